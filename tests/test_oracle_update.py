"""Pins of the oracle's update form o = b + beta * s (the source terms used in
the timestep, section 2.1), checked against the hand-computed source terms and
against the kinetic-energy identity of the Piacsek-Williams form."""
import json
import os

import numpy as np

from paper_2010_01545_amd import inputs
from test_oracle_pins import GOLDEN, H, _example_fields, _random


def _upd(oracle, fields, coef, b, beta, h=H):
    st = [oracle.pad_periodic(f, h) for f in fields]
    sb = [oracle.pad_periodic(x, h) for x in b]
    return [oracle.interior(o, h) for o in oracle.fwd_update(*st, *coef, h, *sb, beta)]


def test_update_of_hand_values(oracle):
    """b + beta * s at the hand-computed cells, with b and beta chosen so that
    every operation is exact: a sign or operand slip (b - beta*s, beta*b + s,
    s alone) changes the value."""
    with open(os.path.join(GOLDEN, "hand_values.json")) as f:
        g = json.load(f)
    c = g["coefficients"]
    n = g["grid"][2]
    coef = (np.full(n, c["tzc1"]), np.full(n, c["tzc2"]), c["tcx"], c["tcy"])
    checked = 0
    for ex in g["examples"]:
        fields = _example_fields(ex["name"])
        b = [np.full((n, n, n), 3.0), np.full((n, n, n), -7.0), np.full((n, n, n), 0.25)]
        o = _upd(oracle, fields, coef, b, 0.5, h=1)
        for cell in ex["cells"]:
            ijk = tuple(cell["ijk"])
            for q, name in enumerate(("su", "sv", "sw")):
                if name in cell:
                    assert o[q][ijk] == b[q][ijk] + 0.5 * cell[name], (ex["name"], ijk, name)
                    checked += 1
    assert checked >= 20


def test_update_special_cases(oracle):
    nx, ny, nz = 7, 5, 9
    fields = _random(21, nx, ny, nz)
    coef = inputs.coefficients(nz)
    b = list(inputs.normal_fields(22, nx, ny, nz))
    st = [oracle.pad_periodic(f, H) for f in fields]
    s = [oracle.interior(a, H) for a in oracle.fwd(*st, *coef, H)]
    # beta = 0 leaves b; b = 0 with beta = 1 gives s; levels whose source term
    # is 0 (level 0; level nz-1 of sw) keep b for any beta
    for x, y in zip(_upd(oracle, fields, coef, b, 0.0), b):
        assert np.array_equal(x, y)
    zero = [np.zeros_like(f) for f in fields]
    for x, y in zip(_upd(oracle, fields, coef, zero, 1.0), s):
        assert np.array_equal(x, y)
    o = _upd(oracle, fields, coef, b, -3.5)
    for q in range(3):
        assert np.array_equal(o[q][:, :, 0], b[q][:, :, 0])
    assert np.array_equal(o[2][:, :, -1], b[2][:, :, -1])


def test_euler_step_energy(oracle):
    """u_new = u + dt * su for the three winds: since the PW form conserves
    kinetic energy (sum of u*su vanishes), the energy grows by exactly
    dt^2 * sum(su^2) up to rounding -- a first-order check that the update adds
    dt * s to the field itself."""
    nx, ny, nz = 12, 10, 16
    fields = _random(23, nx, ny, nz)
    coef = inputs.coefficients(nz)
    st = [oracle.pad_periodic(f, H) for f in fields]
    s = [oracle.interior(a, H) for a in oracle.fwd(*st, *coef, H)]
    dt = 0.75
    new = _upd(oracle, fields, coef, fields, dt)
    for f, sf, nf in zip(fields, s, new):
        growth = np.sum(nf * nf) - np.sum(f * f)
        expect = dt * dt * np.sum(sf * sf)
        assert expect > 0
        # cross term 2 dt sum(f s) is zero up to ~1e-13 of the energy scale
        assert abs(growth - expect) <= 1e-10 * np.sum(f * f), (growth, expect)
    # the same step with the sign flipped gives the same growth: the energy
    # identity alone cannot see the sign, the hand values above do
