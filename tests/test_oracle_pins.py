"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test would fail for a plausible mistake in the oracle: a wrong face
offset (hand values B, C, D), a wrong sign or dropped term (hand values,
energy conservation), a transposed operand or staggering direction (mirror and
transpose symmetries), a wrong top-level rule (hand values at k=nz-1, the
1-D column closed forms), and in the adjoint a wrong or missing scatter
(brute-force Jacobian from the forward alone, Euler identity, finite
differences).
"""
import json
import os

import numpy as np
import pytest

from paper_2010_01545_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
H = 2


def _run(oracle, u, v, w, tzc1, tzc2, tcx, tcy, h=H):
    st = [oracle.pad_periodic(f, h) for f in (u, v, w)]
    return [oracle.interior(s, h) for s in oracle.fwd(*st, tzc1, tzc2, tcx, tcy, h)]


def _random(seed, nx, ny, nz, lids=True):
    u, v, w = inputs.winds(seed, nx, ny, nz)
    if not lids:
        w = inputs.uniform_field(seed, inputs.FIELD_W, nx, ny, nz)
    return u, v, w


def _coef(nz):
    return inputs.coefficients(nz)


# ---------------------------------------------------------------- hand values
def _example_fields(name, n=3):
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = (a.astype(np.float64) for a in (i, j, k))
    one = np.ones_like(i)
    if name == "A":
        return i + 1, j + 1, k
    if name == "B":
        return one, (i * i + 1) * (j + 1), 0 * one
    if name == "C":
        return one, one, i + 2 * j + 4 * k
    if name == "D":
        return i + 3 * k + 1, 2 * j + k + 1, one
    raise KeyError(name)


def test_hand_values(oracle):
    with open(os.path.join(GOLDEN, "hand_values.json")) as f:
        g = json.load(f)
    c = g["coefficients"]
    n = g["grid"][2]
    tz1 = np.full(n, c["tzc1"])
    tz2 = np.full(n, c["tzc2"])
    checked = 0
    for ex in g["examples"]:
        su, sv, sw = _run(oracle, *_example_fields(ex["name"]), tz1, tz2, c["tcx"], c["tcy"], h=1)
        for cell in ex["cells"]:
            ijk = tuple(cell["ijk"])
            for name, arr in (("su", su), ("sv", sv), ("sw", sw)):
                if name in cell:
                    assert arr[ijk] == cell[name], (ex["name"], ijk, name, arr[ijk])
                    checked += 1
    assert checked >= 20


# ------------------------------------------------------------ special cases
def test_zero_winds(oracle):
    z = np.zeros((5, 4, 6))
    tz1, tz2, tcx, tcy = _coef(6)
    for s in _run(oracle, z, z, z, tz1, tz2, tcx, tcy):
        assert np.all(s == 0.0)


def test_uniform_horizontal_flow_is_steady(oracle):
    shape = (4, 5, 7)
    tz1, tz2, tcx, tcy = _coef(7)
    for U, V in ((3.5, -1.25), (-7.0, 2.0)):
        su, sv, sw = _run(oracle, np.full(shape, U), np.full(shape, V), np.zeros(shape),
                          tz1, tz2, tcx, tcy)
        assert np.all(su == 0) and np.all(sv == 0) and np.all(sw == 0)


def test_single_column_closed_form(oracle):
    """nx = ny = 1 with periodic halos: every x and y neighbour is the cell
    itself, the horizontal terms cancel exactly and only the vertical part of
    the scheme remains, which has a short closed form per level."""
    nz = 9
    rng = np.random.default_rng(5)
    u, v, w = (rng.uniform(-10, 10, (1, 1, nz)) for _ in range(3))
    tz1, tz2 = rng.uniform(0.01, 0.05, nz), rng.uniform(0.01, 0.05, nz)
    su, sv, sw = _run(oracle, u, v, w, tz1, tz2, -0.005, -0.004)
    u, v, w, su, sv, sw = (a[0, 0] for a in (u, v, w, su, sv, sw))
    for k in range(nz):
        if k == 0:
            eu = ev = ew = 0.0
        else:
            eu = 2 * (tz1[k] * u[k - 1] * w[k - 1])
            ev = 2 * (tz1[k] * v[k - 1] * w[k - 1])
            if k < nz - 1:
                eu = eu - 2 * (tz2[k] * u[k + 1] * w[k])
                ev = ev - 2 * (tz2[k] * v[k + 1] * w[k])
                ew = tz1[k] * w[k - 1] * (w[k] + w[k - 1]) - tz2[k] * w[k + 1] * (w[k] + w[k + 1])
            else:
                ew = 0.0
        assert su[k] == eu and sv[k] == ev and sw[k] == ew, k


# ------------------------------------------------------------ invariants
def test_quadratic_scaling(oracle):
    nx, ny, nz = 6, 5, 8
    u, v, w = _random(11, nx, ny, nz)
    tz1, tz2, tcx, tcy = _coef(nz)
    base = _run(oracle, u, v, w, tz1, tz2, tcx, tcy)
    for a in (2.0, -1.0):
        sc = _run(oracle, a * u, a * v, a * w, tz1, tz2, tcx, tcy)
        for s0, s1 in zip(base, sc):
            assert np.array_equal(s1, a * a * s0)
    sc = _run(oracle, 3 * u, 3 * v, 3 * w, tz1, tz2, tcx, tcy)
    for s0, s1 in zip(base, sc):
        assert np.max(np.abs(s1 - 9 * s0)) <= 1e-15 * 9 * np.max(np.abs(s0)) * 4


def test_x_mirror(oracle):
    """Reflect x about the u face: u'(i) = -u(N-2-i), v'(i) = v(N-1-i),
    w'(i) = w(N-1-i) (indices mod N); then su'(i) = -su(N-2-i),
    sv'(i) = sv(N-1-i), sw'(i) = sw(N-1-i) exactly."""
    N, M, nz = 7, 6, 8
    u, v, w = _random(12, N, M, nz)
    tz1, tz2, tcx, tcy = _coef(nz)
    su, sv, sw = _run(oracle, u, v, w, tz1, tz2, tcx, tcy)
    iu = (N - 2 - np.arange(N)) % N
    ic = (N - 1 - np.arange(N)) % N
    su2, sv2, sw2 = _run(oracle, -u[iu], v[ic], w[ic], tz1, tz2, tcx, tcy)
    assert np.array_equal(su2, -su[iu])
    assert np.array_equal(sv2, sv[ic])
    assert np.array_equal(sw2, sw[ic])


def test_y_mirror(oracle):
    N, M, nz = 5, 8, 7
    u, v, w = _random(13, N, M, nz)
    tz1, tz2, tcx, tcy = _coef(nz)
    su, sv, sw = _run(oracle, u, v, w, tz1, tz2, tcx, tcy)
    jv = (M - 2 - np.arange(M)) % M
    jc = (M - 1 - np.arange(M)) % M
    su2, sv2, sw2 = _run(oracle, u[:, jc], -v[:, jv], w[:, jc], tz1, tz2, tcx, tcy)
    assert np.array_equal(su2, su[:, jc])
    assert np.array_equal(sv2, -sv[:, jv])
    assert np.array_equal(sw2, sw[:, jc])


def test_xy_transpose(oracle):
    """Swapping the x and y axes (u <-> v, tcx <-> tcy) swaps su and sv."""
    N, M, nz = 6, 9, 8
    u, v, w = _random(14, N, M, nz)
    tz1, tz2, _, _ = _coef(nz)
    tcx, tcy = -0.0043, -0.0061
    su, sv, sw = _run(oracle, u, v, w, tz1, tz2, tcx, tcy)
    T = lambda a: np.ascontiguousarray(a.transpose(1, 0, 2))
    su2, sv2, sw2 = _run(oracle, T(v), T(u), T(w), tz1, tz2, tcy, tcx)
    assert np.array_equal(su2, T(sv))
    assert np.array_equal(sv2, T(su))
    assert np.array_equal(sw2, T(sw))


def test_pw_energy_conservation(oracle):
    """The Piacsek-Williams form conserves kinetic energy: with periodic x/y
    halos, w = 0 on both lids and tzc1[k+1] = tzc2[k], the sums of u*su,
    v*sv and w*sw over the domain vanish in exact arithmetic for any winds
    (each flux telescopes across its face)."""
    nx, ny, nz = 12, 10, 16
    tz1, tz2, tcx, tcy = _coef(nz)
    assert np.array_equal(tz1[1:], tz2[:-1])
    u, v, w = _random(15, nx, ny, nz)
    st = [oracle.pad_periodic(f, H) for f in (u, v, w)]
    s = [oracle.interior(a, H) for a in oracle.fwd(*st, tz1, tz2, tcx, tcy, H)]
    t = [oracle.interior(a, H) for a in oracle.fwd(*st, tz1, tz2, tcx, tcy, H, abs_bound=True)]
    for f, sf, tf in zip((u, v, w), s, t):
        e = np.sum(f * sf)
        scale = np.sum(np.abs(f) * tf)
        assert abs(e) <= 1e-13 * scale, (e, scale)
        # not trivially zero
        assert np.sum(np.abs(f * sf)) > 1e-3 * scale
    # the lids are what makes the vertical flux vanish at the boundaries
    w2 = _random(15, nx, ny, nz, lids=False)[2]
    st2 = [oracle.pad_periodic(f, H) for f in (u, v, w2)]
    sw2 = oracle.interior(oracle.fwd(*st2, tz1, tz2, tcx, tcy, H)[2], H)
    tw2 = oracle.interior(oracle.fwd(*st2, tz1, tz2, tcx, tcy, H, abs_bound=True)[2], H)
    assert abs(np.sum(w2 * sw2)) > 1e-6 * np.sum(np.abs(w2) * tw2)


def test_z_halo_is_never_read(oracle):
    """The scheme reads only interior levels (Listing 1 runs k over the column
    and the top level drops the term that would reach above it): NaN in every
    z-halo level of every input changes no interior result."""
    nx, ny, nz = 6, 5, 7
    coef = _coef(nz)
    u, v, w = _random(25, nx, ny, nz)
    lams = inputs.normal_fields(26, nx, ny, nz)
    st = [oracle.pad_periodic(f, H) for f in (u, v, w)]
    sl = [oracle.pad_periodic(f, H) for f in lams]
    ref_s = oracle.fwd(*st, *coef, H)
    ref_g = oracle.adj(*st, *sl, *coef, H)
    for a in st + sl:
        a[:, :, :H] = np.nan
        a[:, :, -H:] = np.nan
    got_s = oracle.fwd(*st, *coef, H)
    got_g = oracle.adj(*st, *sl, *coef, H)
    for x, y in zip(got_s + got_g, ref_s + ref_g):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))


# ------------------------------------------------------------ coefficients and generator
def test_coefficient_profiles():
    tz1, tz2, tcx, tcy = inputs.coefficients(64)
    assert tcx == -0.25 / 50 and tcy == -0.25 / 50
    assert np.array_equal(tz1[1:], tz2[:-1])
    assert tz2[0] == 0.25 / (10.0 * 1.05 ** 0.5)
    dz = 0.25 / tz2
    np.testing.assert_allclose(dz[1:] / dz[:-1], 1.05, rtol=1e-14)
    # total depth of 64 levels of 10*1.05**k metres
    np.testing.assert_allclose(np.sum(10 * 1.05 ** np.arange(64)), 4340.93, rtol=1e-5)


def test_splitmix64_published_vectors():
    # SplitMix64 reference outputs (Steele, Lea and Flood's generator as
    # distributed with the xorshift/xoshiro family): state 0 and state 1234567
    out0 = inputs.splitmix64_stream(0, 1)
    assert int(out0[0]) == 0xE220A8397B1DCDAF
    out = inputs.splitmix64_stream(1234567, 5)
    assert [int(x) for x in out] == [6457827717110365317, 3203168211198807973,
                                     9817491932198370423, 4593380528125082431,
                                     16408922859458223821]


def test_uniform_field_slabs_and_range():
    nx, ny, nz = 8, 5, 6
    full = inputs.uniform_field(3, inputs.FIELD_V, nx, ny, nz)
    assert full.min() >= -10 and full.max() < 10
    slab = inputs.uniform_field(3, inputs.FIELD_V, nx, ny, nz, x0=-2, x1=3)
    assert np.array_equal(slab, full[np.arange(-2, 3) % nx])
    u, v, w = inputs.winds(3, nx, ny, nz)
    assert np.all(w[:, :, 0] == 0) and np.all(w[:, :, -1] == 0)
    assert abs(u.mean()) < 1.0 and 4 < u.std() < 7
