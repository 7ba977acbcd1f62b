"""Pins of the oracle's rounding-error magnitudes T(c) (pw_oracle_fwd_abs,
pw_oracle_adj_abs).

T(c) is the sum, over the terms coef*A*(B+C) that make up output c, of
|coef|*|A|*(|B|+|C|); for a gradient entry, the sum of the absolute values of
the products it receives.  Every reduced-precision parity bound is a multiple
of it, so a slip here (a dropped or doubled term, a missing absolute value, an
abs mode left switched on) would silently loosen or break those bounds.  The
pins:
  * hand values on the 3x3x3 grid of the source-term hand values (interior,
    top level, periodic wrap, level 0) and, for the adjoint, with a single
    nonzero multiplier, where each entry is one or two products of the su
    terms of one cell (section 2.1, Listing 1);
  * invariance under sign flips of any input cell, multiplier or coefficient
    (only absolute values enter, so the result is bitwise unchanged);
  * the triangle inequality |s(c)| <= T(c), with equality for a cell whose
    terms all share a sign;
  * degree-2 homogeneity in the fields and linearity in the multipliers
    (bitwise for powers of two);
  * the abs entry point leaves the signed adjoint unchanged for later calls;
  * z-halo levels of the inputs are never read.
"""
import json
import os

import numpy as np

from paper_2010_01545_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "hand_values.json")) as f:
        return json.load(f)


def _example(name, n=3):
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = (a.astype(np.float64) for a in (i, j, k))
    if name == "A":
        return i + 1, j + 1, k
    if name == "D":
        return i + 3 * k + 1, 2 * j + k + 1, np.ones_like(i)
    raise KeyError(name)


def _pad(oracle, arrs, h):
    return [oracle.pad_periodic(a, h) for a in arrs]


def _hand_coef(g, n):
    c = g["coefficients"]
    return np.full(n, c["tzc1"]), np.full(n, c["tzc2"]), c["tcx"], c["tcy"]


def test_forward_magnitude_hand_values(oracle):
    g = _golden()
    n = g["grid"][2]
    tz1, tz2, tcx, tcy = _hand_coef(g, n)
    h = 1
    checked = 0
    for cell in g["magnitudes"]["forward"]:
        st = _pad(oracle, _example(cell["example"], n), h)
        t = [oracle.interior(a, h) for a in oracle.fwd(*st, tz1, tz2, tcx, tcy, h, abs_bound=True)]
        ijk = tuple(cell["ijk"])
        for q, name in enumerate(("su", "sv", "sw")):
            if name in cell:
                assert t[q][ijk] == cell[name], (ijk, name, t[q][ijk])
                checked += 1
    assert checked == 13


def test_adjoint_magnitude_hand_values(oracle):
    g = _golden()
    n = g["grid"][2]
    tz1, tz2, tcx, tcy = _hand_coef(g, n)
    h = 1
    st = _pad(oracle, _example("A", n), h)
    lu = np.zeros((n, n, n))
    lu[1, 1, 1] = 1.0
    zero = np.zeros_like(lu)
    sl = _pad(oracle, (lu, zero, zero), h)
    t = [oracle.interior(a, h) for a in oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)]
    expect = [np.zeros((n, n, n)) for _ in range(3)]
    for e in g["magnitudes"]["adjoint"]["entries"]:
        expect["gu gv gw".split().index(e["field"])][tuple(e["ijk"])] = e["value"]
    for q in range(3):
        assert np.array_equal(t[q], expect[q]), (q, t[q], expect[q])


def _random_case(seed, nx, ny, nz):
    u, v, w = inputs.winds(seed, nx, ny, nz)
    lams = inputs.normal_fields(seed + 7, nx, ny, nz)
    return (u, v, w), lams, inputs.coefficients(nz)


def _signs(rng, shape):
    return np.where(rng.random(shape) < 0.5, -1.0, 1.0)


def test_magnitudes_ignore_every_sign(oracle):
    h = 2
    (u, v, w), lams, (tz1, tz2, tcx, tcy) = _random_case(11, 6, 5, 7)
    rng = np.random.default_rng(5)
    ref_f = oracle.fwd(*_pad(oracle, (u, v, w), h), tz1, tz2, tcx, tcy, h, abs_bound=True)
    ref_a = oracle.adj(*_pad(oracle, (u, v, w), h), *_pad(oracle, lams, h), tz1, tz2, tcx, tcy, h,
                       abs_bound=True)
    for trial in range(3):
        f2 = [a * _signs(rng, a.shape) for a in (u, v, w)]
        l2 = [a * _signs(rng, a.shape) for a in lams]
        c1 = tz1 * _signs(rng, tz1.shape)
        c2 = tz2 * _signs(rng, tz2.shape)
        sx, sy = (-tcx, tcy) if trial == 0 else (tcx, -tcy) if trial == 1 else (-tcx, -tcy)
        got_f = oracle.fwd(*_pad(oracle, f2, h), c1, c2, sx, sy, h, abs_bound=True)
        got_a = oracle.adj(*_pad(oracle, f2, h), *_pad(oracle, l2, h), c1, c2, sx, sy, h, abs_bound=True)
        for a, b in zip(got_f + got_a, ref_f + ref_a):
            assert np.array_equal(a, b)


def test_triangle_inequality_and_equality(oracle):
    h = 2
    (u, v, w), lams, (tz1, tz2, tcx, tcy) = _random_case(12, 7, 6, 9)
    st = _pad(oracle, (u, v, w), h)
    sl = _pad(oracle, lams, h)
    s = oracle.fwd(*st, tz1, tz2, tcx, tcy, h)
    t = oracle.fwd(*st, tz1, tz2, tcx, tcy, h, abs_bound=True)
    gsig = oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h)
    gabs = oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)
    for a, b in zip(s + gsig, t + gabs):
        a, b = oracle.interior(a, h), oracle.interior(b, h)
        assert np.all(np.abs(a) <= b * (1 + 1e-14))
        assert np.all(b >= 0)
    # at least one cell's terms do not all share a sign: T is not |s| everywhere
    assert np.any(oracle.interior(t[0], h) > np.abs(oracle.interior(s[0], h)) * (1 + 1e-12))
    # one nonzero term per cell: u = 1, w = 0 and v nonzero at a single cell p;
    # then sv at p +- x and p +- y has exactly one nonzero term (the x terms
    # of sv have the spike as upwind value A, the y terms as A and B), so
    # |sv| == T there, and T == 0 wherever sv has no nonzero term
    n = 4
    one = np.ones((n, n, n))
    vv = np.zeros((n, n, n))
    vv[2, 2, 2] = 3.0
    st = _pad(oracle, (one, vv, 0 * one), h)
    tz1 = np.full(n, 0.5)
    tz2 = np.full(n, 0.25)
    sv = oracle.interior(oracle.fwd(*st, tz1, tz2, 0.75, -1.5, h)[1], h)
    tv = oracle.interior(oracle.fwd(*st, tz1, tz2, 0.75, -1.5, h, abs_bound=True)[1], h)
    hit = tv > 0
    assert sorted(map(tuple, np.argwhere(hit))) == [(1, 2, 2), (2, 1, 2), (2, 3, 2), (3, 2, 2)]
    assert np.array_equal(np.abs(sv[hit]), tv[hit])
    assert tv[3, 2, 2] == 0.75 * 3.0 * 2.0 and tv[2, 3, 2] == 1.5 * 3.0 * 3.0


def test_magnitude_scaling(oracle):
    h = 2
    (u, v, w), lams, (tz1, tz2, tcx, tcy) = _random_case(13, 5, 6, 6)
    st = _pad(oracle, (u, v, w), h)
    sl = _pad(oracle, lams, h)
    t = oracle.fwd(*st, tz1, tz2, tcx, tcy, h, abs_bound=True)
    t2 = oracle.fwd(*[2.0 * a for a in st], tz1, tz2, tcx, tcy, h, abs_bound=True)
    for a, b in zip(t, t2):
        assert np.array_equal(4.0 * a, b)
    ga = oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)
    gb = oracle.adj(*st, *[0.5 * a for a in sl], tz1, tz2, tcx, tcy, h, abs_bound=True)
    for a, b in zip(ga, gb):
        assert np.array_equal(0.5 * a, b)


def test_abs_call_leaves_signed_adjoint_alone(oracle):
    h = 2
    (u, v, w), lams, (tz1, tz2, tcx, tcy) = _random_case(14, 4, 5, 6)
    st = _pad(oracle, (u, v, w), h)
    sl = _pad(oracle, lams, h)
    before = oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h)
    oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)
    after = oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert any(np.any(a < 0) for a in after)


def test_magnitudes_never_read_z_halo(oracle):
    """z-halo levels of the inputs are outside the scheme (su keeps only the
    tzc1 term on the top level, sw is 0 there): NaN in them changes nothing."""
    h = 2
    (u, v, w), lams, (tz1, tz2, tcx, tcy) = _random_case(15, 5, 4, 6)
    st = _pad(oracle, (u, v, w), h)
    sl = _pad(oracle, lams, h)
    ref = oracle.fwd(*st, tz1, tz2, tcx, tcy, h, abs_bound=True) + \
        oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)
    for a in st + sl:
        a[:, :, :h] = np.nan
        a[:, :, -h:] = np.nan
    got = oracle.fwd(*st, tz1, tz2, tcx, tcy, h, abs_bound=True) + \
        oracle.adj(*st, *sl, tz1, tz2, tcx, tcy, h, abs_bound=True)
    for a, b in zip(got, ref):
        assert np.array_equal(oracle.interior(a, h), oracle.interior(b, h))
