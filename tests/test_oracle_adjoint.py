"""Pins of the oracle's scatter-form adjoint, from the forward alone.

Every source term is a sum of products of two field values, so s(x) is a
homogeneous quadratic: s(x + d) = s(x) + J(x) d + s(d) exactly (in real
arithmetic), central differences have no truncation error, and Euler's
theorem gives <x, J(x)^T l> = 2 <s(x), l>.  The brute-force Jacobian below is
built from forward calls only and does not look at how the adjoint is coded.
"""
import numpy as np
import pytest

from paper_2010_01545_amd import inputs

H = 2


def _fwd(oracle, fields, coef):
    st = [oracle.pad_periodic(f, H) for f in fields]
    return [oracle.interior(s, H) for s in oracle.fwd(*st, *coef, H)]


def _adj(oracle, fields, lams, coef):
    st = [oracle.pad_periodic(f, H) for f in fields]
    sl = [oracle.pad_periodic(f, H) for f in lams]
    return [oracle.interior(g, H) for g in oracle.adj(*st, *sl, *coef, H)]


def _dot(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


def _setup(nx, ny, nz, seed):
    fields = list(inputs.winds(seed, nx, ny, nz))
    lams = list(inputs.normal_fields(seed + 100, nx, ny, nz))
    return fields, lams, inputs.coefficients(nz)


@pytest.mark.parametrize("shape", [(4, 4, 5), (3, 5, 4), (1, 2, 3)])
def test_adjoint_matches_bruteforce_jacobian(oracle, shape):
    nx, ny, nz = shape
    fields, lams, coef = _setup(nx, ny, nz, 21)
    # no lids here: the Jacobian must be right for any w
    fields[2] = inputs.uniform_field(21, inputs.FIELD_W, nx, ny, nz)
    s0 = _fwd(oracle, fields, coef)
    grads = _adj(oracle, fields, lams, coef)
    scale = max(np.max(np.abs(g)) for g in grads)
    for f in range(3):
        for p in np.ndindex(shape):
            e = [np.zeros(shape) for _ in range(3)]
            e[f][p] = 1.0
            xp = [a + b for a, b in zip(fields, e)]
            s1 = _fwd(oracle, xp, coef)
            se = _fwd(oracle, e, coef)
            jcol = [a - b - c for a, b, c in zip(s1, s0, se)]
            bf = _dot(lams, jcol)
            assert abs(bf - grads[f][p]) <= 1e-12 * scale, (f, p, bf, grads[f][p])


def test_euler_identity(oracle):
    fields, lams, coef = _setup(16, 12, 10, 22)
    s = _fwd(oracle, fields, coef)
    g = _adj(oracle, fields, lams, coef)
    lhs, rhs = _dot(fields, g), 2.0 * _dot(s, lams)
    mag = _dot([np.abs(a) for a in fields], [np.abs(b) for b in g])
    assert abs(lhs - rhs) <= 1e-13 * mag, (lhs, rhs)


def test_dot_product_identity(oracle):
    fields, lams, coef = _setup(16, 12, 10, 23)
    delta = list(inputs.normal_fields(23 + 200, 16, 12, 10))
    sp = _fwd(oracle, [a + d for a, d in zip(fields, delta)], coef)
    sm = _fwd(oracle, [a - d for a, d in zip(fields, delta)], coef)
    jd = [(a - b) / 2.0 for a, b in zip(sp, sm)]
    g = _adj(oracle, fields, lams, coef)
    lhs, rhs = _dot(jd, lams), _dot(delta, g)
    mag = _dot([np.abs(a) for a in delta], [np.abs(b) for b in g])
    assert abs(lhs - rhs) <= 1e-13 * mag, (lhs, rhs)


def test_central_differences_on_random_cells(oracle):
    nx, ny, nz = 12, 10, 16
    fields, lams, coef = _setup(nx, ny, nz, 24)
    g = _adj(oracle, fields, lams, coef)
    rng = np.random.default_rng(24)
    h = 1e-6
    for _ in range(64):
        f = int(rng.integers(3))
        p = tuple(int(rng.integers(n)) for n in (nx, ny, nz))
        xp = [a.copy() for a in fields]
        xm = [a.copy() for a in fields]
        xp[f][p] += h
        xm[f][p] -= h
        step = xp[f][p] - xm[f][p]
        sp, sm = _fwd(oracle, xp, coef), _fwd(oracle, xm, coef)
        fd = sum(float(np.sum(l * (a - b))) for l, a, b in zip(lams, sp, sm)) / step
        # rounding only: |s| ~ 1 and eps/step ~ 1e-10 per cell of the footprint
        assert abs(fd - g[f][p]) <= 1e-7 * max(1.0, abs(g[f][p])), (f, p, fd, g[f][p])


def test_fold_is_transpose_of_pad(oracle):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 4, 6))
    y = rng.standard_normal((9, 8, 10))
    lhs = float(np.sum(oracle.pad_periodic(x, H) * y))
    g = oracle.fold_periodic(y.copy(), H)
    rhs = float(np.sum(x * oracle.interior(g, H)))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(y))
