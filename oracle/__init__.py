"""Oracle for the PW advection source terms -- TEST INFRASTRUCTURE ONLY.

A ctypes front end over ``pw_oracle.c`` (plain single-threaded FP64 C) plus
the periodic halo fill and its transpose written with numpy.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the GPU library never calls it and shares no code with it.

Every array here is a numpy float64 array.  "Storage" arrays have shape
(nx+2h, ny+2h, nz+2h), C order, z fastest (the Fortran F(k,j,i) layout of
the paper's section 2.1 and the column/y-batch copies of its section 3);
"interior" arrays have shape (nx, ny, nz).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_libs = {}
_override = []   # a library that replaces both builds (see use_library)

_D = ctypes.POINTER(ctypes.c_double)


def _configure(lib):
    fwd_args = [_D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, _D]
    lib.pw_oracle_fwd.argtypes = fwd_args
    lib.pw_oracle_fwd.restype = None
    lib.pw_oracle_fwd_abs.argtypes = fwd_args
    lib.pw_oracle_fwd_abs.restype = None
    lib.pw_oracle_adj.argtypes = [_D] * 8 + [ctypes.c_double, ctypes.c_double] + \
        [ctypes.c_int] * 4 + [_D, _D, _D]
    lib.pw_oracle_adj.restype = None
    lib.pw_oracle_adj_abs.argtypes = lib.pw_oracle_adj.argtypes
    lib.pw_oracle_adj_abs.restype = None
    lib.pw_oracle_fold_periodic.argtypes = [_D] + [ctypes.c_int] * 4
    lib.pw_oracle_fold_periodic.restype = None
    return lib


def _load(threaded=False):
    if _override:
        return _override[-1]
    name = "libpworacle_omp.so" if threaded else "libpworacle.so"
    if name not in _libs:
        path = os.path.join(HERE, name)
        if not os.path.exists(path):
            from .build import build_oracle
            build_oracle()
        _libs[name] = _configure(ctypes.CDLL(path))
    return _libs[name]


class use_library:
    """Context manager: route every oracle call to the shared library at
    ``path`` (a build of a modified pw_oracle.c), for the mutation tests that
    check the pins catch planted mistakes."""

    def __init__(self, path):
        self.lib = _configure(ctypes.CDLL(path))

    def __enter__(self):
        _override.append(self.lib)
        return self

    def __exit__(self, *exc):
        _override.pop()
        return False


def _p(a):
    return a.ctypes.data_as(_D)


def _check_storage(h, *arrays):
    shape = arrays[0].shape
    for a in arrays:
        if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != shape:
            raise ValueError("oracle arrays must be C-contiguous float64 of one storage shape")
    nx, ny, nz = (s - 2 * h for s in shape)
    if nx < 1 or ny < 1 or nz < 2 or h < 1:
        raise ValueError("bad storage shape %r for halo %d" % (shape, h))
    return nx, ny, nz


def _profiles(tzc1, tzc2, nz):
    t1 = np.ascontiguousarray(tzc1, dtype=np.float64)
    t2 = np.ascontiguousarray(tzc2, dtype=np.float64)
    if t1.shape != (nz,) or t2.shape != (nz,):
        raise ValueError("tzc1/tzc2 must have length nz")
    return t1, t2


def pad_periodic(x, h):
    """Interior (nx,ny,nz) -> storage (nx+2h, ny+2h, nz+2h): periodic copies in
    x and y (the halo swap that precedes advection, section 2.1), zeros in the
    z halo (never read by the scheme)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.pad(x, ((h, h), (h, h), (0, 0)), mode="wrap")
    return np.ascontiguousarray(np.pad(s, ((0, 0), (0, 0), (h, h)), mode="constant"))


def interior(s, h):
    return s[h:-h, h:-h, h:-h]


def fwd(u, v, w, tzc1, tzc2, tcx, tcy, h, threaded=False, abs_bound=False):
    """Source terms (su, sv, sw) as storage arrays from storage fields with
    filled halos.  Halo cells of the results are zero.  With ``abs_bound`` the
    rounding-error magnitudes T(c) are returned instead (see pw_oracle.c)."""
    nx, ny, nz = _check_storage(h, u, v, w)
    t1, t2 = _profiles(tzc1, tzc2, nz)
    outs = [np.zeros_like(u) for _ in range(3)]
    lib = _load(threaded)
    f = lib.pw_oracle_fwd_abs if abs_bound else lib.pw_oracle_fwd
    f(_p(u), _p(v), _p(w), _p(t1), _p(t2), float(tcx), float(tcy), nx, ny, nz, h,
      _p(outs[0]), _p(outs[1]), _p(outs[2]))
    return tuple(outs)


def fwd_update(u, v, w, tzc1, tzc2, tcx, tcy, h, bu, bv, bw, beta):
    """Use of the source terms in the timestep (section 2.1: they are
    integrated into the flow fields after the dynamical core): storage arrays
    whose interior cells hold b + beta * s, the product and the sum each
    rounded in FP64 (numpy evaluates them as two operations), and whose halo
    cells are zero.  b arrays are storage arrays (only interiors are used)."""
    s = fwd(u, v, w, tzc1, tzc2, tcx, tcy, h)
    outs = []
    for b, sq in zip((bu, bv, bw), s):
        o = np.zeros_like(sq)
        ob = np.asarray(b, dtype=np.float64)
        t = np.multiply(np.float64(beta), sq[h:-h, h:-h, h:-h])
        o[h:-h, h:-h, h:-h] = np.add(ob[h:-h, h:-h, h:-h], t)
        outs.append(o)
    return tuple(outs)


def adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, h, abs_bound=False):
    """Gradient of sum(lu*su + lv*sv + lw*sw) over interior cells with respect
    to the interior fields of the x/y-periodic problem, as storage arrays whose
    halo cells are zero.  Fields and multipliers are storage arrays with
    filled halos (only interior multipliers matter).  With ``abs_bound`` the
    sums of absolute values of the contributing products are returned."""
    nx, ny, nz = _check_storage(h, u, v, w, lu, lv, lw)
    t1, t2 = _profiles(tzc1, tzc2, nz)
    outs = [np.empty_like(u) for _ in range(3)]
    lib = _load()
    f = lib.pw_oracle_adj_abs if abs_bound else lib.pw_oracle_adj
    f(_p(u), _p(v), _p(w), _p(lu), _p(lv), _p(lw), _p(t1), _p(t2),
                          float(tcx), float(tcy), nx, ny, nz, h,
                          _p(outs[0]), _p(outs[1]), _p(outs[2]))
    return tuple(outs)


def fold_periodic(g, h):
    """Transpose of pad_periodic on a storage array (in place, returned)."""
    nx, ny, nz = _check_storage(h, g)
    _load().pw_oracle_fold_periodic(_p(g), nx, ny, nz, h)
    return g
