"""Seeded synthetic inputs for the PW advection workloads (host side, numpy).

This module holds no part of the advection arithmetic; it only builds the
inputs that both the GPU library and the CPU oracle consume:

* uniform wind fields from a counter-based SplitMix64 generator
  (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014), so any x-slab of any field can be regenerated on
  its own, on the host or on the device (the library's ``pw_fill_uniform``
  implements the same published definition);
* the coefficient profiles tcx, tcy, tzc1(k), tzc2(k) of a stretched vertical
  grid, as the workloads define them (the paper names the coefficients in
  Listing 1 but gives no formula for them);
* standard-normal multiplier / perturbation fields from numpy's default
  generator;
* the smooth large-scale component of the precision workload.

Counter layout.  Value number ``idx`` (the interior linear index
(i*ny + j)*nz + k) of field ``fid`` under seed ``seed`` is the SplitMix64 output
z = mix(S + (idx+1)*GAMMA) with S = seed*256 + fid and
GAMMA = 0x9E3779B97F4A7C15.  Its top 53 bits m give t = (m - 2**52) * 2**-52,
exactly representable in [-1, 1); a field on [-a, a) is a*t, rounded once.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

FIELD_U, FIELD_V, FIELD_W = 0, 1, 2
FIELD_LU, FIELD_LV, FIELD_LW = 3, 4, 5


def splitmix64_mix(z):
    """The SplitMix64 output function (finaliser) on uint64 numpy values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(state, n):
    """First n outputs of SplitMix64 started from ``state``."""
    with np.errstate(over="ignore"):
        ctr = np.uint64(state) + (np.arange(1, n + 1, dtype=np.uint64) * GAMMA)
    return splitmix64_mix(ctr)


def unit_symmetric(seed, fid, idx):
    """t in [-1, 1) for counter values ``idx`` (uint64 array), exact doubles."""
    state = np.uint64(seed * 256 + fid)
    with np.errstate(over="ignore"):
        z = splitmix64_mix(state + (idx.astype(np.uint64) + np.uint64(1)) * GAMMA)
    m = (z >> np.uint64(11)).astype(np.int64) - np.int64(1 << 52)
    return m.astype(np.float64) * (2.0 ** -52)


def uniform_field(seed, fid, nx, ny, nz, amp=10.0, x0=0, x1=None, zero_lids=False):
    """Interior field U(-amp, amp) of shape (x1-x0, ny, nz) for x-planes
    [x0, x1) of an (nx, ny, nz) grid.  Planes outside [0, nx) wrap
    periodically, so x0 may be negative and x1 may exceed nx.  With
    ``zero_lids`` levels 0 and nz-1 are set to 0 (the rigid lids of w)."""
    if x1 is None:
        x1 = nx
    planes = np.arange(x0, x1) % nx
    jk = np.arange(ny * nz, dtype=np.uint64)
    idx = (planes.astype(np.uint64)[:, None] * np.uint64(ny * nz) + jk[None, :])
    out = unit_symmetric(seed, fid, idx.reshape(-1)).reshape(len(planes), ny, nz)
    if amp != 1.0:
        out *= amp
    if zero_lids:
        out[:, :, 0] = 0.0
        out[:, :, nz - 1] = 0.0
    return out


def winds(seed, nx, ny, nz, amp=10.0, x0=0, x1=None):
    """(u, v, w) interior fields U(-amp, amp), w zero on levels 0 and nz-1."""
    u = uniform_field(seed, FIELD_U, nx, ny, nz, amp, x0, x1)
    v = uniform_field(seed, FIELD_V, nx, ny, nz, amp, x0, x1)
    w = uniform_field(seed, FIELD_W, nx, ny, nz, amp, x0, x1, zero_lids=True)
    return u, v, w


def multipliers_uniform(seed, nx, ny, nz, amp=1.0, x0=0, x1=None):
    """(lu, lv, lw) interior fields U(-amp, amp) from the counter generator
    (used where a normal draw of the whole grid would be too slow)."""
    return tuple(uniform_field(seed, f, nx, ny, nz, amp, x0, x1)
                 for f in (FIELD_LU, FIELD_LV, FIELD_LW))


def normal_fields(seed, nx, ny, nz, count=3):
    """``count`` independent N(0,1) interior fields from numpy's default
    generator seeded with ``seed`` (drawn in order)."""
    rng = np.random.default_rng(seed)
    return tuple(rng.standard_normal((nx, ny, nz)) for _ in range(count))


def smooth_u(nx, ny, nz, amp=10.0, x0=0, x1=None):
    """amp*sin(2 pi x/Lx)*cos(2 pi y/Ly) at cell (i, j), x = i*dx, Lx = nx*dx,
    constant in z, evaluated in FP64."""
    if x1 is None:
        x1 = nx
    i = (np.arange(x0, x1) % nx).astype(np.float64)
    j = np.arange(ny, dtype=np.float64)
    plane = amp * np.sin(2.0 * np.pi * i / nx)[:, None] * np.cos(2.0 * np.pi * j / ny)[None, :]
    return np.repeat(plane[:, :, None], nz, axis=2)


def coefficients(nz, dx=50.0, dy=50.0, dz0=10.0, stretch=1.05):
    """Coefficients of the stretched-grid workloads.

    tcx = -0.25/dx, tcy = -0.25/dy (taken literally, sign included).
    With dz(x) = dz0 * stretch**x and interior level index k (0-based),
    tzc1[k] = 0.25/dz(k - 1/2) and tzc2[k] = 0.25/dz(k + 1/2).  Both come from
    one table hz[m] = 0.25/dz(m + 1/2), m = -1..nz-1, so tzc1[k+1] equals
    tzc2[k] bit for bit.
    Returns (tzc1, tzc2, tcx, tcy) with FP64 arrays of length nz.
    """
    m = np.arange(-1, nz, dtype=np.float64)
    hz = 0.25 / (dz0 * np.power(stretch, m + 0.5))
    tzc1 = np.ascontiguousarray(hz[:-1])
    tzc2 = np.ascontiguousarray(hz[1:])
    return tzc1, tzc2, -0.25 / dx, -0.25 / dy


# The five workload shapes (x, y, z) and seeds.
def round_storage(x, kind):
    """Values of ``x`` (float64) as the library's storage type ``kind`` holds
    them, returned as float64: "f64" unchanged; "f32" rounded to float;
    "f16" / "bf16" rounded to float, then to IEEE binary16 / bfloat16 (each
    step round-to-nearest-even, as the device generator defines it)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "f64":
        return x.copy()
    x32 = x.astype(np.float32)
    if kind == "f32":
        return x32.astype(np.float64)
    if kind == "f16":
        return x32.astype(np.float16).astype(np.float64)
    if kind == "bf16":
        b = x32.view(np.uint32).astype(np.uint64)
        nan = np.isnan(x32)
        r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        out = r.astype(np.uint32).view(np.float32).astype(np.float64)
        out[nan] = np.nan
        return out
    raise ValueError(kind)


WORKLOADS = {
    "small": dict(nx=32, ny=32, nz=64, seed=0),
    "medium": dict(nx=256, ny=256, nz=64, seed=1),
    "precision": dict(nx=1024, ny=1024, nz=64, seed=2),
    "differentiation": dict(nx=512, ny=512, nz=64, seed=3),
    "paper_scale": dict(nx=4096, ny=4096, nz=64, seed=4),
}
HALO = 2
