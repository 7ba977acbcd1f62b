"""Shared helpers of the GPU tests: input staging and error measures.

Every GPU result is compared with the oracle on the same seeded inputs; the
inputs are generated on the host (paper_2010_01545_amd.inputs) and copied to
the device, except at the 4096x4096x64 size where the device generator
writes them and the oracle regenerates the x-slabs it needs on the host.
"""
import sys

import numpy as np

import oracle
from paper_2010_01545_amd import inputs

H = inputs.HALO
# every x-marching variant the library builds (PW_TUNE_MARCH_VARIANT values)
MARCH_VARIANTS = list(range(8))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def normwise(got, ref):
    """max |got - ref| / max |ref| (per-cell relative error is meaningless
    where the source term cancels to ~0)."""
    d = np.max(np.abs(got - ref))
    m = np.max(np.abs(ref))
    return float(d / m) if m > 0 else float(d)


def rms_rel(got, ref):
    return float(np.sqrt(np.mean((got - ref) ** 2)) / max(np.sqrt(np.mean(ref ** 2)), 1e-300))


def host_case(nx, ny, nz, seed, smooth=False, lam_seed=None):
    """Interior fields (u, v, w), optional N(0,1) multipliers, coefficients."""
    u, v, w = inputs.winds(seed, nx, ny, nz)
    if smooth:
        u = u + inputs.smooth_u(nx, ny, nz)
    lams = inputs.normal_fields(lam_seed, nx, ny, nz) if lam_seed is not None else None
    return (u, v, w), lams, inputs.coefficients(nz)


def oracle_storage(arrs):
    return [oracle.pad_periodic(a, H) for a in arrs]
