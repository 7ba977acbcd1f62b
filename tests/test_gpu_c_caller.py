"""GPU test of the library from a plain C program (tests/c/pw_c_caller.c,
built by __graft_entry__.build()): device arrays from hipMalloc, the public
header, no Python in the path.  The program fills winds and multipliers on
the device, runs the FP64 forward and fused pass, and checks them against the
C oracle it links (forward bit for bit, adjoint within 1e-12 normwise); it
exits 0 only if every check holds.  Shapes: the default ragged 19x13x64 with
halo 2, a column of 150 levels (the tall-column kernels) with halo 3, and a
tiny 3x2x5 grid with halo 1."""
import os
import subprocess

import pytest

from _helpers import log

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "pw_c_caller")


@pytest.mark.parametrize("shape", [None, (9, 7, 150, 3), (3, 2, 5, 1)], ids=["19x13x64h2", "9x7x150h3", "3x2x5h1"])
def test_c_caller_matches_oracle(shape):
    assert os.path.exists(EXE), "tests/c/pw_c_caller is missing: run __graft_entry__.build() first"
    args = [EXE] + ([str(x) for x in shape] if shape else [])
    log("c caller %s" % (shape,))
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "pw_c_caller ok" in r.stdout
