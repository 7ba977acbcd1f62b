"""Build the plain-C test caller of the library (test infrastructure only).

``pw_c_caller`` (tests/c/pw_c_caller.c) is C99 compiled with gcc against the
public header include/pwadvect.h, linked with the built library
(paper_2010_01545_amd/libpwadvect.so), the oracle (oracle/libpworacle.so)
and the HIP runtime; run-time paths are relative to the program, so the
repository can move.  Build the library and the oracle first.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "pw_c_caller.c")
OUT = os.path.join(HERE, "pw_c_caller")


def build_c_caller(verbose=False):
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), SRC, "-o", OUT + ".tmp",
           "-L" + os.path.join(ROOT, "paper_2010_01545_amd"), "-lpwadvect",
           "-L" + os.path.join(ROOT, "oracle"), "-lpworacle",
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_2010_01545_amd", "-Wl,-rpath,$ORIGIN/../../oracle",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build_c_caller(verbose=True))
