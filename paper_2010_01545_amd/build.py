"""Build libpwadvect.so (HIP, gfx950) in-tree with hipcc.

Every ``csrc/*.hip`` file is compiled to an object and linked into
``paper_2010_01545_amd/libpwadvect.so``.  Packed-FP32 instructions are
disabled (``-target-feature -packed-fp32-ops``); floating-point contraction
follows the source pragmas (the forward stencil switches it off).
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpwadvect.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PW_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=fast-honor-pragmas",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build_library(verbose=False, jobs=8):
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJ_DIR, os.path.basename(s) + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                        and "not a recognized feature" not in l and l.strip())
        if err and verbose:
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def resource_usage(src="pw_march.hip"):
    """Compile one source for the device only with the compiler's
    kernel-resource-usage remarks and return one row per kernel:
    (template arguments, VGPRs, AGPRs, SGPRs, VGPR spill, scratch bytes per
    lane, LDS bytes per workgroup, waves per SIMD)."""
    import re
    cmd = [HIPCC] + CFLAGS + ["--offload-device-only", "-c", os.path.join(CSRC, src), "-o", os.devnull,
                              "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    rows, cur = [], None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            rows.append(cur)
            continue
        m = re.search(r"remark:\s+([A-Za-z /\[\]]+?): (\S+) \[", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return rows


def _march_args(mangled):
    """Template arguments of a march_kernel symbol, readably."""
    import re
    m = re.search(r"march_kernelI(.*?)EEvNS_9MarchArgs", mangled)
    if not m:
        return None
    a = m.group(1)
    types = {"d": "double", "f": "float", "DF16_": "_Float16", "6bf16_t": "bf16", "N12_GLOBAL__N_16bf16_tE": "bf16"}
    out = []
    while a:
        for k in sorted(types, key=len, reverse=True):
            if a.startswith(k):
                out.append(types[k])
                a = a[len(k):]
                break
        else:
            m2 = re.match(r"L([ib])(\d+)E", a)
            if not m2:
                out.append(a)
                break
            v = m2.group(2)
            out.append(("true" if v == "1" else "false") if m2.group(1) == "b" else v)
            a = a[m2.end():]
    return out


def march_resource_table():
    """Markdown table of the x-marching kernels' compile-time resources."""
    lines = ["| T | C | NF | WS | WG | TY | D | EH | UPD | ZW | VGPRs | SGPRs | VGPR spill | SGPR spill | "
             "scratch B/lane | LDS B/WG | waves/SIMD |",
             "|" + "---|" * 17]
    for r in resource_usage("pw_march.hip"):
        a = _march_args(r["name"])
        if not a:
            continue
        lines.append("| " + " | ".join(a + [r.get("VGPRs", "?"), r.get("TotalSGPRs", "?"),
                                           r.get("VGPRs Spill", "?"), r.get("SGPRs Spill", "?"),
                                           r.get("ScratchSize [bytes/lane]", "?"),
                                           r.get("LDS Size [bytes/block]", "?"),
                                           r.get("Occupancy [waves/SIMD]", "?")]) + " |")
    return "\n".join(lines)


if __name__ == "__main__":
    import sys as _sys
    if len(_sys.argv) > 1 and _sys.argv[1] == "--resource-usage":
        print(march_resource_table())
    else:
        print(build_library(verbose=True))
