"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pwadvect.h")
LIB = os.path.join(ROOT, "paper_2010_01545_amd", "libpwadvect.so")

PW_OK, PW_ERR_ARG, PW_ERR_ALIAS, PW_ERR_ALIGN, PW_ERR_SIZE = 0, -1, -2, -3, -4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2010_01545_amd.build import build_library
        build_library()
    L = ctypes.CDLL(LIB)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.pw_advect_fwd.argtypes = [vp] * 5 + [d, d] + [i] * 4 + [vp] * 3 + [i, vp]
    L.pw_advect_adj.argtypes = [vp] * 8 + [d, d] + [i] * 4 + [vp] * 3 + [i, vp]
    L.pw_advect_fwd_adj.argtypes = [vp] * 8 + [d, d] + [i] * 4 + [vp] * 6 + [i, vp]
    L.pw_advect_fwd_update.argtypes = [vp] * 5 + [d, d] + [i] * 4 + [vp] * 3 + [d] + [vp] * 3 + [i, vp]
    L.pw_pad_periodic.argtypes = [vp, vp] + [i] * 5 + [vp]
    L.pw_halo_periodic.argtypes = [vp] + [i] * 5 + [vp]
    L.pw_fill_uniform.argtypes = [vp] + [i] * 4 + [ctypes.c_ulonglong, i, d, i, i, vp]
    L.pw_last_error.restype = ctypes.c_char_p
    return L


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert {"pw_advect_fwd", "pw_advect_adj", "pw_advect_fwd_adj"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_version(lib):
    assert lib.pw_version() >= 100


# fake, well-aligned, non-overlapping "device" addresses: every case below
# must be rejected by host-side checks before any of them is dereferenced
GRID = (8, 6, 64, 2)
STORAGE = (8 + 4) * (6 + 4) * (64 + 4) * 8
ADDR = [0x10000000 + q * 0x01000000 for q in range(16)]


def fwd(lib, ptrs=None, grid=GRID, dtype=0):
    p = list(ADDR[:8]) if ptrs is None else ptrs
    return lib.pw_advect_fwd(p[0], p[1], p[2], p[3], p[4], -0.005, -0.005, *grid, p[5], p[6], p[7],
                             dtype, None)


def test_rejects_null_pointers(lib):
    for q in range(8):
        p = list(ADDR[:8])
        p[q] = None
        assert fwd(lib, p) == PW_ERR_ARG
        assert b"NULL" in lib.pw_last_error()


@pytest.mark.parametrize("grid", [(0, 6, 64, 2), (8, 0, 64, 2), (8, 6, 1, 2), (8, 6, 64, 0), (-3, 6, 64, 2)])
def test_rejects_bad_sizes(lib, grid):
    assert fwd(lib, grid=grid) == PW_ERR_ARG


def test_rejects_bad_dtype(lib):
    assert fwd(lib, dtype=7) == PW_ERR_ARG


def test_dtype_codes(lib):
    """PW_F64..PW_BF16 (0..4) pass the dtype check; the element size follows
    the storage type (8, 4, 4, 2, 2 bytes) in the alignment and overlap checks."""
    assert fwd(lib, dtype=5) == PW_ERR_ARG and b"dtype" in lib.pw_last_error()
    assert fwd(lib, dtype=-1) == PW_ERR_ARG
    cells = STORAGE // 8
    for dtype, es in ((0, 8), (1, 4), (2, 4), (3, 2), (4, 2)):
        p = list(ADDR[:8])
        p[5] += es // 2 if es > 2 else 1      # su misaligned for its element type
        assert fwd(lib, p, dtype=dtype) == PW_ERR_ALIGN, dtype
        p = list(ADDR[:8])
        p[6] = p[5] + cells * es - es         # sv starts on su's last element
        assert fwd(lib, p, dtype=dtype) == PW_ERR_ALIAS, dtype
        p[6] = p[5] + cells * es              # sv starts right after su
        assert fwd(lib, p, dtype=dtype) not in (PW_ERR_ALIAS, PW_ERR_ALIGN), dtype


def test_rejects_size_overflow(lib):
    assert fwd(lib, grid=(2 ** 31 - 3, 6, 64, 2)) == PW_ERR_SIZE
    assert fwd(lib, grid=(8, 2 ** 30, 64, 2)) == PW_ERR_SIZE


def test_rejects_misaligned(lib):
    p = list(ADDR[:8])
    p[6] += 4  # sv misaligned for doubles
    assert fwd(lib, p) == PW_ERR_ALIGN
    p = list(ADDR[:8])
    p[3] += 4  # tzc1 is always double
    assert fwd(lib, p, dtype=1) == PW_ERR_ALIGN


def test_rejects_aliasing(lib):
    p = list(ADDR[:8])
    p[5] = p[0]  # su == u
    assert fwd(lib, p) == PW_ERR_ALIAS
    p = list(ADDR[:8])
    p[6] = p[5] + STORAGE // 2  # sv overlaps su
    assert fwd(lib, p) == PW_ERR_ALIAS
    p = list(ADDR[:8])
    p[7] = p[2] + 8  # sw overlaps w
    assert fwd(lib, p) == PW_ERR_ALIAS
    # inputs may share memory with each other
    p = list(ADDR[:8])
    p[1] = p[0]
    assert fwd(lib, p) not in (PW_ERR_ALIAS, PW_ERR_ALIGN, PW_ERR_SIZE)


def test_adj_and_fused_checks(lib):
    p = ADDR
    rc = lib.pw_advect_adj(p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], -0.005, -0.005, *GRID,
                           p[3], p[8], p[9], 0, None)
    assert rc == PW_ERR_ALIAS  # gu == lu
    rc = lib.pw_advect_fwd_adj(p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], -0.005, -0.005, *GRID,
                               p[8], p[9], p[10], p[11], p[12], p[8], 0, None)
    assert rc == PW_ERR_ALIAS  # gw == su
    rc = lib.pw_advect_fwd_adj(p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], -0.005, -0.005, *GRID,
                               None, p[9], p[10], p[11], p[12], p[13], 0, None)
    assert rc == PW_ERR_ARG


def update(lib, p, b, o):
    return lib.pw_advect_fwd_update(p[0], p[1], p[2], p[3], p[4], -0.005, -0.005, *GRID, b[0], b[1], b[2], 0.5,
                                    o[0], o[1], o[2], 0, None)


def test_update_checks(lib):
    p, o = ADDR[:5], ADDR[8:11]
    # a null or misaligned base array
    assert update(lib, p, [None, ADDR[12], ADDR[13]], o) == PW_ERR_ARG
    assert update(lib, p, [ADDR[11] + 4, ADDR[12], ADDR[13]], o) == PW_ERR_ALIGN
    # bv is the output ou: only ov itself may be passed as bv
    assert update(lib, p, [ADDR[11], o[0], ADDR[13]], o) == PW_ERR_ALIAS
    assert b"bv overlaps output" in lib.pw_last_error()
    # bw straddles ow
    assert update(lib, p, [ADDR[11], ADDR[12], o[2] - 8], o) == PW_ERR_ALIAS
    # an output over an input field is refused as for the plain forward
    assert update(lib, p, list(p[:3]), [p[0], o[1], o[2]]) == PW_ERR_ALIAS
    # accepted by the host-side checks: in place (b = o), Euler (b = u, v, w),
    # separate arrays; they then fail only at the device query
    for b in (list(o), list(p[:3]), ADDR[11:14]):
        assert update(lib, p, b, o) == PW_ERR_ARG
        assert b"device" in lib.pw_last_error()


def test_host_pointer_rejected_without_launch(lib):
    """A host address passes the host-side checks but must be refused as not
    device memory (on a machine without a GPU the runtime query fails, which
    is reported the same way)."""
    bufs = [ctypes.create_string_buffer(STORAGE + 64) for _ in range(6)]
    tz = [ctypes.create_string_buffer(64 * 8 + 16) for _ in range(2)]
    al = lambda b: (ctypes.addressof(b) + 15) // 16 * 16
    p = [al(bufs[0]), al(bufs[1]), al(bufs[2]), al(tz[0]), al(tz[1]), al(bufs[3]), al(bufs[4]), al(bufs[5])]
    assert fwd(lib, p) == PW_ERR_ARG
    assert b"device" in lib.pw_last_error()


def test_utility_checks(lib):
    assert lib.pw_halo_periodic(None, 8, 6, 64, 2, 0, None) == PW_ERR_ARG
    assert lib.pw_pad_periodic(ADDR[0], ADDR[0], 8, 6, 64, 2, 0, None) == PW_ERR_ALIAS
    assert lib.pw_fill_uniform(ADDR[0], 8, 6, 64, 2, 1, 300, 10.0, 0, 0, None) == PW_ERR_ARG
    assert lib.pw_set_kernel(9) == PW_ERR_ARG
    prev = lib.pw_set_kernel(1)
    assert lib.pw_get_kernel() == 1
    lib.pw_set_kernel(prev)


# ---------------------------------------------------------------- tuning knobs
PW_TUNE_KERNEL, PW_TUNE_MARCH_VARIANT, PW_TUNE_MARCH_LX, PW_TUNE_COPY_OUT, PW_TUNE_BLOCK_ORDER, PW_TUNE_TALL_WAVES = \
    0, 1, 2, 3, 4, 5


def _get(lib, knob):
    v = ctypes.c_int(-99)
    rc = lib.pw_get_tuning(knob, ctypes.byref(v))
    return rc, v.value


def test_tuning_knobs_set_get_and_reject(lib):
    lib.pw_get_tuning.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    defaults = {PW_TUNE_KERNEL: 0, PW_TUNE_MARCH_VARIANT: -1, PW_TUNE_MARCH_LX: 0, PW_TUNE_COPY_OUT: 3,
                PW_TUNE_BLOCK_ORDER: -1, PW_TUNE_TALL_WAVES: 0}
    for knob, d in defaults.items():
        assert _get(lib, knob) == (PW_OK, d)
    for knob, good, bad in ((PW_TUNE_KERNEL, 2, 3), (PW_TUNE_MARCH_VARIANT, 7, 8),
                            (PW_TUNE_MARCH_LX, 9, -1), (PW_TUNE_COPY_OUT, 2, 4), (PW_TUNE_BLOCK_ORDER, 16, 65537),
                            (PW_TUNE_TALL_WAVES, 3, 5)):
        assert lib.pw_set_tuning(knob, good) == PW_OK
        assert _get(lib, knob) == (PW_OK, good)
        assert lib.pw_set_tuning(knob, bad) == PW_ERR_ARG
        assert _get(lib, knob) == (PW_OK, good)          # unchanged by a refused value
        assert lib.pw_set_tuning(knob, defaults[knob]) == PW_OK
    assert lib.pw_set_tuning(PW_TUNE_MARCH_VARIANT, -2) == PW_ERR_ARG
    assert lib.pw_set_tuning(PW_TUNE_BLOCK_ORDER, -2) == PW_ERR_ARG
    assert lib.pw_set_tuning(PW_TUNE_TALL_WAVES, 1) == PW_ERR_ARG
    assert lib.pw_set_tuning(17, 0) == PW_ERR_ARG
    assert _get(lib, 17)[0] == PW_ERR_ARG
    assert lib.pw_get_tuning(PW_TUNE_KERNEL, None) == PW_ERR_ARG
    # pw_set_kernel returns the previous family
    assert lib.pw_set_kernel(1) == 0 and lib.pw_get_kernel() == 1
    assert lib.pw_set_kernel(5) == PW_ERR_ARG and lib.pw_get_kernel() == 1
    assert lib.pw_set_kernel(0) == 1


def test_tuning_is_per_thread(lib):
    """A knob set on one thread is invisible to another (the library keeps no
    process-wide selection)."""
    import threading
    lib.pw_get_tuning.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    seen = {}

    def worker():
        seen["before"] = _get(lib, PW_TUNE_MARCH_VARIANT)
        lib.pw_set_tuning(PW_TUNE_MARCH_VARIANT, 4)
        lib.pw_set_kernel(2)
        seen["after"] = _get(lib, PW_TUNE_MARCH_VARIANT)
    assert lib.pw_set_tuning(PW_TUNE_MARCH_VARIANT, 3) == PW_OK
    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert seen == {"before": (PW_OK, -1), "after": (PW_OK, 4)}
    assert _get(lib, PW_TUNE_MARCH_VARIANT) == (PW_OK, 3)
    assert lib.pw_get_kernel() == 0
    lib.pw_set_tuning(PW_TUNE_MARCH_VARIANT, -1)


def test_library_reads_no_environment():
    """No getenv in the library's imports: kernel choice and every other
    setting come from the caller's arguments and tuning calls only."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True, text=True, check=True).stdout
    names = {line.split()[-1].split("@")[0] for line in out.splitlines() if line.strip()}
    assert not {"getenv", "secure_getenv"} & names


# ---------------------------------------------------------------- streaming copy reference
def test_stream_copy_checks(lib):
    vp = ctypes.c_void_p
    lib.pw_stream_copy.argtypes = [vp, vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   vp]

    def call(src, dst, n, nbytes, blocks=0, unit=16, hints=0):
        s = (vp * len(src))(*src)
        d = (vp * len(dst))(*dst)
        return lib.pw_stream_copy(ctypes.cast(s, vp), ctypes.cast(d, vp), n, nbytes, unit, blocks, hints, None)

    src, dst = ADDR[:3], ADDR[3:6]
    assert lib.pw_stream_copy(None, None, 3, 4096, 4, 0, 0, None) == PW_ERR_ARG
    assert call(src, dst, 3, 4096, hints=4) == PW_ERR_ARG               # unknown hint bit
    assert call(src, dst, 3, 4096, hints=-1) == PW_ERR_ARG
    assert call(src, dst, 0, 4096) == PW_ERR_ARG
    assert call(ADDR[:9], ADDR[:9], 9, 4096) == PW_ERR_ARG
    assert call(src, dst, 3, 4100) == PW_ERR_ARG                       # not a multiple of 16
    assert call(src, dst, 3, 4098, unit=4) == PW_ERR_ARG               # not a multiple of 4
    assert call(src, dst, 3, 4096, unit=2) == PW_ERR_ARG               # no 2-byte unit
    assert call(src, dst, 3, 4096, -1) == PW_ERR_ARG
    assert call([ADDR[0] + 8] + src[1:], dst, 3, 4096) == PW_ERR_ALIGN
    assert call([ADDR[0] + 4] + src[1:], dst, 3, 4096, unit=8) == PW_ERR_ALIGN
    assert call(src, [dst[0], dst[1], src[2] + 16], 3, 4096) == PW_ERR_ALIAS   # dst overlaps a source
    assert call(src, [dst[0], dst[0] + 4080, dst[2]], 3, 4096) == PW_ERR_ALIAS  # two destinations overlap
    assert call([0] + src[1:], dst, 3, 4096) == PW_ERR_ARG             # NULL entry
    assert call(src, dst, 3, (1 << 34) + (1 << 33), unit=4) == PW_ERR_SIZE   # 2^32 or more units in one pass


# ---------------------------------------------------------------- C and C++ callers
def _tool(name):
    import shutil
    path = shutil.which(name)
    if not path:
        pytest.fail("%s is needed to check the header" % name)
    return path


def test_header_is_strict_c99_and_cxx(tmp_path):
    """The header compiles on its own as strict C99 and as C++17 (-pedantic
    -Wall -Wextra -Werror)."""
    import subprocess
    body = '#include "pwadvect.h"\nint main(void) { return pw_version() > 0 ? 0 : 1; }\n'
    for compiler, std, name in (("gcc", "-std=c99", "h.c"), ("g++", "-std=c++17", "h.cpp")):
        src = tmp_path / name
        src.write_text(body)
        subprocess.run([_tool(compiler), std, "-pedantic", "-Wall", "-Wextra", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-fsyntax-only", str(src)], check=True)


def test_every_declared_function_links_with_c_linkage(tmp_path):
    """A C++ program that takes the address of every function the header
    declares links against the library: each is defined, and with C linkage
    (a declaration outside the header's extern "C" block would look for a
    mangled name and fail to link)."""
    import subprocess
    names = declared_functions()
    src = tmp_path / "all.cpp"
    src.write_text('#include "pwadvect.h"\n#include <cstdio>\nint main() {\n  const void* fns[] = {\n' +
                   "".join("    (const void*)&%s,\n" % n for n in names) +
                   '  };\n  std::printf("%d\\n", (int)(sizeof fns / sizeof fns[0]));\n  return 0;\n}\n')
    out = tmp_path / "all"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    subprocess.run([_tool("g++"), "-std=c++17", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(out), "-L", os.path.dirname(LIB), "-lpwadvect", "-Wl,-rpath," + os.path.dirname(LIB),
                    "-Wl,-rpath-link," + rocm_lib],
                   check=True)
    ran = subprocess.run([str(out)], capture_output=True, text=True, check=True, timeout=60)
    assert int(ran.stdout.strip()) == len(names)


def test_c_caller_builds():
    """The tests' plain-C caller (tests/c/pw_c_caller.c, run on the GPU by
    test_gpu_c_caller) compiles as C99 against the header and links with the
    library, the oracle and the HIP runtime, finding the in-tree library at
    run time."""
    import importlib.util
    import subprocess
    spec = importlib.util.spec_from_file_location("pw_c_caller_build", os.path.join(ROOT, "tests", "c", "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    exe = m.build_c_caller()
    deps = subprocess.run(["ldd", exe], capture_output=True, text=True, check=True).stdout
    line = [ln for ln in deps.splitlines() if "libpwadvect.so" in ln]
    assert line and os.path.realpath(line[0].split("=>")[1].split("(")[0].strip()) == os.path.realpath(LIB)
