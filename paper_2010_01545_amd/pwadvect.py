"""ctypes binding of libpwadvect (argument marshalling only).

Each function takes torch tensors (on a ROCm device; host tensors for
``fwd_host``), checks that they are contiguous and of one storage shape, and
passes raw pointers, sizes and the current torch stream to the C entry point
of the same name in ``include/pwadvect.h``.  All computation happens in the
HIP library; if it is not built, importing this module raises ImportError.

Storage tensors have shape (nx+2h, ny+2h, nz+2h), z fastest; the grid size is
taken from the shape and the ``halo`` argument.  The storage dtype selects the
element type (float64, float32, float16, bfloat16); ``compute=torch.float64``
with float32 storage selects FP64 arithmetic (PW_F32_F64).
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwadvect.so")

PW_F64, PW_F32, PW_F32_F64, PW_F16, PW_BF16 = 0, 1, 2, 3, 4
KERNELS = {"auto": 0, "direct": 1, "march": 2}
# tuning knobs of the calling thread (pw_set_tuning)
TUNE_KERNEL, TUNE_MARCH_VARIANT, TUNE_MARCH_LX, TUNE_COPY_OUT, TUNE_BLOCK_ORDER, TUNE_TALL_WAVES = 0, 1, 2, 3, 4, 5
MARCH_VARIANTS = 8
COPY_OUT = {"runtime": 0, "kernel": 1, "direct": 2, "auto": 3}
COPY_NT_LOADS, COPY_NT_STORES = 1, 2     # pw_stream_copy hints
ORDERS = {"default": -1, "xcd": 0, "natural": 1}   # or an int G: groups of G strips per XCD
ERRORS = {-1: "PW_ERR_ARG", -2: "PW_ERR_ALIAS", -3: "PW_ERR_ALIGN", -4: "PW_ERR_SIZE",
          -5: "PW_ERR_UNSUPPORTED", -6: "PW_ERR_HIP"}

if not os.path.exists(LIB_PATH):
    raise ImportError("libpwadvect.so is not built (%s); run __graft_entry__.build() "
                      "or python paper_2010_01545_amd/build.py" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
lib.pw_advect_fwd.argtypes = [_vp] * 5 + [_d, _d] + [_i] * 4 + [_vp] * 3 + [_i, _vp]
lib.pw_advect_adj.argtypes = [_vp] * 8 + [_d, _d] + [_i] * 4 + [_vp] * 3 + [_i, _vp]
lib.pw_advect_fwd_adj.argtypes = [_vp] * 8 + [_d, _d] + [_i] * 4 + [_vp] * 6 + [_i, _vp]
lib.pw_advect_fwd_update.argtypes = [_vp] * 5 + [_d, _d] + [_i] * 4 + [_vp] * 3 + [_d] + [_vp] * 3 + [_i, _vp]
lib.pw_halo_periodic.argtypes = [_vp] + [_i] * 5 + [_vp]
lib.pw_pad_periodic.argtypes = [_vp, _vp] + [_i] * 5 + [_vp]
lib.pw_fill_uniform.argtypes = [_vp] + [_i] * 4 + [ctypes.c_ulonglong, _i, _d, _i, _i, _vp]
lib.pw_advect_fwd_host.argtypes = [_vp] * 5 + [_d, _d] + [_i] * 4 + [_vp] * 3 + [_i, _vp, ctypes.c_size_t,
                                                                          _i, _vp]
lib.pw_advect_fwd_host_static.argtypes = [_vp] * 5 + [_d, _d] + [_i] * 4 + [_vp] * 3 + [_i, _i, _vp]
lib.pw_static_scratch_bytes.argtypes = []
lib.pw_static_scratch_bytes.restype = ctypes.c_size_t
lib.pw_offload_workspace_bytes.argtypes = [_i] * 6
lib.pw_offload_workspace_bytes.restype = ctypes.c_size_t
lib.pw_set_kernel.argtypes = [_i]
lib.pw_set_tuning.argtypes = [_i, _i]
lib.pw_get_tuning.argtypes = [_i, ctypes.POINTER(_i)]
lib.pw_stream_copy.argtypes = [_vp, _vp, _i, ctypes.c_size_t, _i, _i, _i, _vp]
lib.pw_last_error.restype = ctypes.c_char_p
for _f in ("pw_advect_fwd", "pw_advect_adj", "pw_advect_fwd_adj", "pw_advect_fwd_host", "pw_advect_fwd_update",
           "pw_advect_fwd_host_static",
           "pw_halo_periodic", "pw_pad_periodic", "pw_fill_uniform", "pw_stream_copy", "pw_set_kernel",
           "pw_get_kernel", "pw_set_tuning", "pw_get_tuning", "pw_version"):
    getattr(lib, _f).restype = ctypes.c_int


class PWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


def _check(rc):
    if rc != 0:
        raise PWError(rc, lib.pw_last_error().decode())


def _dtype_code(t, compute=None):
    """pw_dtype for storage dtype ``t.dtype`` (a tensor or a torch dtype) and
    arithmetic dtype ``compute`` (None: the storage dtype)."""
    st = t if isinstance(t, torch.dtype) else t.dtype
    compute = st if compute is None else compute
    if st == torch.float64 and compute == torch.float64:
        return PW_F64
    if st == torch.float32 and compute == torch.float32:
        return PW_F32
    if st == torch.float32 and compute == torch.float64:
        return PW_F32_F64
    if st == torch.float16 and compute in (torch.float16, torch.float32):
        return PW_F16      # 16-bit storage is always computed in float
    if st == torch.bfloat16 and compute in (torch.bfloat16, torch.float32):
        return PW_BF16
    raise TypeError("unsupported storage/compute dtypes %s/%s" % (st, compute))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _grid(t, halo):
    if t.dim() != 3:
        raise ValueError("storage tensors are 3-D (x, y, z)")
    return tuple(int(s) - 2 * halo for s in t.shape)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _fields(ref, *ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensors must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if t.shape != ref.shape or t.dtype != ref.dtype:
            raise ValueError("all field tensors need one shape and dtype")


def _profile(t, nz, device):
    t = torch.as_tensor(t, dtype=torch.float64, device=device).contiguous()
    if t.shape != (nz,):
        raise ValueError("tzc1/tzc2 need length nz")
    return t


def _out(ref, t):
    return torch.zeros_like(ref) if t is None else t


def fwd(u, v, w, tzc1, tzc2, tcx, tcy, halo, su=None, sv=None, sw=None, compute=None):
    """Forward source terms; returns (su, sv, sw) storage tensors.
    ``compute=torch.float64`` with float32 fields selects PW_F32_F64."""
    nx, ny, nz = _grid(u, halo)
    su, sv, sw = _out(u, su), _out(u, sv), _out(u, sw)
    _fields(u, v, w, su, sv, sw)
    t1, t2 = _profile(tzc1, nz, u.device), _profile(tzc2, nz, u.device)
    _check(lib.pw_advect_fwd(_ptr(u), _ptr(v), _ptr(w), _ptr(t1), _ptr(t2), float(tcx), float(tcy),
                             nx, ny, nz, halo, _ptr(su), _ptr(sv), _ptr(sw), _dtype_code(u, compute), _stream()))
    return su, sv, sw


def fwd_update(u, v, w, tzc1, tzc2, tcx, tcy, halo, bu, bv, bw, beta, ou=None, ov=None, ow=None,
               compute=None):
    """o = b + beta * s for the forward source terms s (not stored); returns
    (ou, ov, ow).  Pass o as b to accumulate in place, or (u, v, w) as b with
    new o arrays for an Euler step u + dt * su."""
    nx, ny, nz = _grid(u, halo)
    ou, ov, ow = _out(u, ou), _out(u, ov), _out(u, ow)
    _fields(u, v, w, bu, bv, bw, ou, ov, ow)
    t1, t2 = _profile(tzc1, nz, u.device), _profile(tzc2, nz, u.device)
    _check(lib.pw_advect_fwd_update(_ptr(u), _ptr(v), _ptr(w), _ptr(t1), _ptr(t2), float(tcx), float(tcy),
                                    nx, ny, nz, halo, _ptr(bu), _ptr(bv), _ptr(bw), float(beta),
                                    _ptr(ou), _ptr(ov), _ptr(ow), _dtype_code(u, compute), _stream()))
    return ou, ov, ow


def adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, halo, gu=None, gv=None, gw=None, compute=None):
    """Gather-form adjoint; returns (gu, gv, gw) storage tensors."""
    nx, ny, nz = _grid(u, halo)
    gu, gv, gw = _out(u, gu), _out(u, gv), _out(u, gw)
    _fields(u, v, w, lu, lv, lw, gu, gv, gw)
    t1, t2 = _profile(tzc1, nz, u.device), _profile(tzc2, nz, u.device)
    _check(lib.pw_advect_adj(_ptr(u), _ptr(v), _ptr(w), _ptr(lu), _ptr(lv), _ptr(lw), _ptr(t1), _ptr(t2),
                             float(tcx), float(tcy), nx, ny, nz, halo, _ptr(gu), _ptr(gv), _ptr(gw),
                             _dtype_code(u, compute), _stream()))
    return gu, gv, gw


def fwd_adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, halo, out=None, compute=None):
    """Forward and adjoint in one launch; returns (su, sv, sw, gu, gv, gw)."""
    nx, ny, nz = _grid(u, halo)
    out = [None] * 6 if out is None else list(out)
    out = [_out(u, t) for t in out]
    _fields(u, v, w, lu, lv, lw, *out)
    t1, t2 = _profile(tzc1, nz, u.device), _profile(tzc2, nz, u.device)
    _check(lib.pw_advect_fwd_adj(_ptr(u), _ptr(v), _ptr(w), _ptr(lu), _ptr(lv), _ptr(lw), _ptr(t1),
                                 _ptr(t2), float(tcx), float(tcy), nx, ny, nz, halo,
                                 *[_ptr(t) for t in out], _dtype_code(u, compute), _stream()))
    return tuple(out)


def offload_workspace_bytes(shape, halo, dtype, chunk, compute=None):
    """Device workspace bytes that fwd_host needs for storage ``shape``."""
    nx, ny, nz = (int(s) - 2 * halo for s in shape)
    code = _dtype_code(dtype, compute)
    return int(lib.pw_offload_workspace_bytes(nx, ny, nz, halo, code, int(chunk)))


def fwd_host(u, v, w, tzc1, tzc2, tcx, tcy, halo, su, sv, sw, chunk, workspace, compute=None):
    """Forward source terms for host storage tensors (pin them for overlap),
    pipelined in x-slabs of ``chunk`` planes through a device ``workspace``
    tensor; returns (su, sv, sw).  Asynchronous on the current stream."""
    nx, ny, nz = _grid(u, halo)
    for t in (u, v, w, su, sv, sw):
        if t.is_cuda or not t.is_contiguous() or t.shape != u.shape or t.dtype != u.dtype:
            raise ValueError("fwd_host takes contiguous host tensors of one storage shape and dtype")
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    t1, t2 = _profile(tzc1, nz, workspace.device), _profile(tzc2, nz, workspace.device)
    _check(lib.pw_advect_fwd_host(_ptr(u), _ptr(v), _ptr(w), _ptr(t1), _ptr(t2), float(tcx), float(tcy),
                                  nx, ny, nz, halo, _ptr(su), _ptr(sv), _ptr(sw), int(chunk),
                                  _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _dtype_code(u, compute), _stream()))
    return su, sv, sw


def fwd_host_static(u, v, w, tzc1, tzc2, tcx, tcy, halo, su, sv, sw, chunk, compute=None):
    """fwd_host with the library's static scratch in place of a workspace
    (allocates no device memory); tzc1/tzc2 must already be device tensors
    of nz doubles.  Raises PWError (PW_ERR_SIZE) when ``chunk`` needs more
    than static_scratch_bytes()."""
    nx, ny, nz = _grid(u, halo)
    for t in (u, v, w, su, sv, sw):
        if t.is_cuda or not t.is_contiguous() or t.shape != u.shape or t.dtype != u.dtype:
            raise ValueError("fwd_host_static takes contiguous host tensors of one storage shape and dtype")
    for t in (tzc1, tzc2):
        if not (torch.is_tensor(t) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.shape == (nz,)):
            raise ValueError("tzc1/tzc2 must be contiguous float64 device tensors of length nz")
    _check(lib.pw_advect_fwd_host_static(_ptr(u), _ptr(v), _ptr(w), _ptr(tzc1), _ptr(tzc2), float(tcx),
                                         float(tcy), nx, ny, nz, halo, _ptr(su), _ptr(sv), _ptr(sw), int(chunk),
                                         _dtype_code(u, compute), _stream()))
    return su, sv, sw


def static_scratch_bytes():
    return int(lib.pw_static_scratch_bytes())


def halo_periodic(storage, halo):
    """Fill the x/y halo columns of ``storage`` periodically, in place."""
    nx, ny, nz = _grid(storage, halo)
    _fields(storage)
    _check(lib.pw_halo_periodic(_ptr(storage), nx, ny, nz, halo, _dtype_code(storage), _stream()))
    return storage


def pad_periodic(interior, halo, out=None):
    """Storage tensor from a compact interior tensor (periodic x/y halos,
    zero z halo)."""
    if not interior.is_cuda or not interior.is_contiguous() or interior.dim() != 3:
        raise ValueError("interior must be a contiguous 3-D GPU tensor")
    nx, ny, nz = (int(s) for s in interior.shape)
    shape = (nx + 2 * halo, ny + 2 * halo, nz + 2 * halo)
    if out is None:
        out = torch.empty(shape, dtype=interior.dtype, device=interior.device)
    elif tuple(out.shape) != shape or out.dtype != interior.dtype or not out.is_contiguous():
        raise ValueError("out has the wrong shape or dtype")
    _check(lib.pw_pad_periodic(_ptr(interior), _ptr(out), nx, ny, nz, halo, _dtype_code(interior),
                               _stream()))
    return out


def fill_uniform(storage, halo, seed, field_id, amp=10.0, zero_lids=False):
    """Write amp * U[-1, 1) counter-based values into the interior columns of
    ``storage`` (see inputs.py for the definition); halos are not filled."""
    nx, ny, nz = _grid(storage, halo)
    _fields(storage)
    _check(lib.pw_fill_uniform(_ptr(storage), nx, ny, nz, halo, int(seed), int(field_id), float(amp),
                               int(bool(zero_lids)), _dtype_code(storage), _stream()))
    return storage


def alloc_fields(count, shape, dtype, device="cuda:0", align=4096):
    """``count`` contiguous tensors of ``shape`` and ``dtype``, carved as
    views from ONE device allocation, each starting on an ``align``-byte
    boundary (a multiple of 256 bytes).

    This is the layout the library's benchmarks give the arrays of one grid.
    On MI355X at 4096 x 4096 x 64 in FP64, the x-marching forward over twelve
    arrays taken from one allocation ran at 9.20-9.31 ms in each of 24
    placements tried (three allocations, eight spacings between the arrays
    from 0 to 8 MiB), against 9.26-9.95 ms over separately allocated arrays,
    whose time depends on where each allocation lands in HBM.  The views
    share one storage, which is freed with the last of them."""
    count = int(count)
    shape = tuple(int(s) for s in shape)
    if count < 1 or any(s < 0 for s in shape):
        raise ValueError("alloc_fields: count >= 1 and a non-negative shape")
    esize = torch.empty((), dtype=dtype).element_size()
    if align < 256 or align % 256:
        raise ValueError("alloc_fields: align must be a multiple of 256 bytes")
    n = 1
    for s in shape:
        n *= s
    step = -(-n * esize // align) * align // esize      # elements from one start to the next
    buf = torch.empty(step * (count - 1) + n + align // esize, dtype=dtype, device=device)
    off = (-buf.data_ptr() % align) // esize
    return [buf[off + q * step: off + q * step + n].view(shape) for q in range(count)]


def stream_copy(src, dst, blocks=0, unit=4, hints=0):
    """One launch of the library's plain streaming copy: dst[q] <- src[q] for
    lists of equally sized contiguous device tensors (the bandwidth reference
    of the advection kernels), in ``unit``-byte units (4, 8 or 16).
    ``blocks`` = 0: one unit per thread and array; > 0: that many workgroups
    striding over the arrays.  ``hints``: 0 or an OR of COPY_NT_LOADS and
    COPY_NT_STORES (non-temporal cache policy on the loads / stores)."""
    if len(src) != len(dst) or not 1 <= len(src) <= 8:
        raise ValueError("1..8 source and destination tensors")
    nbytes = src[0].numel() * src[0].element_size()
    for t in list(src) + list(dst):
        if not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() != nbytes:
            raise ValueError("stream_copy takes contiguous device tensors of one byte size")
    n = len(src)
    sp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in src])
    dp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in dst])
    _check(lib.pw_stream_copy(ctypes.cast(sp, _vp), ctypes.cast(dp, _vp), n, nbytes, int(unit), int(blocks),
                              int(hints), _stream()))


def get_tuning(knob):
    """Current value of tuning knob ``knob`` (TUNE_*) of the calling thread."""
    v = _i(0)
    _check(lib.pw_get_tuning(int(knob), ctypes.byref(v)))
    return v.value


def set_tuning(knob, value):
    """Set tuning knob ``knob`` (TUNE_*) of the calling thread; returns the
    previous value.  No knob changes a result."""
    prev = get_tuning(knob)
    _check(lib.pw_set_tuning(int(knob), int(value)))
    return prev


class tuning:
    """Context manager: set tuning knobs of the calling thread for a block
    and restore them afterwards, e.g. ``with pw.tuning(variant=3, lx=7):``.
    Keywords: kernel ('auto', 'direct', 'march'), variant (-1..7), lx (planes
    per marching workgroup, 0 = automatic), copy_out ('runtime', 'kernel', 'direct', 'auto'),
    order ('default', 'xcd', 'natural', or an int G: groups of G neighbouring
    strips per XCD), tall_waves (wavefronts per column of the tall variant,
    2..4, 0 = automatic)."""

    def __init__(self, kernel=None, variant=None, lx=None, copy_out=None, order=None, tall_waves=None):
        self.want = []
        if kernel is not None:
            self.want.append((TUNE_KERNEL, KERNELS[kernel]))
        if variant is not None:
            self.want.append((TUNE_MARCH_VARIANT, int(variant)))
        if lx is not None:
            self.want.append((TUNE_MARCH_LX, int(lx)))
        if copy_out is not None:
            self.want.append((TUNE_COPY_OUT, COPY_OUT[copy_out]))
        if order is not None:
            self.want.append((TUNE_BLOCK_ORDER, ORDERS[order] if isinstance(order, str) else int(order)))
        if tall_waves is not None:
            self.want.append((TUNE_TALL_WAVES, int(tall_waves)))
        self.saved = []

    def __enter__(self):
        for knob, value in self.want:
            self.saved.append((knob, set_tuning(knob, value)))
        return self

    def __exit__(self, *exc):
        for knob, value in reversed(self.saved):
            set_tuning(knob, value)
        self.saved = []
        return False


def set_kernel(name):
    """Select 'auto', 'direct' or 'march' for the calling thread; returns the
    previous selection."""
    prev = lib.pw_set_kernel(KERNELS[name])
    _check(min(prev, 0))
    return {v: k for k, v in KERNELS.items()}[prev]


def get_kernel():
    return {v: k for k, v in KERNELS.items()}[lib.pw_get_kernel()]


def version():
    return lib.pw_version()
