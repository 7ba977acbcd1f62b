// pw_abi.hip -- the extern "C" entry points of libpwadvect: argument
// validation (all of it before any work is queued), kernel selection and
// launch-error reporting.  See include/pwadvect.h for the contract.
#include <climits>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/pwadvect.h"
#include "pw_half.h"
#include "pw_internal.h"

namespace {

thread_local char g_err[512] = "";

// Tuning state of the calling thread (pw_set_tuning): read by the calls that
// thread makes, so threads never see each other's settings.
struct Tuning {
    int kernel = PW_KERNEL_AUTO;
    int variant = -1;                 // < 0: default variant
    int lx = 0;                       // 0: segment length from the grid
    int copy_out = PW_COPY_OUT_AUTO;
    int order = -1;                   // < 0: default block order, 0: XCD ranges, G: groups of G
    int tall_waves = 0;               // 0: wavefronts per tall column chosen from nz
};
thread_local Tuning g_tune;

MarchTune march_tune() { return MarchTune{g_tune.variant, g_tune.lx, g_tune.order, g_tune.tall_waves}; }

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int ok()
{
    g_err[0] = '\0';
    return PW_OK;
}

size_t elem_size(int dtype)
{
    return dtype == PW_F64 ? 8 : (dtype == PW_F16 || dtype == PW_BF16) ? 2 : 4;
}

// Calls f(T{}, C{}) with the storage type T and arithmetic type C of dtype
// (which check_shape has validated).
template <typename F>
int with_types(int dtype, F&& f)
{
    switch (dtype) {
    case PW_F64: return f(double{}, double{});
    case PW_F32_F64: return f(float{}, double{});
    case PW_F16: return f(_Float16{}, float{});
    case PW_BF16: return f(bf16_t{}, float{});
    default: return f(float{}, float{});
    }
}

// Shape checks shared by every entry point; fills g and the byte count of
// one storage array.
int check_shape(int nx, int ny, int nz, int halo, int dtype, Geom& g, size_t& bytes)
{
    if (dtype != PW_F64 && dtype != PW_F32 && dtype != PW_F32_F64 && dtype != PW_F16 && dtype != PW_BF16)
        return fail(PW_ERR_ARG, "unknown dtype %d", dtype);
    if (nx < 1 || ny < 1) return fail(PW_ERR_ARG, "nx=%d, ny=%d: need nx >= 1 and ny >= 1", nx, ny);
    if (nz < 2) return fail(PW_ERR_ARG, "nz=%d: need nz >= 2", nz);
    if (halo < 1) return fail(PW_ERR_ARG, "halo=%d: need halo >= 1", halo);
    const long long Sx = (long long)nx + 2LL * halo;
    const long long Sy = (long long)ny + 2LL * halo;
    const long long Sz = (long long)nz + 2LL * halo;
    if (Sx > INT_MAX || Sy > INT_MAX || Sz > INT_MAX)
        return fail(PW_ERR_SIZE, "n + 2*halo overflows int");
    // per-plane thread index of the kernels is a 32-bit int
    if (Sy * Sz > (long long)INT_MAX - 1024)
        return fail(PW_ERR_SIZE, "(ny+2h)*(nz+2h) = %lld exceeds the per-plane limit", Sy * Sz);
    const long long es = (long long)elem_size(dtype);
    if (Sx > LLONG_MAX / Sy || Sx * Sy > LLONG_MAX / Sz || Sx * Sy * Sz > LLONG_MAX / es)
        return fail(PW_ERR_SIZE, "storage byte count overflows int64");
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.h = halo;
    g.Sx = (int)Sx;
    g.Sy = (int)Sy;
    g.Sz = (int)Sz;
    g.sy = (int)Sz;
    g.sx = Sy * Sz;
    bytes = (size_t)(Sx * Sy * Sz * es);
    return PW_OK;
}

struct Arr {
    const void* p;
    size_t bytes;
    size_t align;
    const char* name;
};

int check_host_side(const Arr* in, int nin, const Arr* out, int nout)
{
    for (int q = 0; q < nin + nout; q++) {
        const Arr& a = q < nin ? in[q] : out[q - nin];
        if (!a.p) return fail(PW_ERR_ARG, "%s is NULL", a.name);
        if ((uintptr_t)a.p % a.align) return fail(PW_ERR_ALIGN, "%s is not %zu-byte aligned", a.name, a.align);
    }
    for (int o = 0; o < nout; o++) {
        const uintptr_t ob = (uintptr_t)out[o].p, oe = ob + out[o].bytes;
        for (int q = 0; q < nin + nout; q++) {
            if (q == nin + o) continue;
            const Arr& a = q < nin ? in[q] : out[q - nin];
            const uintptr_t ab = (uintptr_t)a.p, ae = ab + a.bytes;
            if (ob < ae && ab < oe)
                return fail(PW_ERR_ALIAS, "output %s overlaps %s", out[o].name, a.name);
        }
    }
    return PW_OK;
}

// Device-pointer and allocation-extent checks (host queries, no GPU work).
// Device address of a pinned host array that is mapped into the current
// device's address space and lies wholly inside one allocation; nullptr
// otherwise (pageable memory, unknown extent).
void* mapped_host(const void* p, size_t bytes)
{
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (attr.type != hipMemoryTypeHost || !attr.devicePointer) return nullptr;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)attr.devicePointer) != hipSuccess || size == 0) {
        (void)hipGetLastError();
        return nullptr;
    }
    const uintptr_t b = (uintptr_t)base, d = (uintptr_t)attr.devicePointer;
    if (d < b || d + bytes > b + size) return nullptr;
    return attr.devicePointer;
}

// Host arrays of pw_advect_fwd_host: pageable or pinned host memory, never
// device memory (the copies are issued as host<->device transfers).
int check_host_memory(const Arr* arrs, int n)
{
    for (int q = 0; q < n; q++) {
        hipPointerAttribute_t attr;
        std::memset(&attr, 0, sizeof attr);
        if (hipPointerGetAttributes(&attr, arrs[q].p) != hipSuccess) {
            (void)hipGetLastError();   // unknown to the runtime: pageable host memory
            continue;
        }
        if (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeArray)
            return fail(PW_ERR_ARG, "%s is device memory; pw_advect_fwd_host takes host arrays", arrs[q].name);
    }
    return PW_OK;
}

int check_device(const Arr* arrs, int n)
{
    for (int q = 0; q < n; q++) {
        const Arr& a = arrs[q];
        hipPointerAttribute_t attr;
        std::memset(&attr, 0, sizeof attr);
        if (hipPointerGetAttributes(&attr, a.p) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PW_ERR_ARG, "%s is not a device pointer", a.name);
        }
        if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
            return fail(PW_ERR_ARG, "%s is not device memory", a.name);
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)a.p) == hipSuccess && size > 0) {
            const uintptr_t b = (uintptr_t)base, p = (uintptr_t)a.p;
            if (p < b || p + a.bytes > b + size)
                return fail(PW_ERR_ARG, "%s (%zu bytes) does not fit inside its device allocation",
                            a.name, a.bytes);
        } else {
            (void)hipGetLastError();
        }
    }
    return PW_OK;
}

int launched(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

// Resolve the kernel family for a shape; -1 if the selection cannot run it.
template <typename T>
int resolve_kernel(const Geom& g, const Arr* arrs, int n)
{
    const int sel = g_tune.kernel;
    if (sel == PW_KERNEL_DIRECT) return PW_KERNEL_DIRECT;
    bool march = march_supported<T>(g);
    for (int q = 0; q < n && march; q++)
        if ((uintptr_t)arrs[q].p % 16) march = false;
    if (sel == PW_KERNEL_MARCH) return march ? PW_KERNEL_MARCH : -1;
    return march ? PW_KERNEL_MARCH : PW_KERNEL_DIRECT;
}

// base == nullptr: plain forward.  Otherwise the update form o = b + beta * s
// (pw_advect_fwd_update): b[q] is o[q] itself, or an array that overlaps no
// output; b == (u, v, w) selects the kernels' field-reuse mode.
template <typename T, typename C>
int do_fwd(const void* u, const void* v, const void* w, const double* tzc1, const double* tzc2,
           double tcx, double tcy, const Geom& g, size_t bytes, void* su, void* sv, void* sw,
           hipStream_t stream, const void* const* base = nullptr, double beta = 0.0)
{
    const Arr in[5] = {{u, bytes, sizeof(T), "u"}, {v, bytes, sizeof(T), "v"}, {w, bytes, sizeof(T), "w"},
                       {tzc1, (size_t)g.nz * 8, 8, "tzc1"}, {tzc2, (size_t)g.nz * 8, 8, "tzc2"}};
    const Arr out[3] = {{su, bytes, sizeof(T), "su"}, {sv, bytes, sizeof(T), "sv"}, {sw, bytes, sizeof(T), "sw"}};
    int rc = check_host_side(in, 5, out, 3);
    if (rc) return rc;
    static const char* const names[3] = {"bu", "bv", "bw"};
    Arr ba[3];
    if (base) {   // host-side checks of the base arrays before any device query
        for (int q = 0; q < 3; q++) ba[q] = Arr{base[q], bytes, sizeof(T), names[q]};
        rc = check_host_side(ba, 3, nullptr, 0);
        if (rc) return rc;
        for (int q = 0; q < 3; q++) {
            if (base[q] == out[q].p) continue;   // accumulate in place
            const uintptr_t bb = (uintptr_t)base[q], be = bb + bytes;
            for (int o = 0; o < 3; o++) {
                const uintptr_t ob = (uintptr_t)out[o].p, oe = ob + bytes;
                if (bb < oe && ob < be)
                    return fail(PW_ERR_ALIAS, "%s overlaps output %s (only %s itself may be passed as %s)",
                                names[q], out[o].name, out[q].name, names[q]);
            }
        }
    }
    const Arr all[8] = {in[0], in[1], in[2], in[3], in[4], out[0], out[1], out[2]};
    rc = check_device(all, 8);
    if (rc) return rc;
    Arr fields[9] = {in[0], in[1], in[2], out[0], out[1], out[2]};
    int nf = 6;
    int upd = 0;
    if (base) {
        rc = check_device(ba, 3);
        if (rc) return rc;
        upd = (base[0] == u && base[1] == v && base[2] == w) ? 2 : 1;
        if (upd == 1)
            for (int q = 0; q < 3; q++) fields[nf++] = ba[q];
    }
    const int kern = resolve_kernel<T>(g, fields, nf);
    if (kern < 0)
        return fail(PW_ERR_UNSUPPORTED,
                    "x-marching kernel needs halo <= 32, columns under 1 GiB and 16-byte aligned arrays");
    FwdArgs<T> a{(const T*)u, (const T*)v, (const T*)w, tzc1, tzc2, tcx, tcy, (T*)su, (T*)sv, (T*)sw, upd,
                 {nullptr, nullptr, nullptr}, beta};
    if (base)
        for (int q = 0; q < 3; q++) a.b[q] = (const T*)base[q];
    (void)hipGetLastError();
    if (kern == PW_KERNEL_MARCH)
        launch_fwd_march<T, C>(a, g, march_tune(), stream);
    else
        launch_fwd_direct<T, C>(a, g, stream);
    return launched(base ? "pw_advect_fwd_update" : "pw_advect_fwd");
}

template <typename T, typename C>
int do_adj(const void* u, const void* v, const void* w, const void* lu, const void* lv, const void* lw,
           const double* tzc1, const double* tzc2, double tcx, double tcy, const Geom& g, size_t bytes,
           void* su, void* sv, void* sw, void* gu, void* gv, void* gw, hipStream_t stream)
{
    const size_t es = sizeof(T);
    const Arr in[8] = {{u, bytes, es, "u"},   {v, bytes, es, "v"},   {w, bytes, es, "w"},
                       {lu, bytes, es, "lu"}, {lv, bytes, es, "lv"}, {lw, bytes, es, "lw"},
                       {tzc1, (size_t)g.nz * 8, 8, "tzc1"}, {tzc2, (size_t)g.nz * 8, 8, "tzc2"}};
    const bool fused = su != nullptr || sv != nullptr || sw != nullptr;
    Arr out[6];
    int nout = 0;
    if (fused) {
        out[nout++] = {su, bytes, es, "su"};
        out[nout++] = {sv, bytes, es, "sv"};
        out[nout++] = {sw, bytes, es, "sw"};
    }
    out[nout++] = {gu, bytes, es, "gu"};
    out[nout++] = {gv, bytes, es, "gv"};
    out[nout++] = {gw, bytes, es, "gw"};
    int rc = check_host_side(in, 8, out, nout);
    if (rc) return rc;
    Arr all[14];
    int n = 0;
    for (int q = 0; q < 8; q++) all[n++] = in[q];
    for (int q = 0; q < nout; q++) all[n++] = out[q];
    rc = check_device(all, n);
    if (rc) return rc;
    Arr fields[12];
    int nf = 0;
    for (int q = 0; q < 6; q++) fields[nf++] = in[q];
    for (int q = 0; q < nout; q++) fields[nf++] = out[q];
    const int kern = resolve_kernel<T>(g, fields, nf);
    if (kern < 0)
        return fail(PW_ERR_UNSUPPORTED,
                    "x-marching kernel needs halo <= 32, columns under 1 GiB and 16-byte aligned arrays");
    AdjArgs<T> a{(const T*)u, (const T*)v, (const T*)w, (const T*)lu, (const T*)lv, (const T*)lw,
                 tzc1, tzc2, tcx, tcy, (T*)su, (T*)sv, (T*)sw, (T*)gu, (T*)gv, (T*)gw};
    (void)hipGetLastError();
    if (kern == PW_KERNEL_MARCH)
        launch_adj_march<T, C>(a, g, march_tune(), stream);
    else
        launch_adj_direct<T, C>(a, g, stream);
    return launched(fused ? "pw_advect_fwd_adj" : "pw_advect_adj");
}

int check_one(const void* p, size_t bytes, size_t align, const char* name)
{
    const Arr a[1] = {{p, bytes, align, name}};
    int rc = check_host_side(a, 1, nullptr, 0);
    if (rc) return rc;
    return check_device(a, 1);
}

// pw_advect_fwd_host and its allocation-free variant: the slab buffers are
// the caller's workspace, or (use_static) the library's static scratch, whose
// calls are then ordered one after another on the device.
int do_fwd_host(const char* name, const void* u, const void* v, const void* w, const double* tzc1,
                const double* tzc2, double tcx, double tcy, int nx, int ny, int nz, int halo, void* su, void* sv,
                void* sw, int chunk, void* workspace, size_t workspace_bytes, bool use_static, int dtype,
                void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    if (chunk < 1) return fail(PW_ERR_ARG, "chunk=%d: need chunk >= 1", chunk);
    if (chunk > nx) chunk = nx;
    const size_t es = elem_size(dtype);
    const size_t need = offload_workspace_bytes(g, chunk, es);
    if (use_static) {
        if (need > kStaticScratchBytes)
            return fail(PW_ERR_SIZE, "%s: chunk %d needs %zu bytes of scratch; the static scratch holds %zu", name,
                        chunk, need, kStaticScratchBytes);
    } else {
        if (!workspace) return fail(PW_ERR_ARG, "workspace is NULL");
        if (workspace_bytes < need)
            return fail(PW_ERR_SIZE, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes,
                        need);
    }
    const Arr in[3] = {{u, bytes, es, "u"}, {v, bytes, es, "v"}, {w, bytes, es, "w"}};
    const Arr out[3] = {{su, bytes, es, "su"}, {sv, bytes, es, "sv"}, {sw, bytes, es, "sw"}};
    rc = check_host_side(in, 3, out, 3);
    if (rc) return rc;
    const Arr host[6] = {in[0], in[1], in[2], out[0], out[1], out[2]};
    rc = check_host_memory(host, 6);
    if (rc) return rc;
    const Arr dev[3] = {{tzc1, (size_t)nz * 8, 8, "tzc1"}, {tzc2, (size_t)nz * 8, 8, "tzc2"},
                        {workspace, need, 16, "workspace"}};
    const int ndev = use_static ? 2 : 3;
    rc = check_host_side(dev, ndev, nullptr, 0);
    if (rc) return rc;
    rc = check_device(dev, ndev);
    if (rc) return rc;
    if (use_static) {
        const hipError_t e = static_scratch_for_current_device(&workspace);
        if (e != hipSuccess)
            return fail(PW_ERR_HIP, "%s: looking up the static scratch: %s", name, hipGetErrorString(e));
    }
    // the slab kernels follow the same selection as pw_advect_fwd
    Geom sg = g;
    sg.nx = chunk;
    const Arr ws[1] = {{workspace, need, 16, "workspace"}};
    const int kern = with_types(dtype, [&](auto t, auto) { return resolve_kernel<decltype(t)>(sg, ws, 1); });
    if (kern < 0) return fail(PW_ERR_UNSUPPORTED, "x-marching kernel needs halo <= 32 and columns under 1 GiB");
    // outputs go back through the runtime's copies unless the copy-out mode
    // (the thread's, or the automatic choice) is the copy kernel or direct
    // writes and they are pinned host memory mapped into the device's address
    // space; direct writes from the x-marching kernels also need every slab's
    // first plane 16-byte aligned
    void* od[3] = {nullptr, nullptr, nullptr};
    const int mode = g_tune.copy_out;
    bool mapped = mode != PW_COPY_OUT_RUNTIME;
    for (int f = 0; f < 3 && mapped; ++f) mapped = (od[f] = mapped_host(out[f].p, bytes)) != nullptr;
    const char* what = "";
    const bool march = kern == PW_KERNEL_MARCH;
    bool direct_ok = mapped;
    if (direct_ok && march) {
        const size_t plane_bytes = (size_t)g.sx * es;
        for (int f = 0; f < 3; ++f)
            if ((uintptr_t)od[f] % 16 || plane_bytes % 16) direct_ok = false;
    }
    const int e = with_types(dtype, [&](auto t, auto c) {
        using T = decltype(t);
        T* const o[3] = {(T*)od[0], (T*)od[1], (T*)od[2]};
        return offload_fwd<T, decltype(c)>((const T*)u, (const T*)v, (const T*)w, tzc1, tzc2, tcx, tcy, g, (T*)su,
                                           (T*)sv, (T*)sw, mapped ? o : nullptr, direct_ok, mode, chunk, workspace,
                                           march, use_static, march_tune(), (hipStream_t)stream, &what);
    });
    if (e) return fail(PW_ERR_HIP, "%s: %s: %s", name, what, hipGetErrorString((hipError_t)e));
    return launched(name);
}

}  // namespace

extern "C" {

int pw_advect_fwd(const void* u, const void* v, const void* w, const double* tzc1, const double* tzc2,
                  double tcx, double tcy, int nx, int ny, int nz, int halo, void* su, void* sv, void* sw,
                  int dtype, void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    return with_types(dtype, [&](auto t, auto c) {
        return do_fwd<decltype(t), decltype(c)>(u, v, w, tzc1, tzc2, tcx, tcy, g, bytes, su, sv, sw,
                                                (hipStream_t)stream);
    });
}

int pw_advect_fwd_update(const void* u, const void* v, const void* w, const double* tzc1, const double* tzc2,
                         double tcx, double tcy, int nx, int ny, int nz, int halo, const void* bu,
                         const void* bv, const void* bw, double beta, void* ou, void* ov, void* ow, int dtype,
                         void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    const void* const base[3] = {bu, bv, bw};
    return with_types(dtype, [&](auto t, auto c) {
        return do_fwd<decltype(t), decltype(c)>(u, v, w, tzc1, tzc2, tcx, tcy, g, bytes, ou, ov, ow,
                                                (hipStream_t)stream, base, beta);
    });
}

int pw_advect_adj(const void* u, const void* v, const void* w, const void* lu, const void* lv,
                  const void* lw, const double* tzc1, const double* tzc2, double tcx, double tcy, int nx,
                  int ny, int nz, int halo, void* gu, void* gv, void* gw, int dtype, void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    if (!gu || !gv || !gw) return fail(PW_ERR_ARG, "gu, gv, gw must not be NULL");
    return with_types(dtype, [&](auto t, auto c) {
        return do_adj<decltype(t), decltype(c)>(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, g, bytes, nullptr,
                                                nullptr, nullptr, gu, gv, gw, (hipStream_t)stream);
    });
}

int pw_advect_fwd_adj(const void* u, const void* v, const void* w, const void* lu, const void* lv,
                      const void* lw, const double* tzc1, const double* tzc2, double tcx, double tcy,
                      int nx, int ny, int nz, int halo, void* su, void* sv, void* sw, void* gu, void* gv,
                      void* gw, int dtype, void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    if (!su || !sv || !sw) return fail(PW_ERR_ARG, "su, sv, sw must not be NULL");
    if (!gu || !gv || !gw) return fail(PW_ERR_ARG, "gu, gv, gw must not be NULL");
    return with_types(dtype, [&](auto t, auto c) {
        return do_adj<decltype(t), decltype(c)>(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, g, bytes, su, sv, sw,
                                                gu, gv, gw, (hipStream_t)stream);
    });
}

size_t pw_offload_workspace_bytes(int nx, int ny, int nz, int halo, int dtype, int chunk)
{
    Geom g;
    size_t bytes;
    if (check_shape(nx, ny, nz, halo, dtype, g, bytes)) return 0;
    if (chunk < 1) return 0;
    if (chunk > nx) chunk = nx;
    return offload_workspace_bytes(g, chunk, elem_size(dtype));
}

int pw_advect_fwd_host(const void* u, const void* v, const void* w, const double* tzc1, const double* tzc2,
                       double tcx, double tcy, int nx, int ny, int nz, int halo, void* su, void* sv, void* sw,
                       int chunk, void* workspace, size_t workspace_bytes, int dtype, void* stream)
{
    return do_fwd_host("pw_advect_fwd_host", u, v, w, tzc1, tzc2, tcx, tcy, nx, ny, nz, halo, su, sv, sw, chunk,
                       workspace, workspace_bytes, false, dtype, stream);
}

size_t pw_static_scratch_bytes(void) { return kStaticScratchBytes; }

int pw_advect_fwd_host_static(const void* u, const void* v, const void* w, const double* tzc1,
                              const double* tzc2, double tcx, double tcy, int nx, int ny, int nz, int halo,
                              void* su, void* sv, void* sw, int chunk, int dtype, void* stream)
{
    return do_fwd_host("pw_advect_fwd_host_static", u, v, w, tzc1, tzc2, tcx, tcy, nx, ny, nz, halo, su, sv, sw,
                       chunk, nullptr, 0, true, dtype, stream);
}

int pw_halo_periodic(void* storage, int nx, int ny, int nz, int halo, int dtype, void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    rc = check_one(storage, bytes, elem_size(dtype), "storage");
    if (rc) return rc;
    (void)hipGetLastError();
    with_types(dtype, [&](auto t, auto) {
        launch_halo_periodic<decltype(t)>((decltype(t)*)storage, g, (hipStream_t)stream);
        return 0;
    });
    return launched("pw_halo_periodic");
}

int pw_pad_periodic(const void* interior, void* storage, int nx, int ny, int nz, int halo, int dtype,
                    void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    const size_t es = elem_size(dtype);
    const Arr in[1] = {{interior, (size_t)nx * (size_t)ny * (size_t)nz * es, es, "interior"}};
    const Arr out[1] = {{storage, bytes, es, "storage"}};
    rc = check_host_side(in, 1, out, 1);
    if (rc) return rc;
    const Arr all[2] = {in[0], out[0]};
    rc = check_device(all, 2);
    if (rc) return rc;
    (void)hipGetLastError();
    with_types(dtype, [&](auto t, auto) {
        using T = decltype(t);
        launch_pad_periodic<T>((const T*)interior, (T*)storage, g, (hipStream_t)stream);
        return 0;
    });
    return launched("pw_pad_periodic");
}

int pw_fill_uniform(void* storage, int nx, int ny, int nz, int halo, unsigned long long seed, int field_id,
                    double amp, int zero_lids, int dtype, void* stream)
{
    Geom g;
    size_t bytes;
    int rc = check_shape(nx, ny, nz, halo, dtype, g, bytes);
    if (rc) return rc;
    if (field_id < 0 || field_id > 255) return fail(PW_ERR_ARG, "field_id=%d outside 0..255", field_id);
    rc = check_one(storage, bytes, elem_size(dtype), "storage");
    if (rc) return rc;
    (void)hipGetLastError();
    with_types(dtype, [&](auto t, auto) {
        launch_fill_uniform<decltype(t)>((decltype(t)*)storage, g, seed, field_id, amp, zero_lids,
                                         (hipStream_t)stream);
        return 0;
    });
    return launched("pw_fill_uniform");
}

int pw_stream_copy(const void* const* src, void* const* dst, int narrays, size_t bytes, int unit, int blocks,
                   int hints, void* stream)
{
    if (!src || !dst) return fail(PW_ERR_ARG, "src and dst must not be NULL");
    if (narrays < 1 || narrays > 8) return fail(PW_ERR_ARG, "narrays=%d outside 1..8", narrays);
    if (unit != 4 && unit != 8 && unit != 16) return fail(PW_ERR_ARG, "unit=%d: need 4, 8 or 16", unit);
    if (bytes % (size_t)unit) return fail(PW_ERR_ARG, "bytes=%zu is not a multiple of the unit %d", bytes, unit);
    if (blocks < 0) return fail(PW_ERR_ARG, "blocks=%d: need 0 or more", blocks);
    if (hints & ~(PW_COPY_NT_LOADS | PW_COPY_NT_STORES))
        return fail(PW_ERR_ARG, "hints=%d: need an OR of PW_COPY_NT_LOADS and PW_COPY_NT_STORES", hints);
    // one pass: one thread per unit, and the grid's thread count must fit 32 bits
    if (blocks == 0 && bytes / (size_t)unit > 0xffffff00ULL)
        return fail(PW_ERR_SIZE, "one pass over %zu bytes in %d-byte units needs 2^32 threads or more", bytes, unit);
    static const char* const sn[8] = {"src[0]", "src[1]", "src[2]", "src[3]", "src[4]", "src[5]", "src[6]", "src[7]"};
    static const char* const dn[8] = {"dst[0]", "dst[1]", "dst[2]", "dst[3]", "dst[4]", "dst[5]", "dst[6]", "dst[7]"};
    Arr in[8], out[8];
    for (int q = 0; q < narrays; ++q) {
        in[q] = Arr{src[q], bytes, (size_t)unit, sn[q]};
        out[q] = Arr{dst[q], bytes, (size_t)unit, dn[q]};
    }
    int rc = check_host_side(in, narrays, out, narrays);
    if (rc) return rc;
    Arr all[16];
    for (int q = 0; q < narrays; ++q) {
        all[q] = in[q];
        all[narrays + q] = out[q];
    }
    rc = check_device(all, 2 * narrays);
    if (rc) return rc;
    (void)hipGetLastError();
    launch_stream_copy(src, dst, narrays, bytes, unit, blocks, hints, (hipStream_t)stream);
    return launched("pw_stream_copy");
}

int pw_set_tuning(int knob, int value)
{
    switch (knob) {
    case PW_TUNE_KERNEL:
        if (value != PW_KERNEL_AUTO && value != PW_KERNEL_DIRECT && value != PW_KERNEL_MARCH)
            return fail(PW_ERR_ARG, "unknown kernel selection %d", value);
        g_tune.kernel = value;
        break;
    case PW_TUNE_MARCH_VARIANT:
        if (value < -1 || value >= PW_MARCH_VARIANTS)
            return fail(PW_ERR_ARG, "march variant %d outside -1..%d", value, PW_MARCH_VARIANTS - 1);
        g_tune.variant = value;
        break;
    case PW_TUNE_MARCH_LX:
        if (value < 0) return fail(PW_ERR_ARG, "segment length %d: need 0 (automatic) or more", value);
        g_tune.lx = value;
        break;
    case PW_TUNE_COPY_OUT:
        if (value != PW_COPY_OUT_RUNTIME && value != PW_COPY_OUT_KERNEL && value != PW_COPY_OUT_DIRECT &&
            value != PW_COPY_OUT_AUTO)
            return fail(PW_ERR_ARG, "unknown copy-out mode %d", value);
        g_tune.copy_out = value;
        break;
    case PW_TUNE_BLOCK_ORDER:
        if (value < -1 || value > PW_ORDER_MAX_GROUP)
            return fail(PW_ERR_ARG, "block order %d outside -1..%d", value, PW_ORDER_MAX_GROUP);
        g_tune.order = value;
        break;
    case PW_TUNE_TALL_WAVES:
        if (value != 0 && (value < 2 || value > 4))
            return fail(PW_ERR_ARG, "wavefronts per tall column %d: need 0 (automatic) or 2..4", value);
        g_tune.tall_waves = value;
        break;
    default:
        return fail(PW_ERR_ARG, "unknown tuning knob %d", knob);
    }
    return ok();
}

int pw_get_tuning(int knob, int* value)
{
    if (!value) return fail(PW_ERR_ARG, "value is NULL");
    switch (knob) {
    case PW_TUNE_KERNEL: *value = g_tune.kernel; break;
    case PW_TUNE_MARCH_VARIANT: *value = g_tune.variant; break;
    case PW_TUNE_MARCH_LX: *value = g_tune.lx; break;
    case PW_TUNE_COPY_OUT: *value = g_tune.copy_out; break;
    case PW_TUNE_BLOCK_ORDER: *value = g_tune.order; break;
    case PW_TUNE_TALL_WAVES: *value = g_tune.tall_waves; break;
    default: return fail(PW_ERR_ARG, "unknown tuning knob %d", knob);
    }
    return ok();
}

int pw_set_kernel(int kernel)
{
    const int prev = g_tune.kernel;
    const int rc = pw_set_tuning(PW_TUNE_KERNEL, kernel);
    return rc ? rc : prev;
}

int pw_get_kernel(void) { return g_tune.kernel; }

const char* pw_last_error(void) { return g_err; }

int pw_version(void) { return 200; }

}  // extern "C"
