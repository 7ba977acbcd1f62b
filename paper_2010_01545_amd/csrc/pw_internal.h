// pw_internal.h -- declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

// Geometry of one storage array: interior (nx, ny, nz), halo h, strides in
// elements of the x planes (sx) and y columns (sy = Sz).
struct Geom {
    int nx, ny, nz, h;
    int Sx, Sy, Sz;   // storage extents
    long long sx;     // Sy * Sz
    int sy;           // Sz
};

// Operand bundles passed to the kernel launchers.  T is the storage type;
// the kernels are also templated on the arithmetic type C (C = T, or
// T = float with C = double), and round tcx, tcy and the profiles to C.
// With `upd` != 0 the forward stores o = b + beta * s instead of s (b[q] is a
// base array, possibly the output itself; upd == 2 means b is (u, v, w) and
// the kernels reuse the values they read).
template <typename T>
struct FwdArgs {
    const T *u, *v, *w;
    const double *tzc1, *tzc2;
    double tcx, tcy;
    T *su, *sv, *sw;
    int upd;
    const T* b[3];
    double beta;
};

template <typename T>
struct AdjArgs {
    const T *u, *v, *w, *lu, *lv, *lw;
    const double *tzc1, *tzc2;
    double tcx, tcy;
    T *su, *sv, *sw;   // forward outputs (fused launch only; null otherwise)
    T *gu, *gv, *gw;
};

// Direct kernels: one thread per storage level of each interior column,
// every operand read from global memory.  Any nz >= 2, any halo >= 1.
template <typename T, typename C> void launch_fwd_direct(const FwdArgs<T>& a, const Geom& g, hipStream_t s);
template <typename T, typename C> void launch_adj_direct(const AdjArgs<T>& a, const Geom& g, hipStream_t s);

// x-marching kernels (any nz >= 2, halo <= 32, 16-byte aligned arrays,
// columns shorter than 1 GiB).  MarchTune carries the calling thread's
// choice of variant (< 0: the default for the type pair and output set),
// segment length in planes (0: chosen from the grid) and block order (< 0:
// the default; 0: XCD ranges; 1: natural) and wavefronts per column of the
// tall variant (0: chosen from nz).
struct MarchTune {
    int variant;
    int lx;
    int order;
    int tall_waves;
};
template <typename T> bool march_supported(const Geom& g);
template <typename T, typename C>
void launch_fwd_march(const FwdArgs<T>& a, const Geom& g, MarchTune t, hipStream_t s);
template <typename T, typename C>
void launch_adj_march(const AdjArgs<T>& a, const Geom& g, MarchTune t, hipStream_t s);

// Utilities.
template <typename T> void launch_halo_periodic(T* st, const Geom& g, hipStream_t s);
template <typename T> void launch_pad_periodic(const T* in, T* st, const Geom& g, hipStream_t s);
template <typename T> void launch_fill_uniform(T* st, const Geom& g, unsigned long long seed,
                                               int field_id, double amp, int zero_lids,
                                               hipStream_t s);

// Plain streaming copy of n arrays in units of 4, 8 or 16 bytes, with
// optional non-temporal loads/stores (pw_copyref.hip), the bandwidth
// reference.
void launch_stream_copy(const void* const* src, void* const* dst, int n, size_t bytes, int unit, int blocks,
                        int hints, hipStream_t s);

// Host-resident fields: chunked, pipelined forward (pw_offload.hip).  out_dev
// holds the device addresses of su, sv, sw when they are mapped pinned host
// memory, else nullptr; direct_ok: the slab kernels may write them directly;
// copy_out: PW_COPY_OUT_* (a mode the outputs do not allow falls back to
// the runtime's copies).
// With after_previous the call's copies and kernels start after the last copy
// out of the offload call queued before it on the device (its buffers may be
// the same).
size_t offload_workspace_bytes(const Geom& g, int chunk, size_t es);
template <typename T, typename C>
int offload_fwd(const T* u, const T* v, const T* w, const double* tzc1, const double* tzc2, double tcx, double tcy,
                const Geom& g, T* su, T* sv, T* sw, T* const* out_dev, bool direct_ok, int copy_out, int chunk,
                void* workspace, bool use_march, bool after_previous, MarchTune tune, hipStream_t stream,
                const char** what);

// Static scratch of pw_advect_fwd_host_static (pw_offload.hip): its size and
// the current device's address of it (looked up once per device).
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
hipError_t static_scratch_for_current_device(void** out);
