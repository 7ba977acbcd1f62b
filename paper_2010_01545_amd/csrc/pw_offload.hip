// pw_offload.hip -- forward source terms for fields held in host memory: the
// offload that the paper measures in its sections 4 and 5 (copy the winds to
// the accelerator, run the kernel, copy the source terms back), with the
// transfer split into x-slabs and pipelined so that the host->device copy of
// one slab, the kernel on the previous one and the device->host copy of the
// one before overlap (the chunked transfer its section 6 proposes).
//
// Slab k covers interior planes [i0, i0 + c).  In the storage layout the
// planes i0 - h .. i0 + c + h - 1 (interior plus the real neighbouring
// planes as x halo) are one contiguous run per field, so each input slab is a
// single copy into a device slab array of c + 2h planes.  The forward kernel
// runs on that slab as a grid of c planes; it writes the interior columns of
// its c planes, which go back with one 2-D copy per field (rows = planes, the
// ny interior columns of a plane being contiguous), so the host arrays' x/y
// halo columns are never written.
//
// Three slab buffers rotate: copies in on one internal stream, kernels on the
// caller's stream, copies out on a second internal stream, ordered by events.
// The internal streams and events are created once per device (default
// priority) and kept for the life of the process.
//
// Copies out, three ways.  The runtime's 2-D copy writes each slab's rows
// back from the copy-out stream.  For output arrays in pinned host memory
// mapped into the device's address space (out_dev holds their device
// addresses), a copy kernel on the copy-out stream can write them instead,
// leaving the copy engines to the inputs; or the slab kernels store straight
// into the mapped host arrays (the slab's planes at their place in the host
// array: the slab geometry has the host array's plane size), so nothing is
// copied out and the kernel's stores cross PCIe while the next slab's inputs
// come in.
//
// Which is fastest depends on the machine: with both directions on copy
// engines the runtime sometimes serialises them on one engine (on one kind
// of machine 148-150 ms per call at 4096 x 1024 x 64 FP64, now and then 258
// ms, against 167 ms with the copy kernel and 170 ms with direct writes; on
// another 214 ms, or 457 ms in three calls of four, against 272 ms with the
// copy kernel).  In the automatic mode (the default) every call is timed
// with two events on the caller's stream; a later call reads the times of
// the calls that have finished (hipEventQuery: it never waits) and takes the
// mode with the lowest mean time per byte over its last eight calls, the
// slowest of them left out, after first trying each mode the call allows
// and trying the others again every eighth call.  That estimates the
// expected time of a mode whose calls are now fast, now slow: a median of
// three stayed on the runtime's copies where they were slow in most calls
// (457 ms against 271 ms for the copy kernel); a plain mean left them for
// several calls after one or two slow calls among fast ones (210 ms in most
// calls, 457 ms in one or two of eight, still below the copy kernel on
// average).
#include <algorithm>
#include <mutex>

#include "../../include/pwadvect.h"
#include "pw_half.h"
#include "pw_internal.h"

namespace {

constexpr int kBuffers = 3;
constexpr int kCopyBlock = 256;

// rows x rowunits units of U from src to dst, both with a pitch of
// pitchunits units; blockIdx.y strides over rows.
template <typename U>
__global__ void __launch_bounds__(kCopyBlock)
copy_rows_kernel(const U* __restrict__ src, U* __restrict__ dst, size_t pitchunits, size_t rowunits, int rows)
{
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        const U* s = src + (size_t)r * pitchunits;
        U* d = dst + (size_t)r * pitchunits;
        for (size_t x = (size_t)blockIdx.x * kCopyBlock + threadIdx.x; x < rowunits; x += (size_t)gridDim.x * kCopyBlock)
            d[x] = s[x];
    }
}

// Widest access unit (16, 8, 4 or 2 bytes) that divides both addresses, the
// pitch and the row length, so every row is copied whole: rows of 16-bit
// elements can be any even number of bytes long.
size_t copy_unit(const void* src, const void* dst, size_t pitch, size_t row)
{
    const uintptr_t all = (uintptr_t)src | (uintptr_t)dst | (uintptr_t)pitch | (uintptr_t)row;
    for (size_t u = 16; u > 2; u /= 2)
        if (all % u == 0) return u;
    return 2;
}

template <typename U>
void copy_rows_as(const void* src, void* dst, size_t pitch, size_t row, int rows, hipStream_t s)
{
    const size_t units = row / sizeof(U);
    unsigned bx = (unsigned)((units + kCopyBlock - 1) / kCopyBlock);
    if (bx > 1024) bx = 1024;
    const dim3 grid(bx, (unsigned)(rows < 65535 ? rows : 65535));
    hipLaunchKernelGGL(copy_rows_kernel<U>, grid, dim3(kCopyBlock), 0, s, (const U*)src, (U*)dst,
                       pitch / sizeof(U), units, rows);
}

// Element sizes are 2, 4 or 8 bytes, so src, dst, pitch and row are even.
void copy_rows(const void* src, void* dst, size_t pitch, size_t row, int rows, hipStream_t s)
{
    switch (copy_unit(src, dst, pitch, row)) {
    case 16: copy_rows_as<uint4>(src, dst, pitch, row, rows, s); break;
    case 8: copy_rows_as<unsigned long long>(src, dst, pitch, row, rows, s); break;
    case 4: copy_rows_as<unsigned>(src, dst, pitch, row, rows, s); break;
    default: copy_rows_as<unsigned short>(src, dst, pitch, row, rows, s); break;
    }
}

constexpr int kModes = 3;       // PW_COPY_OUT_RUNTIME, _KERNEL, _DIRECT
constexpr int kTimed = 8;       // calls whose times may be outstanding
constexpr int kRetryEvery = 8;  // automatic mode: retry the other modes every this many calls
constexpr int kSamples = 8;     // times kept per mode; its cost is their mean without the slowest

struct CallTimer {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int mode = 0;
    double gbytes = 0.0;
    bool live = false;
};

struct DeviceQueues {
    bool ready = false;
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t start = nullptr, done_in[kBuffers] = {}, done_kernel[kBuffers] = {}, done_out[kBuffers] = {},
               end_out = nullptr;
    // automatic copy-out choice: the last kSamples times of each mode in ms
    // per GB, their cost (their mean without the slowest, the expected time of
    // a mode whose calls are now fast, now slow; < 0: no sample yet), the call
    // count at its last sample, and the timers in flight
    double samples[kModes][kSamples] = {};
    int nsamples[kModes] = {0, 0, 0};
    double cost[kModes] = {-1.0, -1.0, -1.0};
    long long sampled_at[kModes] = {-1, -1, -1};
    long long calls = 0;
    CallTimer timers[kTimed];
    int next_timer = 0;
};

std::mutex g_queues_mutex;
std::mutex g_enqueue_mutex;
DeviceQueues g_queues[64];

hipError_t queues_for_current_device(DeviceQueues** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_queues_mutex);
    DeviceQueues& q = g_queues[dev];
    if (!q.ready) {
        const unsigned ev = hipEventDisableTiming;
        if ((e = hipStreamCreateWithFlags(&q.h2d, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipStreamCreateWithFlags(&q.d2h, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&q.start, ev)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&q.end_out, ev)) != hipSuccess) return e;
        for (int b = 0; b < kBuffers; ++b) {
            if ((e = hipEventCreateWithFlags(&q.done_in[b], ev)) != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&q.done_kernel[b], ev)) != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&q.done_out[b], ev)) != hipSuccess) return e;
        }
        for (int t = 0; t < kTimed; ++t) {   // timing events
            if ((e = hipEventCreateWithFlags(&q.timers[t].t0, hipEventDefault)) != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&q.timers[t].t1, hipEventDefault)) != hipSuccess) return e;
        }
        q.ready = true;
    }
    *out = &q;
    return hipSuccess;
}

// Fold the times of finished calls into the per-mode costs (never waits).
void harvest_timers(DeviceQueues* q)
{
    for (CallTimer& t : q->timers) {
        if (!t.live) continue;
        const hipError_t e = hipEventQuery(t.t1);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            continue;
        }
        float ms = 0.0f;
        if (e == hipSuccess && hipEventElapsedTime(&ms, t.t0, t.t1) == hipSuccess && t.gbytes > 0.0) {
            const int m = t.mode;
            double* s = q->samples[m];
            for (int i = kSamples - 1; i > 0; --i) s[i] = s[i - 1];
            s[0] = (double)ms / t.gbytes;
            if (q->nsamples[m] < kSamples) ++q->nsamples[m];
            const int n = q->nsamples[m];
            double sum = 0.0, worst = 0.0;
            for (int i = 0; i < n; ++i) {
                sum += s[i];
                worst = std::max(worst, s[i]);
            }
            // from four samples on, the slowest is left out
            q->cost[m] = n >= 4 ? (sum - worst) / (n - 1) : sum / n;
            q->sampled_at[m] = q->calls;
        }
        (void)hipGetLastError();
        t.live = false;
    }
}

// Copy-out mode for an automatic-mode call: a mode the call allows that has
// no time yet (and none in flight), else every kRetryEvery-th call the
// allowed mode sampled longest ago, else the lowest recent cost.  Without
// exploring (a call being captured into a graph): the lowest cost known.
int choose_copy_out(DeviceQueues* q, const bool allowed[kModes], bool explore)
{
    bool pending[kModes] = {false, false, false};
    for (const CallTimer& t : q->timers)
        if (t.live) pending[t.mode] = true;
    for (int m = 0; m < kModes && explore; ++m)
        if (allowed[m] && q->cost[m] < 0.0 && !pending[m]) return m;
    int best = PW_COPY_OUT_RUNTIME;
    if (explore && q->calls % kRetryEvery == 0) {
        for (int m = 0; m < kModes; ++m)
            if (allowed[m] && q->sampled_at[m] < q->sampled_at[best]) best = m;
        return best;
    }
    for (int m = 0; m < kModes; ++m)
        if (allowed[m] && q->cost[m] >= 0.0 && (q->cost[best] < 0.0 || q->cost[m] < q->cost[best])) best = m;
    return best;
}

}  // namespace

// Scratch of the allocation-free entry point pw_advect_fwd_host_static: its
// three slab buffer sets live in this array instead of a caller's workspace.
// Every device the library runs on holds its own copy from module load until
// the process ends.  In host code `scratch` names a host-side stand-in, never
// the device memory: host code uses only the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mutex;
void* g_scratch_ptr[64] = {};
}  // namespace

hipError_t static_scratch_for_current_device(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Bytes of one slab buffer set: three input and three output slab arrays of
// chunk + 2h planes each.
size_t offload_slab_set_bytes(const Geom& g, int chunk, size_t es)
{
    return (size_t)6 * (size_t)(chunk + 2 * g.h) * (size_t)g.sx * es;
}

size_t offload_workspace_bytes(const Geom& g, int chunk, size_t es)
{
    return (size_t)kBuffers * offload_slab_set_bytes(g, chunk, es);
}

template <typename T, typename C>
int offload_fwd(const T* u, const T* v, const T* w, const double* tzc1, const double* tzc2, double tcx, double tcy,
                const Geom& g, T* su, T* sv, T* sw, T* const* out_dev, bool direct_ok, int copy_out, int chunk,
                void* workspace, bool use_march, bool after_previous, MarchTune tune, hipStream_t stream,
                const char** what)
{
    DeviceQueues* q = nullptr;
    hipError_t e = queues_for_current_device(&q);
    if (e != hipSuccess) {
        *what = "creating the offload streams";
        return (int)e;
    }
    // one enqueue at a time per process: the internal streams and events are
    // shared, and each wait captures the event's latest record when it is queued
    std::lock_guard<std::mutex> lock(g_enqueue_mutex);
    // a call captured into a graph records and queries no timing events
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool timed = hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
    (void)hipGetLastError();
    if (timed) harvest_timers(q);
    const bool allowed[kModes] = {true, out_dev != nullptr, out_dev != nullptr && direct_ok};
    int mode = copy_out == PW_COPY_OUT_AUTO ? choose_copy_out(q, allowed, timed)
             : (copy_out >= 0 && copy_out < kModes && allowed[copy_out]) ? copy_out : PW_COPY_OUT_RUNTIME;
    if (timed) ++q->calls;
    const bool direct = mode == PW_COPY_OUT_DIRECT;
    if (mode == PW_COPY_OUT_RUNTIME) out_dev = nullptr;
    CallTimer* timer = nullptr;
    if (timed) {
        timer = &q->timers[q->next_timer];
        q->next_timer = (q->next_timer + 1) % kTimed;
        timer->live = false;   // (a time still in flight when its slot is reused is dropped)
    }
    // a call whose buffers another call may still use (the static scratch)
    // starts after the last copy out of the call queued before it
    if (after_previous) {
        if ((e = hipStreamWaitEvent(q->h2d, q->end_out, 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
        if ((e = hipStreamWaitEvent(stream, q->end_out, 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
    }
    if (timer && (e = hipEventRecord(timer->t0, stream)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
    const size_t plane = (size_t)g.sx;                       // elements per storage plane
    const size_t slab = (size_t)(chunk + 2 * g.h) * plane;   // elements per slab array
    T* base = (T*)workspace;
    auto buf = [&](int b, int f) -> T* { return base + ((size_t)b * 6 + (size_t)f) * slab; };
    const T* in[3] = {u, v, w};
    T* out[3] = {su, sv, sw};
    const size_t row = (size_t)g.ny * (size_t)g.Sz * sizeof(T);   // interior columns of a plane
    const size_t pitch = plane * sizeof(T);
    const size_t col0 = (size_t)g.h * (size_t)g.Sz;                // first interior column in a plane

    // everything starts after the work already queued on the caller's stream
    if ((e = hipEventRecord(q->start, stream)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
    if ((e = hipStreamWaitEvent(q->h2d, q->start, 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
    if ((e = hipStreamWaitEvent(q->d2h, q->start, 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }

    const int nslabs = (g.nx + chunk - 1) / chunk;
    for (int k = 0; k < nslabs; ++k) {
        const int b = k % kBuffers;
        const int i0 = k * chunk;
        const int c = g.nx - i0 < chunk ? g.nx - i0 : chunk;
        Geom sg = g;
        sg.nx = c;
        sg.Sx = c + 2 * g.h;
        // inputs: storage planes i0 .. i0 + c + 2h - 1 (interior planes i0-h .. i0+c+h-1)
        if (k >= kBuffers && (e = hipStreamWaitEvent(q->h2d, q->done_kernel[b], 0)) != hipSuccess) {
            *what = "hipStreamWaitEvent";
            return (int)e;
        }
        for (int f = 0; f < 3; ++f) {
            e = hipMemcpyAsync(buf(b, f), in[f] + (size_t)i0 * plane, (size_t)(c + 2 * g.h) * pitch,
                               hipMemcpyHostToDevice, q->h2d);
            if (e != hipSuccess) { *what = "hipMemcpyAsync (to device)"; return (int)e; }
        }
        if ((e = hipEventRecord(q->done_in[b], q->h2d)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
        // kernel on the slab
        if ((e = hipStreamWaitEvent(stream, q->done_in[b], 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
        if (!direct && k >= kBuffers && (e = hipStreamWaitEvent(stream, q->done_out[b], 0)) != hipSuccess) {
            *what = "hipStreamWaitEvent";
            return (int)e;
        }
        // direct writes: plane p of the slab is plane i0 + p of the host array
        T* const o0 = direct ? out_dev[0] + (size_t)i0 * plane : buf(b, 3);
        T* const o1 = direct ? out_dev[1] + (size_t)i0 * plane : buf(b, 4);
        T* const o2 = direct ? out_dev[2] + (size_t)i0 * plane : buf(b, 5);
        FwdArgs<T> a{buf(b, 0), buf(b, 1), buf(b, 2), tzc1, tzc2, tcx, tcy, o0, o1, o2};
        (void)hipGetLastError();
        if (use_march)
            launch_fwd_march<T, C>(a, sg, tune, stream);
        else
            launch_fwd_direct<T, C>(a, sg, stream);
        if ((e = hipGetLastError()) != hipSuccess) { *what = "kernel launch"; return (int)e; }
        if ((e = hipEventRecord(q->done_kernel[b], stream)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
        if (direct) continue;
        // outputs: interior columns of the slab's c interior planes
        if ((e = hipStreamWaitEvent(q->d2h, q->done_kernel[b], 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
        for (int f = 0; f < 3; ++f) {
            const T* src = buf(b, 3 + f) + (size_t)g.h * plane + col0;
            const size_t off = (size_t)(i0 + g.h) * plane + col0;
            if (out_dev) {
                copy_rows(src, out_dev[f] + off, pitch, row, c, q->d2h);
                if ((e = hipGetLastError()) != hipSuccess) { *what = "copy kernel launch"; return (int)e; }
            } else {
                e = hipMemcpy2DAsync(out[f] + off, pitch, src, pitch, row, (size_t)c, hipMemcpyDeviceToHost, q->d2h);
                if (e != hipSuccess) { *what = "hipMemcpy2DAsync (to host)"; return (int)e; }
            }
        }
        if ((e = hipEventRecord(q->done_out[b], q->d2h)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
    }
    // later work on the caller's stream sees every copy back (with direct
    // writes the last kernel is the call's last step)
    if ((e = hipEventRecord(q->end_out, direct ? stream : q->d2h)) != hipSuccess) {
        *what = "hipEventRecord";
        return (int)e;
    }
    if ((e = hipStreamWaitEvent(stream, q->end_out, 0)) != hipSuccess) { *what = "hipStreamWaitEvent"; return (int)e; }
    if (timer) {
        if ((e = hipEventRecord(timer->t1, stream)) != hipSuccess) { *what = "hipEventRecord"; return (int)e; }
        timer->mode = mode;
        timer->gbytes = (double)((size_t)2 * 3 * (size_t)g.Sx * plane * sizeof(T)) * 1e-9;
        timer->live = true;
    }
    return 0;
}

#define PW_OFFLOAD_INSTANCE(T, C)                                                                            \
    template int offload_fwd<T, C>(const T*, const T*, const T*, const double*, const double*, double, double, \
                                   const Geom&, T*, T*, T*, T* const*, bool, int, int, void*, bool, bool,     \
                                   MarchTune, hipStream_t, const char**);
PW_OFFLOAD_INSTANCE(double, double)
PW_OFFLOAD_INSTANCE(float, float)
PW_OFFLOAD_INSTANCE(float, double)
PW_OFFLOAD_INSTANCE(_Float16, float)
PW_OFFLOAD_INSTANCE(bf16_t, float)
