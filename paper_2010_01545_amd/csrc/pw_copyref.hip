// pw_copyref.hip -- measurement utility: the plain streaming copy that the
// HBM rate of the advection kernels is read against.  It moves the same
// streams as an advection call (n arrays read, n written, each of one storage
// array's size) with nothing else to do: every thread reads its unit (4, 8
// or 16 bytes) of every source before writing it to every destination, in
// 256-thread workgroups, with the default or the non-temporal (streaming)
// cache policy on its loads and stores.  Measured on MI355X for three FP64
// storage arrays of 4096 x 4096 x 64 in one pass: 4-byte units 8.49-8.58 ms,
// 8.09 ms with streaming loads; 8-byte units 9.46 ms, 16-byte units 8.99 ms;
// 16-byte units in 2048 striding workgroups 9.78 ms.  Six arrays: 4-byte
// units 17.45-17.81 ms, 16.38 ms with streaming loads and stores.
#include "../../include/pwadvect.h"
#include "pw_internal.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr int kMaxArrays = 8;
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

// one unit, with the non-temporal cache policy when NT
template <bool NT, typename U>
__device__ __forceinline__ U load_unit(const U* q)
{
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}
template <bool NT, typename U>
__device__ __forceinline__ void store_unit(U x, U* q)
{
    if constexpr (NT) __builtin_nontemporal_store(x, q);
    else *q = x;
}

// The pointers are named members and the data named registers: an indexed
// array here (of pointers or of loaded values) would be placed in scratch or
// LDS by the compiler, which a plain copy must not touch.
template <typename U>
struct CopyPtrs {
    const U *s0, *s1, *s2, *s3, *s4, *s5, *s6, *s7;
    U *d0, *d1, *d2, *d3, *d4, *d5, *d6, *d7;
};

template <typename U, int N, int H>
__global__ void __launch_bounds__(kCopyThreads) stream_copy_kernel(CopyPtrs<U> p, size_t units)
{
    static_assert(N >= 1 && N <= kMaxArrays, "1..8 arrays");
    constexpr bool L = (H & PW_COPY_NT_LOADS) != 0, S = (H & PW_COPY_NT_STORES) != 0;
    const size_t step = (size_t)gridDim.x * kCopyThreads;
    for (size_t x = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; x < units; x += step) {
        U a0, a1, a2, a3, a4, a5, a6, a7;
        a0 = load_unit<L>(p.s0 + x);
        if constexpr (N > 1) a1 = load_unit<L>(p.s1 + x);
        if constexpr (N > 2) a2 = load_unit<L>(p.s2 + x);
        if constexpr (N > 3) a3 = load_unit<L>(p.s3 + x);
        if constexpr (N > 4) a4 = load_unit<L>(p.s4 + x);
        if constexpr (N > 5) a5 = load_unit<L>(p.s5 + x);
        if constexpr (N > 6) a6 = load_unit<L>(p.s6 + x);
        if constexpr (N > 7) a7 = load_unit<L>(p.s7 + x);
        store_unit<S>(a0, p.d0 + x);
        if constexpr (N > 1) store_unit<S>(a1, p.d1 + x);
        if constexpr (N > 2) store_unit<S>(a2, p.d2 + x);
        if constexpr (N > 3) store_unit<S>(a3, p.d3 + x);
        if constexpr (N > 4) store_unit<S>(a4, p.d4 + x);
        if constexpr (N > 5) store_unit<S>(a5, p.d5 + x);
        if constexpr (N > 6) store_unit<S>(a6, p.d6 + x);
        if constexpr (N > 7) store_unit<S>(a7, p.d7 + x);
    }
}

template <typename U, int N, int H>
void launch_n(const CopyPtrs<U>& p, size_t units, int blocks, hipStream_t s)
{
    const size_t one_pass = (units + kCopyThreads - 1) / kCopyThreads;
    const size_t grid = blocks > 0 ? (size_t)blocks : one_pass;
    hipLaunchKernelGGL((stream_copy_kernel<U, N, H>), dim3((unsigned)grid), dim3(kCopyThreads), 0, s, p, units);
}

template <typename U, int H>
void launch_unit(const void* const* src, void* const* dst, int n, size_t bytes, int blocks, hipStream_t s)
{
    const size_t units = bytes / sizeof(U);
    if (units == 0) return;
    const U* sp[kMaxArrays] = {};
    U* dp[kMaxArrays] = {};
    for (int q = 0; q < n && q < kMaxArrays; ++q) {
        sp[q] = (const U*)src[q];
        dp[q] = (U*)dst[q];
    }
    const CopyPtrs<U> p{sp[0], sp[1], sp[2], sp[3], sp[4], sp[5], sp[6], sp[7],
                        dp[0], dp[1], dp[2], dp[3], dp[4], dp[5], dp[6], dp[7]};
    switch (n) {
    case 1: launch_n<U, 1, H>(p, units, blocks, s); break;
    case 2: launch_n<U, 2, H>(p, units, blocks, s); break;
    case 3: launch_n<U, 3, H>(p, units, blocks, s); break;
    case 4: launch_n<U, 4, H>(p, units, blocks, s); break;
    case 5: launch_n<U, 5, H>(p, units, blocks, s); break;
    case 6: launch_n<U, 6, H>(p, units, blocks, s); break;
    case 7: launch_n<U, 7, H>(p, units, blocks, s); break;
    default: launch_n<U, 8, H>(p, units, blocks, s); break;
    }
}

template <int H>
void launch_hinted(const void* const* src, void* const* dst, int n, size_t bytes, int unit, int blocks,
                   hipStream_t s)
{
    if (unit == 4)
        launch_unit<unsigned, H>(src, dst, n, bytes, blocks, s);
    else if (unit == 8)
        launch_unit<unsigned long long, H>(src, dst, n, bytes, blocks, s);
    else
        launch_unit<u32x4, H>(src, dst, n, bytes, blocks, s);
}

}  // namespace

// n in 1..8, unit 4, 8 or 16 bytes dividing bytes, pointers aligned to the
// unit, hints an OR of PW_COPY_NT_* (checked by the caller); blocks = 0: one
// unit per thread and array.
void launch_stream_copy(const void* const* src, void* const* dst, int n, size_t bytes, int unit, int blocks,
                        int hints, hipStream_t s)
{
    switch (hints & (PW_COPY_NT_LOADS | PW_COPY_NT_STORES)) {
    case PW_COPY_NT_LOADS: launch_hinted<PW_COPY_NT_LOADS>(src, dst, n, bytes, unit, blocks, s); break;
    case PW_COPY_NT_STORES: launch_hinted<PW_COPY_NT_STORES>(src, dst, n, bytes, unit, blocks, s); break;
    case PW_COPY_NT_LOADS | PW_COPY_NT_STORES:
        launch_hinted<PW_COPY_NT_LOADS | PW_COPY_NT_STORES>(src, dst, n, bytes, unit, blocks, s);
        break;
    default: launch_hinted<0>(src, dst, n, bytes, unit, blocks, s); break;
    }
}
