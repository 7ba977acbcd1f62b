// pw_copyref.hip -- measurement utility: the plain streaming copy that the
// HBM rate of the advection kernels is read against.  It moves the same
// streams as an advection call (n arrays read, n written, each of one storage
// array's size) with nothing else to do: every thread reads its unit (4, 8
// or 16 bytes) of every source before writing it to every destination, in
// 256-thread workgroups.  Measured on MI355X for three FP64 storage arrays of
// 4096 x 4096 x 64 in one pass: 4-byte units 8.49-8.58 ms, 8-byte units
// 9.46 ms, 16-byte units 8.99 ms; 16-byte units in 2048 striding workgroups
// 9.78 ms.
#include "pw_internal.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr int kMaxArrays = 8;

// The pointers are named members and the data named registers: an indexed
// array here (of pointers or of loaded values) would be placed in scratch or
// LDS by the compiler, which a plain copy must not touch.
template <typename U>
struct CopyPtrs {
    const U *s0, *s1, *s2, *s3, *s4, *s5, *s6, *s7;
    U *d0, *d1, *d2, *d3, *d4, *d5, *d6, *d7;
};

template <typename U, int N>
__global__ void __launch_bounds__(kCopyThreads) stream_copy_kernel(CopyPtrs<U> p, size_t units)
{
    static_assert(N >= 1 && N <= kMaxArrays, "1..8 arrays");
    const size_t step = (size_t)gridDim.x * kCopyThreads;
    for (size_t x = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; x < units; x += step) {
        U a0, a1, a2, a3, a4, a5, a6, a7;
        a0 = p.s0[x];
        if constexpr (N > 1) a1 = p.s1[x];
        if constexpr (N > 2) a2 = p.s2[x];
        if constexpr (N > 3) a3 = p.s3[x];
        if constexpr (N > 4) a4 = p.s4[x];
        if constexpr (N > 5) a5 = p.s5[x];
        if constexpr (N > 6) a6 = p.s6[x];
        if constexpr (N > 7) a7 = p.s7[x];
        p.d0[x] = a0;
        if constexpr (N > 1) p.d1[x] = a1;
        if constexpr (N > 2) p.d2[x] = a2;
        if constexpr (N > 3) p.d3[x] = a3;
        if constexpr (N > 4) p.d4[x] = a4;
        if constexpr (N > 5) p.d5[x] = a5;
        if constexpr (N > 6) p.d6[x] = a6;
        if constexpr (N > 7) p.d7[x] = a7;
    }
}

template <typename U, int N>
void launch_n(const CopyPtrs<U>& p, size_t units, int blocks, hipStream_t s)
{
    const size_t one_pass = (units + kCopyThreads - 1) / kCopyThreads;
    const size_t grid = blocks > 0 ? (size_t)blocks : one_pass;
    hipLaunchKernelGGL((stream_copy_kernel<U, N>), dim3((unsigned)grid), dim3(kCopyThreads), 0, s, p, units);
}

template <typename U>
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
    case 1: launch_n<U, 1>(p, units, blocks, s); break;
    case 2: launch_n<U, 2>(p, units, blocks, s); break;
    case 3: launch_n<U, 3>(p, units, blocks, s); break;
    case 4: launch_n<U, 4>(p, units, blocks, s); break;
    case 5: launch_n<U, 5>(p, units, blocks, s); break;
    case 6: launch_n<U, 6>(p, units, blocks, s); break;
    case 7: launch_n<U, 7>(p, units, blocks, s); break;
    default: launch_n<U, 8>(p, units, blocks, s); break;
    }
}

}  // namespace

// n in 1..8, unit 4, 8 or 16 bytes dividing bytes, pointers aligned to the
// unit (checked by the caller); blocks = 0: one unit per thread and array.
void launch_stream_copy(const void* const* src, void* const* dst, int n, size_t bytes, int unit, int blocks,
                        hipStream_t s)
{
    if (unit == 4)
        launch_unit<unsigned>(src, dst, n, bytes, blocks, s);
    else if (unit == 8)
        launch_unit<unsigned long long>(src, dst, n, bytes, blocks, s);
    else
        launch_unit<uint4>(src, dst, n, bytes, blocks, s);
}
