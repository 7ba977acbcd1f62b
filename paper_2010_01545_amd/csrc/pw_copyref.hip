// pw_copyref.hip -- measurement utility: the plain streaming copy that the
// HBM rate of the advection kernels is read against.  It moves the same
// streams as an advection call (n arrays read, n written, each of one storage
// array's size) with nothing else to do: 16-byte accesses, every thread
// reading its unit of every source before writing it to every destination.
#include "pw_internal.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr int kMaxArrays = 8;

// The pointers are named members and the data named registers: an indexed
// array here (of pointers or of loaded values) would be placed in scratch or
// LDS by the compiler, which a plain copy must not touch.
struct CopyPtrs {
    const uint4 *s0, *s1, *s2, *s3, *s4, *s5, *s6, *s7;
    uint4 *d0, *d1, *d2, *d3, *d4, *d5, *d6, *d7;
};

template <int N>
__global__ void __launch_bounds__(kCopyThreads) stream_copy_kernel(CopyPtrs p, size_t units)
{
    static_assert(N >= 1 && N <= kMaxArrays, "1..8 arrays");
    const size_t step = (size_t)gridDim.x * kCopyThreads;
    for (size_t x = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; x < units; x += step) {
        uint4 a0, a1, a2, a3, a4, a5, a6, a7;
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

template <int N>
void launch_n(const CopyPtrs& p, size_t units, int blocks, hipStream_t s)
{
    const size_t one_pass = (units + kCopyThreads - 1) / kCopyThreads;
    const size_t grid = blocks > 0 ? (size_t)blocks : one_pass;
    hipLaunchKernelGGL(stream_copy_kernel<N>, dim3((unsigned)grid), dim3(kCopyThreads), 0, s, p, units);
}

}  // namespace

// n in 1..8, bytes a multiple of 16, pointers 16-byte aligned (checked by the
// caller); blocks = 0: one 16-byte unit per thread and array.
void launch_stream_copy(const void* const* src, void* const* dst, int n, size_t bytes, int blocks, hipStream_t s)
{
    const size_t units = bytes / 16;
    if (units == 0) return;
    const uint4* sp[kMaxArrays] = {};
    uint4* dp[kMaxArrays] = {};
    for (int q = 0; q < n && q < kMaxArrays; ++q) {
        sp[q] = (const uint4*)src[q];
        dp[q] = (uint4*)dst[q];
    }
    const CopyPtrs p{sp[0], sp[1], sp[2], sp[3], sp[4], sp[5], sp[6], sp[7],
                     dp[0], dp[1], dp[2], dp[3], dp[4], dp[5], dp[6], dp[7]};
    switch (n) {
    case 1: launch_n<1>(p, units, blocks, s); break;
    case 2: launch_n<2>(p, units, blocks, s); break;
    case 3: launch_n<3>(p, units, blocks, s); break;
    case 4: launch_n<4>(p, units, blocks, s); break;
    case 5: launch_n<5>(p, units, blocks, s); break;
    case 6: launch_n<6>(p, units, blocks, s); break;
    case 7: launch_n<7>(p, units, blocks, s); break;
    default: launch_n<8>(p, units, blocks, s); break;
    }
}
