// pw_copyref.hip -- measurement utility: the plain streaming copy that the
// HBM rate of the advection kernels is read against.  It moves the same
// streams as an advection call (n arrays read, n written, each of one storage
// array's size) with nothing else to do: 16-byte accesses, every thread
// reading its unit of every source before writing it to every destination.
#include "pw_internal.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr int kMaxArrays = 8;

template <int N>
struct CopyPtrs {
    const uint4* src[N];
    uint4* dst[N];
};

template <int N>
__global__ void __launch_bounds__(kCopyThreads) stream_copy_kernel(CopyPtrs<N> p, size_t units)
{
    const size_t step = (size_t)gridDim.x * kCopyThreads;
    for (size_t x = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; x < units; x += step) {
        uint4 v[N];
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = p.src[q][x];
#pragma unroll
        for (int q = 0; q < N; ++q) p.dst[q][x] = v[q];
    }
}

template <int N>
void launch_n(const void* const* src, void* const* dst, size_t units, int blocks, hipStream_t s)
{
    CopyPtrs<N> p;
    for (int q = 0; q < N; ++q) {
        p.src[q] = (const uint4*)src[q];
        p.dst[q] = (uint4*)dst[q];
    }
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
    switch (n) {
    case 1: launch_n<1>(src, dst, units, blocks, s); break;
    case 2: launch_n<2>(src, dst, units, blocks, s); break;
    case 3: launch_n<3>(src, dst, units, blocks, s); break;
    case 4: launch_n<4>(src, dst, units, blocks, s); break;
    case 5: launch_n<5>(src, dst, units, blocks, s); break;
    case 6: launch_n<6>(src, dst, units, blocks, s); break;
    case 7: launch_n<7>(src, dst, units, blocks, s); break;
    default: launch_n<kMaxArrays>(src, dst, units, blocks, s); break;
    }
}
