// pw_util.hip -- storage preparation kernels: periodic halo fill, padding of a
// compact interior array, and the counter-based input generator.
#include "pw_half.h"
#include "pw_internal.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Halo columns, enumerated as: the 2h x-halo planes (all Sy columns each),
// then the 2h y-halo columns of each interior x plane.  Thread per
// (halo column, storage level), level fastest.
template <typename T>
__global__ void __launch_bounds__(kBlock) halo_periodic_kernel(T* __restrict__ st, Geom g,
                                                               long long ncols)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long col = t / g.Sz;
    if (col >= ncols) return;
    const int kk = (int)(t - col * g.Sz);
    const long long nxh = 2LL * g.h * g.Sy;  // columns in x-halo planes
    int si, sj;
    if (col < nxh) {
        const int p = (int)(col / g.Sy);      // 0 .. 2h-1
        sj = (int)(col - (long long)p * g.Sy);
        si = p < g.h ? p : g.nx + p;          // planes 0..h-1 and nx+h..nx+2h-1
    } else {
        const long long r = col - nxh;
        const int p = (int)(r / (2 * g.h));   // interior plane
        const int q = (int)(r - (long long)p * 2 * g.h);
        si = g.h + p;
        sj = q < g.h ? q : g.ny + q;
    }
    const int i = wrap(si - g.h, g.nx) + g.h;
    const int j = wrap(sj - g.h, g.ny) + g.h;
    st[(long long)si * g.sx + (long long)sj * g.sy + kk] = st[(long long)i * g.sx + (long long)j * g.sy + kk];
}

// Storage from a compact interior array; thread per storage element of one
// x plane (blockIdx.y walks planes).
template <typename T>
__global__ void __launch_bounds__(kBlock) pad_periodic_kernel(const T* __restrict__ in,
                                                              T* __restrict__ st, Geom g)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.Sy * g.Sz) return;
    const int sj = t / g.Sz;
    const int kk = t - sj * g.Sz;
    const int k = kk - g.h;
    const int j = wrap(sj - g.h, g.ny);
    for (int si = blockIdx.y; si < g.Sx; si += gridDim.y) {
        const int i = wrap(si - g.h, g.nx);
        T val = T(0);
        if (k >= 0 && k < g.nz) val = in[((long long)i * g.ny + j) * g.nz + k];
        st[(long long)si * g.sx + t] = val;
    }
}

__device__ __forceinline__ unsigned long long splitmix64_mix(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Interior columns of one x plane per blockIdx.y step; thread per level.
template <typename T>
__global__ void __launch_bounds__(kBlock) fill_uniform_kernel(T* __restrict__ st, Geom g,
                                                              unsigned long long state,
                                                              double amp, int zero_lids)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.ny * g.Sz) return;
    const int j = t / g.Sz;
    const int kk = t - j * g.Sz;
    const int k = kk - g.h;
    for (int i = blockIdx.y; i < g.nx; i += gridDim.y) {
        double val = 0.0;
        if (k >= 0 && k < g.nz && !(zero_lids && (k == 0 || k == g.nz - 1))) {
            const unsigned long long idx = ((unsigned long long)i * g.ny + j) * g.nz + k;
            const unsigned long long z = splitmix64_mix(state + (idx + 1ULL) * 0x9E3779B97F4A7C15ULL);
            const long long m = (long long)(z >> 11) - (1LL << 52);
            const double unit = (double)m * 0x1p-52;  // exact
            val = amp * unit;                         // one rounding (then to_storage)
        }
        st[(long long)(i + g.h) * g.sx + (long long)(j + g.h) * g.sy + kk] = to_storage<T>(val);
    }
}

inline unsigned plane_blocks(int n) { return (unsigned)(n < 65535 ? n : 65535); }

}  // namespace

template <typename T>
void launch_halo_periodic(T* st, const Geom& g, hipStream_t s)
{
    const long long ncols = 2LL * g.h * g.Sy + 2LL * g.h * g.nx;
    const long long n = ncols * g.Sz;
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(halo_periodic_kernel<T>, dim3(blocks), dim3(kBlock), 0, s, st, g, ncols);
}

template <typename T>
void launch_pad_periodic(const T* in, T* st, const Geom& g, hipStream_t s)
{
    const unsigned bx = (unsigned)((g.Sy * g.Sz + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(pad_periodic_kernel<T>, dim3(bx, plane_blocks(g.Sx)), dim3(kBlock), 0, s,
                       in, st, g);
}

template <typename T>
void launch_fill_uniform(T* st, const Geom& g, unsigned long long seed, int field_id, double amp,
                         int zero_lids, hipStream_t s)
{
    const unsigned long long state = seed * 256ULL + (unsigned long long)field_id;
    const unsigned bx = (unsigned)((g.ny * g.Sz + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(fill_uniform_kernel<T>, dim3(bx, plane_blocks(g.nx)), dim3(kBlock), 0, s,
                       st, g, state, amp, zero_lids);
}

template void launch_halo_periodic<double>(double*, const Geom&, hipStream_t);
template void launch_halo_periodic<float>(float*, const Geom&, hipStream_t);
template void launch_pad_periodic<double>(const double*, double*, const Geom&, hipStream_t);
template void launch_pad_periodic<float>(const float*, float*, const Geom&, hipStream_t);
template void launch_fill_uniform<double>(double*, const Geom&, unsigned long long, int, double, int,
                                          hipStream_t);
template void launch_fill_uniform<float>(float*, const Geom&, unsigned long long, int, double, int,
                                         hipStream_t);
template void launch_halo_periodic<_Float16>(_Float16*, const Geom&, hipStream_t);
template void launch_halo_periodic<bf16_t>(bf16_t*, const Geom&, hipStream_t);
template void launch_pad_periodic<_Float16>(const _Float16*, _Float16*, const Geom&, hipStream_t);
template void launch_pad_periodic<bf16_t>(const bf16_t*, bf16_t*, const Geom&, hipStream_t);
template void launch_fill_uniform<_Float16>(_Float16*, const Geom&, unsigned long long, int, double, int,
                                            hipStream_t);
template void launch_fill_uniform<bf16_t>(bf16_t*, const Geom&, unsigned long long, int, double, int,
                                          hipStream_t);
