// pw_direct.hip -- the plain GPU form of the PW advection scheme: one thread
// per storage level of every interior column, all operands loaded straight
// from global memory (neighbour reuse is left to the L1/L2 caches).  It runs
// any nz >= 2 and halo >= 1 and is the fallback of the x-marching kernels.
//
// Grid: blockIdx.y walks x-planes (grid-stride), blockIdx.x * 256 + tid walks
// the ny * Sz storage levels of the plane's interior columns, z fastest, so a
// wavefront reads and writes contiguous runs of a column.  z-halo levels of
// interior columns are written with 0.
#include "pw_half.h"
#include "pw_internal.h"
#include "pw_stencil.h"

namespace {

constexpr int kBlock = 256;

// Star of field f around storage element b at interior level k; DIAG
// selects the field's two diagonal neighbours (0: u, 1: v, 2: w; see
// pw_stencil.h).  Operands on levels outside 0..nz-1 (z halo, whatever it
// holds) are replaced by 0; with LAM the adjoint multiplier's level mask is
// applied as well (lu, lv live on 1..nz-1, lw on 1..nz-2).
template <typename T, int DIAG, bool LAM>
__device__ __forceinline__ Star<T> load_star(const T* __restrict__ f, long long b, long long sx, int sy,
                                             int k, int nz)
{
    auto live = [&](int level) -> bool {
        if (LAM) return DIAG == 2 ? lam_w_live(level, nz) : lam_uv_live(level, nz);
        return level >= 0 && level <= nz - 1;
    };
    const bool lk = live(k), lkm = live(k - 1), lkp = live(k + 1);
    const T z = T(0);
    Star<T> s;
    s.c = lk ? f[b] : z;
    s.xm = lk ? f[b - sx] : z;
    s.xp = lk ? f[b + sx] : z;
    s.ym = lk ? f[b - sy] : z;
    s.yp = lk ? f[b + sy] : z;
    s.zm = lkm ? f[b - 1] : z;
    s.zp = lkp ? f[b + 1] : z;
    if (DIAG == 0) {
        s.d1 = lk ? f[b - sx + sy] : z;
        s.d2 = lkp ? f[b - sx + 1] : z;
    } else if (DIAG == 1) {
        s.d1 = lk ? f[b + sx - sy] : z;
        s.d2 = lkp ? f[b - sy + 1] : z;
    } else {
        s.d1 = lkm ? f[b + sx - 1] : z;
        s.d2 = lkm ? f[b + sy - 1] : z;
    }
    return s;
}

template <typename C, typename T>
__device__ __forceinline__ Star<C> widen(const Star<T>& s)
{
    return Star<C>{(C)s.c, (C)s.xm, (C)s.xp, (C)s.ym, (C)s.yp, (C)s.zm, (C)s.zp, (C)s.d1, (C)s.d2};
}

// UPD: 0 stores s; 1 stores b + beta * s with b loaded from a.b (which may be
// the output array itself: the element is read before it is written); 2 the
// same with b = (u, v, w), reusing the star centres.
template <typename T, typename C, int UPD>
__global__ void __launch_bounds__(kBlock) fwd_direct_kernel(FwdArgs<T> a, Geom g)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.ny * g.Sz) return;
    const int j = t / g.Sz;
    const int kk = t - j * g.Sz;
    const int k = kk - g.h;
    for (int i = blockIdx.y; i < g.nx; i += gridDim.y) {
        const long long b = (long long)(i + g.h) * g.sx + (long long)(j + g.h) * g.sy + kk;
        if (k < 0 || k >= g.nz) {
            a.su[b] = T(0);
            a.sv[b] = T(0);
            a.sw[b] = T(0);
            continue;
        }
        const Star<C> u = widen<C>(load_star<T, 0, false>(a.u, b, g.sx, g.sy, k, g.nz));
        const Star<C> v = widen<C>(load_star<T, 1, false>(a.v, b, g.sx, g.sy, k, g.nz));
        const Star<C> w = widen<C>(load_star<T, 2, false>(a.w, b, g.sx, g.sy, k, g.nz));
        const LevelCoef<C> cf = level_coef<C>(a.tzc1, a.tzc2, (C)a.tcx, (C)a.tcy, k, g.nz);
        C su, sv, sw;
        pw_fwd(u, v, w, cf, k, g.nz, su, sv, sw);
        if (UPD != 0) {
            const C beta = (C)a.beta;
            const C bu = UPD == 2 ? u.c : (C)a.b[0][b];
            const C bv = UPD == 2 ? v.c : (C)a.b[1][b];
            const C bw = UPD == 2 ? w.c : (C)a.b[2][b];
            su = pw_update(bu, beta, su);
            sv = pw_update(bv, beta, sv);
            sw = pw_update(bw, beta, sw);
        }
        a.su[b] = store_round<T>(su);
        a.sv[b] = store_round<T>(sv);
        a.sw[b] = store_round<T>(sw);
    }
}

template <typename T, typename C, bool FUSED>
__global__ void __launch_bounds__(kBlock) adj_direct_kernel(AdjArgs<T> a, Geom g)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.ny * g.Sz) return;
    const int j = t / g.Sz;
    const int kk = t - j * g.Sz;
    const int k = kk - g.h;
    for (int i = blockIdx.y; i < g.nx; i += gridDim.y) {
        const long long b = (long long)(i + g.h) * g.sx + (long long)(j + g.h) * g.sy + kk;
        if (k < 0 || k >= g.nz) {
            if (FUSED) {
                a.su[b] = T(0);
                a.sv[b] = T(0);
                a.sw[b] = T(0);
            }
            a.gu[b] = T(0);
            a.gv[b] = T(0);
            a.gw[b] = T(0);
            continue;
        }
        const Star<C> u = widen<C>(load_star<T, 0, false>(a.u, b, g.sx, g.sy, k, g.nz));
        const Star<C> v = widen<C>(load_star<T, 1, false>(a.v, b, g.sx, g.sy, k, g.nz));
        const Star<C> w = widen<C>(load_star<T, 2, false>(a.w, b, g.sx, g.sy, k, g.nz));
        const Star<C> lu = widen<C>(load_star<T, 0, true>(a.lu, b, g.sx, g.sy, k, g.nz));
        const Star<C> lv = widen<C>(load_star<T, 1, true>(a.lv, b, g.sx, g.sy, k, g.nz));
        const Star<C> lw = widen<C>(load_star<T, 2, true>(a.lw, b, g.sx, g.sy, k, g.nz));
        const LevelCoef<C> cf = level_coef<C>(a.tzc1, a.tzc2, (C)a.tcx, (C)a.tcy, k, g.nz);
        if (FUSED) {
            C su, sv, sw;
            pw_fwd(u, v, w, cf, k, g.nz, su, sv, sw);
            a.su[b] = store_round<T>(su);
            a.sv[b] = store_round<T>(sv);
            a.sw[b] = store_round<T>(sw);
        }
        C gu, gv, gw;
        pw_adj_cell(u, v, w, lu, lv, lw, cf, k, g.nz, gu, gv, gw);
        a.gu[b] = store_round<T>(gu);
        a.gv[b] = store_round<T>(gv);
        a.gw[b] = store_round<T>(gw);
    }
}

inline dim3 direct_grid(const Geom& g)
{
    const int per_plane = g.ny * g.Sz;
    const unsigned bx = (unsigned)((per_plane + kBlock - 1) / kBlock);
    const unsigned by = (unsigned)(g.nx < 65535 ? g.nx : 65535);
    return dim3(bx, by, 1);
}

}  // namespace

template <typename T, typename C>
void launch_fwd_direct(const FwdArgs<T>& a, const Geom& g, hipStream_t s)
{
    if (a.upd == 1)
        hipLaunchKernelGGL((fwd_direct_kernel<T, C, 1>), direct_grid(g), dim3(kBlock), 0, s, a, g);
    else if (a.upd == 2)
        hipLaunchKernelGGL((fwd_direct_kernel<T, C, 2>), direct_grid(g), dim3(kBlock), 0, s, a, g);
    else
        hipLaunchKernelGGL((fwd_direct_kernel<T, C, 0>), direct_grid(g), dim3(kBlock), 0, s, a, g);
}

template <typename T, typename C>
void launch_adj_direct(const AdjArgs<T>& a, const Geom& g, hipStream_t s)
{
    if (a.su)
        hipLaunchKernelGGL((adj_direct_kernel<T, C, true>), direct_grid(g), dim3(kBlock), 0, s, a, g);
    else
        hipLaunchKernelGGL((adj_direct_kernel<T, C, false>), direct_grid(g), dim3(kBlock), 0, s, a, g);
}

template void launch_fwd_direct<double, double>(const FwdArgs<double>&, const Geom&, hipStream_t);
template void launch_fwd_direct<float, float>(const FwdArgs<float>&, const Geom&, hipStream_t);
template void launch_fwd_direct<float, double>(const FwdArgs<float>&, const Geom&, hipStream_t);
template void launch_fwd_direct<_Float16, float>(const FwdArgs<_Float16>&, const Geom&, hipStream_t);
template void launch_fwd_direct<bf16_t, float>(const FwdArgs<bf16_t>&, const Geom&, hipStream_t);
template void launch_adj_direct<double, double>(const AdjArgs<double>&, const Geom&, hipStream_t);
template void launch_adj_direct<float, float>(const AdjArgs<float>&, const Geom&, hipStream_t);
template void launch_adj_direct<float, double>(const AdjArgs<float>&, const Geom&, hipStream_t);
template void launch_adj_direct<_Float16, float>(const AdjArgs<_Float16>&, const Geom&, hipStream_t);
template void launch_adj_direct<bf16_t, float>(const AdjArgs<bf16_t>&, const Geom&, hipStream_t);
