// pw_stencil.h -- per-cell arithmetic of the PW advection scheme and of its
// gather-form adjoint, shared by every kernel of the library so that each
// expression tree exists once.
//
// Forward: su follows Listing 1 of section 2.1 with Fortran's left-to-right
// association; sv is its x<->y transpose analogue; sw is the same
// upwind-value-times-face-sum scheme staggered in z (levels 1..nz-2).
// FP contraction is switched off inside these functions: the FP64 forward
// then rounds exactly like a plain evaluation of that expression, and every
// kernel variant gives bitwise identical results.
//
// Operands come as "stars": the value at the cell, its six face neighbours
// and two diagonal neighbours whose position depends on the field:
//   u (staggered at i+1/2): d1 = (i-1, j+1, k), d2 = (i-1, j, k+1)
//   v (staggered at j+1/2): d1 = (i+1, j-1, k), d2 = (i, j-1, k+1)
//   w (staggered at k+1/2): d1 = (i+1, j, k-1), d2 = (i, j+1, k-1)
// The adjoint multipliers lu, lv, lw use the same diagonals as u, v, w.
#pragma once

template <typename T>
struct Star {
    T c, xm, xp, ym, yp, zm, zp, d1, d2;
};

// Coefficients seen by one cell at interior level k.
template <typename T>
struct LevelCoef {
    T tcx, tcy;
    T t1k, t2k;    // tzc1[k], tzc2[k]
    T t1kp, t2km;  // tzc1[k+1] (k+1 <= nz-1), tzc2[k-1] (k >= 1); else unused
};

template <typename T>
__device__ __forceinline__ LevelCoef<T> level_coef(const double* __restrict__ tzc1,
                                                   const double* __restrict__ tzc2,
                                                   T tcx, T tcy, int k, int nz)
{
    LevelCoef<T> c;
    c.tcx = tcx;
    c.tcy = tcy;
    c.t1k = (T)tzc1[k];
    c.t2k = (T)tzc2[k];
    c.t1kp = (T)tzc1[k + 1 < nz ? k + 1 : nz - 1];
    c.t2km = (T)tzc2[k > 0 ? k - 1 : 0];
    return c;
}

// Forward source terms of one interior cell at level k (0 <= k < nz).
template <typename T>
__device__ __forceinline__ void pw_fwd_cell(const Star<T>& u, const Star<T>& v, const Star<T>& w,
                                            const LevelCoef<T>& cf, int k, int nz,
                                            T& su, T& sv, T& sw)
{
#pragma clang fp contract(off)
    const bool top = (k == nz - 1);
    T s;
    // su
    s = cf.tcx * (u.xm * (u.c + u.xm) - u.xp * (u.c + u.xp));
    s = s + cf.tcy * (u.ym * (v.ym + v.d1) - u.yp * (v.c + v.xp));
    s = s + (cf.t1k * u.zm) * (w.zm + w.d1);
    if (!top) s = s - (cf.t2k * u.zp) * (w.c + w.xp);
    su = (k == 0) ? T(0) : s;
    // sv
    s = cf.tcx * (v.xm * (u.xm + u.d1) - v.xp * (u.c + u.yp));
    s = s + cf.tcy * (v.ym * (v.c + v.ym) - v.yp * (v.c + v.yp));
    s = s + (cf.t1k * v.zm) * (w.zm + w.d2);
    if (!top) s = s - (cf.t2k * v.zp) * (w.c + w.yp);
    sv = (k == 0) ? T(0) : s;
    // sw
    s = cf.tcx * (w.xm * (u.xm + u.d2) - w.xp * (u.c + u.zp));
    s = s + cf.tcy * (w.ym * (v.ym + v.d2) - w.yp * (v.c + v.zp));
    s = (s + (cf.t1k * w.zm) * (w.c + w.zm)) - (cf.t2k * w.zp) * (w.c + w.zp);
    sw = (k == 0 || top) ? T(0) : s;
}

// One rounding: a * b + c.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The forward in float arithmetic: the same terms and operands as
// pw_fwd_cell, with each "A (B + C) - D (E + F)" pair and each accumulation
// written as explicit fused multiply-adds (16 operations per source term
// instead of 21; fewer roundings, so within the same error bound).  Float
// kernels are instruction-bound where the FP64 ones are memory-bound, and the
// explicit form keeps every kernel variant bit-identical.
template <typename T>
__device__ __forceinline__ void pw_fwd_cell_fma(const Star<T>& u, const Star<T>& v, const Star<T>& w,
                                                const LevelCoef<T>& cf, int k, int nz,
                                                T& su, T& sv, T& sw)
{
#pragma clang fp contract(off)
    const bool top = (k == nz - 1);
    T s, x, y;
    // su
    x = fmad(u.xm, u.c + u.xm, -(u.xp * (u.c + u.xp)));
    y = fmad(u.ym, v.ym + v.d1, -(u.yp * (v.c + v.xp)));
    s = fmad(cf.tcy, y, cf.tcx * x);
    s = fmad(cf.t1k * u.zm, w.zm + w.d1, s);
    if (!top) s = fmad(-(cf.t2k * u.zp), w.c + w.xp, s);
    su = (k == 0) ? T(0) : s;
    // sv
    x = fmad(v.xm, u.xm + u.d1, -(v.xp * (u.c + u.yp)));
    y = fmad(v.ym, v.c + v.ym, -(v.yp * (v.c + v.yp)));
    s = fmad(cf.tcy, y, cf.tcx * x);
    s = fmad(cf.t1k * v.zm, w.zm + w.d2, s);
    if (!top) s = fmad(-(cf.t2k * v.zp), w.c + w.yp, s);
    sv = (k == 0) ? T(0) : s;
    // sw
    x = fmad(w.xm, u.xm + u.d2, -(w.xp * (u.c + u.zp)));
    y = fmad(w.ym, v.ym + v.d2, -(w.yp * (v.c + v.zp)));
    s = fmad(cf.tcy, y, cf.tcx * x);
    s = fmad(cf.t1k * w.zm, w.c + w.zm, s);
    s = fmad(-(cf.t2k * w.zp), w.c + w.zp, s);
    sw = (k == 0 || top) ? T(0) : s;
}

// The forward the kernels use for arithmetic type T: the plain tree for
// FP64 (bitwise equal to a direct evaluation of Listing 1), the FMA form for
// float.
template <typename T>
__device__ __forceinline__ void pw_fwd(const Star<T>& u, const Star<T>& v, const Star<T>& w,
                                       const LevelCoef<T>& cf, int k, int nz, T& su, T& sv, T& sw)
{
    if constexpr (sizeof(T) == 4)
        pw_fwd_cell_fma(u, v, w, cf, k, nz, su, sv, sw);
    else
        pw_fwd_cell(u, v, w, cf, k, nz, su, sv, sw);
}

// Level masks of the adjoint multipliers.  A term of output cell c exists
// only on c's level range: su, sv terms with tcx, tcy, tzc1 on 1..nz-1; the
// su, sv tzc2 terms and every sw term on 1..nz-2.  The kernels store the
// multipliers with these ranges applied (lu, lv zero on level 0; lw zero on
// levels 0 and nz-1; any operand outside 0..nz-1 zero), which encodes every
// term's range except that of the su, sv tzc2 terms read at the cell's own
// level; pw_adj_cell applies that one through the tzc2[k] coefficient.
__device__ __forceinline__ bool lam_uv_live(int level, int nz) { return level >= 1 && level <= nz - 1; }
__device__ __forceinline__ bool lam_w_live(int level, int nz) { return level >= 1 && level <= nz - 2; }

// Gather-form adjoint of one interior cell p at level k: the derivative of
// L = sum_c lu(c) su(c) + lv(c) sv(c) + lw(c) sw(c) with respect to u(p),
// v(p), w(p).  Each output term coef * A * (B + C) of a cell c that reads
// the field at p contributes lam(c) * coef * (B + C) when A sits at p and
// lam(c) * coef * A when B or C does.  Below, for each coefficient, the
// contributions of all cells c = p - offset that read p are summed (with A
// and C coinciding in the self-advection terms, giving the 2 * F(p) sums);
// the bracket names the output term and the operand that sits at p.
// The multipliers must carry the level masks described above.  Evaluation
// uses explicit fused multiply-adds in a fixed order, so every kernel that
// calls this function produces the same bits.
template <typename T>
__device__ __forceinline__ void pw_adj_cell(const Star<T>& u, const Star<T>& v, const Star<T>& w,
                                            const Star<T>& lu, const Star<T>& lv, const Star<T>& lw,
                                            const LevelCoef<T>& cf, int k, int nz,
                                            T& gu, T& gv, T& gw)
{
#pragma clang fp contract(off)
    const T two = T(2);
    // tzc2[k] multiplies only terms of cells at level k, where the su, sv
    // tzc2 terms need k <= nz-2 (the sw terms are masked through lw)
    const T t2k = (k <= nz - 2) ? cf.t2k : T(0);
    T x, y, z1, z2;

    // ---- d L / d u(p)
    // tcx: su x term (A, C at c = p+x; B at c = p) minus its mirror at p-x,
    //      sv x terms (B at c = p+x / p; C at c = p+x-y / p-y),
    //      sw x terms (B at c = p+x / p; C at c = p+x-z / p-z);
    // three independent partial sums, then combined
    x = lu.xp * fmad(two, u.c, u.xp);
    x = fmad(lu.c, u.xm, x);
    x = fmad(-lu.xm, fmad(two, u.c, u.xm), x);
    x = fmad(-lu.c, u.xp, x);
    y = lv.xp * v.c;
    y = fmad(lv.d1, v.ym, y);
    y = fmad(-lv.c, v.xp, y);
    y = fmad(-lv.ym, v.d1, y);
    z1 = lw.xp * w.c;
    z1 = fmad(lw.d1, w.zm, z1);
    z1 = fmad(-lw.c, w.xp, z1);
    z1 = fmad(-lw.zm, w.d1, z1);
    const T xu = (x + y) + z1;
    // tcy: su y terms, A at c = p+y and c = p-y
    y = lu.yp * (v.c + v.xp);
    y = fmad(-lu.ym, v.ym + v.d1, y);
    // tzc1[k+1]: su z term, A at c = p+z;  tzc2[k-1]: A at c = p-z
    z1 = lu.zp * (w.c + w.xp);
    z2 = lu.zm * (w.zm + w.d1);
    gu = fmad(cf.tcx, xu, fmad(cf.tcy, y, fmad(cf.t1kp, z1, -(cf.t2km * z2))));

    // ---- d L / d v(p)
    // tcy: sv y term (A, C at c = p+y; B at c = p) minus its mirror at p-y,
    //      su y terms (B at c = p+y / p; C at c = p-x+y / p-x),
    //      sw y terms (B at c = p+y / p; C at c = p+y-z / p-z)
    x = lv.yp * fmad(two, v.c, v.yp);
    x = fmad(lv.c, v.ym, x);
    x = fmad(-lv.ym, fmad(two, v.c, v.ym), x);
    x = fmad(-lv.c, v.yp, x);
    y = lu.yp * u.c;
    y = fmad(lu.d1, u.xm, y);
    y = fmad(-lu.c, u.yp, y);
    y = fmad(-lu.xm, u.d1, y);
    z1 = lw.yp * w.c;
    z1 = fmad(lw.d2, w.zm, z1);
    z1 = fmad(-lw.c, w.yp, z1);
    z1 = fmad(-lw.zm, w.d2, z1);
    const T yv = (x + y) + z1;
    // tcx: sv x terms, A at c = p+x and c = p-x
    x = lv.xp * (u.c + u.yp);
    x = fmad(-lv.xm, u.xm + u.d1, x);
    // tzc1[k+1]: sv z term, A at c = p+z;  tzc2[k-1]: A at c = p-z
    z1 = lv.zp * (w.c + w.yp);
    z2 = lv.zm * (w.zm + w.d2);
    gv = fmad(cf.tcy, yv, fmad(cf.tcx, x, fmad(cf.t1kp, z1, -(cf.t2km * z2))));

    // ---- d L / d w(p)
    // tzc1[k+1]: su, sv z terms (B at c = p+z; C at c = p-x+z / p-y+z),
    //            sw z term (A, C at c = p+z)
    z1 = lu.zp * u.c;
    z1 = fmad(lu.d2, u.xm, z1);
    x = lv.zp * v.c;
    x = fmad(lv.d2, v.ym, x);
    z1 = fmad(lw.zp, fmad(two, w.c, w.zp), z1) + x;
    // tzc2[k]: su, sv z terms (B at c = p; C at c = p-x / p-y), sw z term (B at c = p)
    z2 = lu.c * u.zp;
    z2 = fmad(lu.xm, u.d2, z2);
    y = lv.c * v.zp;
    y = fmad(lv.ym, v.d2, y);
    z2 = fmad(lw.c, w.zp, z2) + y;
    // tcx, tcy: sw x and y terms, A at c = p+x / p-x and p+y / p-y
    x = lw.xp * (u.c + u.zp);
    x = fmad(-lw.xm, u.xm + u.d2, x);
    y = lw.yp * (v.c + v.zp);
    y = fmad(-lw.ym, v.ym + v.d2, y);
    // tzc1[k]: sw z term, B at c = p;  tzc2[k-1]: sw z term, A and C at c = p-z
    T g = fmad(cf.t1kp, z1, -(t2k * z2));
    g = fmad(cf.tcx, x, g);
    g = fmad(cf.tcy, y, g);
    g = fmad(cf.t1k, lw.c * w.zm, g);
    gw = fmad(-cf.t2km, lw.zm * fmad(two, w.c, w.zm), g);
}

// Use of a source term in the timestep (the integration that follows the
// dynamical core, section 2.1): base + beta * s, with the product and the sum
// each rounded (no fused multiply-add), so that the result is the plain
// two-operation expression.
template <typename T>
__device__ __forceinline__ T pw_update(T base, T beta, T s)
{
#pragma clang fp contract(off)
    const T t = beta * s;
    return base + t;
}
