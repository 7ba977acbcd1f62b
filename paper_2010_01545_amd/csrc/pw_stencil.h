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

// Gather-form adjoint of one interior cell p at level k: the derivative of
// L = sum_c lu(c) su(c) + lv(c) sv(c) + lw(c) sw(c) with respect to u(p),
// v(p), w(p).  Each output term coef * A * (B + C) of a cell c that reads
// the field at p contributes lam(c) * coef * (B + C) when A sits at p and
// lam(c) * coef * A when B or C does; the sum below lists, for each of the
// eighteen terms of the scheme, every cell c = p - offset that reads p.
// A contribution is kept only when its term exists at c's level:
//   A1(q): 1 <= q <= nz-1   (su, sv terms with tcx, tcy, tzc1)
//   A2(q): 1 <= q <= nz-2   (su, sv tzc2 terms; every sw term)
// Masked contributions are selected away (never multiplied by zero), so
// z-halo values that are read but unused cannot leak NaN into the result.
// Contraction is off here too, so every kernel that uses this function
// (fused or not, direct or x-marching) rounds identically.
template <typename T>
__device__ __forceinline__ void pw_adj_cell(const Star<T>& u, const Star<T>& v, const Star<T>& w,
                                            const Star<T>& lu, const Star<T>& lv, const Star<T>& lw,
                                            const LevelCoef<T>& cf, int k, int nz,
                                            T& gu, T& gv, T& gw)
{
#pragma clang fp contract(off)
    const T tcx = cf.tcx, tcy = cf.tcy;
    const bool a1k = (k >= 1);                 // A1(k)
    const bool a2k = (k >= 1) && (k <= nz - 2); // A2(k)
    const bool a1kp = (k <= nz - 2);           // A1(k+1)
    const bool a2km = (k >= 2);                // A2(k-1)
    const bool a2kp = (k <= nz - 3);           // A2(k+1) (k+1 >= 1 always)
    const T zero = T(0);
    T g, t;

    // ---- d L / d u(p)
    g = zero;
    // su, +tcx u(c-x)(u(c)+u(c-x)):  c = p+x (A and C), c = p (B)
    t = tcx * (lu.xp * (u.xp + u.c) + lu.c * u.xm + lu.xp * u.c);
    g += a1k ? t : zero;
    // su, -tcx u(c+x)(u(c)+u(c+x)):  c = p-x (A and C), c = p (B)
    t = tcx * (lu.xm * (u.xm + u.c) + lu.c * u.xp + lu.xm * u.c);
    g -= a1k ? t : zero;
    // su, +tcy u(c-y)(v(c-y)+v(c+x-y)): A at p, c = p+y
    t = tcy * (lu.yp * (v.c + v.xp));
    g += a1k ? t : zero;
    // su, -tcy u(c+y)(v(c)+v(c+x)): A at p, c = p-y
    t = tcy * (lu.ym * (v.ym + v.d1));
    g -= a1k ? t : zero;
    // su, +tzc1 u(c-z)(w(c-z)+w(c+x-z)): A at p, c = p+z
    t = cf.t1kp * (lu.zp * (w.c + w.xp));
    g += a1kp ? t : zero;
    // su, -tzc2 u(c+z)(w(c)+w(c+x)): A at p, c = p-z
    t = cf.t2km * (lu.zm * (w.zm + w.d1));
    g -= a2km ? t : zero;
    // sv, +tcx v(c-x)(u(c-x)+u(c-x+y)): B at p (c = p+x), C at p (c = p+x-y)
    t = tcx * (lv.xp * v.c + lv.d1 * v.ym);
    g += a1k ? t : zero;
    // sv, -tcx v(c+x)(u(c)+u(c+y)): B at p (c = p), C at p (c = p-y)
    t = tcx * (lv.c * v.xp + lv.ym * v.d1);
    g -= a1k ? t : zero;
    // sw, +tcx w(c-x)(u(c-x)+u(c-x+z)): B at p (c = p+x), C at p (c = p+x-z)
    t = tcx * (a2k ? lw.xp * w.c : zero) + tcx * (a2km ? lw.d1 * w.zm : zero);
    g += t;
    // sw, -tcx w(c+x)(u(c)+u(c+z)): B at p (c = p), C at p (c = p-z)
    t = tcx * (a2k ? lw.c * w.xp : zero) + tcx * (a2km ? lw.zm * w.d1 : zero);
    g -= t;
    gu = g;

    // ---- d L / d v(p)
    g = zero;
    // sv, +tcy v(c-y)(v(c)+v(c-y)): c = p+y (A and C), c = p (B)
    t = tcy * (lv.yp * (v.yp + v.c) + lv.c * v.ym + lv.yp * v.c);
    g += a1k ? t : zero;
    // sv, -tcy v(c+y)(v(c)+v(c+y)): c = p-y (A and C), c = p (B)
    t = tcy * (lv.ym * (v.ym + v.c) + lv.c * v.yp + lv.ym * v.c);
    g -= a1k ? t : zero;
    // sv, +tcx v(c-x)(u(c-x)+u(c-x+y)): A at p, c = p+x
    t = tcx * (lv.xp * (u.c + u.yp));
    g += a1k ? t : zero;
    // sv, -tcx v(c+x)(u(c)+u(c+y)): A at p, c = p-x
    t = tcx * (lv.xm * (u.xm + u.d1));
    g -= a1k ? t : zero;
    // sv, +tzc1 v(c-z)(w(c-z)+w(c+y-z)): A at p, c = p+z
    t = cf.t1kp * (lv.zp * (w.c + w.yp));
    g += a1kp ? t : zero;
    // sv, -tzc2 v(c+z)(w(c)+w(c+y)): A at p, c = p-z
    t = cf.t2km * (lv.zm * (w.zm + w.d2));
    g -= a2km ? t : zero;
    // su, +tcy u(c-y)(v(c-y)+v(c+x-y)): B at p (c = p+y), C at p (c = p-x+y)
    t = tcy * (lu.yp * u.c + lu.d1 * u.xm);
    g += a1k ? t : zero;
    // su, -tcy u(c+y)(v(c)+v(c+x)): B at p (c = p), C at p (c = p-x)
    t = tcy * (lu.c * u.yp + lu.xm * u.d1);
    g -= a1k ? t : zero;
    // sw, +tcy w(c-y)(v(c-y)+v(c-y+z)): B at p (c = p+y), C at p (c = p+y-z)
    t = tcy * (a2k ? lw.yp * w.c : zero) + tcy * (a2km ? lw.d2 * w.zm : zero);
    g += t;
    // sw, -tcy w(c+y)(v(c)+v(c+z)): B at p (c = p), C at p (c = p-z)
    t = tcy * (a2k ? lw.c * w.yp : zero) + tcy * (a2km ? lw.zm * w.d2 : zero);
    g -= t;
    gv = g;

    // ---- d L / d w(p)
    g = zero;
    // su, +tzc1 u(c-z)(w(c-z)+w(c+x-z)): B at p (c = p+z), C at p (c = p-x+z)
    t = cf.t1kp * (lu.zp * u.c + lu.d2 * u.xm);
    g += a1kp ? t : zero;
    // su, -tzc2 u(c+z)(w(c)+w(c+x)): B at p (c = p), C at p (c = p-x)
    t = cf.t2k * (lu.c * u.zp + lu.xm * u.d2);
    g -= a2k ? t : zero;
    // sv, +tzc1 v(c-z)(w(c-z)+w(c+y-z)): B at p (c = p+z), C at p (c = p-y+z)
    t = cf.t1kp * (lv.zp * v.c + lv.d2 * v.ym);
    g += a1kp ? t : zero;
    // sv, -tzc2 v(c+z)(w(c)+w(c+y)): B at p (c = p), C at p (c = p-y)
    t = cf.t2k * (lv.c * v.zp + lv.ym * v.d2);
    g -= a2k ? t : zero;
    // sw, +tcx w(c-x)(u(c-x)+u(c-x+z)): A at p, c = p+x
    t = tcx * (lw.xp * (u.c + u.zp));
    g += a2k ? t : zero;
    // sw, -tcx w(c+x)(u(c)+u(c+z)): A at p, c = p-x
    t = tcx * (lw.xm * (u.xm + u.d2));
    g -= a2k ? t : zero;
    // sw, +tcy w(c-y)(v(c-y)+v(c-y+z)): A at p, c = p+y
    t = tcy * (lw.yp * (v.c + v.zp));
    g += a2k ? t : zero;
    // sw, -tcy w(c+y)(v(c)+v(c+z)): A at p, c = p-y
    t = tcy * (lw.ym * (v.ym + v.d2));
    g -= a2k ? t : zero;
    // sw, +tzc1 w(c-z)(w(c)+w(c-z)): A and C at p (c = p+z), B at p (c = p)
    t = cf.t1kp * (lw.zp * (w.zp + w.c) + lw.zp * w.c);
    g += a2kp ? t : zero;
    t = cf.t1k * (lw.c * w.zm);
    g += a2k ? t : zero;
    // sw, -tzc2 w(c+z)(w(c)+w(c+z)): A and C at p (c = p-z), B at p (c = p)
    t = cf.t2km * (lw.zm * (w.zm + w.c) + lw.zm * w.c);
    g -= a2km ? t : zero;
    t = cf.t2k * (lw.c * w.zp);
    g -= a2k ? t : zero;
    gw = g;
}
