/*
 * pw_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of the Piacsek-Williams
 * (PW) momentum-advection source terms of the MONC model, written from the
 * paper "Exploring the acceleration of the Met Office NERC Cloud model using
 * FPGAs" (N. Brown), section 2.1 and Listing 1.  It exists to check the HIP
 * library; nothing in the product path may call it.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * It shares no code with the GPU library: no headers, helpers or tables.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (and the same source with -fopenmp for the multithreaded host baseline;
 * only the forward loop carries an OpenMP pragma, and every output cell is
 * computed by exactly one thread, so both builds give bitwise equal results).
 *
 * Layout (section 3, Listings 3 and 4, where one memcpy moves a whole column
 * and then consecutive y-columns): every field is a C-contiguous storage array
 * of shape (nx+2h, ny+2h, nz+2h), z fastest, i.e. Fortran F(k,j,i).  Interior
 * cell (i,j,k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, lives at storage index
 * ((i+h)*(ny+2h) + (j+h))*(nz+2h) + (k+h).  Halos are filled by the caller.
 *
 * Readings of the paper used here (the paper prints only su):
 *   - Fortran k = 2..z_size becomes 0-based k = 1..nz-1; level 0 is set to 0.
 *   - su is assigned, not accumulated.
 *   - sv is the x<->y transpose analogue of su; sw follows the same
 *     "upwind value times face sum of the advecting velocity" rule with the
 *     tzc1/tzc2 profiles, on levels 1..nz-2, and is 0 on levels 0 and nz-1.
 *   - Evaluation follows Fortran's left-to-right association of Listing 1.
 * Parity of sv and sw against MONC itself is unpinned (MONC's sv/sw code is
 * not in the paper); they are pinned by hand values, symmetries and PW energy
 * conservation instead.
 */
#include <stddef.h>
#include <math.h>

/* storage index of interior coordinates (i, j, k); i, j may be -h..n+h-1 */
#define SIDX(i, j, k) \
    ((((size_t)((i) + h) * (size_t)(ny + 2 * h)) + (size_t)((j) + h)) * (size_t)(nz + 2 * h) + (size_t)((k) + h))

/*
 * Forward source terms, Listing 1 (su) and the omitted sv, sw (section 2.1).
 * Writes every interior cell of su, sv, sw; halo cells are not touched.
 */
void pw_oracle_fwd(const double *u, const double *v, const double *w,
                   const double *tzc1, const double *tzc2, double tcx, double tcy,
                   int nx, int ny, int nz, int h,
                   double *su, double *sv, double *sw)
{
    int i;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (i = 0; i < nx; i++) {
        int j, k;
        for (j = 0; j < ny; j++) {
            for (k = 0; k < nz; k++) {
                size_t c = SIDX(i, j, k);
                double s;
                if (k == 0) {
                    su[c] = 0.0;
                    sv[c] = 0.0;
                    sw[c] = 0.0;
                    continue;
                }
                /* su: x self-advection, y term with v face sums at i+1/2,
                 * z term with w face sums; the top level drops tzc2 (Listing 1) */
                s = tcx * (u[SIDX(i - 1, j, k)] * (u[c] + u[SIDX(i - 1, j, k)])
                           - u[SIDX(i + 1, j, k)] * (u[c] + u[SIDX(i + 1, j, k)]));
                s = s + tcy * (u[SIDX(i, j - 1, k)] * (v[SIDX(i, j - 1, k)] + v[SIDX(i + 1, j - 1, k)])
                               - u[SIDX(i, j + 1, k)] * (v[c] + v[SIDX(i + 1, j, k)]));
                if (k < nz - 1) {
                    s = s + tzc1[k] * u[SIDX(i, j, k - 1)] * (w[SIDX(i, j, k - 1)] + w[SIDX(i + 1, j, k - 1)])
                          - tzc2[k] * u[SIDX(i, j, k + 1)] * (w[c] + w[SIDX(i + 1, j, k)]);
                } else {
                    s = s + tzc1[k] * u[SIDX(i, j, k - 1)] * (w[SIDX(i, j, k - 1)] + w[SIDX(i + 1, j, k - 1)]);
                }
                su[c] = s;

                /* sv: the same scheme for v, staggered at j+1/2 */
                s = tcx * (v[SIDX(i - 1, j, k)] * (u[SIDX(i - 1, j, k)] + u[SIDX(i - 1, j + 1, k)])
                           - v[SIDX(i + 1, j, k)] * (u[c] + u[SIDX(i, j + 1, k)]));
                s = s + tcy * (v[SIDX(i, j - 1, k)] * (v[c] + v[SIDX(i, j - 1, k)])
                               - v[SIDX(i, j + 1, k)] * (v[c] + v[SIDX(i, j + 1, k)]));
                if (k < nz - 1) {
                    s = s + tzc1[k] * v[SIDX(i, j, k - 1)] * (w[SIDX(i, j, k - 1)] + w[SIDX(i, j + 1, k - 1)])
                          - tzc2[k] * v[SIDX(i, j, k + 1)] * (w[c] + w[SIDX(i, j + 1, k)]);
                } else {
                    s = s + tzc1[k] * v[SIDX(i, j, k - 1)] * (w[SIDX(i, j, k - 1)] + w[SIDX(i, j + 1, k - 1)]);
                }
                sv[c] = s;

                /* sw: the same scheme for w, staggered at k+1/2; zero on both lids */
                if (k == nz - 1) {
                    sw[c] = 0.0;
                    continue;
                }
                s = tcx * (w[SIDX(i - 1, j, k)] * (u[SIDX(i - 1, j, k)] + u[SIDX(i - 1, j, k + 1)])
                           - w[SIDX(i + 1, j, k)] * (u[c] + u[SIDX(i, j, k + 1)]));
                s = s + tcy * (w[SIDX(i, j - 1, k)] * (v[SIDX(i, j - 1, k)] + v[SIDX(i, j - 1, k + 1)])
                               - w[SIDX(i, j + 1, k)] * (v[c] + v[SIDX(i, j, k + 1)]));
                s = s + tzc1[k] * w[SIDX(i, j, k - 1)] * (w[c] + w[SIDX(i, j, k - 1)])
                      - tzc2[k] * w[SIDX(i, j, k + 1)] * (w[c] + w[SIDX(i, j, k + 1)]);
                sw[c] = s;
            }
        }
    }
}

/*
 * Rounding-error magnitude companion of pw_oracle_fwd: the same sums with
 * every coefficient and field value replaced by its absolute value, i.e.
 * T(c) = sum over terms |coef| |A| (|B| + |C|).  A computation of s(c) in a
 * precision with unit roundoff eps that rounds each operation once has error
 * at most about (number of operations on the longest path) * eps * T(c).
 */
void pw_oracle_fwd_abs(const double *u, const double *v, const double *w,
                       const double *tzc1, const double *tzc2, double tcx, double tcy,
                       int nx, int ny, int nz, int h,
                       double *tu, double *tv, double *tw)
{
    int i, j, k;
    double ax = fabs(tcx), ay = fabs(tcy);
#define A(F, ii, jj, kk) fabs(F[SIDX(ii, jj, kk)])
    for (i = 0; i < nx; i++) {
        for (j = 0; j < ny; j++) {
            for (k = 0; k < nz; k++) {
                size_t c = SIDX(i, j, k);
                double t;
                if (k == 0) {
                    tu[c] = tv[c] = tw[c] = 0.0;
                    continue;
                }
                t = ax * (A(u, i - 1, j, k) * (A(u, i, j, k) + A(u, i - 1, j, k))
                          + A(u, i + 1, j, k) * (A(u, i, j, k) + A(u, i + 1, j, k)));
                t += ay * (A(u, i, j - 1, k) * (A(v, i, j - 1, k) + A(v, i + 1, j - 1, k))
                           + A(u, i, j + 1, k) * (A(v, i, j, k) + A(v, i + 1, j, k)));
                t += fabs(tzc1[k]) * A(u, i, j, k - 1) * (A(w, i, j, k - 1) + A(w, i + 1, j, k - 1));
                if (k < nz - 1)
                    t += fabs(tzc2[k]) * A(u, i, j, k + 1) * (A(w, i, j, k) + A(w, i + 1, j, k));
                tu[c] = t;

                t = ax * (A(v, i - 1, j, k) * (A(u, i - 1, j, k) + A(u, i - 1, j + 1, k))
                          + A(v, i + 1, j, k) * (A(u, i, j, k) + A(u, i, j + 1, k)));
                t += ay * (A(v, i, j - 1, k) * (A(v, i, j, k) + A(v, i, j - 1, k))
                           + A(v, i, j + 1, k) * (A(v, i, j, k) + A(v, i, j + 1, k)));
                t += fabs(tzc1[k]) * A(v, i, j, k - 1) * (A(w, i, j, k - 1) + A(w, i, j + 1, k - 1));
                if (k < nz - 1)
                    t += fabs(tzc2[k]) * A(v, i, j, k + 1) * (A(w, i, j, k) + A(w, i, j + 1, k));
                tv[c] = t;

                if (k == nz - 1) {
                    tw[c] = 0.0;
                    continue;
                }
                t = ax * (A(w, i - 1, j, k) * (A(u, i - 1, j, k) + A(u, i - 1, j, k + 1))
                          + A(w, i + 1, j, k) * (A(u, i, j, k) + A(u, i, j, k + 1)));
                t += ay * (A(w, i, j - 1, k) * (A(v, i, j - 1, k) + A(v, i, j - 1, k + 1))
                           + A(w, i, j + 1, k) * (A(v, i, j, k) + A(v, i, j, k + 1)));
                t += fabs(tzc1[k]) * A(w, i, j, k - 1) * (A(w, i, j, k) + A(w, i, j, k - 1));
                t += fabs(tzc2[k]) * A(w, i, j, k + 1) * (A(w, i, j, k) + A(w, i, j, k + 1));
                tw[c] = t;
            }
        }
    }
#undef A
}

/*
 * Adjoint (vector-Jacobian product) in scatter form.
 *
 * Every output is a sum of terms  coef * A * (B + C)  (the terms of Listing 1
 * and of the sv, sw readings above).  For the loss L = sum over interior cells
 * of lu*su + lv*sv + lw*sw, each term of output cell c adds
 *     dL/dA += l(c) * coef * (B + C),  dL/dB += l(c) * coef * A,
 *     dL/dC += l(c) * coef * A
 * to the storage cell holding that operand.  The storage arrays gu, gv, gw
 * (same shape as the fields) are zeroed first and receive these sums,
 * including contributions that land on x/y halo cells.
 *
 * The inputs are the interior fields of a problem that is periodic in x and y:
 * halos are copies of interior cells, so the gradient with respect to an
 * interior value is the sum over that value and all its halo copies.  After
 * the scatter, pw_oracle_fold_periodic adds each halo cell into its periodic
 * image and clears the halo.
 */
static int g_abs_mode = 0; /* set only by pw_oracle_adj_abs */

static void term(double *gA, size_t a, double *gB, size_t b, double *gC, size_t cc,
                 const double *fA, const double *fB, const double *fC,
                 double lam, double coef)
{
    double A = fA[a], B = fB[b], C = fC[cc];
    if (g_abs_mode) {
        A = fabs(A);
        B = fabs(B);
        C = fabs(C);
        lam = fabs(lam);
        coef = fabs(coef);
    }
    gA[a] += lam * coef * (B + C);
    gB[b] += lam * coef * A;
    gC[cc] += lam * coef * A;
}

void pw_oracle_fold_periodic(double *g, int nx, int ny, int nz, int h);

void pw_oracle_adj(const double *u, const double *v, const double *w,
                   const double *lu, const double *lv, const double *lw,
                   const double *tzc1, const double *tzc2, double tcx, double tcy,
                   int nx, int ny, int nz, int h,
                   double *gu, double *gv, double *gw)
{
    size_t n = (size_t)(nx + 2 * h) * (size_t)(ny + 2 * h) * (size_t)(nz + 2 * h);
    size_t q;
    int i, j, k;
    for (q = 0; q < n; q++) {
        gu[q] = 0.0;
        gv[q] = 0.0;
        gw[q] = 0.0;
    }
    for (i = 0; i < nx; i++) {
        for (j = 0; j < ny; j++) {
            for (k = 1; k < nz; k++) {
                size_t c = SIDX(i, j, k);
                double l;
                /* su terms (levels 1..nz-1; tzc2 term only below the top) */
                l = lu[c];
                term(gu, SIDX(i - 1, j, k), gu, c, gu, SIDX(i - 1, j, k), u, u, u, l, tcx);
                term(gu, SIDX(i + 1, j, k), gu, c, gu, SIDX(i + 1, j, k), u, u, u, l, -tcx);
                term(gu, SIDX(i, j - 1, k), gv, SIDX(i, j - 1, k), gv, SIDX(i + 1, j - 1, k), u, v, v, l, tcy);
                term(gu, SIDX(i, j + 1, k), gv, c, gv, SIDX(i + 1, j, k), u, v, v, l, -tcy);
                term(gu, SIDX(i, j, k - 1), gw, SIDX(i, j, k - 1), gw, SIDX(i + 1, j, k - 1), u, w, w, l, tzc1[k]);
                if (k < nz - 1)
                    term(gu, SIDX(i, j, k + 1), gw, c, gw, SIDX(i + 1, j, k), u, w, w, l, -tzc2[k]);

                /* sv terms */
                l = lv[c];
                term(gv, SIDX(i - 1, j, k), gu, SIDX(i - 1, j, k), gu, SIDX(i - 1, j + 1, k), v, u, u, l, tcx);
                term(gv, SIDX(i + 1, j, k), gu, c, gu, SIDX(i, j + 1, k), v, u, u, l, -tcx);
                term(gv, SIDX(i, j - 1, k), gv, c, gv, SIDX(i, j - 1, k), v, v, v, l, tcy);
                term(gv, SIDX(i, j + 1, k), gv, c, gv, SIDX(i, j + 1, k), v, v, v, l, -tcy);
                term(gv, SIDX(i, j, k - 1), gw, SIDX(i, j, k - 1), gw, SIDX(i, j + 1, k - 1), v, w, w, l, tzc1[k]);
                if (k < nz - 1)
                    term(gv, SIDX(i, j, k + 1), gw, c, gw, SIDX(i, j + 1, k), v, w, w, l, -tzc2[k]);

                /* sw terms (levels 1..nz-2 only) */
                if (k == nz - 1)
                    continue;
                l = lw[c];
                term(gw, SIDX(i - 1, j, k), gu, SIDX(i - 1, j, k), gu, SIDX(i - 1, j, k + 1), w, u, u, l, tcx);
                term(gw, SIDX(i + 1, j, k), gu, c, gu, SIDX(i, j, k + 1), w, u, u, l, -tcx);
                term(gw, SIDX(i, j - 1, k), gv, SIDX(i, j - 1, k), gv, SIDX(i, j - 1, k + 1), w, v, v, l, tcy);
                term(gw, SIDX(i, j + 1, k), gv, c, gv, SIDX(i, j, k + 1), w, v, v, l, -tcy);
                term(gw, SIDX(i, j, k - 1), gw, c, gw, SIDX(i, j, k - 1), w, w, w, l, tzc1[k]);
                term(gw, SIDX(i, j, k + 1), gw, c, gw, SIDX(i, j, k + 1), w, w, w, l, -tzc2[k]);
            }
        }
    }
    pw_oracle_fold_periodic(gu, nx, ny, nz, h);
    pw_oracle_fold_periodic(gv, nx, ny, nz, h);
    pw_oracle_fold_periodic(gw, nx, ny, nz, h);
}

/*
 * Transpose of the periodic halo fill in x and y: every storage column outside
 * the interior is added into the interior column it is a copy of, then
 * cleared.  z-halo levels are never read by the scheme and are cleared.
 */
void pw_oracle_fold_periodic(double *g, int nx, int ny, int nz, int h)
{
    int si, sj, k;
    int sx = nx + 2 * h, sy = ny + 2 * h, sz = nz + 2 * h;
    for (si = 0; si < sx; si++) {
        for (sj = 0; sj < sy; sj++) {
            int i = si - h, j = sj - h;
            int ii = ((i % nx) + nx) % nx, jj = ((j % ny) + ny) % ny;
            int interior = (i == ii && j == jj);
            for (k = -h; k < nz + h; k++) {
                size_t s = ((size_t)si * (size_t)sy + (size_t)sj) * (size_t)sz + (size_t)(k + h);
                if (k < 0 || k >= nz) {
                    g[s] = 0.0;
                    continue;
                }
                if (!interior) {
                    g[SIDX(ii, jj, k)] += g[s];
                    g[s] = 0.0;
                }
            }
        }
    }
}

/*
 * Rounding-error magnitude companion of pw_oracle_adj: the same scatter and
 * fold with every coefficient, multiplier and field value replaced by its
 * absolute value, i.e. for each gradient entry the sum of the absolute values
 * of all the products that make it up.  Not thread-safe.
 */
void pw_oracle_adj_abs(const double *u, const double *v, const double *w,
                       const double *lu, const double *lv, const double *lw,
                       const double *tzc1, const double *tzc2, double tcx, double tcy,
                       int nx, int ny, int nz, int h,
                       double *gu, double *gv, double *gw)
{
    g_abs_mode = 1;
    pw_oracle_adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, nx, ny, nz, h, gu, gv, gw);
    g_abs_mode = 0;
}
