/*
 * CPU oracle for the FIt-SNE per-iteration gradient (Linderman et al.,
 * "Efficient Algorithms for t-distributed Stochastic Neighborhood Embedding").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 statement of
 * what the GPU library must compute.  It shares no code, header, table or
 * constant generator with the GPU library and is used only by the tests, the
 * package's smoke check and the benchmark's CPU-baseline leg.
 *
 * Everything is double precision, no fast-math, no blocking or reordering of
 * sums beyond what the definitions state; OpenMP only splits independent
 * output rows.
 *
 * Parts:
 *   (1) direct sums: Z, the repulsive and attractive forces by their definitions
 *       (Section 1.1; Section 2, eq. (frep); Section 3);
 *   (2) the interpolation scheme with Step 2 done directly (Section 2.2 steps
 *       1-3 and Algorithm 1 without the FFT; Section 2.4 for s = 2; the
 *       Appendix for assembling the forces from the s+2 kernel sums);
 *   (3) the gradient-descent update (gradient of Section 1.1 with the
 *       exaggeration factor of Section 1.2 / Section 4; the step rule itself
 *       is not in the paper, see oracle_update).
 *
 * Readings of the paper used here (silent or inconsistent passages):
 *   - sign: F_rep,i = sum_j K2_ij (y_i - y_j) / Z, the sign of the
 *     attractive/repulsive split in Section 1.1, so that the gradient is
 *     4 (alpha F_attr - F_rep); eq. (frep) and the Appendix print the
 *     opposite sign;
 *   - the square box (Section 2.4) of side N_int w is centred on each
 *     dimension's mid-range; nodes of interval l sit at
 *     origin + (l p + m + 1/2) h, m = 0..p-1, the affine image of eq.
 *     (equinodes) on the box;
 *   - a point belongs to interval floor((y - origin)/w), clamped to
 *     [0, N_int - 1];
 *   - Z = sum_i h1_i - N K1(0): the grid sums include the self pair, whose
 *     exact kernel value K1(0) is removed (force numerators cancel the self
 *     pair identically);
 *   - charges are centred at the box centre (translation invariance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Kernel families.  ORACLE_KERNEL_TSNE is the pair of Section 2, eq. (kers):
 * K1 = 1/(1+r^2), K2 = K1^2.  ORACLE_KERNEL_POLY is a test family that keeps
 * the identity K1 = (1 + r^2) K2 but is polynomial (K2 of degree 2 and K1 of
 * degree 4 in each coordinate), so that interpolation with enough nodes per
 * interval is exact and the scheme must reproduce the direct sum to rounding. */
enum { ORACLE_KERNEL_TSNE = 0, ORACLE_KERNEL_POLY = 1 };
/* Charge sets: FORM_A follows the Appendix (K1 with charge 1, K2 with charges
 * 1 and y(d)); FORM_B uses K2 with charges 1, y(d) and |y|^2, and gets the K1
 * sum from K1 = (1 + r^2) K2. */
enum { ORACLE_FORM_A = 0, ORACLE_FORM_B = 1, ORACLE_FORM_V = 2 };
enum { ORACLE_POLICY_PAPER = 0, ORACLE_POLICY_FIXED = 1 };

static double kern1(int kind, double r2)
{
    if (kind == ORACLE_KERNEL_TSNE) return 1.0 / (1.0 + r2);
    return (1.0 + r2) * (2.0 + r2 / 8.0);
}

static double kern2(int kind, double r2)
{
    if (kind == ORACLE_KERNEL_TSNE) {
        double a = 1.0 / (1.0 + r2);
        return a * a;
    }
    return 2.0 + r2 / 8.0;
}

static double sqdist(int s, const double* a, const double* b)
{
    double r2 = 0.0;
    for (int d = 0; d < s; ++d) {
        double t = a[d] - b[d];
        r2 += t * t;
    }
    return r2;
}

/* ------------------------------------------------------------------------ */
/* (1) Direct sums                                                           */
/* ------------------------------------------------------------------------ */

/* Unnormalised per-point sums for the listed rows (all rows if rows == NULL):
 *   h1[r]      = sum_{j != i} K1(|y_i - y_j|^2)                 (Appendix, h1)
 *   num[r*s+d] = sum_{j != i} K2(|y_i - y_j|^2) (y_i(d) - y_j(d))  (eq. (frep)
 *                numerator with the Section 1.1 sign)
 * with i = rows[r].  Y is [n, s] row-major. */
void oracle_direct_sums(int64_t n, int s, const double* Y, int kind,
                        const int64_t* rows, int64_t nrows,
                        double* h1, double* num)
{
    if (rows == NULL) nrows = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        const double* yi = Y + i * s;
        double a = 0.0, f[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double* yj = Y + j * s;
            double r2 = sqdist(s, yi, yj);
            a += kern1(kind, r2);
            double w = kern2(kind, r2);
            for (int d = 0; d < s; ++d) f[d] += w * (yi[d] - yj[d]);
        }
        h1[r] = a;
        for (int d = 0; d < s; ++d) num[r * s + d] = f[d];
    }
}

/* Z = sum_{k != l} K1 (Section 1.1) and F_rep,i = num_i / Z for every point. */
void oracle_direct_rep(int64_t n, int s, const double* Y, int kind,
                       double* F, double* Z)
{
    double* h1 = (double*)malloc((size_t)n * sizeof(double));
    oracle_direct_sums(n, s, Y, kind, NULL, n, h1, F);
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += h1[i];
    for (int64_t k = 0; k < n * s; ++k) F[k] /= z;
    *Z = z;
    free(h1);
}

/* Attractive force over the sparse P (Section 3):
 *   F_attr,i = sum_j p_ij q_ij Z (y_i - y_j) = sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2). */
void oracle_attr(int64_t n, int s, const double* Y, const int64_t* row_ptr,
                 const int32_t* col, const double* val, double* F)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double* yi = Y + i * s;
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const double* yj = Y + (int64_t)col[k] * s;
            double r2 = sqdist(s, yi, yj);
            double w = val[k] / (1.0 + r2);
            for (int d = 0; d < s; ++d) f[d] += w * (yi[d] - yj[d]);
        }
        for (int d = 0; d < s; ++d) F[i * s + d] = f[d];
    }
}

/* Kullback-Leibler divergence of Section 1.1, written out from its
 * definition: C = sum over the non-zeros p_ij of P of p_ij log(p_ij / q_ij),
 * with q_ij = K1(y_i, y_j) / Z and K1 = 1 / (1 + |y_i - y_j|^2).  Z is an
 * argument: the direct sum over ordered pairs i != j (oracle_direct_rep) or
 * the interpolated one of oracle_interp_rep.  Zero entries contribute 0. */
double oracle_kl(int64_t n, int s, const double* Y, const int64_t* row_ptr,
                 const int32_t* col, const double* val, double Z)
{
    double acc = 0.0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : acc)
    for (int64_t i = 0; i < n; ++i) {
        const double* yi = Y + i * s;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const double p = val[k];
            if (p <= 0.0) continue;
            const double q = (1.0 / (1.0 + sqdist(s, yi, Y + (int64_t)col[k] * s))) / Z;
            acc += p * log(p / q);
        }
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Box geometry (the square box of Section 2.4; interval count of Section    */
/* 2.5 or a fixed interval width)                                            */
/* ------------------------------------------------------------------------ */

/* Side L = max_d (max - min), floored at 1e-6.  PAPER: N_int =
 * max(min_intervals, ceil(L)), w = L / N_int.  FIXED: w = interval_width and
 * N_int = ceil(L / w), unless that gives fewer than min_intervals intervals;
 * then N_int = min_intervals and w = L / N_int, so that, as under the
 * interval count of Section 2.5, no interval is wider than L / min_intervals.
 * Every axis gets that N_int (the square box of Section 2.4), or with rect
 * set (s = 2) each narrower axis d gets its own count
 * min(N_int, max(min_intervals, ceil(L_d / w))) at the same w, so the box is
 * a rectangle of equal spacing; n_int[d] receives the per-axis counts.  The square box of side N_int w is
 * centred on the mid-range of each dimension: origin(d) = (min + max)/2 -
 * N_int w / 2 (for the widest dimension under PAPER this is its minimum).
 * Y holds the float32 inputs widened to double. */
void oracle_geometry(int64_t n, int s, const double* Y, int policy,
                     int min_intervals, double interval_width, int rect,
                     double* origin, double* w_int, int* n_int)
{
    double lo[3], hi[3];
    for (int d = 0; d < s; ++d) { lo[d] = Y[d]; hi[d] = Y[d]; }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < s; ++d) {
            double v = Y[i * s + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double L = 0.0;
    for (int d = 0; d < s; ++d)
        if (hi[d] - lo[d] > L) L = hi[d] - lo[d];
    if (L < 1e-6) L = 1e-6;
    int m;
    if (policy == ORACLE_POLICY_PAPER) {
        m = (int)ceil(L);
        if (m < min_intervals) m = min_intervals;
        *w_int = L / m;
    } else if (L < interval_width * min_intervals) {
        m = min_intervals;
        *w_int = L / m;
    } else {
        m = (int)ceil(L / interval_width);
        if (m < min_intervals) m = min_intervals;
        *w_int = interval_width;
    }
    for (int d = 0; d < s; ++d) {
        int md = m;
        double Ld = hi[d] - lo[d];
        if (rect && s == 2 && Ld < L) {
            md = (int)ceil(Ld / *w_int);
            if (md < min_intervals) md = min_intervals;
            if (md > m) md = m;
        }
        n_int[d] = md;
        origin[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * md * (*w_int);
    }
}

/* ------------------------------------------------------------------------ */
/* (2) Interpolation scheme, Step 2 done directly                            */
/* ------------------------------------------------------------------------ */

/* Lagrange basis on the p equispaced nodes tau_m = (m + 1/2)/p of the unit
 * interval (Section 2.1, the Lagrange polynomials; nodes of eq. (equinodes)):
 *   L_m(t) = prod_{k != m} (t - tau_k) / (tau_m - tau_k). */
void oracle_lagrange(int p, double t, double* L)
{
    for (int m = 0; m < p; ++m) {
        double tm = (m + 0.5) / p, a = 1.0;
        for (int k = 0; k < p; ++k) {
            if (k == m) continue;
            double tk = (k + 0.5) / p;
            a *= (t - tk) / (tm - tk);
        }
        L[m] = a;
    }
}

/* Interval index and local coordinate of a coordinate value. */
static void locate(double y, double o, double w, int n_int, int* cell, double* t)
{
    double u = (y - o) / w;
    double f = floor(u);
    int c = (int)f;
    if (f < 0.0) c = 0;
    if (f > (double)(n_int - 1)) c = n_int - 1;
    *cell = c;
    *t = u - (double)c;
}

/* Step 2 directly (eq. (equikereval2)): on a grid with ngv[d] nodes along
 * dimension d and spacing h,
 *   V[g] = sum_{g'} K(h (g - g')) W[g'],
 * where kernel selects K1 (1), K2 (2), or the odd vector kernels
 * G_d(z) = z_d K2(|z|^2) along dimension 0 (3) or 1 (4).  2-D grids are
 * indexed g1*ng0 + g0.  The kernel values come from a table over the lag
 * (|g0-g0'|, |g1-g1'|), with the sign of the lag along d for G_d: the
 * translation invariance that makes the matrix Toeplitz. */
void oracle_grid_conv(int s, const int* ngv, double h, int kind, int kernel,
                      const double* W, double* V)
{
    const int ng = ngv[0], ng1 = (s == 2) ? ngv[1] : 1;
    int64_t tn = (int64_t)ng * ng1;
    double* T = (double*)malloc((size_t)tn * sizeof(double));
    for (int64_t a = 0; a < tn; ++a) {
        double dx = (double)(a % ng), dy = (s == 1) ? 0.0 : (double)(a / ng);
        double r2 = h * h * (dx * dx + dy * dy);
        if (kernel == 1) T[a] = kern1(kind, r2);
        else if (kernel == 2) T[a] = kern2(kind, r2);
        else if (kernel == 3) T[a] = h * dx * kern2(kind, r2);
        else T[a] = h * dy * kern2(kind, r2);
    }
    if (s == 1) {
#pragma omp parallel for schedule(static)
        for (int g = 0; g < ng; ++g) {
            double acc = 0.0;
            for (int q = 0; q < ng; ++q) {
                const double sg = (kernel == 3) ? (double)((g > q) - (g < q)) : 1.0;
                acc += sg * T[abs(g - q)] * W[q];
            }
            V[g] = acc;
        }
    } else {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t g = 0; g < tn; ++g) {
            int g0 = (int)(g % ng), g1 = (int)(g / ng);
            double acc = 0.0;
            for (int q1 = 0; q1 < ng1; ++q1) {
                const double* Trow = T + (int64_t)abs(g1 - q1) * ng;
                const double* Wrow = W + (int64_t)q1 * ng;
                const double s1 = (kernel == 4) ? (double)((g1 > q1) - (g1 < q1)) : 1.0;
                for (int q0 = 0; q0 < ng; ++q0) {
                    const double s0 = (kernel == 3) ? (double)((g0 > q0) - (g0 < q0)) : 1.0;
                    acc += s0 * s1 * Trow[abs(g0 - q0)] * Wrow[q0];
                }
            }
            V[g] = acc;
        }
    }
    free(T);
}

/* The interpolation-based repulsion for s = 1 or 2 with the given box
 * (origin[s], interval width w, n_int[d] intervals along dimension d, p
 * nodes per interval).
 *
 * Charges (centred at the box centre c): form A {1, y'(d)}, form B
 * {1, y'(d), |y'|^2}; y' = y - c.  Potentials (s + 2 of them):
 *   pot[0] = K1 * 1 (form A)  or  K2 * |y'|^2 (form B)
 *   pot[1] = K2 * 1
 *   pot[2+d] = K2 * y'(d)
 * Form V (the vector-kernel variant, not in the paper): the single charge 1
 * and s + 1 potentials pot[0] = K1 * 1, pot[1+d] = G_d * 1 with the odd
 * kernels G_d(z) = z_d K2(|z|^2), so pot[1+d] at y_i is the numerator
 * sum_j (y_i(d) - y_j(d)) K2 itself, with no cancellation.
 * Step 1 spreads each charge onto the nodes of its point's interval (square),
 * Step 2 is oracle_grid_conv, Step 3 interpolates back (Section 2.2,
 * Algorithm 1; tensor-product nodes for s = 2, Section 2.4).  Assembly
 * (Appendix): h1 = pot[0] (form A) or
 * h1 = (1 + |y'|^2) pot[1] - 2 y'.pot[2..] + pot[0] (form B);
 * Z = sum_i h1_i - N K1(0); F_i(d) = (y'_i(d) pot[1]_i - pot[2+d]_i) / Z.
 *
 * Form V: h1 = pot[0], F_i(d) = pot[1+d]_i / Z.
 *
 * Outputs: F [n*s], Z; optional (may be NULL): Wout [C][ng^s] charge grids
 * (C = s+1 form A, s+2 form B, 1 form V; charge order 1, y'(0..s-1), |y'|^2),
 * Vout [P][ng^s] potential grids (P = s+2, or s+1 form V), phi [n][P]
 * potentials at the points, h1 [n].  Returns 0, or -1 on bad arguments. */
int oracle_interp_rep(int64_t n, int s, const double* Y, const double* origin,
                      double w, const int* n_int, int p, int form, int kind,
                      double* F, double* Z, double* Wout, double* Vout,
                      double* phi, double* h1out)
{
    if (s < 1 || s > 2 || p < 1 || n < 1) return -1;
    for (int d = 0; d < s; ++d)
        if (n_int[d] < 1) return -1;
    int ng = n_int[0] * p;
    int ngv[2] = {ng, (s == 2) ? n_int[1] * p : 1};
    int64_t tn = (int64_t)ngv[0] * ngv[1];
    int nc = (form == ORACLE_FORM_A) ? s + 1 : (form == ORACLE_FORM_B) ? s + 2 : 1;
    int np = (form == ORACLE_FORM_V) ? s + 1 : s + 2;
    double h = w / p;
    double centre[2];
    for (int d = 0; d < s; ++d) centre[d] = origin[d] + 0.5 * n_int[d] * w;

    int* cells = (int*)malloc((size_t)n * s * sizeof(int));
    double* wts = (double*)malloc((size_t)n * s * p * sizeof(double));
    double* q = (double*)malloc((size_t)n * nc * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double r2c = 0.0;
        q[i * nc + 0] = 1.0;
        for (int d = 0; d < s; ++d) {
            double t;
            locate(Y[i * s + d], origin[d], w, n_int[d], &cells[i * s + d], &t);
            oracle_lagrange(p, t, wts + (i * s + d) * p);
            double yc = Y[i * s + d] - centre[d];
            if (form != ORACLE_FORM_V) q[i * nc + 1 + d] = yc;
            r2c += yc * yc;
        }
        if (form == ORACLE_FORM_B) q[i * nc + 1 + s] = r2c;
    }

    /* Step 1: w_{m,l} = sum_{y_i in I_l} L_m(y_i) q_i */
    double* W = (double*)calloc((size_t)nc * tn, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        if (s == 1) {
            for (int m = 0; m < p; ++m) {
                int64_t g = (int64_t)cells[i] * p + m;
                double l = wts[i * p + m];
                for (int c = 0; c < nc; ++c) W[c * tn + g] += l * q[i * nc + c];
            }
        } else {
            for (int m1 = 0; m1 < p; ++m1)
                for (int m0 = 0; m0 < p; ++m0) {
                    int64_t g0 = (int64_t)cells[i * 2 + 0] * p + m0;
                    int64_t g1 = (int64_t)cells[i * 2 + 1] * p + m1;
                    double l = wts[(i * 2 + 0) * p + m0] * wts[(i * 2 + 1) * p + m1];
                    for (int c = 0; c < nc; ++c)
                        W[c * tn + g1 * ng + g0] += l * q[i * nc + c];
                }
        }
    }

    /* Step 2: v = K~ w for every (kernel, charge) pair */
    double* V = (double*)malloc((size_t)np * tn * sizeof(double));
    int pk[5], pc[5];
    if (form == ORACLE_FORM_V) {
        pk[0] = 1; pc[0] = 0;
        for (int d = 0; d < s; ++d) { pk[1 + d] = 3 + d; pc[1 + d] = 0; }
    } else {
        if (form == ORACLE_FORM_A) { pk[0] = 1; pc[0] = 0; }
        else                       { pk[0] = 2; pc[0] = s + 1; }
        pk[1] = 2; pc[1] = 0;
        for (int d = 0; d < s; ++d) { pk[2 + d] = 2; pc[2 + d] = 1 + d; }
    }
    for (int k = 0; k < np; ++k)
        oracle_grid_conv(s, ngv, h, kind, pk[k], W + (int64_t)pc[k] * tn, V + (int64_t)k * tn);

    /* Step 3: phi(y_i) = sum_m L_m(y_i) v_{m,l} */
    double* ph = (double*)calloc((size_t)n * np, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < np; ++k) {
            double acc = 0.0;
            if (s == 1) {
                for (int m = 0; m < p; ++m)
                    acc += wts[i * p + m] * V[k * tn + (int64_t)cells[i] * p + m];
            } else {
                for (int m1 = 0; m1 < p; ++m1)
                    for (int m0 = 0; m0 < p; ++m0) {
                        int64_t g0 = (int64_t)cells[i * 2 + 0] * p + m0;
                        int64_t g1 = (int64_t)cells[i * 2 + 1] * p + m1;
                        acc += wts[(i * 2 + 0) * p + m0] * wts[(i * 2 + 1) * p + m1]
                               * V[k * tn + g1 * ng + g0];
                    }
            }
            ph[i * np + k] = acc;
        }
    }

    /* Assembly (Appendix) */
    double z = 0.0;
    double* h1 = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        const double* f = ph + i * np;
        double a;
        if (form == ORACLE_FORM_A || form == ORACLE_FORM_V) {
            a = f[0];
        } else {
            double r2c = q[i * nc + 1 + s], dot = 0.0;
            for (int d = 0; d < s; ++d) dot += q[i * nc + 1 + d] * f[2 + d];
            a = (1.0 + r2c) * f[1] - 2.0 * dot + f[0];
        }
        h1[i] = a;
        z += a;
    }
    z -= (double)n * kern1(kind, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < s; ++d)
            F[i * s + d] = (form == ORACLE_FORM_V)
                               ? ph[i * np + 1 + d] / z
                               : (q[i * nc + 1 + d] * ph[i * np + 1] - ph[i * np + 2 + d]) / z;
    *Z = z;

    if (Wout) memcpy(Wout, W, (size_t)nc * tn * sizeof(double));
    if (Vout) memcpy(Vout, V, (size_t)np * tn * sizeof(double));
    if (phi) memcpy(phi, ph, (size_t)n * np * sizeof(double));
    if (h1out) memcpy(h1out, h1, (size_t)n * sizeof(double));
    free(cells); free(wts); free(q); free(W); free(V); free(ph); free(h1);
    return 0;
}

/* Step 1 alone: the charge grids W [C][ng^s] of oracle_interp_rep. */
int oracle_interp_spread(int64_t n, int s, const double* Y, const double* origin,
                         double w, const int* n_int, int p, int form, double* Wout)
{
    if (s < 1 || s > 2 || p < 1) return -1;
    for (int d = 0; d < s; ++d)
        if (n_int[d] < 1) return -1;
    int ng = n_int[0] * p;
    int64_t tn = (int64_t)ng * ((s == 2) ? n_int[1] * p : 1);
    int nc = (form == ORACLE_FORM_A) ? s + 1 : (form == ORACLE_FORM_B) ? s + 2 : 1;
    double centre[2], L0[16], L1[16];
    for (int d = 0; d < s; ++d) centre[d] = origin[d] + 0.5 * n_int[d] * w;
    memset(Wout, 0, (size_t)nc * tn * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int c0 = 0, c1 = 0;
        double t0, t1 = 0.0, qv[4], r2c = 0.0;
        locate(Y[i * s], origin[0], w, n_int[0], &c0, &t0);
        oracle_lagrange(p, t0, L0);
        if (s == 2) {
            locate(Y[i * s + 1], origin[1], w, n_int[1], &c1, &t1);
            oracle_lagrange(p, t1, L1);
        } else {
            L1[0] = 1.0;
        }
        qv[0] = 1.0;
        for (int d = 0; d < s; ++d) {
            qv[1 + d] = Y[i * s + d] - centre[d];
            r2c += qv[1 + d] * qv[1 + d];
        }
        if (form == ORACLE_FORM_B) qv[1 + s] = r2c;
        int p1 = (s == 2) ? p : 1;
        for (int m1 = 0; m1 < p1; ++m1)
            for (int m0 = 0; m0 < p; ++m0) {
                int64_t g = (int64_t)(c1 * p + m1) * ((s == 2) ? ng : 0) + c0 * p + m0;
                double l = L0[m0] * L1[m1];
                for (int c = 0; c < nc; ++c) Wout[c * tn + g] += l * qv[c];
            }
    }
    return 0;
}

/* Step 3 alone: phi [n][np] at every point from given potential grids
 * V [np][ng^s] (grid layout of oracle_interp_rep), phi_k(y_i) =
 * sum_m L_m(y_i) V_k[node m of the interval of y_i] (Section 2.2, Step 3;
 * tensor-product nodes for s = 2, Section 2.4). */
int oracle_interp_gather(int64_t n, int s, const double* Y, const double* origin,
                         double w, const int* n_int, int p, int np, const double* V,
                         double* phi)
{
    if (s < 1 || s > 2 || p < 1 || np < 1) return -1;
    for (int d = 0; d < s; ++d)
        if (n_int[d] < 1) return -1;
    const int ng = n_int[0] * p;
    const int64_t tn = (int64_t)ng * ((s == 2) ? n_int[1] * p : 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int c0 = 0, c1 = 0;
        double t0, t1 = 0.0, L0[16], L1[16];
        locate(Y[i * s], origin[0], w, n_int[0], &c0, &t0);
        oracle_lagrange(p, t0, L0);
        if (s == 2) {
            locate(Y[i * s + 1], origin[1], w, n_int[1], &c1, &t1);
            oracle_lagrange(p, t1, L1);
        } else {
            L1[0] = 1.0;
        }
        const int p1 = (s == 2) ? p : 1;
        for (int k = 0; k < np; ++k) {
            double acc = 0.0;
            for (int m1 = 0; m1 < p1; ++m1)
                for (int m0 = 0; m0 < p; ++m0) {
                    const int64_t g = (int64_t)(c1 * p + m1) * ((s == 2) ? ng : 0) + c0 * p + m0;
                    acc += L0[m0] * L1[m1] * V[(int64_t)k * tn + g];
                }
            phi[i * np + k] = acc;
        }
    }
    return 0;
}

/* Per-point interpolated sums for a few listed rows, computing V only at the
 * nodes those rows read: each node value is the full direct sum of Step 2
 * over every node.  Needs the complete charge grids W (oracle_interp_spread).
 * Outputs phi [nrows][s+2] in the potential order of oracle_interp_rep. */
int oracle_interp_rows(int64_t n, int s, const double* Y, const double* origin,
                       double w, const int* n_int, int p, int form, int kind,
                       const double* W, const int64_t* rows, int64_t nrows,
                       double* phi)
{
    (void)n;
    if (s < 1 || s > 2 || p < 1) return -1;
    for (int d = 0; d < s; ++d)
        if (n_int[d] < 1) return -1;
    int ng = n_int[0] * p;
    int ng1 = (s == 2) ? n_int[1] * p : 1;
    int64_t tn = (int64_t)ng * ng1;
    int np = (form == ORACLE_FORM_V) ? s + 1 : s + 2;
    double h = w / p;
    int pk[5], pc[5];
    if (form == ORACLE_FORM_V) {
        pk[0] = 1; pc[0] = 0;
        for (int d = 0; d < s; ++d) { pk[1 + d] = 3 + d; pc[1 + d] = 0; }
    } else {
        if (form == ORACLE_FORM_A) { pk[0] = 1; pc[0] = 0; }
        else                       { pk[0] = 2; pc[0] = s + 1; }
        pk[1] = 2; pc[1] = 0;
        for (int d = 0; d < s; ++d) { pk[2 + d] = 2; pc[2 + d] = 1 + d; }
    }
    /* kernel values by lag (|dg0|, |dg1|), as in oracle_grid_conv: K1, K2,
     * then |z_0| K2 and |z_1| K2 (the odd kernels without their sign) */
    double* T = (double*)malloc((size_t)4 * tn * sizeof(double));
    for (int64_t a = 0; a < tn; ++a) {
        double dx = (double)(a % ng), dy = (s == 1) ? 0.0 : (double)(a / ng);
        double r2 = h * h * (dx * dx + dy * dy);
        T[a] = kern1(kind, r2);
        T[tn + a] = kern2(kind, r2);
        T[2 * tn + a] = h * dx * kern2(kind, r2);
        T[3 * tn + a] = h * dy * kern2(kind, r2);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        int c0 = 0, c1 = 0;
        double t0, t1 = 0.0, L0[16], L1[16];
        locate(Y[i * s], origin[0], w, n_int[0], &c0, &t0);
        oracle_lagrange(p, t0, L0);
        if (s == 2) {
            locate(Y[i * s + 1], origin[1], w, n_int[1], &c1, &t1);
            oracle_lagrange(p, t1, L1);
        } else {
            L1[0] = 1.0;
        }
        int p1 = (s == 2) ? p : 1;
        for (int k = 0; k < np; ++k) {
            double acc = 0.0;
            for (int m1 = 0; m1 < p1; ++m1)
                for (int m0 = 0; m0 < p; ++m0) {
                    int g0 = c0 * p + m0, g1 = (s == 2) ? c1 * p + m1 : 0;
                    /* node value by the direct sum over all nodes */
                    const double* Tk = T + (int64_t)(pk[k] - 1) * tn;
                    const double* Wc = W + (int64_t)pc[k] * tn;
                    double v = 0.0;
                    for (int q1 = 0; q1 < ng1; ++q1) {
                        const double* Trow = Tk + (int64_t)abs(g1 - q1) * ng;
                        const double* Wrow = Wc + (int64_t)q1 * ng;
                        const double s1 = (pk[k] == 4) ? (double)((g1 > q1) - (g1 < q1)) : 1.0;
                        for (int q0 = 0; q0 < ng; ++q0) {
                            const double s0 = (pk[k] == 3) ? (double)((g0 > q0) - (g0 < q0)) : 1.0;
                            v += s0 * s1 * Trow[abs(g0 - q0)] * Wrow[q0];
                        }
                    }
                    acc += L0[m0] * L1[m1] * v;
                }
            phi[r * np + k] = acc;
        }
    }
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* (3) Gradient-descent update                                               */
/* ------------------------------------------------------------------------ */

/* One step for every component y_i(d):
 *   grad = 4 (alpha F_attr - F_rep)                 (Section 1.1, Section 1.2)
 *   gain = (grad > 0) != (uY > 0) ? gain + gain_inc : gain * gain_dec,
 *          then max(gain, gain_min)
 *   uY   = mom uY - eta gain grad
 *   Y    = (Y - mean(Y)) + uY   if recentre, else Y + uY
 * The paper does not state the step rule; this is the momentum and
 * per-component-gain descent of the t-SNE implementations it builds on, and
 * its constants come from the caller (parity of the rule itself is unpinned
 * by the paper).  mean(Y) is taken over the Y passed in. */
void oracle_update(int64_t n, int s, double* Y, double* uY, double* gains,
                   const double* Fattr, const double* Frep, double alpha,
                   double mom, double eta, double gain_inc, double gain_dec,
                   double gain_min, int recentre)
{
    double mean[3] = {0.0, 0.0, 0.0};
    if (recentre) {
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < s; ++d) mean[d] += Y[i * s + d];
        for (int d = 0; d < s; ++d) mean[d] /= (double)n;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < s; ++d) {
            int64_t k = i * s + d;
            double g = 4.0 * (alpha * Fattr[k] - Frep[k]);
            double gn = ((g > 0.0) != (uY[k] > 0.0)) ? gains[k] + gain_inc
                                                      : gains[k] * gain_dec;
            if (gn < gain_min) gn = gain_min;
            gains[k] = gn;
            uY[k] = mom * uY[k] - eta * gn * g;
            Y[k] = (Y[k] - mean[d]) + uY[k];
        }
}

/* ------------------------------------------------------------------------ */
/* Input affinities (Section 1.1, restricted to the k nearest neighbours as  */
/* in Section 3)                                                             */
/* ------------------------------------------------------------------------ */

typedef struct { double d; int32_t j; } knn_pair;

static int knn_cmp(const void* a, const void* b)
{
    const knn_pair* x = (const knn_pair*)a;
    const knn_pair* y = (const knn_pair*)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* Exact k nearest neighbours of every row of X [n, dim] (squared Euclidean
 * distance summed over the coordinate differences, the point itself
 * excluded), by computing every distance and sorting; equal distances are
 * ordered by index.  idx [n, k], dist2 [n, k], ascending.  Needs k < n. */
void oracle_knn(int64_t n, int dim, const double* X, int k, int32_t* idx, double* dist2)
{
#pragma omp parallel
    {
        knn_pair* buf = (knn_pair*)malloc(sizeof(knn_pair) * (size_t)n);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double acc = 0.0;
                for (int c = 0; c < dim; ++c) {
                    const double t = X[i * dim + c] - X[j * dim + c];
                    acc += t * t;
                }
                buf[m].d = acc;
                buf[m].j = (int32_t)j;
                ++m;
            }
            qsort(buf, (size_t)m, sizeof(knn_pair), knn_cmp);
            for (int t = 0; t < k; ++t) {
                idx[i * k + t] = buf[t].j;
                dist2[i * k + t] = buf[t].d;
            }
        }
        free(buf);
    }
}

/* oracle_knn for the listed rows only (rows [nr] of X [n, dim]): idx [nr, k],
 * dist2 [nr, k]. */
void oracle_knn_rows(int64_t n, int dim, const double* X, int k, const int64_t* rows, int64_t nr,
                     int32_t* idx, double* dist2)
{
#pragma omp parallel
    {
        knn_pair* buf = (knn_pair*)malloc(sizeof(knn_pair) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nr; ++r) {
            const int64_t i = rows[r];
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double acc = 0.0;
                for (int c = 0; c < dim; ++c) {
                    const double t = X[i * dim + c] - X[j * dim + c];
                    acc += t * t;
                }
                buf[m].d = acc;
                buf[m].j = (int32_t)j;
                ++m;
            }
            qsort(buf, (size_t)m, sizeof(knn_pair), knn_cmp);
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = buf[t].j;
                dist2[r * k + t] = buf[t].d;
            }
        }
        free(buf);
    }
}

/* Conditional affinities of every row from its k squared neighbour
 * distances (ascending): p_{j|i} = exp(-beta_i d_ij) / sum_l exp(-beta_i d_il),
 * beta_i = 1 / (2 sigma_i^2), with beta_i found by bisection so that the
 * perplexity exp(H_i), H_i = -sum_j p_{j|i} ln p_{j|i}, equals the target.
 * Steps: distances are shifted by the row minimum (the p do not change);
 * H = ln S + beta sum_j d'_j w_j / S with w_j = exp(-beta d'_j), S = sum w_j;
 * start at beta = 1 with no bounds; while |H - ln(perplexity)| >= 1e-10 and
 * fewer than 200 steps: if H is too high, the lower bound becomes beta and
 * beta doubles (no upper bound yet) or moves to the midpoint; otherwise the
 * upper bound becomes beta and beta halves (no lower bound) or moves to the
 * midpoint.  beta_out [n] (may be NULL), p [n, k]. */
void oracle_perplexity(int64_t n, int k, const double* dist2, double perplexity,
                       double* beta_out, double* p)
{
    const double target = log(perplexity);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double* d = dist2 + i * k;
        double dmin = d[0];
        for (int t = 1; t < k; ++t) if (d[t] < dmin) dmin = d[t];
        double beta = 1.0, lo = -INFINITY, hi = INFINITY;
        for (int it = 0; it < 200; ++it) {
            double S = 0.0, SD = 0.0;
            for (int t = 0; t < k; ++t) {
                const double w = exp(-beta * (d[t] - dmin));
                S += w;
                SD += (d[t] - dmin) * w;
            }
            const double H = log(S) + beta * SD / S;
            const double diff = H - target;
            if (fabs(diff) < 1e-10) break;
            if (diff > 0.0) {
                lo = beta;
                beta = isinf(hi) ? beta * 2.0 : 0.5 * (beta + hi);
            } else {
                hi = beta;
                beta = isinf(lo) ? beta * 0.5 : 0.5 * (beta + lo);
            }
        }
        double S = 0.0;
        for (int t = 0; t < k; ++t) S += exp(-beta * (d[t] - dmin));
        for (int t = 0; t < k; ++t) p[i * k + t] = exp(-beta * (d[t] - dmin)) / S;
        if (beta_out) beta_out[i] = beta;
    }
}

typedef struct { int64_t r; int32_t c; double v; } coo_entry;

static int coo_cmp(const void* a, const void* b)
{
    const coo_entry* x = (const coo_entry*)a;
    const coo_entry* y = (const coo_entry*)b;
    if (x->r != y->r) return (x->r > y->r) - (x->r < y->r);
    return (x->c > y->c) - (x->c < y->c);
}

/* Symmetric joint affinities p_ij = (p_{j|i} + p_{i|j}) / (2N) from the
 * conditional rows (idx [n, k], p [n, k]), as CSR with columns ascending in
 * each row: every (i, j, p_{j|i}) is counted in row i and in row j, equal
 * (row, column) pairs are summed.  row_ptr [n+1]; col, val hold nnz <= 2nk
 * entries.  Returns nnz. */
int64_t oracle_symmetrize(int64_t n, int k, const int32_t* idx, const double* p,
                          int64_t* row_ptr, int32_t* col, double* val)
{
    const int64_t m = 2 * n * (int64_t)k;
    coo_entry* e = (coo_entry*)malloc(sizeof(coo_entry) * (size_t)m);
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < k; ++t) {
            const int64_t q = i * k + t;
            e[2 * q].r = i;
            e[2 * q].c = idx[q];
            e[2 * q].v = p[q];
            e[2 * q + 1].r = idx[q];
            e[2 * q + 1].c = (int32_t)i;
            e[2 * q + 1].v = p[q];
        }
    qsort(e, (size_t)m, sizeof(coo_entry), coo_cmp);
    int64_t nnz = 0;
    for (int64_t r = 0; r <= n; ++r) row_ptr[r] = 0;
    for (int64_t a = 0; a < m;) {
        int64_t b = a;
        double v = 0.0;
        while (b < m && e[b].r == e[a].r && e[b].c == e[a].c) v += e[b++].v;
        col[nnz] = e[a].c;
        val[nnz] = v / (2.0 * (double)n);
        row_ptr[e[a].r + 1] += 1;
        ++nnz;
        a = b;
    }
    for (int64_t r = 0; r < n; ++r) row_ptr[r + 1] += row_ptr[r];
    free(e);
    return nnz;
}
