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
 *       1-3 and Algorithm 1 without the FFT; Section 2.4 for s = 2 and the
 *       same tensor product for s = 3; the Appendix for assembling the forces
 *       from the s+2 kernel sums);
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

/* Grids of s = 1, 2 or 3 dimensions with ngv[d] nodes along dimension d are
 * stored with dimension 0 fastest: node (g0, g1, g2) at g0 + ng0 (g1 + ng1 g2).
 * Section 2.4 gives the tensor-product scheme for s = 2; the opening of
 * Section 2 states the s + 2 sums for any s, and the same tensor product is
 * used for s = 3. */
static int64_t grid_size(int s, const int* ngv)
{
    int64_t t = 1;
    for (int d = 0; d < s; ++d) t *= ngv[d];
    return t;
}

/* Kernel value at the lag vector dg (in nodes) with spacing h: K1 (kernel 1),
 * K2 (2), or the odd vector kernels G_d(z) = z_d K2(|z|^2) along dimension
 * d = kernel - 3 (3, 4, 5), z = h dg with the sign of the lag. */
static double kern_lag(int s, const int* dg, double h, int kind, int kernel)
{
    double r2 = 0.0;
    for (int d = 0; d < s; ++d) r2 += (double)dg[d] * (double)dg[d];
    r2 *= h * h;
    if (kernel == 1) return kern1(kind, r2);
    if (kernel == 2) return kern2(kind, r2);
    return h * (double)dg[kernel - 3] * kern2(kind, r2);
}

/* Step 2 directly (eq. (equikereval2)): V[g] = sum_{g'} K(h (g - g')) W[g'],
 * the kernel selected as in kern_lag.  The kernel values come from a table
 * over the absolute lags (|dg0|, |dg1|, |dg2|), with the sign of the lag
 * along d restored for G_d: the translation invariance that makes the matrix
 * (block-)Toeplitz. */
void oracle_grid_conv(int s, const int* ngv, double h, int kind, int kernel,
                      const double* W, double* V)
{
    int ng[3] = {1, 1, 1};
    for (int d = 0; d < s; ++d) ng[d] = ngv[d];
    const int64_t tn = (int64_t)ng[0] * ng[1] * ng[2];
    double* T = (double*)malloc((size_t)tn * sizeof(double));
    for (int64_t a = 0; a < tn; ++a) {
        int dg[3] = {(int)(a % ng[0]), (int)((a / ng[0]) % ng[1]), (int)(a / ((int64_t)ng[0] * ng[1]))};
        T[a] = kern_lag(s, dg, h, kind, kernel);     /* odd kernels: |lag| here, sign below */
    }
    const int odd = (kernel >= 3) ? kernel - 3 : -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < tn; ++g) {
        const int g0 = (int)(g % ng[0]), g1 = (int)((g / ng[0]) % ng[1]),
                  g2 = (int)(g / ((int64_t)ng[0] * ng[1]));
        const int gg[3] = {g0, g1, g2};
        double acc = 0.0;
        for (int q2 = 0; q2 < ng[2]; ++q2)
            for (int q1 = 0; q1 < ng[1]; ++q1) {
                const int64_t trow = ((int64_t)abs(g2 - q2) * ng[1] + abs(g1 - q1)) * ng[0];
                const int64_t wrow = ((int64_t)q2 * ng[1] + q1) * ng[0];
                const int qq[3] = {0, q1, q2};
                double sgn12 = 1.0;
                if (odd == 1) sgn12 = (double)((gg[1] > qq[1]) - (gg[1] < qq[1]));
                if (odd == 2) sgn12 = (double)((gg[2] > qq[2]) - (gg[2] < qq[2]));
                for (int q0 = 0; q0 < ng[0]; ++q0) {
                    const double s0 = (odd == 0) ? (double)((g0 > q0) - (g0 < q0)) : 1.0;
                    acc += s0 * sgn12 * T[trow + abs(g0 - q0)] * W[wrow + q0];
                }
            }
        V[g] = acc;
    }
    free(T);
}

/* Cell and Lagrange weights L[d][m] of one point along each dimension. */
static void point_weights(int s, const double* y, const double* origin, double w,
                          const int* n_int, int p, int* cell, double (*L)[16])
{
    for (int d = 0; d < s; ++d) {
        double t;
        locate(y[d], origin[d], w, n_int[d], &cell[d], &t);
        oracle_lagrange(p, t, L[d]);
    }
}

/* Node index and weight of the q-th of the p^s nodes of a point's interval
 * (node offsets m_d = digits of q in base p, dimension 0 fastest); the weight
 * is the product of the per-dimension Lagrange weights, dimension 0 first. */
static int64_t node_of(int s, int q, int p, const int* cell, double (*L)[16], const int* ng,
                       double* wt)
{
    int64_t g = 0, stride = 1;
    double a = 1.0;
    for (int d = 0; d < s; ++d) {
        const int m = q % p;
        q /= p;
        g += (int64_t)(cell[d] * p + m) * stride;
        stride *= ng[d];
        a = (d == 0) ? L[0][m] : a * L[d][m];
    }
    *wt = a;
    return g;
}

static int ipow(int b, int e)
{
    int r = 1;
    for (int k = 0; k < e; ++k) r *= b;
    return r;
}

/* (kernel, charge) of each potential.  Charges (centred at the box centre c,
 * y' = y - c): form A {1, y'(d)}, form B {1, y'(d), |y'|^2}, form V {1}.
 * Potentials: form A/B pot[0] = K1 * 1 (A) or K2 * |y'|^2 (B), pot[1] = K2 * 1,
 * pot[2+d] = K2 * y'(d); form V pot[0] = K1 * 1, pot[1+d] = G_d * 1. */
static void pot_map(int s, int form, int* pk, int* pc)
{
    if (form == ORACLE_FORM_V) {
        pk[0] = 1; pc[0] = 0;
        for (int d = 0; d < s; ++d) { pk[1 + d] = 3 + d; pc[1 + d] = 0; }
    } else {
        if (form == ORACLE_FORM_A) { pk[0] = 1; pc[0] = 0; }
        else                       { pk[0] = 2; pc[0] = s + 1; }
        pk[1] = 2; pc[1] = 0;
        for (int d = 0; d < s; ++d) { pk[2 + d] = 2; pc[2 + d] = 1 + d; }
    }
}

static int n_charges(int s, int form)
{
    return (form == ORACLE_FORM_A) ? s + 1 : (form == ORACLE_FORM_B) ? s + 2 : 1;
}

static int n_pots(int s, int form) { return (form == ORACLE_FORM_V) ? s + 1 : s + 2; }

/* Charges of one point (see pot_map). */
static void charges_of(int s, int form, const double* y, const double* centre, double* q)
{
    double r2c = 0.0;
    q[0] = 1.0;
    for (int d = 0; d < s; ++d) {
        const double yc = y[d] - centre[d];
        if (form != ORACLE_FORM_V) q[1 + d] = yc;
        r2c += yc * yc;
    }
    if (form == ORACLE_FORM_B) q[1 + s] = r2c;
}

static int check_box(int s, int p, const int* n_int)
{
    if (s < 1 || s > 3 || p < 1 || p > 16) return -1;
    for (int d = 0; d < s; ++d)
        if (n_int[d] < 1) return -1;
    return 0;
}

/* Step 1 (Algorithm 1): the charge grids W [C][grid], w_{m,l} = sum over the
 * points y_i of interval l of L_m(y_i) q_c(i) (tensor-product nodes). */
int oracle_interp_spread(int64_t n, int s, const double* Y, const double* origin,
                         double w, const int* n_int, int p, int form, double* Wout)
{
    if (check_box(s, p, n_int)) return -1;
    int ng[3];
    for (int d = 0; d < s; ++d) ng[d] = n_int[d] * p;
    const int64_t tn = grid_size(s, ng);
    const int nc = n_charges(s, form), pps = ipow(p, s);
    double centre[3];
    for (int d = 0; d < s; ++d) centre[d] = origin[d] + 0.5 * n_int[d] * w;
    memset(Wout, 0, (size_t)nc * tn * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int cell[3];
        double L[3][16], qv[5];
        point_weights(s, Y + i * s, origin, w, n_int, p, cell, L);
        charges_of(s, form, Y + i * s, centre, qv);
        for (int q = 0; q < pps; ++q) {
            double l;
            const int64_t g = node_of(s, q, p, cell, L, ng, &l);
            for (int c = 0; c < nc; ++c) Wout[c * tn + g] += l * qv[c];
        }
    }
    return 0;
}

/* Step 3 alone: phi [n][np] at every point from given potential grids
 * V [np][grid], phi_k(y_i) = sum_m L_m(y_i) V_k[node m of the interval of
 * y_i] (Section 2.2, Step 3; tensor-product nodes). */
int oracle_interp_gather(int64_t n, int s, const double* Y, const double* origin,
                         double w, const int* n_int, int p, int np, const double* V,
                         double* phi)
{
    if (check_box(s, p, n_int) || np < 1) return -1;
    int ng[3];
    for (int d = 0; d < s; ++d) ng[d] = n_int[d] * p;
    const int64_t tn = grid_size(s, ng);
    const int pps = ipow(p, s);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int cell[3];
        double L[3][16];
        point_weights(s, Y + i * s, origin, w, n_int, p, cell, L);
        for (int k = 0; k < np; ++k) {
            double acc = 0.0;
            for (int q = 0; q < pps; ++q) {
                double l;
                const int64_t g = node_of(s, q, p, cell, L, ng, &l);
                acc += l * V[(int64_t)k * tn + g];
            }
            phi[i * np + k] = acc;
        }
    }
    return 0;
}

/* The interpolation-based repulsion for s = 1, 2 or 3 with the given box
 * (origin[s], interval width w, n_int[d] intervals along dimension d, p
 * nodes per interval): Step 1 oracle_interp_spread, Step 2 oracle_grid_conv
 * for every (kernel, charge) pair of pot_map, Step 3 oracle_interp_gather,
 * then the assembly of the Appendix:
 *   h1 = pot[0] (forms A and V) or (1 + |y'|^2) pot[1] - 2 y'.pot[2..] + pot[0] (B);
 *   Z = sum_i h1_i - N K1(0);
 *   F_i(d) = (y'_i(d) pot[1]_i - pot[2+d]_i) / Z (A, B) or pot[1+d]_i / Z (V).
 * Outputs: F [n*s], Z; optional (may be NULL): Wout [C][grid] charge grids,
 * Vout [P][grid] potential grids, phi [n][P] potentials at the points,
 * h1 [n].  Returns 0, or -1 on bad arguments. */
int oracle_interp_rep(int64_t n, int s, const double* Y, const double* origin,
                      double w, const int* n_int, int p, int form, int kind,
                      double* F, double* Z, double* Wout, double* Vout,
                      double* phi, double* h1out)
{
    if (check_box(s, p, n_int) || n < 1) return -1;
    int ng[3];
    for (int d = 0; d < s; ++d) ng[d] = n_int[d] * p;
    const int64_t tn = grid_size(s, ng);
    const int nc = n_charges(s, form), np = n_pots(s, form);
    const double h = w / p;
    double centre[3];
    for (int d = 0; d < s; ++d) centre[d] = origin[d] + 0.5 * n_int[d] * w;

    double* W = (double*)malloc((size_t)nc * tn * sizeof(double));
    oracle_interp_spread(n, s, Y, origin, w, n_int, p, form, W);
    double* V = (double*)malloc((size_t)np * tn * sizeof(double));
    int pk[6], pc[6];
    pot_map(s, form, pk, pc);
    for (int k = 0; k < np; ++k)
        oracle_grid_conv(s, ng, h, kind, pk[k], W + (int64_t)pc[k] * tn, V + (int64_t)k * tn);
    double* ph = (double*)malloc((size_t)n * np * sizeof(double));
    oracle_interp_gather(n, s, Y, origin, w, n_int, p, np, V, ph);

    double z = 0.0;
    double* h1 = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        const double* f = ph + i * np;
        double qv[5];
        charges_of(s, form, Y + i * s, centre, qv);
        double a;
        if (form == ORACLE_FORM_A || form == ORACLE_FORM_V) {
            a = f[0];
        } else {
            double dot = 0.0;
            for (int d = 0; d < s; ++d) dot += qv[1 + d] * f[2 + d];
            a = (1.0 + qv[1 + s]) * f[1] - 2.0 * dot + f[0];
        }
        h1[i] = a;
        z += a;
    }
    z -= (double)n * kern1(kind, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        double qv[5];
        charges_of(s, form, Y + i * s, centre, qv);
        for (int d = 0; d < s; ++d)
            F[i * s + d] = (form == ORACLE_FORM_V)
                               ? ph[i * np + 1 + d] / z
                               : (qv[1 + d] * ph[i * np + 1] - ph[i * np + 2 + d]) / z;
    }
    *Z = z;

    if (Wout) memcpy(Wout, W, (size_t)nc * tn * sizeof(double));
    if (Vout) memcpy(Vout, V, (size_t)np * tn * sizeof(double));
    if (phi) memcpy(phi, ph, (size_t)n * np * sizeof(double));
    if (h1out) memcpy(h1out, h1, (size_t)n * sizeof(double));
    free(W); free(V); free(ph); free(h1);
    return 0;
}

/* Per-point interpolated sums for a few listed rows, computing V only at the
 * nodes those rows read: each node value is the full direct sum of Step 2
 * over every node.  Needs the complete charge grids W (oracle_interp_spread).
 * Outputs phi [nrows][P] in the potential order of oracle_interp_rep. */
int oracle_interp_rows(int64_t n, int s, const double* Y, const double* origin,
                       double w, const int* n_int, int p, int form, int kind,
                       const double* W, const int64_t* rows, int64_t nrows,
                       double* phi)
{
    (void)n;
    if (check_box(s, p, n_int)) return -1;
    int ng[3] = {1, 1, 1};
    for (int d = 0; d < s; ++d) ng[d] = n_int[d] * p;
    const int64_t tn = grid_size(s, ng);
    const int np = n_pots(s, form), pps = ipow(p, s);
    const double h = w / p;
    int pk[6], pc[6];
    pot_map(s, form, pk, pc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        int cell[3];
        double L[3][16];
        point_weights(s, Y + i * s, origin, w, n_int, p, cell, L);
        for (int k = 0; k < np; ++k) {
            const double* Wc = W + (int64_t)pc[k] * tn;
            double acc = 0.0;
            for (int q = 0; q < pps; ++q) {
                double l;
                const int64_t g = node_of(s, q, p, cell, L, ng, &l);
                const int gg[3] = {(int)(g % ng[0]), (int)((g / ng[0]) % ng[1]),
                                   (int)(g / ((int64_t)ng[0] * ng[1]))};
                /* node value by the direct sum over all nodes */
                double v = 0.0;
                for (int64_t b = 0; b < tn; ++b) {
                    const int qq[3] = {(int)(b % ng[0]), (int)((b / ng[0]) % ng[1]),
                                       (int)(b / ((int64_t)ng[0] * ng[1]))};
                    int dg[3];
                    for (int d = 0; d < 3; ++d) dg[d] = gg[d] - qq[d];
                    v += kern_lag(s, dg, h, kind, pk[k]) * Wc[b];
                }
                acc += l * v;
            }
            phi[r * np + k] = acc;
        }
    }
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
