// Point-side kernels of one t-SNE gradient iteration on gfx950:
//   box geometry, binning by cell (counting sort), charge spreading (Step 1 of
//   Algorithm 1), interpolation back to the points and the Z reduction
//   (Step 3 and the Appendix assembly) and the descent update.  The sparse
//   attraction and the divergence are in k_attr.hip.
//
// Every kernel walks the virtual blocks of its kind over all instances of the
// launch (VB_BEGIN/VB_END), so one launch serves a single plan or a batch.
#include "k_common.h"

namespace tsne {

// ---------------------------------------------------------------- helpers

// ---------------------------------------------------------------- per-call arguments

__global__ void k_set_args(Inst* inst, CallArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (a.set_ptrs) {
        inst->counting = a.counting;
        inst->Yin = a.Yin;
        inst->Y = a.Y;
        inst->uY = a.uY;
        inst->gains = a.gains;
        inst->Frep = a.Frep;
        inst->Zout = a.Zout;
        inst->Fattr = a.Fattr;
        inst->KLout = a.KLout;
    }
    if (a.set_P) {
        inst->row_ptr = a.row_ptr;
        inst->col = a.col;
        inst->val = a.val;
        inst->tscale = a.tscale;
    }
    if (a.set_sched) *inst->sched = a.sched;
    if (a.set_iter) *inst->iter = a.iter;
    if (a.set_end) inst->iter_end = a.iter_end;
}

hipError_t launch_set_args(Inst* inst, const CallArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_args, dim3(1), dim3(64), 0, st, inst, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- box geometry

// Per-block partial min / max / sum of the coordinates (double) and a
// non-finite flag, kBoxPart doubles per block (minima at 0, maxima at 4,
// sums at 8, the flag at 12).  The geometry kernel reduces them.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_box(LaunchMap map)
{
    __shared__ double sh[4][kBoxPart];
    VB_BEGIN(map, K_BOX)
    if (live_pre(I)) {
        const T* Y = static_cast<const T*>(I.Yin);
        const int64_t n = I.n;
        const int nb = I.nb_box;
        double lo[S], hi[S], sm[S];
        double bad = 0.0;
#pragma unroll
        for (int d = 0; d < S; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; sm[d] = 0.0; }
        // four points a round, their loads in flight together (a point past
        // n loads the round's first point and is not counted)
        const int64_t stride = (int64_t)nb * 256;
        for (int64_t i0 = (int64_t)lb * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
            Pt<T, S> y[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = i0 + q * stride;
                y[q] = Pt<T, S>::load(Y, i < n ? i : i0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (i0 + q * stride >= n) continue;
#pragma unroll
                for (int d = 0; d < S; ++d) {
                    const double v = (double)y[q].v[d];
                    if (!isfinite(v)) bad = 1.0;
                    lo[d] = fmin(lo[d], v);
                    hi[d] = fmax(hi[d], v);
                    sm[d] += v;
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int d = 0; d < S; ++d) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
                sm[d] += __shfl_xor(sm[d], o, 64);
            }
            bad = fmax(bad, __shfl_xor(bad, o, 64));
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) {
            for (int d = 0; d < S; ++d) {
                sh[wv][d] = lo[d];
                sh[wv][4 + d] = hi[d];
                sh[wv][8 + d] = sm[d];
            }
            sh[wv][12] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double* out = I.box_part + (int64_t)lb * kBoxPart;
            for (int d = 0; d < S; ++d) {
                out[d] = fmin(fmin(sh[0][d], sh[1][d]), fmin(sh[2][d], sh[3][d]));
                out[4 + d] = fmax(fmax(sh[0][4 + d], sh[1][4 + d]), fmax(sh[2][4 + d], sh[3][4 + d]));
                out[8 + d] = ((sh[0][8 + d] + sh[1][8 + d]) + sh[2][8 + d]) + sh[3][8 + d];
            }
            out[12] = fmax(fmax(sh[0][12], sh[1][12]), fmax(sh[2][12], sh[3][12]));
        }
    }
    VB_END
}

// Smallest M >= lo of the form 4^a 3^b 5^c with a >= 1 (radix-4, 3 and 5
// stages only).
__device__ __forceinline__ int ladder(int lo)
{
    for (int M = (lo + 3) & ~3;; M += 4) {
        int r = M;
        while (r % 4 == 0) r /= 4;
        while (r % 3 == 0) r /= 3;
        while (r % 5 == 0) r /= 5;
        if (r == 1) return M;
    }
}

// One block per instance: reduce the box partials, decide the iteration
// (status checks, iteration counter) and its geometry.  Square box (Section
// 2.4) of side n_int * w centred on each dimension's mid-range (for the
// widest dimension under the paper policy the origin is its minimum, and a
// narrower dimension keeps its points inside the node hull); interval count by the
// policy (paper: max(min, ceil(L)) as in Section 2.5; fixed: constant width);
// circulant length M from the 2-3-5 ladder with hysteresis, so the tables are
// rebuilt only when the node count leaves [M/3, M/2].  With rect set, a
// narrower second dimension gets its own interval count and FFT length at the
// same spacing.

// Circulant length of one axis with hysteresis, and its radix plan when it
// changes.  Returns true if M changed.
__device__ __forceinline__ bool axis_plan(int nodes, int Mcap, int& Mref, int& half, int& nstages,
                                          int* radix, int* tw_off)
{
    int M = Mref;
    // keep M while 2n <= M <= 3n: the ladder length for 2n is then at least
    // 2M/3, so the hysteresis test below would keep it (and the ladder
    // search, a few microseconds on one lane, is skipped)
    if (M >= 2 * nodes && M <= Mcap && M <= 3 * nodes) return false;
    const int want = ladder(2 * nodes);
    if (M < 2 * nodes || M > Mcap || want * 3 < M * 2) M = want;
    if (M > Mcap) M = Mcap;
    if (M == Mref) return false;
    int r = M, k = 0, n4 = 0, n3 = 0, n5 = 0;
    while (r % 4 == 0) { r /= 4; ++n4; }
    while (r % 3 == 0) { r /= 3; ++n3; }
    while (r % 5 == 0) { r /= 5; ++n5; }
    for (int q = 0; q < n4; ++q) radix[k++] = 4;
    for (int q = 0; q < n3; ++q) radix[k++] = 3;
    for (int q = 0; q < n5; ++q) radix[k++] = 5;
    nstages = k;
    Mref = M;
    half = M / 2 + 1;
    int off = 0, ns = 1;
    for (int q = 0; q < k; ++q) {
        tw_off[q] = off;
        off += ns * (radix[q] - 1);
        ns *= radix[q];
    }
    return true;
}

template <int S>
__global__ __launch_bounds__(256) void k_geom(LaunchMap map)
{
    __shared__ double sh[4][kBoxPart];
    VB_BEGIN(map, K_GEOM)
    Geom& G = *I.geom;
    const bool run = live_pre(I);
    // the record's fields through the constant view: scalar loads, issued
    // together instead of one round trip after each store to the geometry
    const TSNE_CONST Inst& R = *cview<Inst>(&I);
    if (run) {
        const int nb = R.nb_box;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double sm[3] = {0.0, 0.0, 0.0}, bad = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) {
            const double* pp = R.box_part + (int64_t)b * kBoxPart;
            for (int d = 0; d < S; ++d) {
                lo[d] = fmin(lo[d], pp[d]);
                hi[d] = fmax(hi[d], pp[4 + d]);
                sm[d] += pp[8 + d];
            }
            bad = fmax(bad, pp[12]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int d = 0; d < S; ++d) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
                sm[d] += __shfl_xor(sm[d], o, 64);
            }
            bad = fmax(bad, __shfl_xor(bad, o, 64));
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) {
            for (int d = 0; d < S; ++d) {
                sh[wv][d] = lo[d];
                sh[wv][4 + d] = hi[d];
                sh[wv][8 + d] = sm[d];
            }
            sh[wv][12] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double glo[3], ghi[3], gsm[3];
            for (int d = 0; d < S; ++d) {
                glo[d] = fmin(fmin(sh[0][d], sh[1][d]), fmin(sh[2][d], sh[3][d]));
                ghi[d] = fmax(fmax(sh[0][4 + d], sh[1][4 + d]), fmax(sh[2][4 + d], sh[3][4 + d]));
                gsm[d] = ((sh[0][8 + d] + sh[1][8 + d]) + sh[2][8 + d]) + sh[3][8 + d];
            }
            const double gbad = fmax(fmax(sh[0][12], sh[1][12]), fmax(sh[2][12], sh[3][12]));
            int st = 0;
            double L = 0.0;
            for (int d = 0; d < S; ++d) {
                if (ghi[d] - glo[d] > L) L = ghi[d] - glo[d];
                G.mean[d] = gsm[d] / (double)R.n;
            }
            if (gbad != 0.0) st = ST_NONFINITE;
            if (L < 1e-6) L = 1e-6;
            int m;
            double w;
            if (R.policy == 0) {
                m = (int)fmin(ceil(L), 2.0e9);
                if (m < R.min_int) m = R.min_int;
                w = L / m;
            } else if (L < R.interval_width * R.min_int) {
                // a box narrower than min_int intervals: shrink the intervals
                // to L / min_int, as the paper's interval count does
                m = R.min_int;
                w = L / m;
            } else {
                w = R.interval_width;
                m = (int)fmin(ceil(L / w), 2.0e9);
                if (m < R.min_int) m = R.min_int;
            }
            if (st == 0 && m > R.max_int) st = ST_CAPACITY;
            if (st != 0) {
                *R.status = st;            // latched; the iteration is not committed
                G.active = 0;
            } else {
                G.active = 1;
                G.it = *R.iter;
                if (R.counting) *R.iter = G.it + 1;
                G.side = L;
                G.w = w;
                G.inv_w = 1.0 / w;
                G.h = w / R.p;
                // per-axis interval counts: the square box, or a rectangle of
                // the same spacing whose narrower axes get their own counts
                int ma[3] = {m, m, m};
                for (int d = 0; d < S; ++d) {
                    const double Ld = ghi[d] - glo[d];
                    if (R.rect && S == 2 && Ld < L) {
                        int md = (int)ceil(Ld / w);
                        if (md < R.min_int) md = R.min_int;
                        if (md > m) md = m;
                        ma[d] = md;
                    }
                }
                G.n_int = ma[0];
                G.n = ma[0] * R.p;
                // s = 3 has the square box only: every axis has n_int intervals
                G.n_int_y = (S >= 2) ? ma[1] : 1;
                G.n_y = (S >= 2) ? ma[1] * R.p : 1;
                G.n_cells = (S == 3) ? ma[0] * ma[1] * ma[2] : (S == 2) ? ma[0] * ma[1] : ma[0];
                // explicit roundings (no contraction) so the origin is the
                // correctly rounded value of mid - (m/2) w
                for (int d = 0; d < S; ++d) {
                    const double half_side = __dmul_rn(0.5 * ma[d], w);
                    G.origin[d] = __dsub_rn(__dmul_rn(0.5, __dadd_rn(glo[d], ghi[d])), half_side);
                    G.centre[d] = __dadd_rn(G.origin[d], half_side);
                }
                // power-of-two charge scale: |(y - centre) * qscale| < 1
                G.qscale = ldexp(1.0, -(ilogb(0.5 * m * w) + 1));
                // circulant lengths with hysteresis, per axis
                axis_plan(G.n, R.M, G.M, G.half, G.nstages, G.radix, G.tw_off);
                if (S == 2 &&
                    axis_plan(G.n_y, R.M, G.My, G.half_y, G.nstages_y, G.radix_y, G.tw_off_y)) {
                    // columns per block: as many as the LDS holds (power of two)
                    const int csz = 2 * ((R.tile_w == 16) ? 4 : 8);
                    int g = R.tile_w;
                    while (g > 1 && (int64_t)g * lds_stride(G.My) * csz > R.col_lds) g >>= 1;
                    G.col_group = g;
                }
                G.spec_dirty = (G.h != G.spec_h || G.M != G.spec_M || (S == 2 && G.My != G.spec_My)) ? 1 : 0;
                G.spec_h = G.h;
                G.spec_M = G.M;
                G.spec_My = G.My;
                // radix sort of this iteration: digit width for the cell count
                const int nc1 = G.n_cells - 1;
                const int bits = (nc1 > 0) ? 32 - __clz(nc1) : 1;
                G.sort_bits = (bits + R.npass - 1) / R.npass;
            }
        }
    } else if (threadIdx.x == 0) {
        G.active = 0;
    }
    VB_END
}

// ---------------------------------------------------------------- spreading (Step 1)

// One thread per item (up to kpts consecutive sorted points of one cell):
// w_{m,c} += L_m(y_i) q_c(i) accumulated in registers, then a segmented
// reduction across the wave by cell.  A cell whose items all lie in one wave
// is written directly; a cell crossing waves leaves per-wave partials that
// k_spread_fix adds in wave order.  No atomics on floating-point values.
template <typename T, int S, int P, int FORM>
__global__ __launch_bounds__(256) void k_spread(LaunchMap map)
{
    constexpr int NC = Shape<S, FORM>::NC;
    constexpr int NN = (S == 2) ? P * P : P;
    VB_BEGIN(map, K_SPREAD)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int n_int = G.n_int, ncell = G.n_cells, n_cap = I.n_cap;
        const int total = I.item_start[ncell];
        const int t = lb * 256 + threadIdx.x;
        const bool valid = t < total;
        const int lane = threadIdx.x & 63;
        int c = -1;
        T acc[NN][NC];
#pragma unroll
        for (int k = 0; k < NN; ++k)
#pragma unroll
            for (int q = 0; q < NC; ++q) acc[k][q] = (T)0;
        int fi = 0, li = 0;                // the cell's first and one-past-last item
        if (valid) {
            c = I.item_cell[t];
            fi = I.item_start[c];
            li = I.item_start[c + 1];
            const int b = I.cell_start[c] + (t - fi) * I.kpts;
            const int e = min(b + I.kpts, I.cell_start[c + 1]);
            const T* sY = static_cast<const T*>(I.sY);
            const double w = G.w, qs = G.qscale;
            const double o0 = G.origin[0], o1 = G.origin[S - 1];
            const double c0 = G.centre[0], c1 = G.centre[S - 1];
            // positions loaded PF at a time, before the first is used (the
            // first batch before the item's end is known: clamped to the array)
            constexpr int PF = 4;
            const int last = (int)I.n - 1;
            int p0 = b;
            do {
              Pt<T, S> ypf[PF];
#pragma unroll
              for (int u = 0; u < PF; ++u) ypf[u] = Pt<T, S>::load(sY, min(p0 + u, last));
#pragma unroll
              for (int u = 0; u < PF; ++u) {
                if (p0 + u >= e) break;
                T q[NC];
                T tx, ty = (T)0;
                const Pt<T, S> yp = ypf[u];
                const T yx = yp.v[0];
                locate<T>(yx, o0, w, n_int, tx);
                // centred, power-of-two scaled charges, rounded once from double
                const double qx = ((double)yx - c0) * qs;
                double qy = 0.0;
                q[0] = (T)1;
                if (NC > 1) q[1 % NC] = (T)qx;
                if (S == 2) {
                    const T yy = yp.v[S - 1];
                    locate<T>(yy, o1, w, G.n_int_y, ty);
                    qy = ((double)yy - c1) * qs;
                    if (NC > 2) q[2 % NC] = (T)qy;
                }
                if (FORM == 1) q[NC - 1] = (T)(qx * qx + qy * qy);
                T Lx[P];
                lagrange<T, P>(tx, Lx);
                if (S == 2) {
                    T Ly[P];
                    lagrange<T, P>(ty, Ly);
#pragma unroll
                    for (int m1 = 0; m1 < P; ++m1)
#pragma unroll
                        for (int m0 = 0; m0 < P; ++m0) {
                            const T wgt = Ly[m1] * Lx[m0];
#pragma unroll
                            for (int qq = 0; qq < NC; ++qq) acc[m1 * P + m0][qq] += wgt * q[qq];
                        }
                } else {
#pragma unroll
                    for (int m0 = 0; m0 < P; ++m0)
#pragma unroll
                        for (int qq = 0; qq < NC; ++qq) acc[m0][qq] += Lx[m0] * q[qq];
                }
              }
              p0 += PF;
            } while (p0 < e);
        }
        // ---- segmented inclusive scan over the lanes of the wave, by cell
        const int cprev = __shfl_up(c, 1, 64);
        const bool head = (lane == 0) || (cprev != c);
        const unsigned long long hm = __ballot(head);
        const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
        const int run_start = 63 - __clzll(hm & upto);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const bool take = (lane - o) >= run_start;
#pragma unroll
            for (int k = 0; k < NN; ++k)
#pragma unroll
                for (int qq = 0; qq < NC; ++qq) {
                    const T u = __shfl_up(acc[k][qq], o, 64);
                    if (take) acc[k][qq] += u;
                }
        }
        const bool run_end = (lane == 63) || ((hm >> (lane + 1)) & 1ull);
        if (valid && run_end) {
            const int t_first = t - (lane - run_start);
            const bool complete = (t_first == fi) && (t == li - 1);
            if (complete) {
                T* W = static_cast<T*>(I.W);
                const int cx = c % n_int;
                const int cy = (S == 2) ? c / n_int : 0;
#pragma unroll
                for (int qq = 0; qq < NC; ++qq) {
                    if (S == 2) {
#pragma unroll
                        for (int m1 = 0; m1 < P; ++m1)
#pragma unroll
                            for (int m0 = 0; m0 < P; ++m0)
                                W[((int64_t)qq * n_cap + cy * P + m1) * n_cap + cx * P + m0] =
                                    acc[m1 * P + m0][qq];
                    } else {
#pragma unroll
                        for (int m0 = 0; m0 < P; ++m0)
                            W[(int64_t)qq * n_cap + cx * P + m0] = acc[m0][qq];
                    }
                }
            } else {
                const int slot = (run_start == 0) ? 0 : 1;
                T* cr = static_cast<T*>(I.carry) + ((int64_t)(t >> 6) * 2 + slot) * (NN * NC);
#pragma unroll
                for (int k = 0; k < NN; ++k)
#pragma unroll
                    for (int qq = 0; qq < NC; ++qq) cr[k * NC + qq] = acc[k][qq];
            }
        }
    }
    VB_END
}

// Cells whose items cross wave boundaries: add the per-wave partials in wave
// order (the first wave's run is its last run, unless the cell starts the
// wave; every later wave holds the cell as its first run).
template <typename T, int S, int P, int FORM>
__global__ __launch_bounds__(256) void k_spread_fix(LaunchMap map)
{
    constexpr int NC = Shape<S, FORM>::NC;
    constexpr int NN = (S == 2) ? P * P : P;
    constexpr int kSerialWaves = 16;     // cells spanning more waves are summed by the block
    constexpr int NV = NN * NC;
    constexpr int NG = 256 / NV;         // wave groups summed in parallel per value (>= 1)
    __shared__ int nbig;
    __shared__ int bigc[256];
    __shared__ float part[NG > 0 ? NG : 1][NV];
    __shared__ double partd[NG > 0 ? NG : 1][NV];
    static_assert(NG >= 1, "carry vector longer than a block");
    VB_BEGIN(map, K_FIX)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int c = lb * 256 + threadIdx.x;
        if (threadIdx.x == 0) nbig = 0;
        __syncthreads();
        if (c < G.n_cells) {
            const int fi = I.item_start[c], li = I.item_start[c + 1] - 1;
            if (li >= fi && (li >> 6) - (fi >> 6) > kSerialWaves) {
                bigc[atomicAdd(&nbig, 1)] = c;
            } else if (li >= fi && (fi >> 6) != (li >> 6)) {
                const int w0 = fi >> 6, w1 = li >> 6;
                const T* cr = static_cast<const T*>(I.carry);
                T acc[NN * NC];
                const T* first = cr + ((int64_t)w0 * 2 + ((fi & 63) == 0 ? 0 : 1)) * (NN * NC);
#pragma unroll
                for (int k = 0; k < NN * NC; ++k) acc[k] = first[k];
                for (int wv = w0 + 1; wv <= w1; ++wv) {
                    const T* pp = cr + (int64_t)wv * 2 * (NN * NC);
#pragma unroll
                    for (int k = 0; k < NN * NC; ++k) acc[k] += pp[k];
                }
                T* W = static_cast<T*>(I.W);
                const int n_int = G.n_int, n_cap = I.n_cap;
                const int cx = c % n_int;
                const int cy = (S == 2) ? c / n_int : 0;
#pragma unroll
                for (int qq = 0; qq < NC; ++qq) {
                    if (S == 2) {
#pragma unroll
                        for (int m1 = 0; m1 < P; ++m1)
#pragma unroll
                            for (int m0 = 0; m0 < P; ++m0)
                                W[((int64_t)qq * n_cap + cy * P + m1) * n_cap + cx * P + m0] =
                                    acc[(m1 * P + m0) * NC + qq];
                    } else {
#pragma unroll
                        for (int m0 = 0; m0 < P; ++m0)
                            W[(int64_t)qq * n_cap + cx * P + m0] = acc[m0 * NC + qq];
                    }
                }
            }
        }
        __syncthreads();
        // cells spanning many waves: thread (g, v) sums value v over the waves
        // w0 + 1 + g, w0 + 1 + g + NG, ...; the NG partial sums and the first
        // wave's carry are then added in a fixed order (deterministic)
        const T* cr = static_cast<const T*>(I.carry);
        for (int b = 0; b < nbig; ++b) {
            const int cb = bigc[b];
            const int fi = I.item_start[cb], li = I.item_start[cb + 1] - 1;
            const int w0 = fi >> 6, w1 = li >> 6;
            const int g = threadIdx.x / NV, v = threadIdx.x - g * NV;
            if (g < NG) {
                T a = (T)0;
                for (int wv = w0 + 1 + g; wv <= w1; wv += NG) a += cr[(int64_t)wv * 2 * NV + v];
                if constexpr (sizeof(T) == 4) part[g][v] = a; else partd[g][v] = (double)a;
            }
            __syncthreads();
            if (threadIdx.x < NV) {
                const int vv = threadIdx.x;
                T a = cr[((int64_t)w0 * 2 + ((fi & 63) == 0 ? 0 : 1)) * NV + vv];
                for (int gg = 0; gg < NG; ++gg) {
                    if constexpr (sizeof(T) == 4) a += (T)part[gg][vv]; else a += (T)partd[gg][vv];
                }
                T* W = static_cast<T*>(I.W);
                const int n_int = G.n_int, n_cap = I.n_cap;
                const int cx = cb % n_int;
                const int cy = (S == 2) ? cb / n_int : 0;
                const int qq = vv % NC, mm = vv / NC;
                if (S == 2) {
                    const int m1 = mm / P, m0 = mm - m1 * P;
                    W[((int64_t)qq * n_cap + cy * P + m1) * n_cap + cx * P + m0] = a;
                } else {
                    W[(int64_t)qq * n_cap + cx * P + mm] = a;
                }
            }
            __syncthreads();
        }
    }
    VB_END
}

// ---------------------------------------------------------------- gather (Step 3) + Z

// phi_k(y_i) = sum_m L_m(y_i) V_k[node m of i's cell], then the Appendix
// assembly: h1 (the K1 sum), numerators y'(d) h4 - h_{1+d} (form V: the
// numerators are the odd-kernel potentials themselves).  One thread per item
// (up to kpts consecutive sorted points of one cell, the spreading kernel's
// items): the cell's NP p^s node potentials are loaded once (held in
// registers when they fit, FP32 with at most 100 values) and every point of
// the item is interpolated from them; results go to the point's own index.
// (Several threads per item, each loading the potentials, took longer: the
// loads, not the latency, then dominate.)  Z = sum_i h1_i - N, reduced in
// double: per thread over its item's points in order, then per block, then
// over the blocks in k_zsum.
template <typename T, int S, int P, int FORM>
__global__ __launch_bounds__(256) void k_gather(LaunchMap map)
{
    constexpr int NP = Shape<S, FORM>::NP;
    constexpr int NN = (S == 2) ? P * P : P;
    constexpr bool HOLD = (sizeof(T) == 4 && NP * NN <= 100) || NP * NN <= 32;
    constexpr int PF = 8;                                // positions loaded at once
    __shared__ double sh[8];
    VB_BEGIN(map, K_GATHER)
    if (live(I)) {
        // the record and geometry through the constant view (scalar loads),
        // the item tables through the global view (no flat loads)
        const TSNE_CONST Inst& Rc = *cview<Inst>(&I);
        const TSNE_CONST Geom& G = *cview<Geom>(Rc.geom);
        const int ncell = G.n_cells;
        const int total = cview<int>(Rc.item_start)[ncell];
        const int t = lb * 256 + (int)threadIdx.x;
        double h1d = 0.0;
        if (t < total) {
            const TSNE_GLOBAL int* cstart = gview<int>(Rc.cell_start);
            const int n_int = G.n_int, n_cap = Rc.n_cap;
            const int c = gview<int>(Rc.item_cell)[t];
            const int b = cstart[c] + (t - gview<int>(Rc.item_start)[c]) * Rc.kpts;
            const int e = min(b + Rc.kpts, cstart[c + 1]);
            const int cx = c % n_int, cy = (S == 2) ? c / n_int : 0;
            const T* sY = static_cast<const T*>(Rc.sY);
            const T* V = static_cast<const T*>(Rc.V);
            const int64_t plane = (int64_t)n_cap * (S == 2 ? n_cap : 1);
            // node (m1, m0) of the cell in potential k
            auto vidx = [&](int k, int m) -> int64_t {
                const int m1 = (S == 2) ? m / P : 0, m0 = m - m1 * P;
                return (int64_t)k * plane + (int64_t)(cy * P + m1) * (S == 2 ? n_cap : 0) + cx * P + m0;
            };
            T vh[HOLD ? NP : 1][HOLD ? NN : 1];
            if constexpr (HOLD) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
#pragma unroll
                    for (int m = 0; m < NN; ++m) vh[k][m] = V[vidx(k, m)];
            }
            const double w = G.w, qs = G.qscale;
            const double inv_qs = 1.0 / qs;
            // positions PF at a time; the first batch is requested before the
            // item's end is known (indices clamped to the array)
            const int last = (int)I.n - 1;
            int p0 = b;
            do {
                Pt<T, S> yp[PF];
                int ip[PF];
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int pos = min(p0 + u, last);
                    yp[u] = Pt<T, S>::load(sY, pos);
                    ip[u] = I.perm[pos];
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    if (p0 + u >= e) break;
                    T yv[2], tl[2];
#pragma unroll
                    for (int d = 0; d < S; ++d) {
                        yv[d] = yp[u].v[d];
                        locate<T>(yv[d], G.origin[d], w, d == 0 ? n_int : G.n_int_y, tl[d]);
                    }
                    T Lx[P], Ly[P];
                    lagrange<T, P>(tl[0], Lx);
                    if (S == 2) lagrange<T, P>(tl[1], Ly);
                    T phi[NP];
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        T a = (T)0;
                        if (S == 2) {
#pragma unroll
                            for (int m1 = 0; m1 < P; ++m1) {
                                T r = (T)0;
#pragma unroll
                                for (int m0 = 0; m0 < P; ++m0)
                                    r += Lx[m0] * (HOLD ? vh[HOLD ? k : 0][HOLD ? m1 * P + m0 : 0]
                                                        : V[vidx(k, m1 * P + m0)]);
                                a += Ly[m1] * r;
                            }
                        } else {
#pragma unroll
                            for (int m0 = 0; m0 < P; ++m0)
                                a += Lx[m0] * (HOLD ? vh[HOLD ? k : 0][HOLD ? m0 : 0] : V[vidx(k, m0)]);
                        }
                        phi[k] = a;
                    }
                    // potentials: phi[1] = K2*1, phi[2+d] = K2*(y'(d) qs); phi[0] = K1*1 (A)
                    // or K2*(|y'|^2 qs^2) (B); form V: phi[0] = K1*1, phi[1+d] = (z_d K2)*1
                    // assembly in double: the numerator y'(d) h4 - h_{1+d} cancels
                    double yc[2];
                    double r2c = 0.0;
#pragma unroll
                    for (int d = 0; d < S; ++d) {
                        yc[d] = (double)yv[d] - G.centre[d];
                        r2c += yc[d] * yc[d];
                    }
                    double h1;
                    if (FORM == 0 || FORM == 2) {
                        h1 = (double)phi[0];
                    } else {
                        double dot = 0.0;
#pragma unroll
                        for (int d = 0; d < S; ++d) dot += yc[d] * (double)phi[(2 + d) % NP];
                        h1 = (1.0 + r2c) * (double)phi[1] - 2.0 * dot * inv_qs +
                             (double)phi[0] * inv_qs * inv_qs;
                    }
                    const int i = ip[u];
                    Pt<T, S> rv;
#pragma unroll
                    for (int d = 0; d < S; ++d)
                        rv.v[d] = (FORM == 2) ? phi[1 + d]
                                              : (T)(yc[d] * (double)phi[1] - (double)phi[(2 + d) % NP] * inv_qs);
                    rv.store(static_cast<T*>(I.R), i);
                    if (I.h1keep) I.h1keep[i] = h1;
                    h1d += h1;
                }
                p0 += PF;
            } while (p0 < e);
        }
        const double bs = block_sum_d(h1d, sh);
        if (threadIdx.x == 0) I.z_part[lb] = bs;
    }
    VB_END
}

// ---------------------------------------------------------------- s = 3

// Step 1 for s = 3 (Section 2: the s + 2 sums hold for any s; Section 2.4's
// tensor-product nodes on a cube): one thread per (cell, node) of the p^3
// nodes of a cell, summing the cell's points' charges times the node's
// Lagrange weight L_m0(x) L_m1(y) L_m2(z), in sorted (point index) order.
// Every node of every cell is written, an empty cell's with zeros, so the
// grid needs no clearing and no partial sums cross threads.
template <typename T, int P, int FORM>
__global__ __launch_bounds__(256) void k_spread3(LaunchMap map)
{
    constexpr int NC = Shape<3, FORM>::NC;
    constexpr int NN = P * P * P;
    VB_BEGIN(map, K_SPREAD3)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int64_t t = (int64_t)lb * 256 + threadIdx.x;
        const int c = (int)(t / NN), m = (int)(t - (int64_t)c * NN);
        if (c < G.n_cells) {
            const int n_int = G.n_int, n_cap = I.n_cap;
            const int cx = c % n_int, cy = (c / n_int) % n_int, cz = c / (n_int * n_int);
            const int m0 = m % P, m1 = (m / P) % P, m2 = m / (P * P);
            const T* sY = static_cast<const T*>(I.sY);
            const double w = G.w, qs = G.qscale;
            T acc[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) acc[q] = (T)0;
            const int e = I.cell_start[c + 1];
            for (int pos = I.cell_start[c]; pos < e; ++pos) {
                const Pt<T, 3> yp = Pt<T, 3>::load(sY, pos);
                T tl[3], q[NC];
                double qd[3], r2 = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    locate<T>(yp.v[d], G.origin[d], w, n_int, tl[d]);
                    // centred, power-of-two scaled charges, rounded once from double
                    qd[d] = ((double)yp.v[d] - G.centre[d]) * qs;
                    r2 += qd[d] * qd[d];
                }
                q[0] = (T)1;
#pragma unroll
                for (int d = 0; d < 3; ++d) q[1 + d] = (T)qd[d];
                if (FORM == 1) q[NC - 1] = (T)r2;
                T Lx[P], Ly[P], Lz[P];
                lagrange<T, P>(tl[0], Lx);
                lagrange<T, P>(tl[1], Ly);
                lagrange<T, P>(tl[2], Lz);
                const T wgt = Lz[m2] * Ly[m1] * Lx[m0];
#pragma unroll
                for (int qq = 0; qq < NC; ++qq) acc[qq] += wgt * q[qq];
            }
            T* W = static_cast<T*>(I.W);
            const int64_t node = ((int64_t)(cz * P + m2) * n_cap + (cy * P + m1)) * n_cap + cx * P + m0;
            const int64_t plane = (int64_t)n_cap * n_cap * n_cap;
#pragma unroll
            for (int qq = 0; qq < NC; ++qq) W[qq * plane + node] = acc[qq];
        }
    }
    VB_END
}

// Step 3 for s = 3: one thread per sorted position, phi_k = sum over the
// cell's p^3 nodes of L_m0(x) L_m1(y) L_m2(z) V_k, then the Appendix assembly
// as for s = 1, 2 (forms A and B); Z partials per block in double.
template <typename T, int P, int FORM>
__global__ __launch_bounds__(256) void k_gather3(LaunchMap map)
{
    constexpr int NP = Shape<3, FORM>::NP;
    __shared__ double sh[8];
    VB_BEGIN(map, K_GATHER3)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int64_t pos = (int64_t)lb * 256 + threadIdx.x;
        double h1d = 0.0;
        if (pos < I.n) {
            const int n_int = G.n_int, n_cap = I.n_cap;
            const Pt<T, 3> yp = Pt<T, 3>::load(static_cast<const T*>(I.sY), pos);
            T tl[3];
            int cl[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) cl[d] = locate<T>(yp.v[d], G.origin[d], G.w, n_int, tl[d]);
            T Lx[P], Ly[P], Lz[P];
            lagrange<T, P>(tl[0], Lx);
            lagrange<T, P>(tl[1], Ly);
            lagrange<T, P>(tl[2], Lz);
            const T* V = static_cast<const T*>(I.V);
            const int64_t plane = (int64_t)n_cap * n_cap * n_cap;
            T phi[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                T a = (T)0;
#pragma unroll
                for (int m2 = 0; m2 < P; ++m2) {
                    T b = (T)0;
#pragma unroll
                    for (int m1 = 0; m1 < P; ++m1) {
                        const T* row = V + k * plane +
                                       ((int64_t)(cl[2] * P + m2) * n_cap + (cl[1] * P + m1)) * n_cap + cl[0] * P;
                        T r = (T)0;
#pragma unroll
                        for (int m0 = 0; m0 < P; ++m0) r += Lx[m0] * row[m0];
                        b += Ly[m1] * r;
                    }
                    a += Lz[m2] * b;
                }
                phi[k] = a;
            }
            // potentials: phi[1] = K2*1, phi[2+d] = K2*(y'(d) qs); phi[0] = K1*1 (A)
            // or K2*(|y'|^2 qs^2) (B); the assembly in double
            const double inv_qs = 1.0 / G.qscale;
            double yc[3], r2c = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                yc[d] = (double)yp.v[d] - G.centre[d];
                r2c += yc[d] * yc[d];
            }
            double h1;
            if (FORM == 0) {
                h1 = (double)phi[0];
            } else {
                double dot = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) dot += yc[d] * (double)phi[2 + d];
                h1 = (1.0 + r2c) * (double)phi[1] - 2.0 * dot * inv_qs + (double)phi[0] * inv_qs * inv_qs;
            }
            const int i = I.perm[pos];
            Pt<T, 3> rv;
#pragma unroll
            for (int d = 0; d < 3; ++d) rv.v[d] = (T)(yc[d] * (double)phi[1] - (double)phi[2 + d] * inv_qs);
            rv.store(static_cast<T*>(I.R), i);
            if (I.h1keep) I.h1keep[i] = h1;
            h1d = h1;
        }
        const double bs = block_sum_d(h1d, sh);
        if (threadIdx.x == 0) I.z_part[lb] = bs;
    }
    VB_END
}

// One block per instance: Z = sum_i h1_i - N (the self pairs, K1(0) = 1),
// from the gather's block partials in a fixed order.
__global__ __launch_bounds__(256) void k_zsum(LaunchMap map)
{
    __shared__ double sh[8];
    VB_BEGIN(map, K_ZSUM)
    if (live(I)) {
        // four independent partial sums per thread, so their loads are in
        // flight together (a fixed order: the result is reproducible)
        const double* zp = I.z_part;
        const int nb = I.nb_gather;
        double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
        int b = threadIdx.x;
        for (; b + 768 < nb; b += 1024) {
            z0 += zp[b];
            z1 += zp[b + 256];
            z2 += zp[b + 512];
            z3 += zp[b + 768];
        }
        for (; b < nb; b += 256) z0 += zp[b];
        double z = block_sum_d((z0 + z1) + (z2 + z3), sh);
        if (threadIdx.x == 0) {
            z -= (double)I.n;
            I.geom->Z = z;
            if (I.Zout) *I.Zout = z;
        }
    }
    VB_END
}

// F_rep = numerator / Z for the repulsion entry point.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_norm(LaunchMap map)
{
    VB_BEGIN(map, K_NORM)
    if (live(I)) {
        const int64_t i = (int64_t)lb * 256 + threadIdx.x;
        if (i < I.n * S) {
            const double z = I.geom->Z;
            static_cast<T*>(I.Frep)[i] = (T)((double)static_cast<const T*>(I.R)[i] / z);
        }
    }
    VB_END
}

// ---------------------------------------------------------------- update

__device__ __forceinline__ void sched_at(const TSNE_CONST Sched& sc, int it, double& alpha, double& mom)
{
    if (it >= sc.le_start) alpha = sc.le_alpha;
    else if (it < sc.ee_stop) alpha = sc.ee_alpha;
    else alpha = 1.0;
    mom = (it < sc.mom_switch) ? sc.mom0 : sc.mom1;
}

// grad = 4 (alpha F_attr - F_rep); gains, momentum, step; recentring by the
// mean of the Y the forces were computed on.  The schedule is indexed by the
// iteration the geometry kernel assigned.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_update(LaunchMap map)
{
    VB_BEGIN(map, K_UPDATE)
    if (live(I)) {
        // the record, geometry and schedule through the constant view: scalar
        // loads, issued beside the vector loads of the points
        const TSNE_CONST Inst& Rc = *cview<Inst>(&I);
        const TSNE_CONST Geom& G = *cview<Geom>(Rc.geom);
        const TSNE_CONST Sched& sc = *cview<Sched>(Rc.sched);
        double alpha, mom;
        sched_at(sc, G.it, alpha, mom);
        const T invz = (T)(1.0 / G.Z);
        T* Y = static_cast<T*>(Rc.Y);
        T* uY = static_cast<T*>(Rc.uY);
        T* gains = static_cast<T*>(Rc.gains);
        const T* Fa = static_cast<const T*>(Rc.Fattr);
        const T* Fp = static_cast<const T*>(Rc.Fap);
        const T* R = static_cast<const T*>(Rc.R);
        const int64_t n = Rc.n, ns = n * S;
        // kUpdPts points per thread, 256 apart: all their loads are issued
        // first, then the arithmetic, then the stores; each point's S
        // components move as one vector per array (8 or 16 bytes in 2-D)
        const int64_t i0 = (int64_t)lb * (256 * kUpdPts) + threadIdx.x;
        Pt<T, S> fa[kUpdPts], r[kUpdPts], u[kUpdPts], g[kUpdPts], y[kUpdPts];
#pragma unroll
        for (int q = 0; q < kUpdPts; ++q) {
            const int64_t i = min(i0 + (int64_t)q * 256, n - 1);   // past n: a repeat, not stored
            if (Rc.slabs == 1) {
                fa[q] = Pt<T, S>::load(Fa, i);
            } else {
                // every slab's partial in flight at once, then summed in slab order
                constexpr int kMaxSlabs = 8;
                Pt<T, S> p[kMaxSlabs];
#pragma unroll
                for (int sl = 0; sl < kMaxSlabs; ++sl)
                    if (sl < Rc.slabs) p[sl] = Pt<T, S>::load(Fp + (int64_t)sl * ns, i);
                double a[S];
#pragma unroll
                for (int d = 0; d < S; ++d) a[d] = 0.0;
#pragma unroll
                for (int sl = 0; sl < kMaxSlabs; ++sl)
                    if (sl < Rc.slabs) {
#pragma unroll
                        for (int d = 0; d < S; ++d) a[d] += (double)p[sl].v[d];
                    }
#pragma unroll
                for (int d = 0; d < S; ++d) fa[q].v[d] = (T)a[d];
            }
            r[q] = Pt<T, S>::load(R, i);
            u[q] = Pt<T, S>::load(uY, i);
            g[q] = Pt<T, S>::load(gains, i);
            y[q] = Pt<T, S>::load(Y, i);
        }
#pragma unroll
        for (int q = 0; q < kUpdPts; ++q) {
#pragma unroll
            for (int d = 0; d < S; ++d) {
                const T grad = (T)4 * ((T)alpha * fa[q].v[d] - r[q].v[d] * invz);
                T gd = ((grad > (T)0) != (u[q].v[d] > (T)0)) ? g[q].v[d] + (T)sc.gain_inc
                                                             : g[q].v[d] * (T)sc.gain_dec;
                if (gd < (T)sc.gain_min) gd = (T)sc.gain_min;
                g[q].v[d] = gd;
                const T un = (T)mom * u[q].v[d] - (T)sc.eta * gd * grad;
                u[q].v[d] = un;
                const T yd = sc.recentre ? (y[q].v[d] - (T)G.mean[d]) : y[q].v[d];
                y[q].v[d] = yd + un;
            }
        }
#pragma unroll
        for (int q = 0; q < kUpdPts; ++q) {
            const int64_t i = i0 + (int64_t)q * 256;
            if (i < n) {
                g[q].store(gains, i);
                u[q].store(uY, i);
                y[q].store(Y, i);
            }
        }
    }
    VB_END
}

// ---------------------------------------------------------------- dispatch

hipError_t launch_fft_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                           hipStream_t st);
hipError_t launch_attr_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                            hipStream_t st);
hipError_t launch_sort_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                            hipStream_t st);

template <typename T, int S, int P, int FORM>
static hipError_t launch_pts(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                             hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_BOX: hipLaunchKernelGGL((k_box<T, S>), g, b, 0, st, map); break;
    case K_SPREAD: hipLaunchKernelGGL((k_spread<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_FIX: hipLaunchKernelGGL((k_spread_fix<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_GATHER: hipLaunchKernelGGL((k_gather<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_GEOM: hipLaunchKernelGGL((k_geom<S>), g, b, 0, st, map); break;
    case K_ZSUM: hipLaunchKernelGGL(k_zsum, g, b, 0, st, map); break;
    case K_NORM: hipLaunchKernelGGL((k_norm<T, S>), g, b, 0, st, map); break;
    case K_UPDATE: hipLaunchKernelGGL((k_update<T, S>), g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int S, int P>
static hipError_t pts_form(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    switch (c.form) {
    case 0: return launch_pts<T, S, P, 0>(kind, c, m, l, st);
    case 1: return launch_pts<T, S, P, 1>(kind, c, m, l, st);
    case 2: return launch_pts<T, S, P, 2>(kind, c, m, l, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int S>
static hipError_t pts_p(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    switch (c.p) {
    case 2: return pts_form<T, S, 2>(kind, c, m, l, st);
    case 3: return pts_form<T, S, 3>(kind, c, m, l, st);
    case 4: return pts_form<T, S, 4>(kind, c, m, l, st);
    case 5: return pts_form<T, S, 5>(kind, c, m, l, st);
    case 6: return pts_form<T, S, 6>(kind, c, m, l, st);
    default: return hipErrorInvalidValue;
    }
}

// s = 3: forms A and B only
template <typename T, int P, int FORM>
static hipError_t launch_pts3(int kind, const LaunchMap& map, const Launch& l, hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_BOX: hipLaunchKernelGGL((k_box<T, 3>), g, b, 0, st, map); break;
    case K_GEOM: hipLaunchKernelGGL((k_geom<3>), g, b, 0, st, map); break;
    case K_SPREAD3: hipLaunchKernelGGL((k_spread3<T, P, FORM>), g, b, 0, st, map); break;
    case K_GATHER3: hipLaunchKernelGGL((k_gather3<T, P, FORM>), g, b, 0, st, map); break;
    case K_ZSUM: hipLaunchKernelGGL(k_zsum, g, b, 0, st, map); break;
    case K_NORM: hipLaunchKernelGGL((k_norm<T, 3>), g, b, 0, st, map); break;
    case K_UPDATE: hipLaunchKernelGGL((k_update<T, 3>), g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t pts3_form(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    return c.form == 0 ? launch_pts3<T, P, 0>(kind, m, l, st) : launch_pts3<T, P, 1>(kind, m, l, st);
}

template <typename T>
static hipError_t pts3_p(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    switch (c.p) {
    case 2: return pts3_form<T, 2>(kind, c, m, l, st);
    case 3: return pts3_form<T, 3>(kind, c, m, l, st);
    case 4: return pts3_form<T, 4>(kind, c, m, l, st);
    case 5: return pts3_form<T, 5>(kind, c, m, l, st);
    case 6: return pts3_form<T, 6>(kind, c, m, l, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t pts_s(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    if (c.s == 3) return pts3_p<T>(kind, c, m, l, st);
    return c.s == 1 ? pts_p<T, 1>(kind, c, m, l, st) : pts_p<T, 2>(kind, c, m, l, st);
}

hipError_t launch_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                       hipStream_t st)
{
    if (l.grid <= 0) return hipSuccess;
    switch (kind) {
    case K_FFT_ROWS: case K_FFT_COLS: case K_FFT_IROWS: case K_FFT_1D:
    case K_SPEC0: case K_SPEC1: case K_SPEC2:
    case K_F3_X: case K_F3_Y: case K_F3_Z: case K_F3_IY: case K_F3_IX:
    case K_S3_FILL: case K_S3_X: case K_S3_Y: case K_S3_Z: case K_S3_STORE:
        return launch_fft_kind(kind, c, map, l, st);
    case K_ATTR: case K_ATTR_ALL: case K_ATTR_T: case K_ATTR_T_ALL: case K_ASUM: case K_KL_ATTR:
    case K_KL_T:
    case K_KLSUM:
        return launch_attr_kind(kind, c, map, l, st);
    case K_KEY: case K_HIST1: case K_HIST2: case K_TSCAN0: case K_TSCAN1: case K_TSCAN2:
    case K_SORT0: case K_SORT1: case K_SORT2: case K_BOUNDS: case K_SCAN_A: case K_SCAN_B:
        return launch_sort_kind(kind, c, map, l, st);
    default:
        return c.dtype == 0 ? pts_s<float>(kind, c, map, l, st) : pts_s<double>(kind, c, map, l, st);
    }
}

}  // namespace tsne
