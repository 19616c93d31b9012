// Point-side kernels of one t-SNE gradient iteration on gfx950:
//   box geometry, binning by cell (counting sort), charge spreading (Step 1 of
//   Algorithm 1), interpolation back to the points and the Z reduction
//   (Step 3 and the Appendix assembly), sparse attraction (Section 3) and the
//   descent update.
//
// Every kernel walks the virtual blocks of its kind over all instances of the
// launch (VB_BEGIN/VB_END), so one launch serves a single plan or a batch.
#include <math.h>

#include "launch.h"

namespace tsne {

// ---------------------------------------------------------------- helpers

template <typename T> __device__ __forceinline__ T ld(const void* p, int64_t i)
{
    return static_cast<const T*>(p)[i];
}

__device__ __forceinline__ double aload(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the block that finishes last among the
// nblocks blocks sharing this ticket.  Writes made before the call by any of
// those blocks are visible to the last block afterwards.
__device__ __forceinline__ bool last_block(unsigned* ticket, unsigned nblocks, int* flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                            __HIP_MEMORY_SCOPE_AGENT);
        *flag = (t == nblocks - 1);
    }
    __syncthreads();
    const bool last = *flag != 0;
    if (last) __threadfence();
    return last;
}

// Interval of a coordinate value and its local coordinate:
// u = (y - o) / w, l = clamp(floor(u), 0, n_int - 1), t = u - l.
template <typename T>
__device__ __forceinline__ int locate(T y, T o, T w, int n_int, T& t)
{
#pragma clang fp contract(off)
    const T u = (y - o) / w;
    const T f = floor(u);
    int c;
    if (!(f >= (T)0)) c = 0;
    else if (f > (T)(n_int - 1)) c = n_int - 1;
    else c = (int)f;
    t = u - (T)c;
    return c;
}

// 1 / prod_{k != m} (m - k), the denominator of the Lagrange basis on nodes
// m + 1/2 (in units of the node spacing).
__host__ __device__ constexpr double lag_inv_denom(int P, int m)
{
    double d = 1.0;
    for (int k = 0; k < P; ++k)
        if (k != m) d *= (double)(m - k);
    return 1.0 / d;
}

// Lagrange basis of Section 2.1 on the p equispaced nodes (m + 1/2)/p of the
// unit interval, evaluated at t in [0, 1] (eq. (equinodes) for the nodes).
template <typename T, int P>
__device__ __forceinline__ void lagrange(T t, T (&L)[P])
{
    const T sv = t * (T)P;
    T a[P];
#pragma unroll
    for (int k = 0; k < P; ++k) a[k] = sv - ((T)k + (T)0.5);
#pragma unroll
    for (int m = 0; m < P; ++m) {
        T prod = (T)lag_inv_denom(P, m);
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (k != m) prod *= a[k];
        L[m] = prod;
    }
}

template <int S, int FORM> struct Shape {
    static constexpr int NC = (FORM == 0) ? S + 1 : S + 2;   // charges
    static constexpr int NP = S + 2;                          // potentials
};

// ---------------------------------------------------------------- per-call arguments

__global__ void k_set_args(Inst* inst, CallArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (a.set_ptrs) {
        inst->Yin = a.Yin;
        inst->Y = a.Y;
        inst->uY = a.uY;
        inst->gains = a.gains;
        inst->Frep = a.Frep;
        inst->Zout = a.Zout;
        inst->Fattr = a.Fattr;
    }
    if (a.set_P) {
        inst->row_ptr = a.row_ptr;
        inst->col = a.col;
        inst->val = a.val;
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

// ---------------------------------------------------------------- a1: box geometry

// Square box (Section 2.4) with per-dimension origin at the minimum; interval
// count by the policy (paper: max(min, ceil(L)) as in Section 2.5; fixed:
// constant width).  Also the mean (recentring) and the status checks.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_box(LaunchMap map)
{
    __shared__ double sh[4][8];
    __shared__ int flag;
    VB_BEGIN(map, K_BOX)
    if (live(I)) {
        const T* Y = static_cast<const T*>(I.Yin);
        const int64_t n = I.n;
        const int nb = I.nb_box;
        double lo[S], hi[S], sm[S];
        double bad = 0.0;
#pragma unroll
        for (int d = 0; d < S; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; sm[d] = 0.0; }
        for (int64_t i = (int64_t)lb * 256 + threadIdx.x; i < n; i += (int64_t)nb * 256) {
#pragma unroll
            for (int d = 0; d < S; ++d) {
                const double v = (double)Y[i * S + d];
                if (!isfinite(v)) bad = 1.0;
                lo[d] = fmin(lo[d], v);
                hi[d] = fmax(hi[d], v);
                sm[d] += v;
            }
        }
        // wave then block reduction: slots [lo0 lo1 hi0 hi1 sm0 sm1 bad]
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
                sh[wv][2 + d] = hi[d];
                sh[wv][4 + d] = sm[d];
            }
            sh[wv][6] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w)
                for (int d = 0; d < S; ++d) {
                    sh[0][d] = fmin(sh[0][d], sh[w][d]);
                    sh[0][2 + d] = fmax(sh[0][2 + d], sh[w][2 + d]);
                    sh[0][4 + d] += sh[w][4 + d];
                }
            for (int w = 1; w < 4; ++w) sh[0][6] = fmax(sh[0][6], sh[w][6]);
            for (int k = 0; k < 7; ++k) astore(&I.box_part[(int64_t)lb * 8 + k], sh[0][k]);
        }
        if (last_block(&I.tickets[0], (unsigned)nb, &flag)) {
            if (threadIdx.x == 0) {
                double glo[2] = {INFINITY, INFINITY}, ghi[2] = {-INFINITY, -INFINITY};
                double gsm[2] = {0.0, 0.0}, gbad = 0.0;
                for (int b = 0; b < nb; ++b) {
                    const double* pp = I.box_part + (int64_t)b * 8;
                    for (int d = 0; d < S; ++d) {
                        glo[d] = fmin(glo[d], aload(pp + d));
                        ghi[d] = fmax(ghi[d], aload(pp + 2 + d));
                        gsm[d] += aload(pp + 4 + d);
                    }
                    gbad = fmax(gbad, aload(pp + 6));
                }
                Geom& G = *I.geom;
                int st = 0;
                double L = 0.0;
                for (int d = 0; d < S; ++d) {
                    G.origin[d] = glo[d];
                    if (ghi[d] - glo[d] > L) L = ghi[d] - glo[d];
                    G.mean[d] = gsm[d] / (double)n;
                }
                if (gbad != 0.0) st = ST_NONFINITE;
                if (L < 1e-6) L = 1e-6;
                int m;
                double w;
                if (I.policy == 0) {
                    m = (int)fmin(ceil(L), 2.0e9);
                    if (m < I.min_int) m = I.min_int;
                    w = L / m;
                } else {
                    w = I.interval_width;
                    m = (int)fmin(ceil(L / w), 2.0e9);
                    if (m < I.min_int) m = I.min_int;
                }
                if (st == 0 && m > I.max_int) st = ST_CAPACITY;
                if (st != 0) m = I.max_int;   // keep sizes in range for the skipped kernels
                G.side = L;
                G.w = w;
                G.inv_w = 1.0 / w;
                G.h = w / I.p;
                G.n_int = m;
                G.n = m * I.p;
                G.n_cells = (S == 2) ? m * m : m;
                for (int d = 0; d < S; ++d) G.centre[d] = G.origin[d] + 0.5 * m * w;
                // power-of-two charge scale: |(y - centre) * qscale| < 1
                const double halfside = 0.5 * m * w;
                G.qscale = ldexp(1.0, -(ilogb(halfside) + 1));
                G.spec_dirty = (G.h != G.spec_h) ? 1 : 0;
                G.spec_h = G.h;
                if (st != 0)
                    __hip_atomic_store(I.status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&I.tickets[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    VB_END
}

// ---------------------------------------------------------------- a2: binning

// Cell key of each point and its rank among the points of that cell (the
// "for each interval" loops of Algorithm 1 become a counting sort by cell).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_key(LaunchMap map)
{
    VB_BEGIN(map, K_KEY)
    if (live(I)) {
        const int64_t i = (int64_t)lb * 256 + threadIdx.x;
        if (i < I.n) {
            const Geom& G = *I.geom;
            const T* Y = static_cast<const T*>(I.Yin);
            const T w = (T)G.w;
            T t;
            int key = locate<T>(Y[i * S], (T)G.origin[0], w, G.n_int, t);
            if (S == 2) key += G.n_int * locate<T>(Y[i * S + 1], (T)G.origin[1], w, G.n_int, t);
            I.key[i] = key;
            I.rank[i] = atomicAdd(&I.counts[key], 1);
        }
    }
    VB_END
}

// Exclusive scans of the per-cell point counts and item counts (items are
// runs of at most kpts points of one cell), tile sums first.
__device__ __forceinline__ int items_of(int count, int kpts) { return (count + kpts - 1) / kpts; }

__global__ __launch_bounds__(256) void k_scan_a(LaunchMap map)
{
    __shared__ int sh[2][4];
    VB_BEGIN(map, K_SCAN_A)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int base = lb * 1024 + threadIdx.x * 4;
        int c = 0, it = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = base + k;
            if (e < ncell) {
                const int v = I.counts[e];
                c += v;
                it += items_of(v, I.kpts);
            }
        }
        c = wave_sum(c);
        it = wave_sum(it);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) { sh[0][wv] = c; sh[1][wv] = it; }
        __syncthreads();
        if (threadIdx.x == 0) {
            I.scan_part[2 * lb] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
            I.scan_part[2 * lb + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
        }
    }
    VB_END
}

// Inclusive wave scan of an int.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_scan_b(LaunchMap map)
{
    __shared__ int sh[2][4];
    __shared__ int off[2];
    VB_BEGIN(map, K_SCAN_B)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int ntile = (ncell + 1023) / 1024;
        if (lb < ntile) {
            // offset of this tile: sum of earlier tile sums
            int oc = 0, oi = 0;
            for (int k = threadIdx.x; k < lb; k += 256) {
                oc += I.scan_part[2 * k];
                oi += I.scan_part[2 * k + 1];
            }
            oc = wave_sum(oc);
            oi = wave_sum(oi);
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            __syncthreads();
            if (lane == 0) { sh[0][wv] = oc; sh[1][wv] = oi; }
            __syncthreads();
            if (threadIdx.x == 0) {
                off[0] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
                off[1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
            }
            __syncthreads();
            const int base = lb * 1024 + threadIdx.x * 4;
            int cv[4], iv[4], c = 0, it = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = base + k;
                cv[k] = (e < ncell) ? I.counts[e] : 0;
                iv[k] = items_of(cv[k], I.kpts);
                c += cv[k];
                it += iv[k];
            }
            int ic = wave_incl_scan(c), ii = wave_incl_scan(it);
            __syncthreads();
            if (lane == 63) { sh[0][wv] = ic; sh[1][wv] = ii; }
            __syncthreads();
            int pc = off[0], pi = off[1];
            for (int w = 0; w < wv; ++w) { pc += sh[0][w]; pi += sh[1][w]; }
            pc += ic - c;
            pi += ii - it;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = base + k;
                if (e < ncell) {
                    I.cell_start[e] = pc;
                    I.item_start[e] = pi;
                    for (int q = 0; q < iv[k]; ++q) I.item_cell[pi + q] = e;
                    I.counts[e] = 0;          // ready for the next iteration
                    if (e == ncell - 1) {
                        I.cell_start[ncell] = pc + cv[k];
                        I.item_start[ncell] = pi + iv[k];
                    }
                }
                pc += cv[k];
                pi += iv[k];
            }
        }
    }
    VB_END
}

// Scatter: sorted position of every point; sorted copy of Y.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_scatter(LaunchMap map)
{
    VB_BEGIN(map, K_SCATTER)
    if (live(I)) {
        const int64_t i = (int64_t)lb * 256 + threadIdx.x;
        if (i < I.n) {
            const int pos = I.cell_start[I.key[i]] + I.rank[i];
            I.perm[pos] = (int)i;
            const T* Y = static_cast<const T*>(I.Yin);
            T* sY = static_cast<T*>(I.sY);
#pragma unroll
            for (int d = 0; d < S; ++d) sY[(int64_t)pos * S + d] = Y[i * S + d];
        }
    }
    VB_END
}

// ---------------------------------------------------------------- a3: spreading (Step 1)

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
        if (valid) {
            c = I.item_cell[t];
            const int fi = I.item_start[c];
            const int b = I.cell_start[c] + (t - fi) * I.kpts;
            const int e = min(b + I.kpts, I.cell_start[c + 1]);
            const T* sY = static_cast<const T*>(I.sY);
            const T w = (T)G.w, qs = (T)G.qscale;
            const T o0 = (T)G.origin[0], o1 = (T)G.origin[S - 1];
            const T c0 = (T)G.centre[0], c1 = (T)G.centre[S - 1];
            for (int pos = b; pos < e; ++pos) {
                T q[NC];
                T tx, ty = (T)0;
                const T yx = sY[(int64_t)pos * S];
                locate<T>(yx, o0, w, n_int, tx);
                q[0] = (T)1;
                q[1] = (yx - c0) * qs;
                T yy = (T)0;
                if (S == 2) {
                    yy = sY[(int64_t)pos * S + 1];
                    locate<T>(yy, o1, w, n_int, ty);
                    q[2] = (yy - c1) * qs;
                }
                if (FORM == 1) {
                    T r2 = q[1] * q[1];
                    if (S == 2) r2 += q[2] * q[2];
                    q[NC - 1] = r2;
                }
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
            const bool complete = (t_first == I.item_start[c]) && (t == I.item_start[c + 1] - 1);
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
    VB_BEGIN(map, K_FIX)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int c = lb * 256 + threadIdx.x;
        if (c < G.n_cells) {
            const int fi = I.item_start[c], li = I.item_start[c + 1] - 1;
            if (li >= fi && (fi >> 6) != (li >> 6)) {
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
    }
    VB_END
}

// ---------------------------------------------------------------- a8: gather (Step 3) + Z

// phi_k(y_i) = sum_m L_m(y_i) V_k[node m of i's cell], then the Appendix
// assembly: h1 (the K1 sum), numerators y'(d) h4 - h_{1+d}.  One thread per
// sorted position (neighbouring threads share their cell's nodes); results go
// to the point's own index.  Z = sum_i h1_i - N, reduced in double.
template <typename T, int S, int P, int FORM>
__global__ __launch_bounds__(256) void k_gather(LaunchMap map)
{
    constexpr int NP = S + 2;
    __shared__ double sh[8];
    __shared__ int flag;
    VB_BEGIN(map, K_GATHER)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int64_t pos = (int64_t)lb * 256 + threadIdx.x;
        double h1d = 0.0;
        if (pos < I.n) {
            const int n_int = G.n_int, n_cap = I.n_cap;
            const T* sY = static_cast<const T*>(I.sY);
            const T* V = static_cast<const T*>(I.V);
            const T w = (T)G.w, qs = (T)G.qscale;
            T yv[2], tl[2];
            int cl[2] = {0, 0};
#pragma unroll
            for (int d = 0; d < S; ++d) {
                yv[d] = sY[pos * S + d];
                cl[d] = locate<T>(yv[d], (T)G.origin[d], w, n_int, tl[d]);
            }
            T Lx[P], Ly[P];
            lagrange<T, P>(tl[0], Lx);
            if (S == 2) lagrange<T, P>(tl[1], Ly);
            T phi[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                T a = (T)0;
                const T* Vk = V + (int64_t)k * n_cap * (S == 2 ? n_cap : 1);
                if (S == 2) {
#pragma unroll
                    for (int m1 = 0; m1 < P; ++m1) {
                        const T* row = Vk + (int64_t)(cl[1] * P + m1) * n_cap + cl[0] * P;
                        T r = (T)0;
#pragma unroll
                        for (int m0 = 0; m0 < P; ++m0) r += Lx[m0] * row[m0];
                        a += Ly[m1] * r;
                    }
                } else {
                    const T* row = Vk + cl[0] * P;
#pragma unroll
                    for (int m0 = 0; m0 < P; ++m0) a += Lx[m0] * row[m0];
                }
                phi[k] = a;
            }
            // potentials: phi[1] = K2*1, phi[2+d] = K2*(y'(d) qs); phi[0] = K1*1 (A)
            // or K2*(|y'|^2 qs^2) (B)
            T yc[2];
            T r2c = (T)0;
#pragma unroll
            for (int d = 0; d < S; ++d) {
                yc[d] = yv[d] - (T)G.centre[d];
                r2c += yc[d] * yc[d];
            }
            const T inv_qs = (T)1 / qs;
            T h1;
            if (FORM == 0) {
                h1 = phi[0];
            } else {
                T dot = (T)0;
#pragma unroll
                for (int d = 0; d < S; ++d) dot += yc[d] * phi[2 + d];
                h1 = ((T)1 + r2c) * phi[1] - (T)2 * dot * inv_qs + phi[0] * inv_qs * inv_qs;
            }
            const int i = I.perm[pos];
            T* R = static_cast<T*>(I.R);
#pragma unroll
            for (int d = 0; d < S; ++d) R[(int64_t)i * S + d] = yc[d] * phi[1] - phi[2 + d] * inv_qs;
            h1d = (double)h1;
        }
        const double bs = block_sum_d(h1d, sh);
        if (threadIdx.x == 0) astore(&I.z_part[lb], bs);
        if (last_block(&I.tickets[1], (unsigned)I.nb_gather, &flag)) {
            double z = 0.0;
            for (int b = threadIdx.x; b < I.nb_gather; b += 256) z += aload(&I.z_part[b]);
            z = block_sum_d(z, sh);
            if (threadIdx.x == 0) {
                z -= (double)I.n;      // self pairs: K1(0) = 1 per point
                I.geom->Z = z;
                if (I.Zout) *I.Zout = z;
                __hip_atomic_store(&I.tickets[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
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

// ---------------------------------------------------------------- a9: attraction

// F_attr,i = sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2) over row i of the CSR
// P (Section 3).  LPR lanes per row stride over the row's non-zeros; each
// lane accumulates in double, then the lanes of the row are reduced.
template <typename T, int S, int LPR>
__global__ __launch_bounds__(256) void k_attr(LaunchMap map)
{
    VB_BEGIN(map, K_ATTR)
    if (live(I)) {
        constexpr int RPB = 256 / LPR;
        const int64_t i = (int64_t)lb * RPB + threadIdx.x / LPR;
        const int sub = threadIdx.x % LPR;
        double f0 = 0.0, f1 = 0.0;
        const T* Y = static_cast<const T*>(I.Yin);
        if (i < I.n) {
            const T* val = static_cast<const T*>(I.val);
            const T yi0 = Y[i * S];
            const T yi1 = (S == 2) ? Y[i * S + 1] : (T)0;
            const int64_t e = I.row_ptr[i + 1];
            for (int64_t k = I.row_ptr[i] + sub; k < e; k += LPR) {
                const int64_t j = I.col[k];
                const T p = val[k];
                const T d0 = yi0 - Y[j * S];
                T r2 = d0 * d0;
                T d1 = (T)0;
                if (S == 2) {
                    d1 = yi1 - Y[j * S + 1];
                    r2 += d1 * d1;
                }
                const T wgt = p / ((T)1 + r2);
                f0 += (double)(wgt * d0);
                if (S == 2) f1 += (double)(wgt * d1);
            }
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) {
            f0 += __shfl_xor(f0, o, 64);
            if (S == 2) f1 += __shfl_xor(f1, o, 64);
        }
        if (i < I.n && sub == 0) {
            T* F = static_cast<T*>(I.Fattr);
            F[i * S] = (T)f0;
            if (S == 2) F[i * S + 1] = (T)f1;
        }
    }
    VB_END
}

// ---------------------------------------------------------------- a10: update

__device__ __forceinline__ void sched_at(const Sched& sc, int it, double& alpha, double& mom)
{
    if (it >= sc.le_start) alpha = sc.le_alpha;
    else if (it < sc.ee_stop) alpha = sc.ee_alpha;
    else alpha = 1.0;
    mom = (it < sc.mom_switch) ? sc.mom0 : sc.mom1;
}

// grad = 4 (alpha F_attr - F_rep); gains, momentum, step; recentring by the
// mean of the Y the forces were computed on.  The last block advances the
// device iteration counter.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_update(LaunchMap map)
{
    __shared__ int flag;
    VB_BEGIN(map, K_UPDATE)
    if (live(I)) {
        const int it = *I.iter;
        const Sched& sc = *I.sched;
        double alpha, mom;
        sched_at(sc, it, alpha, mom);
        const int64_t i = (int64_t)lb * 256 + threadIdx.x;
        if (i < I.n) {
            const Geom& G = *I.geom;
            const T invz = (T)(1.0 / G.Z);
            T* Y = static_cast<T*>(I.Y);
            T* uY = static_cast<T*>(I.uY);
            T* gains = static_cast<T*>(I.gains);
            const T* Fa = static_cast<const T*>(I.Fattr);
            const T* R = static_cast<const T*>(I.R);
#pragma unroll
            for (int d = 0; d < S; ++d) {
                const int64_t k = i * S + d;
                const T grad = (T)4 * ((T)alpha * Fa[k] - R[k] * invz);
                const T u = uY[k];
                T g = ((grad > (T)0) != (u > (T)0)) ? gains[k] + (T)sc.gain_inc
                                                    : gains[k] * (T)sc.gain_dec;
                if (g < (T)sc.gain_min) g = (T)sc.gain_min;
                gains[k] = g;
                const T un = (T)mom * u - (T)sc.eta * g * grad;
                uY[k] = un;
                const T y = sc.recentre ? (Y[k] - (T)G.mean[d]) : Y[k];
                Y[k] = y + un;
            }
        }
        const unsigned nb = (unsigned)((I.n + 255) / 256);
        if (last_block(&I.tickets[2], nb, &flag)) {
            if (threadIdx.x == 0) {
                *I.iter = it + 1;
                __hip_atomic_store(&I.tickets[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    VB_END
}

// ---------------------------------------------------------------- dispatch

hipError_t launch_fft_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                           hipStream_t st);

template <typename T, int S, int P, int FORM>
static hipError_t launch_pts(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                             hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_BOX: hipLaunchKernelGGL((k_box<T, S>), g, b, 0, st, map); break;
    case K_KEY: hipLaunchKernelGGL((k_key<T, S>), g, b, 0, st, map); break;
    case K_SCAN_A: hipLaunchKernelGGL(k_scan_a, g, b, 0, st, map); break;
    case K_SCAN_B: hipLaunchKernelGGL(k_scan_b, g, b, 0, st, map); break;
    case K_SCATTER: hipLaunchKernelGGL((k_scatter<T, S>), g, b, 0, st, map); break;
    case K_SPREAD: hipLaunchKernelGGL((k_spread<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_FIX: hipLaunchKernelGGL((k_spread_fix<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_GATHER: hipLaunchKernelGGL((k_gather<T, S, P, FORM>), g, b, 0, st, map); break;
    case K_NORM: hipLaunchKernelGGL((k_norm<T, S>), g, b, 0, st, map); break;
    case K_ATTR:
        if (c.lpr == 16) hipLaunchKernelGGL((k_attr<T, S, 16>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr<T, S, 32>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr<T, S, 64>), g, b, 0, st, map);
        break;
    case K_UPDATE: hipLaunchKernelGGL((k_update<T, S>), g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int S, int P>
static hipError_t pts_form(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    return c.form == 0 ? launch_pts<T, S, P, 0>(kind, c, m, l, st)
                       : launch_pts<T, S, P, 1>(kind, c, m, l, st);
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

template <typename T>
static hipError_t pts_s(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    return c.s == 1 ? pts_p<T, 1>(kind, c, m, l, st) : pts_p<T, 2>(kind, c, m, l, st);
}

hipError_t launch_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                       hipStream_t st)
{
    if (l.grid <= 0) return hipSuccess;
    switch (kind) {
    case K_FFT_ROWS: case K_FFT_COLS: case K_FFT_IROWS: case K_FFT_1D:
    case K_SPEC1: case K_SPEC2:
        return launch_fft_kind(kind, c, map, l, st);
    default:
        return c.dtype == 0 ? pts_s<float>(kind, c, map, l, st) : pts_s<double>(kind, c, map, l, st);
    }
}

}  // namespace tsne
