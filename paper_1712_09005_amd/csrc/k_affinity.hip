// Input affinities of Section 1.1 on gfx950, restricted to the k nearest
// neighbours of every point as in Section 3:
//   k_knn   exact k nearest neighbours (squared Euclidean distance, the point
//           itself excluded, equal distances ordered by index): query blocks
//           x candidate tiles staged in LDS, a per-query candidate buffer in
//           LDS that is sorted and cut back to k whenever it could overflow;
//   k_perp  one wave per row: the bandwidth beta_i = 1 / (2 sigma_i^2) by
//           bisection (FP64) so that exp(entropy) of the row equals the
//           target perplexity, then p_{j|i} in FP32;
//   k_sym_* P = (P_cond + P_cond^T) / (2N) as CSR with ascending columns:
//           row counts, a scan, a scatter of both directions, a per-row sort
//           that merges equal columns, a second scan and a compaction.
// Host entry points at the end (declared in tsne.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "../../include/tsne.h"

namespace tsne_aff {

constexpr int QB = 16;       // queries per workgroup
constexpr int CB = 256;      // candidates per tile (one per thread)
constexpr int DC = 32;       // coordinates staged per pass
constexpr int CAP = 512;     // candidate buffer per query (power of two)
constexpr int KMAX = CAP - CB;

// (distance, index) order: ascending distance, then ascending index.
__device__ __forceinline__ bool pair_less(float da, int ia, float db, int ib)
{
    return da < db || (da == db && ia < ib);
}

// Block-wide bitonic sort of the buffers of the flagged queries (CAPv
// entries each, empty slots holding (+inf, INT_MAX)).
template <int QBv, int CAPv>
__device__ void sort_buffers(float* bd, int* bi, const int* flag)
{
    constexpr int PAIRS = QBv * CAPv / 2;
    for (int size = 2; size <= CAPv; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = threadIdx.x; e < PAIRS; e += blockDim.x) {
                const int q = e / (CAPv / 2);
                if (!flag[q]) continue;
                const int r = e - q * (CAPv / 2);
                const int i = 2 * r - (r & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                float* d = bd + q * CAPv;
                int* x = bi + q * CAPv;
                const float di = d[i], dj = d[j];
                const int xi = x[i], xj = x[j];
                if (pair_less(dj, xj, di, xi) == up) {
                    d[i] = dj; d[j] = di;
                    x[i] = xj; x[j] = xi;
                }
            }
            __syncthreads();
        }
    }
}

// Sort the flagged buffers, keep the kk best, reset the rest to empty and
// take the kk-th distance as the new admission threshold.
template <int QBv, int CAPv>
__device__ void compact(float* bd, int* bi, int* cnt, float* thr, int* flag, int kk)
{
    sort_buffers<QBv, CAPv>(bd, bi, flag);
    for (int e = threadIdx.x; e < QBv * CAPv; e += blockDim.x) {
        const int q = e / CAPv, s = e - q * CAPv;
        if (!flag[q] || s < kk) continue;
        bd[e] = INFINITY;
        bi[e] = INT_MAX;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < QBv; q += blockDim.x) {
        if (!flag[q]) continue;
        cnt[q] = min(cnt[q], kk);
        thr[q] = (cnt[q] == kk) ? bd[q * CAPv + kk - 1] : INFINITY;
        flag[q] = 0;
    }
    __syncthreads();
}

// Wave-synchronous step of a sort: the wave's LDS writes are complete and
// visible to its other lanes before it goes on (no block barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of one query's CAPv-entry buffer by one wave.
template <int CAPv>
__device__ void wave_sort(float* d, int* x)
{
    const int lane = threadIdx.x & 63;
    for (int size = 2; size <= CAPv; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int r = lane; r < CAPv / 2; r += 64) {
                const int i = 2 * r - (r & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const float di = d[i], dj = d[j];
                const int xi = x[i], xj = x[j];
                if (pair_less(dj, xj, di, xi) == up) {
                    d[i] = dj; d[j] = di;
                    x[i] = xj; x[j] = xi;
                }
            }
            wave_sync();
        }
    }
}

// Like compact, with each flagged query's buffer sorted by one wave (the
// block's waves take the flagged queries in turn): two block barriers per
// call instead of one per sorting step.
template <int QBv, int CAPv>
__device__ void compact_waves(float* bd, int* bi, int* cnt, float* thr, int* flag, int kk)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int q = threadIdx.x >> 6; q < QBv; q += nw) {
        if (!flag[q]) continue;
        float* d = bd + q * CAPv;
        int* x = bi + q * CAPv;
        wave_sort<CAPv>(d, x);
        for (int s = kk + lane; s < CAPv; s += 64) {
            d[s] = INFINITY;
            x[s] = INT_MAX;
        }
        wave_sync();
        if (lane == 0) {
            cnt[q] = min(cnt[q], kk);
            thr[q] = (cnt[q] == kk) ? d[kk - 1] : INFINITY;
            flag[q] = 0;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_knn(const float* __restrict__ X, int64_t n, int dim, int k,
                                             int32_t* __restrict__ idx, float* __restrict__ dist2)
{
    __shared__ float xq[QB][DC + 1];
    __shared__ float xc[CB][DC + 1];
    __shared__ float bd[QB * CAP];
    __shared__ int bi[QB * CAP];
    __shared__ int cnt[QB];
    __shared__ float thr[QB];
    __shared__ int flag[QB];
    const int64_t q0 = (int64_t)blockIdx.x * QB;
    for (int e = threadIdx.x; e < QB * CAP; e += blockDim.x) {
        bd[e] = INFINITY;
        bi[e] = INT_MAX;
    }
    if (threadIdx.x < QB) {
        cnt[threadIdx.x] = 0;
        thr[threadIdx.x] = INFINITY;
        flag[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += CB) {
        const int64_t c = c0 + threadIdx.x;
        float acc[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) acc[q] = 0.0f;
        for (int d0 = 0; d0 < dim; d0 += DC) {
            for (int e = threadIdx.x; e < QB * DC; e += blockDim.x) {
                const int q = e / DC, dd = e - q * DC;
                xq[q][dd] = (q0 + q < n && d0 + dd < dim) ? X[(q0 + q) * dim + d0 + dd] : 0.0f;
            }
            for (int e = threadIdx.x; e < CB * DC; e += blockDim.x) {
                const int r = e / DC, dd = e - r * DC;
                xc[r][dd] = (c0 + r < n && d0 + dd < dim) ? X[(c0 + r) * dim + d0 + dd] : 0.0f;
            }
            __syncthreads();
            for (int dd = 0; dd < DC; ++dd) {
                const float v = xc[threadIdx.x][dd];
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    const float t = xq[q][dd] - v;
                    acc[q] = fmaf(t, t, acc[q]);
                }
            }
            __syncthreads();
        }
        // admit candidates below each query's threshold (never the query itself)
        if (c < n) {
#pragma unroll
            for (int q = 0; q < QB; ++q) {
                if (q0 + q < n && c != q0 + q && acc[q] < thr[q]) {
                    const int s = atomicAdd(&cnt[q], 1);
                    bd[q * CAP + s] = acc[q];
                    bi[q * CAP + s] = (int)c;
                }
            }
        }
        __syncthreads();
        const bool last = c0 + CB >= n;
        int any = 0;
        if (threadIdx.x < QB) {
            const int q = threadIdx.x;
            flag[q] = (cnt[q] > KMAX || (last && cnt[q] > 0)) ? 1 : 0;
        }
        __syncthreads();
        for (int q = 0; q < QB; ++q) any |= flag[q];
        if (any) compact_waves<QB, CAP>(bd, bi, cnt, thr, flag, k);
    }
    // the buffers now hold the k nearest in order
    for (int e = threadIdx.x; e < QB * k; e += blockDim.x) {
        const int q = e / k, t = e - q * k;
        if (q0 + q < n) {
            idx[(q0 + q) * k + t] = bi[q * CAP + t];
            dist2[(q0 + q) * k + t] = bd[q * CAP + t];
        }
    }
}

// Exact kNN with the dot products on the matrix cores: a 64-query x
// 64-candidate tile per step, each wave one 16-query row of four 16 x 16
// FP32 MFMA tiles (v_mfma_f32_16x16x4f32, K = 4 coordinates per instruction;
// lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and D[4 (l / 16) + r][l % 16]).
// Squared distances |q|^2 + |c|^2 - 2 q.c select the k + 8 best per query
// through the same LDS candidate buffer; those are then recomputed exactly
// over the coordinate differences and re-sorted, so the k returned are
// ordered by their exact FP32 distance (ties by index).  dim <= 56.
constexpr int MQB = 64, MCB = 64, MCAP = 256, MKMAX = MCAP - MCB, MDMAX = 56, MKX = 8;
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_knn_mfma(const float* __restrict__ X, int64_t n, int dim, int k,
                                                  int32_t* __restrict__ idx, float* __restrict__ dist2)
{
    __shared__ float xqT[MDMAX][MQB];
    __shared__ float xcT[MDMAX][MCB + 1];
    __shared__ float qn[MQB], cn[MCB];
    __shared__ float bd[MQB * MCAP];
    __shared__ int bi[MQB * MCAP];
    __shared__ int cnt[MQB], flag[MQB];
    __shared__ float thr[MQB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int dim4 = (dim + 3) & ~3;
    const int kx = k + MKX;
    const int64_t q0 = (int64_t)blockIdx.x * MQB;
    for (int e = tid; e < MQB * dim4; e += 256) {
        const int q = e / dim4, dd = e - q * dim4;
        xqT[dd][q] = (q0 + q < n && dd < dim) ? X[(q0 + q) * dim + dd] : 0.0f;
    }
    for (int e = tid; e < MQB * MCAP; e += 256) {
        bd[e] = INFINITY;
        bi[e] = INT_MAX;
    }
    for (int e = tid; e < MDMAX * (MCB + 1); e += 256) (&xcT[0][0])[e] = 0.0f;   // padding dims stay 0
    const float rdim = 1.0f / (float)dim;
    constexpr int SJ = (MCB * MDMAX + 255) / 256;     // staged values per thread
    __syncthreads();
    if (tid < MQB) {
        float a = 0.0f;
        for (int dd = 0; dd < dim4; ++dd) a = fmaf(xqT[dd][tid], xqT[dd][tid], a);
        qn[tid] = a;
        cnt[tid] = 0;
        flag[tid] = 0;
        thr[tid] = INFINITY;
    }
    const int li = lane & 15, lk = lane >> 4;
    for (int64_t c0 = 0; c0 < n; c0 += MCB) {
        // the chunk is one contiguous run of X: all loads first (coalesced,
        // in flight together), then the transposed LDS stores
        const int64_t base = c0 * dim;
        const int lim = (int)min((int64_t)MCB, n - c0) * dim, tot = MCB * dim;
        float tmp[SJ];
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int e = tid + 256 * j;
            tmp[j] = (e < lim) ? X[base + e] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int e = tid + 256 * j;
            if (e < tot) {
                int c = (int)((float)e * rdim);
                int dd = e - c * dim;
                if (dd < 0) { --c; dd += dim; } else if (dd >= dim) { ++c; dd -= dim; }
                xcT[dd][c] = tmp[j];
            }
        }
        __syncthreads();
        if (tid < MCB) {
            float a = 0.0f;
            for (int dd = 0; dd < dim4; ++dd) a = fmaf(xcT[dd][tid], xcT[dd][tid], a);
            cn[tid] = a;
        }
        v4f acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        for (int kk = 0; kk < dim4; kk += 4) {
            const float a = xqT[kk + lk][16 * w + li];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xcT[kk + lk][16 * t + li], acc[t], 0, 0, 0);
        }
        __syncthreads();                   // cn ready
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qi = 16 * w + 4 * lk + r, cj = 16 * t + li;
                const int64_t cg = c0 + cj;
                const float d = fmaxf(qn[qi] + cn[cj] - 2.0f * acc[t][r], 0.0f);
                if (cg < n && q0 + qi < n && cg != q0 + qi && d < thr[qi]) {
                    const int s = atomicAdd(&cnt[qi], 1);
                    bd[qi * MCAP + s] = d;
                    bi[qi * MCAP + s] = (int)cg;
                }
            }
        }
        __syncthreads();
        if (tid < MQB) flag[tid] = (cnt[tid] > MKMAX) ? 1 : 0;
        __syncthreads();
        int any = 0;
        for (int q = 0; q < MQB; ++q) any |= flag[q];
        if (any) compact_waves<MQB, MCAP>(bd, bi, cnt, thr, flag, kx);
    }
    __syncthreads();
    if (tid < MQB) flag[tid] = 1;
    __syncthreads();
    compact_waves<MQB, MCAP>(bd, bi, cnt, thr, flag, kx);
    // exact distances of the kept candidates, then the final order
    for (int e = tid; e < MQB * kx; e += 256) {
        const int q = e / kx, t = e - q * kx;
        if (q0 + q >= n || t >= cnt[q]) continue;
        const int64_t c = bi[q * MCAP + t];
        const float* xa = X + (q0 + q) * dim;
        const float* xb = X + c * dim;
        float a = 0.0f;
        for (int dd = 0; dd < dim; ++dd) {
            const float u = xa[dd] - xb[dd];
            a = fmaf(u, u, a);
        }
        bd[q * MCAP + t] = a;
    }
    __syncthreads();
    if (tid < MQB) flag[tid] = 1;
    __syncthreads();
    sort_buffers<MQB, MCAP>(bd, bi, flag);
    for (int e = tid; e < MQB * k; e += 256) {
        const int q = e / k, t = e - q * k;
        if (q0 + q < n) {
            idx[(q0 + q) * k + t] = bi[q * MCAP + t];
            dist2[(q0 + q) * k + t] = bd[q * MCAP + t];
        }
    }
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// One wave per row, up to 128 neighbours (two per lane).  The bisection
// follows the definition of perplexity: distances shifted by the row
// minimum, H = ln S + beta sum d' w / S, doubling / halving until the target
// is bracketed, then halving the bracket, until |H - ln perp| < 1e-10 or 200
// steps.
__global__ __launch_bounds__(256) void k_perp(const float* __restrict__ dist2, int64_t n, int k,
                                              double target, float* __restrict__ p,
                                              double* __restrict__ beta_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const float* d = dist2 + row * k;
    const bool h0 = lane < k, h1 = lane + 64 < k;
    double a0 = h0 ? (double)d[lane] : INFINITY;
    double a1 = h1 ? (double)d[lane + 64] : INFINITY;
    const double dmin = wave_min_d(fmin(a0, a1));
    a0 = h0 ? a0 - dmin : 0.0;
    a1 = h1 ? a1 - dmin : 0.0;
    double beta = 1.0, lo = -INFINITY, hi = INFINITY;
    for (int it = 0; it < 200; ++it) {
        const double w0 = h0 ? exp(-beta * a0) : 0.0;
        const double w1 = h1 ? exp(-beta * a1) : 0.0;
        const double S = wave_sum_d(w0 + w1);
        const double SD = wave_sum_d(a0 * w0 + a1 * w1);
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
    const double w0 = h0 ? exp(-beta * a0) : 0.0;
    const double w1 = h1 ? exp(-beta * a1) : 0.0;
    const double S = wave_sum_d(w0 + w1);
    if (h0) p[row * k + lane] = (float)(w0 / S);
    if (h1) p[row * k + lane + 64] = (float)(w1 / S);
    if (beta_out && lane == 0) beta_out[row] = beta;
}

// ---------------------------------------------------------------- symmetrise

__global__ void k_sym_count(const int32_t* __restrict__ idx, int64_t n, int k, int32_t* cnt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    atomicAdd(&cnt[idx[e]], 1);
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) a[e] = v;
}

// Exclusive scan of int32 counts into int64 offsets, three passes: block
// sums of 2048 values, a one-block scan of those sums, then each block's
// values.  out has n + 1 entries (out[n] = total).
constexpr int SCAN_PER = 2048;

__global__ __launch_bounds__(256) void k_scan_sum(const int32_t* __restrict__ a, int64_t n,
                                                  int64_t* __restrict__ bsum)
{
    __shared__ int64_t sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_PER;
    int64_t s = 0;
    for (int t = threadIdx.x; t < SCAN_PER; t += 256)
        if (b0 + t < n) s += a[b0 + t];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t* bsum, int nb)
{
    // one block: exclusive scan of nb block sums in place, in chunks of 256
    __shared__ int64_t sh[256];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const int64_t v = (i < nb) ? bsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int64_t t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ a, int64_t n,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t* __restrict__ out)
{
    // each thread scans 8 consecutive values; the block combines the threads
    __shared__ int64_t sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_PER;
    const int64_t t0 = b0 + (int64_t)threadIdx.x * 8;
    int64_t loc = 0;
    for (int u = 0; u < 8; ++u)
        if (t0 + u < n) loc += a[t0 + u];
    sh[threadIdx.x] = loc;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = bsum[blockIdx.x] + sh[threadIdx.x] - loc;
    for (int u = 0; u < 8; ++u) {
        if (t0 + u < n) {
            out[t0 + u] = run;
            run += a[t0 + u];
        }
        if (t0 + u == n - 1) out[n] = run;
    }
}

// Row i gets its k out-neighbours first (in neighbour order), then the rows
// that list i, in arrival order.
__global__ void k_sym_fill(const int32_t* __restrict__ idx, const float* __restrict__ p, int64_t n,
                           int k, const int64_t* __restrict__ rs, int32_t* cur,
                           int32_t* __restrict__ tcol, float* __restrict__ tval)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int t = (int)(e - i * k);
    const int32_t j = idx[e];
    const float v = p[e];
    tcol[rs[i] + t] = j;
    tval[rs[i] + t] = v;
    const int64_t s = rs[j] + k + atomicAdd(&cur[j], 1);
    tcol[s] = (int32_t)i;
    tval[s] = v;
}

// Sort one row segment by column (bitonic in LDS, length padded to a power of
// two), merge equal columns (sum), scale by 1 / (2N), write the merged row
// back to the start of its segment and its length to len.
template <int MAXL>
__device__ void sort_merge_row(int32_t* tcol, float* tval, int64_t b, int L, int32_t* sc, float* sv,
                               double scale, int32_t* len_out, int nthr, int tid)
{
    int P = 1;
    while (P < L) P <<= 1;
    for (int e = tid; e < P; e += nthr) {
        sc[e] = (e < L) ? tcol[b + e] : INT_MAX;
        sv[e] = (e < L) ? tval[b + e] : 0.0f;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int r = tid; r < P / 2; r += nthr) {
                const int i = 2 * r - (r & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const int ci = sc[i], cj = sc[j];
                if ((cj < ci) == up) {
                    const float vi = sv[i];
                    sc[i] = cj; sc[j] = ci;
                    sv[i] = sv[j]; sv[j] = vi;
                }
            }
            __syncthreads();
        }
    }
    // merge runs of equal columns: a run starts where the column changes
    if (tid == 0) {
        int m = 0;
        for (int e = 0; e < L;) {
            const int c = sc[e];
            double v = 0.0;
            while (e < L && sc[e] == c) v += (double)sv[e++];
            tcol[b + m] = c;
            tval[b + m] = (float)(v * scale);
            ++m;
        }
        *len_out = m;
    }
    __syncthreads();
}

constexpr int ROW_SMALL = 1024;    // rows sorted by one 256-thread block
constexpr int ROW_BIG = 16384;     // rows sorted by one 1024-thread block

__global__ __launch_bounds__(256) void k_sym_sort_small(int32_t* tcol, float* tval,
                                                        const int64_t* __restrict__ rs, int64_t n,
                                                        double scale, int32_t* len)
{
    __shared__ int32_t sc[ROW_SMALL];
    __shared__ float sv[ROW_SMALL];
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t b = rs[i];
        const int L = (int)(rs[i + 1] - b);
        if (L > ROW_SMALL) continue;          // the large-row pass takes it
        sort_merge_row<ROW_SMALL>(tcol, tval, b, L, sc, sv, scale, len + i, 256, threadIdx.x);
    }
}

__global__ __launch_bounds__(1024) void k_sym_sort_big(int32_t* tcol, float* tval,
                                                       const int64_t* __restrict__ rs, int64_t n,
                                                       double scale, int32_t* len, int* status)
{
    extern __shared__ __align__(16) char smem[];
    int32_t* sc = reinterpret_cast<int32_t*>(smem);
    float* sv = reinterpret_cast<float*>(sc + ROW_BIG);
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t b = rs[i];
        const int64_t L = rs[i + 1] - b;
        if (L <= ROW_SMALL) continue;
        if (L > ROW_BIG) {                     // not supported: report, leave the row empty
            if (threadIdx.x == 0) {
                atomicOr(status, 1);
                len[i] = 0;
            }
            continue;
        }
        sort_merge_row<ROW_BIG>(tcol, tval, b, (int)L, sc, sv, scale, len + i, 1024, threadIdx.x);
    }
}

__global__ void k_sym_compact(const int32_t* __restrict__ tcol, const float* __restrict__ tval,
                              const int64_t* __restrict__ rs, const int64_t* __restrict__ rp,
                              int64_t n, int32_t* __restrict__ col, float* __restrict__ val)
{
    // one wave per row
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const int64_t src = rs[i], dst = rp[i], L = rp[i + 1] - rp[i];
    for (int64_t e = lane; e < L; e += 64) {
        col[dst + e] = tcol[src + e];
        val[dst + e] = tval[src + e];
    }
}

// Workspace layout of tsne_symmetrize (bytes, 256-aligned regions).
struct SymLayout {
    size_t cnt, cur, len, rs, bsum, tcol, tval, status, total;
};

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

static SymLayout sym_layout(int64_t n, int32_t k)
{
    SymLayout L;
    const int64_t nb = (n + SCAN_PER) / SCAN_PER + 1;
    size_t off = 0;
    L.cnt = off; off += up256(sizeof(int32_t) * (size_t)n);
    L.cur = off; off += up256(sizeof(int32_t) * (size_t)n);
    L.len = off; off += up256(sizeof(int32_t) * (size_t)n);
    L.rs = off; off += up256(sizeof(int64_t) * (size_t)(n + 1));
    L.bsum = off; off += up256(sizeof(int64_t) * (size_t)nb);
    L.tcol = off; off += up256(sizeof(int32_t) * (size_t)(2 * n * k));
    L.tval = off; off += up256(sizeof(float) * (size_t)(2 * n * k));
    L.status = off; off += 256;
    L.total = off;
    return L;
}

static hipError_t scan_i32(const int32_t* a, int64_t n, int64_t* bsum, int64_t* out, hipStream_t st)
{
    const int nb = (int)((n + SCAN_PER - 1) / SCAN_PER);
    if (nb == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_sum, dim3(nb), dim3(256), 0, st, a, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, a, n, bsum, out);
    return hipGetLastError();
}

}  // namespace tsne_aff

using namespace tsne_aff;

extern "C" {

tsne_status tsne_knn(const float* X, int64_t n, int32_t dim, int32_t k, int32_t* idx, float* dist2,
                     void* stream)
{
    if (!X || !idx || !dist2 || n < 2 || dim < 1 || k < 1 || k >= n || n > INT_MAX)
        return TSNE_E_ARG;
    if (k > KMAX) return TSNE_E_UNSUPPORTED;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (dim <= MDMAX && k + MKX <= MKMAX && k + MKX < n) {
        const int64_t nb = (n + MQB - 1) / MQB;
        hipLaunchKernelGGL(k_knn_mfma, dim3((unsigned)nb), dim3(256), 0, st, X, n, (int)dim, (int)k, idx,
                           dist2);
    } else {
        const int64_t nb = (n + QB - 1) / QB;
        hipLaunchKernelGGL(k_knn, dim3((unsigned)nb), dim3(CB), 0, st, X, n, (int)dim, (int)k, idx, dist2);
    }
    return hipGetLastError() == hipSuccess ? TSNE_OK : TSNE_E_HIP;
}

tsne_status tsne_perplexity(const float* dist2, int64_t n, int32_t k, double perplexity, float* p,
                            double* beta, void* stream)
{
    if (!dist2 || !p || n < 1 || k < 1 || !(perplexity > 0.0)) return TSNE_E_ARG;
    if (k > 128) return TSNE_E_UNSUPPORTED;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nb = (n + 3) / 4;
    hipLaunchKernelGGL(k_perp, dim3((unsigned)nb), dim3(256), 0, st, dist2, n, (int)k, std::log(perplexity),
                       p, beta);
    return hipGetLastError() == hipSuccess ? TSNE_OK : TSNE_E_HIP;
}

size_t tsne_symmetrize_workspace_bytes(int64_t n, int32_t k)
{
    if (n < 2 || k < 1) return 0;
    return sym_layout(n, k).total;
}

tsne_status tsne_symmetrize(const int32_t* idx, const float* p, int64_t n, int32_t k, void* workspace,
                            size_t bytes, void* stream, int64_t* row_ptr, int32_t* col, float* val,
                            int* status)
{
    if (!idx || !p || !row_ptr || !col || !val || n < 2 || k < 1 || n > INT_MAX) return TSNE_E_ARG;
    const SymLayout L = sym_layout(n, k);
    if (!workspace || ((uintptr_t)workspace % 256) != 0 || bytes < L.total) return TSNE_E_WORKSPACE;
    char* w = static_cast<char*>(workspace);
    int32_t* cnt = reinterpret_cast<int32_t*>(w + L.cnt);
    int32_t* cur = reinterpret_cast<int32_t*>(w + L.cur);
    int32_t* len = reinterpret_cast<int32_t*>(w + L.len);
    int64_t* rs = reinterpret_cast<int64_t*>(w + L.rs);
    int64_t* bsum = reinterpret_cast<int64_t*>(w + L.bsum);
    int32_t* tcol = reinterpret_cast<int32_t*>(w + L.tcol);
    float* tval = reinterpret_cast<float*>(w + L.tval);
    int* st_dev = status ? status : reinterpret_cast<int*>(w + L.status);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nk = n * k;
    const unsigned g_n = (unsigned)((n + 255) / 256), g_nk = (unsigned)((nk + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3(g_n), dim3(256), 0, st, cnt, n, (int32_t)k);
    hipLaunchKernelGGL(k_fill_i32, dim3(g_n), dim3(256), 0, st, cur, n, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, st_dev, (int64_t)1, 0);
    hipLaunchKernelGGL(k_sym_count, dim3(g_nk), dim3(256), 0, st, idx, n, (int)k, cnt);
    if (scan_i32(cnt, n, bsum, rs, st) != hipSuccess) return TSNE_E_HIP;
    hipLaunchKernelGGL(k_sym_fill, dim3(g_nk), dim3(256), 0, st, idx, p, n, (int)k, rs, cur, tcol, tval);
    const double scale = 1.0 / (2.0 * (double)n);
    const unsigned g_rows = (unsigned)std::min<int64_t>(n, 4096);
    hipLaunchKernelGGL(k_sym_sort_small, dim3(g_rows), dim3(256), 0, st, tcol, tval, rs, n, scale, len);
    const size_t big_lds = (size_t)ROW_BIG * (sizeof(int32_t) + sizeof(float));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_sym_sort_big),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)big_lds);
    hipLaunchKernelGGL(k_sym_sort_big, dim3((unsigned)std::min<int64_t>(n, 256)), dim3(1024), big_lds, st,
                       tcol, tval, rs, n, scale, len, st_dev);
    if (scan_i32(len, n, bsum, row_ptr, st) != hipSuccess) return TSNE_E_HIP;
    hipLaunchKernelGGL(k_sym_compact, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, tcol, tval, rs,
                       row_ptr, n, col, val);
    return hipGetLastError() == hipSuccess ? TSNE_OK : TSNE_E_HIP;
}

}  // extern "C"
