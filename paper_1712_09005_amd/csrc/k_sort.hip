// Binning of Algorithm 1 on gfx950: the "for each interval" loops of the
// spreading and interpolation steps become one sort of the points by their
// interval cell each iteration.
//
// The sort is a stable least-significant-digit radix sort of (cell, point
// index) pairs, visited in point order, so the result is the canonical order
// by cell and, within a cell, by point index: it depends only on the cells of
// this iteration, not on atomics, launch timing or an earlier iteration, and
// every floating-point sum taken over a cell's points later is reproducible.
//
//   k_key       cell of every point (point order) and the count of every digit
//               value of every pass over all points;
//   k_sort      one launch per pass: a tile of 2048 pairs is ranked stably by
//               its digit in LDS, the tile's digit offsets come from a
//               decoupled look-back over the tiles before it (tiles are taken
//               in launch order from a ticket counter), and the tile is written
//               out digit run by digit run; the last pass writes the sorted
//               point indices, their cells and the sorted positions;
//   k_bounds    first sorted position of every cell;
//   k_scan_a/b  items (runs of at most kpts points of one cell) per cell and
//               the item -> cell table used by the spreading kernel.
#include "k_common.h"

namespace tsne {

// look-back word of one (tile, digit): the sort's epoch in the high 32 bits
// (words of earlier iterations read as "not yet"), a flag and a count
constexpr unsigned long long kLbAgg = 1ull << 30;   // the tile's own count
constexpr unsigned long long kLbInc = 2ull << 30;   // count of this and all earlier tiles
constexpr unsigned kLbCount = (1u << 30) - 1;
constexpr int kSpinLimit = 1 << 20;                 // polls of one word before giving up
constexpr int kLbWindow = 16;                       // earlier tiles requested at once

__device__ __forceinline__ unsigned long long lb_word(unsigned epoch, unsigned long long flag,
                                                      unsigned count)
{
    return ((unsigned long long)epoch << 32) | flag | (unsigned long long)count;
}

// Digits handled by a pass: sort_bits bits from pass * sort_bits up.
__device__ __forceinline__ unsigned digit_of(unsigned key, int shift, unsigned mask)
{
    return (key >> shift) & mask;
}

// Lanes of the wave holding the same digit (among lanes with `valid`), from
// one ballot per digit bit.
__device__ __forceinline__ unsigned long long match_digit(unsigned d, bool valid, int bits)
{
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const unsigned long long set = __ballot(valid && ((d >> b) & 1u));
        m &= ((d >> b) & 1u) ? set : ~set;
    }
    return m;
}

// Exclusive scan over kDigitBins values in LDS by 256 threads (two each),
// in place; returns nothing, the total is not needed.
__device__ __forceinline__ void block_excl_scan_bins(unsigned* v, unsigned* wsum)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const unsigned a = v[2 * t], b = v[2 * t + 1];
    unsigned x = a + b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    unsigned pre = 0;
    for (int w = 0; w < wv; ++w) pre += wsum[w];
    const unsigned ex = pre + x - (a + b);
    v[2 * t] = ex;
    v[2 * t + 1] = ex + a;
    __syncthreads();
}

static_assert(kDigitBins == 2 * 256, "two bins per thread");

// Cell of every point in point order, and the per-pass digit counts over all
// points: the lanes of a wave holding the same digit add their count to LDS
// once (clustered inputs put many points of a block on few digits), and the
// block adds each non-zero count to the global counts once.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_key(LaunchMap map)
{
    __shared__ unsigned hist[kMaxSortPass * kDigitBins];
    VB_BEGIN(map, K_KEY)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int np = I.npass, sb = G.sort_bits;
        const unsigned mask = (1u << sb) - 1u;
        const unsigned long long lt = (1ull << (threadIdx.x & 63)) - 1ull;
        for (int k = threadIdx.x; k < np * kDigitBins; k += 256) hist[k] = 0;
        __syncthreads();
        const T* Y = static_cast<const T*>(I.Yin);
        const int64_t base = (int64_t)lb * kKeyTile;
        for (int r = 0; r < kKeyTile / 256; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            const bool valid = i < I.n;
            unsigned key = 0;
            if (valid) {
                key = (unsigned)cell_of<T, S>(Pt<T, S>::load(Y, i), G);
                I.key[i] = (int)key;
            }
            for (int p = 0; p < np; ++p) {
                const unsigned d = digit_of(key, p * sb, mask);
                const unsigned long long peers = match_digit(d, valid, sb);
                if (valid && (peers & lt) == 0ull)
                    atomicAdd(&hist[p * kDigitBins + d], (unsigned)__popcll(peers));
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < np * kDigitBins; k += 256)
            if (hist[k]) atomicAdd(&I.ghist[k], hist[k]);
        __syncthreads();
    }
    VB_END
}

// One pass of the radix sort over the tiles of one instance (see the file
// comment).  Pass 0 reads the cells of k_key with the identity order; later
// passes read the (cell, index) pairs of the pass before.
template <typename T, int S, int PASS>
__global__ __launch_bounds__(256) void k_sort(LaunchMap map)
{
    constexpr int PER = kSortTile / 256;
    constexpr int KIND = K_SORT0 + PASS;
    __shared__ unsigned wcnt[2][4][kDigitBins];   // per round parity and wave: tag << 16 | count
    __shared__ unsigned run[kDigitBins];          // tile count of each digit so far
    __shared__ unsigned dstart[kDigitBins];       // first LDS slot of each digit in the tile
    __shared__ unsigned dbase[kDigitBins];        // first output position of each digit
    __shared__ uint2 stage[kSortTile];
    __shared__ unsigned wsum[4];
    __shared__ unsigned ticket;
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const Geom& G = *I.geom;
        const int sb = G.sort_bits, shift = PASS * sb;
        const unsigned mask = (1u << sb) - 1u;
        const int nbins = 1 << sb;
        const bool last = (PASS == I.npass - 1);
        const unsigned epoch = G.sort_epoch;
        const int64_t n = I.n;
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        if (t == 0) ticket = atomicAdd(&I.tickets[PASS], 1u);
        for (int k = t; k < 2 * 4 * kDigitBins; k += 256) (&wcnt[0][0][0])[k] = 0;
        run[2 * t] = 0;
        run[2 * t + 1] = 0;
        __syncthreads();
        const int tile = (int)ticket;
        const int64_t base = (int64_t)tile * kSortTile;
        const uint2* kv_in = static_cast<const uint2*>(I.kv) + (int64_t)((PASS + 1) & 1) * n;
        uint2* kv_out = static_cast<uint2*>(I.kv) + (int64_t)(PASS & 1) * n;
        unsigned key[PER];
        int idx[PER];
        unsigned lrank[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int64_t e = base + r * 256 + t;
            key[r] = 0;
            idx[r] = -1;
            lrank[r] = 0;
            if (e < n) {
                if (PASS == 0) {
                    key[r] = (unsigned)I.key[e];
                    idx[r] = (int)e;
                } else {
                    const uint2 q = kv_in[e];
                    key[r] = q.x;
                    idx[r] = (int)q.y;
                }
            }
        }
        // stable ranks within the tile, round by round in element order
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const bool valid = idx[r] >= 0;
            const unsigned d = digit_of(key[r], shift, mask);
            const unsigned long long peers = match_digit(d, valid, sb);
            const unsigned wrank = (unsigned)__popcll(peers & lt);
            const unsigned tag = (unsigned)(r + 1) << 16;
            const int buf = r & 1;
            if (valid && wrank == 0) wcnt[buf][wv][d] = tag | (unsigned)__popcll(peers);
            __syncthreads();
            if (valid) {
                unsigned pre = run[d];
                for (int w = 0; w < wv; ++w) {
                    const unsigned x = wcnt[buf][w][d];
                    if ((x & 0xffff0000u) == tag) pre += x & 0xffffu;
                }
                lrank[r] = pre + wrank;
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int dd = 2 * t + h;
                unsigned add = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const unsigned x = wcnt[buf][w][dd];
                    if ((x & 0xffff0000u) == tag) add += x & 0xffffu;
                }
                run[dd] += add;
            }
        }
        __syncthreads();
        // publish the tile's counts, then look back over earlier tiles for
        // the number of earlier elements of each digit
        unsigned long long* look = I.look + ((int64_t)PASS * I.ntiles_sort + tile) * kDigitBins;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int dd = 2 * t + h;
            if (dd < nbins)
                __hip_atomic_store(look + dd, lb_word(epoch, tile == 0 ? kLbInc : kLbAgg, run[dd]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // digit bases over all points: exclusive scan of the pass's counts
        dbase[2 * t] = (2 * t < nbins) ? I.ghist[PASS * kDigitBins + 2 * t] : 0u;
        dbase[2 * t + 1] = (2 * t + 1 < nbins) ? I.ghist[PASS * kDigitBins + 2 * t + 1] : 0u;
        dstart[2 * t] = run[2 * t];
        dstart[2 * t + 1] = run[2 * t + 1];
        __syncthreads();
        block_excl_scan_bins(dbase, wsum);
        block_excl_scan_bins(dstart, wsum);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int dd = 2 * t + h;
            if (dd >= nbins) continue;
            unsigned excl = 0;
            if (tile > 0) {
                // windows of kLbWindow earlier tiles, nearest first: their words
                // are requested together, then summed in order down to the
                // first inclusive one (an entry not yet published is polled
                // until it is, within kSpinLimit polls)
                const unsigned long long* prev = I.look + ((int64_t)PASS * I.ntiles_sort) * kDigitBins + dd;
                bool found = false;
                for (int j = tile - 1; j >= 0 && !found; j -= kLbWindow) {
                    unsigned long long w[kLbWindow];
#pragma unroll
                    for (int u = 0; u < kLbWindow; ++u)
                        w[u] = (j - u >= 0) ? __hip_atomic_load(prev + (int64_t)(j - u) * kDigitBins,
                                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                            : lb_word(epoch, kLbInc, 0);
#pragma unroll
                    for (int u = 0; u < kLbWindow; ++u) {
                        if (found) break;
                        unsigned long long x = w[u];
                        int spins = 0;
                        while ((unsigned)(x >> 32) != epoch || (x & (3ull << 30)) == 0) {
                            if (++spins > kSpinLimit) {
                                // an earlier tile never published: latch the
                                // condition (the iteration's result is invalid)
                                // instead of waiting for ever
                                atomicCAS(I.status, 0, (int)ST_INTERNAL);
                                x = lb_word(epoch, kLbInc, 0);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            x = __hip_atomic_load(prev + (int64_t)(j - u) * kDigitBins, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                        }
                        excl += (unsigned)(x & kLbCount);
                        if (x & kLbInc) found = true;
                    }
                }
                __hip_atomic_store(look + dd, lb_word(epoch, kLbInc, excl + run[dd]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            dbase[dd] += excl;
        }
        // stage the tile in digit order, then write it out run by run
#pragma unroll
        for (int r = 0; r < PER; ++r)
            if (idx[r] >= 0) stage[dstart[digit_of(key[r], shift, mask)] + lrank[r]] = make_uint2(key[r], (unsigned)idx[r]);
        __syncthreads();
        const int tcount = (int)min<int64_t>(kSortTile, n - base);
        const T* Y = static_cast<const T*>(I.Yin);
        for (int j = t; j < tcount; j += 256) {
            const uint2 q = stage[j];
            const unsigned d = digit_of(q.x, shift, mask);
            const int64_t dst = (int64_t)dbase[d] + (j - (int)dstart[d]);
            if (!last) {
                kv_out[dst] = q;
            } else {
                I.perm[dst] = (int)q.y;
                I.skey[dst] = q.x;
                Pt<T, S>::load(Y, (int64_t)q.y).store(static_cast<T*>(I.sY), dst);
            }
        }
        __syncthreads();
    }
    VB_END
}

// First sorted position of every cell: cell_start[c] = first position whose
// cell is >= c (so empty cells have empty ranges), cell_start[n_cells] = n.
// Each position where the cell changes owns the cells from the previous
// position's cell + 1 to its own; a wave fills the ranges of its positions one
// after another with all 64 lanes, so a long run of empty cells costs one
// store per lane per 64 cells.
__global__ __launch_bounds__(256) void k_bounds(LaunchMap map)
{
    VB_BEGIN(map, K_BOUNDS)
    if (live(I)) {
        const int64_t pos = (int64_t)lb * 256 + threadIdx.x;
        const int lane = threadIdx.x & 63;
        const int ncell = I.geom->n_cells;
        int k = -1, kp = -1;
        if (pos <= I.n) {
            k = (pos < I.n) ? (int)I.skey[pos] : ncell;
            kp = (pos == 0) ? -1 : (int)I.skey[pos - 1];
        }
        unsigned long long m = __ballot(pos <= I.n && k > kp);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const int lo = __shfl(kp, src, 64) + 1, hi = __shfl(k, src, 64);
            const int at = __shfl((int)pos, src, 64);
            for (int c = lo + lane; c <= hi; c += 64) I.cell_start[c] = at;
        }
    }
    VB_END
}

// Exclusive scans of the per-cell item counts (items are runs of at most
// kpts points of one cell), tile sums first.
__device__ __forceinline__ int items_of(int count, int kpts) { return (count + kpts - 1) / kpts; }

__global__ __launch_bounds__(256) void k_scan_a(LaunchMap map)
{
    __shared__ int sh[4];
    VB_BEGIN(map, K_SCAN_A)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int base = lb * 1024 + threadIdx.x * 4;
        int it = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = base + k;
            if (e < ncell) it += items_of(I.cell_start[e + 1] - I.cell_start[e], I.kpts);
        }
        it = wave_sum(it);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) sh[wv] = it;
        __syncthreads();
        if (threadIdx.x == 0) I.scan_part[lb] = sh[0] + sh[1] + sh[2] + sh[3];
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
    constexpr int kSerialItems = 16;     // cells with more items are filled by one wave
    __shared__ int sh[4];
    __shared__ int off;
    __shared__ int nbig;
    __shared__ int big[1024][3];         // (cell, first item, items)
    VB_BEGIN(map, K_SCAN_B)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int ntile = (ncell + 1023) / 1024;
        if (lb < ntile) {
            // offset of this tile: sum of earlier tile sums
            int oi = 0;
            for (int k = threadIdx.x; k < lb; k += 256) oi += I.scan_part[k];
            oi = wave_sum(oi);
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            __syncthreads();
            if (lane == 0) sh[wv] = oi;
            __syncthreads();
            if (threadIdx.x == 0) {
                off = sh[0] + sh[1] + sh[2] + sh[3];
                nbig = 0;
            }
            __syncthreads();
            const int base = lb * 1024 + threadIdx.x * 4;
            int iv[4], it = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = base + k;
                iv[k] = (e < ncell) ? items_of(I.cell_start[e + 1] - I.cell_start[e], I.kpts) : 0;
                it += iv[k];
            }
            const int ii = wave_incl_scan(it);
            __syncthreads();
            if (lane == 63) sh[wv] = ii;
            __syncthreads();
            int pi = off;
            for (int w = 0; w < wv; ++w) pi += sh[w];
            pi += ii - it;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = base + k;
                if (e < ncell) {
                    I.item_start[e] = pi;
                    if (iv[k] <= kSerialItems) {
                        for (int q = 0; q < iv[k]; ++q) I.item_cell[pi + q] = e;
                    } else {
                        const int b = atomicAdd(&nbig, 1);   // at most one per cell of the tile
                        big[b][0] = e;
                        big[b][1] = pi;
                        big[b][2] = iv[k];
                    }
                    if (e == ncell - 1) I.item_start[ncell] = pi + iv[k];
                }
                pi += iv[k];
            }
            // cells with many items (a small box holding many points): the
            // block's four waves take them in turn, each wave's lanes writing
            // one cell's item -> cell entries
            __syncthreads();
            for (int b = wv; b < nbig; b += 4) {
                const int e = big[b][0], p0 = big[b][1], m = big[b][2];
                for (int q = lane; q < m; q += 64) I.item_cell[p0 + q] = e;
            }
            __syncthreads();
        }
    }
    VB_END
}

// ---------------------------------------------------------------- dispatch

template <typename T, int S>
static hipError_t launch_sort_ts(int kind, const LaunchMap& map, const Launch& l, hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_KEY: hipLaunchKernelGGL((k_key<T, S>), g, b, 0, st, map); break;
    case K_SORT0: hipLaunchKernelGGL((k_sort<T, S, 0>), g, b, 0, st, map); break;
    case K_SORT1: hipLaunchKernelGGL((k_sort<T, S, 1>), g, b, 0, st, map); break;
    case K_SORT2: hipLaunchKernelGGL((k_sort<T, S, 2>), g, b, 0, st, map); break;
    case K_BOUNDS: hipLaunchKernelGGL(k_bounds, g, b, 0, st, map); break;
    case K_SCAN_A: hipLaunchKernelGGL(k_scan_a, g, b, 0, st, map); break;
    case K_SCAN_B: hipLaunchKernelGGL(k_scan_b, g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sort_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                            hipStream_t st)
{
    if (c.dtype == 0) return c.s == 1 ? launch_sort_ts<float, 1>(kind, map, l, st)
                                      : launch_sort_ts<float, 2>(kind, map, l, st);
    return c.s == 1 ? launch_sort_ts<double, 1>(kind, map, l, st)
                    : launch_sort_ts<double, 2>(kind, map, l, st);
}

}  // namespace tsne
