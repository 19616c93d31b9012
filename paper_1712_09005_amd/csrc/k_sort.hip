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
// Each pass is reduce, scan, scatter over tiles of 2048 elements, and no
// workgroup ever waits for another:
//   k_key       cell of every point (point order), the first pass's digit
//               count of every tile, and every pass's digit totals;
//   k_hist      (passes after the first) the pass's digit count of every tile
//               of the order the pass before wrote;
//   k_tscan     per digit, an exclusive scan over the tiles of their counts,
//               offset by the count of all smaller digits: each tile's first
//               output position for each digit, in place of the counts;
//   k_sort      a tile ranked stably by its digit in LDS and written out
//               digit run by digit run at the positions k_tscan gave it; the
//               last pass writes the sorted point indices, their cells and
//               the sorted positions;
//   k_bounds    first sorted position of every cell;
//   k_scan_a/b  items (runs of at most kpts points of one cell) per cell and
//               the item -> cell table used by the spreading kernel.
#include "k_common.h"

namespace tsne {

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
// in place.
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
static_assert(kKeyTile == kSortTile, "the first pass's tiles are the key kernel's blocks");

// Digit counts of one tile, per pass, in LDS (a block of 256 threads)
// written out: the tile's row of the count table, all kDigitBins entries.
__device__ __forceinline__ void put_tile_counts(const unsigned* hist, unsigned* row)
{
    const int t = threadIdx.x;
    reinterpret_cast<uint2*>(row)[t] = make_uint2(hist[2 * t], hist[2 * t + 1]);
}

// Cell of every point in point order (stored for the first pass), the first
// pass's digit counts of this tile, and every pass's digit totals over all
// points (one global add per non-zero count of the tile).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_key(LaunchMap map)
{
    __shared__ unsigned hist[kMaxSortPass * kDigitBins];
    VB_BEGIN(map, K_KEY)
    if (live(I)) {
        const Geom& G = *I.geom;
        const int np = I.npass, sb = G.sort_bits;
        const unsigned mask = (1u << sb) - 1u;
        for (int k = threadIdx.x; k < np * kDigitBins; k += 256) hist[k] = 0;
        __syncthreads();
        const T* Y = static_cast<const T*>(I.Yin);
        const int64_t base = (int64_t)lb * kKeyTile;
        constexpr int PER = kKeyTile / 256;
        Pt<T, S> y[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            if (i < I.n) y[r] = Pt<T, S>::load(Y, i);
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            if (i < I.n) {
                const unsigned key = (unsigned)cell_of<T, S>(y[r], G);
                I.key[i] = (int)key;
                for (int p = 0; p < np; ++p)
                    atomicAdd(&hist[p * kDigitBins + digit_of(key, p * sb, mask)], 1u);
            }
        }
        __syncthreads();
        put_tile_counts(hist, I.tcnt + (int64_t)lb * kDigitBins);
        for (int k = threadIdx.x; k < np * kDigitBins; k += 256)
            if (hist[k]) atomicAdd(&I.ghist[k], hist[k]);
        __syncthreads();
    }
    VB_END
}

// Digit counts of every tile for a pass after the first, over the order the
// pass before wrote.
template <int PASS>
__global__ __launch_bounds__(256) void k_hist(LaunchMap map)
{
    constexpr int KIND = (PASS == 1) ? K_HIST1 : K_HIST2;
    constexpr int PER = kSortTile / 256;
    __shared__ unsigned hist[kDigitBins];
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const int sb = I.geom->sort_bits, shift = PASS * sb;
        const unsigned mask = (1u << sb) - 1u;
        const int64_t n = I.n;
        hist[2 * threadIdx.x] = 0;
        hist[2 * threadIdx.x + 1] = 0;
        __syncthreads();
        const uint2* kv_in = static_cast<const uint2*>(I.kv) + (int64_t)((PASS + 1) & 1) * n;
        const int64_t base = (int64_t)lb * kSortTile;
        unsigned key[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int64_t e = base + r * 256 + threadIdx.x;
            key[r] = (e < n) ? kv_in[e].x : 0u;
        }
#pragma unroll
        for (int r = 0; r < PER; ++r)
            if (base + r * 256 + threadIdx.x < n) atomicAdd(&hist[digit_of(key[r], shift, mask)], 1u);
        __syncthreads();
        put_tile_counts(hist, I.tcnt + ((int64_t)PASS * I.ntiles_sort + lb) * kDigitBins);
        __syncthreads();
    }
    VB_END
}

// Tile offsets of one pass, in place: for kScanDigits digits per block (a
// lane each) and kScanWaves segments of the tiles (a wave each), the counts
// are summed per segment, the segment sums scanned across the waves, and the
// segment walked again writing each tile's first output position.
template <int PASS>
__global__ __launch_bounds__(kScanWaves * 64) void k_tscan(LaunchMap map)
{
    constexpr int KIND = K_TSCAN0 + PASS;
    constexpr int U = 8;                               // counts loaded at once
    __shared__ unsigned part[kScanWaves][kScanDigits];
    __shared__ unsigned dbase[kScanDigits];
    static_assert(kScanDigits == 64, "a lane per digit");
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int d0 = lb * kScanDigits;
        if (d0 < (1 << I.geom->sort_bits)) {              // the same for the whole block
            const int d = d0 + lane;
            const int nt = I.ntiles_sort;
            const int seg = (nt + kScanWaves - 1) / kScanWaves;
            const int ta = min(wv * seg, nt), tb = min(ta + seg, nt);
            unsigned* col = I.tcnt + (int64_t)PASS * nt * kDigitBins + d;
            const unsigned* gh = I.ghist + PASS * kDigitBins;
            if (wv == 0) {
                // count of all points with a smaller digit
                unsigned below = 0;
                for (int k = lane; k < d0; k += 64) below += gh[k];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
                const unsigned g = gh[d];
                unsigned x = g;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const unsigned u = __shfl_up(x, o, 64);
                    if (lane >= o) x += u;
                }
                dbase[lane] = below + x - g;
            }
            unsigned sum = 0;
            for (int t = ta; t < tb; t += U) {
                unsigned c[U];
#pragma unroll
                for (int u = 0; u < U; ++u) c[u] = (t + u < tb) ? col[(int64_t)(t + u) * kDigitBins] : 0u;
#pragma unroll
                for (int u = 0; u < U; ++u) sum += c[u];
            }
            part[wv][lane] = sum;
            __syncthreads();
            unsigned off = dbase[lane];
            for (int w = 0; w < wv; ++w) off += part[w][lane];
            for (int t = ta; t < tb; t += U) {
                unsigned c[U];
#pragma unroll
                for (int u = 0; u < U; ++u) c[u] = (t + u < tb) ? col[(int64_t)(t + u) * kDigitBins] : 0u;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (t + u < tb) {
                        col[(int64_t)(t + u) * kDigitBins] = off;
                        off += c[u];
                    }
            }
            __syncthreads();
        }
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
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const Geom& G = *I.geom;
        const int sb = G.sort_bits, shift = PASS * sb;
        const unsigned mask = (1u << sb) - 1u;
        const bool last = (PASS == I.npass - 1);
        const int64_t n = I.n;
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        const int tile = lb;
        for (int k = t; k < 2 * 4 * kDigitBins; k += 256) (&wcnt[0][0][0])[k] = 0;
        run[2 * t] = 0;
        run[2 * t + 1] = 0;
        // this tile's first output position of each digit (from k_tscan)
        const uint2 ofs = reinterpret_cast<const uint2*>(
            I.tcnt + ((int64_t)PASS * I.ntiles_sort + tile) * kDigitBins)[t];
        dbase[2 * t] = ofs.x;
        dbase[2 * t + 1] = ofs.y;
        __syncthreads();
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
        // first LDS slot of each digit: exclusive scan of the tile's counts
        dstart[2 * t] = run[2 * t];
        dstart[2 * t + 1] = run[2 * t + 1];
        __syncthreads();
        block_excl_scan_bins(dstart, wsum);
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
    case K_HIST1: hipLaunchKernelGGL(k_hist<1>, g, b, 0, st, map); break;
    case K_HIST2: hipLaunchKernelGGL(k_hist<2>, g, b, 0, st, map); break;
    case K_TSCAN0: hipLaunchKernelGGL(k_tscan<0>, g, b, 0, st, map); break;
    case K_TSCAN1: hipLaunchKernelGGL(k_tscan<1>, g, b, 0, st, map); break;
    case K_TSCAN2: hipLaunchKernelGGL(k_tscan<2>, g, b, 0, st, map); break;
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
