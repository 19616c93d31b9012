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
//   k_key       cell of every point (point order) and the first pass's digit
//               count of every tile;
//   k_hist      (passes after the first) the pass's digit count of every tile
//               of the order the pass before wrote;
//   k_tscan     the tiles in groups of group_tiles: per group and digit, an
//               exclusive scan of the counts over the group's tiles (in place)
//               and the group's total;
//   k_sort      a tile ranked stably by its digit in LDS and written out
//               digit run by digit run: a digit's run starts at the count of
//               all smaller digits (a scan of the totals over the groups),
//               plus the digit's count in earlier groups, plus its count in
//               earlier tiles of the group; the last pass writes the sorted
//               point indices, their cells and the sorted positions;
//   k_bounds    first sorted position of every cell;
//   k_scan_a/b  items (runs of at most kpts points of one cell) per cell and
//               the item -> cell table used by the spreading and
//               interpolation kernels.
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

// A pair of 32-bit words as a native vector (loads and stores through the
// global view)
typedef unsigned U2 __attribute__((ext_vector_type(2)));

// Digit counts of one tile, per pass, in LDS (a block of 256 threads)
// written out: the tile's row of the count table, all kDigitBins entries.
__device__ __forceinline__ void put_tile_counts(const unsigned* hist, unsigned* row)
{
    const int t = threadIdx.x;
    reinterpret_cast<uint2*>(row)[t] = make_uint2(hist[2 * t], hist[2 * t + 1]);
}

// Cell of every point in point order (stored for the first pass) and the
// first pass's digit counts of this tile.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_key(LaunchMap map)
{
    __shared__ unsigned hist[kDigitBins];
    VB_BEGIN(map, K_KEY)
    if (live(I)) {
        const Geom& G = *I.geom;
        const unsigned mask = (1u << G.sort_bits) - 1u;
        hist[2 * threadIdx.x] = 0;
        hist[2 * threadIdx.x + 1] = 0;
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
                atomicAdd(&hist[digit_of(key, 0, mask)], 1u);
            }
        }
        __syncthreads();
        put_tile_counts(hist, I.tcnt + (int64_t)lb * kDigitBins);
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

// Offsets within the groups of tiles for one pass, in place: a block takes
// one group and kScanDigits digits (a lane each); its four waves split the
// group's tiles, sum their counts, scan the sums across the waves and walk
// their tiles again writing each tile's count of the digit in the group's
// earlier tiles.  The last wave writes the group's total of the digit.
template <int PASS>
__global__ __launch_bounds__(256) void k_tscan(LaunchMap map)
{
    constexpr int KIND = K_TSCAN0 + PASS;
    constexpr int kU = 16;                             // counts loaded at once
    __shared__ unsigned part[4][kScanDigits];
    static_assert(kScanDigits == 64, "a lane per digit");
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        constexpr int nchunk = kDigitBins / kScanDigits;
        const int grp = lb / nchunk, d0 = (lb - grp * nchunk) * kScanDigits;
        if (d0 < (1 << I.geom->sort_bits)) {              // the same for the whole block
            const int d = d0 + lane;
            const int nt = I.ntiles_sort, gt = I.group_tiles;
            const int q = gt / 4;                          // tiles per wave
            const int ta = min(grp * gt + wv * q, nt), tb = min(ta + q, nt);
            unsigned* col = I.tcnt + (int64_t)PASS * nt * kDigitBins + d;
            unsigned c0[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) c0[u] = (ta + u < tb) ? col[(int64_t)(ta + u) * kDigitBins] : 0u;
            unsigned sum = 0;
#pragma unroll
            for (int u = 0; u < kU; ++u) sum += c0[u];
            for (int t = ta + kU; t < tb; t += kU) {
                unsigned c[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) c[u] = (t + u < tb) ? col[(int64_t)(t + u) * kDigitBins] : 0u;
#pragma unroll
                for (int u = 0; u < kU; ++u) sum += c[u];
            }
            part[wv][lane] = sum;
            __syncthreads();
            unsigned off = 0;
            for (int w = 0; w < wv; ++w) off += part[w][lane];
            if (wv == 3) I.gtot[((int64_t)PASS * I.ngroups_sort + grp) * kDigitBins + d] = off + sum;
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (ta + u < tb) {
                    col[(int64_t)(ta + u) * kDigitBins] = off;
                    off += c0[u];
                }
            for (int t = ta + kU; t < tb; t += kU) {
                unsigned c[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) c[u] = (t + u < tb) ? col[(int64_t)(t + u) * kDigitBins] : 0u;
#pragma unroll
                for (int u = 0; u < kU; ++u)
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
//
// Wave w of the block holds the tile's elements w * 512 ... w * 512 + 511 and
// ranks them, 64 at a time in element order, against counts of its own in
// LDS, so the ranking needs no barrier; the waves' counts are then combined
// once per digit (earlier waves first), which keeps the ranks stable.
// FP32 in one or two dimensions: at most 168 registers, three waves per SIMD.
template <typename T, int S> constexpr int kSortWaves = (sizeof(T) == 4 && S <= 2) ? 3 : 1;

template <typename T, int S, int PASS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kSortWaves<T, S>))) void k_sort(LaunchMap map)
{
    constexpr int PER = kSortTile / 256;          // rounds of 64 elements per wave
    constexpr int WCH = kSortTile / 4;            // elements per wave
    constexpr int KIND = K_SORT0 + PASS;
    __shared__ unsigned whist[4][kDigitBins];     // per wave: count of each digit so far, then
                                                  // the wave's first slot within the digit's run
    __shared__ unsigned dstart[kDigitBins];       // first LDS slot of each digit in the tile
    __shared__ unsigned dbase[kDigitBins];        // first output position of each digit
    __shared__ uint2 stage[kSortTile];
    __shared__ unsigned wsum[4];
    VB_BEGIN_IF(map, KIND, (live(I) && PASS < I.npass))
    {
        const Geom& G = *I.geom;
        const int sb = G.sort_bits, shift = PASS * sb;
        const unsigned mask = (1u << sb) - 1u;
        const int nbins = 1 << sb;
        const bool last = (PASS == I.npass - 1);
        const int64_t n = I.n;
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        const int tile = lb;
        for (int k = t; k < 4 * kDigitBins; k += 256) (&whist[0][0])[k] = 0;
        // the digit's count in earlier groups and over all groups (k_tscan)
        const int grp = tile / I.group_tiles, ng = I.ngroups_sort;
        // tables and pairs through the global view: vector-memory accesses,
        // which the LDS waits of the ranking and staging do not wait for
        const TSNE_GLOBAL unsigned* gt = gview<unsigned>(I.gtot) + (int64_t)PASS * ng * kDigitBins;
        unsigned before[2] = {0u, 0u}, total[2] = {0u, 0u};
#pragma unroll
        for (int g = 0; g < kScanGroups; ++g) {
            U2 v = {0u, 0u};
            if (g < ng && 2 * t < nbins) v = reinterpret_cast<const TSNE_GLOBAL U2*>(gt + (int64_t)g * kDigitBins)[t];
            if (g < grp) {
                before[0] += v.x;
                before[1] += v.y;
            }
            total[0] += v.x;
            total[1] += v.y;
        }
        // the digit's count in earlier tiles of the group (k_tscan)
        const U2 ofs = reinterpret_cast<const TSNE_GLOBAL U2*>(
            gview<unsigned>(I.tcnt) + ((int64_t)PASS * I.ntiles_sort + tile) * kDigitBins)[t];
        dbase[2 * t] = total[0];
        dbase[2 * t + 1] = total[1];
        const int64_t base = (int64_t)tile * kSortTile;
        const int64_t wbase = base + (int64_t)wv * WCH;
        const TSNE_GLOBAL U2* kv_in = gview<U2>(I.kv) + (int64_t)((PASS + 1) & 1) * n;
        TSNE_GLOBAL U2* kv_out = (TSNE_GLOBAL U2*)I.kv + (int64_t)(PASS & 1) * n;
        unsigned key[PER];
        int idx[PER];
        unsigned lrank[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int64_t e = wbase + r * 64 + lane;
            key[r] = 0;
            idx[r] = -1;
            lrank[r] = 0;
            if (e < n) {
                if (PASS == 0) {
                    key[r] = (unsigned)gview<int>(I.key)[e];
                    idx[r] = (int)e;
                } else {
                    const U2 q = kv_in[e];
                    key[r] = q.x;
                    idx[r] = (int)q.y;
                }
            }
        }
        __syncthreads();
        // stable ranks within the wave's elements, round by round in element
        // order: each round reads the wave's counts, then the first lane of
        // each digit adds the round's count (one wave: program order suffices)
        unsigned* wh = whist[wv];
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const bool valid = idx[r] >= 0;
            const unsigned d = digit_of(key[r], shift, mask);
            const unsigned long long peers = match_digit(d, valid, sb);
            const unsigned wrank = (unsigned)__popcll(peers & lt);
            const unsigned cur = valid ? wh[d] : 0u;
            lrank[r] = cur + wrank;
            if (valid && wrank == 0) wh[d] = cur + (unsigned)__popcll(peers);
        }
        __syncthreads();
        // per digit: the tile's count and each wave's first slot in the run
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int dd = 2 * t + h;
            unsigned acc = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const unsigned c = whist[w][dd];
                whist[w][dd] = acc;
                acc += c;
            }
            dstart[dd] = acc;
        }
        // first LDS slot of each digit: exclusive scan of the tile's counts;
        // first output position: the scan of the totals plus the counts in
        // earlier groups and earlier tiles of the group
        block_excl_scan_bins(dbase, wsum);
        dbase[2 * t] += before[0] + ofs.x;
        dbase[2 * t + 1] += before[1] + ofs.y;
        block_excl_scan_bins(dstart, wsum);
        // stage the tile in digit order, then write it out run by run
#pragma unroll
        for (int r = 0; r < PER; ++r)
            if (idx[r] >= 0) {
                const unsigned d = digit_of(key[r], shift, mask);
                stage[dstart[d] + wh[d] + lrank[r]] = make_uint2(key[r], (unsigned)idx[r]);
            }
        __syncthreads();
        const int tcount = (int)min<int64_t>(kSortTile, n - base);
        const T* Y = static_cast<const T*>(I.Yin);
        uint2 q[PER];
        int64_t dst[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int j = r * 256 + t;
            dst[r] = -1;
            if (j < tcount) {
                q[r] = stage[j];
                const unsigned d = digit_of(q[r].x, shift, mask);
                dst[r] = (int64_t)dbase[d] + (j - (int)dstart[d]);
            }
        }
        if (!last) {
#pragma unroll
            for (int r = 0; r < PER; ++r)
                if (dst[r] >= 0) {
                    U2 w;
                    w.x = q[r].x;
                    w.y = q[r].y;
                    kv_out[dst[r]] = w;
                }
        } else {
            // every gather of the tile in flight before the first store
            Pt<T, S> y[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r)
                if (dst[r] >= 0) y[r] = Pt<T, S>::load(Y, (int64_t)q[r].y);
#pragma unroll
            for (int r = 0; r < PER; ++r)
                if (dst[r] >= 0) {
                    ((TSNE_GLOBAL int*)I.perm)[dst[r]] = (int)q[r].y;
                    ((TSNE_GLOBAL unsigned*)I.skey)[dst[r]] = q[r].x;
                    y[r].store(static_cast<T*>(I.sY), dst[r]);
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
static_assert(kScanCells == 256, "a thread per cell of a tile");

__global__ __launch_bounds__(256) void k_scan_a(LaunchMap map)
{
    __shared__ int sh[4];
    VB_BEGIN(map, K_SCAN_A)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int e = lb * kScanCells + threadIdx.x;
        int it = (e < ncell) ? items_of(I.cell_start[e + 1] - I.cell_start[e], I.kpts) : 0;
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
    __shared__ int big[kScanCells][3];   // (cell, first item, items)
    VB_BEGIN(map, K_SCAN_B)
    if (live(I)) {
        const int ncell = I.geom->n_cells;
        const int ntile = (ncell + kScanCells - 1) / kScanCells;
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
            // one cell per thread
            const int e = lb * kScanCells + threadIdx.x;
            const int iv = (e < ncell) ? items_of(I.cell_start[e + 1] - I.cell_start[e], I.kpts) : 0;
            const int ii = wave_incl_scan(iv);
            __syncthreads();
            if (lane == 63) sh[wv] = ii;
            __syncthreads();
            int pi = off;
            for (int w = 0; w < wv; ++w) pi += sh[w];
            pi += ii - iv;
            if (e < ncell) {
                I.item_start[e] = pi;
                if (iv <= kSerialItems) {
                    for (int q = 0; q < iv; ++q) I.item_cell[pi + q] = e;
                } else {
                    const int b = atomicAdd(&nbig, 1);   // at most one per cell of the tile
                    big[b][0] = e;
                    big[b][1] = pi;
                    big[b][2] = iv;
                }
                if (e == ncell - 1) I.item_start[ncell] = pi + iv;
            }
            // cells with many items (a small box holding many points): the
            // block's four waves take them in turn, each wave's lanes writing
            // one cell's item -> cell entries
            __syncthreads();
            for (int b = wv; b < nbig; b += 4) {
                const int c = big[b][0], p0 = big[b][1], m = big[b][2];
                for (int q = lane; q < m; q += 64) I.item_cell[p0 + q] = c;
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
                             : c.s == 2 ? launch_sort_ts<float, 2>(kind, map, l, st)
                                        : launch_sort_ts<float, 3>(kind, map, l, st);
    return c.s == 1 ? launch_sort_ts<double, 1>(kind, map, l, st)
         : c.s == 2 ? launch_sort_ts<double, 2>(kind, map, l, st)
                    : launch_sort_ts<double, 3>(kind, map, l, st);
}

}  // namespace tsne
