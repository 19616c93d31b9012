// Host runtime of the t-SNE gradient library: plan layout over a caller
// workspace, launch tables, the C ABI of include/tsne.h, HIP-graph capture of
// an iteration, and the batch of independent embeddings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/tsne.h"
#include "launch.h"

using namespace tsne;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxM = 12288;       // row transforms: 1024 threads x 4 butterflies x radix 3
constexpr int kMaxM3 = 400;        // s = 3 passes: 32 threads x 4 butterflies per stage, so
                                   // M / R <= 128 at every radix R of a ladder length <= 400
constexpr int kMaxBfly = 4;          // must match the kernels' per-thread butterfly bound
constexpr int kGridCap = 4096;       // virtual blocks are looped over beyond this

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Smallest M >= lo of the form 4^a 3^b 5^c, a >= 1: every stage is radix 4, 3
// or 5 (the device picks its per-iteration length from the same ladder).
int fft_len(int lo)
{
    for (int m = std::max((lo + 3) & ~3, 4); m <= kMaxM; m += 4) {
        int r = m;
        while (r % 4 == 0) r /= 4;
        for (int f : {3, 5})
            while (r % f == 0) r /= f;
        if (r == 1) return m;
    }
    return -1;
}

// Radix stages: 4s, then 3s, then 5s.
int radix_plan(int M, int* radix, int* rmin)
{
    int r = M, n4 = 0, n3 = 0, n5 = 0, k = 0;
    while (r % 4 == 0) { r /= 4; ++n4; }
    while (r % 3 == 0) { r /= 3; ++n3; }
    while (r % 5 == 0) { r /= 5; ++n5; }
    if (r != 1) return -1;
    for (int i = 0; i < n4; ++i) radix[k++] = 4;
    for (int i = 0; i < n3; ++i) radix[k++] = 3;
    for (int i = 0; i < n5; ++i) radix[k++] = 5;
    if (k > kMaxStages) return -1;
    int mn = 5;
    for (int i = 0; i < k; ++i) mn = std::min(mn, radix[i]);
    *rmin = mn;
    return k;
}

int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Layout {
    size_t off[48];
    size_t total;
};

enum Region {
    R_INST, R_PREFIX, R_GEOM, R_SCHED, R_SMALL, R_BOX, R_CSTART, R_ISTART, R_SCAN,
    R_ICELL, R_KEY, R_KV, R_SKEY, R_TCNT, R_GTOT, R_PERM, R_SY, R_CARRY, R_W, R_X, R_XC, R_V, R_SPEC,
    R_TW, R_TWY, R_COS, R_CV, R_SPECTMP, R_KTAB, R_CCOS, R_R, R_FA, R_FAP, R_SPLIT, R_TSE, R_TSJ,
    R_TSB, R_EPACK, R_EVAL, R_ZPART, R_KLPART, R_H1, R_N
};
static_assert(R_N <= 48, "workspace regions exceed the layout table");

struct Derived {
    int s, p, nc, np, tsz, max_int, n_cap, M, half, ncell_cap, items_cap, kpts, lpr;
    int npass, ntiles_sort, group_tiles, ngroups_sort;
    int nstages, radix[kMaxStages], rmin;
    int slabs, slab_w;
    int tiled, tile_bi, tile_bj, tile_ni, tile_nj;
    int64_t tile_steps;   // capacity of the sweep step list
    size_t tile_lds;
    int tile_w, ntiles, col_group;
    int nb_box, nb_gather, nb_scan, nwaves, nb_kl;
    int row_threads, col_threads;
    size_t row_lds, col_lds;
    int vb[K_NKINDS];
    Layout L;
};

tsne_status derive(const tsne_desc* d, Derived& o)
{
    if (!d) return TSNE_E_ARG;
    if (d->n < 2 || d->n > (int64_t)INT_MAX / 4) return TSNE_E_ARG;
    if (d->s < 1 || d->s > 3) return TSNE_E_ARG;
    // s = 3: forms A and B, the square box, the CSR attraction in one slab
    if (d->s == 3 && (d->form == TSNE_FORM_V || d->rect != 0 || d->attr_layout == 2 || d->attr_slabs > 1))
        return TSNE_E_UNSUPPORTED;
    if (d->dtype != TSNE_F32 && d->dtype != TSNE_F64) return TSNE_E_ARG;
    if (d->p < 2 || d->p > kMaxP) return TSNE_E_UNSUPPORTED;
    if (d->policy != TSNE_GRID_PAPER && d->policy != TSNE_GRID_FIXED) return TSNE_E_ARG;
    if (d->form != TSNE_FORM_A && d->form != TSNE_FORM_B && d->form != TSNE_FORM_V) return TSNE_E_ARG;
    if (d->min_intervals < 1 || d->max_intervals < d->min_intervals) return TSNE_E_ARG;
    if (d->policy == TSNE_GRID_FIXED && !(d->interval_width > 0.0)) return TSNE_E_ARG;
    if (d->nnz < 0 || d->nnz > (int64_t)INT_MAX * 8) return TSNE_E_ARG;
    if (d->lanes_per_row != 0 && d->lanes_per_row != 4 && d->lanes_per_row != 8 && d->lanes_per_row != 16 &&
        d->lanes_per_row != 32 && d->lanes_per_row != 64)
        return TSNE_E_ARG;
    if (d->points_per_lane != 0 && (d->points_per_lane < 1 || d->points_per_lane > 64))
        return TSNE_E_ARG;
    if (d->attr_slabs < 0 || d->attr_slabs > 64) return TSNE_E_ARG;
    if (d->attr_layout < 0 || d->attr_layout > 2) return TSNE_E_ARG;
    if (d->rect != 0 && d->rect != 1) return TSNE_E_ARG;
    if (d->keep_h1 != 0 && d->keep_h1 != 1) return TSNE_E_ARG;

    o.s = d->s;
    o.p = d->p;
    o.nc = (d->form == TSNE_FORM_A) ? d->s + 1 : (d->form == TSNE_FORM_B) ? d->s + 2 : 1;
    o.np = (d->form == TSNE_FORM_V) ? d->s + 1 : d->s + 2;
    o.tsz = (d->dtype == TSNE_F32) ? 4 : 8;
    o.max_int = d->max_intervals;
    const int64_t ncap64 = (int64_t)d->max_intervals * d->p;
    if (ncap64 * 2 > kMaxM) return TSNE_E_UNSUPPORTED;
    o.n_cap = (int)ncap64;
    if (d->s == 2 && (int64_t)o.max_int * o.max_int > (int64_t)INT_MAX / 8) return TSNE_E_UNSUPPORTED;
    o.M = fft_len(2 * o.n_cap);
    if (o.M < 0) return TSNE_E_UNSUPPORTED;
    o.half = o.M / 2 + 1;
    o.nstages = radix_plan(o.M, o.radix, &o.rmin);
    if (o.nstages < 0) return TSNE_E_UNSUPPORTED;
    // the device picks a smaller ladder length when the box is smaller; every
    // ladder length has radix 3, 4 or 5 stages only
    o.rmin = 3;
    // s = 3: the three-axis passes run 32 threads per transform (kMaxBfly
    // butterflies each at radix 3), and hold M^3 complex grids
    if (d->s == 3 && o.M > kMaxM3) return TSNE_E_UNSUPPORTED;
    o.ncell_cap = (d->s == 3) ? o.max_int * o.max_int * o.max_int
                : (d->s == 2) ? o.max_int * o.max_int : o.max_int;
    // radix passes of the binning: enough digits of at most kDigitBitsMax bits
    // for the largest cell index of the capacity
    {
        int bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < (int64_t)o.ncell_cap) ++bits;
        o.npass = (bits + kDigitBitsMax - 1) / kDigitBitsMax;
        if (o.npass > kMaxSortPass) return TSNE_E_UNSUPPORTED;
    }
    o.kpts = d->points_per_lane ? d->points_per_lane : 8;
    // column slabs: when the positions exceed ~4 MB, 4 slabs of P split over
    // XCD pairs keep each XCD's gathers inside its own 4 MB L2 (measured at
    // N = 1e6: 573 us against 906 us with one slab); short rows per slab then
    // want fewer lanes per row
    {
        const int64_t ybytes = d->n * d->s * ((d->dtype == TSNE_F32) ? 4 : 8);
        const bool big = ybytes >= ((int64_t)4 << 20);
        int sl = d->attr_slabs ? d->attr_slabs : (big ? 4 : 1);
        if (sl != 1 && sl != 2 && sl != 4 && sl != 8) return TSNE_E_ARG;   // slabs map onto XCDs
        if (d->s == 3) sl = 1;
        o.lpr = d->lanes_per_row ? d->lanes_per_row : (sl > 1 ? 4 : 32);
        if (d->nnz >= ((int64_t)1 << 31) || d->nnz == 0) sl = 1;   // split offsets are int32
        if (sl > d->n) sl = (int)d->n;
        o.slabs = sl;
        o.slab_w = (int)((d->n + sl - 1) / sl);
    }
    // attraction layout: CSR rows or row blocks.  Row blocks: each workgroup
    // takes a block of tile_bi rows (their positions and 64-bit fixed-point
    // force sums in LDS) and sweeps column windows of 32 KB (tile_bj points),
    // double-buffered in LDS; the LDS then holds tile_bi s (8 + element) +
    // 64 KB bytes (157 KB for FP32 in 2-D at 3968 rows).
    // Sweep steps are the non-empty (row block, window) tiles, a tile with
    // more than tile_step_edges(tile_bj) edges taking several steps.
    // automatic layout (no CSR knob given): row blocks from 300,000 points in
    // one or two dimensions, where they beat the best CSR rows by 15 % or more
    // (random 90-neighbour P, FP32 and FP64).  At 1e5 the two are level on
    // random P and CSR rows win on a kNN P, whose columns cluster by row.
    const bool auto_rows = d->attr_layout == 0 && d->lanes_per_row == 0 && d->attr_slabs == 0 &&
                           d->s <= 2 && d->n >= 300000;
    o.tiled = (d->nnz > 0) && (d->attr_layout == 2 || auto_rows);
    {
        const int tsz_ = (d->dtype == TSNE_F32) ? 4 : 8;
        // rows per block: enough blocks for every CU (about n / 256, a
        // multiple of 64), at most what the LDS holds beside the windows
        const int64_t cap_bi = (d->dtype == TSNE_F32) ? 3968 : 1984;
        o.tile_bi = (int)std::min<int64_t>(cap_bi, std::max<int64_t>(64, 64 * cdiv(cdiv(d->n, 256), 64)));
        o.tile_bj = kTileWindowBytes / (d->s * tsz_);
        o.tile_ni = (int)((d->n + o.tile_bi - 1) / o.tile_bi);
        o.tile_nj = (int)((d->n + o.tile_bj - 1) / o.tile_bj);
        o.tile_lds = (size_t)o.tile_bi * d->s * (8 + tsz_) + 2 * (size_t)kTileWindowBytes;
        const int se = tile_step_edges(o.tile_bj);
        o.tile_steps = (int64_t)o.tile_ni * o.tile_nj + (d->nnz + se - 1) / se;
    }
    if (o.tiled && o.tile_steps > ((int64_t)1 << 30)) return TSNE_E_UNSUPPORTED;   // int step indices
    if (o.tiled) o.slabs = 1;
    const int64_t n = d->n;
    o.items_cap = cdiv(n, o.kpts) + (int)std::min<int64_t>(n, o.ncell_cap);
    o.nwaves = cdiv(o.items_cap, 64);

    const int csz = 2 * o.tsz;                         // complex element
    o.tile_w = 128 / csz;                              // 16 (float) or 8 (double)
    o.ntiles = cdiv(o.half, o.tile_w);
    // FFT thread counts: every stage must fit kMaxBfly butterflies per thread
    const int need_row = cdiv(o.M, (int64_t)o.rmin * kMaxBfly);
    o.row_threads = std::max(256, pow2_at_least(need_row));
    if (o.row_threads > 1024) return TSNE_E_UNSUPPORTED;
    o.row_lds = (size_t)lds_stride(o.M) * csz;
    // column kernel: LDS for one column at capacity, so several workgroups
    // share a CU and hide each other's barriers and loads; each iteration
    // packs G = (largest power of two) columns of its own M into that space
    const size_t pm = (size_t)lds_stride(o.M) * csz;   // one padded transform
    o.col_lds = pm;
    o.col_group = 1;                                   // columns per block at capacity
    while (o.col_group < o.tile_w && (size_t)(2 * o.col_group) * pm <= o.col_lds) o.col_group *= 2;
    o.col_threads = std::max(256, pow2_at_least(cdiv((int64_t)(o.col_lds / csz), (int64_t)o.rmin * kMaxBfly)));
    // the transforms also hold their stage plan in static LDS (under 256 bytes)
    constexpr size_t kLdsMax = 160 * 1024 - 256;
    if (o.row_lds > kLdsMax) return TSNE_E_UNSUPPORTED;
    if (d->s == 2 && (o.col_threads > 1024 || o.col_lds > kLdsMax)) return TSNE_E_UNSUPPORTED;

    o.nb_box = std::min(512, std::max(1, cdiv(n, 256 * 4)));
    o.nb_gather = (d->s == 3) ? cdiv(n, 256)             // s = 3: one thread per point
                              : cdiv(o.items_cap, 256);   // one thread per item
    o.nb_kl = (int)std::min<int64_t>(2048, cdiv(n, 8));
    o.nb_scan = cdiv(o.ncell_cap, kScanCells);
    o.ntiles_sort = cdiv(n, kSortTile);
    // groups of the offset scan: at most kScanGroups, of a multiple of 4 tiles
    o.group_tiles = 4 * cdiv(cdiv(o.ntiles_sort, kScanGroups), 4);
    o.ngroups_sort = cdiv(o.ntiles_sort, o.group_tiles);

    int* vb = o.vb;
    for (int k = 0; k < K_NKINDS; ++k) vb[k] = 0;
    vb[K_BOX] = o.nb_box;
    vb[K_KEY] = cdiv(n, kKeyTile);
    vb[K_SORT0] = o.ntiles_sort;
    vb[K_SORT1] = (o.npass > 1) ? o.ntiles_sort : 0;
    vb[K_SORT2] = (o.npass > 2) ? o.ntiles_sort : 0;
    vb[K_HIST1] = vb[K_SORT1];
    vb[K_HIST2] = vb[K_SORT2];
    vb[K_TSCAN0] = o.ngroups_sort * (kDigitBins / kScanDigits);
    vb[K_TSCAN1] = (o.npass > 1) ? vb[K_TSCAN0] : 0;
    vb[K_TSCAN2] = (o.npass > 2) ? vb[K_TSCAN0] : 0;
    vb[K_BOUNDS] = cdiv(n + 1, 256);
    vb[K_SCAN_A] = o.nb_scan;
    vb[K_SCAN_B] = o.nb_scan;
    vb[K_SPREAD] = cdiv(o.items_cap, 256);
    vb[K_FIX] = cdiv(o.ncell_cap, 256);
    vb[K_GATHER] = o.nb_gather;
    if (d->s == 3) {
        // node-per-thread spreading, point-per-thread gathering, no items
        vb[K_SCAN_A] = vb[K_SCAN_B] = vb[K_SPREAD] = vb[K_FIX] = vb[K_GATHER] = 0;
        vb[K_SPREAD3] = (int)cdiv((int64_t)o.ncell_cap * o.p * o.p * o.p, 256);
        vb[K_GATHER3] = o.nb_gather;
        const int bpg = (int)((int64_t)o.M * o.M / 16);   // blocks of 16 sequences per grid
        vb[K_F3_X] = vb[K_F3_Y] = o.nc * bpg;
        vb[K_F3_Z] = vb[K_F3_IY] = vb[K_F3_IX] = o.np * bpg;
        vb[K_S3_X] = vb[K_S3_Y] = vb[K_S3_Z] = 2 * bpg;
        vb[K_S3_FILL] = vb[K_S3_STORE] = (int)cdiv(2 * (int64_t)o.M * o.M * o.M, 256);
    } else if (d->s == 2) {
        vb[K_FFT_ROWS] = o.nc * cdiv(o.n_cap, 2);
        // whole tiles of tile_w / col_group groups each, per potential
        vb[K_FFT_COLS] = o.np * o.ntiles * (o.tile_w / o.col_group);
        vb[K_FFT_IROWS] = cdiv(o.np, 2) * o.n_cap;
        // kernel tables: K1 and K2, or K1 and the two odd kernels (form V)
        const int ntab = (d->form == TSNE_FORM_V) ? 3 : 2;
        vb[K_SPEC1] = ntab * cdiv(o.half, 64) * cdiv(o.half, 64);   // 64 x 64 GEMM tiles
        vb[K_SPEC2] = vb[K_SPEC1];
        vb[K_SPEC0] = cdiv(std::max<int64_t>(o.M, (int64_t)ntab * o.half * o.half), 256);
    } else {
        vb[K_FFT_1D] = o.np;
        vb[K_SPEC1] = cdiv(2 * o.half, 256);
        vb[K_SPEC0] = cdiv(std::max(o.M, 2 * o.half), 256);
    }
    vb[K_NORM] = cdiv(n * d->s, 256);
    {
        const int nrb = cdiv(n, 256 / o.lpr);
        // with slabs: 8 * ceil(nrb / (8 / slabs)) virtual blocks, a multiple of 8
        vb[K_ATTR] = (d->nnz == 0 || o.tiled) ? 0 : (o.slabs == 1 ? nrb : 8 * cdiv(nrb, 8 / o.slabs));
        vb[K_ATTR_T] = o.tiled ? o.tile_ni : 0;
        vb[K_ATTR_T_ALL] = vb[K_ATTR_T];
    }
    vb[K_ATTR_ALL] = vb[K_ATTR];
    vb[K_ASUM] = (d->nnz > 0 && o.slabs > 1) ? cdiv(n * d->s, 256) : 0;
    vb[K_UPDATE] = cdiv(n, 256 * kUpdPts);
    vb[K_GEOM] = 1;
    vb[K_ZSUM] = 1;
    // the divergence runs as a mode of the CSR attraction pass (same virtual
    // blocks, one partial each), or over rows for the tiled layout
    vb[K_KL_ATTR] = vb[K_ATTR];
    vb[K_KL_T] = vb[K_ATTR_T];
    // one partial per block of the attraction kernel's divergence mode
    if (vb[K_KL_ATTR] > 0) o.nb_kl = std::min(vb[K_KL_ATTR], kGridCap);
    if (vb[K_KL_T] > 0) o.nb_kl = std::min(vb[K_KL_T], kGridCap);
    vb[K_KLSUM] = (d->nnz > 0) ? 1 : 0;

    // workspace layout
    const int64_t grid = (d->s == 3) ? (int64_t)o.n_cap * o.n_cap * o.n_cap
                       : (d->s == 2) ? (int64_t)o.n_cap * o.n_cap : o.n_cap;
    const int64_t nn = (d->s == 2) ? o.p * o.p : o.p;
    const int64_t M3 = (int64_t)o.M * o.M * o.M;
    size_t sz[R_N];
    sz[R_INST] = sizeof(Inst);
    sz[R_PREFIX] = sizeof(int) * K_NKINDS * 2;
    sz[R_GEOM] = sizeof(Geom);
    sz[R_SCHED] = sizeof(Sched);
    sz[R_SMALL] = 64;                                   // status, iter
    sz[R_BOX] = sizeof(double) * kBoxPart * o.nb_box;
    sz[R_CSTART] = sizeof(int) * (o.ncell_cap + 1);
    sz[R_ISTART] = sizeof(int) * (o.ncell_cap + 1);
    sz[R_SCAN] = sizeof(int) * o.nb_scan;
    sz[R_ICELL] = sizeof(int) * o.items_cap;
    sz[R_KEY] = sizeof(int) * n;
    sz[R_KV] = (o.npass > 1) ? sizeof(uint32_t) * 2 * 2 * (size_t)n : 0;
    sz[R_SKEY] = sizeof(uint32_t) * n;
    sz[R_TCNT] = sizeof(uint32_t) * (size_t)o.npass * o.ntiles_sort * kDigitBins;
    sz[R_GTOT] = sizeof(uint32_t) * (size_t)o.npass * o.ngroups_sort * kDigitBins;
    sz[R_PERM] = sizeof(int) * n;
    sz[R_SY] = (size_t)o.tsz * n * d->s;
    sz[R_CARRY] = (d->s == 3) ? 0 : (size_t)o.tsz * 2 * o.nwaves * nn * o.nc;
    sz[R_W] = (size_t)o.tsz * o.nc * grid;
    if (d->s == 3) {
        // complex M^3 grids per charge and per potential, the two kernel
        // spectra (element type), their FP64 complex build grids
        sz[R_X] = (size_t)csz * o.nc * M3;
        sz[R_XC] = (size_t)csz * o.np * M3;
        sz[R_SPEC] = (size_t)o.tsz * 2 * M3;
        sz[R_SPECTMP] = (size_t)16 * 2 * M3;
        sz[R_KTAB] = 0;
        sz[R_CCOS] = 0;
    } else if (d->s == 2) {
        sz[R_X] = (size_t)csz * o.nc * o.ntiles * o.n_cap * o.tile_w;
        sz[R_XC] = (size_t)csz * o.np * o.ntiles * o.n_cap * o.tile_w;
        // one [half][half] slot per kernel table (form V: a third, the odd
        // kernel along dimension 1); cosine matrices of both axes, and for
        // form V their sine matrices
        const size_t vf = (d->form == TSNE_FORM_V) ? 1 : 0;
        const size_t slot = (size_t)o.half * o.half;
        sz[R_SPEC] = (size_t)o.tsz * (2 + vf) * slot;
        sz[R_SPECTMP] = sizeof(double) * (2 + vf) * slot;
        sz[R_KTAB] = sizeof(double) * (2 + vf) * slot;
        sz[R_CCOS] = sizeof(double) * (2 + 2 * vf) * slot;
    } else {
        sz[R_CCOS] = 0;
        sz[R_X] = 0;
        sz[R_XC] = 0;
        sz[R_SPEC] = (size_t)o.tsz * 2 * o.half;
        sz[R_SPECTMP] = 0;
        sz[R_KTAB] = sizeof(double) * 2 * (size_t)o.half;
    }
    sz[R_V] = (size_t)o.tsz * o.np * grid;
    sz[R_TW] = (size_t)csz * o.M;
    sz[R_TWY] = (d->s == 2) ? (size_t)csz * o.M : (d->s == 3) ? (size_t)16 * o.M : 0;   // s = 3: FP64
    sz[R_COS] = sizeof(double) * 2 * o.M;               // cos, then sin
    sz[R_R] = (size_t)o.tsz * n * d->s;
    sz[R_FA] = (size_t)o.tsz * n * d->s;
    sz[R_FAP] = (o.slabs > 1) ? (size_t)o.tsz * n * d->s * o.slabs : 0;
    sz[R_SPLIT] = (o.slabs > 1) ? sizeof(int) * (size_t)(o.slabs - 1) * n : 0;
    sz[R_TSE] = o.tiled ? sizeof(int64_t) * ((size_t)o.tile_steps + 1) : 0;
    sz[R_TSJ] = o.tiled ? sizeof(int) * (size_t)o.tile_steps : 0;
    sz[R_TSB] = o.tiled ? sizeof(int) * ((size_t)o.tile_ni + 1) : 0;
    // FP32 CSR rows: column and value of each non-zero packed into 8 bytes, so
    // the attraction streams one vector load per non-zero instead of two
    // (one spare pair: the kernel reads pairs two at a time, 16-byte aligned)
    sz[R_CV] = (d->dtype == TSNE_F32 && !o.tiled && d->nnz > 0) ? (size_t)8 * (d->nnz + 1) : 0;
    sz[R_EPACK] = o.tiled ? sizeof(uint32_t) * (size_t)d->nnz : 0;
    sz[R_EVAL] = o.tiled ? (size_t)o.tsz * d->nnz : 0;
    sz[R_ZPART] = sizeof(double) * o.nb_gather;
    sz[R_KLPART] = (d->nnz > 0) ? sizeof(double) * 2 * o.nb_kl : 0;
    sz[R_H1] = d->keep_h1 ? sizeof(double) * n : 0;
    size_t cur = 0;
    for (int r = 0; r < R_N; ++r) {
        o.L.off[r] = cur;
        cur = align_up(cur + sz[r]);
    }
    o.L.total = cur;
    return TSNE_OK;
}

bool hip_ok(hipError_t e) { return e == hipSuccess; }

Cfg cfg_of(const tsne_desc& d, const Derived& o)
{
    return Cfg{d.dtype, d.s, d.p, d.form, o.lpr};
}

Launch launch_of(int kind, const Derived& o, int vblocks)
{
    Launch l{std::min(vblocks, kGridCap), 256, 0};
    switch (kind) {
    case K_SPEC0: case K_SPEC1: case K_SPEC2:
        // usually idle (tables unchanged): one block per CU, each block loops
        // when there is work and checks once when there is none
        l.grid = std::min(vblocks, 256);
        break;
    case K_FFT_ROWS: case K_FFT_IROWS: case K_FFT_1D:
        l.block = o.row_threads;
        l.lds = o.row_lds;
        break;
    case K_FFT_COLS:
        l.block = o.col_threads;
        l.lds = o.col_lds;
        break;
    case K_ATTR_T: case K_ATTR_T_ALL: case K_KL_T:
        l.block = 1024;
        l.lds = o.tile_lds;
        break;
    case K_F3_X: case K_F3_Y: case K_F3_Z: case K_F3_IY: case K_F3_IX:
        l.block = 16 * 32;                                 // 16 sequences, 32 threads each
        l.lds = (size_t)16 * lds_stride(o.M) * 2 * o.tsz;
        break;
    case K_S3_X: case K_S3_Y: case K_S3_Z:
        l.block = 16 * 32;
        l.lds = (size_t)16 * lds_stride(o.M) * 16;         // FP64 complex
        break;
    default:
        break;
    }
    return l;
}

}  // namespace

// ---------------------------------------------------------------- plan

struct tsne_plan {
    tsne_desc d;
    Derived o;
    hipStream_t st;
    char* ws;
    Inst h;                 // host copy of the device record
    Inst* dinst;
    int* dprefix;
    Cfg cfg;
    bool P_bound;
    bool graph_ok;
    hipGraphExec_t gexec;
    hipGraph_t graph;
    bool args_valid;        // last_args mirrors the device record's pointers
    CallArgs last_args;
    double tscale;          // fixed-point scale of the tiled attraction (set with P)
};

// Enqueue the per-call pointer update unless the device record already holds
// exactly these pointers.
static tsne_status set_ptrs(tsne_plan* pl, const CallArgs& a)
{
    if (pl->args_valid && a.Yin == pl->last_args.Yin && a.Y == pl->last_args.Y &&
        a.uY == pl->last_args.uY && a.gains == pl->last_args.gains &&
        a.Frep == pl->last_args.Frep && a.Zout == pl->last_args.Zout &&
        a.Fattr == pl->last_args.Fattr && a.KLout == pl->last_args.KLout &&
        a.counting == pl->last_args.counting)
        return TSNE_OK;
    if (!hip_ok(launch_set_args(pl->dinst, a, pl->st))) return TSNE_E_HIP;
    pl->last_args = a;
    pl->args_valid = true;
    return TSNE_OK;
}

static tsne_status enqueue(tsne_plan* pl, int kind)
{
    const int vb = pl->o.vb[kind];
    if (vb <= 0) return TSNE_OK;
    LaunchMap map{pl->dinst, pl->dprefix, 1};
    const Launch l = launch_of(kind, pl->o, vb);
    return hip_ok(launch_kind(kind, pl->cfg, map, l, pl->st)) ? TSNE_OK : TSNE_E_HIP;
}

// Kernel order of one repulsion.  The table kernels (K_SPEC*) always run;
// they return at once unless the box kernel found a new spacing or length.
static const int kChain2[] = {K_BOX, K_GEOM, K_SPEC0, K_SPEC1, K_SPEC2, K_KEY, K_TSCAN0, K_SORT0,
                              K_HIST1, K_TSCAN1, K_SORT1, K_HIST2, K_TSCAN2, K_SORT2, K_BOUNDS,
                              K_SCAN_A, K_SCAN_B, K_SPREAD, K_FIX, K_FFT_ROWS, K_FFT_COLS,
                              K_FFT_IROWS, K_GATHER, K_ZSUM};
static const int kChain3[] = {K_BOX, K_GEOM, K_S3_FILL, K_S3_X, K_S3_Y, K_S3_Z, K_S3_STORE, K_KEY,
                              K_TSCAN0, K_SORT0, K_HIST1, K_TSCAN1, K_SORT1, K_HIST2, K_TSCAN2,
                              K_SORT2, K_BOUNDS, K_SPREAD3, K_F3_X, K_F3_Y, K_F3_Z, K_F3_IY,
                              K_F3_IX, K_GATHER3, K_ZSUM};
static const int kChain1[] = {K_BOX, K_GEOM, K_SPEC0, K_SPEC1, K_KEY, K_TSCAN0, K_SORT0, K_HIST1,
                              K_TSCAN1, K_SORT1, K_HIST2, K_TSCAN2, K_SORT2, K_BOUNDS, K_SCAN_A,
                              K_SCAN_B, K_SPREAD, K_FIX, K_FFT_1D, K_GATHER, K_ZSUM};

// The repulsion chain of an embedding dimension and its length.
static const int* chain_of(int s, int& nk)
{
    if (s == 3) { nk = (int)(sizeof(kChain3) / sizeof(int)); return kChain3; }
    if (s == 2) { nk = (int)(sizeof(kChain2) / sizeof(int)); return kChain2; }
    nk = (int)(sizeof(kChain1) / sizeof(int));
    return kChain1;
}

static tsne_status enqueue_repulsion(tsne_plan* pl, bool normalise)
{
    int nk;
    const int* ch = chain_of(pl->d.s, nk);
    for (int k = 0; k < nk; ++k) {
        tsne_status s = enqueue(pl, ch[k]);
        if (s != TSNE_OK) return s;
    }
    if (normalise) return enqueue(pl, K_NORM);
    return TSNE_OK;
}

static CallArgs no_args()
{
    CallArgs a;
    std::memset(&a, 0, sizeof(a));
    return a;
}

static void fill_sched(Sched& s, const tsne_sched* c)
{
    s.eta = c->eta;
    s.mom0 = c->mom0;
    s.mom1 = c->mom1;
    s.mom_switch = c->mom_switch;
    s.ee_alpha = c->ee_alpha;
    s.ee_stop = c->ee_stop;
    s.le_alpha = c->le_alpha;
    s.le_start = c->le_start;
    s.gain_inc = c->gain_inc;
    s.gain_dec = c->gain_dec;
    s.gain_min = c->gain_min;
    s.recentre = c->recentre;
}

// Lay a plan over its workspace: the host image of the device record, the
// launch prefix table, and the device state that must start at zero (the
// geometry record, the schedule, status and counters).
// Allocates nothing; synchronises the stream before returning.
static tsne_status plan_init(tsne_plan* pl, const tsne_desc* desc, const Derived& o, char* b,
                             hipStream_t st)
{
    pl->d = *desc;
    pl->o = o;
    pl->st = st;
    pl->ws = b;
    pl->cfg = cfg_of(*desc, o);
    pl->P_bound = false;
    pl->graph_ok = false;
    pl->args_valid = false;

    const size_t* off = o.L.off;
    Inst& h = pl->h;
    std::memset(&h, 0, sizeof(h));
    h.n = desc->n;
    h.nnz = desc->nnz;
    h.s = desc->s;
    h.p = desc->p;
    h.form = desc->form;
    h.rect = (desc->s == 2) ? desc->rect : 0;
    h.nc = o.nc;
    h.np = o.np;
    h.policy = desc->policy;
    h.min_int = desc->min_intervals;
    h.max_int = desc->max_intervals;
    h.n_cap = o.n_cap;
    h.M = o.M;
    h.half = o.half;
    h.ncell_cap = o.ncell_cap;
    h.items_cap = o.items_cap;
    h.kpts = o.kpts;
    h.lpr = o.lpr;
    h.col_group = o.col_group;
    h.col_lds = (int)o.col_lds;
    h.tile_w = o.tile_w;
    h.ntiles = o.ntiles;
    h.interval_width = desc->interval_width;
    h.iter_end = INT_MAX;
    h.geom = reinterpret_cast<Geom*>(b + off[R_GEOM]);
    h.sched = reinterpret_cast<Sched*>(b + off[R_SCHED]);
    h.status = reinterpret_cast<int*>(b + off[R_SMALL]);
    h.iter = reinterpret_cast<int*>(b + off[R_SMALL] + 4);
    h.box_part = reinterpret_cast<double*>(b + off[R_BOX]);
    h.cell_start = reinterpret_cast<int*>(b + off[R_CSTART]);
    h.item_start = reinterpret_cast<int*>(b + off[R_ISTART]);
    h.scan_part = reinterpret_cast<int*>(b + off[R_SCAN]);
    h.item_cell = reinterpret_cast<int*>(b + off[R_ICELL]);
    h.key = reinterpret_cast<int*>(b + off[R_KEY]);
    h.kv = b + off[R_KV];
    h.skey = reinterpret_cast<unsigned*>(b + off[R_SKEY]);
    h.tcnt = reinterpret_cast<unsigned*>(b + off[R_TCNT]);
    h.gtot = reinterpret_cast<unsigned*>(b + off[R_GTOT]);
    h.group_tiles = o.group_tiles;
    h.ngroups_sort = o.ngroups_sort;
    h.npass = o.npass;
    h.ntiles_sort = o.ntiles_sort;
    h.perm = reinterpret_cast<int*>(b + off[R_PERM]);
    h.h1keep = desc->keep_h1 ? reinterpret_cast<double*>(b + off[R_H1]) : nullptr;
    h.sY = b + off[R_SY];
    h.carry = b + off[R_CARRY];
    h.W = b + off[R_W];
    h.X = b + off[R_X];
    h.Xc = b + off[R_XC];
    h.V = b + off[R_V];
    h.spec = b + off[R_SPEC];
    h.tw = b + off[R_TW];
    h.twy = b + off[R_TWY];
    h.costab = reinterpret_cast<double*>(b + off[R_COS]);
    h.spec_tmp = reinterpret_cast<double*>(b + off[R_SPECTMP]);
    h.twd = (desc->s == 3) ? b + off[R_TWY] : nullptr;
    h.specd = (desc->s == 3) ? b + off[R_SPECTMP] : nullptr;
    h.ktab = reinterpret_cast<double*>(b + off[R_KTAB]);
    h.ccos = reinterpret_cast<double*>(b + off[R_CCOS]);
    h.R = b + off[R_R];
    h.Fa_ws = b + off[R_FA];
    h.z_part = reinterpret_cast<double*>(b + off[R_ZPART]);
    h.kl_part = reinterpret_cast<double*>(b + off[R_KLPART]);
    h.KLout = nullptr;
    h.nb_kl = o.nb_kl;
    h.Fap = b + off[R_FAP];
    h.split = reinterpret_cast<const int*>(b + off[R_SPLIT]);
    h.slabs = o.slabs;
    h.slab_w = o.slab_w;
    h.tiled = o.tiled;
    h.tile_bi = o.tile_bi;
    h.tile_bj = o.tile_bj;
    h.tile_ni = o.tile_ni;
    h.tile_nj = o.tile_nj;
    h.tse = reinterpret_cast<const int64_t*>(b + off[R_TSE]);
    h.tsj = reinterpret_cast<const int*>(b + off[R_TSJ]);
    h.tsb = reinterpret_cast<const int*>(b + off[R_TSB]);
    h.tscale = 0.0;
    h.cv = (off[R_CV + 1] > off[R_CV]) ? (const void*)(b + off[R_CV]) : nullptr;
    h.epack = reinterpret_cast<const uint32_t*>(b + off[R_EPACK]);
    h.eval = b + off[R_EVAL];
    h.nb_box = o.nb_box;
    h.nb_gather = o.nb_gather;
    h.nb_scan = o.nb_scan;
    h.nwaves = o.nwaves;
    pl->dinst = reinterpret_cast<Inst*>(b + off[R_INST]);
    pl->dprefix = reinterpret_cast<int*>(b + off[R_PREFIX]);

    // host image of the launch prefix table (one instance)
    int prefix[K_NKINDS * 2];
    for (int k = 0; k < K_NKINDS; ++k) {
        prefix[2 * k] = 0;
        prefix[2 * k + 1] = o.vb[k];
    }
    const bool ok = hip_ok(hipMemcpyAsync(pl->dinst, &h, sizeof(Inst), hipMemcpyHostToDevice, st)) &&
                    hip_ok(hipMemcpyAsync(pl->dprefix, prefix, sizeof(prefix), hipMemcpyHostToDevice, st)) &&
                    hip_ok(hipMemsetAsync(b + off[R_GEOM], 0, sizeof(Geom), st)) &&
                    hip_ok(hipMemsetAsync(b + off[R_SCHED], 0, sizeof(Sched), st)) &&
                    hip_ok(hipMemsetAsync(b + off[R_SMALL], 0, 64, st)) &&
                    hip_ok(hipStreamSynchronize(st));
    return ok ? TSNE_OK : TSNE_E_HIP;
}

extern "C" {

size_t tsne_workspace_bytes(const tsne_desc* desc)
{
    Derived o;
    if (derive(desc, o) != TSNE_OK) return 0;
    return o.L.total;
}

const char* tsne_status_str(tsne_status s)
{
    switch (s) {
    case TSNE_OK: return "ok";
    case TSNE_E_ARG: return "invalid argument";
    case TSNE_E_UNSUPPORTED: return "unsupported configuration";
    case TSNE_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case TSNE_E_CAPACITY: return "box needs more intervals than max_intervals";
    case TSNE_E_NONFINITE: return "non-finite coordinate in Y";
    case TSNE_E_HIP: return "HIP runtime error";
    case TSNE_E_STATE: return "call not valid in this plan state";
    case TSNE_E_INTERNAL: return "internal device error (the binning did not complete)";
    }
    return "unknown status";
}

tsne_status tsne_plan_create(const tsne_desc* desc, void* workspace, size_t bytes, void* stream,
                             tsne_plan** out)
{
    if (!out) return TSNE_E_ARG;
    *out = nullptr;
    Derived o;
    tsne_status rs = derive(desc, o);
    if (rs != TSNE_OK) return rs;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || bytes < o.L.total) return TSNE_E_WORKSPACE;

    tsne_plan* pl = new (std::nothrow) tsne_plan();
    if (!pl) return TSNE_E_HIP;
    rs = plan_init(pl, desc, o, static_cast<char*>(workspace), static_cast<hipStream_t>(stream));
    if (rs != TSNE_OK) {
        delete pl;
        return rs;
    }
    *out = pl;
    return TSNE_OK;
}

tsne_status tsne_plan_destroy(tsne_plan* plan)
{
    if (!plan) return TSNE_E_ARG;
    if (plan->graph_ok) {
        hipGraphExecDestroy(plan->gexec);
        hipGraphDestroy(plan->graph);
    }
    delete plan;
    return TSNE_OK;
}

tsne_status tsne_bind_P(tsne_plan* pl, const int64_t* row_ptr, const int32_t* col, const void* val)
{
    if (!pl) return TSNE_E_ARG;
    if (pl->d.nnz > 0 && (!row_ptr || !col || !val)) return TSNE_E_ARG;
    // host check of the CSR shape: row_ptr[0] = 0, row_ptr[n] = nnz, monotone,
    // columns in range (a device-side read would fault on a bad index)
    if (pl->d.nnz > 0) {
        const int64_t n = pl->d.n;
        std::vector<int64_t> rp(n + 1);
        std::vector<int32_t> cc(pl->d.nnz);
        if (!hip_ok(hipStreamSynchronize(pl->st)) ||
            !hip_ok(hipMemcpy(rp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost)) ||
            !hip_ok(hipMemcpy(cc.data(), col, sizeof(int32_t) * pl->d.nnz, hipMemcpyDeviceToHost)))
            return TSNE_E_HIP;
        if (rp[0] != 0 || rp[n] != pl->d.nnz) return TSNE_E_ARG;
        for (int64_t i = 0; i < n; ++i)
            if (rp[i + 1] < rp[i]) return TSNE_E_ARG;
        for (int64_t k = 0; k < pl->d.nnz; ++k)
            if (cc[k] < 0 || cc[k] >= n) return TSNE_E_ARG;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rp[i] + 1; k < rp[i + 1]; ++k)
                if (cc[k] <= cc[k - 1]) return TSNE_E_ARG;
        // per-row start of each later column slab
        const int S = pl->o.slabs;
        if (S > 1) {
            std::vector<int> split((size_t)(S - 1) * n);
            for (int64_t i = 0; i < n; ++i) {
                const int32_t* r0 = cc.data() + rp[i];
                const int32_t* r1 = cc.data() + rp[i + 1];
                for (int sl = 1; sl < S; ++sl) {
                    const int32_t bound = (int32_t)std::min<int64_t>((int64_t)sl * pl->o.slab_w, n);
                    split[(size_t)(sl - 1) * n + i] = (int)(std::lower_bound(r0, r1, bound) - cc.data());
                }
            }
            if (!hip_ok(hipMemcpy(const_cast<int*>(pl->h.split), split.data(),
                                  split.size() * sizeof(int), hipMemcpyHostToDevice)))
                return TSNE_E_HIP;
        }
        // tiles: edges bucketed by (row block, column window), rows increasing
        // within a tile; the sweep steps of each row block are its non-empty
        // tiles in window order, split into runs of at most tile_step_edges
        if (pl->o.tiled) {
            const Derived& o = pl->o;
            const int64_t nnz = pl->d.nnz;
            const size_t tsz = (size_t)o.tsz;
            std::vector<char> vv(nnz * tsz), vt(nnz * tsz);
            if (!hip_ok(hipMemcpy(vv.data(), val, nnz * tsz, hipMemcpyDeviceToHost))) return TSNE_E_HIP;
            std::vector<int64_t> tse;
            std::vector<int> tsj, tsb(o.tile_ni + 1, 0);
            tse.reserve((size_t)o.tile_steps + 1);
            tsj.reserve((size_t)o.tile_steps);
            std::vector<uint32_t> pack(nnz);
            std::vector<int64_t> cnt(o.tile_nj);
            int64_t cur = 0;
            double rmax = 0.0;   // largest sum of |p| over a row
            for (int I = 0; I < o.tile_ni; ++I) {
                const int64_t r0 = (int64_t)I * o.tile_bi, r1 = std::min<int64_t>(n, r0 + o.tile_bi);
                std::fill(cnt.begin(), cnt.end(), 0);
                for (int64_t i = r0; i < r1; ++i)
                    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) ++cnt[cc[k] / o.tile_bj];
                tsb[I] = (int)tsj.size();
                for (int J = 0; J < o.tile_nj; ++J) {
                    const int64_t c = cnt[J];
                    for (int64_t q = 0; q < c; q += tile_step_edges(o.tile_bj)) {
                        tsj.push_back(J);
                        tse.push_back(cur + q);
                    }
                    cnt[J] = cur;
                    cur += c;
                }
                for (int64_t i = r0; i < r1; ++i) {
                    double ra = 0.0;
                    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                        const int J = cc[k] / o.tile_bj;
                        const int64_t dst = cnt[J]++;
                        pack[dst] = ((uint32_t)(i - r0) << 16) | (uint32_t)(cc[k] - (int64_t)J * o.tile_bj);
                        std::memcpy(vt.data() + dst * tsz, vv.data() + k * tsz, tsz);
                        double v;
                        if (tsz == 4) {
                            float f;
                            std::memcpy(&f, vv.data() + k * tsz, 4);
                            v = f;
                        } else {
                            std::memcpy(&v, vv.data() + k * tsz, 8);
                        }
                        if (!std::isfinite(v)) return TSNE_E_ARG;
                        ra += std::fabs(v);
                    }
                    rmax = std::max(rmax, ra);
                }
            }
            tsb[o.tile_ni] = (int)tsj.size();
            tse.push_back(cur);
            if ((int64_t)tsj.size() > o.tile_steps) return TSNE_E_INTERNAL;
            // |p (y_i - y_j) / (1 + |y_i - y_j|^2)| <= |p| / 2, so a row's sum
            // stays below rmax / 2; a power-of-two scale puts that under 2^60
            // (each term's rounding adds at most 1/2)
            pl->tscale = std::ldexp(1.0, 61 - std::max(-900, std::ilogb(std::max(rmax, 1e-300)) + 1));
            pl->h.tscale = pl->tscale;
            if (!hip_ok(hipMemcpy(const_cast<int64_t*>(pl->h.tse), tse.data(),
                                  tse.size() * sizeof(int64_t), hipMemcpyHostToDevice)) ||
                !hip_ok(hipMemcpy(const_cast<int*>(pl->h.tsj), tsj.data(),
                                  tsj.size() * sizeof(int), hipMemcpyHostToDevice)) ||
                !hip_ok(hipMemcpy(const_cast<int*>(pl->h.tsb), tsb.data(),
                                  tsb.size() * sizeof(int), hipMemcpyHostToDevice)) ||
                !hip_ok(hipMemcpy(const_cast<uint32_t*>(pl->h.epack), pack.data(),
                                  pack.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) ||
                !hip_ok(hipMemcpy(const_cast<void*>(pl->h.eval), vt.data(), vt.size(),
                                  hipMemcpyHostToDevice)))
                return TSNE_E_HIP;
        }
        // FP32 CSR: (column, value) pairs in one array, packed on the device
        if (pl->h.cv &&
            !hip_ok(launch_pack_cv(col, static_cast<const float*>(val), const_cast<void*>(pl->h.cv),
                                   pl->d.nnz, pl->st)))
            return TSNE_E_HIP;
    }
    CallArgs a = no_args();
    a.set_P = 1;
    a.row_ptr = row_ptr;
    a.col = col;
    a.val = val;
    a.tscale = pl->tscale;
    if (!hip_ok(launch_set_args(pl->dinst, a, pl->st))) return TSNE_E_HIP;
    pl->P_bound = pl->d.nnz > 0;
    return TSNE_OK;
}

// Per-point arrays are accessed one point at a time as a vector (s = 1, 2
// elements), so each must be aligned to a whole point; for s = 3 to one
// element.
static bool point_aligned(const tsne_desc& d, const void* p)
{
    // s = 3 points are moved one coordinate at a time: element alignment
    const uintptr_t a = (uintptr_t)((d.s == 3) ? 1 : d.s) * ((d.dtype == TSNE_F32) ? 4 : 8);
    return p && ((uintptr_t)p % a) == 0;
}

tsne_status tsne_repulsive(tsne_plan* pl, const void* Y, void* F_rep, double* Z)
{
    if (!pl || !Y || !F_rep || !point_aligned(pl->d, Y)) return TSNE_E_ARG;
    CallArgs a = no_args();
    a.set_ptrs = 1;
    a.Yin = Y;
    a.Frep = F_rep;
    a.Zout = Z;
    a.Fattr = pl->h.Fa_ws;
    tsne_status s = set_ptrs(pl, a);
    if (s != TSNE_OK) return s;
    return enqueue_repulsion(pl, true);
}

tsne_status tsne_attractive(tsne_plan* pl, const void* Y, void* F_attr)
{
    if (!pl || !Y || !F_attr || !point_aligned(pl->d, Y)) return TSNE_E_ARG;
    if (!pl->P_bound) return TSNE_E_STATE;
    CallArgs a = no_args();
    a.set_ptrs = 1;
    a.Yin = Y;
    a.Fattr = F_attr;
    tsne_status s = set_ptrs(pl, a);
    if (s != TSNE_OK) return s;
    s = enqueue(pl, K_ATTR_ALL);
    if (s != TSNE_OK) return s;
    s = enqueue(pl, K_ATTR_T_ALL);
    if (s != TSNE_OK) return s;
    return enqueue(pl, K_ASUM);
}

tsne_status tsne_kl_divergence(tsne_plan* pl, const void* Y, double* kl)
{
    if (!pl || !Y || !kl || !point_aligned(pl->d, Y)) return TSNE_E_ARG;
    if (!pl->P_bound) return TSNE_E_STATE;
    CallArgs a = no_args();
    a.set_ptrs = 1;
    a.Yin = Y;
    a.Fattr = pl->h.Fa_ws;
    a.KLout = kl;
    tsne_status s = set_ptrs(pl, a);
    if (s != TSNE_OK) return s;
    s = enqueue_repulsion(pl, false);
    if (s != TSNE_OK) return s;
    s = enqueue(pl, pl->o.vb[K_KL_T] > 0 ? K_KL_T : K_KL_ATTR);
    if (s != TSNE_OK) return s;
    return enqueue(pl, K_KLSUM);
}

static tsne_status step_args(tsne_plan* pl, void* Y, void* uY, void* gains, const tsne_sched* sc,
                             int32_t iter)
{
    CallArgs a = no_args();
    a.set_ptrs = 1;
    a.Yin = Y;
    a.Y = Y;
    a.uY = uY;
    a.gains = gains;
    a.Fattr = pl->h.Fa_ws;
    a.set_sched = 1;
    fill_sched(a.sched, sc);
    a.set_iter = 1;
    a.iter = iter;
    a.counting = 1;
    if (!hip_ok(launch_set_args(pl->dinst, a, pl->st))) return TSNE_E_HIP;
    pl->last_args = a;
    pl->args_valid = true;
    return TSNE_OK;
}

static tsne_status enqueue_iteration(tsne_plan* pl)
{
    tsne_status s = enqueue_repulsion(pl, false);
    if (s != TSNE_OK) return s;
    if (pl->P_bound) {
        s = enqueue(pl, K_ATTR);
        if (s != TSNE_OK) return s;
        s = enqueue(pl, K_ATTR_T);
        if (s != TSNE_OK) return s;
    }
    return enqueue(pl, K_UPDATE);
}

static bool sched_ok(const tsne_sched* sc)
{
    return sc && std::isfinite(sc->eta) && std::isfinite(sc->mom0) && std::isfinite(sc->mom1) &&
           std::isfinite(sc->ee_alpha) && std::isfinite(sc->le_alpha) && sc->gain_min >= 0.0;
}

tsne_status tsne_step(tsne_plan* pl, void* Y, void* uY, void* gains, const tsne_sched* sc, int32_t iter)
{
    if (!pl || !Y || !uY || !gains || !sched_ok(sc) || iter < 0) return TSNE_E_ARG;
    if (!point_aligned(pl->d, Y) || !point_aligned(pl->d, uY) || !point_aligned(pl->d, gains)) return TSNE_E_ARG;
    if (pl->d.nnz > 0 && !pl->P_bound) return TSNE_E_STATE;
    tsne_status s = step_args(pl, Y, uY, gains, sc, iter);
    if (s != TSNE_OK) return s;
    return enqueue_iteration(pl);
}

tsne_status tsne_run(tsne_plan* pl, void* Y, void* uY, void* gains, const tsne_sched* sc,
                     int32_t iter0, int32_t n_iter)
{
    if (!pl || !Y || !uY || !gains || !sched_ok(sc) || iter0 < 0 || n_iter < 0) return TSNE_E_ARG;
    if (!point_aligned(pl->d, Y) || !point_aligned(pl->d, uY) || !point_aligned(pl->d, gains)) return TSNE_E_ARG;
    if (pl->d.nnz > 0 && !pl->P_bound) return TSNE_E_STATE;
    if (n_iter == 0) return TSNE_OK;
    tsne_status s = step_args(pl, Y, uY, gains, sc, iter0);
    if (s != TSNE_OK) return s;
    // the first iteration runs eagerly, the rest replay a captured graph of one
    // iteration (the device iteration counter selects the schedule)
    s = enqueue_iteration(pl);
    if (s != TSNE_OK || n_iter == 1) return s;
    if (pl->st == nullptr) {
        for (int32_t i = 1; i < n_iter; ++i) {
            s = enqueue_iteration(pl);
            if (s != TSNE_OK) return s;
        }
        return TSNE_OK;
    }
    if (!pl->graph_ok) {
        if (!hip_ok(hipStreamBeginCapture(pl->st, hipStreamCaptureModeThreadLocal))) return TSNE_E_HIP;
        tsne_status cs = enqueue_iteration(pl);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(pl->st, &g);
        if (cs != TSNE_OK || e != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return cs != TSNE_OK ? cs : TSNE_E_HIP;
        }
        if (!hip_ok(hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0))) {
            hipGraphDestroy(g);
            return TSNE_E_HIP;
        }
        pl->graph = g;
        pl->graph_ok = true;
    }
    for (int32_t i = 1; i < n_iter; ++i)
        if (!hip_ok(hipGraphLaunch(pl->gexec, pl->st))) return TSNE_E_HIP;
    return TSNE_OK;
}

tsne_status tsne_query(tsne_plan* pl, tsne_stats* out)
{
    if (!pl || !out) return TSNE_E_ARG;
    Geom g;
    int small[2];
    if (!hip_ok(hipStreamSynchronize(pl->st)) ||
        !hip_ok(hipMemcpy(&g, pl->h.geom, sizeof(Geom), hipMemcpyDeviceToHost)) ||
        !hip_ok(hipMemcpy(small, pl->h.status, sizeof(small), hipMemcpyDeviceToHost)) ||
        !hip_ok(hipMemset(pl->h.status, 0, sizeof(int))))
        return TSNE_E_HIP;
    std::memset(out, 0, sizeof(*out));
    out->status = small[0];
    out->iter = small[1];
    out->n_int = g.n_int;
    out->n_nodes = g.n;
    out->fft_len = g.M;
    out->max_intervals = pl->d.max_intervals;
    out->origin[0] = g.origin[0];
    out->origin[1] = g.origin[1];
    out->origin_z = g.origin[2];
    out->w_int = g.w;
    out->box_side = g.side;
    out->Z = g.Z;
    out->n_int_y = (pl->d.s >= 2) ? g.n_int_y : 1;
    out->n_nodes_y = (pl->d.s >= 2) ? g.n_y : 1;
    out->fft_len_y = (pl->d.s == 2) ? g.My : 0;
    return TSNE_OK;
}

tsne_status tsne_debug_export(tsne_plan* pl, int32_t what, void* dst, size_t* bytes)
{
    if (!pl || !bytes) return TSNE_E_ARG;
    const Derived& o = pl->o;
    const size_t grid = (pl->d.s == 3) ? (size_t)o.n_cap * o.n_cap * o.n_cap
                      : (pl->d.s == 2) ? (size_t)o.n_cap * o.n_cap : (size_t)o.n_cap;
    const void* src;
    size_t nb;
    switch (what) {
    case 0: src = pl->h.W; nb = (size_t)o.tsz * o.nc * grid; break;
    case 1: src = pl->h.V; nb = (size_t)o.tsz * o.np * grid; break;
    case 2: src = pl->h.R; nb = (size_t)o.tsz * pl->d.n * pl->d.s; break;
    case 4: src = pl->h.perm; nb = sizeof(int) * pl->d.n; break;
    case 5:
        if (!pl->h.h1keep) return TSNE_E_STATE;
        src = pl->h.h1keep;
        nb = sizeof(double) * pl->d.n;
        break;
    case 3: {
        Geom g;
        if (!hip_ok(hipStreamSynchronize(pl->st)) ||
            !hip_ok(hipMemcpy(&g, pl->h.geom, sizeof(Geom), hipMemcpyDeviceToHost)))
            return TSNE_E_HIP;
        src = pl->h.cell_start;
        nb = sizeof(int) * ((size_t)std::min(g.n_cells, o.ncell_cap) + 1);
        break;
    }
    default: return TSNE_E_ARG;
    }
    if (!dst) {
        *bytes = nb;
        return TSNE_OK;
    }
    if (*bytes < nb) return TSNE_E_ARG;
    if (!hip_ok(hipStreamSynchronize(pl->st)) || !hip_ok(hipMemcpy(dst, src, nb, hipMemcpyDeviceToHost)))
        return TSNE_E_HIP;
    *bytes = nb;
    return TSNE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- repulsion without allocation

// Scratch of tsne_repulsive_static: one plan workspace of at most
// TSNE_STATIC_SCRATCH_BYTES in a file-scope device array, one copy per GPU
// (each device holds it until the process ends).  Host code never passes the
// array's name to a kernel or a copy: the name is a host-side stand-in, so its
// device address is looked up once per device and kept in g_scratch.
namespace {
constexpr size_t kScratchBytes = (size_t)TSNE_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static_assert(kScratchBytes % kAlign == 0, "scratch size must keep the workspace alignment");
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];
static char* g_scratch[kMaxDevices];            // device address of scratch, per device
static tsne_plan g_static_plan[kMaxDevices];    // the plan laid over it, per device

extern "C" {

tsne_status tsne_repulsive_static(const tsne_desc* desc, const void* Y, void* F_rep, double* Z,
                                  void* stream)
{
    if (!desc || !Y || !F_rep) return TSNE_E_ARG;
    tsne_desc d = *desc;
    d.nnz = 0;                       // the repulsion does not read P
    Derived o;
    tsne_status rs = derive(&d, o);
    if (rs != TSNE_OK) return rs;
    if (!point_aligned(d, Y) || !point_aligned(d, F_rep)) return TSNE_E_ARG;
    if (o.L.total > kScratchBytes) return TSNE_E_WORKSPACE;
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev))) return TSNE_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return TSNE_E_UNSUPPORTED;
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) || !p) return TSNE_E_HIP;
        g_scratch[dev] = static_cast<char*>(p);
    }
    tsne_plan* pl = &g_static_plan[dev];
    rs = plan_init(pl, &d, o, g_scratch[dev], static_cast<hipStream_t>(stream));
    if (rs != TSNE_OK) return rs;
    return tsne_repulsive(pl, Y, F_rep, Z);
}

}  // extern "C"

// ---------------------------------------------------------------- batch

namespace {

struct Slot {
    bool used;
    tsne_plan* plan;
};

}  // namespace

struct tsne_batch {
    int max_slots, s, dtype, p, form;
    hipStream_t st;
    char* ws;
    Inst* dtable;
    int* dprefix;
    std::vector<Slot> slots;
    std::vector<int> live;              // slot ids in table order
    std::vector<int> prefix_host;       // [K_NKINDS][nlive + 1]
    Launch launch[K_NKINDS];
    Cfg cfg;
    bool dirty;
    bool graph_ok;
    hipGraph_t graph;
    hipGraphExec_t gexec;
};

static size_t batch_table_bytes(int max_slots)
{
    return align_up(sizeof(Inst) * (size_t)max_slots);
}

static void batch_drop_graph(tsne_batch* b)
{
    if (b->graph_ok) {
        hipGraphExecDestroy(b->gexec);
        hipGraphDestroy(b->graph);
        b->graph_ok = false;
    }
}

// Rebuild the device instance table and the per-kind block tables for the
// current set of slots.
static tsne_status batch_refresh(tsne_batch* b)
{
    b->live.clear();
    for (int i = 0; i < b->max_slots; ++i)
        if (b->slots[i].used) b->live.push_back(i);
    const int nl = (int)b->live.size();
    b->prefix_host.assign((size_t)K_NKINDS * (nl + 1), 0);
    for (int k = 0; k < K_NKINDS; ++k) {
        b->launch[k] = Launch{0, 256, 0};
    }
    for (int j = 0; j < nl; ++j) {
        tsne_plan* pl = b->slots[b->live[j]].plan;
        if (!hip_ok(hipMemcpyAsync(b->dtable + j, pl->dinst, sizeof(Inst), hipMemcpyDeviceToDevice, b->st)))
            return TSNE_E_HIP;
        for (int k = 0; k < K_NKINDS; ++k) {
            int* pre = b->prefix_host.data() + (size_t)k * (nl + 1);
            pre[j + 1] = pre[j] + pl->o.vb[k];
            const Launch l = launch_of(k, pl->o, pl->o.vb[k]);
            b->launch[k].block = std::max(b->launch[k].block, l.block);
            b->launch[k].lds = std::max(b->launch[k].lds, l.lds);
        }
    }
    for (int k = 0; k < K_NKINDS; ++k) {
        const int total = b->prefix_host[(size_t)k * (nl + 1) + nl];
        b->launch[k].grid = std::min(total, kGridCap);
    }
    if (nl > 0 &&
        !hip_ok(hipMemcpyAsync(b->dprefix, b->prefix_host.data(), b->prefix_host.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->st)))
        return TSNE_E_HIP;
    if (!hip_ok(hipStreamSynchronize(b->st))) return TSNE_E_HIP;
    batch_drop_graph(b);
    b->dirty = false;
    return TSNE_OK;
}

static tsne_status batch_enqueue_tick(tsne_batch* b)
{
    const int nl = (int)b->live.size();
    LaunchMap map{b->dtable, b->dprefix, nl};
    int nk;
    const int* ch = chain_of(b->s, nk);
    for (int i = 0; i <= nk + 2; ++i) {
        const int k = (i < nk) ? ch[i] : (i == nk ? K_ATTR : (i == nk + 1 ? K_ATTR_T : K_UPDATE));
        if (b->launch[k].grid <= 0) continue;
        if (!hip_ok(launch_kind(k, b->cfg, map, b->launch[k], b->st))) return TSNE_E_HIP;
    }
    return TSNE_OK;
}

extern "C" {

size_t tsne_batch_workspace_bytes(int32_t max_slots)
{
    if (max_slots < 1 || max_slots > 4096) return 0;
    return batch_table_bytes(max_slots) + align_up(sizeof(int) * K_NKINDS * (size_t)(max_slots + 1));
}

tsne_status tsne_batch_create(int32_t max_slots, int32_t s, int32_t dtype, int32_t p, int32_t form,
                              int32_t lanes_per_row, void* workspace, size_t bytes, void* stream,
                              tsne_batch** out)
{
    if (!out) return TSNE_E_ARG;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096 || (s != 1 && s != 2) || (dtype != 0 && dtype != 1) ||
        (form != 0 && form != 1 && form != 2))
        return TSNE_E_ARG;
    if (lanes_per_row == 0) lanes_per_row = 32;
    if (lanes_per_row != 4 && lanes_per_row != 8 && lanes_per_row != 16 && lanes_per_row != 32 &&
        lanes_per_row != 64)
        return TSNE_E_ARG;
    if (p < 2 || p > kMaxP) return TSNE_E_UNSUPPORTED;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || bytes < tsne_batch_workspace_bytes(max_slots))
        return TSNE_E_WORKSPACE;
    tsne_batch* b = new (std::nothrow) tsne_batch();
    if (!b) return TSNE_E_HIP;
    b->max_slots = max_slots;
    b->s = s;
    b->dtype = dtype;
    b->p = p;
    b->form = form;
    b->st = static_cast<hipStream_t>(stream);
    b->ws = static_cast<char*>(workspace);
    b->dtable = reinterpret_cast<Inst*>(b->ws);
    b->dprefix = reinterpret_cast<int*>(b->ws + batch_table_bytes(max_slots));
    b->slots.assign(max_slots, Slot{false, nullptr});
    b->dirty = true;
    b->graph_ok = false;
    b->cfg = Cfg{dtype, s, p, form, lanes_per_row};
    *out = b;
    return TSNE_OK;
}

tsne_status tsne_batch_destroy(tsne_batch* b)
{
    if (!b) return TSNE_E_ARG;
    batch_drop_graph(b);
    for (auto& sl : b->slots)
        if (sl.used) tsne_plan_destroy(sl.plan);
    delete b;
    return TSNE_OK;
}

tsne_status tsne_batch_admit(tsne_batch* b, const tsne_desc* desc, void* plan_ws, size_t plan_ws_bytes,
                             void* Y, void* uY, void* gains, const int64_t* row_ptr,
                             const int32_t* col, const void* val, const tsne_sched* sc,
                             int32_t iter0, int32_t n_iter, int32_t* slot)
{
    if (!b || !desc || !slot || !Y || !uY || !gains || !sched_ok(sc) || iter0 < 0 || n_iter < 0)
        return TSNE_E_ARG;
    if (desc->s != b->s || desc->dtype != b->dtype || desc->p != b->p || desc->form != b->form)
        return TSNE_E_ARG;
    if (!point_aligned(*desc, Y) || !point_aligned(*desc, uY) || !point_aligned(*desc, gains)) return TSNE_E_ARG;
    // every slot shares one attraction launch: CSR rows, the batch's lanes per row, one slab
    if ((desc->lanes_per_row != 0 && desc->lanes_per_row != b->cfg.lpr) ||
        (desc->attr_slabs != 0 && desc->attr_slabs != 1) || desc->attr_layout == 2)
        return TSNE_E_UNSUPPORTED;
    tsne_desc dd = *desc;
    dd.lanes_per_row = b->cfg.lpr;
    dd.attr_slabs = 1;
    dd.attr_layout = 1;
    desc = &dd;
    int free_id = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (!b->slots[i].used) { free_id = i; break; }
    if (free_id < 0) return TSNE_E_CAPACITY;
    tsne_plan* pl = nullptr;
    tsne_status s = tsne_plan_create(desc, plan_ws, plan_ws_bytes, b->st, &pl);
    if (s != TSNE_OK) return s;
    if (desc->nnz > 0) {
        s = tsne_bind_P(pl, row_ptr, col, val);
        if (s != TSNE_OK) { tsne_plan_destroy(pl); return s; }
    }
    s = step_args(pl, Y, uY, gains, sc, iter0);
    CallArgs a = no_args();
    a.set_end = 1;
    a.iter_end = iter0 + n_iter;
    if (s != TSNE_OK || !hip_ok(launch_set_args(pl->dinst, a, b->st))) {
        tsne_plan_destroy(pl);
        return TSNE_E_HIP;
    }
    pl->h.iter_end = iter0 + n_iter;
    b->slots[free_id] = Slot{true, pl};
    b->dirty = true;
    *slot = free_id;
    return TSNE_OK;
}

tsne_status tsne_batch_tick(tsne_batch* b, int32_t n_ticks)
{
    if (!b || n_ticks < 0) return TSNE_E_ARG;
    if (b->dirty) {
        tsne_status s = batch_refresh(b);
        if (s != TSNE_OK) return s;
    }
    if (b->live.empty() || n_ticks == 0) return TSNE_OK;
    int t = 0;
    if (b->st == nullptr) {
        for (; t < n_ticks; ++t) {
            tsne_status s = batch_enqueue_tick(b);
            if (s != TSNE_OK) return s;
        }
        return TSNE_OK;
    }
    if (!b->graph_ok) {
        if (!hip_ok(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal))) return TSNE_E_HIP;
        tsne_status cs = batch_enqueue_tick(b);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->st, &g);
        if (cs != TSNE_OK || e != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return cs != TSNE_OK ? cs : TSNE_E_HIP;
        }
        if (!hip_ok(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0))) {
            hipGraphDestroy(g);
            return TSNE_E_HIP;
        }
        b->graph = g;
        b->graph_ok = true;
    }
    for (; t < n_ticks; ++t)
        if (!hip_ok(hipGraphLaunch(b->gexec, b->st))) return TSNE_E_HIP;
    return TSNE_OK;
}

tsne_status tsne_batch_poll(tsne_batch* b, int32_t slot, int32_t* iters_done, int32_t* status)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return TSNE_E_ARG;
    tsne_plan* pl = b->slots[slot].plan;
    int small[2];
    if (!hip_ok(hipStreamSynchronize(b->st)) ||
        !hip_ok(hipMemcpy(small, pl->h.status, sizeof(small), hipMemcpyDeviceToHost)))
        return TSNE_E_HIP;
    if (iters_done) *iters_done = small[1];
    if (status) *status = small[0];
    return TSNE_OK;
}

tsne_status tsne_batch_retire(tsne_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return TSNE_E_ARG;
    if (!hip_ok(hipStreamSynchronize(b->st))) return TSNE_E_HIP;
    tsne_plan_destroy(b->slots[slot].plan);
    b->slots[slot] = Slot{false, nullptr};
    b->dirty = true;
    return TSNE_OK;
}

}  // extern "C"
