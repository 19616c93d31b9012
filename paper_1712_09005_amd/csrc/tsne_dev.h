// Internal definitions shared by the HIP kernels and the host runtime.
//
// Everything a kernel needs about one embedding ("instance") sits in an Inst
// record in device memory: sizes, the caller's buffers and the workspace
// regions.  A launch covers a list of instances: each kernel kind has a
// per-instance count of virtual blocks and a prefix table over them, so a
// single plan and a batch of uneven embeddings go through the same kernels.
#pragma once

#include <stdint.h>

#ifndef TSNE_HOST_ONLY
#include <hip/hip_runtime.h>
#endif

namespace tsne {

constexpr int kMaxStages = 24;   // FFT radix stages
constexpr int kMaxP = 6;         // Lagrange nodes per interval
constexpr int kWave = 64;

// Binning: stable least-significant-digit radix sort of the points by cell.
constexpr int kBoxPart = 16;      // doubles per block of the box partials
constexpr int kUpdPts = 4;              // points per thread of the update kernel
constexpr int kTileWindowBytes = 32768;   // one LDS column window of the tiled attraction
// non-zeros per sweep step of the tiled attraction: 1024 threads x 2, or x 3
// when a column window holds 8192 points (FP32 in 1-D).  A tile (about n/256
// rows by one window) holds about k w / 256 non-zeros for k per row and w
// points per window: 1440 at k = 90 and w = 4096, 2880 at w = 8192, which
// would take two steps of 2048.
constexpr int tile_step_edges(int window_points) { return window_points >= 8192 ? 3072 : 2048; }
constexpr int kKeyTile = 2048;     // points per block of the key kernel (256 threads x 8)
constexpr int kSortTile = 2048;    // points per tile of a sort pass (256 threads x 8)
constexpr int kScanCells = 256;   // cells per tile of the item scans (a thread each)
constexpr int kScanDigits = 64;    // digits per block of the tile-offset scan (a lane each)
constexpr int kScanGroups = 16;    // at most this many groups of tiles per radix pass
constexpr int kDigitBitsMax = 9;   // at most 512 digit values per pass
constexpr int kDigitBins = 1 << kDigitBitsMax;
constexpr int kMaxSortPass = 3;    // cell indices of up to 27 bits

// Kernel kinds with their own virtual-block tables.
enum Kind : int {
    K_ARGS = 0, K_BOX, K_KEY, K_SORT0, K_SORT1, K_SORT2, K_BOUNDS, K_SCAN_A, K_SCAN_B, K_SPREAD, K_FIX,
    K_FFT_ROWS, K_FFT_COLS, K_FFT_IROWS, K_FFT_1D, K_GATHER, K_NORM, K_ATTR,
    K_UPDATE, K_SPEC0, K_SPEC1, K_SPEC2, K_GEOM, K_ZSUM, K_ATTR_ALL, K_ASUM, K_ATTR_T, K_ATTR_T_ALL,
    K_KLSUM, K_KL_ATTR, K_HIST1, K_HIST2, K_TSCAN0, K_TSCAN1, K_TSCAN2,
    K_F3_X, K_F3_Y, K_F3_Z, K_F3_IY, K_F3_IX, K_S3_FILL, K_S3_X, K_S3_Y, K_S3_Z, K_S3_STORE,
    K_SPREAD3, K_GATHER3, K_KL_T, K_NKINDS
};

// Status bits latched on the device (values of tsne_status).
enum : int { ST_OK = 0, ST_CAPACITY = 4, ST_NONFINITE = 5, ST_INTERNAL = 8 };

// Geometry of the current iteration, written by the box kernel (double).
struct Geom {
    double origin[3];
    double centre[3];
    double mean[3];
    double w;          // interval width
    double inv_w;
    double h;          // node spacing w / p
    double side;       // L
    double qscale;     // power-of-two charge scale
    double Z;          // normalisation of the last repulsion
    int n_int;         // intervals per dimension
    int n;             // nodes per dimension, n_int * p
    int n_cells;       // n_int^s
    int active;        // this iteration runs (set by the geometry kernel)
    int it;            // absolute index of this iteration
    int sort_bits;     // digit bits per radix pass this iteration
    int spec_dirty;    // spacing or FFT length changed: tables must be rebuilt
    double spec_h;     // spacing the current spectra were built for
    int spec_M;        // FFT lengths the current tables were built for
    int spec_My;
    // first axis (x, dimension 0): rows of the grid
    int M;             // circulant length of this iteration (even, 2-3-5 smooth, >= 2n)
    int half;          // M / 2 + 1
    int nstages;
    int radix[kMaxStages];
    int tw_off[kMaxStages];   // offset of each stage's twiddle table in tw
    // second axis (y, dimension 1; s = 2): columns of the grid.  Equal to the
    // first axis' values for the square box.
    int n_int_y;       // intervals along y
    int n_y;           // nodes along y
    int My, half_y, nstages_y;
    int radix_y[kMaxStages];
    int tw_off_y[kMaxStages];  // offsets in twy
    int col_group;     // FFT columns per block this iteration (for My)
};

// LDS index of element i of a transform and the stride between the
// transforms of one block.  Unpadded: measured faster at the lengths in use
// (a pad slot per 8, 16 or 32 values cost more index arithmetic than the bank
// conflicts of the early strided Stockham writes); the odd stride keeps the
// transforms of a block on different banks.
__host__ __device__ constexpr int lds_pad(int i) { return i; }
__host__ __device__ constexpr int lds_stride(int M) { return M + 1; }

struct Sched {
    double eta, mom0, mom1, ee_alpha, le_alpha, gain_inc, gain_dec, gain_min;
    int mom_switch, ee_stop, le_start, recentre;
};

struct Inst {
    // ---- configuration (fixed for the plan)
    int64_t n;
    int64_t nnz;
    int s, p, form, nc, np, policy, rect;
    int min_int, max_int, n_cap, M, half;      // capacity: largest M, M/2 + 1
    int ncell_cap, items_cap, kpts, lpr;
    int col_group, tile_w, ntiles;              // FFT column kernel grouping
    double interval_width;
    int iter_end;                               // iterations stop at this index
    int counting;                               // the geometry kernel advances *iter
    int col_lds;                                // LDS bytes of the FFT column kernel

    // ---- caller buffers (set per call by k_set_args)
    const void* Yin;       // positions read by repulsion / attraction
    void* Y;               // positions updated by the step
    void* uY;
    void* gains;
    void* Frep;            // tsne_repulsive output (normalised)
    double* Zout;          // tsne_repulsive output
    void* Fattr;           // attraction output (caller's or workspace)
    const int64_t* row_ptr;
    const int32_t* col;
    const void* val;
    const void* cv;        // FP32 CSR: [nnz] (column, value bits) pairs packed at bind time

    // ---- workspace regions
    Geom* geom;
    Sched* sched;
    int* status;
    int* iter;
    double* box_part;      // [nb_box][2*s+... ] partial min/max/sum
    int* cell_start;       // [ncell_cap + 1]
    int* item_start;       // [ncell_cap + 1]
    int* scan_part;        // [2 * nb_scan] tile sums
    int* item_cell;        // [items_cap] cell of each item
    int* key;              // [n] cell of each point (point order)
    void* kv;              // [2][n] (cell, point) pairs between radix passes (uint2)
    unsigned* skey;        // [n] cell of each sorted position
    int* perm;             // [n] sorted position -> point
    unsigned* tcnt;        // [npass][ntiles_sort][kDigitBins] digit counts of every tile,
                           // replaced by the tile's first output position per digit
    unsigned* gtot;        // [npass][ngroups_sort][kDigitBins] digit counts of every group of tiles
    int npass, ntiles_sort;    // radix passes (from the cell capacity), sort tiles
    int group_tiles, ngroups_sort;  // tiles per group of the offset scan (a multiple of 4), groups
    void* sY;              // [n][s] sorted positions
    void* carry;           // [2 * nwaves][1 + p^s * nc] spread carries
    void* W;               // [nc][n_cap][n_cap] (s = 2) or [nc][n_cap]
    void* X;               // [nc][ntiles][n_cap][tile_w] complex (row spectra)
    void* Xc;              // [np][ntiles][n_cap][tile_w] complex (after columns)
    void* V;               // [np][n_cap][n_cap] or [np][n_cap]
    void* spec;            // s = 2: [K][half_x][half_y] in slots of the capacity's
                           // half^2; s = 1: [2][half]; pre-scaled
    void* tw;              // [M] stage twiddle tables of this iteration's M (complex)
    void* twy;             // [M] the same for the second axis' length My
    void* twd;             // s = 3: [M] the stage twiddles in double (kernel spectra)
    void* specd;           // s = 3: [2][M^3] complex double, the kernel grids' transforms
    double* costab;        // [2][M] cos and sin(2 pi k / M) in double (s = 1)
    // s = 2 tables, each in a [half][half] slot of the capacity's half:
    double* spec_tmp;      // [K][..] first transform pass (double)
    double* ktab;          // [K][..] kernel values on the lag grid [j1][j0] (double)
    double* ccos;          // [2 or 4][..] weighted cosine matrices of x and y, then
                           // (form V) the sine matrices of x and y (double)
    void* R;               // [n][s] unnormalised repulsion numerators
    void* Fa_ws;           // [n][s] attraction (workspace copy for the step)
    void* Fap;             // [slabs][n][s] attraction partials per column slab
    const int* split;      // [slabs - 1][n] first non-zero of each later slab per row
    int slabs;             // column slabs of P (1: no split)
    int slab_w;            // points per column slab
    int tiled;             // attraction by row blocks sweeping LDS column windows
    int tile_bi, tile_bj;  // rows per row block / points per column window
    int tile_ni, tile_nj;  // row blocks, column windows
    const int* tsb;        // [ni + 1] first sweep step of each row block
    const int* tsj;        // [steps] column window of each step
    const int64_t* tse;    // [steps + 1] first edge of each step
    const uint32_t* epack; // [nnz] (row in block << 16) | column in window, step order
    const void* eval;      // [nnz] values in step order
    double tscale;         // fixed-point scale of the row sums (set with P)
    double* z_part;        // [nb_gather]
    double* h1keep;        // [n] each point's K1 sum h1 of the last repulsion (point order), or null
    double* kl_part;       // [nb_kl][2] divergence partials (sum p log(p/K1), sum p)
    double* KLout;         // caller's divergence output (device, may be null)
    int nb_box, nb_gather, nb_scan, nwaves, nb_kl;
};

// Launch table: first virtual block of each instance per kernel kind.
struct LaunchMap {
    const Inst* insts;     // device array
    const int* prefix;     // device [K_NKINDS][ninst + 1]
    int ninst;
};

#ifndef TSNE_HOST_ONLY

template <typename T> struct cplx { T x, y; };

// Global-memory view of a pointer taken from the instance record: loads
// through it are vector-memory only (a generic pointer gives flat loads,
// which every LDS wait also waits for).
#define TSNE_GLOBAL __attribute__((address_space(1)))
template <typename P> __device__ __forceinline__ const TSNE_GLOBAL P* gview(const void* p)
{
    return (const TSNE_GLOBAL P*)p;
}
// Constant-memory view of read-only data indexed uniformly across the block
// (scalar loads, which the vector-memory waits do not drain).
#define TSNE_CONST __attribute__((address_space(4)))
template <typename P> __device__ __forceinline__ const TSNE_CONST P* cview(const void* p)
{
    return (const TSNE_CONST P*)p;
}

// One complex element through the global view, as one vector load.
template <typename T> __device__ __forceinline__ cplx<T> gload_c(const void* base, int64_t i)
{
    typedef T N __attribute__((ext_vector_type(2)));
    const N q = gview<N>(base)[i];
    return {q.x, q.y};
}
// One complex element stored through the global view, as one vector store.
template <typename T> __device__ __forceinline__ void gstore_c(void* base, int64_t i, cplx<T> v)
{
    typedef T N __attribute__((ext_vector_type(2)));
    N q;
    q.x = v.x;
    q.y = v.y;
    ((TSNE_GLOBAL N*)base)[i] = q;
}

__device__ __forceinline__ int find_inst(const int* __restrict__ pre, int ninst, int vb)
{
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= vb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Before the geometry kernel: no latched status and the iteration counter
// has not reached iter_end.
__device__ __forceinline__ bool live_pre(const Inst& I)
{
    return *I.status == 0 && *I.iter < I.iter_end;
}

// After the geometry kernel: this iteration runs (written once per iteration
// by the geometry kernel; later kernels only read it).
__device__ __forceinline__ bool live(const Inst& I) { return I.geom->active != 0; }

// Iterate over this launch's virtual blocks of kernel kind K:
//   VB_LOOP(map, K) { const Inst& I = ...; int lb = ...; ... }
#define VB_BEGIN(map, KIND)                                                    \
    {                                                                          \
        const int* __pre = (map).prefix + (KIND) * ((map).ninst + 1);          \
        const int __total = __pre[(map).ninst];                                \
        for (int __vb = blockIdx.x; __vb < __total; __vb += gridDim.x) {       \
            const int inst_id = find_inst(__pre, (map).ninst, __vb);           \
            const Inst& I = (map).insts[inst_id];                              \
            const int lb = __vb - __pre[inst_id];                              \
            (void)lb;
#define VB_END \
        }      \
    }

// Like VB_BEGIN, but skips virtual blocks whose instance fails COND; COND is
// evaluated once per instance change (not per virtual block), which keeps
// launches that are usually idle cheap.
#define VB_BEGIN_IF(map, KIND, COND)                                           \
    {                                                                          \
        const int* __pre = (map).prefix + (KIND) * ((map).ninst + 1);          \
        const int __total = __pre[(map).ninst];                                \
        int __last = -1;                                                       \
        bool __ok = false;                                                     \
        for (int __vb = blockIdx.x; __vb < __total; __vb += gridDim.x) {       \
            const int inst_id = find_inst(__pre, (map).ninst, __vb);           \
            const Inst& I = (map).insts[inst_id];                              \
            if (inst_id != __last) {                                           \
                __last = inst_id;                                              \
                __ok = (COND);                                                 \
            }                                                                  \
            if (!__ok) continue;                                               \
            const int lb = __vb - __pre[inst_id];                              \
            (void)lb;

// Like VB_BEGIN_IF, but a failing instance is stepped over in one jump, for
// launches with many virtual blocks per instance that are usually idle.
#define VB_BEGIN_IF_SKIP(map, KIND, COND)                                      \
    {                                                                          \
        const int* __pre = (map).prefix + (KIND) * ((map).ninst + 1);          \
        const int __total = __pre[(map).ninst];                                \
        int __last = -1;                                                       \
        bool __ok = false;                                                     \
        for (int __vb = blockIdx.x; __vb < __total; __vb += gridDim.x) {       \
            const int inst_id = find_inst(__pre, (map).ninst, __vb);           \
            const Inst& I = (map).insts[inst_id];                              \
            if (inst_id != __last) {                                           \
                __last = inst_id;                                              \
                __ok = (COND);                                                 \
            }                                                                  \
            if (!__ok) {                                                       \
                const int __end = __pre[inst_id + 1];                          \
                const int __k = (__end - __vb + (int)gridDim.x - 1) / (int)gridDim.x; \
                __vb += (__k - 1) * (int)gridDim.x;                            \
                continue;                                                      \
            }                                                                  \
            const int lb = __vb - __pre[inst_id];                              \
            (void)lb;

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum of a double (result valid in thread 0).  Needs blockDim.x a
// multiple of 64 and <= 1024.
__device__ __forceinline__ double block_sum_d(double v, double* sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += sh[i];
    }
    return r;
}

#endif  // TSNE_HOST_ONLY

}  // namespace tsne
