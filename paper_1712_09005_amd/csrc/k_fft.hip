// Step 2 of Algorithm 1 on gfx950: the grid sums v = K~ w evaluated as a
// circulant (block-circulant for s = 2) convolution by FFT (Section 2.2,
// Section 2.4).  Hand-written mixed-radix (2, 3, 4, 5) Stockham transforms run
// in LDS; each stage reads its butterflies into registers, synchronises and
// writes them back, so one LDS buffer per transform suffices.
//
// 2-D layout and passes (M = circulant length per dimension, M even):
//   rows:  two real node rows of one charge grid packed into one complex
//          transform; the two half spectra are unpacked and stored in column
//          tiles X[c][k0 / tw][row][k0 % tw] (tw complex = 128 bytes);
//   cols:  for each potential, tiles of columns: forward transform, multiply
//          by the (real, even) kernel spectrum, inverse transform, keep the n
//          node rows;
//   irows: two potentials packed per complex inverse transform (an odd last
//          potential packs two of its rows), keep n nodes.
// The kernel spectra are built in double by direct cosine sums (the circulant
// of an even kernel has a real, even spectrum) and stored pre-scaled by 1/M^s.
#include <math.h>

#include "launch.h"

namespace tsne {

constexpr int kMaxB = 4;   // butterflies per thread per stage (host-enforced)
constexpr int kLd = 8;     // global loads a thread issues before it uses the first

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by -i
template <typename T> __device__ __forceinline__ cplx<T> mnegi(cplx<T> a) { return {a.y, -a.x}; }
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

// Forward DFTs of length R (kernel exp(-2 pi i k n / R)).
template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
    static __device__ __forceinline__ void run(cplx<T> (&v)[2])
    {
        const cplx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T> struct Dft<T, 3> {
    static __device__ __forceinline__ void run(cplx<T> (&v)[3])
    {
        const T s3 = (T)0.86602540378443864676;   // sin(2 pi / 3)
        const cplx<T> t1 = cadd(v[1], v[2]);
        const cplx<T> t2 = csub(v[0], cscale(t1, (T)0.5));
        const cplx<T> t3 = cscale(csub(v[1], v[2]), s3);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, mnegi(t3));
        v[2] = csub(t2, mnegi(t3));
    }
};

template <typename T> struct Dft<T, 4> {
    static __device__ __forceinline__ void run(cplx<T> (&v)[4])
    {
        const cplx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        const cplx<T> c = cadd(v[1], v[3]), d = mnegi(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    }
};

template <typename T> struct Dft<T, 5> {
    static __device__ __forceinline__ void run(cplx<T> (&v)[5])
    {
        const T c1 = (T)0.30901699437494742410;    // cos(2 pi / 5)
        const T c2 = (T)-0.80901699437494742410;   // cos(4 pi / 5)
        const T s1 = (T)0.95105651629515357212;    // sin(2 pi / 5)
        const T s2 = (T)0.58778525229247312917;    // sin(4 pi / 5)
        const cplx<T> a = cadd(v[1], v[4]), b = cadd(v[2], v[3]);
        const cplx<T> c = csub(v[1], v[4]), d = csub(v[2], v[3]);
        const cplx<T> x0 = v[0];
        const cplx<T> p1 = cadd(x0, cadd(cscale(a, c1), cscale(b, c2)));
        const cplx<T> p2 = cadd(x0, cadd(cscale(a, c2), cscale(b, c1)));
        const cplx<T> q1 = mnegi(cadd(cscale(c, s1), cscale(d, s2)));
        const cplx<T> q2 = mnegi(csub(cscale(c, s2), cscale(d, s1)));
        v[0] = cadd(x0, cadd(a, b));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

// floor(j / d) for 0 <= j < 2^21 and 0 < d < 2^21, with h = 1 / (2 d) to
// within one ulp: (j + 1/2) / d lies at least 1 / (2 d) from every integer,
// and the float product (2 j + 1) h is within (j + 1/2) 2^-22 / d of it, which
// is less, so truncating it gives the quotient with no correction step.
__device__ __forceinline__ int fdiv(int j, float h)
{
    return (int)((float)(2 * j + 1) * h);
}

// One Stockham stage of radix R over G transforms of length M stored at
// stride PM (padded indices) in buf; Ns = product of the radices of earlier
// stages.  Butterfly j = a Ns + k reads x[j + r M/R], multiplies by the
// twiddles w^(r k M/(Ns R)) (this stage's table, R-1 values per k), applies
// the length-R DFT and writes to a Ns R + k + r Ns.
template <typename T, int R>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int M, int PM, int G, int Ns,
                                          const cplx<T>* __restrict__ tws)
{
    const int Mr = M / R;
    const float hNs = 0.5f * __builtin_amdgcn_rcpf((float)Ns);   // 1 / (2 Ns), one ulp
    // the threads split evenly over the G transforms (G and the block size are
    // powers of two), so a thread's transform is fixed for the whole stage
    const int lt = __ffs((int)blockDim.x) - __ffs(G);   // log2 of the threads per transform
    const int tpc = 1 << lt;
    const int g = (int)threadIdx.x >> lt;
    const int jt = (int)threadIdx.x & (tpc - 1);
    const int nbt = (Mr + tpc - 1) >> lt;
    const cplx<T>* src = buf + __mul24(g, PM);
    cplx<T> v[kMaxB][R];
    int dst[kMaxB];
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        if (b >= nbt) break;
        const int j = jt + b * tpc;
        dst[b] = -1;
        if (j < Mr) {
            const int k = j - __mul24(fdiv(j, hNs), Ns);   // j = a Ns + k
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = src[lds_pad(j + r * Mr)];
            if (Ns > 1) {
                // through the global view: vector-memory loads, which the LDS
                // waits of the stage do not wait for
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], gload_c<T>(tws, k * (R - 1) + r - 1));
            }
            Dft<T, R>::run(v[b]);
            dst[b] = __mul24(j - k, R) + k;            // a Ns R + k
        }
    }
    __syncthreads();
    cplx<T>* out = buf + __mul24(g, PM);
    // the outputs' offsets r Ns, uniform: scalar registers, added to the
    // thread's index (else the compiler folds them into 64-bit multiply-adds)
    int rns[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rns[r] = __builtin_amdgcn_readfirstlane(r * Ns);
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        if (b >= nbt) break;
        if (dst[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) out[lds_pad(dst[b] + rns[r])] = v[b][r];
        }
    }
    __syncthreads();
}

// Forward transforms (exp(-2 pi i k n / M)) of G length-M sequences in LDS
// (padded layout, transform g at g * lds_stride(M)), M and the radix stages
// being those of this iteration's first axis (Geom), or of its second axis
// with yaxis set.
template <typename T>
__device__ __forceinline__ void block_fft_tw(cplx<T>* buf, int G, int M, int nst, const int* radix,
                                             const int* tw_off, const cplx<T>* tw)
{
    const int PM = lds_stride(M);
    // the stage plan through the constant view: scalar loads
    const TSNE_CONST int* rad = cview<int>(radix);
    const TSNE_CONST int* two = cview<int>(tw_off);
    int Ns = 1;
    for (int s = 0; s < nst; ++s) {
        const int R = rad[s];
        const cplx<T>* tws = tw + two[s];
        switch (R) {
        case 2: fft_stage<T, 2>(buf, M, PM, G, Ns, tws); break;
        case 3: fft_stage<T, 3>(buf, M, PM, G, Ns, tws); break;
        case 4: fft_stage<T, 4>(buf, M, PM, G, Ns, tws); break;
        default: fft_stage<T, 5>(buf, M, PM, G, Ns, tws); break;
        }
        Ns *= R;
    }
}

template <typename T>
__device__ __forceinline__ void block_fft(cplx<T>* buf, int G, const Inst& I, const Geom& Gm,
                                          bool yaxis = false)
{
    // the geometry through the constant view (scalar loads; a generic
    // reference gives flat loads, which the LDS waits also wait for)
    const TSNE_CONST Geom& C = *cview<Geom>(&Gm);
    const cplx<T>* tw = static_cast<const cplx<T>*>((yaxis && C.My != C.M) ? I.twy : I.tw);
    if (yaxis) block_fft_tw<T>(buf, G, C.My, C.nstages_y, &Gm.radix_y[0], &Gm.tw_off_y[0], tw);
    else block_fft_tw<T>(buf, G, C.M, C.nstages, &Gm.radix[0], &Gm.tw_off[0], tw);
}

__device__ __forceinline__ bool okay(const Inst& I) { return live(I); }

__device__ __forceinline__ bool occupied(const int* __restrict__ cs, int c)
{
    return cs[c + 1] > cs[c];
}

// Charge index and kernel spectrum of potential pot.  Forms A and B: kern 0
// is K1, 1 is K2 (real spectra).  Form V (one charge): kern 0 is K1, 1 + d
// the odd kernel z_d K2 along dimension d, whose spectrum is -i times a real
// table (odd along d, even along the other dimension).
template <int S, int FORM>
__device__ __forceinline__ void pot_of(int pot, int& ch, int& kern)
{
    if (FORM == 2) { ch = 0; kern = pot; return; }
    if (pot == 0) { ch = (FORM == 0) ? 0 : S + 1; kern = (FORM == 0) ? 0 : 1; }
    else if (pot == 1) { ch = 0; kern = 1; }
    else { ch = pot - 1; kern = 1; }
}

template <int S, int FORM> struct Pots {
    static constexpr int NP = (FORM == 2) ? S + 1 : S + 2;
};

// ---------------------------------------------------------------- 2-D passes

// Row passes (512 or 1024 threads): FP32 kernels are held to 80 registers, six
// waves per SIMD, where the compiler would take a few more and fit five.
template <typename T> constexpr int kRowWaves = (sizeof(T) == 4) ? 6 : 4;

template <typename T, int P>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kRowWaves<T>))) void k_fft_rows(LaunchMap map)
{
    extern __shared__ __align__(16) char smem[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
    VB_BEGIN(map, K_FFT_ROWS)
    if (okay(I)) {
        const Geom& G = *I.geom;
        const int n = G.n, ny = G.n_y, n_int = G.n_int, M = G.M, n_cap = I.n_cap, tw_ = I.tile_w;
        const int npairs = (n_cap + 1) / 2;
        const int ch = lb / npairs, j = lb - ch * npairs;
        const int ra = 2 * j, rb = 2 * j + 1;
        if (ra < ny) {
            const T* W = static_cast<const T*>(I.W) + (int64_t)ch * n_cap * n_cap;
            const int* cs = I.cell_start;
            const int cya = ra / P, cyb = rb / P;
            // kLd nodes per thread at a time: the cells' occupancy, then the
            // grid values of occupied cells (unoccupied cells were not written)
            const int nthr = blockDim.x;
            for (int g0 = threadIdx.x; g0 < M; g0 += kLd * nthr) {
                int oa[kLd], ob[kLd];
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int g = g0 + u * nthr;
                    oa[u] = ob[u] = 0;
                    if (g < n) {
                        const int cx = g / P;
                        oa[u] = occupied(cs, cya * n_int + cx);
                        if (rb < ny) ob[u] = occupied(cs, cyb * n_int + cx);
                    }
                }
                T a[kLd], b[kLd];
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int g = g0 + u * nthr;
                    a[u] = oa[u] ? W[(int64_t)ra * n_cap + g] : (T)0;
                    b[u] = ob[u] ? W[(int64_t)rb * n_cap + g] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int g = g0 + u * nthr;
                    if (g < M) buf[lds_pad(g)] = {a[u], b[u]};
                }
            }
            __syncthreads();
            block_fft<T>(buf, 1, I, G);
            cplx<T>* X = static_cast<cplx<T>*>(I.X) + (int64_t)ch * I.ntiles * n_cap * tw_;
            const T hlf = (T)0.5;
            const int ltw = __ffs(tw_) - 1;                // tile_w is a power of two
            for (int k = threadIdx.x; k < G.half; k += blockDim.x) {
                const cplx<T> z = buf[lds_pad(k)], zc = buf[lds_pad(k == 0 ? 0 : M - k)];
                const cplx<T> A = {(z.x + zc.x) * hlf, (z.y - zc.y) * hlf};
                const cplx<T> B = {(z.y + zc.y) * hlf, (zc.x - z.x) * hlf};
                const int tile = k >> ltw, kk = k & (tw_ - 1);
                // within one channel every offset fits 31 bits (n_cap <= 6144)
                const int off = __mul24(tile, n_cap * tw_) + kk;
                X[off + ra * tw_] = A;
                if (rb < ny) X[off + rb * tw_] = B;
            }
            __syncthreads();
        }
    }
    VB_END
}

template <typename T, int S, int FORM>
__global__ __launch_bounds__(1024) void k_fft_cols(LaunchMap map)
{
    extern __shared__ __align__(16) char smem[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
    VB_BEGIN(map, K_FFT_COLS)
    if (okay(I)) {
        const Geom& Gm = *I.geom;
        // columns: the half spectrum of the first axis; each column is a
        // transform of length My over the n_y node rows of the second axis
        const int n = Gm.n_y, M = Gm.My, n_cap = I.n_cap, tw_ = I.tile_w, half = Gm.half;
        const int half_y = Gm.half_y;
        const int64_t kslot = (int64_t)I.half * I.half; // one spectrum table
        const int Gc = Gm.col_group;                   // columns per block this iteration
        const int G = tw_ / Gc;                        // blocks per tile of X
        const int ncg = ((half + tw_ - 1) / tw_) * G;  // blocks per potential this iteration
        // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so
        // transposing each run of 8 x G virtual blocks puts the G blocks that
        // share one tile (and so every cache line of it) on the same XCD,
        // one after another.  A bijection on whole runs; the tail is as is.
        constexpr int NP = Pots<S, FORM>::NP;
        const int vtotal = NP * I.ntiles * (tw_ / I.col_group);
        const int run = 8 * G;
        int L = lb;
        if (lb < (vtotal / run) * run) {
            const int r = lb % run;
            L = lb - r + (r & 7) * G + (r >> 3);
        }
        const int pot = L / ncg, cg = L - pot * ncg;
        if (pot < NP && cg * Gc < half) {
        int ch, kern;
        pot_of<S, FORM>(pot, ch, kern);
        const cplx<T>* X = static_cast<const cplx<T>*>(I.X) + (int64_t)ch * I.ntiles * n_cap * tw_;
        const int PM = lds_stride(M);
        // the Gc columns of a block lie in one tile (Gc divides tile_w, both
        // powers of two): element (r, g) of the block is at tile row r, slot kk0 + g
        const int lgc = __ffs(Gc) - 1;
        const int k00 = cg * Gc;
        const int tile = k00 >> (__ffs(tw_) - 1);
        const int64_t t0 = (int64_t)tile * n_cap * tw_ + (k00 - tile * tw_);
        // consecutive threads: columns of a row; kLd loads in flight per thread
        const int nthr = blockDim.x, nel = M << lgc;
        for (int i0 = threadIdx.x; i0 < nel; i0 += kLd * nthr) {
            cplx<T> v[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int idx = i0 + u * nthr;
                const int r = idx >> lgc, g = idx & (Gc - 1);
                v[u] = {(T)0, (T)0};
                if (idx < nel && k00 + g < half && r < n) v[u] = gload_c<T>(X, t0 + (__mul24(r, tw_) + g));
            }
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int idx = i0 + u * nthr;
                const int r = idx >> lgc, g = idx & (Gc - 1);
                if (idx < nel) buf[__mul24(g, PM) + lds_pad(r)] = v[u];
            }
        }
        __syncthreads();
        block_fft<T>(buf, Gc, I, Gm, true);
        // multiply by the real kernel spectrum, conjugate for the inverse; the
        // threads split evenly over the block's columns
        {
            const int tpc = (int)blockDim.x >> lgc;
            const int g = (int)threadIdx.x >> (__ffs(tpc) - 1);
            const int jt = (int)threadIdx.x - g * tpc;
            const int k0 = k00 + g;
            const T* sp = static_cast<const T*>(I.spec) + (int64_t)kern * kslot + (int64_t)k0 * half_y;
            cplx<T>* col = buf + __mul24(g, PM);
            // the spectrum's values kLd at a time, loaded before they are used
            for (int kb = jt; kb < M; kb += kLd * tpc) {
                T sv[kLd];
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int k1 = kb + u * tpc;
                    const bool up = k1 > M - k1;
                    sv[u] = (k1 < M && k0 < half) ? gview<T>(sp)[up ? M - k1 : k1] : (T)0;
                    // times -i b, b odd in k1 for the kernel odd along dimension 1
                    if (FORM == 2 && kern == 2 && up) sv[u] = -sv[u];
                }
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int k1 = kb + u * tpc;
                    if (k1 < M) {
                        const int li = lds_pad(k1);
                        const cplx<T> v = col[li];
                        if (FORM == 2 && kern > 0) col[li] = {v.y * sv[u], v.x * sv[u]};
                        else col[li] = {v.x * sv[u], -v.y * sv[u]};
                    }
                }
            }
        }
        __syncthreads();
        block_fft<T>(buf, Gc, I, Gm, true);
        cplx<T>* Xc = static_cast<cplx<T>*>(I.Xc) + (int64_t)pot * I.ntiles * n_cap * tw_;
        for (int idx = threadIdx.x; idx < (n << lgc); idx += blockDim.x) {
            const int r = idx >> lgc, g = idx & (Gc - 1);
            if (k00 + g < half) gstore_c<T>(Xc, t0 + (__mul24(r, tw_) + g), cconj(buf[__mul24(g, PM) + lds_pad(r)]));
        }
        __syncthreads();
        }
    }
    VB_END
}

template <typename T, int S, int NP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kRowWaves<T>))) void k_fft_irows(LaunchMap map)
{
    extern __shared__ __align__(16) char smem[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
    VB_BEGIN(map, K_FFT_IROWS)
    if (okay(I)) {
        const Geom& G = *I.geom;
        const int n = G.n, M = G.M, n_cap = I.n_cap, tw_ = I.tile_w;
        const int q = lb / n_cap, r = lb - q * n_cap;
        // two real outputs per complex transform: row r of potentials 2q and
        // 2q + 1, or, for an odd last potential, its rows 2r' and 2r' + 1
        int pa = 2 * q, pb = 2 * q + 1, ra = r, rb = r;
        bool has_b = pb < NP;
        if (!has_b) {
            pb = pa;
            ra = 2 * r;
            rb = 2 * r + 1;
            has_b = rb < G.n_y;
        }
        if (ra < G.n_y) {
            const cplx<T>* Xa = static_cast<const cplx<T>*>(I.Xc) + (int64_t)pa * I.ntiles * n_cap * tw_;
            const cplx<T>* Xb = static_cast<const cplx<T>*>(I.Xc) + (int64_t)pb * I.ntiles * n_cap * tw_;
            const int mh = M / 2;
            const int ltw = __ffs(tw_) - 1;                // tile_w is a power of two
            const int nthr = blockDim.x;
            for (int k0 = threadIdx.x; k0 < M; k0 += kLd * nthr) {
                cplx<T> A[kLd], B[kLd];
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int k = k0 + u * nthr;
                    const int kk = (k > mh) ? M - k : k;
                    const int tile = kk >> ltw;
                    const int64_t off = (int64_t)tile * n_cap * tw_ + (kk & (tw_ - 1));
                    A[u] = B[u] = cplx<T>{(T)0, (T)0};
                    if (k < M) {
                        A[u] = Xa[off + (int64_t)ra * tw_];
                        if (has_b) B[u] = Xb[off + (int64_t)rb * tw_];
                    }
                }
#pragma unroll
                for (int u = 0; u < kLd; ++u) {
                    const int k = k0 + u * nthr;
                    if (k < M) {
                        cplx<T> a = A[u], b = B[u];
                        if (k > mh) { a = cconj(a); b = cconj(b); }
                        // Z = A + i B, stored conjugated (inverse by forward transform)
                        buf[lds_pad(k)] = {a.x - b.y, -(a.y + b.x)};
                    }
                }
            }
            __syncthreads();
            block_fft<T>(buf, 1, I, G);
            T* Va = static_cast<T*>(I.V) + (int64_t)pa * n_cap * n_cap + (int64_t)ra * n_cap;
            T* Vb = static_cast<T*>(I.V) + (int64_t)pb * n_cap * n_cap + (int64_t)rb * n_cap;
            for (int g = threadIdx.x; g < n; g += blockDim.x) {
                const cplx<T> z = buf[lds_pad(g)];   // conj of the inverse
                Va[g] = z.x;
                if (has_b) Vb[g] = -z.y;
            }
            __syncthreads();
        }
    }
    VB_END
}

// ---------------------------------------------------------------- 1-D pass

template <typename T, int P, int FORM>
__global__ __launch_bounds__(1024) void k_fft_1d(LaunchMap map)
{
    extern __shared__ __align__(16) char smem[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
    VB_BEGIN(map, K_FFT_1D)
    if (okay(I)) {
        const Geom& G = *I.geom;
        const int n = G.n, M = G.M, n_cap = I.n_cap, half = G.half;
        const int pot = lb;
        int ch, kern;
        pot_of<1, FORM>(pot, ch, kern);
        const T* W = static_cast<const T*>(I.W) + (int64_t)ch * n_cap;
        const int* cs = I.cell_start;
        const int nthr = blockDim.x;
        for (int g0 = threadIdx.x; g0 < M; g0 += kLd * nthr) {
            int oc[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int g = g0 + u * nthr;
                oc[u] = (g < n) ? occupied(cs, g / P) : 0;
            }
            T a[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) a[u] = oc[u] ? W[g0 + u * nthr] : (T)0;
#pragma unroll
            for (int u = 0; u < kLd; ++u)
                if (g0 + u * nthr < M) buf[lds_pad(g0 + u * nthr)] = {a[u], (T)0};
        }
        __syncthreads();
        block_fft<T>(buf, 1, I, G);
        const T* sp = static_cast<const T*>(I.spec) + (int64_t)kern * half;
        for (int k0 = threadIdx.x; k0 < M; k0 += kLd * nthr) {
            T sv[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int k = k0 + u * nthr;
                const bool up = k > M - k;
                sv[u] = (k < M) ? gview<T>(sp)[up ? M - k : k] : (T)0;
                if (FORM == 2 && kern > 0 && up) sv[u] = -sv[u];   // times -i b, b odd in k
            }
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int k = k0 + u * nthr;
                if (k < M) {
                    const cplx<T> v = buf[lds_pad(k)];
                    if (FORM == 2 && kern > 0) buf[lds_pad(k)] = {v.y * sv[u], v.x * sv[u]};
                    else buf[lds_pad(k)] = {v.x * sv[u], -v.y * sv[u]};
                }
            }
        }
        __syncthreads();
        block_fft<T>(buf, 1, I, G);
        T* Vp = static_cast<T*>(I.V) + (int64_t)pot * n_cap;
        for (int g = threadIdx.x; g < n; g += blockDim.x) Vp[g] = buf[lds_pad(g)].x;
        __syncthreads();
    }
    VB_END
}

// ---------------------------------------------------------------- tables and kernel spectra

__device__ __forceinline__ double kern_val(int kern, double r2)
{
    const double a = 1.0 / (1.0 + r2);
    return kern == 0 ? a : a * a;
}

// Value of table kern on the lag grid (j0, j1) with r2 = h^2 (j0^2 + j1^2):
// K1 (0); K2 (1); for form V, table 1 is the odd kernel along dimension 0,
// z_0 K2 at the non-negative lag z_0 = h j0, and table 2 the one along
// dimension 1 (their signs are restored by the sine transforms).
__device__ __forceinline__ double ktab_val(int form, int kern, double h, int j0, int j1, double r2)
{
    if (kern == 0) return kern_val(0, r2);
    const double v = kern_val(1, r2);
    if (form != 2) return v;
    return h * (double)(kern == 1 ? j0 : j1) * v;
}

// The tables are rebuilt when the box kernel found a new node spacing or a
// new circulant length (every call under the paper policy; under a fixed
// width only when the ladder length changes).
__device__ __forceinline__ bool spec_needed(const Inst& I)
{
    return okay(I) && I.geom->spec_dirty != 0;
}

// Stage twiddle tables of one axis: stage s holds w^(r k M/(Ns R)) at
// tw_off[s] + k (R-1) + r - 1, w = exp(-2 pi i / M); idx < M - 1.
template <typename T>
__device__ __forceinline__ void stage_twiddle(int64_t idx, int M, int nstages, const int* radix,
                                              const int* tw_off, void* twv)
{
    int st = 0;
    while (st + 1 < nstages && tw_off[st + 1] <= idx) ++st;
    int ns = 1;
    for (int q = 0; q < st; ++q) ns *= radix[q];
    const int R = radix[st];
    const int e = (int)idx - tw_off[st];
    const int k = e / (R - 1), r = e - k * (R - 1) + 1;
    const int64_t ang = (int64_t)r * k * (M / (ns * R));
    double sv, cv;
    sincospi(2.0 * (double)ang / (double)M, &sv, &cv);
    static_cast<cplx<T>*>(twv)[idx] = {(T)cv, (T)(-sv)};
}

// Entry (j, k) of the weighted cosine matrix wt(j) cos(2 pi j k / M) (wt = 1
// at j = 0 and j = M/2, else 2: the circulant folds j and M - j), or of the
// sine matrix 2 sin(2 pi j k / M) (zero at j = 0, M/2), j, k <= M/2.
__device__ __forceinline__ void cs_entry(int M, int j, int k, double& c, double& sn)
{
    double sv, cv;
    sincospi(2.0 * (double)(((int64_t)j * k) % M) / (double)M, &sv, &cv);
    const bool edge = (j == 0 || 2 * j == M);
    c = (edge ? 1.0 : 2.0) * cv;
    sn = edge ? 0.0 : 2.0 * sv;
}

// Number of kernel tables: K1 and K2, or K1 and the s odd kernels (form V).
__device__ __forceinline__ int n_tables(const Inst& I) { return I.form == 2 ? I.s + 1 : 2; }

// Twiddles exp(-2 pi i k / M) of each axis (element type), the cos and sin
// tables (s = 1) or the weighted cosine and sine matrices of each axis
// (s = 2), and the kernel values on the lag grid j <= M/2 (double).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_spec0(LaunchMap map)
{
    VB_BEGIN_IF_SKIP(map, K_SPEC0, spec_needed(I))
    {
        const Geom& G = *I.geom;
        const int M = G.M, half = G.half;
        // the launch covers the capacity's tables: past this iteration's,
        // step over the rest of the instance's virtual blocks in one jump
        // (the loop variables of VB_BEGIN_IF_SKIP)
        const int64_t hyw = G.half_y;
        const int64_t work = (S == 2) ? std::max(std::max<int64_t>(std::max(M, G.My), (int64_t)half * half),
                                                 std::max(hyw * hyw, (int64_t)n_tables(I) * hyw * half))
                                      : std::max<int64_t>(M, 2 * (int64_t)half);
        if ((int64_t)lb * 256 >= work) {
            const int end = __pre[inst_id + 1];
            __vb += ((end - __vb + (int)gridDim.x - 1) / (int)gridDim.x - 1) * (int)gridDim.x;
            continue;
        }
        const int64_t idx = (int64_t)lb * 256 + threadIdx.x;
        const double h2 = G.h * G.h;
        if (idx < M - 1) stage_twiddle<T>(idx, M, G.nstages, G.radix, G.tw_off, I.tw);
        if (S == 2) {
            const int My = G.My, hy = G.half_y;
            const int64_t slot = (int64_t)I.half * I.half;
            const bool same = (My == M);       // the second axis reuses the first's tables
            if (!same && idx < My - 1) stage_twiddle<T>(idx, My, G.nstages_y, G.radix_y, G.tw_off_y, I.twy);
            // cosine (and form V sine) matrices: x at slots 0 and 2, y at 1 and 3
            if (idx < (int64_t)half * half) {
                const int j = (int)(idx / half), k = (int)(idx - (int64_t)j * half);
                double c, sn;
                cs_entry(M, j, k, c, sn);
                I.ccos[idx] = c;
                if (I.form == 2) I.ccos[2 * slot + idx] = sn;
            }
            if (!same && idx < (int64_t)hy * hy) {
                const int j = (int)(idx / hy), k = (int)(idx - (int64_t)j * hy);
                double c, sn;
                cs_entry(My, j, k, c, sn);
                I.ccos[slot + idx] = c;
                if (I.form == 2) I.ccos[3 * slot + idx] = sn;
            }
            // kernel tables [kern][j1 < half_y][j0 < half]
            const int64_t per = (int64_t)hy * half;
            if (idx < n_tables(I) * per) {
                const int kern = (int)(idx / per);
                const int rem = (int)(idx - (int64_t)kern * per);
                const int j1 = rem / half, j0 = rem - j1 * half;
                I.ktab[kern * slot + rem] =
                    ktab_val(I.form, kern, G.h, j0, j1, h2 * ((double)j1 * j1 + (double)j0 * j0));
            }
        } else {
            if (idx < M) {
                double sv, cv;
                sincospi(2.0 * (double)idx / (double)M, &sv, &cv);
                I.costab[idx] = cv;
                I.costab[I.M + idx] = sv;
            }
            if (idx < 2 * half) {
                const int kern = (int)(idx / half), j = (int)(idx - (int64_t)kern * half);
                I.ktab[idx] = ktab_val(I.form, kern, G.h, j, 0, h2 * (double)j * j);
            }
        }
    }
    VB_END
}

// Weighted cosine matrix C[j][k] = wt(j) cos(2 pi j k / M), j, k <= M/2,
// wt = 1 at j = 0 and j = M/2, else 2 (the circulant folds j and M - j), so
// that for an even sequence c the DFT is sum_j C[j][k] c[j].
__device__ __forceinline__ double cos_w(const double* ct, int M, int j, int k)
{
    const double wt = (j == 0 || 2 * j == M) ? 1.0 : 2.0;
    return wt * ct[(int)(((int64_t)j * k) % M)];
}

// Sine counterpart for an odd sequence s (s[M - j] = -s[j]): the DFT is
// -i sum_j S[j][k] s[j] with S[j][k] = 2 sin(2 pi j k / M), zero at j = 0, M/2.
__device__ __forceinline__ double sin_w(const double* st, int M, int j, int k)
{
    if (j == 0 || 2 * j == M) return 0.0;
    return 2.0 * st[(int)(((int64_t)j * k) % M)];
}

// One 64 x 64 tile of out = op(A) B, op(A) [m x k] and B [k x n] row-major
// double matrices with leading dimensions lda and ldb (op(A) = A, or the
// transpose of a [k x m] A), k staged through LDS 16 at a time; 256 threads,
// 4 x 4 outputs each.  emit(m, n, value) stores a result.
template <bool TA, typename Emit>
__device__ __forceinline__ void gemm_tile(const double* __restrict__ A, int lda,
                                          const double* __restrict__ B, int ldb,
                                          int mdim, int kdim, int ndim, int tm, int tn,
                                          double (*As)[65], double (*Bs)[65], Emit emit)
{
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < kdim; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            int kk, mm;
            if (TA) { kk = e >> 6; mm = e & 63; } else { kk = e & 15; mm = e >> 4; }
            const int m = tm * 64 + mm, k = k0 + kk;
            As[kk][mm] = (m < mdim && k < kdim) ? (TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k])
                                                : 0.0;
            const int nk = e >> 6, nn = e & 63;
            const int n = tn * 64 + nn, k2 = k0 + nk;
            Bs[nk][nn] = (n < ndim && k2 < kdim) ? B[(int64_t)k2 * ldb + n] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = tm * 64 + ty * 4 + i, n = tn * 64 + tx * 4 + j;
            if (m < mdim && n < ndim) emit(m, n, acc[i][j]);
        }
}

// First pass.  s = 2: A[kern] = K[kern] Cx, the transform along dimension 0
// of the kernel grid (K[kern] is [half_y][half_x]; the sine matrix in place
// of Cx for the odd kernel along dimension 0), by tiled GEMM; s = 1: the
// whole spectrum K^[kern][k] = sum_j C[j][k] K[kern][j] / M (sine sums for
// form V's odd kernel).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_spec1(LaunchMap map)
{
    __shared__ double As[16][65], Bs[16][65];
    VB_BEGIN_IF_SKIP(map, K_SPEC1, spec_needed(I))
    {
        const Geom& G = *I.geom;
        const int M = G.M, half = G.half;
        if (S == 2) {
            // tiles of this iteration's [half_y x half] products (the launch
            // covers the capacity's; the rest exit at once)
            const int ntm = (G.half_y + 63) / 64, ntn = (half + 63) / 64;
            const int kern = lb / (ntm * ntn), rem = lb - kern * ntm * ntn;
            const int tm = rem / ntn, tn = rem - tm * ntn;
            const int64_t slot = (int64_t)I.half * I.half;
            if (kern < n_tables(I)) {
                double* out = I.spec_tmp + kern * slot;
                const double* bx = I.ccos + ((I.form == 2 && kern == 1) ? 2 * slot : 0);
                gemm_tile<false>(I.ktab + kern * slot, half, bx, half, G.half_y, half, half, tm, tn, As, Bs,
                                 [&](int m, int n, double v) { out[(int64_t)m * half + n] = v; });
            }
        } else {
            const int idx = lb * 256 + threadIdx.x;
            if (idx < 2 * half) {
                const int kern = idx / half, k = idx - kern * half;
                const double* kt = I.ktab + (int64_t)kern * half;
                double acc = 0.0;
                if (I.form == 2 && kern == 1)
                    for (int j = 0; j < half; ++j) acc += sin_w(I.costab + I.M, M, j, k) * kt[j];
                else
                    for (int j = 0; j < half; ++j) acc += cos_w(I.costab, M, j, k) * kt[j];
                static_cast<T*>(I.spec)[idx] = (T)(acc / M);
            }
        }
    }
    VB_END
}

// Second pass (s = 2): K^[kern] = A[kern]^T Cy / (M My), the transform along
// dimension 1 (the sine matrix of y for form V's odd kernel along dimension
// 1), stored [kern][k0 < half_x][k1 < half_y] in the element type.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_spec2(LaunchMap map)
{
    __shared__ double As[16][65], Bs[16][65];
    VB_BEGIN_IF_SKIP(map, K_SPEC2, S == 2 && spec_needed(I))
    {
        const Geom& G = *I.geom;
        const int M = G.M, half = G.half, hy = G.half_y;
        const int ntm = (half + 63) / 64, ntn = (hy + 63) / 64;   // this iteration's tiles
        const int kern = lb / (ntm * ntn), rem = lb - kern * ntm * ntn;
        const int tm = rem / ntn, tn = rem - tm * ntn;
        const int64_t slot = (int64_t)I.half * I.half;
        if (kern < n_tables(I)) {
            T* out = static_cast<T*>(I.spec) + kern * slot;
            // the second axis' matrices; the first axis' when the lengths agree
            const int64_t ys = (G.My == M) ? 0 : slot;
            const double* by = I.ccos + ((I.form == 2 && kern == 2) ? 2 * slot + ys : ys);
            const double sc = 1.0 / ((double)M * (double)G.My);
            gemm_tile<true>(I.spec_tmp + kern * slot, half, by, hy, half, hy, hy, tm, tn, As, Bs,
                            [&](int m, int n, double v) { out[(int64_t)m * hy + n] = (T)(v * sc); });
        }
    }
    VB_END
}

// ---------------------------------------------------------------- dispatch

// ---------------------------------------------------------------- 3-D convolution (s = 3)

// Step 2 for s = 3 (Section 2, the s + 2 sums for any s; Section 2.4's
// circulant embedding along each axis): the M^3 circulant product by three
// passes of complex transforms over a complex grid per charge, the kernel
// spectrum, and three passes back, each pass over kSeq3 sequences per block
// (consecutive x, so a block's loads along y and z read kSeq3 consecutive
// elements).  Grids are [grid][z][y][x] with this iteration's M per axis.
// The inverse passes are forward transforms of the conjugate (the product's
// conjugate is stored after the z pass); the real part of the last pass is the
// potential, the spectrum being stored pre-scaled by 1/M^3.
//   F3_X   charges:    rows (z, y < n) of W (x < n, rest zero) -> Xg rows
//   F3_Y   charges:    y sequences, all of them (y >= n and z >= n read as
//                      zero, so the z pass finds the zero padding in place)
//   F3_Z   potentials: z sequences of the charge's Xg, times the kernel
//                      spectrum, conjugated, transformed again; z < n kept in Xp
//   F3_IY  potentials: y sequences of Xp for z < n; y < n kept
//   F3_IX  potentials: x rows of Xp for z, y < n; the real part of x < n to V
//   S3_X/Y/Z          the same plain passes over the FP64 kernel grids
enum { F3_X = 0, F3_Y, F3_Z, F3_IY, F3_IX, S3_X, S3_Y, S3_Z };

constexpr int kSeq3 = 16;           // sequences per block of a 3-D pass

template <int MODE> struct F3Kind;
template <> struct F3Kind<F3_X> { static constexpr int K = K_F3_X, AXIS = 0; };
template <> struct F3Kind<F3_Y> { static constexpr int K = K_F3_Y, AXIS = 1; };
template <> struct F3Kind<F3_Z> { static constexpr int K = K_F3_Z, AXIS = 2; };
template <> struct F3Kind<F3_IY> { static constexpr int K = K_F3_IY, AXIS = 1; };
template <> struct F3Kind<F3_IX> { static constexpr int K = K_F3_IX, AXIS = 0; };
template <> struct F3Kind<S3_X> { static constexpr int K = K_S3_X, AXIS = 0; };
template <> struct F3Kind<S3_Y> { static constexpr int K = K_S3_Y, AXIS = 1; };
template <> struct F3Kind<S3_Z> { static constexpr int K = K_S3_Z, AXIS = 2; };

// Kernel value of table kern (0: K1, 1: K2) at squared distance r2.
__device__ __forceinline__ double kern3(int kern, double r2)
{
    const double a = 1.0 / (1.0 + r2);
    return kern == 0 ? a : a * a;
}

// Signed lag of circulant index j: j for j <= M/2, j - M above.
__device__ __forceinline__ int lag3(int j, int M) { return (2 * j <= M) ? j : j - M; }

// One pass of the 3-D convolution (T: the element type of the pass).
// FP32: at most 128 registers (four waves per SIMD); FP64 kernels take two.
template <typename T> constexpr int kF3Waves = (sizeof(T) == 4) ? 4 : 2;

template <typename T, int FORM, int MODE>
__global__ __launch_bounds__(kSeq3 * 32) __attribute__((amdgpu_waves_per_eu(kF3Waves<T>))) void k_f3(LaunchMap map)
{
    constexpr int AXIS = F3Kind<MODE>::AXIS;
    constexpr bool SPEC = MODE >= S3_X;
    extern __shared__ __align__(16) char smem[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
    VB_BEGIN_IF_SKIP(map, F3Kind<MODE>::K, (SPEC ? spec_needed(I) : okay(I)))
    {
        const Geom& G = *I.geom;
        const int M = G.M, n = G.n, n_cap = I.n_cap, PM = lds_stride(M);
        const int64_t M2 = (int64_t)M * M, M3 = M2 * M;
        const int nthr = blockDim.x;
        const int ngrid = SPEC ? 2 : (MODE == F3_X || MODE == F3_Y) ? I.nc : I.np;
        const int bpg = (int)(M2 / kSeq3);                 // blocks per grid (16 divides M^2)
        const int g = lb / bpg, j0 = (lb - g * bpg) * kSeq3;
        if (g < ngrid) {
            int ch = g, kern = 0;
            if (MODE == F3_Z) {
                // potential g: its charge and kernel (forms A and B)
                if (g == 0) { ch = (FORM == 0) ? 0 : 4; kern = (FORM == 0) ? 0 : 1; }
                else if (g == 1) { ch = 0; kern = 1; }
                else { ch = g - 1; kern = 1; }
            }
            // sequence j (0 <= j < M^2) of the pass: its two fixed indices
            // (a, b) = (z, y) for x rows, (z, x) for y, (y, x) for z; base
            // offset and element stride in the grid
            auto seq = [&](int j, int& a, int& b, int64_t& base, int64_t& stride) {
                a = j / M;
                b = j - a * M;
                if (AXIS == 0) { base = (int64_t)a * M2 + (int64_t)b * M; stride = 1; }
                else if (AXIS == 1) { base = (int64_t)a * M2 + b; stride = M; }
                else { base = (int64_t)a * M + b; stride = M2; }
            };
            // is sequence j wanted at all / read as all zero
            auto wanted = [&](int a, int b) -> bool {
                if (MODE == F3_X || MODE == F3_IX) return a < n && b < n;
                if (MODE == F3_IY) return a < n;
                return true;
            };
            bool any = false;
            for (int q = 0; q < kSeq3; ++q) {
                int a, b;
                int64_t base, stride;
                seq(j0 + q, a, b, base, stride);
                any = any || wanted(a, b);
            }
            if (any) {
                typedef cplx<T> C;
                const C* src;
                C* dst;
                if (SPEC) {
                    src = static_cast<const C*>(I.specd) + (int64_t)g * M3;
                    dst = static_cast<C*>(I.specd) + (int64_t)g * M3;
                } else if (MODE == F3_X) {
                    src = nullptr;
                    dst = static_cast<C*>(I.X) + (int64_t)g * M3;
                } else if (MODE == F3_Y) {
                    src = static_cast<const C*>(I.X) + (int64_t)g * M3;
                    dst = static_cast<C*>(I.X) + (int64_t)g * M3;
                } else if (MODE == F3_Z) {
                    src = static_cast<const C*>(I.X) + (int64_t)ch * M3;
                    dst = static_cast<C*>(I.Xc) + (int64_t)g * M3;
                } else {
                    src = static_cast<const C*>(I.Xc) + (int64_t)g * M3;
                    dst = static_cast<C*>(I.Xc) + (int64_t)g * M3;
                }
                const T* W = static_cast<const T*>(I.W) + (int64_t)g * n_cap * n_cap * n_cap;
                // load: x rows element-major (consecutive threads along a row),
                // y and z sequences sequence-major (consecutive x)
                for (int idx = threadIdx.x; idx < kSeq3 * M; idx += nthr) {
                    const int q = (AXIS == 0) ? idx / M : idx % kSeq3;
                    const int r = (AXIS == 0) ? idx - q * M : idx / kSeq3;
                    int a, b;
                    int64_t base, stride;
                    seq(j0 + q, a, b, base, stride);
                    C v = {(T)0, (T)0};
                    if (MODE == F3_X) {
                        if (a < n && b < n && r < n)
                            v.x = W[((int64_t)a * n_cap + b) * n_cap + r];
                    } else if (MODE == F3_Y) {
                        if (a < n && r < n) v = src[base + (int64_t)r * stride];
                    } else if (wanted(a, b)) {
                        v = src[base + (int64_t)r * stride];
                    }
                    buf[__mul24(q, PM) + lds_pad(r)] = v;
                }
                __syncthreads();
                const C* tw = SPEC ? static_cast<const C*>(I.twd) : static_cast<const C*>(I.tw);
                block_fft_tw<T>(buf, kSeq3, M, G.nstages, G.radix, G.tw_off, tw);
                if (MODE == F3_Z) {
                    // times the real kernel spectrum, conjugated; then the
                    // transform of the conjugate (the inverse along z)
                    const T* sp = static_cast<const T*>(I.spec) + (int64_t)kern * M3;
                    for (int idx = threadIdx.x; idx < kSeq3 * M; idx += nthr) {
                        const int q = idx % kSeq3, r = idx / kSeq3;
                        int a, b;
                        int64_t base, stride;
                        seq(j0 + q, a, b, base, stride);
                        const T sv = sp[base + (int64_t)r * stride];
                        const C v = buf[__mul24(q, PM) + lds_pad(r)];
                        buf[__mul24(q, PM) + lds_pad(r)] = {v.x * sv, -v.y * sv};
                    }
                    __syncthreads();
                    block_fft_tw<T>(buf, kSeq3, M, G.nstages, G.radix, G.tw_off, tw);
                }
                // store
                for (int idx = threadIdx.x; idx < kSeq3 * M; idx += nthr) {
                    const int q = (AXIS == 0) ? idx / M : idx % kSeq3;
                    const int r = (AXIS == 0) ? idx - q * M : idx / kSeq3;
                    int a, b;
                    int64_t base, stride;
                    seq(j0 + q, a, b, base, stride);
                    const C v = buf[__mul24(q, PM) + lds_pad(r)];
                    if (MODE == F3_IX) {
                        if (a < n && b < n && r < n)
                            static_cast<T*>(I.V)[(((int64_t)g * n_cap + a) * n_cap + b) * n_cap + r] = v.x;
                    } else if (MODE == F3_Z || MODE == F3_IY) {
                        if (r < n && wanted(a, b)) dst[base + (int64_t)r * stride] = v;
                    } else if (wanted(a, b)) {
                        dst[base + (int64_t)r * stride] = v;
                    }
                }
                __syncthreads();
            }
        }
    }
    VB_END
}

// Kernel grids for the spectra (FP64, when the spacing or M changed): the
// circulant samples K(h lag) of K1 and K2 at every (z, y, x) of M^3, and the
// stage twiddles of M in double and in the element type.
template <typename T>
__global__ __launch_bounds__(256) void k_s3_fill(LaunchMap map)
{
    VB_BEGIN_IF_SKIP(map, K_S3_FILL, spec_needed(I))
    {
        const Geom& G = *I.geom;
        const int M = G.M;
        const int64_t M2 = (int64_t)M * M, M3 = M2 * M;
        const int64_t idx = (int64_t)lb * 256 + threadIdx.x;
        if (idx < M - 1) {
            stage_twiddle<double>(idx, M, G.nstages, G.radix, G.tw_off, I.twd);
            stage_twiddle<T>(idx, M, G.nstages, G.radix, G.tw_off, I.tw);
        }
        if (idx < 2 * M3) {
            const int kern = (int)(idx / M3);
            const int64_t e = idx - kern * M3;
            const int z = (int)(e / M2), y = (int)((e - (int64_t)z * M2) / M), x = (int)(e % M);
            const double lx = lag3(x, M), ly = lag3(y, M), lz = lag3(z, M);
            const double r2 = G.h * G.h * (lx * lx + ly * ly + lz * lz);
            static_cast<cplx<double>*>(I.specd)[idx] = {kern3(kern, r2), 0.0};
        }
    }
    VB_END
}

// The spectra: real parts of the transformed kernel grids, scaled by 1/M^3,
// in the element type.
template <typename T>
__global__ __launch_bounds__(256) void k_s3_store(LaunchMap map)
{
    VB_BEGIN_IF_SKIP(map, K_S3_STORE, spec_needed(I))
    {
        const Geom& G = *I.geom;
        const int64_t M3 = (int64_t)G.M * G.M * G.M;
        const int64_t idx = (int64_t)lb * 256 + threadIdx.x;
        if (idx < 2 * M3)
            static_cast<T*>(I.spec)[idx] = (T)(static_cast<const cplx<double>*>(I.specd)[idx].x / (double)M3);
    }
    VB_END
}

// Allow up to the full 160 KB of LDS for a kernel's dynamic allocation.
template <typename K>
static void allow_lds(K kernel, size_t lds)
{
    if (lds > 48 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T, int S, int P, int FORM>
static hipError_t fft_go(int kind, const LaunchMap& map, const Launch& l, hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_FFT_ROWS:
        if (S == 2) {
            allow_lds(k_fft_rows<T, P>, l.lds);
            hipLaunchKernelGGL((k_fft_rows<T, P>), g, b, l.lds, st, map);
        }
        break;
    case K_FFT_COLS:
        if (S == 2) {
            allow_lds(k_fft_cols<T, S, FORM>, l.lds);
            hipLaunchKernelGGL((k_fft_cols<T, S, FORM>), g, b, l.lds, st, map);
        }
        break;
    case K_FFT_IROWS:
        if (S == 2) {
            constexpr int NP = Pots<S, FORM>::NP;
            allow_lds(k_fft_irows<T, S, NP>, l.lds);
            hipLaunchKernelGGL((k_fft_irows<T, S, NP>), g, b, l.lds, st, map);
        }
        break;
    case K_FFT_1D:
        if (S == 1) {
            allow_lds(k_fft_1d<T, P, FORM>, l.lds);
            hipLaunchKernelGGL((k_fft_1d<T, P, FORM>), g, b, l.lds, st, map);
        }
        break;
    case K_SPEC0: hipLaunchKernelGGL((k_spec0<T, S>), g, b, 0, st, map); break;
    case K_SPEC1: hipLaunchKernelGGL((k_spec1<T, S>), g, b, 0, st, map); break;
    case K_SPEC2: hipLaunchKernelGGL((k_spec2<T, S>), g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int S, int P>
static hipError_t fft_form(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    switch (c.form) {
    case 0: return fft_go<T, S, P, 0>(kind, m, l, st);
    case 1: return fft_go<T, S, P, 1>(kind, m, l, st);
    case 2: return fft_go<T, S, P, 2>(kind, m, l, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int S>
static hipError_t fft_p(int kind, const Cfg& c, const LaunchMap& m, const Launch& l, hipStream_t st)
{
    switch (c.p) {
    case 2: return fft_form<T, S, 2>(kind, c, m, l, st);
    case 3: return fft_form<T, S, 3>(kind, c, m, l, st);
    case 4: return fft_form<T, S, 4>(kind, c, m, l, st);
    case 5: return fft_form<T, S, 5>(kind, c, m, l, st);
    case 6: return fft_form<T, S, 6>(kind, c, m, l, st);
    default: return hipErrorInvalidValue;
    }
}

// s = 3 kinds: the convolution passes in the element type, the spectrum
// passes in double.
template <typename T, int FORM>
static hipError_t f3_go(int kind, const LaunchMap& map, const Launch& l, hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_F3_X: allow_lds(k_f3<T, FORM, F3_X>, l.lds); hipLaunchKernelGGL((k_f3<T, FORM, F3_X>), g, b, l.lds, st, map); break;
    case K_F3_Y: allow_lds(k_f3<T, FORM, F3_Y>, l.lds); hipLaunchKernelGGL((k_f3<T, FORM, F3_Y>), g, b, l.lds, st, map); break;
    case K_F3_Z: allow_lds(k_f3<T, FORM, F3_Z>, l.lds); hipLaunchKernelGGL((k_f3<T, FORM, F3_Z>), g, b, l.lds, st, map); break;
    case K_F3_IY: allow_lds(k_f3<T, FORM, F3_IY>, l.lds); hipLaunchKernelGGL((k_f3<T, FORM, F3_IY>), g, b, l.lds, st, map); break;
    case K_F3_IX: allow_lds(k_f3<T, FORM, F3_IX>, l.lds); hipLaunchKernelGGL((k_f3<T, FORM, F3_IX>), g, b, l.lds, st, map); break;
    case K_S3_X: allow_lds(k_f3<double, 0, S3_X>, l.lds); hipLaunchKernelGGL((k_f3<double, 0, S3_X>), g, b, l.lds, st, map); break;
    case K_S3_Y: allow_lds(k_f3<double, 0, S3_Y>, l.lds); hipLaunchKernelGGL((k_f3<double, 0, S3_Y>), g, b, l.lds, st, map); break;
    case K_S3_Z: allow_lds(k_f3<double, 0, S3_Z>, l.lds); hipLaunchKernelGGL((k_f3<double, 0, S3_Z>), g, b, l.lds, st, map); break;
    case K_S3_FILL: hipLaunchKernelGGL((k_s3_fill<T>), g, b, 0, st, map); break;
    case K_S3_STORE: hipLaunchKernelGGL((k_s3_store<T>), g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                           hipStream_t st)
{
    if (c.s == 3) {
        if (c.dtype == 0) return c.form == 0 ? f3_go<float, 0>(kind, map, l, st) : f3_go<float, 1>(kind, map, l, st);
        return c.form == 0 ? f3_go<double, 0>(kind, map, l, st) : f3_go<double, 1>(kind, map, l, st);
    }
    if (c.dtype == 0)
        return c.s == 1 ? fft_p<float, 1>(kind, c, map, l, st) : fft_p<float, 2>(kind, c, map, l, st);
    return c.s == 1 ? fft_p<double, 1>(kind, c, map, l, st) : fft_p<double, 2>(kind, c, map, l, st);
}

}  // namespace tsne
