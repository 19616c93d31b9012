// Sparse-P kernels on gfx950: the attraction of Section 3 (CSR rows, with
// optional XCD-aware column slabs, or row blocks sweeping LDS column windows)
// and the Kullback-Leibler divergence of Section 1.1.
//
// Every kernel walks the virtual blocks of its kind over all instances of the
// launch (VB_BEGIN/VB_END), so one launch serves a single plan or a batch.
#include "k_common.h"

namespace tsne {

// ---------------------------------------------------------------- attraction

template <typename T, int S> struct Vec;
template <> struct Vec<float, 1> { typedef float t; };
template <> struct Vec<float, 2> { typedef float2 t; };
template <> struct Vec<double, 1> { typedef double t; };
template <> struct Vec<double, 2> { typedef double2 t; };

template <typename V> __device__ __forceinline__ double cx(const V& v) { return (double)v.x; }
template <> __device__ __forceinline__ double cx<float>(const float& v) { return (double)v; }
template <> __device__ __forceinline__ double cx<double>(const double& v) { return v; }

// 1 / x: the hardware reciprocal (1 ulp) for float, IEEE division for double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// F_attr,i = sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2) over row i of the CSR
// P (Section 3).  LPR lanes per row; each lane takes U non-zeros per round and
// issues all their loads (column, value, then the neighbours' positions as one
// vector load each) before using them, so LPR * U should cover a typical row.
// Each lane sums its few terms in the element type; the row's lanes are
// reduced in double.  Optionally the columns are split into slabs (virtual
// blocks run slab-major, each row's slab range from the split table) and each
// slab writes a partial force.  PK: the (column, value) pairs come packed in
// one 8-byte array (FP32), loaded two at a time.  KL: the same pass computes
// the Kullback-Leibler sums of Section 1.1 instead, sum p log(p (1 + d^2))
// and sum p over the edges of all the block's virtual blocks (log in the
// element type, FP64 sums), left as the block's two partials for k_klsum.
template <typename T, int S, int LPR, int U, bool GATED, bool PK, bool KL = false>
__global__ __launch_bounds__(256) void k_attr(LaunchMap map)
{
    constexpr int RPB = 256 / LPR;
    typedef typename Vec<T, S>::t V;
    __shared__ double klsh[8];
    double kla = 0.0, klp = 0.0;
    double* klout = nullptr;
    VB_BEGIN_IF(map, GATED ? K_ATTR : K_ATTR_ALL, (!GATED || live(I)))
    {
        if (KL) klout = I.kl_part;
        // one edge's contribution: the force term, or the divergence terms
        auto edge = [&](T pk, T d0, T d1, T& a0, T& a1) {
            const T q = (T)1 + d0 * d0 + d1 * d1;
            if constexpr (KL) {
                if (pk > (T)0) {
                    kla += (double)pk * (double)log(pk * q);
                    klp += (double)pk;
                }
            } else {
                const T wgt = pk * recip(q);
                a0 += wgt * d0;
                if (S == 2) a1 += wgt * d1;
            }
        };
        const int64_t n = I.n;
        const int nrb = (int)((n + RPB - 1) / RPB);
        // XCD-aware slab assignment: workgroups go to the 8 XCDs round-robin
        // (block b -> XCD b mod 8, and launches keep virtual block = b mod 8),
        // so virtual block v works on slab (v mod 8) / (8 / slabs): each XCD's
        // L2 then only holds the positions of its own slab.
        int slab = 0, rb = lb;
        if (I.slabs > 1) {
            const int per = 8 / I.slabs;
            const int x = lb & 7, q = lb >> 3;
            slab = x / per;
            rb = q * per + (x - slab * per);
        }
        const int i = rb * RPB + (int)threadIdx.x / LPR;
        const int sub = (int)threadIdx.x % LPR;
        T a0 = (T)0, a1 = (T)0;
        const V* Y = static_cast<const V*>(I.Yin);
        if (i < n && rb < nrb) {
            const T* val = static_cast<const T*>(I.val);
            const int32_t* col = I.col;
            const V yi = Y[i];
            T yi0, yi1 = (T)0;
            if constexpr (S == 2) { yi0 = yi.x; yi1 = yi.y; } else { yi0 = yi; }
            const int64_t b = (slab == 0) ? I.row_ptr[i] : (int64_t)I.split[(int64_t)(slab - 1) * n + i];
            const int64_t e = (slab == I.slabs - 1) ? I.row_ptr[i + 1]
                                                     : (int64_t)I.split[(int64_t)slab * n + i];
            if constexpr (PK) {
                // two (column, value) pairs per 16-byte load: lane `sub` takes
                // the aligned pair couples q0 + v LPR, each covering entries
                // 2q and 2q + 1 (entries outside [b, e) are masked)
                constexpr int UH = (U + 1) / 2;
                const uint4* cv4 = static_cast<const uint4*>(I.cv);
                for (int64_t q0 = (b >> 1) + sub; 2 * q0 < e; q0 += (int64_t)LPR * UH) {
                    int jj[2 * UH];
                    T pp[2 * UH];
#pragma unroll
                    for (int v = 0; v < UH; ++v) {
                        const int64_t q = q0 + (int64_t)v * LPR;
                        const bool any = 2 * q < e;
                        const uint4 w = any ? cv4[q] : make_uint4((unsigned)i, 0u, (unsigned)i, 0u);
                        const bool ok0 = any && 2 * q >= b, ok1 = 2 * q + 1 < e;
                        jj[2 * v] = ok0 ? (int)w.x : i;
                        pp[2 * v] = ok0 ? (T)__uint_as_float(w.y) : (T)0;
                        jj[2 * v + 1] = ok1 ? (int)w.z : i;
                        pp[2 * v + 1] = ok1 ? (T)__uint_as_float(w.w) : (T)0;
                    }
                    V yj[2 * UH];
#pragma unroll
                    for (int u = 0; u < 2 * UH; ++u) yj[u] = Y[jj[u]];
#pragma unroll
                    for (int u = 0; u < 2 * UH; ++u) {
                        T d0, d1 = (T)0;
                        if constexpr (S == 2) { d0 = yi0 - yj[u].x; d1 = yi1 - yj[u].y; }
                        else { d0 = yi0 - yj[u]; }
                        edge(pp[u], d0, d1, a0, a1);
                    }
                }
            } else {
            for (int64_t k0 = b + sub; k0 < e; k0 += (int64_t)LPR * U) {
                int jj[U];
                T pp[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t k = k0 + (int64_t)u * LPR;
                    const bool ok = k < e;
                    jj[u] = ok ? col[k] : i;
                    pp[u] = ok ? val[k] : (T)0;
                }
                V yj[U];
#pragma unroll
                for (int u = 0; u < U; ++u) yj[u] = Y[jj[u]];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T d0, d1 = (T)0;
                    if constexpr (S == 2) { d0 = yi0 - yj[u].x; d1 = yi1 - yj[u].y; }
                    else { d0 = yi0 - yj[u]; }
                    edge(pp[u], d0, d1, a0, a1);
                }
            }
            }
        }
        if constexpr (KL) continue;
        double f0 = (double)a0, f1 = (double)a1;
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) {
            f0 += __shfl_xor(f0, o, 64);
            if (S == 2) f1 += __shfl_xor(f1, o, 64);
        }
        if (i < n && rb < nrb && sub == 0) {
            T* F = (I.slabs == 1) ? static_cast<T*>(I.Fattr)
                                  : static_cast<T*>(I.Fap) + (int64_t)slab * n * S;
            F[(int64_t)i * S] = (T)f0;
            if (S == 2) F[(int64_t)i * S + 1] = (T)f1;
        }
    }
    VB_END
    if constexpr (KL) {
        // a single-instance launch: the block's partials (klout is this
        // instance's array once the block has run a virtual block)
        kla = block_sum_d(kla, klsh);
        klp = block_sum_d(klp, klsh);
        if (threadIdx.x == 0 && klout) {
            klout[2 * blockIdx.x] = kla;
            klout[2 * blockIdx.x + 1] = klp;
        }
    }
}

// The attraction and the divergence terms for s = 3 over CSR rows (Section 3;
// Section 1.1 for the divergence): LPR lanes per row, each taking U
// non-zeros per round with all their loads issued first (column and value
// from the bound CSR, the neighbours' three coordinates); the row's lanes are
// reduced in double.  One slab (the whole row).
template <typename T, int LPR, int U, bool GATED, bool KL = false>
__global__ __launch_bounds__(256) void k_attr3(LaunchMap map)
{
    constexpr int RPB = 256 / LPR;
    __shared__ double klsh[8];
    double kla = 0.0, klp = 0.0;
    double* klout = nullptr;
    VB_BEGIN_IF(map, GATED ? K_ATTR : K_ATTR_ALL, (!GATED || live(I)))
    {
        if (KL) klout = I.kl_part;
        const int64_t n = I.n;
        const int i = lb * RPB + (int)threadIdx.x / LPR;
        const int sub = (int)threadIdx.x % LPR;
        T a[3] = {(T)0, (T)0, (T)0};
        const T* Y = static_cast<const T*>(I.Yin);
        if (i < n) {
            const T* val = static_cast<const T*>(I.val);
            const int32_t* col = I.col;
            const Pt<T, 3> yi = Pt<T, 3>::load(Y, i);
            const int64_t b = I.row_ptr[i], e = I.row_ptr[i + 1];
            for (int64_t k0 = b + sub; k0 < e; k0 += (int64_t)LPR * U) {
                int jj[U];
                T pp[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t k = k0 + (int64_t)u * LPR;
                    const bool ok = k < e;
                    jj[u] = ok ? col[k] : i;
                    pp[u] = ok ? val[k] : (T)0;
                }
                Pt<T, 3> yj[U];
#pragma unroll
                for (int u = 0; u < U; ++u) yj[u] = Pt<T, 3>::load(Y, jj[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T d[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) d[q] = yi.v[q] - yj[u].v[q];
                    const T qv = (T)1 + d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if constexpr (KL) {
                        if (pp[u] > (T)0) {
                            kla += (double)pp[u] * (double)log(pp[u] * qv);
                            klp += (double)pp[u];
                        }
                    } else {
                        const T wgt = pp[u] * recip(qv);
#pragma unroll
                        for (int q = 0; q < 3; ++q) a[q] += wgt * d[q];
                    }
                }
            }
        }
        if constexpr (KL) continue;
        double f[3] = {(double)a[0], (double)a[1], (double)a[2]};
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1)
#pragma unroll
            for (int q = 0; q < 3; ++q) f[q] += __shfl_xor(f[q], o, 64);
        if (i < n && sub == 0) {
            T* F = static_cast<T*>(I.Fattr);
#pragma unroll
            for (int q = 0; q < 3; ++q) F[(int64_t)i * 3 + q] = (T)f[q];
        }
    }
    VB_END
    if constexpr (KL) {
        kla = block_sum_d(kla, klsh);
        klp = block_sum_d(klp, klsh);
        if (threadIdx.x == 0 && klout) {
            klout[2 * blockIdx.x] = kla;
            klout[2 * blockIdx.x + 1] = klp;
        }
    }
}

// Barrier for hand-offs through LDS only: each wave waits for its own LDS
// accesses, not for its global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One point of an [n][S] array through the global view, as one vector load
// (a native vector type: the HIP vector structs cannot be copied out of a
// qualified address space).
template <typename T, int S> struct NativeVec { typedef T t; };
template <> struct NativeVec<float, 2> { typedef float t __attribute__((ext_vector_type(2))); };
template <> struct NativeVec<double, 2> { typedef double t __attribute__((ext_vector_type(2))); };
template <typename T, int S>
__device__ __forceinline__ typename Vec<T, S>::t gpoint(const void* base, int64_t i)
{
    typedef typename NativeVec<T, S>::t N;
    const N q = gview<N>(base)[i];
    if constexpr (S == 2) {
        typename Vec<T, S>::t v;
        v.x = q.x;
        v.y = q.y;
        return v;
    } else {
        return q;
    }
}

// Attraction by row blocks (the sum over the non-zeros of P of Section 3,
// arranged for LDS): each virtual block takes tile_bi rows, keeps their
// positions and force sums in LDS and sweeps the column windows (tile_bj
// points, 32 KB) that hold its non-zeros, in the sweep steps fixed at bind
// time (one step: at most tile_step_edges non-zeros of one window, rows
// increasing).  Windows are double-buffered in LDS: step t takes its
// non-zeros against buffer t mod 2 and stores window t + 1 (requested a step
// earlier) into the other buffer, while window t + 2 and the non-zeros of
// step t + 1 are in flight; one LDS-only barrier per step.  Every neighbour position is thus an LDS read instead of
// a random L2 gather, the cost that bounds the CSR rows on a graph with no
// locality.  Row sums are 64-bit fixed point (scale tscale, a power of two
// chosen at bind time so that no row sum can overflow) added with LDS integer
// atomics: integer addition commutes, so the result has the same bits in
// whatever order the atomics land.  All loads are unconditional, at clamped
// addresses (slots past a step's non-zeros carry weight zero), so the
// compiler's wait counts leave the prefetches outstanding.  KL: the same
// sweep computes the Kullback-Leibler sums of Section 1.1 instead (as the CSR
// kernel's divergence mode: FP64 per-thread sums, one pair of partials per
// block for k_klsum), with no force sums.
template <typename T, int S, bool GATED, bool KL = false>
__global__ __launch_bounds__(1024) void k_attr_tile(LaunchMap map)
{
    typedef typename Vec<T, S>::t V;
    constexpr int NT = 1024;
    constexpr int WQ = kTileWindowBytes / (S * (int)sizeof(T)) / NT;     // window points per thread
    constexpr int UE = tile_step_edges(WQ * NT) / NT;                   // non-zeros per thread and step
    extern __shared__ __align__(16) char smem[];
    __shared__ double klsh[NT / 64];
    double kla = 0.0, klp = 0.0;
    double* klout = nullptr;
    VB_BEGIN_IF(map, KL ? K_KL_T : GATED ? K_ATTR_T : K_ATTR_T_ALL, (!GATED || live(I)))
    {
        if (KL) klout = I.kl_part;
        // the record's fields through a constant view: scalar loads, kept in
        // scalar registers (a vector copy of a base pointer would make the
        // compiler wait for in-flight loads whenever it reuses registers)
        const TSNE_CONST Inst& R = *cview<Inst>(&I);
        const int BI = R.tile_bi, BJ = R.tile_bj;   // BJ = WQ NT
        const int n = (int)R.n;
        const int tid = (int)threadIdx.x;
        unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem);   // [BI][S]
        V* yI = reinterpret_cast<V*>(acc + (size_t)BI * S);
        V* win = yI + BI;                                                        // [2][BJ]
        const void* Y = R.Yin;
        const TSNE_GLOBAL uint32_t* ep = gview<uint32_t>(R.epack);
        const TSNE_GLOBAL T* ev = gview<T>(R.eval);
        const TSNE_CONST int* tsj = cview<int>(R.tsj);           // uniform: scalar loads
        const TSNE_CONST int64_t* tse = cview<int64_t>(R.tse);
        const double scale = R.tscale;
        const int i0 = lb * BI;
        for (int r = tid; r < BI; r += NT) {
#pragma unroll
            for (int d = 0; d < S; ++d) acc[r * S + d] = 0ull;
            yI[r] = gpoint<T, S>(Y, min(i0 + r, n - 1));   // rows past n: never referenced
        }
        const int s0 = cview<int>(R.tsb)[lb], s1 = cview<int>(R.tsb)[lb + 1];
        // window registers: the window of the step after next is requested
        // while this step's non-zeros are taken, and stored a step later
        V wA[WQ], wB[WQ];
        // loads at a uniform base plus a 32-bit offset (scalar base address,
        // no 64-bit index arithmetic per lane)
        auto wload = [&](int J, V (&w)[WQ]) {
            const int j0 = J * BJ, lim = n - 1 - j0;   // >= 0: windows start below n
            const void* base = static_cast<const char*>(Y) + (size_t)j0 * S * sizeof(T);
#pragma unroll
            for (int q = 0; q < WQ; ++q) w[q] = gpoint<T, S>(base, min(tid + q * NT, lim));
        };
        auto wstore = [&](int buf, const V (&w)[WQ]) {
#pragma unroll
            for (int q = 0; q < WQ; ++q) win[buf * BJ + tid + q * NT] = w[q];
        };
        // a slot past the step's non-zeros loads the last non-zero and gets
        // mask 0 (applied where the value is used, so the load stays in flight)
        auto eload = [&](int st, uint32_t (&k)[UE], T (&v)[UE], T (&m)[UE]) {
            const int64_t e0 = tse[st];
            const int cnt = (int)(tse[st + 1] - e0);   // >= 1: steps hold non-zeros
            const TSNE_GLOBAL uint32_t* epb = ep + e0;
            const TSNE_GLOBAL T* evb = ev + e0;
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                const int e = tid + u * NT, ec = min(e, cnt - 1);
                k[u] = epb[ec];
                v[u] = evb[ec];
                m[u] = (e < cnt) ? (T)1 : (T)0;
            }
        };
        auto fx = [&](T c) -> unsigned long long {
            return (unsigned long long)__double2ll_rn((double)c * scale);
        };
        // a step's slots: every LDS read first, then the arithmetic, then the
        // atomics of the slots with a non-zero term (masked slots have none)
        // A wave whose lanes all lie past the step's non-zeros in a slot
        // skips that slot (a wave-uniform branch; steps fill about 70% of
        // their slots at C3).
        auto edges = [&](const uint32_t (&key)[UE], const T (&pv)[UE], const T (&m)[UE], const V* w) {
            V a[UE], b[UE];
            bool any[UE];
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                any[u] = __builtin_amdgcn_ballot_w64(m[u] != (T)0) != 0;
                if (any[u]) {
                    a[u] = yI[key[u] >> 16];
                    b[u] = w[key[u] & 0xffffu];
                }
            }
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                if (!any[u]) continue;
                T d0, d1 = (T)0;
                if constexpr (S == 2) { d0 = a[u].x - b[u].x; d1 = a[u].y - b[u].y; }
                else { d0 = a[u] - b[u]; }
                const T q = (T)1 + d0 * d0 + d1 * d1;
                const T pk = pv[u] * m[u];
                if constexpr (KL) {
                    if (pk > (T)0) {
                        kla += (double)pk * (double)log(pk * q);
                        klp += (double)pk;
                    }
                } else {
                    const T wgt = pk * recip(q);
                    const T c0 = wgt * d0, c1 = wgt * d1;
                    if (c0 != (T)0 || c1 != (T)0) {
                        const int lr = (int)(key[u] >> 16);
                        atomicAdd(&acc[lr * S], fx(c0));
                        if (S == 2) atomicAdd(&acc[lr * S + 1], fx(c1));
                    }
                }
            }
        };
        uint32_t kA[UE], kB[UE];
        T vA[UE], vB[UE], mA[UE], mB[UE];
        // step t: holds window t + 1 and the non-zeros of t in registers;
        // requests window t + 2 and the non-zeros of t + 1, takes its own
        // non-zeros against LDS buffer t mod 2, stores window t + 1 into the
        // other buffer, barrier
        auto step = [&](int st, const V (&wc)[WQ], V (&wn)[WQ], const uint32_t (&kc)[UE],
                        const T (&vc)[UE], const T (&mc)[UE], uint32_t (&kn)[UE], T (&vn)[UE],
                        T (&mn)[UE]) {
            const V* w = win + ((st - s0) & 1) * BJ;
            wload(tsj[min(st + 2, s1 - 1)], wn);
            eload(min(st + 1, s1 - 1), kn, vn, mn);
            edges(kc, vc, mc, w);
            wstore((st + 1 - s0) & 1, wc);
            lds_barrier();
        };
        if (s1 > s0) {
            wload(tsj[s0], wA);
            wstore(0, wA);
            wload(tsj[min(s0 + 1, s1 - 1)], wA);
            eload(s0, kA, vA, mA);
            // the sweep starts with nothing in flight: the loop's registers
            // then carry no load from before it, so the compiler places no
            // full wait at the top of every iteration
            __builtin_amdgcn_s_waitcnt(0);
        }
        lds_barrier();
        // steps in pairs, the registers' roles swapped in the second (every
        // path into the loop's top then comes from the same point), and a
        // last single step
        int st = s0;
        for (; st + 1 < s1; st += 2) {
            step(st, wA, wB, kA, vA, mA, kB, vB, mB);
            step(st + 1, wB, wA, kB, vB, mB, kA, vA, mA);
        }
        if (st < s1) step(st, wA, wB, kA, vA, mA, kB, vB, mB);
        if constexpr (!KL) {
            TSNE_GLOBAL T* F = (TSNE_GLOBAL T*)R.Fattr;
            const int rows = min(BI, n - i0);
            for (int r = tid; r < rows * S; r += NT)
                F[(int64_t)i0 * S + r] = (T)((double)(long long)acc[r] / scale);
        }
        __syncthreads();   // the LDS is reused by the next virtual block
    }
    VB_END
    if constexpr (KL) {
        // a single-instance launch: the block's partials (klout is the
        // instance's array once the block has run a virtual block)
        kla = block_sum_d(kla, klsh);
        klp = block_sum_d(klp, klsh);
        if (threadIdx.x == 0 && klout) {
            klout[2 * blockIdx.x] = kla;
            klout[2 * blockIdx.x + 1] = klp;
        }
    }
}

// Attraction entry point with slabs: F_attr = sum of the slab partials.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_asum(LaunchMap map)
{
    VB_BEGIN(map, K_ASUM)
    {
        const int64_t k = (int64_t)lb * 256 + threadIdx.x;
        const int64_t ns = I.n * S;
        if (k < ns) {
            const T* Fp = static_cast<const T*>(I.Fap);
            // every slab's partial in flight at once, then summed in slab order
            constexpr int kMaxSlabs = 8;
            T q[kMaxSlabs];
#pragma unroll
            for (int sl = 0; sl < kMaxSlabs; ++sl)
                if (sl < I.slabs) q[sl] = Fp[(int64_t)sl * ns + k];
            double a = 0.0;
#pragma unroll
            for (int sl = 0; sl < kMaxSlabs; ++sl)
                if (sl < I.slabs) a += (double)q[sl];
            static_cast<T*>(I.Fattr)[k] = (T)a;
        }
    }
    VB_END
}

// ---------------------------------------------------------------- KL divergence

// C = sum p_ij log(p_ij / q_ij) with q_ij = K1_ij / Z (Section 1.1), split as
// sum p log(p (1 + |y_i - y_j|^2)) + (sum p) log Z: the attraction kernel's
// divergence mode leaves the first two sums as FP64 partials per block; this
// kernel adds them in block order and applies the Z of the same call.
__global__ __launch_bounds__(256) void k_klsum(LaunchMap map)
{
    __shared__ double sh[8];
    VB_BEGIN(map, K_KLSUM)
    if (live(I)) {
        double a = 0.0, ps = 0.0;
        for (int b = threadIdx.x; b < I.nb_kl; b += 256) {
            a += I.kl_part[2 * b];
            ps += I.kl_part[2 * b + 1];
        }
        a = block_sum_d(a, sh);
        ps = block_sum_d(ps, sh);
        if (threadIdx.x == 0 && I.KLout) *I.KLout = a + ps * log(I.geom->Z);
    }
    VB_END
}

// ---------------------------------------------------------------- packing

// (column, value bits) pairs of an FP32 CSR, for the packed attraction.
__global__ __launch_bounds__(256) void k_pack_cv(const int32_t* __restrict__ col,
                                                 const float* __restrict__ val, uint2* __restrict__ cv,
                                                 int64_t nnz)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256)
        cv[k] = make_uint2((unsigned)col[k], __float_as_uint(val[k]));
}

hipError_t launch_pack_cv(const int32_t* col, const float* val, void* cv, int64_t nnz, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nnz + 255) / 256, 8192);
    hipLaunchKernelGGL(k_pack_cv, dim3((unsigned)blocks), dim3(256), 0, st, col, val,
                       static_cast<uint2*>(cv), nnz);
    return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch

template <typename T, int S>
static hipError_t launch_attr(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                              hipStream_t st)
{
    constexpr bool PK = sizeof(T) == 4;   // FP32 plans bind P packed (the CSR layout)
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_ATTR:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr<T, S, 4, 10, true, PK>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr<T, S, 8, 4, true, PK>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr<T, S, 16, 3, true, PK>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr<T, S, 32, 3, true, PK>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr<T, S, 64, 2, true, PK>), g, b, 0, st, map);
        break;
    case K_ATTR_ALL:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr<T, S, 4, 10, false, PK>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr<T, S, 8, 4, false, PK>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr<T, S, 16, 3, false, PK>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr<T, S, 32, 3, false, PK>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr<T, S, 64, 2, false, PK>), g, b, 0, st, map);
        break;
    case K_ASUM: hipLaunchKernelGGL((k_asum<T, S>), g, b, 0, st, map); break;
    case K_KL_ATTR:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr<T, S, 4, 10, true, PK, true>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr<T, S, 8, 4, true, PK, true>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr<T, S, 16, 3, true, PK, true>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr<T, S, 32, 3, true, PK, true>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr<T, S, 64, 2, true, PK, true>), g, b, 0, st, map);
        break;
    case K_KLSUM: hipLaunchKernelGGL(k_klsum, g, b, 0, st, map); break;
    case K_ATTR_T:
        if (l.lds > 48 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_attr_tile<T, S, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)l.lds);
        hipLaunchKernelGGL((k_attr_tile<T, S, true>), g, b, l.lds, st, map);
        break;
    case K_ATTR_T_ALL:
        if (l.lds > 48 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_attr_tile<T, S, false>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)l.lds);
        hipLaunchKernelGGL((k_attr_tile<T, S, false>), g, b, l.lds, st, map);
        break;
    case K_KL_T:
        if (l.lds > 48 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_attr_tile<T, S, true, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)l.lds);
        hipLaunchKernelGGL((k_attr_tile<T, S, true, true>), g, b, l.lds, st, map);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// s = 3: the CSR rows at the plan's lanes per row, one slab
template <typename T>
static hipError_t launch_attr3(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                               hipStream_t st)
{
    dim3 g(l.grid), b(l.block);
    switch (kind) {
    case K_ATTR:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr3<T, 4, 8, true>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr3<T, 8, 4, true>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr3<T, 16, 3, true>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr3<T, 32, 3, true>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr3<T, 64, 2, true>), g, b, 0, st, map);
        break;
    case K_ATTR_ALL:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr3<T, 4, 8, false>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr3<T, 8, 4, false>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr3<T, 16, 3, false>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr3<T, 32, 3, false>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr3<T, 64, 2, false>), g, b, 0, st, map);
        break;
    case K_KL_ATTR:
        if (c.lpr == 4) hipLaunchKernelGGL((k_attr3<T, 4, 8, true, true>), g, b, 0, st, map);
        else if (c.lpr == 8) hipLaunchKernelGGL((k_attr3<T, 8, 4, true, true>), g, b, 0, st, map);
        else if (c.lpr == 16) hipLaunchKernelGGL((k_attr3<T, 16, 3, true, true>), g, b, 0, st, map);
        else if (c.lpr == 32) hipLaunchKernelGGL((k_attr3<T, 32, 3, true, true>), g, b, 0, st, map);
        else hipLaunchKernelGGL((k_attr3<T, 64, 2, true, true>), g, b, 0, st, map);
        break;
    case K_KLSUM: hipLaunchKernelGGL(k_klsum, g, b, 0, st, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_attr_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                            hipStream_t st)
{
    if (c.s == 3) return c.dtype == 0 ? launch_attr3<float>(kind, c, map, l, st)
                                      : launch_attr3<double>(kind, c, map, l, st);
    if (c.dtype == 0)
        return c.s == 1 ? launch_attr<float, 1>(kind, c, map, l, st) : launch_attr<float, 2>(kind, c, map, l, st);
    return c.s == 1 ? launch_attr<double, 1>(kind, c, map, l, st) : launch_attr<double, 2>(kind, c, map, l, st);
}

}  // namespace tsne
