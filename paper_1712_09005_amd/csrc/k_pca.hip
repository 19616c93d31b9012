// Randomised PCA of Section 6 (Algorithm 2) on gfx950, FP64.
//
// The big matrix A enters only through two skinny products on the FP64
// matrix cores:
//   k_mm_mfma   C (rows x nc) = M (rows x K, row-major) S (K x nc)   A X, Z W
//   k_mmt_mfma  C (p x l)    (+)= M^T T, M rows x p, T rows x l       A^T T, Z^T Z
// and the small l x l eigenproblems run in one workgroup (cyclic Jacobi).
// The host side walks A in b-row blocks (copied from host memory when A is
// there), so each power iteration reads every block once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "tsne.h"
#include "tsne_pca.h"

namespace pca {

constexpr int TILE = 64;      // output tile edge (rows or columns) per workgroup, and the max l
constexpr int KC = 32;        // reduction chunk staged in LDS
constexpr int GSPLIT = 256;   // row splits of a Gram product
constexpr int MSPLIT = 8;     // most row splits of an A^T T product (partials of n x l each)
constexpr double kDrop = 1e-12;

// The two products on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 v + l / 16][l % 16] in its v-th accumulator).  A workgroup computes a
// 64 x 64 output tile; each of its four waves owns a 16-row strip of it as
// four 16 x 16 blocks.  Operands are staged through LDS in chunks of KC
// along the reduction:
//   k_mm_mfma   C[r][c] = sum_k M[r][k] S[k][c], r < rows, c < nc <= 64;
//   k_mmt_mfma  C[c][j] (+)= sum_r M[r][c] T[r][j], c < p, j < l, over the
//               rows of the workgroup's split (blockIdx.y; split s writes
//               C + s * split_stride).
// Both kernels are held to three waves per SIMD (three workgroups per CU,
// 39 or 41 KB of LDS each): the accumulators then live in VGPRs and the
// occupancy hides more of the global latency than the default two waves.
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int SMP = KC + 4;     // LDS row pitch of the 64 x 32 tile
constexpr int SSP = TILE + 16;  // LDS row pitch of the 32 x 64 tile

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_mm_mfma(const double* __restrict__ M, int64_t ldm, int64_t rows,
                                                 int64_t K, const double* __restrict__ S, int64_t lds,
                                                 int nc, double* __restrict__ C, int64_t ldc)
{
    __shared__ double sm[TILE * SMP];
    __shared__ double ss[KC * SSP];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * TILE;
    dbl4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    // the next chunk is loaded into registers while the current one is multiplied
    constexpr int QA = TILE * KC / 256, QS = KC * TILE / 256;
    double ra[QA], rs[QS];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + 256 * q, rr = e / KC, kk = e % KC;
            const int64_t r = r0 + rr, k = k0 + kk;
            ra[q] = (r < rows && k < K) ? M[r * ldm + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const int e = tid + 256 * q, kk = e / TILE, c = e % TILE;
            const int64_t k = k0 + kk;
            rs[q] = (k < K && c < nc) ? S[k * lds + c] : 0.0;
        }
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + 256 * q;
            sm[(e / KC) * SMP + e % KC] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const int e = tid + 256 * q;
            ss[(e / TILE) * SSP + e % TILE] = rs[q];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const double a = sm[(wv * 16 + li) * SMP + kk + lk];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ss[(kk + lk) * SSP + t * 16 + li], acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + wv * 16 + 4 * v + lk;
        if (r >= rows) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = t * 16 + li;
            if (c < nc) C[r * ldc + c] = acc[t][v];
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_mmt_mfma(const double* __restrict__ M, int64_t ldm, int64_t rows,
                                                  int64_t p, const double* __restrict__ T, int64_t ldt, int l,
                                                  double* __restrict__ C, int64_t ldc, int accumulate,
                                                  int64_t rows_per_split, int64_t split_stride)
{
    __shared__ double sm[KC * SSP];
    __shared__ double st[KC * SSP];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * TILE;
    const int64_t rb = (int64_t)blockIdx.y * rows_per_split;
    const int64_t re = std::min(rows, rb + rows_per_split);
    dbl4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    // the next chunk is loaded into registers while the current one is multiplied
    constexpr int Q = KC * TILE / 256;
    double rm[Q], rt[Q];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q, rr = e / TILE, cc = e % TILE;
            const int64_t r = r0 + rr, c = c0 + cc;
            rm[q] = (r < re && c < p) ? M[r * ldm + c] : 0.0;
            rt[q] = (r < re && cc < l) ? T[r * ldt + cc] : 0.0;
        }
    };
    if (rb < re) fetch(rb);
    for (int64_t r0 = rb; r0 < re; r0 += KC) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q;
            sm[(e / TILE) * SSP + e % TILE] = rm[q];
            st[(e / TILE) * SSP + e % TILE] = rt[q];
        }
        __syncthreads();
        if (r0 + KC < re) fetch(r0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const double a = sm[(kk + lk) * SSP + wv * 16 + li];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, st[(kk + lk) * SSP + t * 16 + li], acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    double* Cs = C + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t c = c0 + wv * 16 + 4 * v + lk;
        if (c >= p) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int jj = t * 16 + li;
            if (jj < l) {
                double* o = Cs + c * ldc + jj;
                *o = accumulate ? *o + acc[t][v] : acc[t][v];
            }
        }
    }
}

// G[e] (+)= sum over splits s (in order) of part[s][e], e < count.
__global__ __launch_bounds__(256) void k_sum_splits(const double* __restrict__ part, int splits,
                                                    int64_t stride, int64_t count, double* __restrict__ G,
                                                    int accumulate)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    double a = 0.0;
    for (int s = 0; s < splits; ++s) a += part[(int64_t)s * stride + e];
    G[e] = accumulate ? G[e] + a : a;
}

// Eigenpairs of the symmetric l x l matrix G (l <= 64) by cyclic Jacobi
// rotations, sorted by decreasing eigenvalue.  Outputs, row-major l x l:
//   W   the eigenvectors (columns);
//   Ws  mode 0: W[:, j] lambda_j^(-1/2); mode 1: W[:, j] / sqrt(lambda_j);
//       both zero for a dropped direction (lambda_j <= kDrop lambda_max);
//   sv  (mode 1 only, the first nsv entries) sqrt(max(lambda_j, 0)).
// One workgroup; each rotation J = [c s; -s c] in the (p, q) plane updates
// the columns of G and W, then the rows of G.
__global__ __launch_bounds__(256) void k_symeig(const double* __restrict__ G, int l, int mode,
                                                double* __restrict__ W, double* __restrict__ Ws,
                                                double* __restrict__ sv, int nsv)
{
    __shared__ double a[TILE][TILE + 1];
    __shared__ double w[TILE][TILE + 1];
    __shared__ double red[2][256];
    __shared__ double rot[2];
    __shared__ int go;
    __shared__ int order[TILE];
    __shared__ double lam[TILE];
    const int tid = threadIdx.x;
    for (int e = tid; e < l * l; e += 256) {
        const int i = e / l, j = e % l;
        a[i][j] = 0.5 * (G[i * l + j] + G[j * l + i]);
        w[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < l * l; e += 256) {
            const int i = e / l, j = e % l;
            const double v = a[i][j] * a[i][j];
            tot += v;
            if (i != j) off += v;
        }
        red[0][tid] = off;
        red[1][tid] = tot;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
            }
            __syncthreads();
        }
        const bool done = !(red[0][0] > 1e-30 * red[1][0]);
        __syncthreads();
        if (done) break;
        for (int p = 0; p < l - 1; ++p) {
            for (int q = p + 1; q < l; ++q) {
                if (tid == 0) {
                    const double apq = a[p][q];
                    const double scale = fabs(a[p][p]) + fabs(a[q][q]);
                    go = (apq != 0.0 && fabs(apq) > 1e-300 + 1e-18 * scale) ? 1 : 0;
                    if (go) {
                        const double tau = (a[q][q] - a[p][p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        const double c = 1.0 / sqrt(1.0 + t * t);
                        rot[0] = c;
                        rot[1] = t * c;
                    }
                }
                __syncthreads();
                // every thread reads the same flag, so the barrier inside is uniform;
                // the last barrier keeps thread 0 from overwriting it too early
                const int g = go;
                const double c = rot[0], s = rot[1];
                if (g) {
                    if (tid < l) {
                        const double rp = a[tid][p], rq = a[tid][q];
                        a[tid][p] = c * rp - s * rq;
                        a[tid][q] = s * rp + c * rq;
                    } else if (tid >= 128 && tid < 128 + l) {
                        const int r = tid - 128;
                        const double wp = w[r][p], wq = w[r][q];
                        w[r][p] = c * wp - s * wq;
                        w[r][q] = s * wp + c * wq;
                    }
                    __syncthreads();
                    if (tid < l) {
                        const double pr = a[p][tid], qr = a[q][tid];
                        a[p][tid] = c * pr - s * qr;
                        a[q][tid] = s * pr + c * qr;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (tid == 0) {
        for (int j = 0; j < l; ++j) {
            order[j] = j;
            lam[j] = a[j][j];
        }
        for (int i = 0; i < l; ++i) {          // selection sort, decreasing
            int best = i;
            for (int j = i + 1; j < l; ++j)
                if (lam[order[j]] > lam[order[best]]) best = j;
            const int t = order[i];
            order[i] = order[best];
            order[best] = t;
        }
    }
    __syncthreads();
    const double lmax = lam[order[0]];
    for (int e = tid; e < l * l; e += 256) {
        const int i = e / l, j = e % l;
        const double lj = lam[order[j]];
        const double v = w[i][order[j]];
        const bool keep = lmax > 0.0 && lj > kDrop * lmax;
        W[i * l + j] = v;
        Ws[i * l + j] = keep ? v / sqrt(lj) : 0.0;
    }
    if (mode == 1)
        for (int j = tid; j < nsv; j += 256) sv[j] = sqrt(std::max(lam[order[j]], 0.0));
}

// ---------------------------------------------------------------- host side

struct Ws {
    double *X, *X2, *Y, *Q, *G, *W, *Wsc, *part, *stage;
};

static size_t up(size_t v) { return (v + 31) & ~size_t(31); }   // doubles, to 256 bytes

static int64_t block_rows(const tsne_pca_desc* d)
{
    if (d->b > 0) return std::min(d->b, d->m);
    return d->a_host ? std::min<int64_t>(16384, d->m) : d->m;
}

static bool valid(const tsne_pca_desc* d)
{
    return d && d->m > 0 && d->n > 0 && d->lda >= d->n && d->l > 0 && d->k > 0 && d->k <= d->l &&
           d->l < std::min(d->m, d->n) && d->its >= 0 && d->b >= 0 && (d->a_host == 0 || d->a_host == 1);
}

static size_t layout(const tsne_pca_desc* d, char* base, Ws* w)
{
    const size_t l = (size_t)d->l, m = (size_t)d->m, n = (size_t)d->n;
    const size_t parts = std::max((size_t)GSPLIT * l * l, (size_t)MSPLIT * n * l);
    const size_t sizes[9] = {up(n * l), up(n * l), up(m * l), up(m * l), up(l * l), up(l * l), up(l * l),
                             up(parts), d->a_host ? up((size_t)block_rows(d) * n) : 0};
    size_t off = 0;
    double** slots[9] = {&w->X, &w->X2, &w->Y, &w->Q, &w->G, &w->W, &w->Wsc, &w->part, &w->stage};
    for (int i = 0; i < 9; ++i) {
        if (w) *slots[i] = base ? reinterpret_cast<double*>(base) + off : nullptr;
        off += sizes[i];
    }
    return off * sizeof(double);
}

struct Runner {
    const tsne_pca_desc* d;
    const double* A;
    Ws w;
    hipStream_t st;
    int64_t b;
    bool ok = true;

    void check(hipError_t e) { if (e != hipSuccess) ok = false; }
    void launched() { check(hipGetLastError()); }

    // the rows [r0, r0 + rows) of A in device memory (copied there if A is on the host)
    const double* block(int64_t r0, int64_t rows, int64_t& ld)
    {
        if (!d->a_host) {
            ld = d->lda;
            return A + r0 * d->lda;
        }
        ld = d->n;
        check(hipMemcpy2DAsync(w.stage, (size_t)d->n * sizeof(double), A + r0 * d->lda,
                               (size_t)d->lda * sizeof(double), (size_t)d->n * sizeof(double),
                               (size_t)rows, hipMemcpyHostToDevice, st));
        return w.stage;
    }
    void mm(const double* M, int64_t ldm, int64_t rows, int64_t K, const double* S, int64_t lds, int nc,
            double* C, int64_t ldc)
    {
        if (rows <= 0) return;
        const dim3 g((unsigned)((rows + TILE - 1) / TILE));
        hipLaunchKernelGGL(k_mm_mfma, g, dim3(256), 0, st, M, ldm, rows, K, S, lds, nc, C, ldc);
        launched();
    }
    // C (+)= M^T T with C p x l.  When the column tiles alone leave the chip
    // underfilled the rows are split (at most MSPLIT ways, each split at
    // least 4096 rows) into partials that are then added in a fixed order.
    void mmt(const double* M, int64_t ldm, int64_t rows, int64_t p, const double* T, int64_t ldt,
             double* C, int accumulate)
    {
        if (rows <= 0) return;
        const int64_t tiles = (p + TILE - 1) / TILE;
        int64_t splits = std::min<int64_t>({(int64_t)MSPLIT, (2048 + tiles - 1) / tiles, rows / 4096});
        if (splits < 2) {
            hipLaunchKernelGGL(k_mmt_mfma, dim3((unsigned)tiles, 1), dim3(256), 0, st, M, ldm, rows, p, T, ldt,
                               d->l, C, (int64_t)d->l, accumulate, rows, (int64_t)0);
            launched();
            return;
        }
        int64_t per = (rows + splits - 1) / splits;
        per = ((per + KC - 1) / KC) * KC;
        splits = (rows + per - 1) / per;
        const int64_t cnt = p * d->l;
        hipLaunchKernelGGL(k_mmt_mfma, dim3((unsigned)tiles, (unsigned)splits), dim3(256), 0, st, M, ldm, rows, p, T,
                           ldt, d->l, w.part, (int64_t)d->l, 0, per, cnt);
        launched();
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, w.part,
                           (int)splits, cnt, cnt, C, accumulate);
        launched();
    }
    // G = Z^T Z for Z rows x l, split over row ranges, summed in a fixed order
    void gram(const double* Z, int64_t rows)
    {
        const int l = d->l;
        int64_t per = (rows + GSPLIT - 1) / GSPLIT;
        per = ((per + KC - 1) / KC) * KC;
        const int splits = (int)((rows + per - 1) / per);
        hipLaunchKernelGGL(k_mmt_mfma, dim3(1, splits), dim3(256), 0, st, Z, (int64_t)l, rows, (int64_t)l, Z,
                           (int64_t)l, l, w.part, (int64_t)l, 0, per, (int64_t)l * l);
        launched();
        const int64_t cnt = (int64_t)l * l;
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, w.part, splits,
                           cnt, cnt, w.G, 0);
        launched();
    }
    void eig(int mode, double* sv, int nsv)
    {
        hipLaunchKernelGGL(k_symeig, dim3(1), dim3(256), 0, st, w.G, d->l, mode, w.W, w.Wsc, sv, nsv);
        launched();
    }
    // Zout = Z W diag(lambda)^(-1/2): orthonormal columns spanning Z's range
    void orth(const double* Z, int64_t rows, double* Zout)
    {
        gram(Z, rows);
        eig(0, nullptr, 0);
        mm(Z, d->l, rows, d->l, w.Wsc, d->l, d->l, Zout, d->l);
    }
    // Xout = A^T (A Xin), one pass over the blocks of A (A_b X into Q's rows)
    void ata(const double* Xin, double* Xout)
    {
        for (int64_t r0 = 0; r0 < d->m; r0 += b) {
            const int64_t rows = std::min(b, d->m - r0);
            int64_t ld;
            const double* Ab = block(r0, rows, ld);
            double* Tb = w.Q + r0 * d->l;
            mm(Ab, ld, rows, d->n, Xin, d->l, d->l, Tb, d->l);
            mmt(Ab, ld, rows, d->n, Tb, d->l, Xout, r0 > 0);
        }
    }
    void apply_A(const double* Xin, double* Yout)
    {
        for (int64_t r0 = 0; r0 < d->m; r0 += b) {
            const int64_t rows = std::min(b, d->m - r0);
            int64_t ld;
            const double* Ab = block(r0, rows, ld);
            mm(Ab, ld, rows, d->n, Xin, d->l, d->l, Yout + r0 * d->l, d->l);
        }
    }
    void apply_At(const double* Z, double* Out)
    {
        for (int64_t r0 = 0; r0 < d->m; r0 += b) {
            const int64_t rows = std::min(b, d->m - r0);
            int64_t ld;
            const double* Ab = block(r0, rows, ld);
            mmt(Ab, ld, rows, d->n, Z + r0 * d->l, d->l, Out, r0 > 0);
        }
    }
};

}  // namespace pca

using namespace pca;

extern "C" size_t tsne_pca_workspace_bytes(const tsne_pca_desc* d)
{
    if (!valid(d) || d->l > TILE) return 0;
    return layout(d, nullptr, nullptr);
}

extern "C" int tsne_pca(const tsne_pca_desc* d, const double* A, const double* omega, double* U, double* s,
                        double* V, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!valid(d) || !A || !omega || !U || !s || !V) return TSNE_E_ARG;
    if (d->l > TILE) return TSNE_E_UNSUPPORTED;
    const size_t need = layout(d, nullptr, nullptr);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return TSNE_E_WORKSPACE;
    Runner R;
    R.d = d;
    R.A = A;
    R.st = static_cast<hipStream_t>(stream);
    R.b = block_rows(d);
    layout(d, static_cast<char*>(workspace), &R.w);
    const int64_t m = d->m, n = d->n;
    const int l = d->l, k = d->k;
    // power iterations on the n side: X_i = orth(A^T A X_{i-1}), X_0 = Omega
    const double* X = omega;
    for (int i = 1; i <= d->its; ++i) {
        R.ata(X, R.w.X2);
        R.orth(R.w.X2, n, R.w.X);
        X = R.w.X;
    }
    // Y = A X, then two orthonormalisations (the second restores orthogonality)
    R.apply_A(X, R.w.Y);
    R.orth(R.w.Y, m, R.w.Q);
    R.orth(R.w.Q, m, R.w.Y);
    const double* Qf = R.w.Y;
    // B^T = A^T Q (n x l); B B^T = W diag(lambda) W^T
    R.apply_At(Qf, R.w.X2);
    R.gram(R.w.X2, n);
    R.eig(1, s, k);
    // U = Q W, V = B^T W diag(1/s), first k columns
    R.mm(Qf, l, m, l, R.w.W, l, k, U, k);
    R.mm(R.w.X2, l, n, l, R.w.Wsc, l, k, V, k);
    return R.ok ? TSNE_OK : TSNE_E_HIP;
}
