/*
 * tsne_pca.h - C ABI of the randomised PCA of the MI355X t-SNE library.
 *
 * Out-of-core randomised PCA, Algorithm 2 of Section 6 (Linderman et al.,
 * FIt-SNE): the top k principal components of an m x n matrix A from l
 * random vectors and `its` power iterations, touching A only through
 * block-wise products, b rows at a time (Section 6.2).
 *
 * Computation (FP64 throughout, as the section's matrices of doubles):
 *   X_0 = Omega;  X_i = orth(A^T (A X_{i-1})) for i = 1 .. its,
 *   Y = A X_its;  Q = orth(orth(Y));  B^T = A^T Q;
 *   B B^T = W diag(lambda) W^T;  s = sqrt(lambda);  U = Q W;  V = B^T W diag(1/s).
 * Each power iteration reads A once: every b-row block A_b is used for
 * A_b X and then for A_b^T (A_b X) while it is in device memory, so the
 * product with A A^T costs one pass, as Section 6.2 arranges it.  The span
 * of Y equals that of Algorithm 2's Y_its ((A A^T)^its A Omega); the
 * renormalisations (LU and QR in the paper) are orthonormalisations here:
 * Z <- Z W diag(lambda)^(-1/2) from the eigenpairs of Z^T Z, directions with
 * lambda <= 1e-12 lambda_max dropped (their columns set to zero).  k is
 * therefore at most the numerical rank of A for nonzero output columns.
 *
 * Layouts: A row-major with row stride lda >= n (A[i*lda + j]); Omega n x l,
 * U m x k, V n x k row-major with row strides l, k, k; s has k entries in
 * decreasing order.  Columns of U and V are orthonormal and defined up to a
 * common sign per column; A ~ U diag(s) V^T.
 *
 * Pointers are device pointers except A when a_host = 1 (host memory,
 * pinned or pageable, copied to the workspace b rows at a time).  All
 * arrays are owned by the caller and must stay valid until the enqueued
 * work has completed on `stream` (hipStream_t or NULL).  The library
 * allocates no memory: the caller passes a device workspace of at least
 * tsne_pca_workspace_bytes bytes, 256-byte aligned.  Work is enqueued
 * asynchronously; the call returns TSNE_OK (0), TSNE_E_ARG (1) for invalid
 * sizes, TSNE_E_UNSUPPORTED (2) for l > 64, TSNE_E_WORKSPACE (3) for a
 * missing or short workspace, or TSNE_E_HIP (6) if a launch or copy fails.
 */
#ifndef TSNE_PCA_MI355X_H
#define TSNE_PCA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsne_pca_desc {
    int64_t m, n;      /* A is m x n, 0 < l < min(m, n) */
    int64_t lda;       /* row stride of A in doubles, >= n */
    int32_t k;         /* components returned, 0 < k <= l */
    int32_t l;         /* random vectors, l <= 64 (the paper's default is k + 2) */
    int32_t its;       /* power iterations, >= 0 */
    int32_t a_host;    /* 1: A in host memory, streamed in b-row blocks */
    int64_t b;         /* rows per block of A; 0 = all rows (device A) or 16384 (host A) */
} tsne_pca_desc;

/* Workspace bytes for tsne_pca with this descriptor (0 if it is invalid). */
size_t tsne_pca_workspace_bytes(const tsne_pca_desc* d);

/* Algorithm 2 of Section 6 as described above.  omega: n x l, the random
 * matrix of the algorithm's first step (uniform random numbers drawn by the
 * caller).  Outputs U (m x k), s (k), V (n x k). */
int tsne_pca(const tsne_pca_desc* d, const double* A, const double* omega,
             double* U, double* s, double* V,
             void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif
