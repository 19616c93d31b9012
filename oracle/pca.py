"""CPU oracle for the out-of-core randomised PCA of Section 6 (Algorithm 2).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the benchmark's CPU-baseline
leg, never by the GPU library, and it shares no code with it.  Plain FP64
numpy/scipy: every product with the big matrix A is formed a block of b rows
at a time, exactly as the algorithm states, and the renormalisations are the
library's LU with partial pivoting and Householder QR, the small SVD the
library's SVD.

Algorithm 2 (Section 6.1 for the background, 6.2 for the blocking), with
A of size m x n, l random vectors and its power iterations:

1. Omega, n x l, uniform random: an input here (the caller draws it).
2. Y_0 = A Omega, block-wise; L_0 U_0 = Y_0 (LU, L with its rows permuted).
3. For i = 1 .. its: Y_i = A (A^* L_{i-1}), block-wise; for i < its,
   L_i U_i = Y_i.
4. Q R = Y_its (Y_0 when its = 0); U' Sigma V^* = Q^* A; U = Q U'.
5. The first k columns of U and V and the first k singular values.

A^* L is formed as the sum over row blocks of A_b^T L_b, so each product
reads A one block at a time (Section 6.2).  No mean centring: the section
lists centring as an optional pre-processing step outside the algorithm.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _blocks(m: int, b: int):
    b = max(1, int(b))
    for r0 in range(0, m, b):
        yield r0, min(m, r0 + b)


def apply_A(A: np.ndarray, X: np.ndarray, b: int) -> np.ndarray:
    """A X, filled in b rows at a time (Section 6.2)."""
    out = np.empty((A.shape[0], X.shape[1]), dtype=np.float64)
    for r0, r1 in _blocks(A.shape[0], b):
        out[r0:r1] = np.asarray(A[r0:r1], dtype=np.float64) @ X
    return out


def apply_At(A: np.ndarray, Y: np.ndarray, b: int) -> np.ndarray:
    """A^* Y as the sum over row blocks of A_b^T Y_b (Section 6.2)."""
    out = np.zeros((A.shape[1], Y.shape[1]), dtype=np.float64)
    for r0, r1 in _blocks(A.shape[0], b):
        out += np.asarray(A[r0:r1], dtype=np.float64).T @ Y[r0:r1]
    return out


def lu_renorm(Y: np.ndarray) -> np.ndarray:
    """L of the LU factorisation with partial pivoting, rows permuted back
    (the renormalisation of Algorithm 2)."""
    PL, _ = scipy.linalg.lu(Y, permute_l=True)
    return PL


def oocpca(A: np.ndarray, omega: np.ndarray, k: int, its: int, b: int):
    """Algorithm 2.  Returns (U, s, V): U m x k and V n x k with orthonormal
    columns, s the k largest singular values in decreasing order, so that
    A ~ U diag(s) V^T."""
    A = np.asarray(A)
    m, n = A.shape
    omega = np.asarray(omega, dtype=np.float64)
    l = omega.shape[1]
    if omega.shape[0] != n or not (0 < k <= l < min(m, n)) or its < 0:
        raise ValueError("oocpca: need omega n x l and 0 < k <= l < min(m, n), its >= 0")
    Y = apply_A(A, omega, b)
    for i in range(1, its + 1):
        L = lu_renorm(Y)
        Y = apply_A(A, apply_At(A, L, b), b)
    Q, _ = np.linalg.qr(Y)
    B = apply_At(A, Q, b).T                      # Q^* A, l x n
    Up, s, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Up
    return U[:, :k], s[:k], Vt[:k].T
