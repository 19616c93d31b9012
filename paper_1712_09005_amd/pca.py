"""Python binding of the randomised PCA (Section 6, Algorithm 2) in
``libtsne_mi355x.so``: argument marshalling only, every step runs in the
library's kernels (``csrc/k_pca.hip``)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import tsne


class Desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("its", ctypes.c_int32),
                ("a_host", ctypes.c_int32), ("b", ctypes.c_int64)]


def make_desc(m: int, n: int, k: int, l: int | None = None, its: int = 2, lda: int | None = None,
              a_host: bool = False, b: int = 0) -> Desc:
    return Desc(m, n, n if lda is None else lda, k, k + 2 if l is None else l, its,
                1 if a_host else 0, b)


def oocpca(A, omega, k: int, its: int = 2, b: int = 0, device=None):
    """Top-k principal components of A (no centring).

    A: a CUDA float64 tensor with unit column stride (device mode), or a
    C-contiguous float64 numpy array (host mode: streamed to the device b
    rows at a time).  omega: the n x l random matrix (numpy or CUDA tensor).
    Returns CUDA tensors U (m x k), s (k), V (n x k), enqueued on the current
    stream."""
    on_host = isinstance(A, np.ndarray)
    if on_host:
        if A.dtype != np.float64 or A.ndim != 2 or not A.flags["C_CONTIGUOUS"]:
            raise ValueError("host A must be a C-contiguous float64 matrix")
        m, n = A.shape
        lda = n
        dev = torch.device(device if device is not None else "cuda:0")
        a_ptr = A.ctypes.data
    else:
        if A.dtype != torch.float64 or A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
            raise ValueError("device A must be a CUDA float64 matrix with unit column stride")
        m, n = A.shape
        lda = A.stride(0)
        dev = A.device
        a_ptr = A.data_ptr()
    om = torch.as_tensor(omega, dtype=torch.float64, device=dev).contiguous()
    if om.dim() != 2 or om.shape[0] != n:
        raise ValueError("omega must be n x l")
    l = om.shape[1]
    d = make_desc(m, n, k, l, its, lda=lda, a_host=on_host, b=b)
    L = tsne.lib()
    nb = L.tsne_pca_workspace_bytes(ctypes.byref(d))
    if nb == 0:
        raise ValueError("invalid PCA sizes (need 0 < k <= l <= 64, l < min(m, n), its >= 0)")
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    U = torch.empty((m, k), dtype=torch.float64, device=dev)
    s = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    P = ctypes.c_void_p
    rc = L.tsne_pca(ctypes.byref(d), P(a_ptr), P(om.data_ptr()), P(U.data_ptr()), P(s.data_ptr()),
                    P(V.data_ptr()), P(ws.data_ptr()), nb, P(st))
    if rc != 0:
        raise RuntimeError("tsne_pca failed: %s" % L.tsne_status_str(rc).decode())
    if on_host:
        torch.cuda.current_stream(dev).synchronize()   # A's pages are read by the copies
    return U, s, V
