"""CPU oracle for the FIt-SNE per-iteration t-SNE gradient.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path; both are fed from ``paper_1712_09005_amd.inputs``, which
holds no gradient arithmetic.

The arithmetic lives in ``oracle.c`` (plain FP64 C, OpenMP over independent
rows), loaded here with ctypes.  Function-by-function citations of the paper
are in that file.  Every routine is pinned by the ``-m "not gpu"`` tests
against closed forms, hand-computed values, brute force on tiny inputs and
invariants, except the constants of the descent step (``update``), which the
paper does not state: the rule is pinned by hand-computed steps, its constants
are a reading (parity unpinned by the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KERNEL_TSNE, KERNEL_POLY = 0, 1
FORM_A, FORM_B, FORM_V = 0, 1, 2
POLICY_PAPER, POLICY_FIXED = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        sig = {
            "oracle_direct_sums": [i64, i32, P, i32, P, i64, P, P],
            "oracle_direct_rep": [i64, i32, P, i32, P, P],
            "oracle_attr": [i64, i32, P, P, P, P, P],
            "oracle_kl": [i64, i32, P, P, P, P, f64],
            "oracle_knn": [i64, i32, P, i32, P, P],
            "oracle_knn_rows": [i64, i32, P, i32, P, i64, P, P],
            "oracle_perplexity": [i64, i32, P, f64, P, P],
            "oracle_symmetrize": [i64, i32, P, P, P, P, P],
            "oracle_geometry": [i64, i32, P, i32, i32, f64, i32, P, P, P],
            "oracle_lagrange": [i32, f64, P],
            "oracle_grid_conv": [i32, P, f64, i32, i32, P, P],
            "oracle_interp_rep": [i64, i32, P, P, f64, P, i32, i32, i32,
                                  P, P, P, P, P, P],
            "oracle_interp_spread": [i64, i32, P, P, f64, P, i32, i32, P],
            "oracle_interp_rows": [i64, i32, P, P, f64, P, i32, i32, i32,
                                   P, P, i64, P],
            "oracle_interp_gather": [i64, i32, P, P, f64, P, i32, i32, P, P],
            "oracle_update": [i64, i32, P, P, P, P, P, f64, f64, f64, f64,
                              f64, f64, i32],
        }
        for name, args in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int if name.startswith("oracle_interp") else None
        _lib.oracle_kl.restype = f64
        _lib.oracle_symmetrize.restype = i64
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data if a is not None else None


def threads() -> int:
    """OpenMP threads the oracle will use."""
    n = os.environ.get("OMP_NUM_THREADS")
    return int(n) if n else (os.cpu_count() or 1)


# ---------------------------------------------------------------- direct sums
def direct_sums(Y, rows=None, kind=KERNEL_TSNE):
    """Per-row h1 [r] and unnormalised repulsive numerators [r, s] by the direct
    O(N) sum per row.  ``rows`` None means every row."""
    Y = _f64(Y)
    n, s = Y.shape
    if rows is None:
        r = None
        nr = n
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = r.shape[0]
    h1 = np.empty(nr)
    num = np.empty((nr, s))
    _load().oracle_direct_sums(n, s, _ptr(Y), kind, _ptr(r), nr, _ptr(h1), _ptr(num))
    return h1, num


def direct_rep(Y, kind=KERNEL_TSNE):
    """(F_rep [N, s], Z) by the O(N^2) definitions."""
    Y = _f64(Y)
    n, s = Y.shape
    F = np.empty((n, s))
    Z = ctypes.c_double()
    _load().oracle_direct_rep(n, s, _ptr(Y), kind, _ptr(F), ctypes.addressof(Z))
    return F, Z.value


def attr(Y, P):
    """F_attr [N, s] over the CSR P (``inputs.CSR``)."""
    Y = _f64(Y)
    n, s = Y.shape
    rp = np.ascontiguousarray(P.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(P.col, dtype=np.int32)
    val = _f64(P.val)
    F = np.empty((n, s))
    _load().oracle_attr(n, s, _ptr(Y), _ptr(rp), _ptr(col), _ptr(val), _ptr(F))
    return F


def kl(Y, P, Z=None):
    """KL(P || Q) over the non-zeros of P with q_ij = K1(y_i, y_j) / Z
    (Section 1.1).  Z defaults to the direct sum over ordered pairs."""
    Y = _f64(Y)
    n, s = Y.shape
    if Z is None:
        Z = direct_rep(Y)[1]
    rp = np.ascontiguousarray(P.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(P.col, dtype=np.int32)
    val = _f64(P.val)
    return float(_load().oracle_kl(n, s, _ptr(Y), _ptr(rp), _ptr(col), _ptr(val), float(Z)))


# ---------------------------------------------------------------- affinities
def knn(X, k):
    """Exact k nearest neighbours (self excluded, ties by index): (idx int32
    [n, k], squared distances [n, k]) in ascending order."""
    X = _f64(X)
    n, dim = X.shape
    if not 0 < k < n:
        raise ValueError("need 0 < k < n")
    idx = np.empty((n, k), np.int32)
    d2 = np.empty((n, k))
    _load().oracle_knn(n, dim, _ptr(X), int(k), _ptr(idx), _ptr(d2))
    return idx, d2


def knn_rows(X, rows, k):
    """knn for the listed rows only: (idx int32 [r, k], dist2 [r, k])."""
    X = _f64(X)
    n, dim = X.shape
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    idx = np.empty((r.shape[0], k), np.int32)
    d2 = np.empty((r.shape[0], k))
    _load().oracle_knn_rows(n, dim, _ptr(X), int(k), _ptr(r), r.shape[0], _ptr(idx), _ptr(d2))
    return idx, d2


def perplexity(dist2, perp):
    """Conditional affinities [n, k] and bandwidths beta [n] by bisection to
    the target perplexity (Section 1.1)."""
    d2 = _f64(dist2)
    n, k = d2.shape
    p = np.empty((n, k))
    beta = np.empty(n)
    _load().oracle_perplexity(n, k, _ptr(d2), float(perp), _ptr(beta), _ptr(p))
    return p, beta


def symmetrize(idx, p):
    """Joint P = (P_cond + P_cond^T) / (2N) as CSR (row_ptr int64, col int32,
    val float64), columns ascending in each row."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    p = _f64(p)
    n, k = idx.shape
    rp = np.empty(n + 1, np.int64)
    col = np.empty(2 * n * k, np.int32)
    val = np.empty(2 * n * k)
    nnz = _load().oracle_symmetrize(n, k, _ptr(idx), _ptr(p), _ptr(rp), _ptr(col), _ptr(val))
    return rp, col[:nnz].copy(), val[:nnz].copy()


# ---------------------------------------------------------------- geometry
def geometry(Y, policy, min_intervals=1, interval_width=1.0, rect=False):
    """(origin [s], w_int, N_int) of the box policy; N_int is an int for the
    square box, or a tuple of per-axis counts with ``rect``."""
    Y = _f64(Y)
    n, s = Y.shape
    o = np.empty(s)
    w = ctypes.c_double()
    m = np.zeros(s, dtype=np.int32)
    pol = POLICY_PAPER if policy in ("paper", POLICY_PAPER) else POLICY_FIXED
    _load().oracle_geometry(n, s, _ptr(Y), pol, int(min_intervals), float(interval_width),
                            int(bool(rect)), _ptr(o), ctypes.addressof(w), _ptr(m))
    return o, w.value, (tuple(int(x) for x in m) if rect else int(m[0]))


def _axes(n_int, s):
    """Per-axis interval counts as an int32 array of length s."""
    a = np.atleast_1d(np.asarray(n_int, dtype=np.int32))
    if a.shape[0] == 1:
        a = np.repeat(a, s)
    if a.shape[0] != s:
        raise ValueError("n_int must be one count or one per axis")
    return np.ascontiguousarray(a)


# ---------------------------------------------------------------- interpolation
def lagrange(p, t):
    L = np.empty(p)
    _load().oracle_lagrange(p, float(t), _ptr(L))
    return L


def grid_conv(W, h, kernel, kind=KERNEL_TSNE):
    """Step 2 directly on a 1-D [ng], 2-D [ng1, ng0] (index [g1, g0]) or 3-D
    [ng2, ng1, ng0] grid.  kernel: 1 = K1, 2 = K2, 3 / 4 / 5 = the odd kernels
    z_0 K2, z_1 K2, z_2 K2."""
    W = _f64(W)
    s = W.ndim
    ngv = np.array(W.shape[::-1], dtype=np.int32)         # [ng0(, ng1)]
    V = np.empty_like(W)
    _load().oracle_grid_conv(s, _ptr(ngv), float(h), kind, int(kernel), _ptr(W), _ptr(V))
    return V


def interp_rep(Y, origin, w_int, n_int, p=3, form=FORM_A, kind=KERNEL_TSNE,
               want_grids=False):
    """Interpolation scheme with direct Step 2.  n_int: one interval count
    (square box) or one per axis.  Returns a dict with F [N, s], Z,
    phi [N, P], h1 [N] and (``want_grids``) W [C, (ng1,) ng0], V [P, ...]."""
    Y = _f64(Y)
    n, s = Y.shape
    o = _f64(origin)
    ax = _axes(n_int, s)
    shape = tuple(int(x) * p for x in ax[::-1])           # (ng1,) ng0
    tn = int(np.prod(shape))
    nc = s + 1 if form == FORM_A else (s + 2 if form == FORM_B else 1)
    npot = s + 1 if form == FORM_V else s + 2
    F = np.empty((n, s))
    Z = ctypes.c_double()
    phi = np.empty((n, npot))
    h1 = np.empty(n)
    W = np.empty((nc, tn)) if want_grids else None
    V = np.empty((npot, tn)) if want_grids else None
    rc = _load().oracle_interp_rep(n, s, _ptr(Y), _ptr(o), float(w_int), _ptr(ax), int(p),
                                   int(form), int(kind), _ptr(F), ctypes.addressof(Z),
                                   _ptr(W), _ptr(V), _ptr(phi), _ptr(h1))
    if rc != 0:
        raise ValueError("oracle_interp_rep: bad arguments")
    out = dict(F=F, Z=Z.value, phi=phi, h1=h1)
    if want_grids:
        out["W"] = W.reshape((nc,) + shape)
        out["V"] = V.reshape((npot,) + shape)
    return out


def interp_spread(Y, origin, w_int, n_int, p=3, form=FORM_A):
    Y = _f64(Y)
    n, s = Y.shape
    ax = _axes(n_int, s)
    nc = s + 1 if form == FORM_A else (s + 2 if form == FORM_B else 1)
    W = np.empty((nc, int(np.prod(ax * p))))
    rc = _load().oracle_interp_spread(n, s, _ptr(Y), _ptr(_f64(origin)), float(w_int),
                                      _ptr(ax), int(p), int(form), _ptr(W))
    if rc != 0:
        raise ValueError("oracle_interp_spread: bad arguments")
    return W


def interp_rows(Y, origin, w_int, n_int, rows, W, p=3, form=FORM_A, kind=KERNEL_TSNE):
    """phi [len(rows), P] at the listed points (P = s+2, or s+1 for form V),
    node values by direct sums."""
    Y = _f64(Y)
    n, s = Y.shape
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    phi = np.empty((r.shape[0], s + 1 if form == FORM_V else s + 2))
    rc = _load().oracle_interp_rows(n, s, _ptr(Y), _ptr(_f64(origin)), float(w_int),
                                    _ptr(_axes(n_int, s)), int(p), int(form), int(kind), _ptr(_f64(W)),
                                    _ptr(r), r.shape[0], _ptr(phi))
    if rc != 0:
        raise ValueError("oracle_interp_rows: bad arguments")
    return phi


def _kernel_fn(kind, kernel):
    """Kernel of Step 2 as a function of the lag vector (z_0(, z_1)) in Y units:
    1 = K1, 2 = K2, 3 / 4 = the odd kernels z_0 K2, z_1 K2 (the pair of
    Section 2, eq. (kers); KERNEL_POLY is the polynomial test family)."""
    def k(z):
        r2 = sum(c * c for c in z)
        if kind == KERNEL_TSNE:
            k1 = 1.0 / (1.0 + r2)
            k2 = k1 * k1
        else:
            k2 = 2.0 + r2 / 8.0
            k1 = (1.0 + r2) * k2
        if kernel == 1:
            return k1
        if kernel == 2:
            return k2
        return z[kernel - 3] * k2
    return k


def grid_conv_fft(W, h, kernel, kind=KERNEL_TSNE):
    """Step 2 (eq. (equikereval2)) as a circulant convolution by FFT (Section
    2.2): the Toeplitz kernel matrix of an ng-node axis is embedded in a
    circulant of length 2 ng per axis, lag j at index j mod 2 ng (the lag ng
    is never used by an ng-node grid and is set to zero), and applied with
    numpy's FFT in FP64.  Same grid layout and kernels as ``grid_conv``, which
    it must reproduce to rounding."""
    W = _f64(W)
    shape = W.shape                                       # (ng1,) ng0
    Lx = tuple(2 * g for g in shape)
    # lag of each circulant index along each axis: j for j < ng, j - 2 ng above
    lags = []
    for g, L in zip(shape, Lx):
        j = np.arange(L)
        lag = np.where(j < g, j, j - L).astype(np.float64)
        lag[g] = 0.0
        lags.append(lag)
    grids = np.meshgrid(*lags, indexing="ij")             # axis order (g2, g1,) g0
    z = [h * grids[W.ndim - 1 - d] for d in range(W.ndim)]  # (z_0, z_1, z_2)
    T = np.asarray(_kernel_fn(kind, kernel)(z), dtype=np.float64)
    if T.ndim == 0:
        T = np.full(Lx, float(T))
    # the unused lag ng of each axis carries no kernel value
    for ax, g in enumerate(shape):
        idx = [slice(None)] * W.ndim
        idx[ax] = g
        T[tuple(idx)] = 0.0
    Wp = np.zeros(Lx)
    Wp[tuple(slice(0, g) for g in shape)] = W
    axes = tuple(range(W.ndim))
    V = np.fft.irfftn(np.fft.rfftn(Wp, axes=axes) * np.fft.rfftn(T, axes=axes), s=Lx, axes=axes)
    return np.ascontiguousarray(V[tuple(slice(0, g) for g in shape)])


def interp_gather(Y, origin, w_int, n_int, V, p=3):
    """Step 3 alone: phi [N, P] at every point from the potential grids
    V [P, (ng1,) ng0] (``interp_rep(want_grids=True)['V']`` layout)."""
    Y = _f64(Y)
    n, s = Y.shape
    V = _f64(V)
    npot = V.shape[0]
    phi = np.empty((n, npot))
    rc = _load().oracle_interp_gather(n, s, _ptr(Y), _ptr(_f64(origin)), float(w_int),
                                      _ptr(_axes(n_int, s)), int(p), int(npot),
                                      _ptr(np.ascontiguousarray(V.reshape(npot, -1))), _ptr(phi))
    if rc != 0:
        raise ValueError("oracle_interp_gather: bad arguments")
    return phi


def _pots(form, s):
    """(kernel, charge) of each potential, in the order of interp_rep."""
    if form == FORM_V:
        return [(1, 0)] + [(3 + d, 0) for d in range(s)]
    first = (1, 0) if form == FORM_A else (2, s + 1)
    return [first, (2, 0)] + [(2, 1 + d) for d in range(s)]


def interp_rep_fft(Y, origin, w_int, n_int, p=3, form=FORM_A, kind=KERNEL_TSNE,
                   want_grids=False):
    """``interp_rep`` with Step 2 by FFT (``grid_conv_fft``) instead of the
    direct double sum, for grids too large for the direct sum (N = 1e6 boxes):
    Step 1 ``interp_spread``, Step 2 ``grid_conv_fft`` per potential, Step 3
    ``interp_gather``, the Appendix assembly (``assemble_rows``), Z = sum h1
    - N K1(0) and F = numerator / Z.  Same outputs as ``interp_rep``."""
    Y = _f64(Y)
    n, s = Y.shape
    ax = _axes(n_int, s)
    shape = tuple(int(x) * p for x in ax[::-1])
    Wf = interp_spread(Y, origin, w_int, ax, p, form)
    W = Wf.reshape((Wf.shape[0],) + shape)
    h = w_int / p
    V = np.stack([grid_conv_fft(W[c], h, k, kind) for k, c in _pots(form, s)])
    phi = interp_gather(Y, origin, w_int, ax, V, p)
    h1, num = assemble_rows(Y, origin, w_int, ax, phi, form)
    k10 = 1.0 if kind == KERNEL_TSNE else 2.0
    Z = float(h1.sum() - n * k10)
    out = dict(F=num / Z, Z=Z, phi=phi, h1=h1)
    if want_grids:
        out["W"] = W
        out["V"] = V
    return out


def centre(origin, w_int, n_int):
    """Box centre used to centre the charges (n_int: one count or per axis)."""
    o = _f64(origin)
    return o + 0.5 * _axes(n_int, o.shape[0]).astype(np.float64) * w_int


def assemble_rows(Y, origin, w_int, n_int, phi, form=FORM_A):
    """Unnormalised (h1 [r], numerator [r, s]) for rows whose potentials are
    ``phi`` (Appendix assembly; see oracle_interp_rep)."""
    Y = _f64(Y)
    s = Y.shape[1]
    yc = Y - centre(origin, w_int, n_int)
    if form == FORM_V:
        return phi[:, 0].copy(), phi[:, 1:1 + s].copy()
    if form == FORM_A:
        h1 = phi[:, 0].copy()
    else:
        r2 = (yc * yc).sum(1)
        h1 = (1.0 + r2) * phi[:, 1] - 2.0 * (yc * phi[:, 2:2 + s]).sum(1) + phi[:, 0]
    num = yc * phi[:, 1:2] - phi[:, 2:2 + s]
    return h1, num


# ---------------------------------------------------------------- update
def update(Y, uY, gains, Fattr, Frep, alpha, mom, eta, gain_inc=0.2, gain_dec=0.8,
           gain_min=0.01, recentre=True):
    """One descent step; returns new (Y, uY, gains) as float64 arrays."""
    Y = _f64(Y).copy()
    uY = _f64(uY).copy()
    gains = _f64(gains).copy()
    n, s = Y.shape
    _load().oracle_update(n, s, _ptr(Y), _ptr(uY), _ptr(gains), _ptr(_f64(Fattr)),
                          _ptr(_f64(Frep)), float(alpha), float(mom), float(eta),
                          float(gain_inc), float(gain_dec), float(gain_min), int(bool(recentre)))
    return Y, uY, gains


def schedule(it, ee_alpha=12.0, ee_stop=250, le_alpha=1.0, le_start=1 << 30,
             mom0=0.5, mom1=0.8, mom_switch=250):
    """(alpha, momentum) at iteration ``it`` (early exaggeration Section 1.2,
    late exaggeration Section 4; the momentum switch is not in the paper)."""
    if it >= le_start:
        alpha = le_alpha
    elif it < ee_stop:
        alpha = ee_alpha
    else:
        alpha = 1.0
    mom = mom0 if it < mom_switch else mom1
    return alpha, mom
