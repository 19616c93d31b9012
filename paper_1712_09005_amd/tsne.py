"""Python binding of the C ABI in ``include/tsne.h`` (ctypes).

Argument marshalling only: every step of the gradient runs in the HIP kernels
of ``libtsne_mi355x.so``.  PyTorch provides device memory (workspace, outputs)
and the stream.  There is no fallback: without the built library (or without a
GPU) the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsne_mi355x.so")

F32, F64 = 0, 1
STATIC_SCRATCH_BYTES = 128 << 20     # TSNE_STATIC_SCRATCH_BYTES of include/tsne.h
GRID_PAPER, GRID_FIXED = 0, 1
FORM_A, FORM_B, FORM_V = 0, 1, 2
_FORMS = {"A": FORM_A, "B": FORM_B, "V": FORM_V, FORM_A: FORM_A, FORM_B: FORM_B, FORM_V: FORM_V}


def form_code(form):
    """Form name ("A", "B", "V") or code to the tsne_form code."""
    if form not in _FORMS:
        raise ValueError("form must be one of A, B, V")
    return _FORMS[form]

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported configuration",
          3: "workspace", 4: "capacity exceeded", 5: "non-finite coordinate",
          6: "HIP runtime error", 7: "invalid state", 8: "internal device error"}


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("s", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("p", ctypes.c_int32), ("policy", ctypes.c_int32), ("form", ctypes.c_int32),
                ("min_intervals", ctypes.c_int32), ("max_intervals", ctypes.c_int32),
                ("interval_width", ctypes.c_double), ("nnz", ctypes.c_int64),
                ("lanes_per_row", ctypes.c_int32), ("points_per_lane", ctypes.c_int32),
                ("attr_slabs", ctypes.c_int32), ("attr_layout", ctypes.c_int32),
                ("rect", ctypes.c_int32), ("keep_h1", ctypes.c_int32)]


class Sched(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("mom0", ctypes.c_double), ("mom1", ctypes.c_double),
                ("mom_switch", ctypes.c_int32), ("ee_alpha", ctypes.c_double),
                ("ee_stop", ctypes.c_int32), ("le_alpha", ctypes.c_double),
                ("le_start", ctypes.c_int32), ("gain_inc", ctypes.c_double),
                ("gain_dec", ctypes.c_double), ("gain_min", ctypes.c_double),
                ("recentre", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_int", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("fft_len", ctypes.c_int32), ("iter", ctypes.c_int32),
                ("max_intervals", ctypes.c_int32), ("origin", ctypes.c_double * 2),
                ("w_int", ctypes.c_double), ("box_side", ctypes.c_double), ("Z", ctypes.c_double),
                ("n_int_y", ctypes.c_int32), ("n_nodes_y", ctypes.c_int32),
                ("fft_len_y", ctypes.c_int32), ("origin_z", ctypes.c_double)]


@dataclass
class Schedule:
    """Descent schedule (see tsne_sched in include/tsne.h)."""
    eta: float = 200.0
    mom0: float = 0.5
    mom1: float = 0.8
    mom_switch: int = 250
    ee_alpha: float = 12.0
    ee_stop: int = 250
    le_alpha: float = 1.0
    le_start: int = 1 << 30
    gain_inc: float = 0.2
    gain_dec: float = 0.8
    gain_min: float = 0.01
    recentre: bool = True

    def c(self) -> Sched:
        return Sched(self.eta, self.mom0, self.mom1, self.mom_switch, self.ee_alpha, self.ee_stop,
                     self.le_alpha, self.le_start, self.gain_inc, self.gain_dec, self.gain_min,
                     int(bool(self.recentre)))


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtsne_mi355x.so is not built; run __graft_entry__.build() "
                              "or python -m paper_1712_09005_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        sig = {
            "tsne_workspace_bytes": ([P], ctypes.c_size_t),
            "tsne_plan_create": ([P, P, ctypes.c_size_t, P, P], i32),
            "tsne_plan_destroy": ([P], i32),
            "tsne_bind_P": ([P, P, P, P], i32),
            "tsne_repulsive": ([P, P, P, P], i32),
            "tsne_repulsive_static": ([P, P, P, P, P], i32),
            "tsne_attractive": ([P, P, P], i32),
            "tsne_kl_divergence": ([P, P, P], i32),
            "tsne_knn": ([P, i64, i32, i32, P, P, P], i32),
            "tsne_perplexity": ([P, i64, i32, ctypes.c_double, P, P, P], i32),
            "tsne_symmetrize_workspace_bytes": ([i64, i32], ctypes.c_size_t),
            "tsne_symmetrize": ([P, P, i64, i32, P, ctypes.c_size_t, P, P, P, P, P], i32),
            "tsne_step": ([P, P, P, P, P, i32], i32),
            "tsne_run": ([P, P, P, P, P, i32, i32], i32),
            "tsne_query": ([P, P], i32),
            "tsne_debug_export": ([P, i32, P, P], i32),
            "tsne_status_str": ([i32], ctypes.c_char_p),
            "tsne_batch_workspace_bytes": ([i32], ctypes.c_size_t),
            "tsne_batch_create": ([i32, i32, i32, i32, i32, i32, P, ctypes.c_size_t, P, P], i32),
            "tsne_batch_destroy": ([P], i32),
            "tsne_batch_admit": ([P, P, P, ctypes.c_size_t, P, P, P, P, P, P, P, i32, i32, P], i32),
            "tsne_batch_tick": ([P, i32], i32),
            "tsne_batch_poll": ([P, i32, P, P], i32),
            "tsne_batch_retire": ([P, i32], i32),
            "tsne_pca_workspace_bytes": ([P], ctypes.c_size_t),
            "tsne_pca": ([P, P, P, P, P, P, P, ctypes.c_size_t, P], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class TsneError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (status %d)" % (what, STATUS.get(code, "?"), code))


def _check(code: int, what: str):
    if code != 0:
        raise TsneError(code, what)


def _dt(dtype) -> int:
    if dtype in (torch.float32, "f32", F32):
        return F32
    if dtype in (torch.float64, "f64", F64):
        return F64
    raise ValueError("dtype must be float32 or float64")


def make_desc(n, s, dtype=torch.float32, p=5, policy="fixed", form="A", min_intervals=1,
              max_intervals=512, interval_width=0.75, nnz=0, lanes_per_row=0,
              points_per_lane=0, attr_slabs=0, attr_layout=0, rect=False, keep_h1=False) -> Desc:
    pol = GRID_PAPER if policy in ("paper", GRID_PAPER) else GRID_FIXED
    frm = form_code(form)
    return Desc(int(n), int(s), _dt(dtype), int(p), pol, frm, int(min_intervals),
                int(max_intervals), float(interval_width), int(nnz), int(lanes_per_row),
                int(points_per_lane), int(attr_slabs), int(attr_layout), int(bool(rect)),
                int(bool(keep_h1)))


def workspace_bytes(desc: Desc) -> int:
    return int(lib().tsne_workspace_bytes(ctypes.byref(desc)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """One embedding: workspace, stream and the C plan.  Inputs may come from
    any stream; each call orders the plan's stream after the caller's current
    stream and the caller's current stream after the plan's work."""

    def __init__(self, n, s, dtype=torch.float32, p=5, policy="fixed", form="A",
                 min_intervals=1, max_intervals=512, interval_width=0.75, nnz=0,
                 lanes_per_row=0, points_per_lane=0, attr_slabs=0, attr_layout=0, device="cuda",
                 stream=None, rect=False, keep_h1=False):
        self.desc = make_desc(n, s, dtype, p, policy, form, min_intervals, max_intervals,
                              interval_width, nnz, lanes_per_row, points_per_lane, attr_slabs,
                              attr_layout, rect, keep_h1)
        self.n, self.s = int(n), int(s)
        self.dtype = torch.float32 if self.desc.dtype == F32 else torch.float64
        self.device = torch.device(device)
        if not torch.cuda.is_available():
            raise RuntimeError("the t-SNE library needs a GPU")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nbytes = workspace_bytes(self.desc)
        if nbytes == 0:
            raise TsneError(1, "tsne_workspace_bytes")
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        _check(lib().tsne_plan_create(ctypes.byref(self.desc), _ptr(self.ws), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(self._h)), "tsne_plan_create")
        self._P = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self.stream.synchronize()
                lib().tsne_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # stream ordering around each call
    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _vec(self, t, name):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or \
                t.numel() != self.n * self.s:
            raise ValueError("%s must be a contiguous %s tensor with n*s elements on %s"
                             % (name, self.dtype, self.device))

    def bind_P(self, row_ptr, col, val):
        if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != self.dtype:
            raise ValueError("P must be (int64 row_ptr, int32 col, %s val)" % self.dtype)
        if tuple(row_ptr.shape) != (self.n + 1,) or col.dim() != 1 or \
                tuple(val.shape) != tuple(col.shape) or col.numel() != self.desc.nnz:
            raise ValueError("P must have row_ptr [n+1] and col, val [nnz] with nnz = %d"
                             % self.desc.nnz)
        for t in (row_ptr, col, val):
            if t.device != self.device or not t.is_contiguous():
                raise ValueError("P arrays must be contiguous on the plan's device")
        self._enter()
        _check(lib().tsne_bind_P(self._h, _ptr(row_ptr), _ptr(col), _ptr(val)), "tsne_bind_P")
        self._P = (row_ptr, col, val)

    def repulsive(self, Y, F=None, Z=None):
        self._vec(Y, "Y")
        with torch.cuda.stream(self.stream):
            if F is None:
                F = torch.empty_like(Y)
            if Z is None:
                Z = torch.empty(1, dtype=torch.float64, device=self.device)
        self._enter()
        _check(lib().tsne_repulsive(self._h, _ptr(Y), _ptr(F), _ptr(Z)), "tsne_repulsive")
        self._leave()
        return F, Z

    def attractive(self, Y, F=None):
        self._vec(Y, "Y")
        with torch.cuda.stream(self.stream):
            if F is None:
                F = torch.empty_like(Y)
        self._enter()
        _check(lib().tsne_attractive(self._h, _ptr(Y), _ptr(F)), "tsne_attractive")
        self._leave()
        return F

    def kl_divergence(self, Y, out=None):
        """KL(P || Q) at Y as a one-element float64 device tensor."""
        self._vec(Y, "Y")
        with torch.cuda.stream(self.stream):
            if out is None:
                out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._enter()
        _check(lib().tsne_kl_divergence(self._h, _ptr(Y), _ptr(out)), "tsne_kl_divergence")
        self._leave()
        return out

    def step(self, Y, uY, gains, sched: Schedule, it: int):
        for t, nm in ((Y, "Y"), (uY, "uY"), (gains, "gains")):
            self._vec(t, nm)
        sc = (sched if sched is not None else Schedule()).c()
        self._enter()
        _check(lib().tsne_step(self._h, _ptr(Y), _ptr(uY), _ptr(gains), ctypes.byref(sc), int(it)),
               "tsne_step")
        self._leave()

    def run(self, Y, uY, gains, sched: Schedule, it0: int, n_it: int):
        for t, nm in ((Y, "Y"), (uY, "uY"), (gains, "gains")):
            self._vec(t, nm)
        sc = (sched if sched is not None else Schedule()).c()
        self._enter()
        _check(lib().tsne_run(self._h, _ptr(Y), _ptr(uY), _ptr(gains), ctypes.byref(sc),
                              int(it0), int(n_it)), "tsne_run")
        self._leave()

    def query(self) -> dict:
        st = Stats()
        _check(lib().tsne_query(self._h, ctypes.byref(st)), "tsne_query")
        return dict(status=st.status, n_int=st.n_int, n_nodes=st.n_nodes, fft_len=st.fft_len,
                    iter=st.iter, max_intervals=st.max_intervals,
                    origin=(st.origin[0], st.origin[1]), w_int=st.w_int,
                    box_side=st.box_side, Z=st.Z, n_int_y=st.n_int_y, n_nodes_y=st.n_nodes_y,
                    fft_len_y=st.fft_len_y, origin_z=st.origin_z)

    def export(self, what: int):
        """Internal array of the last iteration as a flat host buffer (bytes)."""
        nb = ctypes.c_size_t(0)
        _check(lib().tsne_debug_export(self._h, int(what), None, ctypes.byref(nb)), "export")
        buf = (ctypes.c_char * nb.value)()
        _check(lib().tsne_debug_export(self._h, int(what), buf, ctypes.byref(nb)), "export")
        return bytes(buf)


def repulsive_static(Y, desc: Desc, F=None, Z=None, stream=None):
    """tsne_repulsive_static: the repulsion of desc at Y with the plan's
    workspace in the library's fixed device scratch (nothing is allocated by
    the call; F and Z may be passed in).  Returns (F_rep, Z)."""
    n, s = int(desc.n), int(desc.s)
    dt = torch.float32 if desc.dtype == F32 else torch.float64
    if Y.dtype != dt or not Y.is_cuda or not Y.is_contiguous() or Y.numel() != n * s:
        raise ValueError("Y must be a contiguous %s GPU tensor with n*s elements" % dt)
    st = stream if stream is not None else torch.cuda.current_stream(Y.device)
    with torch.cuda.stream(st):
        if F is None:
            F = torch.empty_like(Y)
        if Z is None:
            Z = torch.empty(1, dtype=torch.float64, device=Y.device)
    _check(lib().tsne_repulsive_static(ctypes.byref(desc), _ptr(Y), _ptr(F), _ptr(Z),
                                       ctypes.c_void_p(st.cuda_stream)), "tsne_repulsive_static")
    return F, Z


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream)


def knn(X, k, stream=None):
    """Exact k nearest neighbours of the rows of X (contiguous FP32 [n, dim]
    on a GPU): (idx int32 [n, k], dist2 float32 [n, k]) in ascending order."""
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_cuda or not X.is_contiguous():
        raise ValueError("X must be a contiguous float32 [n, dim] GPU tensor")
    n, dim = X.shape
    st = stream if stream is not None else torch.cuda.current_stream(X.device)
    with torch.cuda.stream(st):
        idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
        d2 = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check(lib().tsne_knn(_ptr(X), n, dim, int(k), _ptr(idx), _ptr(d2), _stream_ptr(st)), "tsne_knn")
    return idx, d2


def perplexity(dist2, perp, stream=None, want_beta=False):
    """Conditional affinities [n, k] (float32) by bisection to the perplexity."""
    if dist2.dtype != torch.float32 or dist2.dim() != 2 or not dist2.is_contiguous():
        raise ValueError("dist2 must be a contiguous float32 [n, k] GPU tensor")
    n, k = dist2.shape
    st = stream if stream is not None else torch.cuda.current_stream(dist2.device)
    with torch.cuda.stream(st):
        p = torch.empty_like(dist2)
        beta = torch.empty(n, dtype=torch.float64, device=dist2.device) if want_beta else None
    _check(lib().tsne_perplexity(_ptr(dist2), n, k, float(perp), _ptr(p), _ptr(beta),
                                 _stream_ptr(st)), "tsne_perplexity")
    return (p, beta) if want_beta else p


def symmetrize(idx, p, stream=None):
    """Joint CSR P from conditional rows: (row_ptr int64 [n+1], col int32
    [nnz], val float32 [nnz]) on the GPU."""
    if idx.dtype != torch.int32 or p.dtype != torch.float32 or idx.shape != p.shape or \
            not idx.is_contiguous() or not p.is_contiguous():
        raise ValueError("idx int32 and p float32 of one shape [n, k], contiguous")
    n, k = idx.shape
    dev = idx.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    nb = int(lib().tsne_symmetrize_workspace_bytes(n, k))
    if nb == 0:
        raise TsneError(1, "tsne_symmetrize_workspace_bytes")
    with torch.cuda.stream(st):
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(2 * n * k, dtype=torch.int32, device=dev)
        val = torch.empty(2 * n * k, dtype=torch.float32, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(lib().tsne_symmetrize(_ptr(idx), _ptr(p), n, k, _ptr(ws), nb, _stream_ptr(st), _ptr(rp),
                                 _ptr(col), _ptr(val), _ptr(status)), "tsne_symmetrize")
    st.synchronize()
    if int(status.item()) != 0:
        raise TsneError(2, "tsne_symmetrize: a row exceeds 16384 entries")
    nnz = int(rp[n].item())
    return rp, col[:nnz].clone(), val[:nnz].clone()


def affinities(X, k=90, perp=30.0, stream=None):
    """Joint P (CSR on the GPU) from the points X: kNN, perplexity, symmetrise."""
    idx, d2 = knn(X, k, stream)
    p = perplexity(d2, perp, stream)
    return symmetrize(idx, p, stream)


class Batch:
    """Independent embeddings sharing every launch (tsne_batch_*)."""

    def __init__(self, max_slots, s=2, dtype=torch.float32, p=5, form="A", lanes_per_row=32,
                 device="cuda", stream=None):
        self.device = torch.device(device)
        self.lanes_per_row = int(lanes_per_row)
        self.dtype = torch.float32 if _dt(dtype) == F32 else torch.float64
        self.s, self.p = int(s), int(p)
        self.form = form_code(form)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nb = int(lib().tsne_batch_workspace_bytes(int(max_slots)))
        if nb == 0:
            raise TsneError(1, "tsne_batch_workspace_bytes")
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        _check(lib().tsne_batch_create(int(max_slots), self.s, _dt(self.dtype), self.p, self.form,
                                       self.lanes_per_row, _ptr(self.ws), nb,
                                       ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(self._h)), "tsne_batch_create")
        self.jobs = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self.stream.synchronize()
                lib().tsne_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    @staticmethod
    def footprint(n, nnz, s=2, dtype=torch.float32, p=5, policy="fixed", max_intervals=512,
                  interval_width=0.75, min_intervals=1, form="A"):
        """Device bytes a job holds: plan workspace plus Y, uY, gains and P."""
        d = make_desc(n, s, dtype, p, policy, form, min_intervals, max_intervals, interval_width, nnz,
                      lanes_per_row=32, attr_slabs=1, attr_layout=1)
        tsz = 4 if d.dtype == F32 else 8
        return workspace_bytes(d) + 3 * n * s * tsz + 8 * (n + 1) + (4 + tsz) * nnz

    def admit(self, Y, P, sched: Schedule, it0, n_it, policy="fixed", min_intervals=1,
              max_intervals=512, interval_width=0.75, uY=None, gains=None, points_per_lane=0):
        """Admit a job: Y (host or device), P = (row_ptr, col, val) arrays,
        optionally the uY and gains of a job being resumed.  Returns the slot;
        the job's tensors stay alive in ``self.jobs``."""
        n = Y.shape[0]
        row_ptr, col, val = P
        if len(Y.shape) != 2 or Y.shape[1] != self.s:
            raise ValueError("Y must be [n, %d]" % self.s)
        if tuple(row_ptr.shape) != (n + 1,) or len(col.shape) != 1 or \
                tuple(val.shape) != tuple(col.shape):
            raise ValueError("P must have row_ptr [n+1] and col, val [nnz]")
        # every slot shares one attraction launch: CSR rows, one slab
        d = make_desc(n, self.s, self.dtype, self.p, policy, self.form, min_intervals,
                      max_intervals, interval_width, int(col.shape[0]),
                      lanes_per_row=self.lanes_per_row, points_per_lane=points_per_lane,
                      attr_slabs=1, attr_layout=1)
        nbytes = workspace_bytes(d)
        if nbytes == 0:
            raise TsneError(1, "tsne_workspace_bytes")
        with torch.cuda.stream(self.stream):
            job = dict(
                ws=torch.empty(nbytes, dtype=torch.uint8, device=self.device),
                Y=torch.as_tensor(Y, dtype=self.dtype).to(self.device).contiguous(),
                rp=torch.as_tensor(row_ptr, dtype=torch.int64).to(self.device).contiguous(),
                col=torch.as_tensor(col, dtype=torch.int32).to(self.device).contiguous(),
                val=torch.as_tensor(val, dtype=self.dtype).to(self.device).contiguous())
            job["uY"] = torch.zeros_like(job["Y"]) if uY is None else \
                torch.as_tensor(uY, dtype=self.dtype).to(self.device).contiguous()
            job["gains"] = torch.ones_like(job["Y"]) if gains is None else \
                torch.as_tensor(gains, dtype=self.dtype).to(self.device).contiguous()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        slot = ctypes.c_int32(-1)
        sc = (sched if sched is not None else Schedule()).c()
        _check(lib().tsne_batch_admit(self._h, ctypes.byref(d), _ptr(job["ws"]), nbytes,
                                      _ptr(job["Y"]), _ptr(job["uY"]), _ptr(job["gains"]),
                                      _ptr(job["rp"]), _ptr(job["col"]), _ptr(job["val"]),
                                      ctypes.byref(sc), int(it0), int(n_it), ctypes.byref(slot)),
               "tsne_batch_admit")
        job["end"] = int(it0) + int(n_it)
        self.jobs[slot.value] = job
        return slot.value

    def tick(self, n=1):
        _check(lib().tsne_batch_tick(self._h, int(n)), "tsne_batch_tick")

    def poll(self, slot):
        it = ctypes.c_int32(0)
        st = ctypes.c_int32(0)
        _check(lib().tsne_batch_poll(self._h, int(slot), ctypes.byref(it), ctypes.byref(st)),
               "tsne_batch_poll")
        return it.value, st.value

    def retire(self, slot):
        _check(lib().tsne_batch_retire(self._h, int(slot)), "tsne_batch_retire")
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return self.jobs.pop(slot)
