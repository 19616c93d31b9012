"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.

Tolerances (relative L2 over all N*s entries; per component where stated):
  - FP64 mode vs the interpolation oracle (same geometry, Step 2 direct):
    contract 1e-5; tested at 1e-9 (FFT rounding in double is ~1e-13).
  - FP32 mode vs the interpolation oracle: 1e-4.  The FFT's FP32 rounding is
    ~eps32 * log2(M) = 6e-8 * 12 relative to the grid's norm; the form-A
    numerator y'(d) h4 - h_{1+d} cancels by up to |y'| / (force scale), about
    50-100 on these boxes, so 1e-4 bounds it (observed 2-5e-5, larger in 1-D
    where |y'| reaches ~80 intervals).
  - default settings (p = 5, interval width 0.75) vs the direct O(N^2) sum:
    1e-3 (the accuracy target); the paper's settings of the 2,048-point check
    (p = 3, max(50, ceil(width)) intervals) reach only ~1.6e-2 and are tested
    at 3e-2.
  - attraction vs oracle: 1e-6 (FP32 terms, double accumulation).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1712_09005_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09005_amd import tsne
    tsne.lib()
    return tsne


DEV = "cuda:0"


def gpu_rep(T, Y, dtype=torch.float32, p=5, policy="fixed", w=0.75, min_int=1, max_int=256,
            form="A", P=None, ppl=0):
    n, s = Y.shape
    plan = T.Plan(n, s, dtype, p=p, policy=policy, form=form, min_intervals=min_int,
                  max_intervals=max_int, interval_width=w, nnz=(P.nnz if P is not None else 0),
                  points_per_lane=ppl, device=DEV)
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to(DEV, dtype)
    F, Z = plan.repulsive(Yt)
    torch.cuda.synchronize()
    st = plan.query()
    return plan, Yt, F.cpu().numpy().astype(np.float64), float(Z.item()), st


def oracle_rep(Y, p, policy, w, min_int, form="A"):
    Yd = np.asarray(Y, np.float64)
    o, ww, m = oracle.geometry(Yd, policy, min_int, w)
    code = {"A": oracle.FORM_A, "B": oracle.FORM_B, "V": oracle.FORM_V}[form]
    r = oracle.interp_rep(Yd, o, ww, m, p, code, want_grids=True)
    return (o, ww, m), r


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
@pytest.mark.parametrize("n", [2048, 1000, 3001])
def test_repulsion_2d_vs_interp_oracle(T, dtype, tol, n):
    print("case: repulsion 2-D n=%d %s" % (n, dtype), flush=True)
    Y = inputs.mixture_embedding(n, 2, 10, -30, 30, 2.0, seed=0)
    plan, _, F, Z, st = gpu_rep(T, Y, dtype, p=5, policy="fixed", w=0.75, max_int=128)
    assert st["status"] == 0, st
    (o, w, m), r = oracle_rep(Y, 5, "fixed", 0.75, 1)
    assert st["n_int"] == m and st["w_int"] == w
    np.testing.assert_array_equal(st["origin"], o)
    e = rel(F, r["F"])
    ez = abs(Z - r["Z"]) / r["Z"]
    print("  rel err F %.3e  Z %.3e" % (e, ez))
    assert e < tol and ez < tol
    for d in range(2):
        assert rel(F[:, d], r["F"][:, d]) < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grids_match_oracle(T, dtype):
    """Charge grids W on occupied cells and potential grids V on every node."""
    print("case: grids %s" % dtype, flush=True)
    n = 2500
    Y = inputs.mixture_embedding(n, 2, 6, -12, 12, 1.5, seed=5)
    plan, _, F, Z, st = gpu_rep(T, Y, dtype, p=4, policy="paper", min_int=20, max_int=64)
    (o, w, m), r = oracle_rep(Y, 4, "paper", 1.0, 20)
    assert st["n_int"] == m
    ng = m * 4
    ncap = 64 * 4
    npdt = np.float64 if dtype == torch.float64 else np.float32
    Wg = np.frombuffer(plan.export(0), npdt).reshape(3, ncap, ncap)[:, :ng, :ng]
    Vg = np.frombuffer(plan.export(1), npdt).reshape(4, ncap, ncap)[:, :ng, :ng]
    Yd = Y.astype(np.float64)
    cells = np.clip(np.floor((Yd - o) / w), 0, m - 1).astype(int)
    occ = np.zeros((m, m), bool)
    occ[cells[:, 1], cells[:, 0]] = True
    mask = np.kron(occ, np.ones((4, 4), bool))
    qs = 2.0 ** -(np.floor(np.log2(0.5 * m * w)) + 1)      # charge scale of the library
    scale = np.array([1.0, qs, qs])[:, None, None]
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    for c in range(3):
        assert rel(Wg[c][mask], (r["W"][c] * scale[c])[mask]) < tol, c
    vscale = np.array([1.0, 1.0, qs, qs])[:, None, None]
    for k in range(4):
        assert rel(Vg[k], r["V"][k] * vscale[k]) < (1e-9 if dtype == torch.float64 else 2e-5), k
    cs = np.frombuffer(plan.export(3), np.int32)
    counts = np.bincount(cells[:, 1] * m + cells[:, 0], minlength=m * m)
    np.testing.assert_array_equal(np.diff(cs), counts)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-5)])
@pytest.mark.parametrize("n", [2048, 3001])
def test_repulsion_form_v_2d(T, dtype, tol, n):
    """Vector-kernel form against the oracle's form V on the same geometry.
    No cancellation in the numerators, so FP32 is held to 1e-5."""
    print("case: repulsion form V 2-D n=%d %s" % (n, dtype), flush=True)
    Y = inputs.mixture_embedding(n, 2, 10, -30, 30, 2.0, seed=1)
    _, _, F, Z, st = gpu_rep(T, Y, dtype, p=5, policy="fixed", w=0.75, max_int=128, form="V")
    assert st["status"] == 0, st
    (o, w, m), r = oracle_rep(Y, 5, "fixed", 0.75, 1, "V")
    assert st["n_int"] == m
    e = rel(F, r["F"])
    ez = abs(Z - r["Z"]) / r["Z"]
    print("  rel err F %.3e  Z %.3e" % (e, ez))
    assert e < tol and ez < tol
    for d in range(2):
        assert rel(F[:, d], r["F"][:, d]) < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, None)])
@pytest.mark.parametrize("form", ["A", "B", "V"])
@pytest.mark.parametrize("wide", [0, 1])
def test_rect_box_vs_oracle(T, dtype, tol, form, wide):
    """Rectangular box (per-axis interval counts and FFT lengths at equal
    spacing) on a flat cloud, wide along x or along y: geometry exactly as
    the oracle's, forces and Z against the oracle's rectangular scheme."""
    print("case: rect box %s form %s wide axis %d" % (dtype, form, wide), flush=True)
    Y = inputs.mixture_embedding(3001, 2, 8, -30, 30, 1.5, seed=4)
    Y[:, 1 - wide] *= 0.25                                     # the other axis a quarter as wide
    n = Y.shape[0]
    plan = T.Plan(n, 2, dtype, p=5, policy="fixed", interval_width=0.75, max_intervals=128,
                  form=form, rect=True, device=DEV)
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to(DEV, dtype)
    F, Z = plan.repulsive(Yt)
    torch.cuda.synchronize()
    st = plan.query()
    assert st["status"] == 0, st
    Yd = Y.astype(np.float64)
    o, w, m = oracle.geometry(Yd, "fixed", 1, 0.75, rect=True)
    assert (st["n_int"], st["n_int_y"]) == m and st["w_int"] == w
    np.testing.assert_array_equal(st["origin"], o)
    narrow = st["fft_len_y"] if wide == 0 else st["fft_len"]
    wide_len = st["fft_len"] if wide == 0 else st["fft_len_y"]
    assert narrow < wide_len
    code = {"A": oracle.FORM_A, "B": oracle.FORM_B, "V": oracle.FORM_V}[form]
    r = oracle.interp_rep(Yd, o, w, m, 5, code)
    F = F.cpu().numpy().astype(np.float64)
    e, ez = rel(F, r["F"]), abs(float(Z.item()) - r["Z"]) / r["Z"]
    print("  n_int %s, FFT %d x %d: rel err F %.2e Z %.2e" % (m, st["fft_len"], st["fft_len_y"], e, ez))
    if tol is None:
        tol = 1e-5 if form == "V" else 1e-4
    assert e < tol and ez < tol
    Fd, _ = oracle.direct_rep(Yd)
    assert rel(F, Fd) < 1e-3


def test_rect_on_square_box_is_the_square_path(T):
    """With equal extents on both axes the rectangular box is the square box:
    same geometry and FFT lengths, and the same forces up to the summation
    order inside a cell (the counting sort ranks points with atomics, so two
    runs of either path differ at rounding level; FP64 here)."""
    print("case: rect on a square box", flush=True)
    Y = inputs.mixture_embedding(2000, 2, 6, -20, 20, 1.5, seed=8)
    Y[0] = [Y[:, 0].min(), Y[:, 1].min()]
    side = np.ptp(Y, axis=0).max()
    Y[1] = Y[0] + side                                          # both axes exactly `side` wide
    outs = []
    for rect in (False, True):
        plan = T.Plan(Y.shape[0], 2, torch.float64, p=5, interval_width=0.75, max_intervals=128,
                      form="V", rect=rect, device=DEV)
        F, Z = plan.repulsive(torch.from_numpy(np.ascontiguousarray(Y)).to(DEV, torch.float64))
        torch.cuda.synchronize()
        st = plan.query()
        assert st["n_int"] == st["n_int_y"] and st["fft_len"] == st["fft_len_y"]
        outs.append((F.cpu().numpy(), float(Z.item()), st))
    assert outs[0][2]["n_int"] == outs[1][2]["n_int"] and outs[0][2]["origin"] == outs[1][2]["origin"]
    assert rel(outs[1][0], outs[0][0]) < 1e-13
    assert abs(outs[1][1] - outs[0][1]) < 1e-13 * outs[0][1]


@pytest.mark.parametrize("form", ["A", "V"])
@pytest.mark.parametrize("min_int", [1, 6])
def test_small_box_fixed_policy(T, form, min_int):
    """A box narrower than min_int intervals of the fixed width (the start of
    a run from a tiny random embedding): the intervals shrink to L / min_int
    on the device exactly as in the oracle, and the forces meet the accuracy
    target against the direct sum in both forms."""
    print("case: small box form %s min_int %d" % (form, min_int), flush=True)
    rng = np.random.default_rng(12)
    Y = (1e-2 * rng.standard_normal((3000, 2))).astype(np.float32)
    _, _, F, Z, st = gpu_rep(T, Y, torch.float32, p=5, policy="fixed", w=0.75, min_int=min_int,
                             max_int=64, form=form)
    assert st["status"] == 0
    (o, w, m), r = oracle_rep(Y, 5, "fixed", 0.75, min_int, form)
    assert st["n_int"] == m == min_int and st["w_int"] == w < 0.75
    np.testing.assert_array_equal(st["origin"], o)
    Fd, Zd = oracle.direct_rep(Y.astype(np.float64))
    e = rel(F, Fd)
    print("  vs direct %.2e, vs interpolation oracle %.2e" % (e, rel(F, r["F"])))
    assert e < 1e-3 and abs(Z - Zd) / Zd < 1e-3


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grids_form_v_match_oracle(T, dtype):
    """Form V: the one charge grid and the K1 and odd-kernel potential grids
    (no charge scaling: the charge is 1)."""
    print("case: grids form V %s" % dtype, flush=True)
    n = 2500
    Y = inputs.mixture_embedding(n, 2, 6, -12, 12, 1.5, seed=5)
    plan, _, F, Z, st = gpu_rep(T, Y, dtype, p=4, policy="paper", min_int=20, max_int=64, form="V")
    (o, w, m), r = oracle_rep(Y, 4, "paper", 1.0, 20, "V")
    assert st["n_int"] == m
    ng, ncap = m * 4, 64 * 4
    npdt = np.float64 if dtype == torch.float64 else np.float32
    Wg = np.frombuffer(plan.export(0), npdt).reshape(1, ncap, ncap)[:, :ng, :ng]
    Vg = np.frombuffer(plan.export(1), npdt).reshape(3, ncap, ncap)[:, :ng, :ng]
    Yd = Y.astype(np.float64)
    cells = np.clip(np.floor((Yd - o) / w), 0, m - 1).astype(int)
    occ = np.zeros((m, m), bool)
    occ[cells[:, 1], cells[:, 0]] = True
    mask = np.kron(occ, np.ones((4, 4), bool))
    assert rel(Wg[0][mask], r["W"][0][mask]) < (1e-10 if dtype == torch.float64 else 1e-5)
    for k in range(3):
        assert rel(Vg[k], r["V"][k]) < (1e-9 if dtype == torch.float64 else 2e-5), k


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("form", ["A", "B", "V"])
@pytest.mark.parametrize("s", [1, 2])
def test_repulsion_p_and_form(T, p, form, s):
    """Every node count the library accepts (2..6), every form, 1-D and 2-D,
    against the interpolation oracle in FP64 (and FP32 for the 2-D case)."""
    print("case: p=%d form %s s=%d" % (p, form, s), flush=True)
    Y = inputs.mixture_embedding(1500, s, 5, -10, 10, 1.0, seed=2)
    _, _, F, Z, st = gpu_rep(T, Y, torch.float64, p=p, policy="paper", min_int=20, max_int=64,
                             form=form)
    assert st["status"] == 0
    (o, w, m), r = oracle_rep(Y, p, "paper", 1.0, 20, form)
    assert st["n_int"] == m
    assert rel(F, r["F"]) < 1e-9 and abs(Z - r["Z"]) / r["Z"] < 1e-9
    if s == 2:
        _, _, F32, Z32, st = gpu_rep(T, Y, torch.float32, p=p, policy="paper", min_int=20,
                                     max_int=64, form=form)
        tol = 1e-5 if form == "V" else 1e-4
        assert rel(F32, r["F"]) < tol and abs(Z32 - r["Z"]) / r["Z"] < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
@pytest.mark.parametrize("form", ["A", "B", "V"])
def test_repulsion_1d(T, dtype, tol, form):
    print("case: 1-D %s %s" % (dtype, form), flush=True)
    Y = inputs.mixture_embedding(4000, 1, 12, -60, 60, 1.5, seed=0)
    _, _, F, Z, st = gpu_rep(T, Y, dtype, p=5, policy="fixed", w=0.75, max_int=256, form=form)
    assert st["status"] == 0
    (o, w, m), r = oracle_rep(Y, 5, "fixed", 0.75, 1, form)
    assert st["n_int"] == m
    assert rel(F, r["F"]) < tol and abs(Z - r["Z"]) / r["Z"] < tol


def test_c1_against_direct_sum(T):
    """The 2,048-point check: FP32 GPU against the direct O(N^2) sum, at the
    paper's settings and at the default settings."""
    print("case: c1 vs direct", flush=True)
    c1 = inputs.config_inputs("c1")
    Y, P = c1["Y"], c1["P"]
    Fd, Zd = oracle.direct_rep(Y.astype(np.float64))
    _, _, F, Z, st = gpu_rep(T, Y, torch.float32, p=3, policy="paper", min_int=50, max_int=128)
    e_paper = rel(F, Fd)
    _, _, F2, Z2, _ = gpu_rep(T, Y, torch.float32, p=5, policy="fixed", w=0.75, max_int=128)
    e_def = rel(F2, Fd)
    print("  paper settings %.3e (Z %.2e); default %.3e (Z %.2e)"
          % (e_paper, abs(Z - Zd) / Zd, e_def, abs(Z2 - Zd) / Zd))
    assert e_paper < 3e-2 and e_def < 1e-3
    assert abs(Z2 - Zd) / Zd < 1e-4
    for d in range(2):
        assert rel(F2[:, d], Fd[:, d]) < 1e-3
    # FP64 mode and the vector-kernel form at the default settings, per component
    for dt, form in ((torch.float64, "A"), (torch.float32, "V"), (torch.float64, "V")):
        _, _, F3, Z3, _ = gpu_rep(T, Y, dt, p=5, policy="fixed", w=0.75, max_int=128, form=form)
        print("  %s form %s: %.3e (Z %.2e)" % (dt, form, rel(F3, Fd), abs(Z3 - Zd) / Zd))
        assert abs(Z3 - Zd) / Zd < 1e-4
        for d in range(2):
            assert rel(F3[:, d], Fd[:, d]) < 1e-3


ATTR_LAYOUTS = [  # (lanes per row, slabs, layout): CSR rows, XCD slabs, LDS tiles
    (4, 1, 1), (8, 1, 1), (16, 1, 1), (32, 1, 1), (64, 1, 1), (4, 4, 1), (8, 4, 1), (16, 2, 1),
    (32, 8, 1), (0, 0, 2)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("lpr,slabs,layout", ATTR_LAYOUTS)
@pytest.mark.parametrize("n,s", [(3001, 2), (20011, 2), (9001, 1)])
def test_attraction(T, dtype, lpr, slabs, layout, n, s):
    """Every attraction layout against the oracle, with ragged row and tile
    counts (n not a multiple of any block size)."""
    print("case: attraction %s n=%d s=%d lpr=%d slabs=%d layout=%d" % (dtype, n, s, lpr, slabs, layout),
          flush=True)
    Y = inputs.mixture_embedding(n, s, 10, -30, 30, 2.0, seed=0)
    P = inputs.random_graph_P(n, 90, seed=1)
    plan = T.Plan(n, s, dtype, nnz=P.nnz, lanes_per_row=lpr, attr_slabs=slabs, attr_layout=layout,
                  max_intervals=128, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    Yt = torch.from_numpy(Y).to(DEV, dtype)
    Fa = plan.attractive(Yt).cpu().numpy()
    Pd = inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64))
    ref = oracle.attr(Y.astype(np.float64), Pd)
    assert rel(Fa, ref) < (1e-6 if dtype == torch.float32 else 1e-13)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("s", [1, 2])
def test_attraction_row_blocks_sparse(T, dtype, s):
    """The row-block sweep (layout 2) where whole row blocks and many rows have
    no non-zeros: rows 3000..8199 of 9000 have none, so with 64-row blocks at
    this n some 80 blocks sweep no window at all.  Those rows get exactly zero,
    the rest match the oracle, and a second call gives the same bits (the row
    sums are fixed point)."""
    print("case: attraction row blocks with empty blocks %s s=%d" % (dtype, s), flush=True)
    n = 9000
    rng = np.random.default_rng(11)
    live = np.concatenate([np.arange(0, 3000), np.arange(8200, n)])
    r = rng.choice(live, 40000)
    c = rng.choice(live, 40000)
    keep = r != c
    P = inputs._csr_from_edges(n, r[keep], c[keep], np.exp(-rng.uniform(0, 5, keep.sum())))
    Y = inputs.mixture_embedding(n, s, 10, -30, 30, 2.0, seed=2)
    plan = T.Plan(n, s, dtype, nnz=P.nnz, attr_layout=2, max_intervals=128, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    Yt = torch.from_numpy(Y).to(DEV, dtype)
    Fa1 = plan.attractive(Yt)
    Fa2 = plan.attractive(Yt)
    torch.cuda.synchronize()
    assert torch.equal(Fa1, Fa2)
    Fa = Fa1.cpu().numpy().reshape(n, s)
    ref = oracle.attr(Y.astype(np.float64), inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64)))
    ref = np.asarray(ref).reshape(n, s)
    assert np.all(Fa[3000:8200] == 0)
    assert rel(Fa, ref) < (1e-6 if dtype == torch.float32 else 1e-13)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("s", [1, 2])
def test_attraction_row_blocks_step_splits(T, dtype, s):
    """The row-block sweep cuts a tile's non-zeros into steps of 2048 (3072
    where a 32 KB window holds 8192 points: FP32 in 1-D).  Three tiles hold
    exactly two steps, one step and one non-zero, and one non-zero short of a
    step; the remaining rows get random non-zeros.  Against the oracle, and the
    same bits on a second call."""
    n = 20000
    el = 4 if dtype == torch.float32 else 8
    wpts = 32768 // (s * el)                         # points per column window
    step = 3072 if wpts >= 8192 else 2048
    bi = 64 * -(-(-(-n // 256)) // 64)               # rows per block at this n: 128
    print("case: attraction step splits %s s=%d step=%d" % (dtype, s, step), flush=True)
    rng = np.random.default_rng(17)
    rs, cs = [], []
    # windows past the first: no tile of these rows meets the diagonal
    wins = (1, 2, 1)
    for blk, win, cnt in ((0, wins[0], 2 * step), (1, wins[1], step + 1), (2, wins[2], step - 1)):
        r0, c0 = blk * bi, win * wpts
        ncol = min(wpts, n - c0)
        cells = rng.choice(bi * ncol, cnt, replace=False)
        r, c = r0 + cells // ncol, c0 + cells % ncol
        keep = r != c
        rs.append(r[keep])
        cs.append(c[keep])
    r = rng.integers(3 * bi, n, 40000)
    c = rng.integers(0, n, 40000)
    keep = r != c
    rs.append(r[keep])
    cs.append(c[keep])
    r, c = np.concatenate(rs), np.concatenate(cs)
    import scipy.sparse as sp
    a = sp.csr_matrix((np.exp(-rng.uniform(0, 5, r.size)), (r, c)), shape=(n, n))
    a.sum_duplicates()
    a.sort_indices()
    P = inputs.CSR(a.indptr.astype(np.int64), a.indices.astype(np.int32),
                   (a.data / a.data.sum()).astype(np.float32))
    tiles = [np.count_nonzero((P.col[P.row_ptr[k * bi]:P.row_ptr[(k + 1) * bi]] // wpts) == wins[k])
             for k in range(3)]
    assert tiles == [2 * step, step + 1, step - 1]
    Y = inputs.mixture_embedding(n, s, 10, -30, 30, 2.0, seed=3)
    plan = T.Plan(n, s, dtype, nnz=P.nnz, attr_layout=2, max_intervals=128, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    Yt = torch.from_numpy(Y).to(DEV, dtype)
    Fa1 = plan.attractive(Yt)
    Fa2 = plan.attractive(Yt)
    torch.cuda.synchronize()
    assert torch.equal(Fa1, Fa2)
    ref = oracle.attr(Y.astype(np.float64), inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64)))
    assert rel(Fa1.cpu().numpy(), ref) < (1e-6 if dtype == torch.float32 else 1e-13)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
@pytest.mark.parametrize("form", ["A", "V"])
def test_step_vs_oracle(T, dtype, tol, form):
    """One full iteration (repulsion, attraction, update) against the oracle
    composed step by step, in the early-exaggeration phase and after it."""
    n = 2048
    c1 = inputs.config_inputs("c1")
    Y, P = c1["Y"], c1["P"]
    plan = T.Plan(n, 2, dtype, p=5, policy="fixed", interval_width=0.75, max_intervals=128,
                  form=form, nnz=P.nnz, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    rng = np.random.default_rng(3)
    uY0 = rng.standard_normal((n, 2)) * 0.1
    g0 = 1.0 + rng.uniform(0, 0.5, (n, 2))
    for it in (0, 300):
        print("case: step it=%d %s form %s" % (it, dtype, form), flush=True)
        Yt = torch.from_numpy(Y).to(DEV, dtype)
        uY = torch.from_numpy(uY0).to(DEV, dtype)
        gains = torch.from_numpy(g0).to(DEV, dtype)
        sched = T.Schedule()
        plan.step(Yt, uY, gains, sched, it)
        torch.cuda.synchronize()
        st = plan.query()
        assert st["status"] == 0 and st["iter"] == it + 1
        Yd = Y.astype(np.float64)
        o, w, m = oracle.geometry(Yd, "fixed", 1, 0.75)
        r = oracle.interp_rep(Yd, o, w, m, 5, oracle.FORM_A if form == "A" else oracle.FORM_V)
        Fa = oracle.attr(Yd, inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64)))
        alpha, mom = oracle.schedule(it)
        Y1, u1, g1 = oracle.update(Yd, uY0, g0, Fa, r["F"], alpha, mom, 200.0)
        assert rel(uY.cpu().numpy(), u1) < tol
        assert rel(gains.cpu().numpy(), g1) < tol
        assert rel(Yt.cpu().numpy(), Y1) < tol


@pytest.mark.parametrize("form", ["A", "V"])
def test_run_matches_steps(T, form):
    """tsne_run (graph replay, device iteration counter) against the same
    iterations issued one tsne_step at a time."""
    print("case: run vs steps form %s" % form, flush=True)
    c1 = inputs.config_inputs("c1")
    Y, P = c1["Y"], c1["P"]
    n = Y.shape[0]
    outs = []
    for mode in ("steps", "run"):
        plan = T.Plan(n, 2, torch.float64, p=5, interval_width=0.75, max_intervals=256,
                      form=form, nnz=P.nnz, device=DEV)
        plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                    torch.from_numpy(P.val).to(DEV, torch.float64))
        Yt = torch.from_numpy(Y).to(DEV, torch.float64)
        uY = torch.zeros_like(Yt)
        gains = torch.ones_like(Yt)
        sched = T.Schedule(ee_stop=3, mom_switch=4)
        if mode == "steps":
            for it in range(8):
                plan.step(Yt, uY, gains, sched, it)
        else:
            plan.run(Yt, uY, gains, sched, 0, 8)
        torch.cuda.synchronize()
        st = plan.query()
        assert st["status"] == 0 and st["iter"] == 8
        outs.append(Yt.cpu().numpy())
    assert rel(outs[1], outs[0]) < 1e-9


def test_edge_two_points_and_coincident(T):
    print("case: edges", flush=True)
    Y = np.array([[0.3, -1.2], [2.1, 0.4]])
    _, _, F, Z, st = gpu_rep(T, Y, torch.float64, p=5, policy="paper", min_int=50, max_int=64)
    r2 = ((Y[0] - Y[1]) ** 2).sum()
    # interpolation at 50 intervals on a 1.8-wide box is accurate to ~1e-9
    assert abs(Z - 2 / (1 + r2)) / (2 / (1 + r2)) < 1e-7
    np.testing.assert_allclose(F[0], (Y[0] - Y[1]) / (2 * (1 + r2)), rtol=1e-6)
    Yc = np.full((777, 2), 3.25)
    _, _, F, Z, st = gpu_rep(T, Yc, torch.float32, p=5, policy="paper", min_int=50, max_int=64)
    assert st["status"] == 0
    assert np.abs(F).max() < 1e-6 and abs(Z - 777 * 776) / (777 * 776) < 1e-3


def test_status_capacity_and_nonfinite(T):
    print("case: status", flush=True)
    Y = inputs.mixture_embedding(1000, 2, 4, -40, 40, 1.0, seed=9)
    n = 1000
    plan = T.Plan(n, 2, torch.float32, p=3, policy="fixed", interval_width=1.0, max_intervals=16,
                  device=DEV)
    Yt = torch.from_numpy(Y).to(DEV)
    F = torch.full_like(Yt, 7.0)
    plan.repulsive(Yt, F)
    torch.cuda.synchronize()
    st = plan.query()
    assert st["status"] == 4
    assert torch.all(F == 7.0)             # nothing committed
    assert plan.query()["status"] == 0     # cleared by the query
    Y2 = Y.copy()
    Y2[17, 1] = np.nan
    plan2 = T.Plan(n, 2, torch.float32, p=3, policy="paper", min_intervals=20, max_intervals=128,
                   device=DEV)
    F2 = torch.full_like(Yt, 7.0)
    plan2.repulsive(torch.from_numpy(Y2).to(DEV), F2)
    torch.cuda.synchronize()
    assert plan2.query()["status"] == 5
    assert torch.all(F2 == 7.0)


def test_misaligned_point_arrays_rejected(T):
    # per-point arrays move as one vector per point: a pointer that is not
    # aligned to a whole point is refused on the host, before any launch
    print("case: misaligned point arrays", flush=True)
    import ctypes
    n = 1000
    plan = T.Plan(n, 2, torch.float32, p=3, max_intervals=64, device=DEV)
    buf = torch.zeros(2 * n + 2, dtype=torch.float32, device=DEV)
    good, bad = buf[:2 * n], buf[1:2 * n + 1]
    sc = T.Schedule().c()
    L = T.lib()
    P = ctypes.c_void_p
    assert L.tsne_step(plan._h, P(bad.data_ptr()), P(good.data_ptr()), P(good.data_ptr()),
                       ctypes.byref(sc), 0) == 1
    assert L.tsne_run(plan._h, P(good.data_ptr()), P(bad.data_ptr()), P(good.data_ptr()),
                      ctypes.byref(sc), 0, 3) == 1
    assert L.tsne_step(plan._h, P(good.data_ptr()), P(good.data_ptr()), P(bad.data_ptr()),
                       ctypes.byref(sc), 0) == 1
    assert L.tsne_repulsive(plan._h, P(bad.data_ptr()), P(good.data_ptr()), None) == 1
    torch.cuda.synchronize()
    assert torch.all(buf == 0)
