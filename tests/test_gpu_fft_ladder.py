"""Step 2's circulant convolution at every FFT length the library can pick.

The device chooses the circulant length M per iteration from the 4^a 3^b 5^c
ladder (a >= 1, M <= 12288), so every radix sequence the transforms support
is reached by some box.  With p = 2 nodes per interval and a box of exactly
M/4 unit intervals the node count is n = M/2 and the chosen length is M
itself, which lets each ladder length be forced in turn.  The potential
grids V (the FFT's output after the spectral product and the crop) are
compared in FP64 with the interpolation oracle: Step 2 summed directly in
1-D (every length, the two forms' even and odd kernels, at the exact
capacity and at the largest capacity, whose transforms use the most
threads), and by numpy's FFT (pinned to the direct sum on the CPU) in 2-D
for every length up to 2560, where rows and columns run in different
kernels; FP32 at every 1-D length."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

LADDER = sorted({4 ** a * 3 ** b * 5 ** c for a in range(1, 8) for b in range(10) for c in range(7)
                 if 4 ** a * 3 ** b * 5 ** c <= 12288})
FORMS = {"A": oracle.FORM_A, "V": oracle.FORM_V}


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09005_amd import tsne
    tsne.lib()
    return tsne


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _box(n_int, s, npts, seed):
    """Points spanning n_int - 1/2 in every dimension, so that a unit width
    gives exactly n_int intervals.  The coordinates are FP32 values, so the
    FP32 and FP64 plans and the oracle bin the same positions (a point moved
    across an interval boundary by rounding changes its node weights by the
    interpolation error, which at p = 2 is large)."""
    rng = np.random.default_rng(seed)
    L = n_int - 0.5
    Y = rng.uniform(0.0, L, size=(npts, s)).astype(np.float32)
    Y[0] = 0.0
    Y[1] = L
    return np.ascontiguousarray(Y.astype(np.float64))


def _gpu_V(T, Y, dtype, form, cap):
    n, s = Y.shape
    plan = T.Plan(n, s, dtype, p=2, policy="fixed", interval_width=1.0, min_intervals=1,
                  max_intervals=cap, form=form, device=DEV)
    plan.repulsive(torch.from_numpy(Y).to(DEV, dtype))
    torch.cuda.synchronize()
    st = plan.query()
    el = np.float32 if dtype == torch.float32 else np.float64
    V = np.frombuffer(plan.export(1), el)
    return st, V


def test_ladder_is_what_the_plans_accept(T):
    assert len(LADDER) == 69 and LADDER[0] == 4 and LADDER[-1] == 12288
    # the largest length is reached by the largest 1-D capacity at p = 2
    assert T.workspace_bytes(T.make_desc(1000, 1, p=2, max_intervals=3072)) > 0
    assert T.workspace_bytes(T.make_desc(1000, 1, p=2, max_intervals=3073)) == 0


def _largest_capacity(T, dtype):
    """Largest 1-D interval count at p = 2 whose plan fits (an FP64 transform
    of length M needs 16 (M + 1) bytes of LDS, so FP64 stops below 12288)."""
    cap = 3072
    while T.workspace_bytes(T.make_desc(1000, 1, dtype, p=2, max_intervals=cap)) == 0:
        cap -= 1
    return cap


@pytest.mark.parametrize("form", ["A", "V"])
def test_every_length_1d(T, form):
    caps = {dt: _largest_capacity(T, dt) for dt in (torch.float64, torch.float32)}
    assert caps[torch.float32] == 3072 and caps[torch.float64] >= 2500
    for M in LADDER:
        m = M // 4
        Y = _box(m, 1, 3000, seed=M)
        o, w, mo = oracle.geometry(Y, "fixed", 1, 1.0)
        assert mo == m
        r = oracle.interp_rep(Y, o, w, m, 2, FORMS[form], want_grids=True)
        cases = {(m, torch.float64, 1e-10), (caps[torch.float64], torch.float64, 1e-10),
                 (m, torch.float32, 2e-5), (caps[torch.float32], torch.float32, 2e-5)}
        for cap, dtype, tol in sorted(cases, key=lambda c: (str(c[1]), c[0])):
            if cap < m or cap > caps[dtype]:
                continue                     # FP64 lengths beyond its largest transform
            print("case: fft ladder 1-D M=%d form %s %s capacity %d" % (M, form, dtype, cap), flush=True)
            st, V = _gpu_V(T, Y, dtype, form, cap)
            assert st["status"] == 0 and st["n_int"] == m and st["fft_len"] == M, (M, st)
            n_cap = cap * 2
            Vg = V.reshape(-1, n_cap)[:, :2 * m]
            # the library scales the y charges by a power of two,
            # 2^-(floor(log2(box half-width)) + 1), undone at the assembly
            qs = 2.0 ** -(np.floor(np.log2(0.5 * m * w)) + 1)
            vscale = [1.0] * Vg.shape[0] if form == "V" else [1.0, 1.0, qs]
            for k in range(Vg.shape[0]):
                e = rel(Vg[k], r["V"][k] * vscale[k])
                assert e < tol, (M, cap, dtype, k, e)


def test_every_length_2d(T):
    for M in [x for x in LADDER if x <= 2560]:
        m = M // 4
        print("case: fft ladder 2-D M=%d" % M, flush=True)
        Y = _box(m, 2, 20000, seed=M + 1)
        o, w, mo = oracle.geometry(Y, "fixed", 1, 1.0)
        assert mo == m
        st, V = _gpu_V(T, Y, torch.float64, "V", m)
        assert st["status"] == 0 and st["n_int"] == m and st["fft_len"] == M, (M, st)
        ng = 2 * m
        W = oracle.interp_spread(Y, o, w, m, 2, oracle.FORM_V).reshape(ng, ng)
        Vg = V.reshape(3, ng, ng)
        for k, kern in enumerate((1, 3, 4)):             # K1 and the two odd kernels
            ref = oracle.grid_conv_fft(W, w / 2, kern)
            e = rel(Vg[k], ref)
            assert e < 1e-10, (M, k, e)
