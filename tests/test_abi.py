"""The C-ABI library loads and exports every entry point that include/*.h
declares; host-side argument checks work without a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def L():
    from paper_1712_09005_amd import tsne
    if not os.path.exists(tsne.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return tsne.lib()


def declared():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsne_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("tsne_plan_create", "tsne_repulsive", "tsne_attractive", "tsne_step",
                 "tsne_run", "tsne_batch_tick", "tsne_pca", "tsne_pca_workspace_bytes"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    for name in declared():
        assert hasattr(L, name), name


def test_workspace_bytes_and_argument_checks(L):
    from paper_1712_09005_amd import tsne
    d = tsne.make_desc(1_000_000, 2, p=5, max_intervals=320, nnz=90_000_000)
    nb = tsne.workspace_bytes(d)
    assert 100 << 20 < nb < 4 << 30
    # invalid descriptors: zero bytes
    for kw in (dict(n=1, s=2), dict(n=100, s=4), dict(n=100, s=2, p=9),
               dict(n=100, s=2, max_intervals=0)):
        n = kw.pop("n")
        s = kw.pop("s")
        assert tsne.workspace_bytes(tsne.make_desc(n, s, **kw)) == 0
    # 1-D plans need no 2-D FFT buffers
    assert tsne.workspace_bytes(tsne.make_desc(10_000, 1, max_intervals=600)) < \
        tsne.workspace_bytes(tsne.make_desc(10_000, 2, max_intervals=600))
    # plan creation rejects a missing or misaligned workspace before any device work
    out = ctypes.c_void_p()
    assert L.tsne_plan_create(ctypes.byref(d), None, 0, None, ctypes.byref(out)) == 3
    assert L.tsne_plan_create(ctypes.byref(d), ctypes.c_void_p(4096 + 8), 1 << 40, None,
                              ctypes.byref(out)) == 3
    bad = tsne.make_desc(100, 2, p=7)
    assert L.tsne_plan_create(ctypes.byref(bad), ctypes.c_void_p(4096), 1 << 30, None,
                              ctypes.byref(out)) == 2
    assert L.tsne_status_str(4) == b"box needs more intervals than max_intervals"
    assert L.tsne_batch_workspace_bytes(0) == 0 and L.tsne_batch_workspace_bytes(64) > 0


def test_fft_length_ladder(L):
    """Capacity determines the circulant length: the smallest even 2^a 3^b 5^c
    at least twice the node count."""
    from paper_1712_09005_amd import tsne
    small = tsne.workspace_bytes(tsne.make_desc(5000, 1, p=5, max_intervals=100))
    large = tsne.workspace_bytes(tsne.make_desc(5000, 1, p=5, max_intervals=1200))
    assert large > small
    # a circulant longer than the supported 12288 is refused
    assert tsne.workspace_bytes(tsne.make_desc(5000, 1, p=6, max_intervals=1100)) == 0


def test_pca_workspace_and_argument_checks(L):
    from paper_1712_09005_amd import pca
    d = pca.make_desc(1_000_000, 30_000, k=50, l=52, its=2)
    nb = L.tsne_pca_workspace_bytes(ctypes.byref(d))
    # X, X2 (n x l), Y, Q (m x l), l x l matrices and the partial sums (8 n x l)
    assert 2 * 1_000_000 * 52 * 8 + 10 * 30_000 * 52 * 8 < nb < \
        2 * 1_000_000 * 52 * 8 + 10 * 30_000 * 52 * 8 + (1 << 20)
    host = pca.make_desc(1_000_000, 30_000, k=50, l=52, its=2, a_host=True, b=1000)
    assert L.tsne_pca_workspace_bytes(ctypes.byref(host)) == nb + 1000 * 30_000 * 8
    for kw in (dict(k=0), dict(k=53), dict(l=30_000), dict(its=-1)):
        args = dict(k=50, l=52, its=2)
        args.update(kw)
        assert L.tsne_pca_workspace_bytes(ctypes.byref(pca.make_desc(1000, 30_000, **args))) == 0
    big = pca.make_desc(1000, 1000, k=50, l=65, its=2)
    assert L.tsne_pca_workspace_bytes(ctypes.byref(big)) == 0
    z = ctypes.c_void_p(4096)
    assert L.tsne_pca(ctypes.byref(big), z, z, z, z, z, z, 1 << 40, None) == 2
    assert L.tsne_pca(ctypes.byref(d), z, z, z, z, z, None, 0, None) == 3
    assert L.tsne_pca(ctypes.byref(d), z, z, z, z, z, ctypes.c_void_p(4096 + 64), 1 << 40, None) == 3
    bad = pca.make_desc(10, 10, k=5, l=12, its=1)
    assert L.tsne_pca(ctypes.byref(bad), z, z, z, z, z, z, 1 << 40, None) == 1


def test_static_repulsion_argument_checks(L):
    """tsne_repulsive_static validates its descriptor and the scratch size on
    the host, before any device work."""
    from paper_1712_09005_amd import tsne
    z = ctypes.c_void_p(4096)
    assert L.tsne_repulsive_static(None, z, z, None, None) == 1
    assert L.tsne_repulsive_static(ctypes.byref(tsne.make_desc(100, 4)), z, z, None, None) == 1
    assert L.tsne_repulsive_static(ctypes.byref(tsne.make_desc(100, 2, p=9)), z, z, None, None) == 2
    # a plan larger than the scratch array is refused with TSNE_E_WORKSPACE
    big = tsne.make_desc(1_000_000, 2, p=5, max_intervals=512)
    assert tsne.workspace_bytes(big) > tsne.STATIC_SCRATCH_BYTES
    assert L.tsne_repulsive_static(ctypes.byref(big), z, z, None, None) == 3
    # misaligned Y (FP32 2-D points are 8 bytes)
    small = tsne.make_desc(1000, 2, p=5, max_intervals=64)
    assert tsne.workspace_bytes(small) <= tsne.STATIC_SCRATCH_BYTES
    assert L.tsne_repulsive_static(ctypes.byref(small), ctypes.c_void_p(4100), z, None, None) == 1
