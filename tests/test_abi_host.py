"""Host-side checks of the C ABI: the library loads without a GPU, exports every
symbol the header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mecuco.h")


def _lib():
    from paper_2606_06329_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libmecuco.so not built")
    return L


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(mc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mc_knn", "mc_curvature_fast", "mc_curvature_exact", "mc_curvature_backward",
              "mc_workspace_bytes", "mc_status_string", "mc_version"):
        assert f in names


def test_every_declared_symbol_is_exported():
    L = _lib()
    raw = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    assert set(L.EXPORTS) <= set(declared_functions())


def test_version_and_status_strings():
    L = _lib()
    assert L.lib().mc_version() == 100
    for st in range(9):
        assert len(L.status_string(st)) > 0
    assert L.status_string(99) == "unknown status"


def test_workspace_query():
    L = _lib()
    lib = L.lib()
    assert lib.mc_workspace_bytes(L.MC_OP_KNN, 20000, 784, 11, L.MC_FP32, 2) > 20000 * 784 * 4
    # the GEMM input copy shrinks with the element size (float32 > bf16 > fp8)
    w32, w16, w8 = (lib.mc_workspace_bytes(L.MC_OP_KNN, 20000, 784, 11, p, 2)
                    for p in (L.MC_FP32, L.MC_BF16, L.MC_FP8))
    assert w32 > w16 > w8 > 0
    assert lib.mc_workspace_bytes(L.MC_OP_KNN, 10, 4, 11, L.MC_FP32, 2) == 0     # k >= n
    assert lib.mc_workspace_bytes(L.MC_OP_KNN, 100, 4, 40, L.MC_FP32, 1) == 0    # k > 32
    assert lib.mc_workspace_bytes(L.MC_OP_KNN, 1000, 4, 20, L.MC_FP32, 4) == 0   # K' > 64
    assert lib.mc_workspace_bytes(7, 1000, 4, 20, L.MC_FP32, 1) == 0
    # 0 doubles as the support query of the on-chip limits
    assert lib.mc_workspace_bytes(L.MC_OP_EXACT, 1000, 784, 11, L.MC_FP32, 1) > 0
    assert lib.mc_workspace_bytes(L.MC_OP_EXACT, 1000, 4096, 32, L.MC_FP32, 1) == 0
    assert lib.mc_workspace_bytes(L.MC_OP_FAST, 1000, 64, 28, L.MC_FP64, 1) > 0
    assert lib.mc_workspace_bytes(L.MC_OP_FAST, 1000, 64, 29, L.MC_FP64, 1) == 0
    assert lib.mc_workspace_bytes(L.MC_OP_BACKWARD, 1000, 64, 16, L.MC_FP32, 1) > 0
    assert lib.mc_workspace_bytes(L.MC_OP_BACKWARD, 1000, 64, 17, L.MC_FP32, 1) == 0
    assert lib.mc_workspace_bytes(L.MC_OP_KNN, 1000, 64, 11, L.MC_FP64, 2) == 0


@pytest.mark.parametrize("n", [128, 129, 20000, 100000, 131072, 131073, 140000])
def test_knn_schedule_workspace(n):
    """The symmetric tile-pair schedule keeps one 64 KiB transposed score tile per unordered
    pair of 128-point tiles in the workspace; knn_symmetric mirrors the library's limit."""
    import paper_2606_06329_amd as P
    L = _lib()
    T = -(-n // 128)
    tiles = T * (T - 1) // 2 * 65536
    ws = L.lib().mc_workspace_bytes(L.MC_OP_KNN, n, 8, 4, L.MC_FP32, 2)
    assert P.knn_symmetric(n) == (ws > tiles > 0)
    assert P.knn_symmetric(n) == (2 <= T <= 1024)


def test_exact_support_boundary():
    """The documented example: at k = 11 exact mode holds m <= 1038 on chip."""
    L = _lib()
    from paper_2606_06329_amd import api
    assert api.exact_supported(1038, 11)
    assert not api.exact_supported(1039, 11)


FAKE = 0x100000  # never dereferenced: validation fails before any device access


@pytest.mark.parametrize("args,code", [
    (dict(X=None), 1), (dict(n=0), 1), (dict(m=0), 1), (dict(ldx=3), 1), (dict(k=1), 1),
    (dict(k=33), 1), (dict(k=100), 1), (dict(precision=7), 1), (dict(precision=2, rerank=1), 1),
    (dict(rerank=0), 1), (dict(rerank=5), 1), (dict(flags=8), 1), (dict(idx=None), 1),
    (dict(ws=None), 1), (dict(ws_bytes=16), 4), (dict(ws=FAKE + 8), 4),
    (dict(precision=1, rerank=1), 1), (dict(k=20, rerank=4), 1), (dict(n=2**31), 2),
    (dict(precision=3), 3),
])
def test_knn_rejects(args, code):
    L = _lib()
    a = dict(X=FAKE, n=100, m=4, ldx=4, k=5, precision=0, rerank=2, flags=0, idx=FAKE, ws=FAKE,
             ws_bytes=1 << 40)
    a.update(args)
    st = L.lib().mc_knn(a["X"], a["n"], a["m"], a["ldx"], a["k"], a["precision"], a["rerank"],
                        a["flags"], a["idx"], None, None, a["ws"], a["ws_bytes"], None)
    assert st == code


@pytest.mark.parametrize("args,code", [
    (dict(X=None), 1), (dict(idx=None), 1), (dict(kappa=None), 1), (dict(k=1), 1),
    (dict(k=100), 1), (dict(variant=2), 1), (dict(precision=2), 3), (dict(precision=9), 1),
    (dict(flags=1), 1), (dict(ldx=2), 1), (dict(precision=3, k=29), 2), (dict(precision=3, k=32), 2),
])
def test_fast_rejects(args, code):
    L = _lib()
    a = dict(X=FAKE, n=100, m=4, ldx=4, k=5, precision=0, variant=0, flags=0, idx=FAKE, kappa=FAKE)
    a.update(args)
    st = L.lib().mc_curvature_fast(a["X"], a["n"], a["m"], a["ldx"], a["idx"], a["k"],
                                   a["precision"], a["variant"], a["flags"], a["kappa"], None,
                                   FAKE, 1 << 20, None)
    assert st == code


@pytest.mark.parametrize("args,code", [
    (dict(X=None), 1), (dict(ws=None), 1), (dict(precision=1), 3), (dict(ws_bytes=0), 4),
    (dict(k=2, n=2), 1), (dict(precision=3), 3),
])
def test_exact_rejects(args, code):
    L = _lib()
    a = dict(X=FAKE, n=100, m=4, ldx=4, k=5, precision=0, idx=FAKE, kappa=FAKE, ws=FAKE,
             ws_bytes=1 << 40)
    a.update(args)
    st = L.lib().mc_curvature_exact(a["X"], a["n"], a["m"], a["ldx"], a["idx"], a["k"],
                                    a["precision"], 0, a["kappa"], None, a["ws"], a["ws_bytes"], None)
    assert st == code


@pytest.mark.parametrize("args,code", [
    (dict(gk=None), 1), (dict(grad=None), 1), (dict(gap=-1.0), 1), (dict(gap=float("nan")), 1),
    (dict(variant=3), 1), (dict(k=0), 1), (dict(k=17), 2), (dict(k=32), 2),
])
def test_backward_rejects(args, code):
    L = _lib()
    a = dict(X=FAKE, n=100, m=4, ldx=4, k=5, variant=0, idx=FAKE, gk=FAKE, gap=0.0, grad=FAKE)
    a.update(args)
    st = L.lib().mc_curvature_backward(a["X"], a["n"], a["m"], a["ldx"], a["idx"], a["k"],
                                       a["variant"], a["gk"], a["gap"], a["grad"], FAKE, 1 << 20, None)
    assert st == code


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2606_06329_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()
