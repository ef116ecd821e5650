"""mc_curvature_fast_noalloc (no workspace argument, static device scratch) against
mc_curvature_fast on the same inputs, through the C ABI: identical results on two calls in a
row, the second smaller, and a clear rejection of sizes beyond the static scratch."""
import ctypes

import numpy as np
import pytest

from oracle import knn as ok
from paper_2606_06329_amd import synth
from tests.gpu_common import to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(X, idx, variant, precision):
    from paper_2606_06329_amd import _lib as L
    n, m = X.shape
    k = idx.shape[1]
    kap = torch.empty(n, dtype=torch.float32, device=X.device)
    fl = torch.empty(n, dtype=torch.uint8, device=X.device)
    prec = {"fp32": L.MC_FP32, "bf16": L.MC_BF16, "fp64": L.MC_FP64}[precision]
    var = {"paper": L.MC_FAST_PAPER, "haar": L.MC_FAST_HAAR}[variant]
    st = L.lib().mc_curvature_fast_noalloc(X.data_ptr(), n, m, X.stride(0), idx.data_ptr(), k, prec, var, 0,
                                           kap.data_ptr(), fl.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
    return st, kap, fl


@pytest.mark.parametrize("name,n,m,k,precision", [("blobs", 1500, 300, 32, "fp32"), ("blobs", 1500, 300, 32, "bf16"),
                                                  ("torus", 3000, 96, 16, "fp64"), ("swissroll", 2000, 40, 8, "fp32")])
def test_noalloc_matches_workspace_entry_point(name, n, m, k, precision):
    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib as L
    for nn, seed in ((n, 31), (n // 3, 32)):           # the second call is smaller
        X = synth.WORKLOADS[name][0](n=nn, m=m, seed=seed)
        idx, _, _, _ = ok.knn(X.astype(np.float64), k)
        Xd = to_dev(X)
        idd = torch.from_numpy(idx.astype(np.int32)).cuda()
        print(f"noalloc {name} n={nn} m={m} k={k} {precision}", flush=True)
        st, kap, fl = _noalloc(Xd, idd, "paper", precision)
        assert st == L.MC_OK, L.status_string(st)
        want, wfl = P.curvature_fast(Xd, idd, "paper", precision)
        torch.cuda.synchronize()
        assert torch.equal(kap, want)
        assert torch.equal(fl, wfl)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    from paper_2606_06329_amd import _lib as L
    lib = L.lib()
    k, m = 32, 64
    n = 100
    while lib.mc_workspace_bytes(L.MC_OP_FAST, n, m, k, L.MC_FP32, 1) <= L.MC_NOALLOC_SCRATCH_BYTES:
        n *= 2
    X = torch.zeros((n, m), device="cuda")
    idx = torch.zeros((n, k), dtype=torch.int32, device="cuda")
    st, _, _ = _noalloc(X, idx, "paper", "fp32")
    assert st == L.MC_ESCRATCH
    assert "scratch" in L.status_string(st)
