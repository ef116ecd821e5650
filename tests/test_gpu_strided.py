"""Row-strided inputs (ldx > m): column-slice views of a wider matrix, with a row stride that
keeps 16-byte alignment, one that does not, and a base pointer off the 16-byte grid, give the
same neighbours as the contiguous copy and, on the same neighbour lists, the same curvatures
bit for bit (every kernel reads row r at X + r * ldx).  The re-rank's distances depend on its
column grouping only through rounding, and the adjoint's atomic scatter-add leaves its
summation order free."""
import numpy as np
import pytest

from paper_2606_06329_amd import synth
from tests.gpu_common import to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pad,offset", [(3, 0), (5, 0), (4, 1)],
                         ids=["stride-aligned", "stride-odd", "base-misaligned"])
def test_strided_views_bit_identical(pad, offset):
    import paper_2606_06329_amd as P
    n, m, k = 700, 61, 9
    X = synth.swissroll(n=n, m=m, seed=8080)
    wide = np.zeros((n, m + pad + offset), np.float32)
    wide[:, offset:offset + m] = X
    Wd = to_dev(wide)
    Xv = Wd[:, offset:offset + m]                 # a view: stride(0) = m + pad + offset
    Xc = to_dev(X)
    assert Xv.stride(0) == m + pad + offset and Xv.stride(1) == 1
    assert (Xv.stride(0) % 4 == 0 and offset == 0) == (pad == 3)   # only the first is 16-byte aligned
    print(f"strided view ldx={Xv.stride(0)} offset={offset}", flush=True)
    i1, d1, f1 = P.knn(Xv, k)
    i2, d2, f2 = P.knn(Xc, k)
    # the re-rank sums 16-byte groups of columns when rows are 16-byte aligned (ldx % 4 == 0
    # and an aligned base) and single columns otherwise: the neighbours agree (up to ties
    # within float32 rounding, which are flagged ambiguous) and the distances to rounding
    amb = ((f1 | f2) & 16).bool()
    assert torch.equal(i1[~amb], i2[~amb])
    assert torch.allclose(d1, d2, rtol=2.0 ** -20, atol=0.0)
    for variant in ("paper", "haar"):
        a, fa = P.curvature_fast(Xv, i2, variant)
        b, fb = P.curvature_fast(Xc, i2, variant)
        assert torch.equal(a, b) and torch.equal(fa, fb)
    a, _ = P.curvature_exact(Xv, i2)
    b, _ = P.curvature_exact(Xc, i2)
    assert torch.equal(a, b)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal(n).astype(np.float32)).cuda()
    gv = torch.zeros_like(Wd)[:, offset:offset + m]
    P.curvature_backward(Xv, i2, w, "paper", 0.0, gv)
    gc = P.curvature_backward(Xc, i2, w, "paper", 0.0)
    # the adjoint scatter-adds with float atomics, so only the summation order may differ
    tol = 1e-5 * float(gc.abs().max())
    assert torch.allclose(gv.contiguous(), gc, rtol=1e-5, atol=tol)
