"""The allocation-free product (h2x_matmul_noalloc) against h2x_matmul, through the C ABI.
Named to be collected last, so that a failure here cannot hide the other GPU tests.

Two calls in a row share the library's static scratch array: the first on the
n = 20000, k = 64 sphere operator with 32 columns, the second on a smaller operator
(n = 3000, k = 27) with 5 columns, so the second call meets the first one's stale
contents.  Each must equal the workspace product (the same kernels: bitwise, and in
any case within 1e-12 per column) and the oracle within 1e-12 per column.  A product
whose scratch exceeds the array is refused with H2X_ENOMEM before anything runs.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


CASES = [("sphere-n20000-k64-m32", 20000, 151, dict(ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4), 32),
         ("sphere-n3000-k27-m5", 3000, 152, dict(ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3), 5)]


def test_noalloc_matches_workspace_product_twice():
    import paper_2509_17257_amd as h2x
    lib = h2x.load_library()
    for name, n, seed, prm, m in CASES:
        print(f"[noalloc] {name}", flush=True)
        P = W.sphere_points(n, seed)
        A = h2x.H2Matrix(P, **prm)
        assert lib.h2x_matmul_workspace_bytes(A._h, m) <= h2x.NOALLOC_MAX_BYTES
        X = torch.from_numpy(W.rhs(n, m, seed + 1)).cuda()
        Y0 = torch.from_numpy(W.rhs(n, m, seed + 2)).cuda()
        ref = h2x.h2_matmul(A, X, alpha=0.75, beta=0.5, out=Y0.clone())
        got = h2x.h2_matmul_noalloc(A, X, alpha=0.75, beta=0.5, out=Y0.clone())
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        o = oracle.OracleH2(P, **prm)
        orc = o.matmul(X.cpu().numpy(), alpha=0.75, beta=0.5, Y=Y0.cpu().numpy())
        e_ws, e_orc = _colrel(g, r), _colrel(g, orc)
        print(f"[noalloc] {name}: vs workspace product {e_ws:.2e} (bitwise {np.array_equal(g, r)}), "
              f"vs oracle {e_orc:.2e}", flush=True)
        assert e_ws <= 1e-12 and e_orc <= 1e-12


def test_noalloc_refuses_scratch_beyond_the_array():
    import paper_2509_17257_amd as h2x
    lib = h2x.load_library()
    P = W.sphere_points(20000, 151)
    A = h2x.H2Matrix(P, ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
    m = 256
    assert lib.h2x_matmul_workspace_bytes(A._h, m) > h2x.NOALLOC_MAX_BYTES
    X = torch.zeros((A.n, m), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(h2x.H2xError, match="status 2"):
        h2x.h2_matmul_noalloc(A, X, out=Y)
