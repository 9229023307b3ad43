"""Complex (K = C) operator on the GPU: the Helmholtz single-layer kernel with equal
quadrature weights (H2X_KERNEL_HELMHOLTZ), products and block GMRES over C, against
the oracle's complex product and complex GMRES (section 5.2's complex setting).

* Products (k = 27 and k = 64, two wavenumbers, an odd number of complex columns,
  alpha / beta): per complex column relative error <= 1e-12 against the oracle;
  complex linearity A (i X) = i A X.
* GMRES over C: fixed step budgets agree with the oracle <= 1e-11 per column with
  equal step counts and estimates; end to end to 1e-10 true residuals within rtol,
  step counts within one cycle of the oracle's, solutions within 10 kappa rtol.
* Refused: CG (needs a Hermitian positive definite operator), the adjoint and
  gradients, low-precision storage, batching, an odd number of real columns.
* Full size (sphere n = 65536, k = 64, 16 complex columns): the product against the
  oracle and GMRES(30) to 1e-8 with true residuals within rtol.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _h2x():
    import paper_2509_17257_amd as h2x
    return h2x


def _cplx(n, m, seed):
    return W.rhs(n, m, seed) + 1j * W.rhs(n, m, seed + 1)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _colrel(a, b):
    den = np.linalg.norm(b, axis=0)
    den[den == 0] = 1.0
    return (np.linalg.norm(a - b, axis=0) / den).max()


CASES = [
    ("sphere-n4096-k27", lambda: W.sphere_points(4096, 121), dict(leaf=32, p=3), 1.0, 3),
    ("sphere-n5000-k64", lambda: W.sphere_points(5000, 122), dict(leaf=64, p=4), 1.0, 5),
    ("sphere-n3000-k64-kappa4", lambda: W.sphere_points(3000, 123), dict(leaf=64, p=4), 4.0, 4),
]


@pytest.mark.parametrize("name,pts,prm,kappa,m", CASES, ids=[c[0] for c in CASES])
def test_complex_product_matches_oracle(name, pts, prm, kappa, m):
    h2x = _h2x()
    P = pts()
    n = P.shape[0]
    kw = dict(kernel="helmholtz", ell=kappa, shift=1.0, eta=1.0, **prm)
    o = oracle.OracleH2(P, **kw)
    A = h2x.H2Matrix(P, **kw)
    X = _cplx(n, m, 124)
    ref = o.matmul_complex(X)
    got = h2x.h2_matmul(A, _dev(X)).cpu().numpy()
    err = _colrel(got, ref)
    Y0 = _cplx(n, m, 126)
    got_ab = h2x.h2_matmul(A, _dev(X), alpha=-0.5, beta=2.0, out=_dev(Y0)).cpu().numpy()
    err_ab = _colrel(got_ab, 2.0 * Y0 - 0.5 * ref)
    lin = _colrel(h2x.h2_matmul(A, _dev(1j * X)).cpu().numpy(), 1j * got)
    print(f"{name}: product {err:.2e} alpha/beta {err_ab:.2e} linearity {lin:.2e}")
    assert err <= 1e-12 and err_ab <= 1e-12 and lin <= 1e-14


@pytest.mark.parametrize("name,pts,prm,kappa,m", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_complex_row_split_leaf_stage(name, pts, prm, kappa, m):
    """The row-split leaf stage (leaf_kind 2) on the complex operator: each near block's
    imaginary plane applied to J X while X is staged."""
    h2x = _h2x()
    P = pts()
    n = P.shape[0]
    kw = dict(kernel="helmholtz", ell=kappa, shift=1.0, eta=1.0, **prm)
    o = oracle.OracleH2(P, **kw)
    A = h2x.H2Matrix(P, **kw)
    X = _cplx(n, m, 134)
    ref = o.matmul_complex(X)
    errs = []
    for npl in (1, 2):
        A.set_tune(2 * m, leaf_kind=2, np_leaf=npl)
        errs.append(_colrel(h2x.h2_matmul(A, _dev(X)).cpu().numpy(), ref))
    print(f"{name}: row-split leaf stage {max(errs):.2e}")
    assert max(errs) <= 1e-12


def test_complex_split_coupling():
    """Both coupling passes (real plane, imaginary plane on J x-hat) of each part of the
    split rows: bitwise the one-launch result, and the oracle's."""
    h2x = _h2x()
    P = W.sphere_points(4096, 121)
    kw = dict(kernel="helmholtz", ell=1.0, shift=1.0, eta=1.0, leaf=32, p=3)
    A = h2x.H2Matrix(P, **kw)
    assert A.plan.split_depth > 0
    X = _cplx(4096, 3, 136)
    A.set_tune(6, split=2)
    one = h2x.h2_matmul(A, _dev(X)).cpu().numpy()
    A.set_tune(6, split=1)
    got = h2x.h2_matmul(A, _dev(X)).cpu().numpy()
    err = _colrel(got, oracle.OracleH2(P, **kw).matmul_complex(X))
    print(f"complex split coupling: {err:.2e}")
    assert np.array_equal(got, one) and err <= 1e-12


@pytest.fixture(scope="module")
def helm():
    h2x = _h2x()
    P = W.sphere_points(4096, 127)
    kw = dict(kernel="helmholtz", ell=1.0, shift=1.0, eta=1.0, leaf=32, p=3)
    return oracle.OracleH2(P, **kw), h2x.H2Matrix(P, **kw)


@pytest.mark.parametrize("restart,steps", [(6, 6), (4, 10)])
def test_complex_gmres_fixed_steps(helm, restart, steps):
    h2x = _h2x()
    o, A = helm
    B = _cplx(o.n, 3, 128)
    Xo, io = o.block_gmres_complex(B, rtol=0.0, restart=restart, max_iter=steps)
    Xg, ig = h2x.block_gmres_solve(A, _dev(B), rtol=0.0, restart=restart, max_iter=steps, check_every=1)
    err = _colrel(Xg.cpu().numpy(), Xo)
    print(f"complex GMRES restart {restart} steps {steps}: {err:.2e}")
    assert ig.iters == io["iters"] == steps and ig.cycles == io["cycles"]
    np.testing.assert_array_equal(ig.col_iters, io["col_iters"])
    assert err <= 1e-11
    np.testing.assert_allclose(ig.col_res, io["res_est"], rtol=1e-8)


def test_complex_gmres_end_to_end():
    h2x = _h2x()
    P = W.sphere_points(2000, 129)
    kw = dict(kernel="helmholtz", ell=2.0, shift=1.0, eta=1.0, leaf=32, p=3)
    o = oracle.OracleH2(P, **kw)
    A = h2x.H2Matrix(P, **kw)
    B = _cplx(2000, 3, 130)
    rtol = 1e-10
    Xo, io = o.block_gmres_complex(B, rtol=rtol, restart=10)
    Xg, ig = h2x.block_gmres_solve(A, _dev(B), rtol=rtol, restart=10)
    Xg = Xg.cpu().numpy()
    D = o.dense_complex()
    kappa = np.linalg.cond(D)
    res = np.linalg.norm(B - o.matmul_complex(Xg), axis=0) / np.linalg.norm(B, axis=0)
    print(f"complex end to end: steps {ig.col_iters.tolist()} oracle {io['col_iters'].tolist()}, kappa {kappa:.2f}, "
          f"true residual {res.max():.2e}, X vs oracle {_colrel(Xg, Xo):.2e}")
    assert ig.status == 0 and (ig.col_status == 0).all()
    assert (res <= rtol).all()
    assert (np.abs(ig.col_iters - io["col_iters"]) <= 10 + 2).all()
    assert _colrel(Xg, Xo) <= 10 * kappa * rtol


def test_complex_refusals(helm):
    h2x = _h2x()
    o, A = helm
    B = _dev(_cplx(o.n, 2, 131))
    with pytest.raises(h2x.H2xError, match="complex"):
        h2x.block_cg_solve(A, torch.view_as_real(B).reshape(o.n, 4))
    with pytest.raises(h2x.H2xError, match="complex"):
        h2x.h2_matmul_adjoint(A, torch.view_as_real(B).reshape(o.n, 4))
    with pytest.raises(h2x.H2xError, match="even"):
        h2x.h2_matmul(A, torch.zeros((o.n, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(h2x.H2xError):
        h2x.H2Matrix(W.sphere_points(1000, 132), storage="f32", kernel="helmholtz", ell=1.0, leaf=64, p=4)
    with pytest.raises(h2x.H2xError):
        h2x.Plan.merge([A.plan, A.plan])


def test_complex_full_size():
    h2x = _h2x()
    w = W.FP64
    P = w.points()
    kw = dict(kernel="helmholtz", ell=1.0, shift=1.0, eta=1.0, leaf=64, p=4)
    A = h2x.H2Matrix(P, **kw)
    X = _cplx(w.n, 16, 133)
    print("[full] complex product", flush=True)
    got = h2x.h2_matmul(A, _dev(X)).cpu().numpy()
    o = oracle.OracleH2(P, **kw)
    err = _colrel(got, o.matmul_complex(X))
    del o
    B = _dev(_cplx(w.n, 16, 135))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xs, info = h2x.block_gmres_solve(A, B, rtol=1e-8, restart=30)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    R = B - h2x.h2_matmul(A, Xs)
    res = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(B, dim=0)).cpu().numpy()
    print(f"[full] product vs oracle {err:.2e}; GMRES steps {info.iters} cycles {info.cycles} time {dt:.3f} s, "
          f"true residual {res.max():.2e}")
    assert err <= 1e-12
    assert info.status == 0 and (res <= 1e-8).all()
