"""Pins of the oracle's complex (K = C) operator and complex block GMRES (section 5.2
with the paper's Helmholtz setting; point-cloud single-layer kernel with equal
quadrature weights, g(x, y) = (4 pi / n) exp(i kappa r) / (4 pi r), self-interaction
excluded, shift on the diagonal).

* The fast product (real bases on interleaved real / imaginary column pairs, complex
  coupling and near-field blocks) equals the densely assembled complex H^2 matrix.
* Its distance to the exact kernel matrix decays geometrically over p = 2..5 (the
  absolute interpolation error is parity unpinned: the paper prints no value for
  this kernel).
* Complex linearity A (i x) = i A x, which fails if the imaginary planes are applied
  with the wrong sign or to the wrong component; the assembled matrix is complex
  symmetric (g(x, y) = g(y, x), S_(s,t) = S_(t,s)^T) and not Hermitian.
* Complex block GMRES: after k steps of one cycle the iterate is the least-squares
  minimiser over the complex Krylov space (numpy QR / lstsq); restarted to 1e-11 it
  matches a dense complex solve; column i of the block run is bit-for-bit GMRES on b_i
  alone; restart semantics as in the real case.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W


def _cplx(n, m, seed):
    return W.rhs(n, m, seed) + 1j * W.rhs(n, m, seed + 1)


@pytest.fixture(scope="module")
def helm():
    P = W.sphere_points(700, 111)
    o = oracle.OracleH2(P, kernel="helmholtz", ell=1.0, shift=1.0, eta=1.0, leaf=32, p=3)
    return o, o.dense_complex()


def test_fast_product_equals_dense_assembly(helm):
    o, D = helm
    X = _cplx(o.n, 4, 112)
    Y = o.matmul_complex(X)
    assert np.linalg.norm(Y - D @ X) <= 1e-13 * np.linalg.norm(Y)


def test_interpolation_error_decays_geometrically():
    P = W.sphere_points(600, 113)
    K = oracle.kernel_matrix(P, kernel="helmholtz", ell=1.0, shift=1.0)
    X = _cplx(600, 3, 114)
    errs = []
    for p in (2, 3, 4, 5):
        o = oracle.OracleH2(P, kernel="helmholtz", ell=1.0, shift=1.0, eta=1.0, leaf=32, p=p)
        errs.append(np.linalg.norm(o.matmul_complex(X) - K @ X) / np.linalg.norm(K @ X))
    print("errors", errs)
    assert all(b < 0.2 * a for a, b in zip(errs, errs[1:]))


def test_complex_linearity_and_symmetry(helm):
    o, D = helm
    X = _cplx(o.n, 3, 115)
    Y = o.matmul_complex(X)
    assert np.linalg.norm(o.matmul_complex(1j * X) - 1j * Y) <= 1e-14 * np.linalg.norm(Y)
    assert np.abs(D - D.T).max() <= 1e-15 * np.abs(D).max()
    assert np.abs(D - D.conj().T).max() > 1e-3 * np.abs(D).max()  # not Hermitian
    assert np.abs(D.imag).max() > 1e-3 * np.abs(D).max()


@pytest.mark.parametrize("k", [1, 4, 8])
def test_complex_gmres_krylov_minimiser(helm, k):
    o, D = helm
    B = _cplx(o.n, 2, 116)
    X, info = o.block_gmres_complex(B, rtol=0.0, restart=k, max_iter=k)
    assert info["iters"] == k
    for i in range(B.shape[1]):
        b = B[:, i]
        K = np.empty((len(b), k), complex)
        v = b / np.linalg.norm(b)
        for j in range(k):
            K[:, j] = v
            v = D @ v
            v -= K[:, : j + 1] @ (K[:, : j + 1].conj().T @ v)
            v -= K[:, : j + 1] @ (K[:, : j + 1].conj().T @ v)
            v /= np.linalg.norm(v)
        y = np.linalg.lstsq(D @ K, b, rcond=None)[0]
        x = K @ y
        assert np.linalg.norm(X[:, i] - x) <= 1e-9 * np.linalg.norm(x)
        rmin = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
        assert abs(info["res_est"][i] - rmin) <= 1e-9 * rmin


def test_complex_gmres_dense_solve_and_columns(helm):
    o, D = helm
    B = _cplx(o.n, 3, 117)
    rtol = 1e-11
    X, info = o.block_gmres_complex(B, rtol=rtol, restart=10)
    assert (info["status"] == 0).all()
    ref = np.linalg.solve(D, B)
    cond = np.linalg.cond(D)
    for i in range(3):
        assert np.linalg.norm(B[:, i] - D @ X[:, i]) <= rtol * np.linalg.norm(B[:, i])
        assert np.linalg.norm(X[:, i] - ref[:, i]) <= 10 * cond * rtol * np.linalg.norm(ref[:, i])
        x1, i1 = o.block_gmres_complex(B[:, i : i + 1], rtol=rtol, restart=10)
        np.testing.assert_array_equal(X[:, i], x1[:, 0])
        assert i1["col_iters"][0] == info["col_iters"][i]


def test_complex_gmres_restart(helm):
    o, _ = helm
    B = _cplx(o.n, 2, 118)
    X4, i4 = o.block_gmres_complex(B, rtol=0.0, restart=3, max_iter=4)
    X3, _ = o.block_gmres_complex(B, rtol=0.0, restart=3, max_iter=3)
    X31, _ = o.block_gmres_complex(B, X0=X3, rtol=0.0, restart=3, max_iter=1)
    assert i4["cycles"] == 2
    np.testing.assert_array_equal(X31, X4)
