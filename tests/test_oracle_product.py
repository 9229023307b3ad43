"""Pins of the oracle's H^2 x X product (Algorithm "H2_mvm" in its matrix form,
section 4; forward/backward transformations and the list-wise multiplication
phase of section 3).

* Fast product == the explicitly assembled dense H^2 matrix (its definition).
* Polynomial kernel (1 + x.y)^2, reproduced exactly by order >= 3 interpolation:
  fast product == the dense kernel matrix, which pins forward, transfer,
  coupling, backward and near field independently of interpolation error.
* eta -> 0 (nothing admissible) and leaf >= n: the product is a dense GEMM.
* Column i of H^2 X == H^2 x_i; parallel == sequential recursion.
* Exponential kernel: error against the dense kernel decays geometrically in p
  (its absolute size is parity unpinned: the paper gives no value for it).
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W


def _rel_cols(A, B):
    return (np.linalg.norm(A - B, axis=0) / np.linalg.norm(B, axis=0)).max()


@pytest.mark.parametrize("p,leaf,eta", [(2, 16, 1.0), (3, 32, 1.0), (3, 20, 2.0), (4, 40, 0.7)])
def test_fast_equals_dense_assembly(p, leaf, eta):
    P = W.sphere_points(1800, 41)
    h = oracle.OracleH2(P, leaf=leaf, eta=eta, p=p, ell=0.5, shift=1.0)
    X = W.rhs(1800, 5, 42)
    A = h.dense()
    assert _rel_cols(h.matmul(X), A @ X) < 1e-13
    # the assembled H^2 matrix is symmetric (S_ts = S_st^T, W == V)
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("geom", ["sphere", "cube"])
def test_polynomial_kernel_exact(geom):
    n = 2000
    P = W.sphere_points(n, 43) if geom == "sphere" else W.cube_points(n, 44)
    X = W.rhs(n, 3, 45)
    for p in (3, 4):
        h = oracle.OracleH2(P, kernel="poly", leaf=24, p=p, shift=0.75)
        ref = oracle.kernel_matrix(P, kernel="poly", shift=0.75) @ X
        assert h.n_adm > 0
        assert _rel_cols(h.matmul(X), ref) < 1e-13


def test_planted_coupling_error_is_caught():
    n = 1200
    P = W.sphere_points(n, 46)
    X = W.rhs(n, 2, 47)
    h = oracle.OracleH2(P, kernel="poly", leaf=24, p=3, shift=0.5)
    ref = oracle.kernel_matrix(P, kernel="poly", shift=0.5) @ X
    S = h.S()
    S[len(S) // 2] = S[len(S) // 2].T.copy() * 1.001  # transposed and scaled block
    h.set_S(S)
    assert _rel_cols(h.matmul(X), ref) > 1e-6


def test_no_admissible_is_dense_gemm():
    n = 700
    P = W.sphere_points(n, 48)
    X = W.rhs(n, 4, 49)
    ref = oracle.kernel_matrix(P, ell=0.5, shift=1.0) @ X
    for kw in (dict(leaf=16, eta=1e-12), dict(leaf=n)):
        h = oracle.OracleH2(P, p=3, ell=0.5, shift=1.0, **kw)
        assert h.n_adm == 0
        assert _rel_cols(h.matmul(X), ref) < 1e-14


def test_columns_independent_and_recursion():
    n = 1500
    P = W.sphere_points(n, 50)
    X = W.rhs(n, 6, 51)
    h = oracle.OracleH2(P, leaf=32, p=3)
    Y = h.matmul(X)
    for i in range(6):
        np.testing.assert_array_equal(Y[:, i], h.matmul(X[:, i:i + 1])[:, 0])
    np.testing.assert_array_equal(Y, h.matmul(X, recursive=True))


def test_alpha_beta():
    n = 900
    P = W.sphere_points(n, 52)
    X = W.rhs(n, 3, 53)
    Y0 = W.rhs(n, 3, 54)
    h = oracle.OracleH2(P, leaf=32, p=3)
    AX = h.matmul(X)
    Y = h.matmul(X, alpha=-0.7, beta=1.3, Y=Y0)
    np.testing.assert_allclose(Y, 1.3 * Y0 - 0.7 * AX, rtol=0, atol=1e-12 * np.abs(AX).max())


def test_exp_kernel_error_decays_geometrically():
    n = 2500
    P = W.sphere_points(n, 55)
    X = W.rhs(n, 3, 56)
    ref = oracle.kernel_matrix(P, ell=0.5, shift=1.0) @ X
    errs = []
    for p in (2, 3, 4, 5, 6):
        h = oracle.OracleH2(P, leaf=32, p=p, ell=0.5, shift=1.0)
        errs.append(_rel_cols(h.matmul(X), ref))
    errs = np.array(errs)
    ratios = errs[1:] / errs[:-1]
    assert np.all(ratios < 0.6), (errs, ratios)
    assert errs[-1] < 1e-4
