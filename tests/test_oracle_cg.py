"""Pins of the oracle's block CG (section 5.1: CG for one right-hand side, and the
block CG for m right-hand sides that shares one H^2 x P product per iteration).

* Column i of block CG is bit-for-bit the single-RHS CG on b_i.
* The converged block agrees with a dense Cholesky solve of the assembled H^2
  matrix (a textbook LAPACK routine) within the tolerance times the condition.
* Constant kernel: A = shift I + 1 1^T exactly, whose inverse is known in closed
  form (Sherman-Morrison) and on which CG converges in two steps (two distinct
  eigenvalues).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2509_17257_amd import workloads as W


@pytest.fixture(scope="module")
def small():
    n = 1200
    P = W.sphere_points(n, 61)
    h = oracle.OracleH2(P, leaf=32, p=3, ell=0.5, shift=1.0)
    return h, W.rhs(n, 4, 62)


def test_block_cg_column_equals_single_cg(small):
    h, B = small
    X, info = h.block_cg(B, rtol=1e-8)
    for i in range(B.shape[1]):
        x1, it1 = h.cg1(B[:, i], rtol=1e-8)
        # same iteration count for the column while it is unconverged
        assert info["col_iters"][i] == it1
        if it1 == info["iters"]:
            np.testing.assert_array_equal(X[:, i], x1)


def test_block_cg_matches_dense_cholesky(small):
    h, B = small
    A = h.dense()
    c = sla.cho_factor(A)  # succeeds only if A_H2 is SPD
    Xd = sla.cho_solve(c, B)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    rtol = 1e-8
    X, info = h.block_cg(B, rtol=rtol)
    assert np.all(info["status"] == 0)
    rel = np.linalg.norm(X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    assert rel.max() <= kappa * rtol
    res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 2 * rtol


def test_constant_kernel_closed_form():
    n, sigma = 800, 0.8
    P = W.sphere_points(n, 63)
    h = oracle.OracleH2(P, kernel="const", leaf=32, p=2, shift=sigma)
    assert h.n_adm > 0
    B = W.rhs(n, 3, 64)
    X, info = h.block_cg(B, rtol=1e-12)
    Xcf = (B - np.ones((n, 1)) * (B.sum(0, keepdims=True) / (sigma + n))) / sigma
    np.testing.assert_allclose(X, Xcf, rtol=0, atol=1e-9 * np.abs(Xcf).max())
    assert info["iters"] <= 2


def test_nonzero_initial_guess_and_max_iter(small):
    h, B = small
    X0 = 0.1 * W.rhs(h.n, 4, 65)
    X, info = h.block_cg(B, X0=X0, rtol=1e-8)
    res = np.linalg.norm(B - h.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 2e-8
    X1, info1 = h.block_cg(B, rtol=1e-8, max_iter=1)
    assert info1["iters"] == 1 and np.all(info1["status"] == 2)


def test_indefinite_shift_flags_breakdown():
    n = 600
    P = W.sphere_points(n, 66)
    h = oracle.OracleH2(P, leaf=32, p=3, shift=-200.0)  # shift below -lambda_min
    B = W.rhs(n, 3, 67)
    X, info = h.block_cg(B, rtol=1e-8, max_iter=500)
    assert np.any(info["status"] != 0)


# ---- block CG over one shared block Krylov space (m x m Gram matrices) ----

def test_shared_block_cg_matches_dense_and_beats_independent(small):
    h, B = small
    A = h.dense()
    Xd = sla.cho_solve(sla.cho_factor(A), B)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    X, info = h.block_cg_shared(B, rtol=1e-8)
    _, ind = h.block_cg(B, rtol=1e-8)
    assert np.all(info["status"] == 0) and info["rank_min"] == B.shape[1]
    rel = np.linalg.norm(X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    assert rel.max() <= kappa * 1e-8
    res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 1e-8
    # the shared space contains every column's own Krylov space
    assert info["iters"] < ind["iters"]


def test_shared_block_cg_single_column_is_cg(small):
    h, B = small
    x1, it1 = h.cg1(B[:, 0], rtol=1e-10)
    X1, info = h.block_cg_shared(B[:, :1].copy(), rtol=1e-10)
    assert abs(info["iters"] - it1) <= 1
    assert np.abs(X1[:, 0] - x1).max() <= 1e-9 * np.abs(x1).max()


def test_shared_block_cg_deflates_dependent_columns(small):
    h, B = small
    ref, rinfo = h.block_cg_shared(np.ascontiguousarray(B[:, [0, 2]]), rtol=1e-8)
    cases = {
        "duplicate": np.ascontiguousarray(B[:, [0, 0, 2]]),
        "zero": np.c_[B[:, [0, 2]], np.zeros(h.n)],
        "combination": np.c_[B[:, [0, 2]], B[:, 0] - 2.0 * B[:, 2]],
    }
    for name, Bx in cases.items():
        X, info = h.block_cg_shared(Bx, rtol=1e-8)
        assert np.all(info["status"] == 0), name
        assert info["rank_min"] == 2, name
        assert abs(info["iters"] - rinfo["iters"]) <= 3, (name, info, rinfo)
        res = np.linalg.norm(Bx - h.matmul(X), axis=0) / np.maximum(np.linalg.norm(Bx, axis=0), 1e-300)
        assert res.max() <= 1e-8, name


def test_shared_block_cg_constant_kernel():
    n, sigma = 800, 0.8
    P = W.sphere_points(n, 63)
    h = oracle.OracleH2(P, kernel="const", leaf=32, p=2, shift=sigma)
    B = W.rhs(n, 3, 64)
    X, info = h.block_cg_shared(B, rtol=1e-12)
    Xcf = (B - np.ones((n, 1)) * (B.sum(0, keepdims=True) / (sigma + n))) / sigma
    np.testing.assert_allclose(X, Xcf, rtol=0, atol=1e-9 * np.abs(Xcf).max())
    assert info["iters"] <= 2
