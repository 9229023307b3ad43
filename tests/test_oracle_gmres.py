"""Pins of the oracle's block GMRES(ell) (section 5.2: GMRES with restarts, and its
block form for m right-hand sides that shares one product per Arnoldi step; no
preconditioner).

* After k steps of one cycle the iterate is the minimiser of ||b - A x|| over the
  Krylov space span{b, Ab, ..., A^(k-1) b}: a least-squares problem solved here by
  numpy (QR of the Krylov matrix, lstsq), on a non-symmetric operator.  The
  estimate |rhat_k| equals that minimal residual.
* Restarted to convergence it agrees with a dense LU solve of the assembled H^2
  matrix within the tolerance times the condition number, for a symmetric and a
  non-symmetric operator, with true residuals below the tolerance.
* Constant kernel: A = shift I + 1 1^T has two distinct eigenvalues, so GMRES
  ends after at most two steps, at the Sherman-Morrison closed form.
* Column i of the block run is bit-for-bit GMRES on b_i alone.
* Restarting from the iterate after three steps with one more step gives the
  iterate of a three-step cycle followed by a one-step cycle (the residual is
  recomputed from the improved iterate); the step budget counts Arnoldi steps.
* A zero right-hand side converges before any step, with x = 0.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W


def _perturbed(n, seed):
    """A small operator made non-symmetric by perturbing some coupling blocks."""
    P = W.sphere_points(n, seed)
    h = oracle.OracleH2(P, leaf=32, p=3, ell=0.5, shift=1.0)
    S = h.S()
    rng = np.random.default_rng(seed + 1)
    for b in rng.choice(S.shape[0], max(1, S.shape[0] // 4), replace=False):
        S[b] += 0.2 * rng.standard_normal(S[b].shape)
    h.set_S(S)
    return h


@pytest.fixture(scope="module")
def nonsym():
    h = _perturbed(500, 71)
    A = h.dense()
    assert np.abs(A - A.T).max() > 1e-3  # the operator really is non-symmetric
    return h, A, W.rhs(500, 3, 72)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_gmres_iterate_is_krylov_least_squares_minimiser(nonsym, k):
    h, A, B = nonsym
    X, info = h.block_gmres(B, rtol=0.0, restart=k, max_iter=k)
    assert info["iters"] == k and info["cycles"] == 1
    for i in range(B.shape[1]):
        b = B[:, i]
        K = np.empty((len(b), k))
        v = b / np.linalg.norm(b)
        for j in range(k):  # Krylov vectors, orthonormalised as they are formed
            K[:, j] = v
            v = A @ v
            v -= K[:, : j + 1] @ (K[:, : j + 1].T @ v)
            v -= K[:, : j + 1] @ (K[:, : j + 1].T @ v)
            v /= np.linalg.norm(v)
        y = np.linalg.lstsq(A @ K, b, rcond=None)[0]
        x = K @ y
        assert np.linalg.norm(X[:, i] - x) <= 1e-9 * np.linalg.norm(x)
        rmin = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert abs(info["res_est"][i] - rmin) <= 1e-9 * rmin


@pytest.mark.parametrize("kind", ["symmetric", "nonsymmetric"])
def test_gmres_matches_dense_solve(nonsym, kind):
    if kind == "symmetric":
        h = oracle.OracleH2(W.sphere_points(700, 73), leaf=32, p=3, ell=0.5, shift=1.0)
        A, B = h.dense(), W.rhs(700, 3, 74)
    else:
        h, A, B = nonsym
    rtol = 1e-11
    X, info = h.block_gmres(B, rtol=rtol, restart=15, max_iter=2000)
    assert (info["status"] == 0).all()
    ref = np.linalg.solve(A, B)
    cond = np.linalg.cond(A)
    for i in range(B.shape[1]):
        res = np.linalg.norm(B[:, i] - A @ X[:, i]) / np.linalg.norm(B[:, i])
        assert res <= rtol
        assert np.linalg.norm(X[:, i] - ref[:, i]) <= 10 * cond * rtol * np.linalg.norm(ref[:, i])


def test_gmres_constant_kernel_two_steps():
    n, shift = 800, 0.5
    h = oracle.OracleH2(W.sphere_points(n, 75), kernel="const", leaf=32, p=3, shift=shift)
    B = W.rhs(n, 3, 76)
    X, info = h.block_gmres(B, rtol=1e-12, restart=10)
    assert (info["status"] == 0).all()
    assert info["col_iters"].max() <= 2
    ones = np.ones(n)
    for i in range(B.shape[1]):
        b = B[:, i]
        ref = (b - ones * (ones @ b) / (shift + n)) / shift
        assert np.linalg.norm(X[:, i] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_gmres_block_column_equals_single_column(nonsym):
    h, _, B = nonsym
    X, info = h.block_gmres(B, rtol=1e-9, restart=8, max_iter=400)
    for i in range(B.shape[1]):
        x1, info1 = h.block_gmres(B[:, i : i + 1], rtol=1e-9, restart=8, max_iter=400)
        assert info1["col_iters"][0] == info["col_iters"][i]
        np.testing.assert_array_equal(X[:, i], x1[:, 0])


def test_gmres_restart_from_improved_iterate(nonsym):
    h, _, B = nonsym
    X4, info4 = h.block_gmres(B, rtol=0.0, restart=3, max_iter=4)
    assert info4["iters"] == 4 and info4["cycles"] == 2 and (info4["status"] == 2).all()
    X3, _ = h.block_gmres(B, rtol=0.0, restart=3, max_iter=3)
    X31, info31 = h.block_gmres(B, X0=X3, rtol=0.0, restart=3, max_iter=1)
    assert info31["iters"] == 1
    np.testing.assert_array_equal(X31, X4)


def test_gmres_zero_rhs_column():
    h = oracle.OracleH2(W.sphere_points(400, 77), leaf=32, p=3, ell=0.5, shift=1.0)
    B = W.rhs(400, 3, 78)
    B[:, 1] = 0.0
    X, info = h.block_gmres(B, rtol=1e-8, restart=10)
    assert info["col_iters"][1] == 0 and info["status"][1] == 0
    assert not X[:, 1].any()
    assert (info["status"] == 0).all()
