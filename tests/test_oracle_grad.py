"""Pins of the oracle's adjoint product and gradients.

* Adjoint dot-product identity <dY, A X> = <A^T dY, X>, and A^T dY = A dY (the
  H^2 matrix is exactly symmetric: S_ts = S_st^T, W == V, symmetric near field).
* dS: L(S) = <dY, A(S) X> is linear in S, so a difference quotient in one
  coupling entry reproduces dS exactly (up to rounding).  Same for dN.
* d ell: equals <dY, (dA/d ell) X> of the densely assembled derivative, and a
  central finite difference (h = 1e-6) of L(ell) with a refilled operator.
* Implicit adjoint of X = A^{-1} B: d <C, X> / d ell = -<lambda, (dA/d ell) X>,
  lambda = A^{-1} C, against a central finite difference of dense solves.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W


@pytest.fixture(scope="module")
def tiny():
    P = W.sphere_points(900, 141)
    h = oracle.OracleH2(P, leaf=24, p=3, ell=0.5, shift=1.0)
    return h, W.rhs(900, 3, 142), W.rhs(900, 3, 143)


def test_adjoint(tiny):
    h, X, dY = tiny
    AX = h.matmul(X)
    AtdY = h.matmul_adjoint(dY)
    lhs, rhs = np.sum(dY * AX), np.sum(AtdY * X)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    np.testing.assert_allclose(AtdY, h.matmul(dY), rtol=0, atol=1e-13 * np.abs(AtdY).max())
    Ad = h.dense()
    np.testing.assert_allclose(AtdY, Ad.T @ dY, rtol=0, atol=1e-12 * np.abs(AtdY).max())
    # with one coupling block perturbed (A no longer symmetric) the adjoint must follow
    # the transpose, not A itself
    S = h.S()
    S2 = S.copy()
    S2[7] = S[7] + 0.01 * np.arange(h.k * h.k).reshape(h.k, h.k) / (h.k * h.k)
    h.set_S(S2)
    try:
        Ans = h.dense()
        At = h.matmul_adjoint(dY)
        assert np.abs(Ans - Ans.T).max() > 1e-6
        np.testing.assert_allclose(At, Ans.T @ dY, rtol=0, atol=1e-12 * np.abs(At).max())
        assert np.abs(At - h.matmul(dY)).max() > 1e-8
        assert abs(np.sum(dY * h.matmul(X)) - np.sum(At * X)) <= 1e-12 * abs(lhs)
    finally:
        h.set_S(S)


def test_dS_and_dN_are_exact_difference_quotients(tiny):
    h, X, dY = tiny
    dS, dN, _ = h.grad(X, dY)
    S, N = h.S(), h.N()
    L0 = np.sum(dY * h.matmul(X))
    g = np.random.default_rng(144)
    for _ in range(4):
        b, i, j = g.integers(h.n_adm), g.integers(h.k), g.integers(h.k)
        S2 = S.copy()
        S2[b, i, j] += 1.0
        h.set_S(S2)
        d = np.sum(dY * h.matmul(X)) - L0
        h.set_S(S)
        assert abs(d - dS[b, i, j]) <= 1e-9 * max(1.0, abs(dS[b, i, j]))
        e = g.integers(h.near_entries)
        N2 = N.copy()
        N2[e] += 1.0
        h.set_N(N2)
        d = np.sum(dY * h.matmul(X)) - L0
        h.set_N(N)
        assert abs(d - dN[e]) <= 1e-9 * max(1.0, abs(dN[e]))


def test_dell_dense_and_finite_difference(tiny):
    h, X, dY = tiny
    _, _, dl = h.grad(X, dY, want_dS=False, want_dN=False)
    dense = np.sum(dY * (h.dense_dell() @ X))
    assert abs(dl - dense) <= 1e-12 * abs(dense)
    ell, eps = h.ell, 1e-6
    h.set_ell(ell + eps)
    Lp = np.sum(dY * h.matmul(X))
    h.set_ell(ell - eps)
    Lm = np.sum(dY * h.matmul(X))
    h.set_ell(ell)
    fd = (Lp - Lm) / (2 * eps)
    assert abs(fd - dl) <= 1e-7 * abs(dl)


def test_implicit_adjoint(tiny):
    h, B, C = tiny
    A = h.dense()
    X = np.linalg.solve(A, B)
    lam = np.linalg.solve(A.T, C)
    dl = -np.sum(lam * (h.dense_dell() @ X))
    # the same through the fast gradient with dY = lambda
    _, _, dl_fast = h.grad(X, lam, want_dS=False, want_dN=False)
    assert abs(-dl_fast - dl) <= 1e-10 * abs(dl)
    ell, eps = h.ell, 1e-6
    vals = []
    for e in (eps, -eps):
        h.set_ell(ell + e)
        vals.append(np.sum(C * np.linalg.solve(h.dense(), B)))
    h.set_ell(ell)
    fd = (vals[0] - vals[1]) / (2 * eps)
    assert abs(fd - dl) <= 1e-6 * abs(dl)
