"""Pins of the oracle's cluster basis: Chebyshev nodes, leaf matrices V_t and
transfer matrices E_t (section 2, Definition "Cluster basis"; the H^2 matrix is
built by interpolation, which the paper names as an alternative construction).

Checks are facts of interpolation, not re-evaluations of the oracle's formulas:
nodes are the roots of T_p; Lagrange bases sum to one and reproduce every
polynomial of coordinate degree < p; the basis is nested, V_t|t' = V_t' E_t'.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W


@pytest.fixture(scope="module", params=[2, 3, 4])
def h(request):
    P = W.sphere_points(1500, 31)
    return oracle.OracleH2(P, leaf=24, p=request.param), P


def test_nodes_are_chebyshev_roots(h):
    h, _ = h
    tr, nodes = h.tree(), h.nodes()
    p = h.p
    for c in range(0, h.C, 7):
        for d in range(3):
            lo, hi = tr["ilo"][c][d], tr["ihi"][c][d]
            assert hi > lo
            x = nodes[c, :, d]
            xt = (x - 0.5 * (lo + hi)) / (0.5 * (hi - lo))
            assert np.all(np.abs(np.cos(p * np.arccos(np.clip(xt, -1, 1)))) < 1e-10)
            assert len(np.unique(np.round(xt, 12))) == p


def test_partition_of_unity(h):
    h, _ = h
    V = h.V()
    np.testing.assert_allclose(V.sum(1), 1.0, atol=1e-13, rtol=0)


def _poly_values(coef, pts, p):
    # f(x) = sum_{a,b,c < p} coef[a,b,c] x^a y^b z^c
    out = np.zeros(pts.shape[0])
    for a in range(p):
        for b in range(p):
            for c in range(p):
                out += coef[a, b, c] * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c
    return out


def test_polynomial_reproduction_leaf(h):
    h, P = h
    tr, V, nodes = h.tree(), h.V(), h.nodes()
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((h.p,) * 3)
    for c in range(h.C):
        if tr["son0"][c] >= 0:
            continue
        rows = np.arange(tr["first"][c], tr["first"][c] + tr["size"][c])
        fx = _poly_values(coef, P[tr["perm"][rows]], h.p)
        fn = _poly_values(coef, nodes[c], h.p)
        np.testing.assert_allclose(V[rows] @ fn, fx, atol=1e-11 * max(1, np.abs(fx).max()), rtol=0)


def test_transfer_reproduces_polynomials(h):
    h, _ = h
    tr, E, nodes = h.tree(), h.E(), h.nodes()
    rng = np.random.default_rng(8)
    coef = rng.standard_normal((h.p,) * 3)
    for c in range(1, h.C):
        par = tr["parent"][c]
        f_par = _poly_values(coef, nodes[par], h.p)
        f_son = _poly_values(coef, nodes[c], h.p)
        np.testing.assert_allclose(E[c] @ f_par, f_son, atol=1e-11 * max(1, np.abs(f_son).max()), rtol=0)


def test_nestedness(h):
    h, _ = h
    tr, E, V = h.tree(), h.E(), h.V()
    # V_t for an inner cluster t, evaluated directly, restricted to a son t'
    # equals the son's basis times its transfer matrix.
    for c in range(h.C):
        if tr["son0"][c] < 0 or c % 3:
            continue
        Vt = h.basis_direct(c)
        for s in (tr["son0"][c], tr["son1"][c]):
            Vs = h.basis_direct(s)
            off = tr["first"][s] - tr["first"][c]
            ref = Vt[off:off + tr["size"][s]]
            np.testing.assert_allclose(Vs @ E[s], ref, atol=1e-12 * np.abs(ref).max(), rtol=0)
    # and the stored leaf matrices are the direct bases of the leaves
    for c in range(h.C):
        if tr["son0"][c] < 0:
            rows = slice(tr["first"][c], tr["first"][c] + tr["size"][c])
            np.testing.assert_array_equal(V[rows], h.basis_direct(c))


def _lagrange_1d(nodes, x):
    """L[i, j] = the j-th Lagrange polynomial of `nodes` at x[i] (product formula)."""
    p = len(nodes)
    L = np.ones((len(x), p))
    for j in range(p):
        for q in range(p):
            if q != j:
                L[:, j] *= (x - nodes[q]) / (nodes[j] - nodes[q])
    return L


def test_transfer_is_a_kronecker_product(h):
    """Tensor nodes and tensor Lagrange polynomials make each transfer matrix the
    Kronecker product of three one-dimensional matrices, E_c = F^2 (x) F^1 (x) F^0 with
    F^d[i, j] = the father's j-th polynomial on axis d at the son's i-th node on that axis
    (node index a = a0 + p a1 + p^2 a2): the structure the device's transfer passes use."""
    h, _ = h
    tr, E, nodes = h.tree(), h.E(), h.nodes()
    p = h.p
    for c in range(1, h.C):
        par = tr["parent"][c]
        F = []
        for d in range(3):
            stride = p ** d
            nd_par = nodes[par, [stride * j for j in range(p)], d]
            nd_son = nodes[c, [stride * i for i in range(p)], d]
            F.append(_lagrange_1d(nd_par, nd_son))
        np.testing.assert_allclose(E[c], np.kron(F[2], np.kron(F[1], F[0])), atol=1e-13, rtol=0)


def test_planted_transposed_transfer_is_caught():
    """A transposed E (a plausible indexing slip) must break nestedness."""
    P = W.sphere_points(600, 32)
    h = oracle.OracleH2(P, leaf=24, p=3)
    tr = h.tree()
    E = h.E()
    h.set_E(np.ascontiguousarray(np.transpose(E, (0, 2, 1))))
    Eb = h.E()
    c = 0
    s = tr["son0"][c]
    Vt = h.basis_direct(c)[: tr["size"][s]]
    assert np.abs(h.basis_direct(s) @ Eb[s] - Vt).max() > 1e-3
