"""Pins of the oracle's low-precision operator and mixed-precision refinement.

* The bfloat16 rounding helper agrees with torch's FP32 -> bfloat16 conversion
  (round to nearest even) on random, tie and special values.
* The emulated FP32 / BF16 operators differ from the FP64 product by an amount of
  the storage type's size (nonzero, and within a small multiple of its unit
  roundoff), and are exactly the FP64 product when every stored factor and every
  rounded operand is exact in that type (constant kernel, integer right-hand sides).
* Refinement reaches an FP64 true residual of 1e-10 and agrees with the FP64
  block-CG solution to within the condition number times the tolerance.
* CG with residual replacement (iterations with the emulated operator, residual
  recomputed in FP64) meets 1e-10 on the true residual, agrees with a dense
  Cholesky solve within kappa * rtol, and solves sigma I + 1 1^T in a few steps.
* The rounding points of the emulation (reading R16) are pinned by a hand-worked
  product (tests/golden/lowp_line16.json): 16 points on a line, p = 1, constant
  kernel, right-hand sides whose x-hat and y-hat at inner clusters are not
  bfloat16 numbers.  Switching off any one rounding point (a planted slip)
  changes the product.
* A refinement or residual-replacement run that cannot converge (a bfloat16
  operator on a system whose condition number times the operator error exceeds
  1) returns, per column, its iterate with the smallest true residual, so the
  returned residual is at most that of X0 = 0.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def test_bf16_rounding_matches_torch():
    g = np.random.default_rng(5)
    vals = np.concatenate([
        g.standard_normal(100000).astype(np.float32) * np.float32(10.0) ** g.integers(-20, 20, 100000).astype(np.float32),
        # exact ties between two bfloat16 values (low 16 bits = 0x8000)
        (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 1.0, 3.0e38, 1e-40], np.float32),
    ])
    ours = oracle.round_bf16(vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(ours, ref)
    assert np.isnan(oracle.round_bf16(np.array([np.nan], np.float32))[0])


@pytest.fixture(scope="module")
def h():
    P = W.sphere_points(2000, 121)
    return oracle.OracleH2(P, leaf=32, p=3, ell=0.5, shift=1.0)


@pytest.mark.parametrize("prec,lo,hi", [("f32", 1e-9, 2e-6), ("bf16", 1e-4, 3e-2)])
def test_lowp_error_size(h, prec, lo, hi):
    X = W.rhs(h.n, 4, 122)
    e = _colrel(h.matmul_lowp(X, prec), h.matmul(X))
    assert lo < e < hi, e


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_lowp_exact_when_everything_is_representable(prec):
    # constant kernel: S = 1, near field = 1 + shift on the diagonal (exact in both types
    # for shift = 0.5); with p = 1 every basis entry and transfer entry is exactly 1; X holds
    # small integers, so every partial sum is an integer below 2^24 and exact in FP32.
    P = W.sphere_points(700, 123)
    hc = oracle.OracleH2(P, kernel="const", leaf=16, p=1, shift=0.5)
    assert hc.n_adm > 0
    X = np.random.default_rng(124).integers(-3, 4, (700, 3)).astype(np.float64)
    np.testing.assert_array_equal(hc.matmul_lowp(X, prec), hc.matmul(X))


def test_refinement_reaches_fp64_accuracy(h):
    B = W.rhs(h.n, 3, 125)
    Xf, _ = h.block_cg(B, rtol=1e-12)
    A = h.dense()
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    for prec, inner in (("f32", 1e-5), ("bf16", 1e-2)):
        X, info = h.refine_cg(B, prec, rtol=1e-10, inner_rtol=inner)
        res = np.linalg.norm(B - h.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
        assert res.max() <= 1e-10, (prec, info, res)
        assert _colrel(X, Xf) <= kappa * 2e-10
        assert info["outer"] >= 2


# ---- mixed precision in one CG run (residual replacement) ----

@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_cg_reaches_fp64_accuracy(h, prec):
    """Iterations with the low-precision operator, residual recomputed in FP64: the
    solve meets 1e-10 on the FP64 true residual and agrees with a dense Cholesky
    solve of the assembled H^2 matrix within the condition number times rtol."""
    import scipy.linalg as sla
    B = W.rhs(h.n, 3, 191)
    X, info = h.block_cg_mixed(B, prec, rtol=1e-10)
    res = np.linalg.norm(B - h.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 1e-10
    assert info["replacements"] >= 1
    A = h.dense()
    ev = np.linalg.eigvalsh(A)
    Xd = sla.cho_solve(sla.cho_factor(A), B)
    assert _colrel(X, Xd) <= (ev[-1] / ev[0]) * 1e-10
    # a replacement restarts nothing: the iteration count stays near the FP64 one
    _, i64 = h.block_cg(B, rtol=1e-10)
    assert info["iters"] <= 3 * i64["iters"]


def test_mixed_cg_constant_kernel_closed_form():
    """A = sigma I + 1 1^T has two eigenvalues, so CG on it converges in two steps.
    With the FP32 operator (relative error 7e-7 here, kappa ~800) a replacement
    cycle cuts the true residual by about kappa times that error, so the
    Sherman-Morrison solution is reached to 1e-10 within a few short cycles (13
    iterations and 7 replacements with a check every iteration)."""
    n, sigma = 700, 0.9
    o = oracle.OracleH2(W.sphere_points(n, 192), kernel="const", leaf=32, p=2, shift=sigma)
    B = W.rhs(n, 2, 193)
    X, info = o.block_cg_mixed(B, "f32", rtol=1e-11, check=1)
    Xcf = (B - B.sum(0, keepdims=True) / (sigma + n)) / sigma
    assert _colrel(X, Xcf) <= 1e-10
    assert info["iters"] <= 20 and info["replacements"] <= 10


# ---- hand-worked rounding points (reading R16) ----

def _line16():
    g = json.load(open(os.path.join(GOLD, "lowp_line16.json")))
    P = np.zeros((16, 3))
    P[:, 0] = g["points_x"]
    o = oracle.OracleH2(P, kernel="const", leaf=g["leaf_size"], p=1, eta=g["eta"], shift=g["shift"])
    X = np.zeros((16, len(g["columns"])))
    for j, col in enumerate(g["columns"]):
        for i, v in col["x_nonzero"].items():
            X[int(i), j] = v
    Yb = np.array([c["y_bf16"] for c in g["columns"]], dtype=np.float64).T
    Ye = np.array([c["y_exact"] for c in g["columns"]], dtype=np.float64).T
    return g, o, X, Yb, Ye


def test_line16_structure_is_the_hand_worked_one():
    """The derivation assumes this tree and these lists: check them first."""
    g, o, X, Yb, Ye = _line16()
    tr = o.tree()
    assert o.C == len(g["clusters_preorder"])
    for c in g["clusters_preorder"]:
        i = c["id"]
        lo, hi = c["members"]
        assert tr["first"][i] == lo and tr["size"][i] == hi - lo + 1
        sons = [int(tr["son0"][i]), int(tr["son1"][i])] if tr["son0"][i] >= 0 else []
        assert sons == c["sons"]
    assert list(tr["perm"]) == list(range(16))
    b = o.blocks()
    for t in range(o.C):
        got = [[int(b["s"][q]), "adm" if b["adm"][q] else "near"]
               for q in b["list_blk"][b["list_ptr"][t]:b["list_ptr"][t + 1]]]
        assert got == g["lists"].get(str(t), []), t


def test_lowp_rounding_points_hand_worked():
    """BF16 emulation equals the hand-worked product exactly; FP32 storage equals the
    exact product where every value is an FP32 number (columns 1-3) and the hand-worked
    FP32 sums in column 4; the FP64 product is the exact A = 11^T + 0.5 I product."""
    g, o, X, Yb, Ye = _line16()
    np.testing.assert_array_equal(o.matmul_lowp(X, "bf16"), Yb)
    Yf = o.matmul_lowp(X, "f32")
    np.testing.assert_array_equal(Yf[:, :3], Ye[:, :3])
    np.testing.assert_array_equal(Yf[:, 3], Yb[:, 3])
    np.testing.assert_array_equal(o.matmul(X), Ye)
    # the exact product is the closed form (1 1^T + 0.5 I) X
    np.testing.assert_array_equal(Ye, X.sum(0, keepdims=True) + 0.5 * X)


@pytest.mark.parametrize("slip", sorted(oracle.LOWP_OMIT))
def test_lowp_planted_rounding_slip_is_caught(slip):
    g, o, X, Yb, Ye = _line16()
    Yp = o.matmul_lowp(X, "bf16", omit=oracle.LOWP_OMIT[slip])
    assert not np.array_equal(Yp, Yb), slip


# ---- solves that cannot converge return their best iterate ----

@pytest.fixture(scope="module")
def hard():
    """Unit-cube points, length scale 1 and shift 1e-3: the dense H^2 matrix has
    lambda_min 6.2e-3 and lambda_max 798 (kappa 1.3e5), and the bfloat16 operator's
    error is 2.2e-3 of the product, so kappa times the error is far above 1: neither
    refinement nor residual replacement can converge (refinement diverges at once)."""
    P = np.random.default_rng(131).random((1500, 3))
    return oracle.OracleH2(P, leaf=32, p=3, ell=1.0, shift=1e-3)


def _true_rel(o, B, X):
    return np.linalg.norm(B - o.matmul(X), axis=0) / np.linalg.norm(B, axis=0)


def test_refinement_returns_best_iterate_when_it_stalls(hard):
    B = W.rhs(hard.n, 3, 132)
    X, info = hard.refine_cg(B, "bf16", rtol=1e-10, inner_rtol=1e-2, max_outer=8, max_inner=150)
    rel = _true_rel(hard, B, X)
    assert info["status"] == 5
    np.testing.assert_allclose(info["col_relres"], rel, rtol=1e-12)
    assert (rel <= 1.0).all()
    # the returned columns are the best outer iterates: no later outer step of the same
    # (deterministic) run is better than what was returned
    for outer in range(0, info["outer"] + 1):
        Xo, io = hard.refine_cg(B, "bf16", rtol=1e-10, inner_rtol=1e-2, max_outer=outer, max_inner=150)
        assert (rel <= _true_rel(hard, B, Xo) * (1 + 1e-12)).all(), outer


def test_mixed_cg_returns_best_iterate_on_breakdown_or_budget(hard):
    B = W.rhs(hard.n, 3, 133)
    X, info = hard.block_cg_mixed(B, "bf16", rtol=1e-10, max_iter=300, check=4)
    rel = _true_rel(hard, B, X)
    assert info["status"] in (4, 5)
    np.testing.assert_allclose(info["col_relres"], rel, rtol=1e-12)
    assert (rel <= 1.0).all()


def test_best_iterate_rule_leaves_converged_solves_alone(h):
    """When every column converges the returned iterate meets rtol (the rule picks the
    smallest true residual, which is then at most rtol)."""
    B = W.rhs(h.n, 2, 134)
    for fn in (lambda: h.refine_cg(B, "f32", rtol=1e-10, inner_rtol=1e-5),
               lambda: h.block_cg_mixed(B, "f32", rtol=1e-10)):
        X, info = fn()
        assert info["status"] == 0
        rel = _true_rel(h, B, X)
        assert rel.max() <= 1e-10
        np.testing.assert_allclose(info["col_relres"], rel, rtol=0, atol=1e-13)
