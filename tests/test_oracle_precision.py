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
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")


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
