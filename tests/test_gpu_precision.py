"""Mixed precision on the GPU: FP32 / BF16 operators (FP32 accumulation) against
the oracle's emulation of the same operator, and FP64 iterative refinement.

Bars: the GPU low-precision product agrees with the oracle's emulated one to
1e-5 (FP32) / 1e-4 (BF16) per column -- both accumulate in FP32 in different
orders, and a bfloat16 rounding of an FP32 intermediate can fall on either side
of a tie between the two orders; both differ from the FP64 product by an amount
of the storage type's size; refinement reaches an FP64 true residual of 1e-10.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-4}
ERR_RANGE = {"f32": (1e-9, 2e-6), "bf16": (1e-4, 3e-2)}


def _colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


CASES = [
    ("small-k27-m4", lambda: W.SMALL.points(), W.SMALL.params(), 4),
    ("sphere-k64-m32", lambda: W.sphere_points(5000, 131), dict(ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4), 32),
    ("cube-k64-m7", lambda: W.cube_points(6000, 132), dict(ell=0.25, shift=0.5, eta=1.0, leaf=64, p=4), 7),
    # k <= 32 matrix-core coupling: several column slabs with a ragged last one, and k = 8
    # (one group of four k-steps)
    ("sphere-k27-m37", lambda: W.sphere_points(4000, 134), dict(ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3), 37),
    ("cube-k8-m20", lambda: W.cube_points(3000, 135), dict(ell=0.3, shift=1.0, eta=1.0, leaf=16, p=2), 20),
    # leaves above 64 points (several 64-row chunks per leaf) and 64 columns per work-group
    ("cube-k64-leaf100-m40", lambda: W.cube_points(5000, 136), dict(ell=0.25, shift=0.5, eta=1.0, leaf=100, p=4), 40),
]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("name,pts,prm,m", CASES, ids=[c[0] for c in CASES])
def test_lowp_product(name, pts, prm, m, prec):
    """Both leaf-stage forms of the low-precision operator (0: the built-in one contraction
    per leaf; 1: a 64-row tile per wave and term), with 32 and 64 columns per work-group,
    against the oracle's emulation of the same operator and against FP64."""
    import paper_2509_17257_amd as h2x
    P = pts()
    o = oracle.OracleH2(P, **prm)
    A = h2x.H2Matrix(P, storage=prec, **prm)
    X = W.rhs(P.shape[0], m, 133)
    emu = o.matmul_lowp(X, prec)
    ref = o.matmul(X)
    Xd = torch.from_numpy(X).cuda()
    for kind in (0, 1):
        for npl in ((1, 2) if m > 32 else (1,)):
            A.set_tune(m, leaf_kind=kind, np_leaf=npl)
            got = h2x.h2_matmul(A, Xd).cpu().numpy()
            e_emu, e64 = _colrel(got, emu), _colrel(got, ref)
            print(f"{name} {prec} leaf form {kind} np {npl}: vs emulated {e_emu:.2e}, vs FP64 {e64:.2e}")
            assert e_emu <= TOL[prec]
            lo, hi = ERR_RANGE[prec]
            assert lo < e64 < hi
    A.set_tune(m)


@pytest.mark.parametrize("prec,inner", [("f32", 1e-5), ("bf16", 1e-2)])
def test_refinement(prec, inner):
    import paper_2509_17257_amd as h2x
    w = W.SMALL
    P = w.points()
    o = oracle.OracleH2(P, **w.params())
    plan = h2x.Plan(P, **w.params())
    A = h2x.H2Matrix(plan, storage="f64")
    A_lo = h2x.H2Matrix(plan, storage=prec)
    B = w.rhs()
    X, info = h2x.block_cg_refine(A, A_lo, torch.from_numpy(B).cuda(), rtol=1e-10, inner_rtol=inner)
    X = X.cpu().numpy()
    res = np.linalg.norm(B - o.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
    print(f"refine {prec}: outer {info.outer_iters}, inner {info.iters}, oracle residual {res.max():.2e}")
    assert info.status == 0 and res.max() <= 1.5e-10
    assert np.all(info.col_relres <= 1e-10)
    Xf, _ = o.block_cg(B, rtol=1e-12)
    assert _colrel(X, Xf) <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_cg_residual_replacement(prec):
    """One CG run with the low-precision operator and FP64 residual replacement:
    FP64 true residual 1e-10 (oracle product), iteration count near the oracle's
    run of the same method on its emulated operator, graph replay bitwise equal."""
    import paper_2509_17257_amd as h2x
    w = W.SMALL
    P = w.points()
    o = oracle.OracleH2(P, **w.params())
    plan = h2x.Plan(P, **w.params())
    A = h2x.H2Matrix(plan, storage="f64")
    A_lo = h2x.H2Matrix(plan, storage=prec)
    B = w.rhs()
    Bd = torch.from_numpy(B).cuda()
    X, info = h2x.block_cg_mixed(A, A_lo, Bd, rtol=1e-10)
    Xg, ig = h2x.block_cg_mixed(A, A_lo, Bd, rtol=1e-10, graph=True)
    assert torch.equal(X, Xg) and ig.iters == info.iters
    X = X.cpu().numpy()
    res = np.linalg.norm(B - o.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
    _, oi = o.block_cg_mixed(B, prec, rtol=1e-10)
    _, i64 = o.block_cg(B, rtol=1e-10)
    print(f"mixed {prec}: gpu {info.iters} it / {info.outer_iters} replacements, oracle {oi['iters']} it / "
          f"{oi['replacements']}, FP64 CG {i64['iters']} it, true residual {res.max():.2e}")
    assert info.status == 0 and res.max() <= 1.5e-10
    assert np.all(info.col_relres <= 1e-10)
    assert abs(info.iters - oi["iters"]) <= max(5, 0.1 * oi["iters"])


def test_precision_workload_full_size():
    """The precision workload at full size (cube, n = 262144, k = 64, m = 64), products in
    FP64, FP32 and BF16 storage as the bench times them (64 columns).  The oracle runs on a
    sample of four of the columns (each column of the product depends on its own column
    of X only): FP64 to 1e-12 per column; FP32 and BF16 against the FP64 product within the
    ranges their storage gives (the emulated low-precision operator is checked on the
    smaller cases above)."""
    import paper_2509_17257_amd as h2x
    w = W.PRECISION
    P = w.points()
    X = w.rhs()
    cols = [0, 21, 42, 63]
    plan = h2x.Plan(P, **w.params())
    got = {}
    for prec in ("f64", "f32", "bf16"):
        print(f"[full] precision workload, {prec} product, m = {X.shape[1]}", flush=True)
        A = h2x.H2Matrix(plan, storage=prec)
        got[prec] = h2x.h2_matmul(A, torch.from_numpy(X).cuda()).cpu().numpy()
        del A
        torch.cuda.empty_cache()
    print("[full] oracle on the sampled columns", flush=True)
    o = oracle.OracleH2(P, **w.params())
    ref = o.matmul(np.ascontiguousarray(X[:, cols]))
    del o
    e64 = _colrel(got["f64"][:, cols], ref)
    errs = {p: _colrel(got[p], got["f64"]) for p in ("f32", "bf16")}
    print(f"[full] FP64 vs oracle {e64:.2e}; FP32 vs FP64 {errs['f32']:.2e}; BF16 vs FP64 {errs['bf16']:.2e}")
    assert e64 <= 1e-12
    # an entry of the product sums K ~ 10^3 .. 10^4 FP32 products (the lists and near blocks
    # of a row, the transfer levels): the rounding grows like sqrt(K) u, u = 2^-24 (FP32) or
    # 2^-8 (BF16 storage), so the full size gets the bounds 1e-5 and 3e-2
    full = {"f32": (1e-9, 1e-5), "bf16": (1e-4, 3e-2)}
    for p, e in errs.items():
        lo, hi = full[p]
        assert lo < e < hi


# ---- the hand-worked rounding points (reading R16), on the GPU ----

@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_lowp_rounding_points_hand_worked(prec):
    """The GPU's BF16 / FP32 operators on the hand-worked case of tests/golden/lowp_line16.json
    (16 points on a line, p = 1, constant kernel): the product equals the values worked by
    hand from the rounding points, independently of the oracle."""
    import json
    import os
    import paper_2509_17257_amd as h2x
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lowp_line16.json")))
    P = np.zeros((16, 3))
    P[:, 0] = g["points_x"]
    A = h2x.H2Matrix(P, kernel="const", storage=prec, ell=1.0, shift=g["shift"], eta=g["eta"],
                     leaf=g["leaf_size"], p=1)
    X = np.zeros((16, len(g["columns"])))
    for j, col in enumerate(g["columns"]):
        for i, v in col["x_nonzero"].items():
            X[int(i), j] = v
    got = h2x.h2_matmul(A, torch.from_numpy(X).cuda()).cpu().numpy()
    yb = np.array([c["y_bf16"] for c in g["columns"]]).T
    ye = np.array([c["y_exact"] for c in g["columns"]]).T
    want = yb if prec == "bf16" else np.concatenate([ye[:, :3], yb[:, 3:]], axis=1)
    for j in range(X.shape[1]):
        print(f"{prec} column {j}: got {got[:, j].tolist()}")
    np.testing.assert_array_equal(got, want)


# ---- solves that cannot converge return their best iterate ----

def test_recovery_returns_best_iterate_when_it_cannot_converge():
    """Unit-cube points, length scale 1, shift 1e-3 (kappa 1.3e5, BF16 operator error
    2e-3): BF16 refinement and BF16 residual replacement cannot converge.  Both report
    it, and every returned column has a true residual (oracle product) at most that of
    X0 = 0; the reported residuals are those of the returned columns."""
    import paper_2509_17257_amd as h2x
    P = np.random.default_rng(131).random((1500, 3))
    prm = dict(ell=1.0, shift=1e-3, eta=1.0, leaf=32, p=3)
    o = oracle.OracleH2(P, **prm)
    plan = h2x.Plan(P, **prm)
    A = h2x.H2Matrix(plan, storage="f64")
    A_lo = h2x.H2Matrix(plan, storage="bf16")
    B = W.rhs(1500, 3, 132)
    Bd = torch.from_numpy(B).cuda()
    runs = {
        "refine": h2x.block_cg_refine(A, A_lo, Bd, rtol=1e-10, inner_rtol=1e-2, max_outer=8, max_inner=150),
        "mixed": h2x.block_cg_mixed(A, A_lo, Bd, rtol=1e-10, max_iter=300),
    }
    for name, (X, info) in runs.items():
        X = X.cpu().numpy()
        rel = np.linalg.norm(B - o.matmul(X), axis=0) / np.linalg.norm(B, axis=0)
        print(f"{name}: status {info.status}, returned true residuals {rel}, reported {info.col_relres}")
        assert info.status in (4, 5)
        assert (rel <= 1.0).all()
        np.testing.assert_allclose(info.col_relres, rel, rtol=1e-8)


# ---- FP64 recovery at the precision workload's full size ----

def test_precision_workload_solves():
    """The precision workload at full size (cube, n = 262144, k = 64, m = 64).  FP32 storage:
    residual replacement and restarted refinement both reach an FP64 true residual of 1e-10,
    measured with the FP64 product (pinned against the oracle by the full-size product test).
    BF16 storage: the operator's error (1e-2 of the product) times the condition number
    (lambda_min >= 0.5 from the shift, lambda_max ~ 2e4) is far above 1, so neither method
    can converge; both say so and return iterates no worse than X0 = 0."""
    import paper_2509_17257_amd as h2x
    w = W.PRECISION
    P = w.points()
    plan = h2x.Plan(P, **w.params())
    B = torch.from_numpy(w.rhs()).cuda()
    A = h2x.H2Matrix(plan, storage="f64")

    def true_rel(X):
        R = B - h2x.h2_matmul(A, X)
        return (R.norm(dim=0) / B.norm(dim=0)).cpu().numpy()

    for prec in ("f32", "bf16"):
        A_lo = h2x.H2Matrix(plan, storage=prec)
        legs = [("mixed", lambda: h2x.block_cg_mixed(A, A_lo, B, rtol=1e-10, max_iter=3000 if prec == "f32" else 400,
                                                      graph=True)),
                ("refine", lambda: h2x.block_cg_refine(A, A_lo, B, rtol=1e-10, inner_rtol=1e-6 if prec == "f32" else 1e-2,
                                                        max_outer=8, max_inner=2000 if prec == "f32" else 300))]
        for name, run in legs:
            print(f"[full] {prec} {name}", flush=True)
            X, info = run()
            rel = true_rel(X)
            print(f"[full] {prec} {name}: status {info.status}, iters {info.iters}, outer {info.outer_iters}, "
                  f"max true residual {rel.max():.3e}", flush=True)
            np.testing.assert_allclose(info.col_relres, rel, rtol=1e-6, atol=1e-14)
            if prec == "f32":
                assert info.status == 0 and rel.max() <= 1e-10
            else:
                assert info.status in (4, 5) and rel.max() <= 1.0
        del A_lo
        torch.cuda.empty_cache()
