"""GPU parity of the H^2 x X product (C ABI h2x_matmul) against the CPU oracle.

Bar (FP64): per column, ||Y_gpu - Y_oracle|| / ||Y_oracle|| <= 1e-12, on the same
seeded inputs, at sizes that span several tiles and ragged tails, at the full
FP64 throughput size, and on the edge cases (m = 1, ragged m, leaves larger
than one tile, no admissible block, a single leaf, alpha/beta, tree order).
The main cases and the full size also bound every entry: per column,
max_i |Y_gpu - Y_oracle|_i <= 1e-12 max_i |Y_oracle|_i, so that an error confined
to a few rows cannot hide in a column norm.
"""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _h2x():
    import paper_2509_17257_amd as h2x
    return h2x


def _colrel(a, b):
    den = np.linalg.norm(b, axis=0)
    den[den == 0] = 1.0
    return (np.linalg.norm(a - b, axis=0) / den).max()


def _entrel(a, b):
    """Largest entry-wise difference of each column over that column's largest entry."""
    den = np.abs(b).max(axis=0)
    den[den == 0] = 1.0
    return (np.abs(a - b).max(axis=0) / den).max()


def _pair(P, **kw):
    h2x = _h2x()
    return oracle.OracleH2(P, **kw), h2x.H2Matrix(P, **kw)


def _gpu(A, X, **kw):
    h2x = _h2x()
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    if "out" in kw and isinstance(kw["out"], np.ndarray):
        kw["out"] = torch.from_numpy(np.ascontiguousarray(kw["out"])).cuda()
    Y = h2x.h2_matmul(A, Xd, **kw)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


CASES = [
    # name, points, params, m
    ("small-k27-m4", lambda: W.SMALL.points(), W.SMALL.params(), 4),
    ("small-k27-m1", lambda: W.SMALL.points(), W.SMALL.params(), 1),
    ("small-k27-m37", lambda: W.SMALL.points(), W.SMALL.params(), 37),
    ("sphere-k64-m32", lambda: W.sphere_points(6000, 81), dict(ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4), 32),
    ("cube-k64-m5", lambda: W.cube_points(7000, 82), dict(ell=0.25, shift=0.5, eta=1.0, leaf=64, p=4), 5),
    ("cube-k8-leaf100", lambda: W.cube_points(3000, 83), dict(ell=0.3, shift=0.5, eta=1.5, leaf=100, p=2), 3),
    ("line-k27", lambda: W.line_points(2000, 84), dict(ell=0.2, shift=1.0, eta=1.0, leaf=16, p=3), 7),
    ("sphere-k125-m9", lambda: W.sphere_points(3000, 85), dict(ell=0.5, shift=1.0, eta=1.0, leaf=64, p=5), 9),
    ("cube-k64-m64", lambda: W.cube_points(5000, 101), dict(ell=0.25, shift=0.5, eta=1.0, leaf=64, p=4), 64),
    ("sphere-k64-m100", lambda: W.sphere_points(4000, 102), dict(ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4), 100),
    ("sphere-k64-leaf150-m17", lambda: W.sphere_points(4000, 103), dict(ell=0.5, shift=1.0, eta=1.0, leaf=150, p=4),
     17),
    ("line-k64-m3", lambda: W.line_points(3000, 104), dict(ell=0.2, shift=1.0, eta=1.0, leaf=40, p=4), 3),
]


@pytest.mark.parametrize("name,pts,prm,m", CASES, ids=[c[0] for c in CASES])
def test_matmul_matches_oracle(name, pts, prm, m):
    P = pts()
    o, A = _pair(P, **prm)
    X = W.rhs(P.shape[0], m, 90 + m)
    ref = o.matmul(X)
    got = _gpu(A, X)
    err, ent = _colrel(got, ref), _entrel(got, ref)
    print(f"{name}: n={P.shape[0]} adm={o.n_adm} near={o.n_near} max col rel err={err:.3e}, entries {ent:.3e}")
    assert err <= TOL and ent <= TOL


ROWS = [c for c in CASES if c[0] in ("small-k27-m37", "sphere-k64-m32", "cube-k64-m5", "cube-k8-leaf100",
                                      "line-k27", "cube-k64-m64", "sphere-k64-m100", "sphere-k64-leaf150-m17")]


# leaf-stage forms: 1 a 64-row tile per wave and term, 2 a wave per 32-row band, 3 the near
# blocks and the basis as one contraction per leaf (16-row tiles; its near field also in
# shares inside the transfer-level launches, overlap 5, on the second stream, overlap 1, or
# in two halves on the second stream beside the upward and the downward pass, overlap 6)
LEAF_FORMS = [(1, (2, 1)), (2, (2, 1)), (3, (2, 1, 5, 6))]


@pytest.mark.parametrize("kind,overlaps", LEAF_FORMS, ids=[f"kind{k}" for k, _ in LEAF_FORMS])
@pytest.mark.parametrize("name,pts,prm,m", ROWS, ids=[c[0] for c in ROWS])
def test_leaf_forms_match_oracle(name, pts, prm, m, kind, overlaps):
    """Every leaf-stage form, with 32 and 64 columns per work-group, alone and with each
    placement of the near field, against the oracle per column and entry by entry; alpha /
    beta in original and in tree order (leaves above 64 points: several row chunks)."""
    h2x = _h2x()
    P = pts()
    o, A = _pair(P, **prm)
    n = P.shape[0]
    X = W.rhs(n, m, 190 + m)
    ref = o.matmul(X)
    errs = []
    for npl in (1, 2):
        for ov in overlaps:
            A.set_tune(m, leaf_kind=kind, np_leaf=npl, overlap=ov)
            assert A.get_tune(m)["np_leaf"] == npl
            got = _gpu(A, X)
            errs.append(max(_colrel(got, ref), _entrel(got, ref)))
    Y0 = W.rhs(n, m, 191)
    A.set_tune(m, leaf_kind=kind)
    err_ab = _colrel(_gpu(A, X, alpha=0.75, beta=-1.5, out=Y0), 0.75 * ref - 1.5 * Y0)
    perm = A.plan.perm()
    got_t = _gpu(A, X[perm], alpha=2.0, tree_order=True)
    err_t = _colrel(got_t, 2.0 * ref[perm])
    A.set_tune(m)
    print(f"{name}: leaf form {kind} max err {max(errs):.3e}, alpha/beta {err_ab:.3e}, tree order {err_t:.3e}")
    assert max(errs) <= TOL and err_ab <= TOL and err_t <= TOL


SPLIT = [c for c in CASES if c[0] in ("small-k27-m37", "cube-k64-m5", "cube-k64-m64")] + [
    ("sphere20000-k27-m9", lambda: W.sphere_points(20000, 5), dict(ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3), 9)]


@pytest.mark.parametrize("name,pts,prm,m", SPLIT, ids=[c[0] for c in SPLIT])
def test_split_coupling_matches_oracle(name, pts, prm, m):
    """The coupling rows in two parts (split 1, with the LDS reserve, and 3): the deep part
    on the operator's second stream beside the upper transfer levels, the other rows and
    the upper downward levels on the caller's stream.  Against the oracle, and bitwise equal to the one
    launch (each row's blocks are summed in the same order); alpha / beta."""
    P = pts()
    o, A = _pair(P, **prm)
    assert A.plan.split_depth > A.plan.adm_depth + 1 and 0 < A.plan.deep_blocks < A.plan.n_adm
    n = P.shape[0]
    X = W.rhs(n, m, 200 + m)
    ref = o.matmul(X)
    # the near field in the leaf stage in every run (the split schedule does not place it in
    # shares beside the transfer levels), so that the three runs sum alike
    A.set_tune(m, split=2, overlap=2)
    one = _gpu(A, X)
    A.set_tune(m, split=3, overlap=2)
    got3 = _gpu(A, X)
    A.set_tune(m, split=1, overlap=2)
    got = _gpu(A, X)
    Y0 = W.rhs(n, m, 201)
    err_ab = _colrel(_gpu(A, X, alpha=-1.25, beta=0.5, out=Y0), 0.5 * Y0 - 1.25 * ref)
    A.set_tune(m)
    err = _colrel(got, ref)
    print(f"{name}: split depth {A.plan.split_depth} (deep blocks {A.plan.deep_blocks} of {A.plan.n_adm}), "
          f"err {err:.3e}, alpha/beta {err_ab:.3e}")
    assert np.array_equal(got, one) and np.array_equal(got3, one)
    assert err <= TOL and err_ab <= TOL


def test_set_get_tune():
    h2x = _h2x()
    A = h2x.H2Matrix(W.sphere_points(2000, 192), ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
    assert all(v == 0 for v in A.get_tune(20).values())
    A.set_tune(20, nj_coupling=2, leaf_kind=2, np_leaf=1, overlap=1, split=2)
    # one entry per ceil(m / 16): 17..32 share it, 16 and 33 do not
    assert A.get_tune(17) == A.get_tune(32) == dict(nj_transfer=0, nj_coupling=2, np_leaf=1, overlap=1, fuse_up=0,
                                                    leaf_kind=2, split=2)
    assert A.get_tune(16)["leaf_kind"] == 0 and A.get_tune(33)["leaf_kind"] == 0
    for bad in (dict(nj_coupling=5), dict(leaf_kind=4), dict(split=4), dict(np_leaf=-1), dict(overlap=7), dict(fuse_up=3)):
        with pytest.raises(h2x.H2xError, match="out of range"):
            A.set_tune(20, **bad)
    with pytest.raises(ValueError):
        A.set_tune(20, nj_foo=1)
    A.set_tune(20)
    assert all(v == 0 for v in A.get_tune(20).values())


def test_polynomial_kernel_equals_dense():
    P = W.sphere_points(3000, 86)
    h2x = _h2x()
    A = h2x.H2Matrix(P, kernel="poly", shift=0.75, leaf=32, p=3)
    X = W.rhs(3000, 6, 87)
    ref = oracle.kernel_matrix(P, kernel="poly", shift=0.75) @ X
    assert _colrel(_gpu(A, X), ref) <= TOL


@pytest.mark.parametrize("kw", [dict(leaf=16, eta=1e-12), dict(leaf=1000)])
def test_dense_only_cases(kw):
    P = W.sphere_points(700, 88)
    h2x = _h2x()
    A = h2x.H2Matrix(P, ell=0.5, shift=1.0, p=3, **kw)
    assert A.plan.n_adm == 0
    X = W.rhs(700, 33, 89)
    ref = oracle.kernel_matrix(P, ell=0.5, shift=1.0) @ X
    assert _colrel(_gpu(A, X), ref) <= TOL


def test_alpha_beta_and_tree_order():
    P = W.SMALL.points()
    o, A = _pair(P, **W.SMALL.params())
    X = W.rhs(P.shape[0], 6, 91)
    Y0 = W.rhs(P.shape[0], 6, 92)
    ref = o.matmul(X, alpha=-0.7, beta=1.3, Y=Y0)
    got = _gpu(A, X, alpha=-0.7, beta=1.3, out=Y0.copy())
    assert _colrel(got, ref) <= TOL
    # beta = 0 ignores NaN in the output buffer
    nanY = np.full_like(Y0, np.nan)
    got = _gpu(A, X, alpha=2.0, beta=0.0, out=nanY)
    assert _colrel(got, 2.0 * o.matmul(X)) <= TOL
    # tree-ordered input and output
    perm = A.plan.perm()
    got_t = _gpu(A, X[perm], tree_order=True)
    back = np.empty_like(got_t)
    back[perm] = got_t
    assert _colrel(back, o.matmul(X)) <= TOL


def test_bitwise_deterministic_and_column_independent():
    P = W.sphere_points(5000, 93)
    h2x = _h2x()
    A = h2x.H2Matrix(P, leaf=64, p=4)
    X = W.rhs(5000, 16, 94)
    a = _gpu(A, X)
    b = _gpu(A, X)
    np.testing.assert_array_equal(a, b)
    for i in (0, 7, 15):
        c = _gpu(A, X[:, i:i + 1].copy())
        assert _colrel(c, a[:, i:i + 1]) <= 1e-14


def test_full_fp64_workload():
    """The FP64 throughput workload at full size (n = 65536, k = 64, m = 32)."""
    w = W.FP64
    P = w.points()
    o, A = _pair(P, **w.params())
    X = w.rhs()
    ref = o.matmul(X)
    got = _gpu(A, X)
    err, ent = _colrel(got, ref), _entrel(got, ref)
    print(f"{w.name}: adm={o.n_adm} near={o.n_near} max col rel err={err:.3e}, entries {ent:.3e}")
    assert err <= TOL and ent <= TOL


def test_invalid_arguments_on_gpu():
    h2x = _h2x()
    P = W.sphere_points(500, 95)
    A = h2x.H2Matrix(P, leaf=32, p=3)
    X = torch.zeros((500, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(h2x.H2xError):
        h2x.h2_matmul(A, X, out=X)  # X and Y overlap
    with pytest.raises(ValueError):
        h2x.h2_matmul(A, torch.zeros((499, 4), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("storage,m", [("f64", 32), ("f64", 5), ("f64", 64), ("f32", 40), ("bf16", 20)])
def test_autotune_keeps_results(storage, m):
    """Autotuned tile shapes change only the work distribution (fixed summation order
    per element); the placement of the near field changes only whether the near and
    basis terms reach Y in one step or two, and the leaf-stage forms sum the terms in
    different orders: rounding-level changes.  A choice with the built-in leaf form and
    near-field placement is bitwise the built-in product."""
    h2x = _h2x()
    P = W.sphere_points(8000, 121)
    A = h2x.H2Matrix(P, storage=storage, ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
    X = torch.from_numpy(W.rhs(8000, m, 122)).cuda()
    before = h2x.h2_matmul(A, X).clone()
    info = A.autotune(m)
    after = h2x.h2_matmul(A, X)
    torch.cuda.synchronize()
    print(f"{storage} m={m}: {info}")
    assert info["ms_tuned"] <= info["ms_default"] * 1.0001
    builtin_form = info["leaf_kind"] in (0, 3) and (storage != "f64" or info["overlap"] in (0, 5))
    if builtin_form:
        assert torch.equal(before, after)
    else:
        # another leaf-stage form or near-field placement: the same terms summed in another
        # order (FP64 sums; FP32 sums for the low-precision operators, whose last stage is the
        # leaf stage, so no rounding to BF16 follows the changed sums)
        rel = ((after - before).norm(dim=0) / before.norm(dim=0)).max().item()
        assert rel <= (1e-14 if storage == "f64" else 1e-5)


def test_stage_timer():
    """h2x_matmul_marked: the same product as h2x_matmul (bitwise), stage boundaries recorded
    per slot without waiting; h2x_timer_read returns positive stage times whose sum is the
    product's time; bad slots are refused."""
    h2x = _h2x()
    P = W.sphere_points(6000, 81)
    A = h2x.H2Matrix(P, ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
    X = torch.from_numpy(W.rhs(6000, 32, 205)).cuda()
    ref = h2x.h2_matmul(A, X).clone()
    T = h2x.Timer(3)
    outs = [h2x.h2_matmul(A, X, timer=T, slot=i).clone() for i in range(3)]
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(outs[i], ref)
        st = T.read(i)
        assert st.shape == (len(h2x.STAGES),) and (st > 0).all() and st.sum() < 100.0
    with pytest.raises(h2x.H2xError):
        h2x.h2_matmul(A, X, timer=T, slot=3)
    with pytest.raises(h2x.H2xError):
        T.read(-1)
