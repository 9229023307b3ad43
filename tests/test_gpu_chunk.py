"""Right-hand-side chunking on the GPU (section 5, memory-footprint remarks): chunked
block CG and block GMRES against the unchunked solves and the oracle, the plan-only
workspace sizes against the operators' own, and the throughput curve.

Columns of both solvers are independent processes that share only the products, so a
chunked solve (columns frozen once converged for CG) reaches the unchunked solution
within the end-to-end bound of the solver (the row blocking of the reductions, and so
the rounding, may differ with the column count), with per-column iteration counts
within the bound used for CG parity, and true residuals within the tolerance."""
import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _h2x():
    import paper_2509_17257_amd as h2x
    return h2x


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _colrel(a, b):
    den = np.linalg.norm(b, axis=0)
    den[den == 0] = 1.0
    return (np.linalg.norm(a - b, axis=0) / den).max()


@pytest.fixture(scope="module")
def setup():
    h2x = _h2x()
    P = W.sphere_points(3000, 93)
    prm = dict(ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3)
    return oracle.OracleH2(P, **prm), h2x.H2Matrix(P, **prm), W.rhs(3000, 10, 94)


def test_plan_workspace_matches_operator(setup):
    h2x = _h2x()
    _, A, _ = setup
    lib = h2x.load_library()
    for m in (1, 7, 32):
        assert h2x.solve_workspace_bytes(A.plan, m, solver="cg") == lib.h2x_block_cg_workspace_bytes(A._h, m)
        assert h2x.solve_workspace_bytes(A.plan, m, solver="gmres", restart=12) == \
            lib.h2x_block_gmres_workspace_bytes(A._h, m, 12)


def test_throughput_curve(setup):
    _, A, _ = setup
    ms = A.product_times([1, 8, 32], reps=3)
    print("curve", ms)
    assert all(t > 0 for t in ms)


def test_chunked_cg_matches_unchunked_and_oracle(setup):
    h2x = _h2x()
    o, A, B = setup
    Bd = _dev(B)
    rtol = 1e-9
    Xu, iu = h2x.block_cg_solve(A, Bd, rtol=rtol, freeze_converged=True)
    Xc, ic = h2x.block_cg_solve_chunked(A, Bd, 4, rtol=rtol, freeze_converged=True)
    Xu, Xc = Xu.cpu().numpy(), Xc.cpu().numpy()
    err = _colrel(Xc, Xu)
    Xo, io = o.block_cg(B, rtol=rtol, freeze_converged=True)
    print(f"CG chunked vs unchunked {err:.2e}, vs oracle {_colrel(Xc, Xo):.2e}; chunk iters {ic.iters}")
    assert err <= 100 * rtol
    assert (np.abs(ic.col_iters - iu.col_iters) <= np.maximum(2, iu.col_iters // 20)).all()
    assert ic.status == 0 and (ic.col_status == 0).all()
    res = np.linalg.norm(B - o.matmul(Xc), axis=0) / np.linalg.norm(B, axis=0)
    assert (res <= 1.01 * rtol).all()
    assert (np.abs(ic.col_iters - io["col_iters"]) <= np.maximum(2, io["col_iters"] // 20)).all()


def test_chunked_gmres_matches_unchunked_and_oracle(setup):
    h2x = _h2x()
    o, A, B = setup
    Bd = _dev(B)
    rtol = 1e-9
    Xu, iu = h2x.block_gmres_solve(A, Bd, rtol=rtol, restart=12)
    Xc, ic = h2x.block_gmres_solve_chunked(A, Bd, 3, rtol=rtol, restart=12)
    Xu, Xc = Xu.cpu().numpy(), Xc.cpu().numpy()
    err = _colrel(Xc, Xu)
    Xo, io = o.block_gmres(B, rtol=rtol, restart=12)
    print(f"GMRES chunked vs unchunked {err:.2e}, vs oracle {_colrel(Xc, Xo):.2e}; steps {ic.col_iters.tolist()} "
          f"oracle {io['col_iters'].tolist()}; estimates {ic.col_res.tolist()} oracle {io['res_est'].tolist()}")
    assert err <= 100 * rtol
    assert (np.abs(ic.col_iters - iu.col_iters) <= 2).all()
    assert ic.status == 0 and (ic.col_status == 0).all()
    res = np.linalg.norm(B - o.matmul(Xc), axis=0) / np.linalg.norm(B, axis=0)
    assert (res <= rtol).all()
    # restarted GMRES: two summation orders can put a cycle-start residual on different
    # sides of rtol; where the residual stagnates across restarts near rtol (as it does at
    # GMRES(12) here), that moves convergence by up to two cycles (measured: 144 against
    # 163 steps on one column, both below rtol in the true residual)
    assert (np.abs(ic.col_iters - io["col_iters"]) <= 2 * 12 + 2).all()
    res_o = np.linalg.norm(B - o.matmul(Xo), axis=0) / np.linalg.norm(B, axis=0)
    assert (res_o <= rtol).all()


def test_policy_end_to_end(setup):
    h2x = _h2x()
    o, A, B = setup
    budget = h2x.solve_workspace_bytes(A.plan, 4, solver="gmres", restart=12)
    X, info, mc = h2x.solve_chunked(A, _dev(B), budget, solver="gmres", restart=12, candidates=(2, 4, 8), rtol=1e-9)
    print("chosen chunk", mc)
    assert mc in (2, 4)  # 8 columns do not fit the budget
    assert info.status == 0
    res = np.linalg.norm(B - o.matmul(X.cpu().numpy()), axis=0) / np.linalg.norm(B, axis=0)
    assert (res <= 1e-9).all()
    # a workspace smaller than the chunk needs is refused
    lib = h2x.load_library()
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    Bd = _dev(B)
    X = torch.zeros_like(Bd)
    prm = h2x._GmresParams(1e-9, 12, 100, 4, 0)
    import ctypes as C
    st = lib.h2x_block_gmres_chunked(A._h, C.byref(prm), 10, 4, C.c_void_p(Bd.data_ptr()), 10,
                                     C.c_void_p(X.data_ptr()), 10, C.c_void_p(ws.data_ptr()), ws.numel(), None, None)
    assert st == 2 and b"too small" in lib.h2x_last_error()
