"""Right-hand-side chunk policy (section 5, memory-footprint remarks of block CG and
block GMRES), host side: workspace sizes from the plan alone and the choice of
m_chunk under a memory budget, with and without a throughput curve.  No GPU."""
import math

import numpy as np
import pytest

import paper_2509_17257_amd as h2x
from paper_2509_17257_amd import workloads as W


@pytest.fixture(scope="module")
def plan():
    return h2x.Plan(W.sphere_points(3000, 91), ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3)


def test_workspace_grows_linearly(plan):
    n = plan.n
    for solver, restart in (("cg", 30), ("gmres", 10), ("gmres", 30)):
        ws = [h2x.solve_workspace_bytes(plan, m, solver=solver, restart=restart) for m in (1, 2, 8, 32, 33, 64)]
        assert all(b > 0 for b in ws) and ws == sorted(ws)
        # per column at least the solver's n x m blocks: CG keeps B, X, R, P, AP (5 n);
        # GMRES B, X and restart + 1 basis blocks
        per_col = (ws[5] - ws[4]) / 31
        floor = 5 * 8 * n if solver == "cg" else (restart + 3) * 8 * n
        assert per_col >= floor
    assert h2x.solve_workspace_bytes(plan, 16, solver="gmres", restart=30) > h2x.solve_workspace_bytes(
        plan, 16, solver="cg")
    lib = h2x.load_library()
    assert lib.h2x_solve_workspace_bytes(plan._h, 0, 0, 0, 0) == 0  # m = 0
    assert lib.h2x_solve_workspace_bytes(plan._h, 0, 1, 4, 0) == 0  # GMRES needs restart >= 1


def test_memory_rule(plan):
    ws = lambda m: h2x.solve_workspace_bytes(plan, m, solver="cg")
    assert h2x.choose_chunk(plan, 100, ws(32)) == 32
    assert h2x.choose_chunk(plan, 100, ws(32) - 1) == 31
    assert h2x.choose_chunk(plan, 20, ws(64)) == 20  # never more than m
    assert h2x.choose_chunk(plan, 100, 1 << 62) == 100
    with pytest.raises(h2x.H2xError):
        h2x.choose_chunk(plan, 100, ws(1) - 1)  # a single column does not fit


def test_throughput_rule(plan):
    big = 1 << 62
    curve = {16: 1.0, 32: 1.1, 64: 2.2, 100: 3.5}
    # predicted times ceil(100 / c) * t(c): 7.0, 4.4, 4.4, 3.5
    assert h2x.choose_chunk(plan, 100, big, curve=curve) == 100
    curve[100] = 4.5  # 7.0, 4.4, 4.4, 4.5: a tie goes to the larger chunk
    assert h2x.choose_chunk(plan, 100, big, curve=curve) == 64
    # a budget that admits chunks up to 40 columns: 16 or 32
    wsg = lambda m: h2x.solve_workspace_bytes(plan, m, solver="gmres", restart=10)
    assert h2x.choose_chunk(plan, 100, wsg(40), solver="gmres", restart=10, curve=curve) == 32
    # no measured candidate fits: the memory rule
    assert h2x.choose_chunk(plan, 100, wsg(12), solver="gmres", restart=10, curve=curve) == 12
    # candidates above m count as m
    assert h2x.choose_chunk(plan, 10, big, curve={16: 1.0, 4: 0.5}) == 10
    # brute force over random curves and budgets
    rng = np.random.default_rng(92)
    for _ in range(20):
        cands = sorted(rng.choice(np.arange(1, 129), 5, replace=False).tolist())
        ms = rng.uniform(0.5, 5.0, 5).tolist()
        m = int(rng.integers(1, 300))
        budget = h2x.solve_workspace_bytes(plan, int(rng.integers(1, 200)), solver="cg")
        got = h2x.choose_chunk(plan, m, budget, curve=dict(zip(cands, ms)))
        fit = [(min(c, m), t) for c, t in zip(cands, ms)
               if h2x.solve_workspace_bytes(plan, min(c, m), solver="cg") <= budget]
        if fit:
            best = min(fit, key=lambda ct: (math.ceil(m / ct[0]) * ct[1], -ct[0]))
            assert got == best[0]
        else:
            assert got == h2x.choose_chunk(plan, m, budget)


def test_bad_arguments(plan):
    lib = h2x.load_library()
    out = np.zeros(1, np.int64)
    assert lib.h2x_choose_chunk(None, 0, 0, 0, 10, 1 << 40, 0, None, None, out.ctypes.data) == 1
    assert lib.h2x_choose_chunk(plan._h, 0, 5, 0, 10, 1 << 40, 0, None, None, out.ctypes.data) == 1  # solver
    assert lib.h2x_choose_chunk(plan._h, 0, 1, 0, 10, 1 << 40, 0, None, None, out.ctypes.data) == 1  # restart
    assert lib.h2x_choose_chunk(plan._h, 0, 0, 0, 0, 1 << 40, 0, None, None, out.ctypes.data) == 1  # m
