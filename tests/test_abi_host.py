"""Host-side checks of the C-ABI library (no GPU needed).

* libh2x.so loads and exports every function declared in include/h2x.h.
* The native planner reproduces the oracle's cluster tree, block tree and lists
  exactly (same rules, written independently): permutation, cluster ranges,
  and the set of admissible / near-field leaves with the within-row order of
  the prepare_addeval lists.
* Argument validation returns H2X_EINVAL without touching a GPU.
* The split of the coupling rows (plan stats): recomputed from the cluster tree and
  the block lists, the deep part is the rows at depth >= D whose inner column clusters
  all lie at depth >= D, it holds >= 60 % of the admissible blocks, and D is the
  deepest such depth above the shallowest admissible depth + 1.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2509_17257_amd as h2x
from paper_2509_17257_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "h2x.h")).read()
    return sorted(set(re.findall(r"\b(h2x_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = h2x.load_library()
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
    assert lib.h2x_version().decode().startswith("h2x")


@pytest.mark.parametrize("wl,n", [("sphere", 3000), ("cube", 5000), ("line", 700)])
@pytest.mark.parametrize("leaf,eta,p", [(32, 1.0, 3), (64, 1.0, 4), (16, 2.0, 2), (8, 0.5, 3)])
def test_planner_matches_oracle_structure(wl, n, leaf, eta, p):
    P = {"sphere": W.sphere_points, "cube": W.cube_points, "line": W.line_points}[wl](n, 71)
    o = oracle.OracleH2(P, leaf=leaf, eta=eta, p=p)
    pl = h2x.Plan(P, leaf=leaf, eta=eta, p=p)
    assert (pl.n, pl.C, pl.leaves, pl.n_adm, pl.n_near, pl.near_entries, pl.depth) == \
        (o.n, o.C, o.leaves, o.n_adm, o.n_near, o.near_entries, o.depth)
    ot = o.tree()
    np.testing.assert_array_equal(pl.perm(), ot["perm"])
    cl = pl.clusters()
    for nm in ("first", "size", "parent", "son0", "son1", "depth"):
        np.testing.assert_array_equal(cl[nm], ot[nm], err_msg=nm)
    ob = o.blocks()
    # oracle lists grouped by row cluster, in block pre-order within a row
    lists_adm = [(int(ob["t"][b]), int(ob["s"][b])) for b in ob["list_blk"] if ob["adm"][b]]
    lists_near = [(int(ob["t"][b]), int(ob["s"][b])) for b in ob["list_blk"] if not ob["adm"][b]]
    pb = pl.blocks()
    assert list(zip(pb["adm_t"].tolist(), pb["adm_s"].tolist())) == lists_adm
    assert list(zip(pb["near_t"].tolist(), pb["near_s"].tolist())) == lists_near


def test_stats_bytes():
    P = W.sphere_points(2000, 72)
    pl = h2x.Plan(P, leaf=32, p=3)
    k = 27
    ent = pl.n * k + (pl.C - 1) * k * k + pl.n_adm * k * k
    assert pl.bytes_operator == [8 * ent, 4 * ent, 2 * ent]
    assert pl.bytes_near == 8 * pl.near_entries


def test_invalid_arguments_rejected():
    P = W.sphere_points(100, 73)
    for kw in (dict(p=0), dict(p=9), dict(leaf=0), dict(eta=0.0), dict(ell=-1.0)):
        with pytest.raises(h2x.H2xError):
            h2x.Plan(P, **kw)
    bad = P.copy()
    bad[3, 1] = np.nan
    with pytest.raises(h2x.H2xError):
        h2x.Plan(bad)
    lib = h2x.load_library()
    h = C.c_void_p()
    assert lib.h2x_plan_create(None, 10, None, C.byref(h)) == 1
    assert b"NULL" in lib.h2x_last_error()
    # workspace queries on NULL handles return 0 instead of crashing
    assert lib.h2x_mat_workspace_bytes(None, 0) == 0
    assert lib.h2x_matmul_workspace_bytes(None, 4) == 0
    # tuning and timer entry points refuse NULL handles and bad sizes before any GPU call
    info = h2x._TuneInfo()
    assert lib.h2x_mat_set_tune(None, 8, C.byref(info)) == 1
    assert lib.h2x_mat_get_tune(None, 8, C.byref(info)) == 1
    t = C.c_void_p()
    assert lib.h2x_timer_create(0, C.byref(t)) == 1 and not t.value
    assert lib.h2x_timer_create(4, None) == 1
    out = np.zeros(5)
    assert lib.h2x_timer_read(None, 0, out.ctypes.data_as(C.c_void_p)) == 1
    lib.h2x_timer_destroy(None)


def test_merged_plan_is_the_concatenation_of_its_systems():
    specs = [(W.sphere_points(900, 401), dict(leaf=32, p=3, ell=0.5)),
             (W.cube_points(1500, 402), dict(leaf=16, p=3, ell=0.3, eta=1.5, shift=0.5)),
             (W.line_points(300, 403), dict(leaf=8, p=3, ell=0.2)),
             (W.sphere_points(2000, 404), dict(leaf=64, p=3, ell=0.9))]
    parts = [h2x.Plan(P, **kw) for P, kw in specs]
    mp = h2x.Plan.merge(parts)
    assert mp.n == sum(p.n for p in parts) and mp.C == sum(p.C for p in parts)
    assert (mp.n_adm, mp.n_near, mp.near_entries) == (sum(p.n_adm for p in parts), sum(p.n_near for p in parts),
                                                       sum(p.near_entries for p in parts))
    assert mp.depth == max(p.depth for p in parts)
    np.testing.assert_array_equal(mp.systems(), np.r_[0, np.cumsum([p.n for p in parts])])
    n0 = c0 = 0
    cl, pb, perm = mp.clusters(), mp.blocks(), mp.perm()
    a0 = q0 = 0
    for p in parts:
        c = p.clusters()
        sl = slice(c0, c0 + p.C)
        np.testing.assert_array_equal(cl["first"][sl], c["first"] + n0)
        np.testing.assert_array_equal(cl["size"][sl], c["size"])
        np.testing.assert_array_equal(cl["depth"][sl], c["depth"])
        for nm in ("parent", "son0", "son1"):
            np.testing.assert_array_equal(cl[nm][sl], np.where(c[nm] < 0, -1, c[nm] + c0), err_msg=nm)
        np.testing.assert_array_equal(perm[n0:n0 + p.n], p.perm() + n0)
        b = p.blocks()
        np.testing.assert_array_equal(pb["adm_t"][a0:a0 + p.n_adm], b["adm_t"] + c0)
        np.testing.assert_array_equal(pb["adm_s"][a0:a0 + p.n_adm], b["adm_s"] + c0)
        np.testing.assert_array_equal(pb["near_t"][q0:q0 + p.n_near], b["near_t"] + c0)
        np.testing.assert_array_equal(pb["near_s"][q0:q0 + p.n_near], b["near_s"] + c0)
        n0 += p.n
        c0 += p.C
        a0 += p.n_adm
        q0 += p.n_near
    with pytest.raises(h2x.H2xError):
        h2x.Plan.merge([parts[0], h2x.Plan(W.sphere_points(500, 405), leaf=32, p=4)])


def _deep_blocks(c, b, D):
    depth, son0 = c["depth"], c["son0"]
    at, as_ = b["adm_t"], b["adm_s"]
    inner = son0[as_] >= 0
    # shallowest inner column cluster per row
    ready = np.full(len(depth), 1 << 30, dtype=np.int64)
    np.minimum.at(ready, at[inner], depth[as_[inner]])
    deep = (depth >= D) & (ready >= D)
    return int(deep[at].sum())


@pytest.mark.parametrize("wl,n,leaf,p", [("sphere", 20000, 32, 3), ("cube", 7000, 64, 4), ("sphere", 4096, 32, 3),
                                         ("sphere", 4000, 64, 4), ("line", 3000, 16, 2)])
def test_coupling_split_rule(wl, n, leaf, p):
    pts = {"sphere": W.sphere_points, "cube": W.cube_points, "line": W.line_points}[wl](n, 41)
    P = h2x.Plan(pts, ell=0.5, shift=1.0, eta=1.0, leaf=leaf, p=p)
    c, b = P.clusters(), P.blocks()
    D = P.split_depth
    cands = [d for d in range(P.depth, P.adm_depth + 1, -1) if 10 * _deep_blocks(c, b, d) >= 6 * P.n_adm]
    print(f"{wl} n={n}: depth {P.depth}, adm {P.adm_depth}, split {D}, deep {P.deep_blocks} of {P.n_adm}")
    if D == 0:
        assert not cands and P.deep_blocks == 0
    else:
        assert D == cands[0] and P.deep_blocks == _deep_blocks(c, b, D)
        assert 10 * P.deep_blocks >= 6 * P.n_adm
