"""Pins of the oracle's cluster tree, block tree and lists.

Every check here is fixed by the paper's definitions (section 2: cluster tree,
block tree, admissibility; section 3: prepare_addeval lists) or by brute force,
not by re-running the oracle's own code.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2509_17257_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _line8():
    g = json.load(open(os.path.join(GOLD, "tree_line8.json")))
    P = np.zeros((8, 3))
    P[:, 0] = g["points_x"]
    return g, P


@pytest.mark.parametrize("eta", [1.0, 0.5])
def test_hand_worked_line8(eta):
    g, P = _line8()
    h = oracle.OracleH2(P, kernel="exp", ell=1.0, shift=1.0, eta=eta, leaf=g["leaf_size"], p=2)
    tr = h.tree()
    assert h.C == len(g["clusters_preorder"])
    for c in g["clusters_preorder"]:
        i = c["id"]
        mem = sorted(tr["perm"][tr["first"][i]: tr["first"][i] + tr["size"][i]].tolist())
        assert mem == c["members"]
        sons = [] if tr["son0"][i] < 0 else [int(tr["son0"][i]), int(tr["son1"][i])]
        assert sons == c["sons"]
    bl = h.blocks()
    got = [[int(t), int(s), "adm" if a else "near"] for t, s, a in zip(bl["t"], bl["s"], bl["adm"])]
    assert got == g[f"blocks_eta_{eta}"]
    if eta == 1.0:
        lists = {}
        for c in range(h.C):
            ids = bl["list_blk"][bl["list_ptr"][c]: bl["list_ptr"][c + 1]]
            lists[str(c)] = [[int(bl["t"][b]), int(bl["s"][b])] for b in ids]
        assert lists == g["lists_eta_1.0"]


def _tree_checks(h, P):
    tr = h.tree()
    n = P.shape[0]
    assert sorted(tr["perm"].tolist()) == list(range(n))
    assert tr["first"][0] == 0 and tr["size"][0] == n and tr["parent"][0] == -1
    for c in range(h.C):
        f, sz = tr["first"][c], tr["size"][c]
        pts = P[tr["perm"][f:f + sz]]
        # tight box of the cluster's points
        np.testing.assert_array_equal(tr["blo"][c], pts.min(0))
        np.testing.assert_array_equal(tr["bhi"][c], pts.max(0))
        s0, s1 = tr["son0"][c], tr["son1"][c]
        if s0 < 0:
            assert sz <= h.leaf or np.all(pts == pts[0])
            continue
        # pre-order: first son follows its parent
        assert s0 == c + 1
        # sons partition the parent, disjointly and contiguously
        assert tr["first"][s0] == f and tr["first"][s1] == f + tr["size"][s0]
        assert tr["size"][s0] + tr["size"][s1] == sz
        assert tr["parent"][s0] == c and tr["parent"][s1] == c
        # split along the widest box dimension at the box midpoint
        ext = tr["bhi"][c] - tr["blo"][c]
        d = int(np.argmax(ext))
        mid = 0.5 * (tr["blo"][c][d] + tr["bhi"][c][d])
        a = P[tr["perm"][f:f + tr["size"][s0]], d]
        b = P[tr["perm"][f + tr["size"][s0]:f + sz], d]
        assert np.all(a < mid) and np.all(b >= mid)
    return tr


@pytest.mark.parametrize("geom,n,leaf", [("sphere", 300, 8), ("cube", 400, 16), ("sphere", 4096, 32)])
def test_cluster_tree_definition(geom, n, leaf):
    P = W.sphere_points(n, 11) if geom == "sphere" else W.cube_points(n, 12)
    h = oracle.OracleH2(P, leaf=leaf, p=2)
    _tree_checks(h, P)


def _adm_np(P, perm, first, size, t, s, eta):
    A = P[perm[first[t]:first[t] + size[t]]]
    B = P[perm[first[s]:first[s] + size[s]]]
    lo_a, hi_a, lo_b, hi_b = A.min(0), A.max(0), B.min(0), B.max(0)
    gap = np.maximum(0.0, np.maximum(lo_b - hi_a, lo_a - hi_b))
    dist = np.sqrt((gap ** 2).sum())
    diam = max(np.sqrt(((hi_a - lo_a) ** 2).sum()), np.sqrt(((hi_b - lo_b) ** 2).sum()))
    return dist > 0 and diam <= eta * dist


@pytest.mark.parametrize("eta", [1.0, 2.0, 0.5])
def test_block_leaves_partition_and_admissibility(eta):
    n = 400
    P = W.sphere_points(n, 21)
    h = oracle.OracleH2(P, leaf=8, eta=eta, p=2)
    tr, bl = h.tree(), h.blocks()
    cover = np.zeros((n, n), np.int32)
    seen = set()
    for t, s, a in zip(bl["t"], bl["s"], bl["adm"]):
        rt = tr["perm"][tr["first"][t]:tr["first"][t] + tr["size"][t]]
        rs = tr["perm"][tr["first"][s]:tr["first"][s] + tr["size"][s]]
        cover[np.ix_(rt, rs)] += 1
        assert _adm_np(P, tr["perm"], tr["first"], tr["size"], t, s, eta) == bool(a)
        if not a:
            assert tr["son0"][t] < 0 and tr["son0"][s] < 0
        seen.add((int(t), int(s), bool(a)))
    assert np.all(cover == 1), "leaf blocks must partition I x J"
    for t, s, a in seen:  # symmetric structure
        assert (s, t, a) in seen
    # lists: every block once, grouped by row cluster, in block pre-order
    lp, lb = bl["list_ptr"], bl["list_blk"]
    assert sorted(lb.tolist()) == list(range(h.nb))
    for c in range(h.C):
        ids = lb[lp[c]:lp[c + 1]]
        assert np.all(bl["t"][ids] == c) and np.all(np.diff(ids) > 0)


def test_single_leaf_and_no_admissible():
    P = W.sphere_points(200, 5)
    h = oracle.OracleH2(P, leaf=200, p=2)
    assert h.C == 1 and h.nb == 1 and h.n_near == 1 and h.n_adm == 0
    h2 = oracle.OracleH2(P, leaf=8, eta=1e-12, p=2)
    assert h2.n_adm == 0 and h2.near_entries == 200 * 200


def test_coincident_points_stay_leaf():
    P = np.tile(np.array([[0.3, -0.2, 0.1]]), (50, 1))
    h = oracle.OracleH2(P, leaf=4, p=2)
    assert h.C == 1 and h.leaves == 1
