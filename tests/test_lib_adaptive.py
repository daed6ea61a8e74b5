"""The library's adaptive tree and lists against the oracle's (CPU only).

Host-only plans (opts.device = -1, opts.adaptive = 1) build the adaptive
octree and its U, V, W, X lists in C++; oracle/adaptive.py builds them from
their definitions by direct search. Both must give the same cubes, the same
leaf for every point and the same lists, pair for pair, on point sets whose
leaves span many levels (a Gaussian cluster in a sparse background, the
2:1:0.5 ellipsoid surface, a sparse corner whose octant stays a level-1 leaf)
and on the degenerate cases (one point, coincident points, one leaf).
"""
import functools

import numpy as np
import pytest

import workloads
import paper_1211_2517_amd as K
from oracle.adaptive import build_adaptive_tree


def _sets():
    return {
        "clustered": (workloads.clustered_points(1500, 2500, 3), 24),
        "clustered_small_leaf": (workloads.clustered_points(400, 600, 4), 12),
        "ellipsoid": (workloads.ellipsoid_points(6000, 5), 32),
        "corner": (workloads.corner_clusters(3000, 20, 7), 32),
    }


@functools.lru_cache(maxsize=None)
def _pair(name):
    x, s = _sets()[name]
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=s, device=-1, adaptive=True)
    return x, plan, build_adaptive_tree(x, s)


def _box_keys(plan):
    b = plan.export_boxes()
    return [(int(r[0]), (int(r[1]), int(r[2]), int(r[3]))) for r in b], b[:, 4]


@pytest.mark.parametrize("name", list(_sets()))
def test_tree_matches_oracle(name):
    x, plan, t = _pair(name)
    keys, leaf_idx = _box_keys(plan)
    assert len(set(keys)) == len(keys)
    assert set(keys) == {(lv, b) for lv in t.by_level for b in t.by_level[lv]}
    assert {keys[i] for i in np.flatnonzero(leaf_idx >= 0)} == set(t.leaf_points)
    # leaves of a level come first among its cubes; leaf indices are a permutation
    levels = np.array([k[0] for k in keys])
    assert np.all(np.diff(levels) >= 0)
    for lv in np.unique(levels):
        lf = leaf_idx[levels == lv] >= 0
        assert not np.any(lf[1:] & ~lf[:-1])
    assert sorted(leaf_idx[leaf_idx >= 0].tolist()) == list(range(len(t.leaf_points)))
    pl = plan.export_point_leaves()
    assert all((int(r[0]), (int(r[1]), int(r[2]), int(r[3]))) == t.leaf_of_point[i] for i, r in enumerate(pl))
    info = plan.info()
    assert info["adaptive"] == 1
    assert info["leaf_level_min"] == min(lf[0] for lf in t.leaf_points)
    assert info["depth"] == t.depth
    assert info["n_leaf"] == len(t.leaf_points)


@pytest.mark.parametrize("name", list(_sets()))
def test_lists_match_oracle(name):
    x, plan, t = _pair(name)
    keys, _ = _box_keys(plan)
    boxes = [(lv, b) for lv in t.by_level for b in t.by_level[lv]]
    want = {
        "U": {(lf, c) for lf in t.leaf_points for c in t.U(lf)},
        "V": {(bx, c) for bx in boxes for c in t.V(bx)},
        "W": {(lf, c) for lf in t.leaf_points for c in t.W(lf)},
    }
    want["X"] = {(c, lf) for (lf, c) in want["W"]}
    for which, ref in want.items():
        got = plan.export_list(which)
        pairs = [(keys[a], keys[b]) for a, b in got]
        assert len(pairs) == len(set(pairs)), which
        assert set(pairs) == ref, which
    info = plan.info()
    assert info["w_pairs"] == len(want["W"])
    assert info["v_pairs"] == len(want["V"])
    assert info["near_pairs"] == len(want["U"])
    if name == "corner":
        # the sparse octant is a level-1 leaf whose far field comes from W alone
        lvl1 = [lf for lf in t.leaf_points if lf[0] == 1]
        assert lvl1 and all(t.W(lf) for lf in lvl1)


def test_degenerate_cases():
    # one point: the root is the only cube and leaf, no far field
    p1 = K.Plan(np.array([[0.3, -0.2, 0.1]]), p=4, eps=1e-6, leaf_size=8, device=-1, adaptive=True)
    assert p1.info()["depth"] == 0 and p1.info()["n_leaf"] == 1
    assert p1.export_list("U").tolist() == [[0, 0]]
    # coincident points beyond the leaf size: one chain of cubes down to max_depth
    x = np.tile([[0.5, 0.5, 0.5]], (40, 1))
    x = np.concatenate([x, [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]])
    p2 = K.Plan(x, p=4, eps=1e-6, leaf_size=8, device=-1, adaptive=True, max_depth=6)
    t2 = build_adaptive_tree(x, 8, max_depth=6)
    keys, leaf_idx = _box_keys(p2)
    assert set(keys) == {(lv, b) for lv in t2.by_level for b in t2.by_level[lv]}
    assert p2.info()["depth"] == 6
    # leaf size >= n: one leaf
    x3 = workloads.uniform_cube(50, 1)
    p3 = K.Plan(x3, p=4, eps=1e-6, leaf_size=64, device=-1, adaptive=True)
    assert p3.info()["n_leaf"] == 1 and p3.info()["v_pairs"] == 0 and p3.info()["w_pairs"] == 0


def test_uniform_lists_exported():
    # the same exports on a uniform plan: every leaf at the leaf level, no W or X
    x = workloads.uniform_cube(3000, 2)
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=32, device=-1)
    keys, leaf_idx = _box_keys(plan)
    d = plan.info()["depth"]
    assert all((k[0] == d) == (li >= 0) for k, li in zip(keys, leaf_idx))
    assert plan.export_list("W").shape == (0, 2) and plan.export_list("X").shape == (0, 2)
    assert len(plan.export_list("U")) == plan.info()["near_pairs"]
    assert len(plan.export_list("V")) == plan.info()["v_pairs"]


def test_adaptive_rejects_forced_depth():
    x = workloads.uniform_cube(100, 3)
    with pytest.raises(K.KifmmError):
        K.Plan(x, p=4, eps=1e-6, leaf_size=8, device=-1, adaptive=True, depth=3)
