"""Pins of the adaptive-tree oracle (oracle/adaptive.py; CPU only).

The adaptive KIFMM is pinned to things other than itself:
* tree invariants: every point in exactly one leaf, leaves hold at most s
  points (below the depth cap), no leaf shares a vertex with a leaf two or
  more levels finer (2:1 balance);
* the lists cover every ordered pair of leaves exactly once: directly (U), at
  one pair of same-level ancestors (V), from a cube above the source into the
  target leaf (W), or from the source leaf into a cube above the target (X);
* the FMM against the O(N^2) direct sum on a clustered set (leaves over seven
  levels) and the 2:1:0.5 ellipsoid, with the error falling with p;
* when every leaf sits at one level the adaptive tree is the uniform tree and
  the result equals the uniform-tree oracle's (W and X empty);
* planted mistakes (no W/X lists, near field restricted to one level, M2T
  without the U~ expansion) fail the direct-sum pin.
"""
import functools

import numpy as np
import pytest

import oracle
import workloads
from oracle.adaptive import build_adaptive_tree, fmm_adaptive, is_ancestor_or_self, touches


@functools.lru_cache(maxsize=None)
def clustered(n_bg=1500, n_cl=2500, seed=3):
    """Sparse uniform background plus a dense Gaussian cluster: leaves from
    level 2 to level 8."""
    x = workloads.clustered_points(n_bg, n_cl, seed)
    return x, workloads.uniform_density(x.shape[0], seed + 100)


@functools.lru_cache(maxsize=None)
def clustered_tree(leaf=24):
    return build_adaptive_tree(clustered()[0], leaf)


def test_tree_invariants():
    x, _ = clustered()
    t = clustered_tree()
    count = np.zeros(x.shape[0], dtype=int)
    for lf, idx in t.leaf_points.items():
        count[idx] += 1
        assert idx.size <= 24 or lf[0] == 16
    assert np.all(count == 1)
    levels = {lf[0] for lf in t.leaf_points}
    assert min(levels) <= 3 and max(levels) >= 7, levels
    leaves = t.leaves()
    for a in leaves:
        for b in leaves:
            if b[0] >= a[0] + 2:
                assert not touches(a, b), (a, b)


def test_lists_cover_every_leaf_pair_once():
    x, _ = clustered(400, 600, 4)
    t = build_adaptive_tree(x, 12)
    leaves = t.leaves()
    boxes = [(lv, b) for lv in t.by_level for b in t.by_level[lv]]
    V = {bx: t.V(bx) for bx in boxes}
    W = {lf: t.W(lf) for lf in leaves}
    X = {}
    for lf, ws in W.items():
        for c in ws:
            X.setdefault(c, []).append(lf)
    anc = {lf: [bx for bx in boxes if is_ancestor_or_self(bx, lf)] for lf in leaves}
    assert sum(len(v) for v in W.values()) > 0
    for T in leaves:
        U = set(t.U(T))
        for S in leaves:
            n = int(S in U)
            n += sum(1 for Ta in anc[T] for Sa in V[Ta] if is_ancestor_or_self(Sa, S))
            n += sum(1 for c in W[T] if is_ancestor_or_self(c, S))
            n += sum(1 for Ta in anc[T] for c in X.get(Ta, []) if c == S)
            assert n == 1, (T, S, n)


@functools.lru_cache(maxsize=None)
def _ops(p, eps, leaf, mode):
    return oracle.build_operators(p, eps, leaf, mode=mode)


@pytest.mark.parametrize("mode", ["dense", "svd"])
def test_fmm_vs_direct_clustered(mode):
    x, s = clustered()
    t = clustered_tree()
    d = oracle.direct(x, s)
    errs = []
    for p in (4, 6):
        phi = fmm_adaptive(x, s, _ops(p, 1e-8, 24, mode), t)
        errs.append(float(np.linalg.norm(phi - d) / np.linalg.norm(d)))
    print(f"clustered {mode}: p=4 {errs[0]:.3e}, p=6 {errs[1]:.3e}")
    assert errs[0] < 5e-4 and errs[1] < 1e-5 and errs[1] < errs[0] / 10


def test_stage2_adaptive_vs_direct_and_dense():
    # stage-2 factors (Sec. 3.2, C2 = 10) on the adaptive tree: within the
    # uniform tree's stage-2 bar of the dense result, and of the direct sum
    x, s = clustered()
    t = clustered_tree()
    d = oracle.direct(x, s)
    dense = fmm_adaptive(x, s, _ops(6, 1e-8, 24, "dense"), t)
    ops2 = oracle.build_operators(6, 1e-6, 24, mode="svd2", c2=10.0)
    phi = fmm_adaptive(x, s, ops2, t)
    e_dense = float(np.linalg.norm(phi - dense) / np.linalg.norm(dense))
    e_direct = float(np.linalg.norm(phi - d) / np.linalg.norm(d))
    print(f"stage 2 adaptive: vs dense {e_dense:.3e}, vs direct {e_direct:.3e}")
    assert e_dense < 5e-6 and e_direct < 1e-5


def test_fmm_vs_direct_ellipsoid():
    x = workloads.ellipsoid_points(6000, 5)
    s = workloads.uniform_density(6000, 6)
    t = build_adaptive_tree(x, 32)
    assert len({lf[0] for lf in t.leaf_points}) >= 2
    d = oracle.direct(x, s)
    phi = fmm_adaptive(x, s, _ops(6, 1e-6, 32, "svd"), t)
    e = float(np.linalg.norm(phi - d) / np.linalg.norm(d))
    print(f"ellipsoid 6000 p=6: {e:.3e}")
    assert e < 1e-5


def jittered_grid(m=16, seed=8):
    """m^3 points, one near the centre of each cell of an m^3 grid over
    [0, 1]^3, plus the corners (0,0,0) and (1,1,1) that fix the bounding box."""
    rng = np.random.default_rng(seed)
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5
         + 0.3 * rng.uniform(-1, 1, (m ** 3, 3))) / m
    return np.concatenate([g, [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]])


def test_adaptive_equals_uniform_when_leaves_share_a_level():
    x = jittered_grid()
    s = workloads.uniform_density(x.shape[0], 9)
    t = build_adaptive_tree(x, 9)
    assert {lf[0] for lf in t.leaf_points} == {3}
    assert all(not t.W(lf) for lf in t.leaf_points)
    ops = _ops(4, 1e-6, 9, "svd")
    pa = fmm_adaptive(x, s, ops, t)
    pu, info = oracle.fmm(x, s, 4, 1e-6, 9, ops=ops)
    assert info["tree"].depth == 3
    assert np.allclose(pa, pu, rtol=1e-12, atol=1e-12 * np.abs(pu).max())


# ------------------------------------------------------- planted mistakes
def _err_with(monkeypatch, patch):
    x, s = clustered()
    t = build_adaptive_tree(x, 24)
    patch(monkeypatch, t)
    d = oracle.direct(x, s)
    phi = fmm_adaptive(x, s, _ops(6, 1e-8, 24, "svd"), t)
    return float(np.linalg.norm(phi - d) / np.linalg.norm(d))


def _no_w(mp, t):
    mp.setattr(t, "W", lambda leaf: [])


def _same_level_near(mp, t):
    orig = t.U
    mp.setattr(t, "U", lambda leaf: [c for c in orig(leaf) if c[0] == leaf[0]])


@pytest.mark.parametrize("patch", [_no_w, _same_level_near])
def test_planted_list_mistakes_fail(monkeypatch, patch):
    assert _err_with(monkeypatch, patch) > 1e-4


def test_planted_missing_expansion_fails():
    x, s = clustered()
    t = clustered_tree()
    ops = _ops(6, 1e-8, 24, "svd")
    import copy
    wrong = copy.copy(ops)
    wrong.U = np.eye(ops.n_eq)[:, :ops.k]   # M2T and S2L without the U~ basis
    d = oracle.direct(x, s)
    phi = fmm_adaptive(x, s, wrong, t)
    assert float(np.linalg.norm(phi - d) / np.linalg.norm(d)) > 1e-4
