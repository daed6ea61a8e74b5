"""KIFMM evaluation following the complete algorithm of Sec. 4.3 (test infrastructure only).

Step 1 (setup): octree and lists (``tree.py``), surfaces and operators
(``operators.py``).
Step 2 (upward pass): S2M at every leaf, then M2M child -> parent up to level 2.
Step 3 (downward pass): M2L into every cube from its interaction field, L2L
parent -> child, L2T at the leaves.
Step 4 (near field): S2T from the near field of every leaf by eq. (1).

Reading taken where the algorithm listing is incomplete: M2L is applied to the
leaf cubes as well as to the non-leaf ones (otherwise the interaction fields of
the leaves would never be evaluated and far pairs at the finest level would be
lost); M2L starts at level 2 because the interaction fields of levels 0 and 1
are empty.

The potential is evaluated at the points themselves (targets = sources), the
self pair contributing 0. ``sample`` restricts Steps 3-4 to the leaves holding
the listed points (the upward pass is always complete), which gives the same
values for those points at a fraction of the cost.
"""
from __future__ import annotations

import numpy as np

from .direct import kernel_matrix
from .operators import build_operators
from .tree import build_tree


def _sign(o01):
    return tuple(2.0 * v - 1.0 for v in o01)


def fmm(x: np.ndarray, sigma: np.ndarray, p: int, eps: float, leaf_size: int,
        mode: str = "dense", cd: float = 0.5, rcond: float = 1e-10,
        depth: int | None = None, max_depth: int = 16, sample: np.ndarray | None = None,
        ops=None, tree=None, c2: float = 0.0, source_field=None, near_field=None):
    """Potential phi (N,) or (N,m) at every point (or at `sample` indices).

    The sources are point charges at the points unless `source_field` and
    `near_field` say otherwise (the boundary elements of Sec. 4):
    source_field(P, idx) is the matrix of the potentials at the points P of
    the unit densities of sources idx (S2M's check potential, Sec. 4.2), and
    near_field(tidx, sidx) that at points tidx of sources sidx (S2T).

    Returns (phi, info) where info holds the tree and the operators.
    """
    x = np.asarray(x, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    vec = s.ndim == 1
    if vec:
        s = s[:, None]
    nrhs = s.shape[1]
    if tree is None:
        tree = build_tree(x, leaf_size, depth=depth, max_depth=max_depth)
    if ops is None:
        ops = build_operators(p, eps, leaf_size, mode=mode, cd=cd, rcond=rcond, c2=c2)
    L = tree.depth

    # ---- Step 2: upward pass -------------------------------------------------
    up = [dict() for _ in range(L + 1)]
    if L >= 2:
        rL = tree.half_width(L)
        for b, idx in tree.leaf_points.items():
            c = tree.box_centre(L, b)
            P = c + rL * ops.UC
            G = kernel_matrix(P, x[idx]) if source_field is None else source_field(P, idx)
            check = G @ s[idx]                                          # S2M, Sec. 2.2
            up[L][b] = rL * (ops.S @ check)
        for level in range(L - 1, 1, -1):                               # M2M, Sec. 2.2
            for b in tree.boxes[level]:
                acc = np.zeros((ops.k, nrhs))
                for o in [(0, 0, 0), (0, 0, 1), (0, 1, 0), (0, 1, 1),
                          (1, 0, 0), (1, 0, 1), (1, 1, 0), (1, 1, 1)]:
                    ch = (2 * b[0] + o[0], 2 * b[1] + o[1], 2 * b[2] + o[2])
                    if ch in up[level + 1]:
                        acc += ops.M[_sign(o)] @ up[level + 1][ch]
                up[level][b] = acc

    # ---- which leaves to evaluate -------------------------------------------
    if sample is None:
        leaves = list(tree.leaf_points.keys())
    else:
        leaves = sorted({tree.leaf_of_point[int(i)] for i in np.asarray(sample)})
    need = [set() for _ in range(L + 1)]
    need[L] = set(leaves)
    for level in range(L - 1, -1, -1):
        need[level] = {(b[0] >> 1, b[1] >> 1, b[2] >> 1) for b in need[level + 1]}

    # ---- Step 3: downward pass ----------------------------------------------
    down = [dict() for _ in range(L + 1)]
    for level in range(2, L + 1):
        r = tree.half_width(level)
        for b in need[level]:
            acc = np.zeros((ops.k, nrhs))
            if level > 2:                                               # L2L, Sec. 2.2
                parent = (b[0] >> 1, b[1] >> 1, b[2] >> 1)
                o = (b[0] & 1, b[1] & 1, b[2] & 1)
                acc += ops.L[_sign(o)] @ down[level - 1][parent]
            for c in tree.interaction(level, b):                       # M2L, Sec. 2.2
                t = (b[0] - c[0], b[1] - c[1], b[2] - c[2])
                if ops.K2 is not None:                                  # stage 2, Sec. 3.2
                    Uh, Vh = ops.K2[t]
                    acc += (Uh @ (Vh @ up[level][c])) / r
                else:
                    acc += (ops.K[t] @ up[level][c]) / r
            down[level][b] = acc

    # ---- L2T (Sec. 2.2) and Step 4 S2T ----------------------------------------
    phi = np.zeros((x.shape[0], nrhs))
    rL = tree.half_width(L)
    for b in leaves:
        idx = tree.leaf_points[b]
        if L >= 2:
            c = tree.box_centre(L, b)
            e = rL * (ops.T @ down[L][b])
            phi[idx] += kernel_matrix(x[idx], c + rL * ops.DE) @ e
        for nb in tree.near(L, b):
            j = tree.leaf_points[nb]
            G = kernel_matrix(x[idx], x[j]) if near_field is None else near_field(idx, j)
            phi[idx] += G @ s[j]
    if sample is not None:
        phi = phi[np.asarray(sample)]
    if vec:
        phi = phi[:, 0]
    return phi, {"tree": tree, "ops": ops}
