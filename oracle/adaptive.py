"""Adaptive octree and the KIFMM evaluated on it (test infrastructure only).

Sec. 2.1 splits the root cube into 8 children and continues "until the
particles contained in each leaf cube is no more than s". Read cube by cube
this gives an adaptive tree: a cube is split only while it holds more than s
points, so leaves sit at several levels (on a surface, and more so on the
2:1:0.5 ellipsoid, the points per cube vary by orders of magnitude). The near
and interaction fields of Sec. 2.1 relate cubes of one level; between leaves
of different levels the far field is covered by two more lists, those of the
kernel-independent FMM the paper builds on. For a cube B:

* U(B), B a leaf: the leaves of any level that share at least one vertex with
  B (B included) -- the near field, evaluated directly (S2T);
* V(B): children of the same-level neighbours of B's parent that do not share
  a vertex with B -- the interaction field of Sec. 2.1 (M2L);
* W(B), B a leaf: cubes C inside a same-level neighbour of B whose parent
  shares a vertex with B but which do not themselves -- C's upward equivalent
  densities are evaluated at B's points (M2T);
* X(B): the leaves C with B in W(C) -- C's points give B's downward check
  potential directly (S2L).

Readings taken here and by the GPU library (which has its own implementation):

* the root cube and integer coordinates are those of the uniform tree
  (oracle.tree): 21-bit integer coordinates, the level-l cube of a point is
  q >> (21 - l);
* a cube holding more than s points is split, down to `max_depth` (larger
  leaves are allowed there); empty children are not created;
* 2:1 balance, in rounds: every leaf of the current tree that shares a
  vertex with a leaf two or more levels finer is split, all of them at once;
  rounds repeat until no such pair is left. (The rounds fix the result: a
  leaf split in the same round as the finer leaf it touches might not have
  needed it had that leaf been split first, since empty children are not
  created.)
* the downward pass runs at levels >= 2 as in the uniform tree (V is empty
  at levels 0 and 1); a leaf above level 2 takes its far field from W only.

Boxes are (level, (i, j, k)) keys of plain dictionaries; lists are built from
their definitions by direct search, which is fine for the sizes the tests use.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .direct import kernel_matrix
from .tree import QBITS, integer_coords, root_cube

CHILD_OFFSETS = list(itertools.product((0, 1), repeat=3))
NEIGHBOUR_OFFSETS = list(itertools.product((-1, 0, 1), repeat=3))


def _parent(box):
    level, b = box
    return (level - 1, (b[0] >> 1, b[1] >> 1, b[2] >> 1))


def touches(a, b) -> bool:
    """Whether two cubes (level, triple) share at least one point (closed
    cubes); for two cubes of one tree that is 'share a vertex' or nesting."""
    la, ia = a
    lb, ib = b
    m = max(la, lb)
    sa, sb = 1 << (m - la), 1 << (m - lb)
    for d in range(3):
        alo, ahi = ia[d] * sa, (ia[d] + 1) * sa
        blo, bhi = ib[d] * sb, (ib[d] + 1) * sb
        if alo > bhi or blo > ahi:
            return False
    return True


def is_ancestor_or_self(a, b) -> bool:
    """Whether cube a contains cube b."""
    la, ia = a
    lb, ib = b
    if la > lb:
        return False
    s = lb - la
    return all((ib[d] >> s) == ia[d] for d in range(3))


@dataclass
class AdaptiveTree:
    centre: np.ndarray
    r0: float
    q: np.ndarray
    children: dict = field(default_factory=dict)       # box -> list of child boxes (empty for leaves)
    leaf_points: dict = field(default_factory=dict)    # leaf box -> np.ndarray of point indices
    by_level: dict = field(default_factory=dict)       # level -> set of triples
    leaf_of_point: list = field(default_factory=list)  # point index -> leaf box

    @property
    def depth(self) -> int:
        return max(self.by_level)

    def half_width(self, level: int) -> float:
        return self.r0 / float(2 ** level)

    def box_centre(self, box) -> np.ndarray:
        level, b = box
        r = self.half_width(level)
        return (self.centre - self.r0) + (2.0 * np.asarray(b, dtype=np.float64) + 1.0) * r

    def is_leaf(self, box) -> bool:
        return box in self.leaf_points

    def exists(self, box) -> bool:
        level, b = box
        return b in self.by_level.get(level, ())

    def leaves(self):
        return list(self.leaf_points.keys())

    # ------------------------------------------------------------------ lists
    def colleagues(self, box):
        """Same-level cubes sharing a vertex with `box` (box included)."""
        level, b = box
        out = []
        for d in NEIGHBOUR_OFFSETS:
            c = (b[0] + d[0], b[1] + d[1], b[2] + d[2])
            if c in self.by_level.get(level, ()):
                out.append((level, c))
        return out

    def U(self, leaf):
        """Leaves sharing a vertex with `leaf` (itself included)."""
        return [c for c in self.leaf_points if touches(leaf, c)]

    def V(self, box):
        level, b = box
        if level < 2:
            return []
        out = []
        for pn in self.colleagues(_parent(box)):
            for o in CHILD_OFFSETS:
                c = (2 * pn[1][0] + o[0], 2 * pn[1][1] + o[1], 2 * pn[1][2] + o[2])
                if c in self.by_level.get(level, ()) and not touches(box, (level, c)):
                    out.append((level, c))
        return out

    def W(self, leaf):
        """Cubes below the leaf's same-level neighbours that do not share a
        vertex with it while their parents do."""
        out = []
        stack = []
        for c0 in self.colleagues(leaf):
            if c0 != leaf:
                stack.extend(self.children.get(c0, []))
        while stack:
            c = stack.pop()
            if not touches(leaf, c):
                out.append(c)
            else:
                stack.extend(self.children.get(c, []))
        return out


def build_adaptive_tree(x: np.ndarray, leaf_size: int, max_depth: int = 16, balance: bool = True) -> AdaptiveTree:
    x = np.asarray(x, dtype=np.float64)
    centre, r0 = root_cube(x)
    q = integer_coords(x, centre, r0)
    t = AdaptiveTree(centre=centre, r0=r0, q=q)
    root = (0, (0, 0, 0))
    t.children[root] = []
    t.by_level = {0: {(0, 0, 0)}}
    pts = {root: np.arange(x.shape[0], dtype=np.int64)}

    def split(box):
        level, b = box
        idx = pts[box]
        cells = q[idx] >> (QBITS - level - 1)
        kids = []
        for o in CHILD_OFFSETS:
            c = (2 * b[0] + o[0], 2 * b[1] + o[1], 2 * b[2] + o[2])
            sel = idx[np.all(cells == np.asarray(c), axis=1)]
            if sel.size == 0:
                continue
            kid = (level + 1, c)
            pts[kid] = sel
            t.children[kid] = []
            t.by_level.setdefault(level + 1, set()).add(c)
            kids.append(kid)
        t.children[box] = kids
        return kids

    # split while a cube holds more than s points
    work = [root]
    while work:
        box = work.pop()
        if pts[box].size > leaf_size and box[0] < max_depth:
            work.extend(split(box))
    # 2:1 balance: split leaves that share a vertex with a leaf >= 2 levels finer
    if balance:
        changed = True
        while changed:
            changed = False
            leaves = [b for b, ch in t.children.items() if not ch]
            deep = {}
            for lf in leaves:
                deep.setdefault(lf[0], []).append(lf)
            for lf in leaves:
                if lf[0] >= max_depth:
                    continue
                finer = [c for lv, cs in deep.items() if lv >= lf[0] + 2 for c in cs]
                if any(touches(lf, c) for c in finer):
                    split(lf)
                    changed = True
    for box, ch in t.children.items():
        if not ch:
            t.leaf_points[box] = pts[box]
    t.leaf_of_point = [None] * x.shape[0]
    for lf, idx in t.leaf_points.items():
        for i in idx:
            t.leaf_of_point[int(i)] = lf
    return t


def fmm_adaptive(x: np.ndarray, sigma: np.ndarray, ops, tree: AdaptiveTree) -> np.ndarray:
    """Potential at every point by the KIFMM on the adaptive tree, FP64, with
    the operators `ops` (oracle.operators.build_operators: dense, svd or svd2
    mode; svd2 applies each M2L matrix as its stage-2 factors).

    Upward: S2M at every leaf at its own level, M2M for every split cube
    (finest level first). Downward, levels >= 2: L2L from the parent, M2L from
    V, S2L from X; at every leaf L2T (level >= 2), M2T from W and S2T from U.
    In svd mode the upward and downward coefficients are compressed: the
    equivalent densities of a cube are U~ q~ and its downward check potential
    enters as U~^T p (the projection the compressed M2L produces)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    vec = s.ndim == 1
    if vec:
        s = s[:, None]
    Ut = ops.U if ops.U is not None else np.eye(ops.n_eq)
    up = {}
    # ---- upward pass
    for lf, idx in tree.leaf_points.items():
        level = lf[0]
        r = tree.half_width(level)
        c = tree.box_centre(lf)
        up[lf] = r * (ops.S @ (kernel_matrix(c + r * ops.UC, x[idx]) @ s[idx]))   # S2M
    for level in sorted(tree.by_level, reverse=True):
        for b in tree.by_level[level]:
            box = (level, b)
            kids = tree.children.get(box, [])
            if not kids:
                continue
            acc = np.zeros((ops.k, s.shape[1]))
            for kid in kids:                                                         # M2M
                o = tuple(2.0 * (kid[1][d] - 2 * b[d]) - 1.0 for d in range(3))
                acc += ops.M[o] @ up[kid]
            up[box] = acc
    # X lists from the W lists of the leaves
    X = {}
    W = {lf: tree.W(lf) for lf in tree.leaf_points}
    for lf, ws in W.items():
        for c in ws:
            X.setdefault(c, []).append(lf)
    # ---- downward pass
    down = {}
    for level in sorted(tree.by_level):
        if level < 2:
            continue
        r = tree.half_width(level)
        for b in tree.by_level[level]:
            box = (level, b)
            acc = np.zeros((ops.k, s.shape[1]))
            par = _parent(box)
            if par[0] >= 2:                                                          # L2L
                o = tuple(2.0 * (b[d] - 2 * par[1][d]) - 1.0 for d in range(3))
                acc += ops.L[o] @ down[par]
            for c in tree.V(box):                                                    # M2L
                tvec = tuple(b[d] - c[1][d] for d in range(3))
                if ops.K2 is not None:                                               # stage 2, Sec. 3.2
                    Uh, Vh = ops.K2[tvec]
                    acc += (Uh @ (Vh @ up[c])) / r
                else:
                    acc += (ops.K[tvec] @ up[c]) / r
            if box in X:                                                             # S2L
                dc = tree.box_centre(box) + r * ops.DC
                for src in X[box]:
                    j = tree.leaf_points[src]
                    acc += Ut.T @ (kernel_matrix(dc, x[j]) @ s[j])
            down[box] = acc
    # ---- leaves: L2T, M2T, S2T
    phi = np.zeros((x.shape[0], s.shape[1]))
    for lf, idx in tree.leaf_points.items():
        level = lf[0]
        if level >= 2:                                                               # L2T
            r = tree.half_width(level)
            c = tree.box_centre(lf)
            e = r * (ops.T @ down[lf])
            phi[idx] += kernel_matrix(x[idx], c + r * ops.DE) @ e
        for src in W[lf]:                                                            # M2T
            rs = tree.half_width(src[0])
            ue = tree.box_centre(src) + rs * ops.UE
            phi[idx] += kernel_matrix(x[idx], ue) @ (Ut @ up[src])
        for nb in tree.U(lf):                                                        # S2T
            j = tree.leaf_points[nb]
            phi[idx] += kernel_matrix(x[idx], x[j]) @ s[j]
    return phi[:, 0] if vec else phi
