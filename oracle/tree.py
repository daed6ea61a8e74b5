"""Octree, near fields and interaction fields (test infrastructure only).

Sec. 2.1: the points are enclosed in a root cube that is split into 8 equal
children level after level until every leaf holds at most s points. For a cube
C the near field N^C is the set of same-level cubes sharing at least one vertex
with C (C included); the far field F^C is everything else; with B the parent of
C the interaction field is I^C = F^C minus F^B.

Readings where the paper is silent (also taken by the GPU library, which has
its own implementation of them):

* root cube: centre = midpoint of the axis-aligned bounding box, half-width
  r0 = max extent / 2 * (1 + 2**-20) (r0 = 1 for a zero extent);
* integer coordinates q = min(floor((x - (centre - r0)) / (2 r0) * 2**21), 2**21 - 1)
  per axis in FP64; the level-l cube of a point is q >> (21 - l);
* uniform depth: L is the smallest level >= 0 at which every nonempty cube
  holds at most s points, capped at `max_depth` (oversize leaves allowed
  then); every leaf sits at level L;
* cube index vectors are integer triples; half-width at level l is r0 / 2**l
  and the centre of cube b is (centre - r0) + (2 b + 1) r_l.

Boxes are plain dictionaries keyed by integer triples: no Morton order, no
sorting beyond what is needed to list them.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

QBITS = 21


def root_cube(x: np.ndarray):
    """Centre (3,) and half-width r0 of the root cube."""
    lo = x.min(axis=0)
    hi = x.max(axis=0)
    centre = (lo + hi) / 2.0
    ext = float((hi - lo).max())
    r0 = ext / 2.0 * (1.0 + 2.0 ** -20) if ext > 0 else 1.0
    return centre, r0


def integer_coords(x: np.ndarray, centre: np.ndarray, r0: float) -> np.ndarray:
    """21-bit integer coordinates of the points (N,3) int64."""
    lo = centre - r0
    q = np.floor((x - lo) / (2.0 * r0) * float(1 << QBITS)).astype(np.int64)
    return np.clip(q, 0, (1 << QBITS) - 1)


NEIGHBOUR_OFFSETS = list(itertools.product((-1, 0, 1), repeat=3))
CHILD_OFFSETS = list(itertools.product((0, 1), repeat=3))


@dataclass
class OracleTree:
    centre: np.ndarray
    r0: float
    depth: int
    q: np.ndarray                     # (N,3) integer coordinates
    leaf_of_point: list               # point index -> leaf triple
    leaf_points: dict                 # leaf triple -> np.ndarray of point indices
    boxes: list = field(default_factory=list)   # boxes[l] = set of triples at level l

    def half_width(self, level: int) -> float:
        return self.r0 / float(2 ** level)

    def box_centre(self, level: int, b) -> np.ndarray:
        r = self.half_width(level)
        return (self.centre - self.r0) + (2.0 * np.asarray(b, dtype=np.float64) + 1.0) * r

    def near(self, level: int, b):
        """N^b: nonempty same-level cubes sharing a vertex with b (b included)."""
        out = []
        for d in NEIGHBOUR_OFFSETS:
            c = (b[0] + d[0], b[1] + d[1], b[2] + d[2])
            if c in self.boxes[level]:
                out.append(c)
        return out

    def interaction(self, level: int, b):
        """I^b = F^b minus F^parent: children of the parent's near field that
        are not in b's own near field (nonempty cubes only)."""
        if level < 1:
            return []
        parent = (b[0] >> 1, b[1] >> 1, b[2] >> 1)
        out = []
        for pn in self.near(level - 1, parent):
            for o in CHILD_OFFSETS:
                c = (2 * pn[0] + o[0], 2 * pn[1] + o[1], 2 * pn[2] + o[2])
                if c not in self.boxes[level]:
                    continue
                if max(abs(c[0] - b[0]), abs(c[1] - b[1]), abs(c[2] - b[2])) >= 2:
                    out.append(c)
        return out


def choose_depth(q: np.ndarray, leaf_size: int, max_depth: int) -> int:
    for level in range(0, max_depth + 1):
        cells = q >> (QBITS - level)
        _, counts = np.unique(cells, axis=0, return_counts=True)
        if counts.max() <= leaf_size:
            return level
    return max_depth


def build_tree(x: np.ndarray, leaf_size: int, depth: int | None = None,
               max_depth: int = 16) -> OracleTree:
    x = np.asarray(x, dtype=np.float64)
    centre, r0 = root_cube(x)
    q = integer_coords(x, centre, r0)
    L = choose_depth(q, leaf_size, max_depth) if depth is None else int(depth)
    leaf_cells = q >> (QBITS - L)
    leaf_of_point = [tuple(int(v) for v in row) for row in leaf_cells]
    leaf_points: dict = {}
    for i, b in enumerate(leaf_of_point):
        leaf_points.setdefault(b, []).append(i)
    leaf_points = {b: np.asarray(v, dtype=np.int64) for b, v in leaf_points.items()}
    boxes = [set() for _ in range(L + 1)]
    boxes[L] = set(leaf_points.keys())
    for level in range(L - 1, -1, -1):
        boxes[level] = {(b[0] >> 1, b[1] >> 1, b[2] >> 1) for b in boxes[level + 1]}
    return OracleTree(centre=centre, r0=r0, depth=L, q=q, leaf_of_point=leaf_of_point,
                      leaf_points=leaf_points, boxes=boxes)
