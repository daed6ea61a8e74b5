"""Seeded synthetic point sets and densities shaped like the paper's BEM workloads.

This module only generates inputs (geometry and densities). It holds none of
the fast multipole method's arithmetic and is shared by the oracle, the tests
and the benchmark, so that both sides of every parity check see the same data.

The paper's workloads are collocation points of triangulated surfaces (element
centroids, Sec. 4.1) of an ellipsoid refined from 512 triangles (Sec. 5.1),
a shaft and an engine block (Sec. 5.2-5.3; meshes not available). The
generators below stand in for them with seeded meshes of the same kind:
icosphere and ellipsoid centroids, cube and torus surfaces.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosphere",
    "icosphere_centroids",
    "sphere_points",
    "ellipsoid_points",
    "uniform_cube",
    "cube_surface",
    "torus_grid_centroids",
    "torus_random",
    "sphere_density",
    "uniform_density",
    "batch_sets",
    "SEED_BASE",
]

SEED_BASE = 1211


def icosphere(level: int):
    """Vertices (V,3) on the unit sphere and faces (F,3) of a level-`level`
    subdivided icosahedron (20*4**level faces)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
         [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
         [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        key = e[:, 0] * (nv + 1) + e[:, 1]
        uk, inv = np.unique(key, return_inverse=True)
        a = uk // (nv + 1)
        b = uk % (nv + 1)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = inv.reshape(3, -1) + nv  # midpoint ids of edges (01, 12, 20)
        m01, m12, m20 = m[0], m[1], m[2]
        v = np.concatenate([v, mid], axis=0)
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)], axis=0)
    return v, f


def icosphere_centroids(level: int, scale=(1.0, 1.0, 1.0)):
    """Centroids (F,3) and areas (F,) of the flat triangles of a level-`level`
    icosphere whose vertices are scaled per axis by `scale`."""
    v, f = icosphere(level)
    v = v * np.asarray(scale, dtype=np.float64)[None, :]
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    cen = (a + b + c) / 3.0
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return cen, area


def _subset(n_total: int, n: int, rng: np.random.Generator) -> np.ndarray:
    if n > n_total:
        raise ValueError(f"requested {n} of {n_total} faces")
    return rng.choice(n_total, size=n, replace=False)


def _level_for(n: int) -> int:
    lev = 0
    while 20 * 4 ** lev < n:
        lev += 1
    return lev


def sphere_points(n: int, seed: int, return_area: bool = False):
    """n centroids drawn without replacement from the smallest icosphere with
    at least n faces (radius 1). n = 2**20 uses the level-8 icosphere
    (1,310,720 faces). Returned in the drawn (unsorted) order."""
    rng = np.random.default_rng(seed)
    cen, area = icosphere_centroids(_level_for(n))
    idx = _subset(cen.shape[0], n, rng)
    if return_area:
        return cen[idx].copy(), area[idx].copy()
    return cen[idx].copy()


def ellipsoid_points(n: int, seed: int, axes=(2.0, 1.0, 0.5)):
    """n centroids of an icosphere whose vertices are scaled by `axes`."""
    rng = np.random.default_rng(seed)
    cen, _ = icosphere_centroids(_level_for(n), scale=axes)
    idx = _subset(cen.shape[0], n, rng)
    return cen[idx].copy()


def ellipsoid_surface_mesh(level: int, axes=(2.0, 1.0, 3.0)):
    """Triangulated ellipsoid: the octahedron (8 faces) refined `level` times by
    edge midpoints pushed out to the unit sphere, vertices scaled by `axes`.
    8 * 4^level triangles (level 3: 512, each further level x4), outward
    orientation (counterclockwise seen from outside). Returns (vertices (nv, 3)
    float64, triangles (nt, 3) int32)."""
    v = [np.array(a, dtype=np.float64) for a in
         ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
    f = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    for _ in range(level):
        mid = {}

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                w = v[a] + v[b]
                v.append(w / np.linalg.norm(w))
                mid[key] = len(v) - 1
            return mid[key]
        nf = []
        for a, b, c in f:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    verts = np.asarray(v) * np.asarray(axes, dtype=np.float64)
    return verts, np.asarray(f, dtype=np.int32)


def clustered_points(n_bg: int, n_cl: int, seed: int, centre=(0.5, 0.5, 0.5), width: float = 0.02):
    """n_bg iid uniform points in [-1,1]^3 and a Gaussian cluster of n_cl
    points (standard deviation `width`) around `centre`: a point set whose
    cube occupancy varies by orders of magnitude (adaptive-tree workloads)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, (n_bg, 3))
    b = width * rng.standard_normal((n_cl, 3)) + np.asarray(centre, dtype=np.float64)
    return np.concatenate([a, b])


def corner_clusters(n_dense: int, n_sparse: int, seed: int):
    """A dense Gaussian cluster near (0.9, 0.9, 0.9) and a sparse one near
    (-0.9, -0.9, -0.9): the sparse octant stays a leaf at level 1."""
    rng = np.random.default_rng(seed)
    a = 0.03 * rng.standard_normal((n_dense, 3)) + 0.9
    b = 0.05 * rng.standard_normal((n_sparse, 3)) - 0.9
    return np.concatenate([a, b])


def uniform_cube(n: int, seed: int):
    """n iid points uniform in the unit cube [0,1]^3."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3))


def cube_surface(n: int, seed: int):
    """n points area-uniform on the surface of [-1,1]^3."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-1.0, 1.0, size=(n, 2))
    x = np.empty((n, 3))
    ax = face // 2
    sgn = np.where(face % 2 == 0, -1.0, 1.0)
    for a in range(3):
        sel = ax == a
        others = [b for b in range(3) if b != a]
        x[sel, a] = sgn[sel]
        x[sel, others[0]] = uv[sel, 0]
        x[sel, others[1]] = uv[sel, 1]
    return x


def _torus_xyz(u, v, big_r, small_r):
    u, v = np.broadcast_arrays(u, v)
    return np.stack([(big_r + small_r * np.cos(v)) * np.cos(u),
                     (big_r + small_r * np.cos(v)) * np.sin(u),
                     small_r * np.sin(v)], axis=-1)


def torus_grid_centroids(nu: int, nv: int, big_r: float = 1.0, small_r: float = 0.3):
    """Centroids of the 2*nu*nv triangles of a (u,v)-grid triangulation of a
    torus (major radius big_r, minor radius small_r)."""
    u = 2 * np.pi * np.arange(nu + 1) / nu
    v = 2 * np.pi * np.arange(nv + 1) / nv
    P = _torus_xyz(u[:, None], v[None, :], big_r, small_r)  # (nu+1, nv+1, 3)
    p00 = P[:-1, :-1]
    p10 = P[1:, :-1]
    p01 = P[:-1, 1:]
    p11 = P[1:, 1:]
    c1 = (p00 + p10 + p11) / 3.0
    c2 = (p00 + p11 + p01) / 3.0
    return np.concatenate([c1.reshape(-1, 3), c2.reshape(-1, 3)], axis=0)


def torus_random(n: int, seed: int, big_r: float = 1.0, small_r: float = 0.3):
    """n points area-uniform on a torus (rejection sampling on the v angle)."""
    rng = np.random.default_rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 16
        u = rng.uniform(0, 2 * np.pi, m)
        v = rng.uniform(0, 2 * np.pi, m)
        w = rng.uniform(0, 1, m)
        keep = w < (big_r + small_r * np.cos(v)) / (big_r + small_r)
        out = np.concatenate([out, _torus_xyz(u[keep], v[keep], big_r, small_r)], axis=0)
    return out[:n].copy()


def sphere_density(x: np.ndarray, seed: int):
    """1 + 0.5*Y_2^0(theta) + N(0, 0.01) noise, theta the polar angle of x."""
    rng = np.random.default_rng(seed)
    r = np.linalg.norm(x, axis=1)
    cth = x[:, 2] / np.where(r > 0, r, 1.0)
    y20 = math.sqrt(5.0 / (16.0 * math.pi)) * (3.0 * cth * cth - 1.0)
    return 1.0 + 0.5 * y20 + rng.normal(0.0, 0.1, size=x.shape[0])


def uniform_density(n: int, seed: int, nrhs: int | None = None):
    """iid U[-1,1] densities, shape (n,) or (n, nrhs) (column j = RHS j)."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        return rng.uniform(-1.0, 1.0, size=n)
    return rng.uniform(-1.0, 1.0, size=(nrhs, n)).T.copy()


def batch_sets(count: int = 24, seed: int = SEED_BASE + 3, lo_log2: int = 12, hi_log2: int = 19):
    """`count` independent surface point sets: shape i mod 3 is a sphere, a cube
    surface or a torus (R=1, r=0.3); sizes N_i = round(2**(lo + (hi-lo)*u_i))
    with u_i ~ U[0,1) drawn from `seed`. Returns a list of (points, name)."""
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    sizes = [int(round(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * ui))) for ui in u]
    out = []
    for i, n in enumerate(sizes):
        s = seed * 1000 + i
        kind = i % 3
        if kind == 0:
            out.append((sphere_points(n, s), "sphere"))
        elif kind == 1:
            out.append((cube_surface(n, s), "cube_surface"))
        else:
            out.append((torus_random(n, s), "torus"))
    return out
