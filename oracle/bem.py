"""Collocation BEM for the Laplace single- and double-layer operators (Sec. 4;
test infrastructure only).

The boundary is a triangulated surface with piecewise-constant densities
q_j on the triangles and collocation points x_i at the centroids. The
operators are

    single layer   (A q)_i = sum_j q_j int_{T_j} G(x_i, y) dS_y,
    double layer   (B q)_i = sum_j q_j int_{T_j} dG(x_i, y)/dn(y) dS_y,

G = 1/(4 pi |x - y|), n the unit normal of T_j (the orientation of its
vertices), the self term of B its principal value (0 on a flat triangle).

* ``single_layer_integral`` - int_T 1/|x - y| dS_y in closed form, summed over
  the edges: for the projection x0 of x on the plane of T and its height h,
  each edge with in-plane outward normal m and unit tangent t contributes
  p ln((R+ + s+)/(R- + s-)) - |h| (atan(p s+ / (R0^2 + |h| R+)) -
  atan(p s- / (R0^2 + |h| R-))), p = (a - x0).m, s = (end - x0).t,
  R0^2 = p^2 + h^2, R = sqrt(s^2 + R0^2) (Wilton et al., IEEE Trans. AP 1984).
* ``solid_angle`` - the signed solid angle Omega = int_T n.(y - x)/|y - x|^3 dS_y
  by the formula of Van Oosterom and Strackee (IEEE Trans. BME 1983):
  tan(Omega/2) = det[R1 R2 R3] / (|R1||R2||R3| + (R1.R2)|R3| + (R1.R3)|R2| +
  (R2.R3)|R1|), R_k = v_k - x; int_T dG/dn(y) dS_y = -Omega / (4 pi).
* ``QUAD7`` - the 7-point degree-5 rule on a triangle (Radon, 1948), used for
  the far-field source integrals of S2M (Sec. 4.2): a triangle's sources are
  its seven points with weights w_k area_j.
* ``dense_operator`` - A or B in full (the exact integrals for every pair).
* ``bem_fmm`` - the KIFMM matvec of Sec. 4: the octree over the centroids, S2M
  by the 7-point rule over the triangles of the leaf (Sec. 4.2, with the
  double-layer kernel in its first step for B, eq. of Sec. 4.2), S2T by the
  exact integrals over the near-field triangles, the other steps as for points.
* ``conductor_density`` - the charge density on an ellipsoid held at potential
  V in closed form: Q = 8 pi V / I0, I0 = int_0^inf ds / sqrt((a^2+s)(b^2+s)(c^2+s)),
  sigma(x) = Q / (4 pi a b c sqrt(x^2/a^4 + y^2/b^4 + z^2/c^4)).
* ``gmres_solve`` - the linear system by GMRES (scipy's routine as one step).
"""
from __future__ import annotations

import math

import numpy as np

from .fmm import fmm

FOUR_PI = 4.0 * math.pi

_s15 = math.sqrt(15.0)
_a1, _b1 = (6.0 - _s15) / 21.0, (9.0 + 2.0 * _s15) / 21.0
_a2, _b2 = (6.0 + _s15) / 21.0, (9.0 - 2.0 * _s15) / 21.0
_w1, _w2 = (155.0 - _s15) / 1200.0, (155.0 + _s15) / 1200.0
# barycentric coordinates (7, 3) and weights (7,) summing to 1
QUAD7_BARY = np.array([[1 / 3, 1 / 3, 1 / 3],
                       [_a1, _a1, _b1], [_a1, _b1, _a1], [_b1, _a1, _a1],
                       [_a2, _a2, _b2], [_a2, _b2, _a2], [_b2, _a2, _a2]])
QUAD7_W = np.array([9.0 / 40.0, _w1, _w1, _w1, _w2, _w2, _w2])


def triangles(vertices, tris):
    """(v0, v1, v2) arrays (n, 3) of the triangles."""
    V = np.asarray(vertices, dtype=np.float64)
    F = np.asarray(tris)
    return V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]


def geometry(vertices, tris):
    """Centroids (n, 3), areas (n,), unit normals (n, 3)."""
    v0, v1, v2 = triangles(vertices, tris)
    cr = np.cross(v1 - v0, v2 - v0)
    ar = 0.5 * np.linalg.norm(cr, axis=1)
    return (v0 + v1 + v2) / 3.0, ar, cr / (2.0 * ar[:, None])


def quad_points(vertices, tris):
    """Quadrature points (n, 7, 3) and weights w_k * area (n, 7)."""
    v0, v1, v2 = triangles(vertices, tris)
    _, ar, _ = geometry(vertices, tris)
    P = (QUAD7_BARY[None, :, 0, None] * v0[:, None] + QUAD7_BARY[None, :, 1, None] * v1[:, None]
         + QUAD7_BARY[None, :, 2, None] * v2[:, None])
    return P, ar[:, None] * QUAD7_W[None, :]


def single_layer_integral(x, v0, v1, v2):
    """int_{T_j} 1/|x_i - y| dS_y for points x (m, 3) and triangles (n, 3) each:
    (m, n), in closed form (see the module docstring)."""
    x = np.asarray(x, dtype=np.float64)[:, None, :]
    cr = np.cross(v1 - v0, v2 - v0)
    nrm = cr / np.linalg.norm(cr, axis=1)[:, None]
    h = np.einsum("mnk,nk->mn", x - v0[None], nrm)
    x0 = x - h[..., None] * nrm[None]
    ah = np.abs(h)
    total = np.zeros(h.shape)
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        ed = b - a
        t = ed / np.linalg.norm(ed, axis=1)[:, None]
        m = np.cross(t, nrm)                                  # in-plane, outward
        p = np.einsum("mnk,nk->mn", a[None] - x0, m)
        sm = np.einsum("mnk,nk->mn", a[None] - x0, t)
        sp = np.einsum("mnk,nk->mn", b[None] - x0, t)
        r0 = p * p + h * h
        rm = np.sqrt(sm * sm + r0)
        rp = np.sqrt(sp * sp + r0)
        # ln((R+ + s+)/(R- + s-)), in the form without cancellation: for s < 0,
        # R + s = R0^2 / (R - s)
        with np.errstate(divide="ignore", invalid="ignore"):
            num = np.where(sp >= 0, rp + sp, r0 / (rp - sp))
            den = np.where(sm >= 0, rm + sm, r0 / (rm - sm))
            lg = np.where(np.abs(p) > 0, p * np.log(num / den), 0.0)
            at = np.where((ah > 0) & (np.abs(p) > 0),
                          np.arctan(p * sp / (r0 + ah * rp)) - np.arctan(p * sm / (r0 + ah * rm)), 0.0)
        total += lg - ah * at
    return total


def solid_angle(x, v0, v1, v2):
    """Signed solid angle int_{T_j} n.(y - x_i)/|y - x_i|^3 dS_y, (m, n)."""
    x = np.asarray(x, dtype=np.float64)[:, None, :]
    R1, R2, R3 = v0[None] - x, v1[None] - x, v2[None] - x
    l1, l2, l3 = (np.linalg.norm(R, axis=2) for R in (R1, R2, R3))
    num = np.einsum("mnk,mnk->mn", R1, np.cross(R2, R3))
    den = (l1 * l2 * l3 + np.einsum("mnk,mnk->mn", R1, R2) * l3 + np.einsum("mnk,mnk->mn", R1, R3) * l2
           + np.einsum("mnk,mnk->mn", R2, R3) * l1)
    return 2.0 * np.arctan2(num, den)


def layer_integral(x, v0, v1, v2, layer):
    """int_{T_j} K(x_i, y) dS_y with K = G (layer "single") or dG/dn(y) ("double")."""
    if layer == "single":
        return single_layer_integral(x, v0, v1, v2) / FOUR_PI
    if layer == "double":
        return -solid_angle(x, v0, v1, v2) / FOUR_PI
    raise ValueError(layer)


def dense_operator(vertices, tris, layer="single", chunk=256):
    """The collocation matrix (n, n) of the layer at the centroids, exact integrals."""
    v0, v1, v2 = triangles(vertices, tris)
    c, _, _ = geometry(vertices, tris)
    n = c.shape[0]
    A = np.empty((n, n))
    for i0 in range(0, n, chunk):
        A[i0:i0 + chunk] = layer_integral(c[i0:i0 + chunk], v0, v1, v2, layer)
    if layer == "double":
        A[np.arange(n), np.arange(n)] = 0.0       # principal value on the flat self triangle
    return A


def kernel_at(P, Y, nrm, layer):
    """K(P_a, Y_b) (m, n) for points P, sources Y with unit normals nrm (n, 3)."""
    d = P[:, None, :] - Y[None, :, :]
    r = np.linalg.norm(d, axis=2)
    if layer == "single":
        return 1.0 / (FOUR_PI * r)
    return np.einsum("mnk,nk->mn", d, nrm) / (FOUR_PI * r ** 3)


def bem_fmm(vertices, tris, q, p, eps, leaf_size, layer="single", mode="svd", ops=None, tree=None):
    """The KIFMM BEM matvec (Sec. 4) at the centroids: (phi, info)."""
    c, _, nrm = geometry(vertices, tris)
    v0, v1, v2 = triangles(vertices, tris)
    QP, QW = quad_points(vertices, tris)

    def source_field(P, idx):
        # S2M check potential of unit densities on triangles idx: the 7-point rule
        out = np.zeros((P.shape[0], len(idx)))
        for k in range(7):
            out += kernel_at(P, QP[idx, k], nrm[idx], layer) * QW[idx, k][None, :]
        return out

    def near_field(tidx, sidx):
        G = layer_integral(c[tidx], v0[sidx], v1[sidx], v2[sidx], layer)
        if layer == "double":
            G[np.asarray(tidx)[:, None] == np.asarray(sidx)[None, :]] = 0.0
        return G

    return fmm(c, q, p, eps, leaf_size, mode=mode, ops=ops, tree=tree, source_field=source_field,
               near_field=near_field)


def conductor_charge(axes, V=1.0):
    """Total charge of the ellipsoid with semi-axes `axes` at potential V."""
    from scipy.integrate import quad
    a, b, cc = axes
    I0, _ = quad(lambda s: 1.0 / math.sqrt((a * a + s) * (b * b + s) * (cc * cc + s)), 0.0, math.inf,
                 epsabs=0.0, epsrel=1e-13, limit=500)
    return 8.0 * math.pi * V / I0


def conductor_density(x, axes, V=1.0):
    """Closed-form surface charge density at points x (n, 3) on the ellipsoid."""
    a, b, cc = axes
    x = np.asarray(x, dtype=np.float64)
    g = np.sqrt(x[:, 0] ** 2 / a ** 4 + x[:, 1] ** 2 / b ** 4 + x[:, 2] ** 2 / cc ** 4)
    return conductor_charge(axes, V) / (4.0 * math.pi * a * b * cc * g)


def gmres_solve(matvec, b, rtol=1e-10, restart=200, maxiter=2000):
    """x with matvec(x) = b by GMRES (scipy); returns (x, iterations)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    n = b.shape[0]
    count = [0]

    def mv(v):
        count[0] += 1
        return matvec(np.asarray(v, dtype=np.float64).ravel())
    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    x, info = gmres(op, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"GMRES did not converge (info {info})")
    return x, count[0]
