"""Pins of the BEM oracle (oracle/bem.py; CPU only).

The collocation BEM of Sec. 4 is pinned to things other than itself:
* the ellipsoid mesh: 8 * 4^level triangles, closed (every edge in exactly two
  triangles, Euler characteristic 2), outward orientation, vertices on the
  ellipsoid;
* the 7-point rule integrates every monomial of degree <= 5 exactly on a
  triangle and fails at degree 6 (the exact moments are x^i y^j -> i! j! /
  (i + j + 2)! on the unit right triangle);
* the closed-form single-layer integral: sqrt(3) s ln(2 + sqrt(3)) at the
  centroid of an equilateral triangle of side s, and adaptive subdivision
  quadrature at points off the triangle and in its plane outside it;
* the solid angle: Gauss's theorem on the closed mesh (4 pi inside, 0
  outside, 2 pi from a face's centroid with the face itself left out), and
  subdivision quadrature of the dipole kernel off the triangle;
* the conductor: the closed form on a sphere (Q = 4 pi R V, uniform density),
  the density integrating to Q on a fine mesh, and the dense BEM solution
  converging to it as the mesh is refined;
* the double layer applied to q = 1 is exactly -1/2 at every centroid;
* the KIFMM BEM matvec against the dense operators, the error falling with p;
* planted mistakes (no arctan term, flipped orientation, the single-layer
  kernel in the first step of S2M for the double layer) fail these pins.
"""
import functools
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import bem

AXES = (2.0, 1.0, 3.0)


@functools.lru_cache(maxsize=None)
def mesh(level, axes=AXES):
    return workloads.ellipsoid_surface_mesh(level, axes)


def test_mesh_closed_oriented_on_surface():
    for level in (2, 3):
        V, F = mesh(level)
        assert F.shape == (8 * 4 ** level, 3)
        edges = {}
        for a, b, c in F:
            for e in ((a, b), (b, c), (c, a)):
                k = (min(e), max(e))
                edges[k] = edges.get(k, 0) + 1
        assert set(edges.values()) == {2}
        assert V.shape[0] - len(edges) + F.shape[0] == 2
        c, ar, nrm = bem.geometry(V, F)
        assert np.all(np.einsum("ij,ij->i", nrm, c) > 0) and np.all(ar > 0)
        r = (V / np.asarray(AXES)) ** 2
        assert np.allclose(r.sum(axis=1), 1.0, atol=1e-14)


def test_quad7_degree_five():
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    P = bem.QUAD7_BARY @ v
    w = 0.5 * bem.QUAD7_W
    assert abs(bem.QUAD7_W.sum() - 1.0) < 1e-15
    worst6 = 0.0
    for deg in range(7):
        for i in range(deg + 1):
            j = deg - i
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            got = float((w * P[:, 0] ** i * P[:, 1] ** j).sum())
            if deg <= 5:
                assert abs(got - exact) < 1e-15, (i, j)
            else:
                worst6 = max(worst6, abs(got - exact))
    assert worst6 > 1e-6


def _subdiv_quad(x, a, b, c, lev, f):
    tris = [(a, b, c)]
    for _ in range(lev):
        nt = []
        for (p, q, r) in tris:
            pq, qr, rp = (p + q) / 2, (q + r) / 2, (r + p) / 2
            nt += [(p, pq, rp), (q, qr, pq), (r, rp, qr), (pq, qr, rp)]
        tris = nt
    tot = 0.0
    for (p, q, r) in tris:
        ar = 0.5 * np.linalg.norm(np.cross(q - p, r - p))
        for k in range(7):
            y = bem.QUAD7_BARY[k] @ np.stack([p, q, r])
            tot += bem.QUAD7_W[k] * ar * f(x, y)
    return tot


TRI = (np.array([[0.1, -0.2, 0.05]]), np.array([[1.4, 0.1, -0.1]]), np.array([[0.5, 1.2, 0.3]]))
POINTS = [(0.4, 0.3, 0.6), (2.0, -1.0, 0.5), (0.6, 0.3, -0.4), (-1.0, 0.2, 0.0)]


def test_single_layer_closed_forms():
    s = 1.3
    v0, v1, v2 = np.array([[0, 0, 0.0]]), np.array([[s, 0, 0.0]]), np.array([[s / 2, s * math.sqrt(3) / 2, 0.0]])
    c = (v0 + v1 + v2) / 3
    assert abs(bem.single_layer_integral(c, v0, v1, v2)[0, 0] - math.sqrt(3) * s * math.log(2 + math.sqrt(3))) < 1e-13
    # in-plane point outside the triangle and off-plane points: subdivision quadrature
    n = np.cross(TRI[1][0] - TRI[0][0], TRI[2][0] - TRI[0][0])
    inplane = TRI[0][0] + 1.7 * (TRI[1][0] - TRI[0][0]) - 0.4 * (TRI[2][0] - TRI[0][0])
    assert abs(n @ (inplane - TRI[0][0])) < 1e-12
    for x in POINTS + [tuple(inplane)]:
        x = np.array(x)
        an = bem.single_layer_integral(x[None], *TRI)[0, 0]
        nu = _subdiv_quad(x, TRI[0][0], TRI[1][0], TRI[2][0], 4, lambda x, y: 1 / np.linalg.norm(x - y))
        assert abs(an - nu) < 1e-9 * abs(nu), (x, an, nu)


def test_solid_angle_gauss_and_quadrature():
    V, F = mesh(3)
    v0, v1, v2 = bem.triangles(V, F)
    for x, want in (([0.0, 0.0, 0.0], 4 * math.pi), ([0.5, 0.2, 1.0], 4 * math.pi), ([5.0, 0.0, 0.0], 0.0)):
        assert abs(bem.solid_angle(np.array([x]), v0, v1, v2).sum() - want) < 1e-12
    c, _, _ = bem.geometry(V, F)
    om = bem.solid_angle(c[:40], v0, v1, v2)
    for i in range(40):
        assert abs(om[i].sum() - om[i, i] - 2 * math.pi) < 1e-12
    nrm = np.cross(TRI[1][0] - TRI[0][0], TRI[2][0] - TRI[0][0])
    nrm /= np.linalg.norm(nrm)
    for x in POINTS:
        x = np.array(x)
        an = bem.solid_angle(x[None], *TRI)[0, 0]
        nu = _subdiv_quad(x, TRI[0][0], TRI[1][0], TRI[2][0], 4,
                          lambda x, y: nrm @ (y - x) / np.linalg.norm(y - x) ** 3)
        assert abs(an - nu) < 1e-8 * max(1.0, abs(nu)), (x, an, nu)


def test_conductor_closed_form():
    assert abs(bem.conductor_charge((1.0, 1.0, 1.0)) - 4 * math.pi) < 1e-10
    assert abs(bem.conductor_charge((2.0, 2.0, 2.0), V=3.0) - 24 * math.pi) < 1e-9
    x = np.array([[0.0, 0.0, 1.0], [0.6, 0.8, 0.0]])
    assert np.allclose(bem.conductor_density(x, (1.0, 1.0, 1.0)), 1.0, rtol=1e-12)
    V, F = mesh(6)
    c, ar, _ = bem.geometry(V, F)
    # the centroids lie inside the ellipsoid; their radial projection carries the density
    s = np.sqrt(((c / np.asarray(AXES)) ** 2).sum(axis=1))
    Q = float((bem.conductor_density(c / s[:, None], AXES) * ar).sum())
    assert abs(Q - bem.conductor_charge(AXES)) < 2e-3 * bem.conductor_charge(AXES)


@functools.lru_cache(maxsize=None)
def dense(level, layer):
    V, F = mesh(level)
    return bem.dense_operator(V, F, layer)


def test_dense_solution_converges_to_closed_form():
    errs = []
    for level in (3, 4):
        V, F = mesh(level)
        c, ar, _ = bem.geometry(V, F)
        q = np.linalg.solve(dense(level, "single"), np.ones(F.shape[0]))
        ex = bem.conductor_density(c, AXES)
        errs.append(float(np.linalg.norm(q - ex) / np.linalg.norm(ex)))
        Qex = bem.conductor_charge(AXES)
        assert abs(float((q * ar).sum()) - Qex) < 0.01 * Qex
    print("density errors", errs)
    assert errs[0] < 0.03 and errs[1] < 0.01 and errs[1] < errs[0] / 2


def test_double_layer_of_constant_is_minus_half():
    B = dense(3, "double")
    assert np.allclose(B @ np.ones(B.shape[0]), -0.5, atol=1e-13)


def test_gmres_matches_direct_solve():
    A = dense(3, "single")
    b = np.ones(A.shape[0])
    x, it = bem.gmres_solve(lambda v: A @ v, b, rtol=1e-12)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9) and it > 3


@pytest.mark.parametrize("layer,tol4,tol6", [("single", 5e-4, 3e-5), ("double", 3e-2, 3e-3)])
def test_fmm_matvec_vs_dense(layer, tol4, tol6):
    V, F = mesh(4)
    M = dense(4, layer)
    x = workloads.uniform_density(F.shape[0], 3)
    want = M @ x
    errs = []
    for p, tol in ((4, tol4), (6, tol6)):
        phi, _ = bem.bem_fmm(V, F, x, p, 1e-8, 32, layer=layer)
        errs.append(float(np.linalg.norm(phi - want) / np.linalg.norm(want)))
        assert errs[-1] < tol, (p, errs)
    print(layer, "fmm vs dense p=4/6", errs)
    assert errs[1] < errs[0] / 5
    if layer == "double":
        phi1, _ = bem.bem_fmm(V, F, np.ones(F.shape[0]), 6, 1e-8, 32, layer=layer)
        assert np.abs(phi1 + 0.5).max() < 1e-3


# ------------------------------------------------------- planted mistakes
def test_planted_mistakes_fail(monkeypatch):
    # (a) the arctan term dropped: off-plane values wrong
    x = np.array(POINTS[0])
    good = bem.single_layer_integral(x[None], *TRI)[0, 0]
    monkeypatch.setattr(np, "arctan", lambda z: 0.0 * z)
    bad = bem.single_layer_integral(x[None], *TRI)[0, 0]
    monkeypatch.undo()
    assert abs(bad - good) > 1e-3 * abs(good)
    # (b) orientation flipped: Gauss sum has the wrong sign
    V, F = mesh(2)
    v0, v1, v2 = bem.triangles(V, F)
    assert abs(bem.solid_angle(np.zeros((1, 3)), v0, v2, v1).sum() + 4 * math.pi) < 1e-12
    # (c) the double layer with the single-layer kernel in the first step of S2M
    V, F = mesh(4)
    B = dense(4, "double")
    q = workloads.uniform_density(F.shape[0], 3)
    orig = bem.kernel_at
    monkeypatch.setattr(bem, "kernel_at", lambda P, Y, nrm, layer: orig(P, Y, nrm, "single"))
    phi, _ = bem.bem_fmm(V, F, q, 6, 1e-8, 32, layer="double")
    monkeypatch.undo()
    assert np.linalg.norm(phi - B @ q) / np.linalg.norm(B @ q) > 1e-1


def green_data(level, x0=(3.0, 0.5, 4.0)):
    """u = 1/|y - x0| (harmonic inside the ellipsoid, x0 outside) and its
    outward normal derivative at the centroids."""
    V, F = mesh(level)
    c, _, nrm = bem.geometry(V, F)
    d = c - np.asarray(x0)
    r = np.linalg.norm(d, axis=1)
    return V, F, 1.0 / r, -np.einsum("ij,ij->i", d, nrm) / r ** 3


def test_green_identity_single_and_double_layer():
    # Green's third identity on the boundary (n outward): for u harmonic inside,
    # S[du/dn] - B[u] = u / 2 at every smooth boundary point; the collocation
    # residual falls with the mesh size (the mixed-condition problems of Sec. 5.2
    # combine exactly these two operators)
    res = []
    for level in (3, 4):
        V, F, u, dn = green_data(level)
        r = dense(level, "single") @ dn - dense(level, "double") @ u - 0.5 * u
        res.append(float(np.linalg.norm(r) / np.linalg.norm(0.5 * u)))
    print("Green identity residuals", res)
    assert res[0] < 0.05 and res[1] < res[0] / 1.8
