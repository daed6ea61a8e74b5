"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
* FP64 device mode against the oracle in the same mode: 1e-10 relative L2 at
  p=4 and 1e-8 at p=6 (both evaluate the same operators in double; they differ
  by the rounding of two independent SVD/pseudo-inverse routes and summation
  order, amplified by the conditioning of the check-to-equivalent systems).
* FP32 device mode against the FP64 dense-M2L oracle: 1e-5 relative L2, the
  bar set for this matvec. The SVD truncation at eps = 1e-6 contributes about
  1e-6 of it and FP32 rounding the rest.
"""
import functools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sphere1m_p6_samples.json")


def _k():
    import paper_1211_2517_amd as K
    return K


def _torch():
    import torch
    return torch


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    """max |a - b| / max |b| (a wrong value at one point is not diluted)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_apply(x, s, p, eps, leaf, precision="fp32", dense=False, adjoint=False, **kw):
    torch = _torch()
    plan = _k().Plan(x, p=p, eps=eps, leaf_size=leaf, precision=precision, dense_m2l=dense, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    sd = torch.tensor(np.asarray(s), dtype=dt, device="cuda:0")
    out = plan.apply_adjoint(sd) if adjoint else plan.apply(sd)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), plan


@functools.lru_cache(maxsize=None)
def oracle_ops(p, eps, leaf, mode):
    return oracle.build_operators(p, eps, leaf, mode=mode)


@functools.lru_cache(maxsize=None)
def cube(n=4096):
    x = workloads.uniform_cube(n, workloads.SEED_BASE)
    s = workloads.uniform_density(n, workloads.SEED_BASE + 100)
    return x, s


@functools.lru_cache(maxsize=None)
def oracle_phi(kind, n, p, eps, leaf, mode):
    x, s = cube(n) if kind == "cube" else sphere(n)
    return oracle.fmm(x, s, p, eps, leaf, ops=oracle_ops(p, eps, leaf, mode))[0]


@functools.lru_cache(maxsize=None)
def sphere(n):
    x = workloads.sphere_points(n, workloads.SEED_BASE + 1)
    return x, workloads.sphere_density(x, workloads.SEED_BASE + 101)


# ------------------------------------------------------------------ FP64 mode
@pytest.mark.parametrize("mode", ["dense", "svd"])
def test_fp64_matches_oracle_same_mode(mode):
    x, s = cube()
    want = oracle_phi("cube", 4096, 4, 1e-6, 64, mode)
    got, _ = gpu_apply(x, s, 4, 1e-6, 64, precision="fp64", dense=(mode == "dense"))
    assert rel(got, want) < 1e-10


# ------------------------------------------------------------------ FP32 mode
@pytest.mark.parametrize("p", [4, 6])
def test_fp32_svd_vs_dense_oracle_cube(p):
    x, s = cube()
    want = oracle_phi("cube", 4096, p, 1e-6, 64, "dense")
    got, plan = gpu_apply(x, s, p, 1e-6, 64)
    e = rel(got, want)
    print(f"p={p} k={plan.info()['k']} fp32-svd vs fp64-dense oracle: {e:.3e}")
    assert e < 1e-5


# ------------------------------------------------------------ split-BF16 M2L
# Bound for the split-BF16 M2L: each product drops the lo*lo term and rounds
# the low parts to BF16, a relative error of order 2^-16 ~ 1.5e-5 per product
# entry; the M2L contribution is a fraction of the potential and the errors of
# the 32-term BF16 sums are not aligned, so the matvec stays well inside 2e-5
# (measured 3.4e-6 on this case, 3.3e-7 on the benchmark sphere).
@pytest.mark.parametrize("p", [4, 6])
def test_bf16x3_svd_vs_dense_oracle_cube(p):
    x, s = cube()
    want = oracle_phi("cube", 4096, p, 1e-6, 64, "dense")
    got, plan = gpu_apply(x, s, p, 1e-6, 64, precision="bf16x3")
    info = plan.info()
    assert info["k_pad"] % 32 == 0
    e = rel(got, want)
    print(f"p={p} k={info['k']} bf16x3-svd vs fp64-dense oracle: {e:.3e}")
    assert e < 2e-5


# Every M2L kernel shape that exists for FP32 data, forced: the staged shapes
# (0: 8 waves, 3: 4 waves x 32 rows) and the row-slab shapes (4: 4 waves x 32
# rows, 5: 8 waves x 16 rows), in FP32 (p = 4 and 6; p = 6 takes the trimmed
# last K-chunk, k = 119 <= 120) and split BF16, forward and adjoint, one and
# eight right-hand sides, against the FP64 dense oracle (bars as above).
@pytest.mark.parametrize("shape", [0, 3, 4, 5])
@pytest.mark.parametrize("precision,p,tol", [("fp32", 4, 1e-5), ("fp32", 6, 1e-5), ("bf16x3", 6, 2e-5)])
def test_m2l_shapes_vs_oracle(shape, precision, p, tol):
    torch = _torch()
    K = _k()
    x, s = cube()
    want = oracle_phi("cube", 4096, p, 1e-6, 64, "dense")
    plan = K.Plan(x, p=p, eps=1e-6, leaf_size=64, precision=precision, m2l_shape=shape, max_nrhs=8)
    assert plan.info()["m2l_variant"] == shape
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    fwd = plan.apply(sd).double().cpu().numpy()
    adj = plan.apply_adjoint(sd).double().cpu().numpy()
    S = workloads.uniform_density(4096, 40 + shape, nrhs=7)
    wantS = oracle.fmm(x, S, p, 1e-6, 64, ops=oracle_ops(p, 1e-6, 64, "dense"))[0]
    gotS = plan.apply_batched(torch.tensor(S, dtype=torch.float32, device="cuda:0")).double().cpu().numpy()
    eb = max(max(rel(gotS[:, j], wantS[:, j]), maxrel(gotS[:, j], wantS[:, j])) for j in range(7))
    print(f"shape {shape} {precision} p={p}: forward {rel(fwd, want):.3e} (max {maxrel(fwd, want):.3e}), "
          f"adjoint {rel(adj, want):.3e}, 7 rhs {eb:.3e}")
    assert rel(fwd, want) < tol and maxrel(fwd, want) < tol
    assert rel(adj, want) < tol
    assert eb < tol


def test_m2l_row_slab_shapes_sphere_ragged_and_stage2():
    # many tiles with a ragged tail (tile_targets = 96), and the stage-2 second
    # phase (K = 48) on the row-slab shapes
    torch = _torch()
    K = _k()
    x, s = sphere(20000)
    want = oracle_phi("sphere", 20000, 6, 1e-6, 32, "dense")
    for shape in (4, 5):
        for c2 in (0.0, 10.0):
            plan = K.Plan(x, p=6, eps=1e-6, leaf_size=32, tile_targets=96, m2l_shape=shape, c2=c2)
            got = plan.apply(torch.tensor(s, dtype=torch.float32, device="cuda:0")).double().cpu().numpy()
            e = rel(got, want)
            print(f"sphere 20000 shape {shape} c2={c2}: {e:.3e}")
            assert e < 1e-5 and maxrel(got, want) < 1e-5


def test_fp64_dense_gpu_vs_dense_oracle_cube_p6():
    # The uncompressed operators amplify rounding (pseudo-inverse of the
    # check-to-equivalent systems): only FP64 reaches the oracle's accuracy.
    x, s = cube()
    want = oracle_phi("cube", 4096, 6, 1e-6, 64, "dense")
    got, _ = gpu_apply(x, s, 6, 1e-6, 64, precision="fp64", dense=True)
    # measured 1.5e-9: the two sides' pseudo-inverses (Jacobi vs LAPACK SVD,
    # rcond 1e-10) differ by rounding amplified by the conditioning of the
    # check-to-equivalent systems; 1e-8 leaves a factor of about 6.
    assert rel(got, want) < 1e-8


def test_fp32_dense_gpu_p4_within_operator_rounding():
    # FP32 uncompressed operators: the oracle evaluated with the same operators
    # rounded to FP32 is off by about 3e-4 at p=4 (and 0.45 at p=6), so the
    # dense FP32 path is held to 1e-3 at p=4 only.
    x, s = cube()
    want = oracle_phi("cube", 4096, 4, 1e-6, 64, "dense")
    got, _ = gpu_apply(x, s, 4, 1e-6, 64, dense=True)
    assert rel(got, want) < 1e-3


def test_fp32_sphere_many_tiles_ragged():
    # 20000 points, leaf 32: depth 5, thousands of boxes, M2L tiles with a ragged tail
    x, s = sphere(20000)
    want = oracle_phi("sphere", 20000, 6, 1e-6, 32, "dense")
    got, plan = gpu_apply(x, s, 6, 1e-6, 32, tile_targets=96)
    info = plan.info()
    assert info["depth"] >= 5 and info["n_box"] > 2000
    assert rel(got, want) < 1e-5


def test_full_size_sphere_sampled():
    # 2**20 icosphere centroids, p=6, eps=1e-6, leaf 64 (the benchmark workload),
    # checked at 256 sampled points against the oracle (tests/golden, written
    # by tests/golden/make_sphere_samples.py from the oracle alone).
    g = json.load(open(GOLDEN))
    x, s = sphere(g["n"])
    idx = np.asarray(g["sample"])
    for dense, prec, tol, c2 in ((False, "fp32", 1e-5, 0.0), (False, "bf16x3", 1e-5, 0.0), (True, "fp64", 1e-8, 0.0),
                                 (False, "fp32", 1e-5, 10.0)):
        got, plan = gpu_apply(x, s, g["p"], g["eps"], g["leaf_size"], precision=prec, dense=dense, c2=c2)
        assert plan.info()["depth"] == g["depth"]
        e, m = rel(got[idx], g["phi_dense"]), maxrel(got[idx], g["phi_dense"])
        print(f"dense_m2l={dense} {prec} c2={c2} sampled rel err vs fp64 dense oracle {e:.3e} "
              f"(max {m:.3e}); vs direct {rel(got[idx], g['phi_direct']):.3e}")
        assert e < tol and m < tol


# ------------------------------------------------ stage-2 low rank (Sec. 3.2)
@functools.lru_cache(maxsize=None)
def oracle_phi_svd2(p, c2):
    x, s = cube()
    ops = oracle.build_operators(p, 1e-6, 64, mode="svd2", c2=c2)
    return oracle.fmm(x, s, p, 1e-6, 64, ops=ops)[0]


@pytest.mark.parametrize("p,tol", [(4, 1e-10), (6, 3e-9)])
def test_stage2_fp64_matches_oracle_svd2(p, tol):
    # two thin products per pair (w = V^ q per chunk slot, then U^ w) against
    # the oracle's stage-2 M2L with the same C2 (ranks equal on both sides here).
    # A wrong factor or rank would show at the size of the dropped singular
    # values (eps2 ~ 1e-7 relative); FP64 rounding of the two sides' operators
    # is amplified by the reduced S~ (|S~| ~ 1e5 at p = 6): measured 6.5e-10.
    x, s = cube()
    got, plan = gpu_apply(x, s, p, 1e-6, 64, precision="fp64", c2=10.0)
    want = oracle_phi_svd2(p, 10.0)
    info = plan.info()
    assert 0 < info["m2l_rank_max"] < info["k"]
    assert rel(got, want) < tol


@pytest.mark.parametrize("p", [4, 6])
def test_stage2_fp32_vs_dense_oracle_cube(p):
    x, s = cube()
    want = oracle_phi("cube", 4096, p, 1e-6, 64, "dense")
    got, plan = gpu_apply(x, s, p, 1e-6, 64, c2=10.0)
    e = rel(got, want)
    print(f"p={p} fp32 stage-2 (C2=10, mean rank {plan.info()['m2l_rank_mean']:.1f}) vs dense oracle: {e:.3e}")
    assert e < 1e-5


def test_stage2_adjoint_dot_product_fp64():
    torch = _torch()
    x, s = cube()
    g = workloads.uniform_density(4096, 77)
    plan = _k().Plan(x, p=6, eps=1e-6, leaf_size=64, precision="fp64", c2=10.0)
    sd = torch.tensor(s, dtype=torch.float64, device="cuda:0")
    gd = torch.tensor(g, dtype=torch.float64, device="cuda:0")
    fs = plan.apply(sd).double().cpu().numpy()
    ftg = plan.apply_adjoint(gd).double().cpu().numpy()
    # the stage-2 factors of t and -t are transposes of each other up to rounding
    assert abs(g @ fs - ftg @ s) <= 1e-10 * np.linalg.norm(g) * np.linalg.norm(fs)


def test_stage2_without_far_field():
    # depth < 2 (no interaction fields): the stage-2 plan is the direct sum
    x = workloads.uniform_cube(60, 5)
    s = workloads.uniform_density(60, 6)
    got, plan = gpu_apply(x, s, 4, 1e-6, 64, precision="fp64", c2=10.0)
    assert plan.info()["depth"] < 2
    assert rel(got, oracle.direct(x, s)) < 1e-13


def test_stage2_batched_columns_match_single():
    # 3 right-hand sides through the per-slot product buffer (rows slot*R + r)
    torch = _torch()
    K = _k()
    x, _ = cube()
    S = workloads.uniform_density(4096, 9, nrhs=3)
    plan = K.Plan(x, p=6, eps=1e-6, leaf_size=64, max_nrhs=4, c2=10.0)
    single = K.Plan(x, p=6, eps=1e-6, leaf_size=64, c2=10.0)
    Sd = torch.tensor(S, dtype=torch.float32, device="cuda:0")
    out = plan.apply_batched(Sd).cpu().numpy()
    for j in range(3):
        one = single.apply(Sd[:, j].contiguous()).cpu().numpy()
        assert np.allclose(out[:, j], one, rtol=1e-6, atol=1e-6 * np.abs(one).max())


# ----------------------------------------------------------------- adjoint
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_adjoint_dot_product(precision, tol):
    torch = _torch()
    x, s = cube()
    g = workloads.uniform_density(4096, 77)
    plan = _k().Plan(x, p=4, eps=1e-6, leaf_size=64, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    sd = torch.tensor(s, dtype=dt, device="cuda:0")
    gd = torch.tensor(g, dtype=dt, device="cuda:0")
    fs = plan.apply(sd).double().cpu().numpy()
    ftg = plan.apply_adjoint(gd).double().cpu().numpy()
    lhs, rhs = g @ fs, ftg @ s
    assert abs(lhs - rhs) <= tol * np.linalg.norm(g) * np.linalg.norm(fs)


def test_adjoint_equals_forward_fp64():
    # With the paper's surfaces the FMM operator is symmetric, so the
    # transposed passes must reproduce the forward passes to rounding.
    x, s = cube()
    fwd, _ = gpu_apply(x, s, 6, 1e-6, 64, precision="fp64")
    adj, _ = gpu_apply(x, s, 6, 1e-6, 64, precision="fp64", adjoint=True)
    # measured 3.3e-10: the reduced operators reach |S~| ~ 3e5 while phi is
    # O(1-10), so FP64 rounding is amplified by about 1e5-1e6
    assert rel(adj, fwd) < 1e-8


def test_adjoint_vs_dense_direct_transpose_torus():
    # F^T g against the dense K^T g (= K g, the kernel is symmetric) at N=16384.
    x = workloads.torus_grid_centroids(128, 64)
    g = workloads.uniform_density(x.shape[0], 5)
    want = oracle.direct(x, g)
    got, _ = gpu_apply(x, g, 6, 1e-6, 64, adjoint=True)
    e = rel(got, want)
    print(f"adjoint vs dense K^T g: {e:.3e}")
    assert e < 1e-4


def test_autograd_backward_is_adjoint_and_fd():
    torch = _torch()
    K = _k()
    x = workloads.torus_grid_centroids(64, 32)
    n = x.shape[0]
    plan = K.Plan(x, p=6, eps=1e-6, leaf_size=64, precision="fp64")
    rng = np.random.default_rng(3)
    sig = torch.tensor(rng.uniform(-1, 1, n), dtype=torch.float64, device="cuda:0", requires_grad=True)
    star = torch.tensor(rng.uniform(-1, 1, n), dtype=torch.float64, device="cuda:0")
    b = plan.apply(star)

    def loss_of(s):
        r = K.KifmmMatvec.apply(plan, s) - b
        return 0.5 * (r * r).sum()

    loss = loss_of(sig)
    loss.backward()
    grad = sig.grad.detach()
    want = plan.apply_adjoint(plan.apply(sig.detach()) - b)
    assert torch.allclose(grad, want, rtol=0, atol=0)
    h = 1e-3
    for d in range(4):
        v = torch.tensor(rng.normal(size=n), dtype=torch.float64, device="cuda:0")
        v *= sig.detach().norm() / v.norm()
        with torch.no_grad():
            fd = (loss_of(sig.detach() + h * v) - loss_of(sig.detach() - h * v)) / (2 * h)
        an = (grad * v).sum()
        assert abs(float(fd - an)) <= 1e-8 * abs(float(an)) + 1e-12


# ------------------------------------------------------------------ batching
def test_batched_columns_match_single_applies():
    torch = _torch()
    K = _k()
    x, _ = cube()
    S = workloads.uniform_density(4096, 9, nrhs=3)
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=64, max_nrhs=4)
    single = K.Plan(x, p=4, eps=1e-6, leaf_size=64)
    Sd = torch.tensor(S, dtype=torch.float32, device="cuda:0")
    out = plan.apply_batched(Sd).cpu().numpy()
    for j in range(3):
        one = single.apply(Sd[:, j].contiguous()).cpu().numpy()
        assert np.allclose(out[:, j], one, rtol=1e-6, atol=1e-6 * np.abs(one).max())
        assert rel(out[:, j], oracle.fmm(x, S[:, j], 4, 1e-6, 64, ops=oracle_ops(4, 1e-6, 64, "dense"))[0]) < 1e-5


# Several right-hand sides per launch at every padded width R (2, 4, 8; a
# ragged count below the width) and in every precision, each column against
# the FP64 oracle evaluated on all columns at once: the FP64 plan against the
# oracle's compressed (svd) mode with the same operators (1e-8: operator
# rounding of the two sides, as in the dense FP64 test), FP32 (1e-5) and
# BF16X3 (2e-5) against the dense mode.
@pytest.mark.parametrize("precision,max_nrhs,nrhs,tol", [
    ("fp32", 2, 2, 1e-5), ("fp32", 8, 5, 1e-5), ("fp32", 8, 8, 1e-5),
    ("fp64", 4, 3, 1e-8), ("bf16x3", 8, 6, 2e-5), ("bf16x3", 2, 1, 2e-5)])
def test_batched_widths_and_precisions_vs_oracle(precision, max_nrhs, nrhs, tol):
    torch = _torch()
    K = _k()
    x, _ = cube()
    S = workloads.uniform_density(4096, 31 + nrhs, nrhs=nrhs)
    mode = "svd" if precision == "fp64" else "dense"
    want = oracle.fmm(x, S, 6, 1e-6, 64, ops=oracle_ops(6, 1e-6, 64, mode))[0]
    plan = K.Plan(x, p=6, eps=1e-6, leaf_size=64, precision=precision, max_nrhs=max_nrhs)
    dt = torch.float64 if precision == "fp64" else torch.float32
    got = plan.apply_batched(torch.tensor(S, dtype=dt, device="cuda:0")).double().cpu().numpy()
    errs = [max(rel(got[:, j], want[:, j]), maxrel(got[:, j], want[:, j])) for j in range(nrhs)]
    print(f"{precision} R<={max_nrhs} nrhs={nrhs}: worst column error vs oracle {max(errs):.3e}")
    assert max(errs) < tol


# The split-BF16 adjoint multiplies by the split table of the transposed class
# matrices. Both products carry relative errors of order 2^-16 per entry, so
# the adjoint identity and adjoint = forward (the FMM operator is symmetric)
# hold to that level: bound 2e-5, the BF16X3 bar.
def test_bf16x3_adjoint_identity_and_symmetry():
    torch = _torch()
    x, s = cube()
    g = workloads.uniform_density(4096, 77)
    plan = _k().Plan(x, p=6, eps=1e-6, leaf_size=64, precision="bf16x3")
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    gd = torch.tensor(g, dtype=torch.float32, device="cuda:0")
    fs = plan.apply(sd).double().cpu().numpy()
    ftg = plan.apply_adjoint(gd).double().cpu().numpy()
    fts = plan.apply_adjoint(sd).double().cpu().numpy()
    ident = abs(g @ fs - ftg @ s) / (np.linalg.norm(g) * np.linalg.norm(fs))
    sym = rel(fts, fs)
    want = oracle_phi("cube", 4096, 6, 1e-6, 64, "dense")
    print(f"bf16x3 adjoint: identity {ident:.3e}, adjoint vs forward {sym:.3e}, adjoint vs oracle {rel(fts, want):.3e}")
    assert ident < 2e-5 and sym < 2e-5 and rel(fts, want) < 2e-5


def test_profiled_plan_refuses_capture():
    # profiled applies record timing events that must not be captured: a
    # group holding a profiled plan is refused before any capture begins
    torch = _torch()
    K = _k()
    x, s = cube()
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=64)
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    out = torch.empty_like(sd)
    plan.profile(True)
    grp = K.Group([plan])
    with pytest.raises(K.KifmmError) as err:
        grp.apply([sd], [out])
    assert err.value.code == -5
    plan.profile(False)
    grp.apply([sd], [out])
    torch.cuda.synchronize()
    assert torch.equal(out, plan.apply(sd))


def test_binding_rejects_bad_outputs():
    # outputs are written in place by the kernels: wrong shape, dtype or a
    # strided view is an error, raised before anything is launched
    torch = _torch()
    K = _k()
    x, s = cube()
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=64)
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    for bad, exc in ((torch.empty(4095, device="cuda:0"), ValueError),
                     (torch.empty(4096, dtype=torch.float64, device="cuda:0"), TypeError),
                     (torch.empty(8192, device="cuda:0")[::2], ValueError),
                     (torch.empty(4096), TypeError)):
        with pytest.raises(exc):
            plan.apply(sd, out=bad)
        with pytest.raises(exc):
            plan.apply_adjoint(sd, out=bad)
    with pytest.raises(ValueError):
        plan.apply(sd, out=sd)
    grp = K.Group([plan])
    with pytest.raises(ValueError):
        grp.apply([sd[:100]], [torch.empty_like(sd)])
    with pytest.raises(ValueError):
        grp.apply([sd], [torch.empty(4095, device="cuda:0")])


# ------------------------------------------------------------- edge cases
def test_single_point_and_pair():
    got, _ = gpu_apply(np.array([[0.3, 0.1, -0.2]]), np.array([2.0]), 4, 1e-6, 64, precision="fp64")
    assert got[0] == 0.0
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.0]])
    got, _ = gpu_apply(x, np.array([1.0, -3.0]), 4, 1e-6, 64, precision="fp64")
    f = 1.0 / (4 * math.pi * 0.5)
    assert np.allclose(got, [-3.0 * f, f], rtol=1e-14)


def test_one_leaf_equals_direct_fp32():
    x = workloads.uniform_cube(60, 4)
    s = workloads.uniform_density(60, 5)
    got, plan = gpu_apply(x, s, 4, 1e-6, 64)
    assert plan.info()["depth"] == 0
    assert rel(got, oracle.direct(x, s)) < 1e-6


def test_duplicates_and_clusters():
    # exact duplicates contribute 0 on both sides; two far clusters exercise M2L alone
    a = workloads.uniform_cube(1500, 6) * 0.01
    b = a + np.array([1.0, 1.0, 1.0])
    x = np.concatenate([a, b, a[:200]], axis=0)
    s = workloads.uniform_density(x.shape[0], 7)
    want = oracle.fmm(x, s, 6, 1e-6, 32, ops=oracle_ops(6, 1e-6, 32, "dense"))[0]
    got, _ = gpu_apply(x, s, 6, 1e-6, 32)
    assert rel(got, want) < 1e-5


def test_bitwise_deterministic():
    torch = _torch()
    x, s = sphere(20000)
    plan = _k().Plan(x, p=6, eps=1e-6, leaf_size=32)
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    a = plan.apply(sd).clone()
    b = plan.apply(sd).clone()
    assert torch.equal(a, b)


@pytest.mark.parametrize("c2", [0.0, 10.0])
def test_group_graph_replays_match_eager(c2):
    # c2 > 0: the stage-2 M2L launches (per-slot products, then U^ w) inside the graph
    torch = _torch()
    K = _k()
    sets = [workloads.sphere_points(3000, 1), workloads.cube_surface(5000, 2), workloads.torus_random(7000, 3)]
    plans = [K.Plan(x, p=4, eps=1e-6, leaf_size=32, c2=c2) for x in sets]
    sig = [torch.tensor(workloads.uniform_density(x.shape[0], i), dtype=torch.float32, device="cuda:0")
           for i, x in enumerate(sets)]
    eager = [p.apply(s).clone() for p, s in zip(plans, sig)]
    outs = [torch.empty_like(s) for s in sig]
    grp = K.Group(plans)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        grp.apply(sig, outs)
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            if c2 > 0:
                # stage-2 plans are not merged: each plan's own launches, bitwise
                assert torch.equal(o, e), f"replay {rep}"
            else:
                # merged group: other M2L work tiles, so another summation order
                assert float((o - e).abs().max() / e.abs().max()) < 1e-6, f"replay {rep}"
        _ = [p.apply(s) for p, s in zip(plans, sig)]   # eager work between replays
        torch.cuda.synchronize()


def test_stage_profile_counts():
    torch = _torch()
    x, s = cube()
    plan = _k().Plan(x, p=4, eps=1e-6, leaf_size=64)
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    plan.profile(True)
    for _ in range(3):
        plan.apply(sd)
    ms, calls = plan.profile_read()
    assert calls == 3 and ms["m2l"] > 0 and ms["p2p"] > 0
    plan.profile(False)


@pytest.mark.parametrize("kind", ["sphere", "adaptive", "bem"])
def test_fused_leaf_kernels_match_separate_launches(kind):
    # S2M (check potentials + S~) and L2P (T~ + far field) as one launch each
    # compute the same sums in the same order as the separate launches: the
    # results agree bitwise, forward and adjoint, eager and in a group graph
    torch = _torch()
    K = _k()
    if kind == "bem":
        V, F = workloads.ellipsoid_surface_mesh(5, (2.0, 1.0, 3.0))
        mk = lambda fused: K.Plan.bem(V, F, "single", p=6, eps=1e-6, leaf_size=32, fused_leaf=3 if fused else 0)
        n = F.shape[0]
    else:
        x = sphere(20000)[0] if kind == "sphere" else workloads.clustered_points(1500, 2500, 3)
        mk = lambda fused: K.Plan(x, p=6, eps=1e-6, leaf_size=32, adaptive=(kind == "adaptive"),
                                  fused_leaf=3 if fused else 0)
        n = x.shape[0]
    a, b = mk(True), mk(False)
    s = torch.tensor(workloads.uniform_density(n, 9), dtype=torch.float32, device="cuda:0")
    assert torch.equal(a.apply(s), b.apply(s))
    if kind != "bem":
        assert torch.equal(a.apply_adjoint(s), b.apply_adjoint(s))
    ga, gb = K.Group([a]), K.Group([b])
    oa, ob = torch.empty_like(s), torch.empty_like(s)
    ga.apply([s], [oa])
    gb.apply([s], [ob])
    torch.cuda.synchronize()
    assert torch.equal(oa, ob) and torch.equal(oa, a.apply(s))


@pytest.mark.parametrize("kind", ["sphere", "adaptive", "group"])
def test_direct_passes_match_grouped_gemm(kind):
    # M2M as one product per parent and L2L by octant segments with the
    # operator rows in registers (opts.direct_passes) against the grouped GEMM
    # forms: the same products summed in another order, so the results agree
    # to FP32 rounding, forward and adjoint (L2L^T, M2M^T), on a uniform tree,
    # an adaptive tree (M2M into split cubes only) and a merged group of plans
    # of different depths (rows offset per plan, segments across plans)
    torch = _torch()
    K = _k()
    xs = [sphere(20000)[0]] if kind == "sphere" else [workloads.clustered_points(1500, 2500, 3)]
    if kind == "group":
        xs = [sphere(20000)[0], workloads.uniform_cube(3000, 4), workloads.clustered_points(1500, 2500, 3)]
    mk = lambda x, d: K.Plan(x, p=6, eps=1e-6, leaf_size=32, adaptive=(kind == "adaptive"), direct_passes=d)
    a, b = [mk(x, True) for x in xs], [mk(x, False) for x in xs]
    sig = [torch.tensor(workloads.uniform_density(x.shape[0], 11 + i), dtype=torch.float32, device="cuda:0")
           for i, x in enumerate(xs)]
    mr = lambda u, v: float((u - v).abs().max() / v.abs().max())
    if kind == "group":
        assert len({p.info()["depth"] for p in a}) > 1
        ga, gb = K.Group(a), K.Group(b)
        oa, ob = [torch.empty_like(s) for s in sig], [torch.empty_like(s) for s in sig]
        ga.apply(sig, oa)
        gb.apply(sig, ob)
        torch.cuda.synchronize()
        for u, v in zip(oa, ob):
            assert mr(u, v) < 2e-6
        return
    assert a[0].info()["depth"] >= 4
    assert mr(a[0].apply(sig[0]), b[0].apply(sig[0])) < 2e-6
    assert mr(a[0].apply_adjoint(sig[0]), b[0].apply_adjoint(sig[0])) < 2e-6


@pytest.mark.parametrize("p,eps", [(4, 1e-6), (5, 1e-6), (6, 1e-8)])
def test_direct_passes_other_widths(p, eps):
    # k padded to 64, 96 and 160 (k = 56, 94, 152): one, two and three row
    # blocks per wave in the direct kernels, the last ones partly past k_pad,
    # against the grouped GEMM forms, forward and adjoint
    torch = _torch()
    K = _k()
    x, s = sphere(20000)
    a = K.Plan(x, p=p, eps=eps, leaf_size=32)
    b = K.Plan(x, p=p, eps=eps, leaf_size=32, direct_passes=False)
    assert a.info()["k"] == b.info()["k"]
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    u, v = a.apply(sd), b.apply(sd)
    assert float((u - v).abs().max() / v.abs().max()) < 2e-6, a.info()["k"]
    ua, va = a.apply_adjoint(sd), b.apply_adjoint(sd)
    assert float((ua - va).abs().max() / va.abs().max()) < 2e-6, a.info()["k"]


NEAR_SETS = {
    # name: (points, leaf size); the leaf sizes span every split of a wave's
    # lanes between targets and sources, leaves of more than 64 points (several
    # target blocks per wave) and near lists of more than 64 sources (several
    # staged batches)
    "sphere": (lambda: sphere(20000)[0], 32),
    "cube": (lambda: workloads.uniform_cube(30000, workloads.SEED_BASE + 7), 100),
    "clustered": (lambda: workloads.clustered_points(3000, 5000, workloads.SEED_BASE + 8), 8),
}


@pytest.mark.parametrize("name", list(NEAR_SETS))
def test_near_field_overlap_is_bitwise_the_same(name):
    # the near field with register-staged sources forked just before M2L
    # (opts.near_overlap, the default) against the LDS-staged one forked after
    # the permute: the same sums in the same order, so the matvec, its adjoint
    # and the no-allocation apply agree bit for bit
    torch = _torch()
    K = _k()
    gen, leaf = NEAR_SETS[name]
    x = gen()
    s = workloads.uniform_density(x.shape[0], workloads.SEED_BASE + 9) if name != "sphere" else sphere(20000)[1]
    a = K.Plan(x, p=6, eps=1e-6, leaf_size=leaf)
    b = K.Plan(x, p=6, eps=1e-6, leaf_size=leaf, near_overlap=False)
    sd = torch.tensor(s, dtype=torch.float32, device="cuda:0")
    fa = a.apply(sd).clone()
    assert torch.equal(fa, b.apply(sd))
    assert torch.equal(a.apply_adjoint(sd), b.apply_adjoint(sd))
    o = torch.full_like(sd, float("nan"))
    a.apply_noalloc(sd, o)
    torch.cuda.synchronize()
    assert torch.equal(o, fa)
    if name == "sphere":
        want = oracle_phi("sphere", 20000, 6, 1e-6, 32, "dense")
        assert rel(fa.double().cpu().numpy(), want) < 1e-5
