"""GPU tests at the sizes of the precision, batching and differentiation
workloads (2**20-point sphere and ellipsoid at p = 8; 24 independent surfaces
plus 16 right-hand sides; a 262,144-point torus), through the C-ABI.

Every expected value comes from the oracle: stored samples written by
tests/golden/make_p8_samples.py and tests/golden/make_batch_samples.py, or
oracle calls made here."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


# ------------------------------------------------------ p = 8 precision modes
# Error of each device precision against the FP64 dense-M2L oracle at 256
# sampled points (eps = 1e-8). Bounds: FP64 - the stage-1 truncation at eps =
# 1e-8 (the SVD oracle and the dense oracle differ by O(eps)); FP32 - the 1e-5
# bar of the FP32 mode; BF16X3 - the split-BF16 M2L's stated bound 1e-4
# (products accurate to O(2^-16)).
@pytest.mark.parametrize("shape", ["sphere", "ellipsoid"])
def test_p8_precision_modes_vs_oracle(shape):
    torch = _torch()
    K = _k()
    g = json.load(open(os.path.join(HERE, "golden", "p8_samples.json")))
    gen = workloads.sphere_points if shape == "sphere" else workloads.ellipsoid_points
    x = gen(g["n"], g["seed"])
    sig = workloads.sphere_density(x, g["seed"] + 100)
    gs = g[shape]
    idx = np.asarray(gs["sample"])
    want = np.asarray(gs["phi_dense"])
    for prec, tol in (("fp64", 1e-7), ("fp32", 1e-5), ("bf16x3", 1e-4)):
        dt = torch.float64 if prec == "fp64" else torch.float32
        plan = K.Plan(x, p=g["p"], eps=g["eps"], leaf_size=g["leaf_size"], precision=prec)
        assert plan.info()["depth"] == gs["depth"]
        sd = torch.tensor(sig, dtype=dt, device="cuda:0")
        got = plan.apply(sd).double().cpu().numpy()[idx]
        e = rel(got, want)
        print(f"{shape} p=8 eps=1e-8 {prec}: k={plan.info()['k']} rel err vs fp64 dense oracle {e:.3e}, "
              f"vs direct sum {rel(got, gs['phi_direct']):.3e}")
        plan.close()
        assert e < tol


def test_p8_stage2_products_beyond_2gib():
    # stage 2 (C2 = 10) at the p=8, eps=1e-8 configuration on the 2^20-point
    # sphere: k = 234 and ranks up to 84 (padded to 96) make 2.25 GB of
    # per-pair products in FP32, past the 32-bit offsets of one launch, so the
    # second phase runs as two launches over tile ranges. Forward against the
    # dense oracle at the sampled points to the FP32 bar, and the adjoint
    # (the same ranges over the transposed factors) against the forward: the
    # operator is symmetric
    torch = _torch()
    K = _k()
    g = json.load(open(os.path.join(HERE, "golden", "p8_samples.json")))
    x = workloads.sphere_points(g["n"], g["seed"])
    sig = workloads.sphere_density(x, g["seed"] + 100)
    gs = g["sphere"]
    idx = np.asarray(gs["sample"])
    plan = K.Plan(x, p=g["p"], eps=g["eps"], leaf_size=g["leaf_size"], precision="fp32", c2=10.0)
    info = plan.info()
    assert info["k"] == 234 and info["m2l_rank_max"] > 80
    sd = torch.tensor(sig, dtype=torch.float32, device="cuda:0")
    fwd = plan.apply(sd).double().cpu().numpy()
    adj = plan.apply_adjoint(sd).double().cpu().numpy()
    plan.close()
    e = rel(fwd[idx], np.asarray(gs["phi_dense"]))
    print(f"sphere p=8 eps=1e-8 fp32 stage 2 (ranks <= {info['m2l_rank_max']}): rel err vs dense oracle {e:.3e}, "
          f"adjoint vs forward {rel(adj, fwd):.3e}")
    assert e < 1e-5
    assert rel(adj, fwd) < 1e-5


# ----------------------------------------------------------------- batching
def maxrel(a, b):
    """max |a - b| / max |b|: a wrong value at one point is not diluted by the
    number of points, unlike the relative L2 error."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


# Every set and every right-hand side against the FP64 dense-M2L oracle at its
# sampled points (tests/golden/batch_samples.json, written by
# tests/golden/make_batch_samples.py from the oracle alone): the FP32 bar 1e-5
# for the relative L2 error and for the largest error relative to the largest
# potential (FP32 rounding and the eps = 1e-6 truncation are spread over all
# points; a wrong leaf or column shows at O(1e-2) or more).
def test_24_surfaces_one_graph_and_16_rhs():
    torch = _torch()
    K = _k()
    g = json.load(open(os.path.join(HERE, "golden", "batch_samples.json")))
    sets = workloads.batch_sets(24)
    assert len(sets) == g["count"]
    big = g["big"]
    plans, sig, eager = [], [], []
    for i, (x, _) in enumerate(sets):
        plans.append(K.Plan(x, p=g["p"], eps=g["eps"], leaf_size=g["leaf_size"]))
        sig.append(torch.tensor(workloads.uniform_density(x.shape[0], 100 + i), dtype=torch.float32,
                                device="cuda:0"))
    for p, s in zip(plans, sig):
        eager.append(p.apply(s).clone())
    torch.cuda.synchronize()
    grp = K.Group(plans)
    outs = [torch.empty_like(s) for s in sig]
    # the 24 plans share their operators, so the group is merged: every stage
    # one launch over all of them; equal to the plans' own applies up to the
    # summation order of M2L, and replays agree bitwise
    first = None
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        grp.apply(sig, outs)
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            assert float((o - e).abs().max() / e.abs().max()) < 1e-6, f"replay {rep}, set {i}"
        if first is None:
            first = [o.clone() for o in outs]
        else:
            assert all(torch.equal(a, b) for a, b in zip(first, outs)), f"replay {rep}"
    worst = 0.0
    for i, (x, name) in enumerate(sets):
        gs = g["sets"][i]
        assert gs["n"] == x.shape[0] and gs["name"] == name
        assert plans[i].info()["depth"] == gs["depth"]
        idx = np.asarray(gs["sample"])
        got = outs[i].double().cpu().numpy()[idx]
        e, m = rel(got, gs["phi_dense"]), maxrel(got, gs["phi_dense"])
        worst = max(worst, e)
        print(f"set {i} ({name}, N={x.shape[0]}): rel L2 {e:.3e}, max {m:.3e} vs fp64 dense oracle")
        assert e < 1e-5 and m < 1e-5, f"set {i}"
    print(f"24 sets in one merged group: worst rel L2 vs oracle {worst:.3e}")
    # 16 right-hand sides on the largest set, each column against the oracle
    xb = sets[big][0]
    gb = g["sets"][big]
    idx = np.asarray(gb["sample"])
    want = np.asarray(gb["phi_rhs"])
    assert want.shape == (idx.size, g["nrhs"])
    S = torch.tensor(workloads.uniform_density(xb.shape[0], 7, nrhs=16), dtype=torch.float32, device="cuda:0")
    plan16 = K.Plan(xb, p=g["p"], eps=g["eps"], leaf_size=g["leaf_size"], max_nrhs=16)
    outb = plan16.apply_batched(S).double().cpu().numpy()[idx]
    worst = max(max(rel(outb[:, j], want[:, j]), maxrel(outb[:, j], want[:, j])) for j in range(16))
    print(f"largest set N={xb.shape[0]}: 16 right-hand sides vs oracle, worst column error {worst:.3e}")
    assert worst < 1e-5


# ---------------------------------------------------------- differentiation
# loss(s) = 0.5 |F s - b|^2 on the 262,144-point torus (b = F s* for a random
# s*, loss summed in FP64); its gradient F^T (F s - b) through the autograd
# function against central differences (h = 1e-3) along 64 random directions
# v scaled to |v| = |s|. The loss is quadratic, so the difference quotient has
# no truncation error; what remains is the rounding of the two loss values.
#  - FP64 plans: rounding ~1e-16 of |F s|, so |fd - grad.v| / |grad.v| stays
#    below ~1e-10 even where grad.v is small: bound 1e-8.
#  - FP32 plans: the two evaluations of F carry rounding errors of ~1e-7
#    |F s|, which enter the difference divided by 2h; against the scale
#    |grad| |v| of a directional derivative that is at most ~1e-4 (grad.v
#    itself can be far smaller than that scale for a random v, where the plain
#    relative error reaches 1e-2, so the quotient is normalised by
#    |grad| |v|): bound 1e-5, measured 4.9e-7. The sharp FP32 check is the
#    adjoint identity <g, F s> = <F^T g, s> to rounding (bound 2e-6 of
#    |g| |F s|, measured 7e-10).
def _torus_plan_and_data(precision):
    torch = _torch()
    K = _k()
    x = workloads.torus_grid_centroids(512, 256)
    n = x.shape[0]
    assert n == 262144
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = K.Plan(x, p=6, eps=1e-6, leaf_size=64, precision=precision)
    rng = np.random.default_rng(11)
    star = torch.tensor(rng.uniform(-1, 1, n), dtype=dt, device="cuda:0")
    b = plan.apply(star).double()
    s0 = torch.tensor(rng.uniform(-1, 1, n), dtype=dt, device="cuda:0", requires_grad=True)
    return K, plan, b, s0, rng, dt


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_fd_gradient_full_size(precision):
    torch = _torch()
    K, plan, b, s0, rng, dt = _torus_plan_and_data(precision)
    n = s0.shape[0]

    def loss_of(s):
        r = K.KifmmMatvec.apply(plan, s).double() - b
        return 0.5 * (r * r).sum()

    loss = loss_of(s0)
    loss.backward()
    grad = s0.grad.detach().double()
    h = 1e-3
    worst_raw = worst_norm = 0.0
    for d in range(64):
        v = torch.tensor(rng.normal(size=n), dtype=torch.float64, device="cuda:0")
        v *= s0.detach().double().norm() / v.norm()
        with torch.no_grad():
            lp = loss_of((s0.detach().double() + h * v).to(dt))
            lm = loss_of((s0.detach().double() - h * v).to(dt))
        fd = float((lp - lm) / (2 * h))
        an = float((grad * v).sum())
        worst_raw = max(worst_raw, abs(fd - an) / abs(an))
        worst_norm = max(worst_norm, abs(fd - an) / float(grad.norm() * v.norm()))
    print(f"torus N={n} {precision}: 64 directions, max |fd - grad.v| / |grad.v| = {worst_raw:.3e}, "
          f"max |fd - grad.v| / (|grad| |v|) = {worst_norm:.3e}")
    if precision == "fp64":
        assert worst_raw < 1e-8
    else:
        assert worst_norm < 1e-5
        g = torch.tensor(rng.uniform(-1, 1, n), dtype=dt, device="cuda:0")
        s = s0.detach()
        fs = plan.apply(s).double()
        ftg = plan.apply_adjoint(g).double()
        lhs = float((g.double() * fs).sum())
        rhs = float((ftg * s.double()).sum())
        e = abs(lhs - rhs) / float(g.double().norm() * fs.norm())
        print(f"torus N={n} fp32: adjoint identity |<g,Fs> - <F^T g,s>| / (|g||Fs|) = {e:.3e}")
        assert e < 2e-6
