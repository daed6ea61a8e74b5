"""Parity of the adaptive-tree HIP path (opts.adaptive) with the adaptive oracle.

The oracle (oracle/adaptive.py) evaluates the KIFMM on the adaptive tree in
FP64 with U/V/W/X lists built from their definitions; the library builds the
same tree and lists in C++ and runs S2M/M2M/M2L/L2L/L2T plus M2T (W) and S2L
(X) in its kernels. Tolerances as for the uniform tree: FP64 against the
oracle in the same operator mode 1e-10 (p = 4) and 1e-8 (p = 6); FP32 and
BF16X3 against the FP64 dense oracle 1e-5 (relative L2 and max-relative).
At 2^20 points (the 2:1:0.5 ellipsoid of the precision workload, p = 8,
eps = 1e-8) the oracle's direct sum and dense-M2L potentials at 256 sampled
points (tests/golden/p8_samples.json) bound the result.
"""
import functools
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle.adaptive import build_adaptive_tree, fmm_adaptive

pytestmark = pytest.mark.gpu

P8 = os.path.join(os.path.dirname(__file__), "golden", "p8_samples.json")


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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


SETS = {
    # name: (points, leaf size)
    "clustered": (lambda: workloads.clustered_points(1500, 2500, 3), 24),
    "ellipsoid": (lambda: workloads.ellipsoid_points(6000, 5), 32),
    "corner": (lambda: workloads.corner_clusters(3000, 20, 7), 32),
}


@functools.lru_cache(maxsize=None)
def case(name):
    gen, leaf = SETS[name]
    x = gen()
    s = workloads.uniform_density(x.shape[0], 77)
    return x, s, leaf


@functools.lru_cache(maxsize=None)
def oracle_ops(p, eps, leaf, mode, c2=0.0):
    if mode == "svd2":
        return oracle.build_operators(p, eps, leaf, mode=mode, c2=c2)
    return oracle.build_operators(p, eps, leaf, mode=mode)


@functools.lru_cache(maxsize=None)
def oracle_phi(name, p, eps, mode, c2=0.0):
    x, s, leaf = case(name)
    return fmm_adaptive(x, s, oracle_ops(p, eps, leaf, mode, c2), build_adaptive_tree(x, leaf))


def gpu(name, p, eps, precision="fp32", dense=False, adjoint=False, s=None, **kw):
    torch = _torch()
    x, s0, leaf = case(name)
    s = s0 if s is None else s
    plan = _k().Plan(x, p=p, eps=eps, leaf_size=leaf, precision=precision, dense_m2l=dense, adaptive=True, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    sd = torch.tensor(np.asarray(s), dtype=dt, device="cuda:0")
    out = plan.apply_adjoint(sd) if adjoint else plan.apply(sd)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), plan


@pytest.mark.parametrize("name,p,tol", [("clustered", 4, 1e-10), ("clustered", 6, 1e-8), ("ellipsoid", 6, 1e-8),
                                        ("corner", 4, 1e-10)])
@pytest.mark.parametrize("mode", ["svd", "dense"])
def test_fp64_matches_adaptive_oracle(name, p, tol, mode):
    want = oracle_phi(name, p, 1e-6, mode)
    got, plan = gpu(name, p, 1e-6, precision="fp64", dense=(mode == "dense"))
    info = plan.info()
    assert info["adaptive"] == 1 and info["w_pairs"] > 0
    e, m = rel(got, want), maxrel(got, want)
    print(f"{name} p={p} {mode} fp64: rel {e:.3e} max {m:.3e}; levels {info['leaf_level_min']}..{info['depth']}")
    assert e < tol and m < 10 * tol


@pytest.mark.parametrize("name", ["clustered", "ellipsoid", "corner"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_fp32_vs_dense_adaptive_oracle(name, precision):
    want = oracle_phi(name, 6, 1e-6, "dense")
    got, _ = gpu(name, 6, 1e-6, precision=precision)
    e, m = rel(got, want), maxrel(got, want)
    print(f"{name} p=6 {precision}: rel {e:.3e} max {m:.3e}")
    assert e < 1e-5 and m < 1e-5


def test_stage2_fp64_matches_oracle():
    want = oracle_phi("clustered", 6, 1e-6, "svd2", 10.0)
    got, plan = gpu("clustered", 6, 1e-6, precision="fp64", c2=10.0)
    assert plan.info()["m2l_rank_max"] > 0
    assert rel(got, want) < 3e-9


def test_adjoint_identity_and_symmetry_fp64():
    # <F x, y> = <x, F^T y>; the adaptive operator is symmetric as the uniform
    # one (M2T and S2L are each other's transposes)
    x, s, leaf = case("clustered")
    y = workloads.uniform_density(x.shape[0], 78)
    fx, _ = gpu("clustered", 4, 1e-6, precision="fp64")
    fty, _ = gpu("clustered", 4, 1e-6, precision="fp64", adjoint=True, s=y)
    fy, _ = gpu("clustered", 4, 1e-6, precision="fp64", s=y)
    a, b = float(fx @ y), float(s @ fty)
    assert abs(a - b) < 1e-12 * abs(a) * 10
    assert rel(fty, fy) < 1e-10


def test_batched_columns_match_single():
    torch = _torch()
    x, s, leaf = case("clustered")
    K = _k()
    S = np.stack([workloads.uniform_density(x.shape[0], 80 + r) for r in range(3)], axis=1)
    plan = K.Plan(x, p=4, eps=1e-6, leaf_size=leaf, adaptive=True, max_nrhs=4)
    single = K.Plan(x, p=4, eps=1e-6, leaf_size=leaf, adaptive=True)
    st = torch.tensor(S, dtype=torch.float32, device="cuda:0")
    got = plan.apply_batched(st).double().cpu().numpy()
    for r in range(3):
        one = single.apply(st[:, r].contiguous()).double().cpu().numpy()
        assert maxrel(got[:, r], one) < 1e-6, r
    want = np.stack([oracle_phi_cols(r) for r in range(3)], axis=1)
    assert rel(got, want) < 1e-5


@functools.lru_cache(maxsize=None)
def oracle_phi_cols(r):
    x, _, leaf = case("clustered")
    s = workloads.uniform_density(x.shape[0], 80 + r)
    return fmm_adaptive(x, s, oracle_ops(4, 1e-6, leaf, "dense"), build_adaptive_tree(x, leaf))


def test_group_graph_and_noalloc_match_eager():
    torch = _torch()
    K = _k()
    plans, sig = [], []
    for i, name in enumerate(["clustered", "corner", "ellipsoid"]):
        x, s, leaf = case(name)
        plans.append(K.Plan(x, p=4, eps=1e-6, leaf_size=leaf, adaptive=True))
        sig.append(torch.tensor(s, dtype=torch.float32, device="cuda:0"))
    eager = [p.apply(s).clone() for p, s in zip(plans, sig)]
    outs = [torch.empty_like(s) for s in sig]
    grp = K.Group(plans)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        grp.apply(sig, outs)
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            # the captured apply evaluates near and far fields in one kernel:
            # the same sums in another grouping
            assert float((o - e).abs().max() / e.abs().max()) < 1e-6, f"replay {rep}"
        _ = [p.apply(s) for p, s in zip(plans, sig)]
        torch.cuda.synchronize()
    for p, s, e in zip(plans, sig, eager):
        o = torch.full_like(s, float("nan"))
        p.apply_noalloc(s, o)
        torch.cuda.synchronize()
        assert torch.equal(o, e)


def test_equals_uniform_when_leaves_share_a_level():
    # a jittered grid whose adaptive leaves all sit at level 3: no W/X lists,
    # the same tree, and the uniform plan's result
    torch = _torch()
    K = _k()
    rng = np.random.default_rng(8)
    m = 16
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5
         + 0.3 * rng.uniform(-1, 1, (m ** 3, 3))) / m
    x = np.concatenate([g, [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]])
    s = workloads.uniform_density(x.shape[0], 9)
    pa = K.Plan(x, p=4, eps=1e-6, leaf_size=9, adaptive=True, precision="fp64")
    pu = K.Plan(x, p=4, eps=1e-6, leaf_size=9, precision="fp64")
    assert pa.info()["w_pairs"] == 0 and pa.info()["leaf_level_min"] == 3 == pu.info()["depth"]
    sd = torch.tensor(s, dtype=torch.float64, device="cuda:0")
    assert rel(pa.apply(sd).cpu().numpy(), pu.apply(sd).cpu().numpy()) < 1e-13


def test_full_size_ellipsoid_sampled():
    # 2^20-point 2:1:0.5 ellipsoid, p = 8, eps = 1e-8, leaf 64: the adaptive
    # plan against the oracle's direct sum and uniform dense-M2L KIFMM at 256
    # sampled points
    g = json.load(open(P8))
    x = workloads.ellipsoid_points(g["n"], g["seed"])
    s = workloads.sphere_density(x, g["seed"] + 100)
    e = g["ellipsoid"]
    idx = np.asarray(e["sample"])
    torch = _torch()
    K = _k()
    for prec, tol in (("fp64", 1e-7), ("fp32", 1e-5)):
        plan = K.Plan(x, p=g["p"], eps=g["eps"], leaf_size=g["leaf_size"], precision=prec, adaptive=True)
        dt = torch.float64 if prec == "fp64" else torch.float32
        got = plan.apply(torch.tensor(s, dtype=dt, device="cuda:0")).double().cpu().numpy()[idx]
        info = plan.info()
        ed, ek = rel(got, e["phi_direct"]), rel(got, e["phi_dense"])
        print(f"ellipsoid 2^20 adaptive {prec}: vs direct {ed:.3e}, vs uniform dense {ek:.3e}; leaves "
              f"{info['n_leaf']} levels {info['leaf_level_min']}..{info['depth']} W pairs {info['w_pairs']}")
        assert ed < tol and ek < tol and maxrel(got, e["phi_direct"]) < 10 * tol
        del plan
