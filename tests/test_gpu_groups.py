"""Merged groups: plans with equal operators run as one merged plan (every
stage one launch over all their cubes). Their results must equal each plan's
own apply up to the summation order of M2L (FP64: 1e-12 relative; FP32:
1e-6 of the largest value), for uniform and adaptive members together, a
member without far field (one leaf) and a member whose tree is deeper than
the rest; replays of the captured graph must agree with each other bitwise."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _k():
    import paper_1211_2517_amd as K
    return K


def _members(K, precision, **kw):
    sets = [
        (workloads.sphere_points(3000, 1), {}),
        (workloads.cube_surface(5000, 2), {"adaptive": True}),
        (workloads.torus_random(7000, 3), {}),
        (workloads.clustered_points(1500, 2500, 3), {"adaptive": True}),
        (workloads.uniform_cube(40, 4), {}),                 # one leaf: no far field
        (workloads.corner_clusters(3000, 20, 7), {"adaptive": True}),
    ]
    plans = [K.Plan(x, p=4, eps=1e-6, leaf_size=32, precision=precision, **o, **kw) for x, o in sets]
    return [x for x, _ in sets], plans


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_merged_group_matches_member_applies(precision, tol):
    import torch
    K = _k()
    sets, plans = _members(K, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    sig = [torch.tensor(workloads.uniform_density(x.shape[0], 50 + i), dtype=dt, device="cuda:0")
           for i, x in enumerate(sets)]
    eager = [p.apply(s).clone() for p, s in zip(plans, sig)]
    outs = [torch.full_like(s, float("nan")) for s in sig]
    grp = K.Group(plans)
    first = None
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        grp.apply(sig, outs)
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            err = float((o - e).abs().max() / e.abs().max())
            assert err < tol, (rep, i, err)
        if first is None:
            first = [o.clone() for o in outs]
        else:
            assert all(torch.equal(a, b) for a, b in zip(first, outs)), rep
        _ = [p.apply(s) for p, s in zip(plans, sig)]
        torch.cuda.synchronize()
    grp.close()


def test_merged_group_new_pointers_and_widths():
    # members with max_nrhs 4 (right-hand-side width 4) merge too; new output
    # pointers re-capture the graph
    import torch
    K = _k()
    sets, plans = _members(K, "fp32", max_nrhs=4)
    sig = [torch.tensor(workloads.uniform_density(x.shape[0], 70 + i), dtype=torch.float32, device="cuda:0")
           for i, x in enumerate(sets)]
    eager = [p.apply(s).clone() for p, s in zip(plans, sig)]
    grp = K.Group(plans)
    for _ in range(2):
        outs = [torch.full_like(s, float("nan")) for s in sig]
        grp.apply(sig, outs)
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert float((o - e).abs().max() / e.abs().max()) < 1e-6
    grp.close()
