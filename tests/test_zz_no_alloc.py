"""kifmm_apply_noalloc through the C ABI against kifmm_apply."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_noalloc_matches_apply_two_calls_then_smaller():
    # two calls in a row on one plan, then a plan with fewer points (the
    # static workspace keeps the previous call's contents): each output is
    # bitwise equal to kifmm_apply's (same kernels, same order) and within
    # the FP32 bar of it
    import torch
    import paper_1211_2517_amd as K
    big = K.Plan(workloads.uniform_cube(4096, 21), p=6, eps=1e-6, leaf_size=64)
    small = K.Plan(workloads.sphere_points(2500, 22), p=4, eps=1e-6, leaf_size=32)
    for plan, seeds in ((big, (1, 2)), (small, (3,))):
        for sd in seeds:
            s = torch.tensor(workloads.uniform_density(plan.n, sd), dtype=torch.float32, device="cuda:0")
            ref = plan.apply(s).clone()
            out = torch.full_like(s, float("nan"))
            plan.apply_noalloc(s, out)
            torch.cuda.synchronize()
            e = float((out.double() - ref.double()).norm() / ref.double().norm())
            print(f"noalloc N={plan.n} seed {sd}: bitwise equal {torch.equal(out, ref)}, rel diff {e:.3e}")
            assert torch.equal(out, ref)


def test_noalloc_refuses_oversized_and_stage2_plans():
    import torch
    import paper_1211_2517_amd as K
    x = workloads.sphere_points(40000, 23)
    wide = K.Plan(x, p=6, eps=1e-6, leaf_size=64, max_nrhs=16)   # workspace of 16 right-hand sides
    s = torch.ones(x.shape[0], dtype=torch.float32, device="cuda:0")
    out = torch.empty_like(s)
    with pytest.raises(K.KifmmError) as err:
        wide.apply_noalloc(s, out)
    assert err.value.code == -1
    st2 = K.Plan(x, p=6, eps=1e-6, leaf_size=64, c2=10.0)
    with pytest.raises(K.KifmmError) as err:
        st2.apply_noalloc(s, out)
    assert err.value.code == -1
