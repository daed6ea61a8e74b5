"""Host-side checks of the C-ABI library (CPU only, no device calls).

The library is loaded and every symbol declared in include/kifmm.h must be
exported. Host-only plans (opts.device = -1) build the tree, lists and FP64
operators without touching a GPU; they are compared with the oracle, which
computes the same quantities independently.
"""
import ctypes
import functools
import os
import re

import numpy as np
import pytest

import oracle
import workloads
import paper_1211_2517_amd as K

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "kifmm.h")


def test_library_exports_every_declared_symbol():
    lib = K.load_library()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(kifmm_[a-z_]+)\s*\(", text))
    assert declared, "no declarations parsed"
    assert declared == set(K.EXPORTED_SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


@functools.lru_cache(maxsize=None)
def _host_plan(kind, n, p, eps, leaf, dense=False):
    x = {"cube": workloads.uniform_cube, "sphere": workloads.sphere_points}[kind](n, 1211)
    return x, K.Plan(x, p=p, eps=eps, leaf_size=leaf, device=-1, dense_m2l=dense)


@functools.lru_cache(maxsize=None)
def _oracle_ops(p, eps, leaf, mode):
    return oracle.build_operators(p, eps, leaf, mode=mode)


@pytest.mark.parametrize("kind,n,leaf", [("cube", 4096, 64), ("sphere", 20000, 32), ("cube", 50, 64)])
def test_tree_identical_to_oracle(kind, n, leaf):
    x, pl = _host_plan(kind, n, 4, 1e-6, leaf)
    tr = oracle.build_tree(x, leaf)
    info = pl.info()
    assert info["depth"] == tr.depth
    lc = pl.export_tree()
    want = np.array(tr.leaf_of_point, dtype=np.int64).reshape(-1, 3)
    assert np.array_equal(lc.astype(np.int64), want)
    assert info["n_leaf"] == len(tr.leaf_points)
    assert info["boxes_level"] == [len(tr.boxes[l]) for l in range(tr.depth + 1)]
    vl = [sum(len(tr.interaction(l, b)) for b in tr.boxes[l]) if l >= 2 else 0 for l in range(tr.depth + 1)]
    assert info["v_pairs_level"] == vl
    near = sum(len(tr.near(tr.depth, b)) for b in tr.boxes[tr.depth])
    assert info["near_pairs"] == near


@pytest.mark.parametrize("p,eps", [(4, 1e-6), (6, 1e-6), (6, 1e-4)])
def test_svd_operators_match_oracle(p, eps):
    _, pl = _host_plan("cube", 4096, p, eps, 64)
    ops = _oracle_ops(p, eps, 64, "svd")
    k = ops.k
    assert pl.info()["k"] == k
    s = pl.export_operator(0)
    assert np.allclose(s[:k], ops.sing[:k], rtol=1e-9, atol=0)
    U = pl.export_operator(1).reshape(ops.n_eq, k)
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-12)
    # singular vectors are unique up to sign: compare sign-free products
    assert np.abs(U @ U.T - ops.U @ ops.U.T).max() < 1e-9
    Kl = pl.export_operator(6).reshape(316, k, k)
    scale = max(np.abs(v).max() for v in ops.K_full.values())
    for i, t in enumerate(oracle.offset_classes()):
        assert np.abs(U @ Kl[i] @ U.T - ops.U @ ops.K[t] @ ops.U.T).max() < 1e-9 * scale
    S = pl.export_operator(2).reshape(k, ops.n_eq)
    T = pl.export_operator(3).reshape(ops.n_eq, k)
    ref = np.abs(ops.U @ ops.S).max()
    assert np.abs(U @ S - ops.U @ ops.S).max() < 1e-7 * ref
    assert np.abs(T @ U.T - ops.T @ ops.U.T).max() < 1e-7 * ref
    M = pl.export_operator(4).reshape(8, k, k)
    L = pl.export_operator(5).reshape(8, k, k)
    for o in range(8):
        sign = tuple(2.0 * ((o >> s) & 1) - 1.0 for s in (2, 1, 0))
        assert np.abs(U @ M[o] @ U.T - ops.U @ ops.M[sign] @ ops.U.T).max() < 1e-8
        assert np.abs(U @ L[o] @ U.T - ops.U @ ops.L[sign] @ ops.U.T).max() < 1e-8


def test_dense_operators_match_oracle():
    _, pl = _host_plan("cube", 4096, 4, 1e-6, 64, dense=True)
    ops = _oracle_ops(4, 1e-6, 64, "dense")
    n = ops.n_eq
    assert pl.info()["k"] == n
    Kl = pl.export_operator(6).reshape(316, n, n)
    for i, t in enumerate(oracle.offset_classes()):
        assert np.allclose(Kl[i], ops.K[t], rtol=1e-13, atol=1e-16)
    S = pl.export_operator(2).reshape(n, n)
    assert np.abs(S - ops.S).max() < 1e-8 * np.abs(ops.S).max()


def test_single_leaf_depth_zero():
    x, pl = _host_plan("cube", 50, 4, 1e-6, 64)
    info = pl.info()
    assert info["depth"] == 0 and info["n_leaf"] == 1 and info["v_pairs"] == 0


def _err(fn):
    with pytest.raises(K.KifmmError) as e:
        fn()
    return e.value.code


def test_invalid_arguments_are_rejected():
    x = workloads.uniform_cube(100, 1)
    assert _err(lambda: K.Plan(x, p=1, device=-1)) == -1
    assert _err(lambda: K.Plan(x, p=6, eps=1.0, device=-1)) == -1
    assert _err(lambda: K.Plan(x, p=6, eps=-1e-3, device=-1)) == -1
    assert _err(lambda: K.Plan(x, leaf_size=0, device=-1)) == -1
    assert _err(lambda: K.Plan(x[:0], device=-1)) == -1
    bad = x.copy()
    bad[17, 1] = np.nan
    assert _err(lambda: K.Plan(bad, device=-1)) == -4
    bad[17, 1] = np.inf
    assert _err(lambda: K.Plan(bad, device=-1)) == -4
    assert _err(lambda: K.Plan(x, max_nrhs=17, device=-1)) == -1
    assert _err(lambda: K.Plan(x, p=9, device=-1)) == -1     # n_eq 386 beyond the device kernels


def test_flag_options_out_of_range_are_rejected():
    # through the C ABI directly (the binding passes these as booleans):
    # fused_leaf outside [0, 3], direct_passes or near_overlap outside {0, 1}
    import ctypes
    lib = K.load_library()
    x = np.ascontiguousarray(workloads.uniform_cube(100, 1))
    for field, value in (("fused_leaf", 4), ("fused_leaf", -1), ("direct_passes", 2), ("near_overlap", 2),
                         ("near_overlap", -1)):
        o = K._Opts()
        lib.kifmm_opts_default(ctypes.byref(o))
        o.device = -1
        setattr(o, field, value)
        h = ctypes.c_void_p()
        rc = lib.kifmm_plan_ex(x.ctypes.data, x.shape[0], 4, 1e-6, 16, ctypes.byref(o), ctypes.byref(h))
        assert rc == -1 and not h.value, (field, value, rc)
    o = K._Opts()
    lib.kifmm_opts_default(ctypes.byref(o))
    assert (o.fused_leaf, o.direct_passes, o.near_overlap) == (3, 1, 1)


def test_host_only_plan_refuses_apply():
    lib = K.load_library()
    _, pl = _host_plan("cube", 4096, 4, 1e-6, 64)
    rc = lib.kifmm_apply(pl._h, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert rc == -5
    assert b"host-only" in lib.kifmm_last_error()
    lib.kifmm_destroy(None)       # NULL-safe
    lib.kifmm_group_destroy(None)


def test_duplicate_points_cap_depth():
    x = np.repeat(workloads.uniform_cube(10, 2), 20, axis=0)   # 20 copies of 10 points
    pl = K.Plan(x, p=4, eps=1e-6, leaf_size=8, device=-1, max_depth=6)
    assert pl.info()["depth"] == 6


@pytest.mark.parametrize("p,eps,c2", [(4, 1e-6, 10.0), (6, 1e-6, 10.0), (6, 1e-6, 100.0)])
def test_stage2_factors_match_oracle(p, eps, c2):
    # stage-2 low rank (Sec. 3.2): same ranks as the oracle and the same factored
    # matrices U^ V^ (in the U~ basis, which is unique up to signs)
    x = workloads.uniform_cube(4096, 1211)
    pl = K.Plan(x, p=p, eps=eps, leaf_size=64, device=-1, c2=c2)
    ops = oracle.build_operators(p, eps, 64, mode="svd2", c2=c2)
    k = ops.k
    info = pl.info()
    ranks = pl.export_operator(7).astype(int)
    want = np.array([ops.K2[t][0].shape[1] for t in oracle.offset_classes()])
    # a singular value within rounding of the cutoff may fall on either side
    assert np.abs(ranks - want).max() <= 1 and np.mean(ranks != want) < 0.02
    assert info["m2l_rank_max"] == ranks.max() and abs(info["m2l_rank_mean"] - ranks.mean()) < 1e-12
    rm = info["m2l_rank_max"]
    U = pl.export_operator(1).reshape(ops.n_eq, k)
    U2 = pl.export_operator(8).reshape(316, k, rm)
    V2 = pl.export_operator(9).reshape(316, rm, k)
    scale = max(np.abs(v).max() for v in ops.K_full.values())
    for i, t in enumerate(oracle.offset_classes()):
        r = ranks[i]
        assert not U2[i][:, r:].any() and not V2[i][r:].any()
        Uh, Vh = ops.K2[t]
        mine = U @ U2[i] @ V2[i] @ U.T
        ref = ops.U @ Uh @ Vh @ ops.U.T
        # equal ranks: the same truncated matrix; one more or fewer singular
        # value: they differ by that value, which is within rounding of the cutoff
        assert np.abs(mine - ref).max() <= 1e-9 * scale + (0 if r == Uh.shape[1] else 2 * ops.eps2)
    # flops of the two thin products
    assert info["flops"]["m2l"] < 2 * k * k * info["v_pairs"]


@pytest.mark.parametrize("p,dense", [(4, False), (6, False), (4, True)])
def test_m2l_spectra_invariant_under_cube_symmetries(p, dense):
    # singular values of the exported M2L matrices (compressed K~, or the
    # uncompressed K) agree across each orbit of the 48 cube symmetries
    x = workloads.uniform_cube(2000, 7)
    pl = K.Plan(x, p=p, eps=1e-6, leaf_size=64, device=-1, dense_m2l=dense)
    k = pl.info()["k"]
    sv = np.linalg.svd(pl.export_operator(6).reshape(316, k, k), compute_uv=False)
    offs = [(a, b, c) for a in range(-3, 4) for b in range(-3, 4) for c in range(-3, 4)
            if max(abs(a), abs(b), abs(c)) >= 2]
    orbits = {}
    for i, t in enumerate(offs):
        orbits.setdefault(tuple(sorted(map(abs, t))), []).append(i)
    assert len(orbits) == 16
    for idx in orbits.values():
        assert np.max(np.abs(sv[idx] - sv[idx[0]])) <= 1e-12 * sv[idx[0]][0]


@pytest.mark.parametrize("p", [4, 6])
def test_stage2_spectra_invariant_under_cube_symmetries(p):
    # cube surfaces: offsets in one orbit of the 48 axis permutations and
    # reflections (same sorted |t_a|) have M2L operators related by
    # orthogonal maps, hence equal stage-2 ranks and kept singular values
    # (the row norms of V^ = S^ Q^^T); offsets in lexicographic order over
    # [-3,3]^3 with max |t_a| >= 2
    x = workloads.uniform_cube(2000, 7)
    pl = K.Plan(x, p=p, eps=1e-6, leaf_size=64, device=-1, c2=10.0)
    info = pl.info()
    k, r = info["k"], info["m2l_rank_max"]
    ranks = pl.export_operator(7).astype(int)
    sv = np.linalg.norm(pl.export_operator(9).reshape(316, r, k), axis=2)
    offs = [(a, b, c) for a in range(-3, 4) for b in range(-3, 4) for c in range(-3, 4)
            if max(abs(a), abs(b), abs(c)) >= 2]
    orbits = {}
    for i, t in enumerate(offs):
        orbits.setdefault(tuple(sorted(map(abs, t))), []).append(i)
    assert len(orbits) == 16
    for idx in orbits.values():
        assert len(set(ranks[idx])) == 1
        ref = sv[idx[0]]
        assert np.max(np.abs(sv[idx] - ref)) <= 1e-10 * ref[0]


def test_stage2_rejected_with_dense_or_bf16x3():
    x = workloads.uniform_cube(500, 1211)
    with pytest.raises(K.KifmmError):
        K.Plan(x, p=4, eps=1e-6, leaf_size=64, device=-1, c2=10.0, dense_m2l=True)
    with pytest.raises(K.KifmmError):
        K.Plan(x, p=4, eps=1e-6, leaf_size=64, device=-1, c2=10.0, precision="bf16x3")
    with pytest.raises(K.KifmmError):
        K.Plan(x, p=4, eps=1e-6, leaf_size=64, device=-1, c2=-1.0)
    pl = K.Plan(x, p=4, eps=1e-6, leaf_size=64, device=-1)
    with pytest.raises(K.KifmmError):
        pl.export_operator(7)


def test_fp32_arctangent_coefficients_match_fit():
    # the FP32 arctangent of the BEM element integrals (eval.hip, bem_atan2)
    # uses the polynomial that csrc/fit_atan.py fits: the coefficients in the
    # source equal the script's, the FP32 evaluation stays within 1e-7 of
    # atan on [0, 1], and the octant reduction reproduces atan2 to 4e-7
    import importlib.util
    import os
    import re
    here = os.path.join(os.path.dirname(K.__file__), "csrc")
    spec = importlib.util.spec_from_file_location("fit_atan", os.path.join(here, "fit_atan.py"))
    fa = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fa)
    cf = fa.fit()
    src = open(os.path.join(here, "eval.hip")).read()
    body = src[src.index("__device__ __forceinline__ float bem_atan2"):]
    body = body[:body.index("return copysignf")]
    # Horner order in the source: the highest-degree coefficient, then one per fmaf step
    lits = [float(re.search(r"float p = (-?\d+\.\d+)f;", body).group(1))]
    lits += [float(v) for v in re.findall(r"__builtin_fmaf\(p, s, (-?\d+\.\d+)f\)", body)]
    assert np.array_equal(np.float32(lits), cf[::-1]), (lits, cf)
    assert fa.fp32_error(cf) < 1e-7

    def atan2_32(y, x):
        ax, ay = np.abs(x), np.abs(y)
        mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
        t = np.where(mx > 0, mn / np.where(mx > 0, mx, 1), 0).astype(np.float32)
        s = (t * t).astype(np.float32)
        p = np.full_like(t, cf[-1])
        for k in range(len(cf) - 2, -1, -1):
            p = (p * s + cf[k]).astype(np.float32)
        r = (t * p).astype(np.float32)
        r = np.where(ay > ax, np.float32(np.pi / 2) - r, r)
        r = np.where(x < 0, np.float32(np.pi) - r, r)
        return np.copysign(r, y)

    rng = np.random.default_rng(0)
    y, x = (rng.normal(size=(2, 100000)) * 10.0 ** rng.uniform(-3, 3, (2, 100000))).astype(np.float32)
    assert np.abs(atan2_32(y, x) - np.arctan2(y.astype(np.float64), x.astype(np.float64))).max() < 4e-7
