"""MI355X (gfx950) SVD-accelerated kernel-independent FMM: Python binding.

Thin ctypes marshalling over the C ABI declared in include/kifmm.h. Every step
of the evaluation runs in the library's HIP kernels; PyTorch only provides
device memory and the current stream. There is no CPU fallback: if the
library is not built, loading fails with an error.

    plan = Plan(points, p=6, eps=1e-6, leaf_size=64)      # points: (N,3) float64, host
    phi = plan.apply(sigma)                               # sigma: (N,) cuda float32
    g = plan.apply_adjoint(r)
    KifmmMatvec.apply(plan, sigma)                        # autograd: backward = adjoint
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Plan", "Group", "KifmmMatvec", "KifmmError", "load_library", "library_path",
           "FP64", "FP32", "BF16X3", "STAGES", "EXPORTED_SYMBOLS"]

FP64, FP32, BF16X3 = 0, 1, 2
STAGES = ("p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "perm")
_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}

EXPORTED_SYMBOLS = (
    "kifmm_opts_default", "kifmm_plan", "kifmm_plan_ex", "kifmm_apply", "kifmm_apply_adjoint",
    "kifmm_apply_batched", "kifmm_group_create", "kifmm_group_apply", "kifmm_group_destroy",
    "kifmm_plan_info", "kifmm_plan_export_tree", "kifmm_plan_export_operator", "kifmm_profile",
    "kifmm_profile_read", "kifmm_destroy", "kifmm_last_error", "kifmm_apply_noalloc",
    "kifmm_plan_export_point_leaves", "kifmm_plan_export_boxes", "kifmm_plan_export_list",
    "kifmm_plan_bem", "kifmm_solve_gmres",
)


class KifmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kifmm error {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("cd", ctypes.c_double), ("pinv_rcond", ctypes.c_double),
                ("depth", ctypes.c_int), ("max_depth", ctypes.c_int), ("dense_m2l", ctypes.c_int),
                ("max_nrhs", ctypes.c_int), ("device", ctypes.c_int), ("mem_limit", ctypes.c_size_t),
                ("tile_targets", ctypes.c_int), ("m2l_shape", ctypes.c_int), ("c2", ctypes.c_double),
                ("adaptive", ctypes.c_int), ("fused_leaf", ctypes.c_int), ("direct_passes", ctypes.c_int), ("near_overlap", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("k", ctypes.c_int), ("n_eq", ctypes.c_int), ("k_pad", ctypes.c_int),
                ("precision", ctypes.c_int), ("dense_m2l", ctypes.c_int), ("n", ctypes.c_int64),
                ("n_leaf", ctypes.c_int64), ("n_box", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("p2p_interactions", ctypes.c_int64), ("v_pairs", ctypes.c_int64),
                ("v_pairs_level", ctypes.c_int64 * 21), ("boxes_level", ctypes.c_int64 * 21),
                ("r0", ctypes.c_double), ("flops", ctypes.c_double * 7), ("bytes", ctypes.c_double * 7),
                ("device_bytes", ctypes.c_size_t), ("m2l_tile_targets", ctypes.c_int),
                ("sigma0", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("m2l_variant", ctypes.c_int), ("m2l_tiles", ctypes.c_int),
                ("m2l_rank_max", ctypes.c_int), ("m2l_rank_mean", ctypes.c_double),
                ("adaptive", ctypes.c_int), ("leaf_level_min", ctypes.c_int), ("w_pairs", ctypes.c_int64),
                ("w_cubes", ctypes.c_int64), ("m2t_flops", ctypes.c_double), ("s2l_flops", ctypes.c_double),
                ("layer", ctypes.c_int), ("m2l_chunks", ctypes.c_int64), ("m2l_blocks", ctypes.c_int64)]


_LIB = None


def library_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkifmm.so")


def load_library():
    """Load libkifmm.so (built in-tree by paper_1211_2517_amd/build.py)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P, I, D, I64, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    lib.kifmm_opts_default.argtypes = [ctypes.POINTER(_Opts)]
    lib.kifmm_plan.argtypes = [P, I64, I, D, I, ctypes.POINTER(V)]
    lib.kifmm_plan_ex.argtypes = [P, I64, I, D, I, ctypes.POINTER(_Opts), ctypes.POINTER(V)]
    lib.kifmm_apply.argtypes = [V, P, P, P]
    lib.kifmm_apply_adjoint.argtypes = [V, P, P, P]
    lib.kifmm_apply_noalloc.argtypes = [V, P, P, P]
    lib.kifmm_apply_batched.argtypes = [V, P, P, I, I64, P]
    lib.kifmm_group_create.argtypes = [ctypes.POINTER(V), I, ctypes.POINTER(V)]
    lib.kifmm_group_apply.argtypes = [V, ctypes.POINTER(P), ctypes.POINTER(P), P]
    lib.kifmm_group_destroy.argtypes = [V]
    lib.kifmm_group_destroy.restype = None
    lib.kifmm_plan_info.argtypes = [V, ctypes.POINTER(_Info)]
    lib.kifmm_plan_export_tree.argtypes = [V, P]
    lib.kifmm_plan_export_operator.argtypes = [V, I, P, ctypes.POINTER(I64)]
    lib.kifmm_plan_export_point_leaves.argtypes = [V, P]
    lib.kifmm_plan_export_boxes.argtypes = [V, P, ctypes.POINTER(I64)]
    lib.kifmm_plan_export_list.argtypes = [V, I, P, ctypes.POINTER(I64)]
    lib.kifmm_solve_gmres.argtypes = [V, P, P, D, I, I, P, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.kifmm_plan_bem.argtypes = [P, I64, P, I64, I, I, D, I, ctypes.POINTER(_Opts), ctypes.POINTER(V)]
    lib.kifmm_profile.argtypes = [V, I]
    lib.kifmm_profile_read.argtypes = [V, P, ctypes.POINTER(I64)]
    lib.kifmm_destroy.argtypes = [V]
    lib.kifmm_destroy.restype = None
    lib.kifmm_last_error.restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if not hasattr(lib, name):
            raise ImportError(f"{path} does not export {name}")
    _LIB = lib
    return lib


def _check(rc):
    if rc != 0:
        raise KifmmError(rc, load_library().kifmm_last_error().decode())


def _torch():
    import torch
    return torch


class Plan:
    """A KIFMM plan over a fixed point set (tree, lists, operators on the device)."""

    def __init__(self, points, p: int = 6, eps: float = 1e-6, leaf_size: int = 64, *,
                 precision: str = "fp32", dense_m2l: bool = False, max_nrhs: int = 1, device: int = 0,
                 depth: int = 0, max_depth: int = 16, cd: float = 0.5, pinv_rcond: float = 1e-10,
                 mem_limit: int = 0, tile_targets: int = 0, m2l_shape: int = -1, c2: float = 0.0,
                 adaptive: bool = False, fused_leaf: int = 3, direct_passes: bool = True, near_overlap: bool = True, _mesh=None):
        lib = load_library()
        pts = np.ascontiguousarray(np.asarray(points.cpu().numpy() if hasattr(points, "cpu") else points,
                                              dtype=np.float64))
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must have shape (N, 3)")
        o = _Opts()
        lib.kifmm_opts_default(ctypes.byref(o))
        o.precision = _PREC[precision]
        o.dense_m2l = int(bool(dense_m2l))
        o.max_nrhs = int(max_nrhs)
        o.device = int(device)
        o.depth = int(depth)
        o.max_depth = int(max_depth)
        o.cd = float(cd)
        o.pinv_rcond = float(pinv_rcond)
        o.mem_limit = int(mem_limit)
        o.tile_targets = int(tile_targets)
        o.m2l_shape = int(m2l_shape)
        o.c2 = float(c2)
        o.adaptive = int(bool(adaptive))
        o.fused_leaf = int(fused_leaf)
        o.direct_passes = int(bool(direct_passes))
        o.near_overlap = int(bool(near_overlap))
        h = ctypes.c_void_p()
        if _mesh is None:
            _check(lib.kifmm_plan_ex(pts.ctypes.data, pts.shape[0], int(p), float(eps), int(leaf_size),
                                     ctypes.byref(o), ctypes.byref(h)))
        else:
            verts, tris, layer = _mesh
            _check(lib.kifmm_plan_bem(verts.ctypes.data, verts.shape[0], tris.ctypes.data, tris.shape[0], layer,
                                      int(p), float(eps), int(leaf_size), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.n = pts.shape[0]
        self.p, self.eps, self.leaf_size = p, eps, leaf_size
        self.precision = precision
        self.device = device
        self.max_nrhs = max_nrhs

    @classmethod
    def bem(cls, vertices, triangles, layer: str = "single", p: int = 6, eps: float = 1e-6, leaf_size: int = 64,
            **kw):
        """BEM plan (kifmm_plan_bem): point i is the centroid of triangle i;
        apply(q) gives sum_j q_j int_{T_j} K(x_i, y) dS_y, K the single layer
        G or the double layer dG/dn(y)."""
        verts = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64))
        tris = np.ascontiguousarray(np.asarray(triangles, dtype=np.int32))
        if verts.ndim != 2 or verts.shape[1] != 3 or tris.ndim != 2 or tris.shape[1] != 3:
            raise ValueError("vertices must be (nv, 3) and triangles (nt, 3)")
        lay = {"single": 0, "double": 1}[layer]
        centroids = verts[tris].mean(axis=1) if tris.size and tris.min() >= 0 and tris.max() < len(verts) \
            else np.zeros((tris.shape[0], 3))
        return cls(centroids, p=p, eps=eps, leaf_size=leaf_size, _mesh=(verts, tris, lay), **kw)

    # ------------------------------------------------------------------ info
    def info(self) -> dict:
        i = _Info()
        _check(self._lib.kifmm_plan_info(self._h, ctypes.byref(i)))
        d = {f: getattr(i, f) for f, _ in _Info._fields_}
        d["v_pairs_level"] = list(i.v_pairs_level)[: i.depth + 1]
        d["boxes_level"] = list(i.boxes_level)[: i.depth + 1]
        d["flops"] = dict(zip(STAGES, list(i.flops)))
        d["bytes"] = dict(zip(STAGES, list(i.bytes)))
        return d

    def export_tree(self) -> np.ndarray:
        out = np.empty((self.n, 3), dtype=np.int32)
        _check(self._lib.kifmm_plan_export_tree(self._h, out.ctypes.data))
        return out

    def export_point_leaves(self) -> np.ndarray:
        """(level, i, j, k) of every point's leaf, caller order."""
        out = np.empty((self.n, 4), dtype=np.int32)
        _check(self._lib.kifmm_plan_export_point_leaves(self._h, out.ctypes.data))
        return out

    def export_boxes(self) -> np.ndarray:
        """Cubes in the plan's global order: (level, i, j, k, leaf index or -1)."""
        cnt = ctypes.c_int64()
        _check(self._lib.kifmm_plan_export_boxes(self._h, None, ctypes.byref(cnt)))
        out = np.empty((cnt.value, 5), dtype=np.int32)
        _check(self._lib.kifmm_plan_export_boxes(self._h, out.ctypes.data, ctypes.byref(cnt)))
        return out

    def export_list(self, which: str) -> np.ndarray:
        """(target, source) global cube indices of list "U", "V", "W" or "X"."""
        w = {"U": 0, "V": 1, "W": 2, "X": 3}[which]
        cnt = ctypes.c_int64()
        _check(self._lib.kifmm_plan_export_list(self._h, w, None, ctypes.byref(cnt)))
        out = np.empty((cnt.value, 2), dtype=np.int32)
        if cnt.value:
            _check(self._lib.kifmm_plan_export_list(self._h, w, out.ctypes.data, ctypes.byref(cnt)))
        return out

    def export_operator(self, which: int) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check(self._lib.kifmm_plan_export_operator(self._h, which, None, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=np.float64)
        _check(self._lib.kifmm_plan_export_operator(self._h, which, out.ctypes.data, ctypes.byref(cnt)))
        return out

    def profile(self, enable: bool = True):
        """Switch per-stage HIP-event timing on/off (clears the totals)."""
        _check(self._lib.kifmm_profile(self._h, int(bool(enable))))

    def profile_read(self) -> tuple[dict, int]:
        """(summed ms per stage since profiling was enabled, profiled applies)."""
        ms = (ctypes.c_double * 7)()
        calls = ctypes.c_int64()
        _check(self._lib.kifmm_profile_read(self._h, ms, ctypes.byref(calls)))
        return dict(zip(STAGES, list(ms))), calls.value

    # ----------------------------------------------------------------- apply
    def _dtype(self):
        torch = _torch()
        return torch.float64 if self.precision == "fp64" else torch.float32

    def _check_vec(self, x, name):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if x.dtype != self._dtype():
            raise TypeError(f"{name} must be {self._dtype()} for a {self.precision} plan")
        if x.device.index != self.device:
            raise ValueError(f"{name} is on device {x.device.index}, plan on {self.device}")
        return x.contiguous()

    def _check_out(self, out, name, shape):
        """An output tensor is written in place by the kernels: it must already
        have the plan's dtype and device, the exact shape and a contiguous
        layout (no copy is made, so a mismatch is an error)."""
        torch = _torch()
        if not isinstance(out, torch.Tensor) or not out.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if out.dtype != self._dtype():
            raise TypeError(f"{name} must be {self._dtype()} for a {self.precision} plan")
        if out.device.index != self.device:
            raise ValueError(f"{name} is on device {out.device.index}, plan on {self.device}")
        if tuple(out.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(out.shape)}")
        if not out.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return out

    def _stream(self):
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def apply(self, sigma, out=None):
        sigma = self._check_vec(sigma, "sigma")
        if sigma.shape != (self.n,):
            raise ValueError(f"sigma must have shape ({self.n},)")
        if out is None:
            out = _torch().empty_like(sigma)
        else:
            self._check_out(out, "out", (self.n,))
        if out.data_ptr() == sigma.data_ptr():
            raise ValueError("out must not alias sigma")
        _check(self._lib.kifmm_apply(self._h, sigma.data_ptr(), out.data_ptr(), self._stream()))
        return out

    def apply_noalloc(self, sigma, out):
        """phi = F sigma through kifmm_apply_noalloc: the library allocates
        nothing (its workspace is a static device array shared by every such
        call on the GPU). `out` is the caller's preallocated result."""
        sigma = self._check_vec(sigma, "sigma")
        if sigma.shape != (self.n,):
            raise ValueError(f"sigma must have shape ({self.n},)")
        self._check_out(out, "out", (self.n,))
        if out.data_ptr() == sigma.data_ptr():
            raise ValueError("out must not alias sigma")
        _check(self._lib.kifmm_apply_noalloc(self._h, sigma.data_ptr(), out.data_ptr(), self._stream()))
        return out

    def apply_adjoint(self, g, out=None):
        g = self._check_vec(g, "g")
        if g.shape != (self.n,):
            raise ValueError(f"g must have shape ({self.n},)")
        if out is None:
            out = _torch().empty_like(g)
        else:
            self._check_out(out, "out", (self.n,))
        if out.data_ptr() == g.data_ptr():
            raise ValueError("out must not alias g")
        _check(self._lib.kifmm_apply_adjoint(self._h, g.data_ptr(), out.data_ptr(), self._stream()))
        return out

    def apply_batched(self, sigma, out=None):
        """sigma: (N, nrhs) tensor; column j is right-hand side j."""
        torch = _torch()
        if sigma.dim() != 2 or sigma.shape[0] != self.n:
            raise ValueError(f"sigma must have shape ({self.n}, nrhs)")
        nrhs = sigma.shape[1]
        if not 1 <= nrhs <= self.max_nrhs:
            raise ValueError(f"nrhs must be in [1, {self.max_nrhs}] (max_nrhs of the plan)")
        if out is not None:
            # filled by a copy from the library's column-major result, so any
            # layout will do; dtype, device and shape must match
            self._check_vec(out, "out")
            if tuple(out.shape) != (self.n, nrhs):
                raise ValueError(f"out must have shape ({self.n}, {nrhs})")
        colmajor = self._check_vec(sigma.t().contiguous(), "sigma")   # (nrhs, N): column-major N x nrhs
        res = torch.empty_like(colmajor)
        _check(self._lib.kifmm_apply_batched(self._h, colmajor.data_ptr(), res.data_ptr(), nrhs, self.n,
                                             self._stream()))
        res = res.t()
        if out is not None:
            out.copy_(res)
            return out
        return res.contiguous()

    def apply_batched_colmajor(self, sigma_cm, out_cm):
        """Several right-hand sides without layout copies: sigma_cm and out_cm
        are (nrhs, N) contiguous tensors, i.e. column-major N x nrhs; row j
        of out_cm receives F sigma_cm[j]."""
        sigma_cm = self._check_vec(sigma_cm, "sigma_cm")
        if sigma_cm.dim() != 2 or sigma_cm.shape[1] != self.n:
            raise ValueError(f"sigma_cm must have shape (nrhs, {self.n})")
        nrhs = sigma_cm.shape[0]
        if not 1 <= nrhs <= self.max_nrhs:
            raise ValueError(f"nrhs must be in [1, {self.max_nrhs}] (max_nrhs of the plan)")
        self._check_out(out_cm, "out_cm", (nrhs, self.n))
        if out_cm.data_ptr() == sigma_cm.data_ptr():
            raise ValueError("out_cm must not alias sigma_cm")
        _check(self._lib.kifmm_apply_batched(self._h, sigma_cm.data_ptr(), out_cm.data_ptr(), nrhs, self.n,
                                             self._stream()))
        return out_cm

    def solve_gmres(self, b, x0=None, tol: float = 1e-6, restart: int = 50, max_iter: int = 500):
        """x with A x = b (kifmm_solve_gmres): returns (x, applies used, final relative residual)."""
        b = self._check_vec(b, "b")
        torch = _torch()
        x = torch.zeros_like(b) if x0 is None else self._check_vec(x0, "x0").clone()
        it = ctypes.c_int()
        res = ctypes.c_double()
        _check(self._lib.kifmm_solve_gmres(self._h, b.data_ptr(), x.data_ptr(), float(tol), int(restart),
                                           int(max_iter), self._stream(), ctypes.byref(it), ctypes.byref(res)))
        return x, it.value, res.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.kifmm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Several plans whose applies run from one captured HIP graph."""

    def __init__(self, plans):
        lib = load_library()
        self._plans = list(plans)
        arr = (ctypes.c_void_p * len(self._plans))(*[p._h.value for p in self._plans])
        h = ctypes.c_void_p()
        _check(lib.kifmm_group_create(arr, len(self._plans), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    def apply(self, sigmas, outs):
        n = len(self._plans)
        if len(sigmas) != n or len(outs) != n:
            raise ValueError("need one sigma and one output per plan")
        # the graph captures raw device pointers: every sigma is checked (and
        # made contiguous, the copy kept alive here until the call returns;
        # a replay with other pointers re-captures), every out must be exactly
        # the plan's vector since it is written in place
        ins = []
        for i, (pl, s, o) in enumerate(zip(self._plans, sigmas, outs)):
            s = pl._check_vec(s, f"sigmas[{i}]")
            if tuple(s.shape) != (pl.n,):
                raise ValueError(f"sigmas[{i}] must have shape ({pl.n},)")
            pl._check_out(o, f"outs[{i}]", (pl.n,))
            if o.data_ptr() == s.data_ptr():
                raise ValueError(f"outs[{i}] must not alias sigmas[{i}]")
            ins.append(s)
        sp = (ctypes.c_void_p * n)(*[s.data_ptr() for s in ins])
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        _check(self._lib.kifmm_group_apply(self._h, sp, op, self._plans[0]._stream()))
        return outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.kifmm_group_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_autograd():
    torch = _torch()

    class KifmmMatvec(torch.autograd.Function):
        """phi = F sigma with d(loss)/d(sigma) = F^T (d loss / d phi) by the
        hand-written adjoint passes. F is linear in sigma, so nothing from the
        forward pass is kept for the backward pass."""

        @staticmethod
        def forward(ctx, plan, sigma):
            ctx.plan = plan
            return plan.apply(sigma.detach())

        @staticmethod
        def backward(ctx, grad_phi):
            return None, ctx.plan.apply_adjoint(grad_phi.contiguous())

    return KifmmMatvec


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


KifmmMatvec = _LazyAutograd()
