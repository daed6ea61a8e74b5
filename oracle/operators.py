"""Equivalent/check surfaces and translation operators (test infrastructure only).

Surfaces (Sec. 2.1): for a cube of half-width r the upward equivalent surface
and the downward check surface are cube boundaries of half-width (1+d) r; the
upward check surface and the downward equivalent surface have half-width
(3-2d) r. Sec. 4.1 sets d = C_d / sqrt(s) with C_d = 0.5. Points are sampled
on the surfaces with p points per cube side (Sec. 1): the boundary nodes of a
uniform p x p x p grid, n_eq = p^3 - (p-2)^3 of them, in lexicographic order.

All operators are built for the cube of unit half-width centred at 0; the
kernel 1/(4 pi r) is homogeneous of degree -1 (Sec. 3.1), which gives the
level scalings used by the evaluation:

* S2M (Sec. 2.2): q^u = r * P_up * (upward check potential), P_up the
  pseudo-inverse of G(upward check, upward equivalent);
* M2M (Sec. 2.2): M^o = P_up G(UC, (o + UE)/2), o in {-1,1}^3 the child offset;
* M2L (Sec. 2.2): K^(t) = G(DC + 2t, UE), t the integer centre offset in units
  of the cube width, scaled by 1/r at half-width r; the 316 offsets with
  max |t_a| in {2,3} are the classes;
* L2L (Sec. 2.2): L^o = G((o + DC)/2, DE) P_dn, P_dn = pinv(G(DC, DE));
* L2T (Sec. 2.2): e = r * P_dn * p^d, then the potential of e on DE.

Stage-1 compression (Sec. 3.1: the fat/thin SVDs and the compressed K~): U from the SVD of
K_fat = [K^(1) ... K^(316)]; keep the columns whose singular value is at least
eps * Sigma_00. Because the downward check and upward equivalent surfaces
coincide, K^(-t) = K^(t)^T, so K_thin is a block permutation of K_fat^T and its
right factor R equals U: one SVD suffices (the reading of the symmetry remark
in Sec. 3.1). Then K~ = U~^T K U~ and, from Sec. 3.3, S~ = U~^T S,
M~ = U~^T M U~, L~ = U~^T L U~, T~ = T U~ (the printed "T~ = T~ U~" is read as
T~ = T U~).

Stage-2 low rank (Sec. 3.2, mode "svd2"): each compressed M2L matrix is
factored by its own SVD, K~^(t) = U S Q^T, and the singular values below
eps2 * ||K_fat||_2 are dropped, eps2 = C2 * eps / k (eq. for eps2 in Sec. 3.2,
with eps the stage-1 threshold and k the compressed dimension). M2L then applies
U^ (V^ q) with V^ = S^ Q^^T: two thin products of rank r_t instead of one k x k
product. The 2-norm error of each factored matrix is the first dropped singular
value, at most eps2 * ||K_fat||_2.

The pseudo-inverse is a truncated SVD with relative cutoff `rcond` (the paper
does not say how the check-to-equivalent systems are solved).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .direct import kernel_matrix

CHILD_SIGNS = list(itertools.product((-1.0, 1.0), repeat=3))


def n_equiv(p: int) -> int:
    return p ** 3 - (p - 2) ** 3 if p >= 2 else 0


def surface_template(p: int) -> np.ndarray:
    """Boundary nodes of the p^3 grid on [-1,1]^3, lexicographic (i,j,k)."""
    g = np.linspace(-1.0, 1.0, p)
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if min(i, j, k) == 0 or max(i, j, k) == p - 1:
                    pts.append((g[i], g[j], g[k]))
    return np.asarray(pts, dtype=np.float64)


def offset_classes():
    """The 316 integer offsets t in [-3,3]^3 with max |t_a| >= 2 (Sec. 3.1)."""
    return [t for t in itertools.product(range(-3, 4), repeat=3) if max(abs(v) for v in t) >= 2]


@dataclass
class Operators:
    p: int
    n_eq: int
    d: float
    rcond: float
    mode: str
    k: int                     # reduced dimension (n_eq when mode == "dense")
    UE: np.ndarray             # unit upward equivalent surface (1+d)
    UC: np.ndarray             # unit upward check surface (3-2d)
    DC: np.ndarray             # unit downward check surface (1+d)
    DE: np.ndarray             # unit downward equivalent surface (3-2d)
    S: np.ndarray              # (k, n_eq)  check potential -> (reduced) equivalent density
    M: dict                    # child sign o -> (k,k)
    K: dict                    # offset t -> (k,k)
    L: dict                    # child sign o -> (k,k)
    T: np.ndarray              # (n_eq, k)  (reduced) check potential -> downward equivalent density
    sing: np.ndarray | None = None   # singular values of K_fat (svd mode)
    U: np.ndarray | None = None      # U~ (n_eq, k) (svd mode)
    K_full: dict | None = None       # uncompressed K^(t) (svd mode keeps them for checks)
    K2: dict | None = None           # svd2 mode: offset t -> (U^ (k, r_t), V^ (r_t, k))
    eps2: float | None = None        # svd2 mode: absolute stage-2 cutoff eps2 * ||K_fat||_2


def stage2_factors(K: dict, sigma0: float, eps: float, k: int, c2: float):
    """Per-class low-rank factors of the compressed M2L matrices (Sec. 3.2).

    Returns ({t: (U^, V^)}, cutoff) with cutoff = C2 * eps / k * sigma0, keeping
    the singular values not below the cutoff (V^ = S^ Q^^T).
    """
    cut = c2 * eps / k * sigma0
    out = {}
    for t, Kt in K.items():
        U, S, Qt = np.linalg.svd(Kt)
        r = int(np.count_nonzero(S >= cut))
        out[t] = (U[:, :r], S[:r, None] * Qt[:r, :])
    return out, cut


def build_operators(p: int, eps: float, leaf_size: int, mode: str = "dense",
                    cd: float = 0.5, rcond: float = 1e-10, c2: float = 0.0) -> Operators:
    """Operators of `mode`: "dense" (uncompressed), "svd" (stage 1, Sec. 3.1 and
    3.3) or "svd2" (stage 1 plus the stage-2 factors of Sec. 3.2 with constant c2)."""
    if mode not in ("dense", "svd", "svd2"):
        raise ValueError(mode)
    E = surface_template(p)
    n = E.shape[0]
    d = cd / np.sqrt(float(leaf_size))
    inner = (1.0 + d) * E
    outer = (3.0 - 2.0 * d) * E
    UE, UC, DC, DE = inner, outer, inner, outer
    P_up = np.linalg.pinv(kernel_matrix(UC, UE), rcond=rcond)
    P_dn = np.linalg.pinv(kernel_matrix(DC, DE), rcond=rcond)
    M = {o: P_up @ kernel_matrix(UC, 0.5 * (np.asarray(o) + UE)) for o in CHILD_SIGNS}
    L = {o: kernel_matrix(0.5 * (np.asarray(o) + DC), DE) @ P_dn for o in CHILD_SIGNS}
    K = {t: kernel_matrix(DC + 2.0 * np.asarray(t, dtype=np.float64), UE) for t in offset_classes()}
    if mode == "dense":
        return Operators(p=p, n_eq=n, d=d, rcond=rcond, mode=mode, k=n, UE=UE, UC=UC, DC=DC,
                         DE=DE, S=P_up, M=M, K=K, L=L, T=P_dn)
    K_fat = np.concatenate([K[t] for t in offset_classes()], axis=1)
    U, sing, _ = np.linalg.svd(K_fat, full_matrices=False)
    k = int(np.count_nonzero(sing >= eps * sing[0]))
    Ut = U[:, :k]
    Kc = {t: Ut.T @ K[t] @ Ut for t in K}
    K2, cut = stage2_factors(Kc, sing[0], eps, k, c2) if mode == "svd2" else (None, None)
    return Operators(
        p=p, n_eq=n, d=d, rcond=rcond, mode=mode, k=k, UE=UE, UC=UC, DC=DC, DE=DE,
        S=Ut.T @ P_up,
        M={o: Ut.T @ M[o] @ Ut for o in CHILD_SIGNS},
        K=Kc,
        L={o: Ut.T @ L[o] @ Ut for o in CHILD_SIGNS},
        T=P_dn @ Ut,
        sing=sing, U=Ut, K_full=K, K2=K2, eps2=cut)
