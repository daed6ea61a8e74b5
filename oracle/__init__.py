"""Plain FP64 CPU oracle for the SVD-accelerated kernel-independent FMM.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg do. It shares
no code, tables or constants with the GPU library: the two agree only because
both follow the paper.

What it computes (Cao, Wen, Rong, "A SVD accelerated kernel-independent fast
multipole method and its application to BEM"):

* ``direct``    - the O(N^2) sum of eq. (1) with the single-layer Laplace kernel
                  G(x,y) = 1/(4 pi |x-y|) of Sec. 4 (pairs at distance 0 add 0).
* ``fmm``       - the KIFMM of Sec. 2 evaluated step by step as in the complete
                  algorithm of Sec. 4.3, either uncompressed (``mode="dense"``,
                  M2L matrices K of Sec. 2.2) or with the stage-1 SVD compression
                  of Sec. 3.1 and the reduced upward/downward operators of
                  Sec. 3.3 (``mode="svd"``).

* ``bem``       - the collocation BEM of Sec. 4 (triangles, piecewise-constant
                  densities, single- and double-layer operators with closed-form
                  triangle integrals, the KIFMM BEM matvec, the ellipsoid
                  conductor in closed form, GMRES).
* ``adaptive``  - the KIFMM on an adaptive 2:1-balanced octree (U/V/W/X lists).

Library primitives used as single steps: ``numpy.linalg.svd`` and
``numpy.linalg.pinv`` (truncated-SVD pseudo-inverse), matrix products, sorting.

Pinned by the ``-m "not gpu"`` tests against brute force, closed forms
(uniform charge on a sphere), exact special cases (one leaf; eps -> 0),
exact invariances (dyadic scaling, translation, permutation) and the
stage-1 truncation bound. See each function for the passage it follows.
"""
from .direct import direct, kernel_matrix
from .tree import OracleTree, build_tree, root_cube, integer_coords
from .operators import Operators, surface_template, n_equiv, offset_classes, build_operators
from .fmm import fmm

__all__ = [
    "direct", "kernel_matrix", "OracleTree", "build_tree", "root_cube", "integer_coords",
    "Operators", "surface_template", "n_equiv", "offset_classes", "build_operators", "fmm",
]
