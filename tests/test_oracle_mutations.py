"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's operators (a transposed
operand, a wrong child sign, a wrong class, a dropped term, swapped surfaces,
a wrong level scaling) and checks that the FMM-vs-direct-sum pin, which the
correct oracle meets, then fails.
"""
import copy
import functools

import numpy as np
import pytest

import oracle
import workloads
from oracle.fmm import fmm
from oracle.operators import build_operators, offset_classes

P, EPS, LEAF, BOUND = 6, 1e-6, 64, 1e-5


@functools.lru_cache(maxsize=None)
def _setup():
    x = workloads.uniform_cube(4096, 1211)
    q = workloads.uniform_density(4096, 1311)
    ops = build_operators(P, EPS, LEAF, mode="svd")
    return x, q, oracle.direct(x, q), ops


def _err(ops):
    x, q, ref, _ = _setup()
    phi, _ = fmm(x, q, P, EPS, LEAF, ops=ops)
    return float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))


def test_unmutated_meets_bound():
    assert _err(_setup()[3]) < BOUND


def _m_transposed(o):
    o.M = {k: v.T.copy() for k, v in o.M.items()}


def _l_wrong_child(o):
    o.L = {k: o.L[(-k[0], k[1], k[2])] for k in o.L}


def _k_negated_class(o):
    o.K = {t: o.K[(-t[0], -t[1], -t[2])] for t in o.K}


def _k_dropped_class(o):
    o.K = dict(o.K)
    o.K[(2, 0, 0)] = np.zeros_like(o.K[(2, 0, 0)])


def _k_level_scale(o):
    o.K = {t: 2.0 * v for t, v in o.K.items()}


def _s_unscaled_transpose(o):
    o.S = o.T.T.copy() * 1.001


def _surfaces_swapped(o):
    o.UC, o.UE = o.UE, o.UC


@pytest.mark.parametrize("mutate", [_m_transposed, _l_wrong_child, _k_negated_class,
                                    _k_dropped_class, _k_level_scale, _s_unscaled_transpose,
                                    _surfaces_swapped])
def test_planted_mistake_is_caught(mutate):
    ops = copy.copy(_setup()[3])
    mutate(ops)
    assert _err(ops) > BOUND


# stage-2 factors (Sec. 3.2): planted mistakes in the factored M2L matrices
@functools.lru_cache(maxsize=None)
def _setup2():
    return build_operators(P, EPS, LEAF, mode="svd2", c2=10.0)


def test_stage2_unmutated_meets_bound():
    assert _err(_setup2()) < BOUND


def _k2_unscaled(o):
    # V^ without the singular values (Q^^T instead of S^ Q^^T)
    o.K2 = {t: (U, V / np.linalg.norm(V, axis=1, keepdims=True)) for t, (U, V) in o.K2.items()}


def _k2_transposed_factors(o):
    # the class of -t (the transposed matrix) applied for t
    o.K2 = {t: o.K2[(-t[0], -t[1], -t[2])] for t in o.K2}


def _k2_rank_one(o):
    o.K2 = {t: (U[:, :1], V[:1]) for t, (U, V) in o.K2.items()}


@pytest.mark.parametrize("mutate", [_k2_unscaled, _k2_transposed_factors, _k2_rank_one])
def test_stage2_planted_mistake_is_caught(mutate):
    ops = copy.copy(_setup2())
    mutate(ops)
    assert _err(ops) > BOUND
