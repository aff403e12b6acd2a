"""The PCG host loop's chunk rule (lpcg_next_chunk, host code in the library):
the decay of log(||r||^2 / ||b||^2) between two looks at the done flag,
extrapolated to tol^2 and shortened by 15%, capped at four times the measured
span and at the iteration cap, at least one; 8 without a decay to measure."""
import math

import numpy as np
import pytest

from paper_2305_16432_amd import lpcg


def _rule(it, res, prev_it, prev_res, tol, maxit):
    span = it - prev_it
    if span <= 0 or not (res > 0) or not (prev_res > 0) or not math.isfinite(res):
        return 8, False
    rate = (math.log(res) - math.log(prev_res)) / span
    if not rate < -1e-6:
        return 8, False
    cap = min(4.0 * span, max(1, maxit - it + 1))
    if tol <= 0:
        return int(max(1, cap)), False
    need = math.ceil(0.85 * (math.log(tol * tol) - math.log(res)) / rate)
    return int(max(1, min(need, cap))), need <= cap


def test_geometric_decay_extrapolated():
    # 1e-4 after 8 iterations from 1: 16 more to 1e-12, 15% shorter -> 14
    assert lpcg.next_chunk(8, 1e-4, 0, 1.0, 1e-6, 1000) == (14, True)


@pytest.mark.parametrize("case", [
    (2, 0.5, 0, 1.0, 1e-10, 1000),        # capped at 4 x span
    (8, 1e-4, 0, 1.0, 1e-6, 10),          # capped at the iteration cap
    (8, 1e-4, 0, 1.0, 0.0, 1000),         # tol 0: the cap
    (8, 1.0001e-12, 0, 1.0, 1e-6, 1000),  # almost there: at least one
    (8, 2.0, 0, 1.0, 1e-6, 1000),         # growth: 8
    (8, 1.0, 0, 1.0, 1e-6, 1000),         # stagnation: 8
    (0, 0.5, 0, 1.0, 1e-6, 1000),         # no span: 8
    (8, 0.0, 0, 1.0, 1e-6, 1000),         # zero residual: 8
    (8, float("nan"), 0, 1.0, 1e-6, 1000),
    (8, 1e-4, 0, -1.0, 1e-6, 1000),       # no previous residual: 8
    (40, 1e-9, 12, 1e-3, 1e-8, 5000),
])
def test_rule_cases(case):
    got = lpcg.next_chunk(*case)
    assert got == _rule(*case), (case, got)


def test_random_histories_match_rule():
    rng = np.random.default_rng(4)
    for _ in range(500):
        prev_it = int(rng.integers(0, 200))
        it = prev_it + int(rng.integers(1, 40))
        prev_res = float(np.float32(10.0 ** rng.uniform(-12, 0)))
        res = float(np.float32(prev_res * 10.0 ** rng.uniform(-6, 0.5)))
        tol = float(10.0 ** rng.uniform(-10, -2))
        maxit = int(rng.integers(it, it + 300))
        assert lpcg.next_chunk(it, res, prev_it, prev_res, tol, maxit) == _rule(it, res, prev_it, prev_res, tol, maxit)
