"""Pins for the oracle's local solve: eq. godonuv (Sec. 1.1) in the closed
form of the coarse solver C_H (Sec. 3.2), with the wind rules of
Alg. fineupdate2D (fine) and Alg. update2D (coarse).

The pins do not re-type the closed form: they check it against the
defining equation sum_a ((u - m_a)^+)^2 = (r Delta)^2 solved by a bracketing
root finder, against its special cases, and against the monotonicity fact
used in the proof of Theorem choosetheta (Sec. 4.1)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle

ULP = np.finfo(np.float64).eps


def godunov_root(m, rd):
    """Solve sum_a max(u - m_a, 0)^2 = rd^2 for u >= min(m) by bisection on
    the monotone left-hand side (the upwind form of eq. godonuv)."""
    m = np.asarray([x for x in m if np.isfinite(x)], dtype=np.float64)
    if m.size == 0:
        return math.inf
    lo = float(m.min())
    hi = lo + 2 * rd

    def f(u):
        return float(np.sum(np.maximum(u - m, 0.0) ** 2) - rd * rd)

    return brentq(f, lo, hi, xtol=1e-300, rtol=4 * ULP, maxiter=500)


def test_one_sided_is_min_plus_rd():
    rng = np.random.default_rng(0)
    for _ in range(500):
        rd = rng.uniform(0.01, 2.0)
        a = rng.uniform(0, 5)
        b = a + rd * rng.uniform(1.0, 4.0) * rng.choice([-1, 1])
        u, w = oracle.local([a, b], [1, -1], rd)
        assert u == min(a, b) + rd
        assert (w[0] != 0) != (w[1] != 0)
        assert (w[0] != 0) == (a < b)


def test_equal_neighbours_give_rd_over_sqrt2():
    for a in [0.0, 0.3, 1.7, 12.5]:
        for rd in [0.001, 0.1, 1.0]:
            u, w = oracle.local([a, a], [1, 1], rd)
            assert abs(u - (a + rd / math.sqrt(2.0))) <= 4 * ULP * max(1.0, a)
            assert list(w) == [1, 1]


@pytest.mark.parametrize("d", [2, 3])
def test_matches_root_of_godunov_equation(d):
    rng = np.random.default_rng(1 + d)
    for _ in range(2000):
        rd = rng.uniform(0.01, 1.0)
        m = rng.uniform(0.0, 2.0, d)
        if rng.uniform() < 0.3:
            m[rng.integers(0, d)] = np.inf
        ws = rng.choice([-1, 1], d)
        u, w = oracle.local(list(m), list(ws), rd)
        ref = godunov_root(m, rd)
        assert abs(u - ref) <= 8 * ULP * max(1.0, abs(ref)), (m, rd, u, ref)
        # winds: exactly the axes whose neighbour lies below u (the terms
        # that are active in eq. godonuv), each with the sign of its side
        for a in range(d):
            gap = u - m[a]
            if abs(gap) < 1e-9:
                continue  # a tie: either choice is a solution
            assert (w[a] != 0) == (gap > 0)
            assert w[a] in (0, ws[a])


def test_two_sided_residual_identity():
    rng = np.random.default_rng(7)
    for _ in range(1000):
        rd = rng.uniform(0.01, 1.0)
        a = rng.uniform(0, 3)
        b = a + rng.uniform(-0.99, 0.99) * rd
        u, _ = oracle.local([a, b], [1, 1], rd)
        lhs = (u - a) ** 2 + (u - b) ** 2
        assert abs(lhs - rd * rd) <= 16 * ULP * max(1.0, u) ** 2


def test_monotone_in_neighbours():
    # the fact used in the proof of Theorem choosetheta: a <= b implies
    # C_H(a, c) <= C_H(b, c)
    rng = np.random.default_rng(11)
    for _ in range(2000):
        rd = rng.uniform(0.01, 1.0)
        a, b, c = np.sort(rng.uniform(0, 2, 3))
        ua, _ = oracle.local([a, c], [1, 1], rd)
        ub, _ = oracle.local([b, c], [1, 1], rd)
        assert ua <= ub


def test_coarse_and_fine_wind_rules_agree_off_ties():
    rng = np.random.default_rng(5)
    for d in (2, 3):
        for _ in range(2000):
            rd = rng.uniform(0.01, 1.0)
            m = rng.uniform(0, 2, d)
            ws = rng.choice([-1, 1], d)
            u0, w0 = oracle.local(list(m), list(ws), rd, rule=0)
            u1, w1 = oracle.local(list(m), list(ws), rd, rule=1)
            assert u0 == u1
            if np.min(np.abs(u0 - m)) > 1e-9:
                assert list(w0) == list(w1)


def test_no_finite_neighbour_gives_infinity():
    for d in (2, 3):
        u, w = oracle.local([np.inf] * d, [1] * d, 0.5)
        assert u == np.inf


def test_fp32_build_rounds_the_same_expressions():
    rng = np.random.default_rng(9)
    for d in (2, 3):
        for _ in range(500):
            rd = np.float32(rng.uniform(0.01, 1.0))
            m = rng.uniform(0, 2, d).astype(np.float32)
            u32, _ = oracle.local(list(m), [1] * d, rd, dtype=np.float32)
            u64, _ = oracle.local(list(m.astype(np.float64)), [1] * d, float(rd))
            assert abs(float(u32) - u64) <= 8 * np.finfo(np.float32).eps * max(1.0, u64)
