"""Pins for Sec. 4's model problem, evaluated as the paper writes it
(oracle/model_problem.py: eq. modelprob with eqs. modelBC1, modelBC2, the
coarse solver that looks left and down, fine subdomain solves with the left
column held at U^k).  What the paper states about it
(tests/golden/paper_values.json, "model_problem"):
  * Theorem exactness: U^k_{i,j} = u^f_{i,j} once k >= i, for any weights;
  * Fig. theta1 (theta = 1, H = 1/20, h = 1/1000): the maximum error is
    above its starting value from k = 1 on, keeps rising and is largest near
    k = 10, then falls as the columns become exact one by one;
  * small weights converge (Fig. vartheta's comparison).
The min over X of M-bar^1 the paper prints (5.6e-3) is not reproduced by
the readings tried (see test_min_mbar_at_k1_is_recorded)."""
import json
import os

import numpy as np
import pytest

from oracle.model_problem import ModelStrip, c_h

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def _golden():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        return json.load(f)["model_problem"]


@pytest.fixture(scope="module")
def strip():
    g = _golden()
    return ModelStrip(g["N"], g["M"])


def test_coarse_solver_closed_forms():
    H = 0.05
    assert c_h(1.0, 5.0, H) == 1.0 + H                       # one-sided
    assert c_h(1.0, 1.0, H) == 1.0 + H / np.sqrt(2)          # equal neighbours (to rounding below)
    u = c_h(1.0, 1.02, H)
    assert abs((u - 1.0) ** 2 + (u - 1.02) ** 2 - H * H) <= 8 * EPS


def test_coarse_init_is_the_l1_distance(strip):
    """U^0 = C_H recursion from the left edge: along j < M each step adds H,
    so U^0_{i,j} = jh + iH (x + y), summed in order."""
    U0 = strip.coarse_init()
    for i in (1, 5, 20):
        for j in (1, 17, 49):
            v = strip.uf[0, j]
            for _ in range(i):
                v = v + strip.H
            assert U0[i, j] == v


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.1])
def test_theorem_exactness(strip, theta):
    Us, _ = strip.run(theta, strip.N + 1)
    for k, U in enumerate(Us):
        for i in range(0, min(k, strip.N) + 1):
            assert np.max(np.abs(U[i, 1:] - strip.uf[i, 1:])) <= 16 * EPS, (k, i)


def test_theta_one_error_grows_and_peaks_near_k10(strip):
    g = _golden()
    Us, _ = strip.run(1.0, strip.N + 2)
    e = np.array(strip.errors(Us))
    assert e[1] > e[0]                                       # above the start at k = 1 ...
    k_peak = int(np.argmax(e))
    assert abs(k_peak - g["theta1_error_peak_k"]) <= 2, e    # ... largest near k = 10 ...
    assert np.all(np.diff(e[: k_peak + 1]) > 0)              # ... growing until then
    assert np.all(e[strip.N:] <= 16 * EPS)                   # exact from k = N on


@pytest.mark.parametrize("theta", [0.05, 0.1])
def test_small_weights_converge_monotonically(strip, theta):
    Us, _ = strip.run(theta, strip.N + 1)
    e = np.array(strip.errors(Us))
    assert np.all(np.diff(e[: strip.N + 1]) < 0), e
    assert e[strip.N] <= 16 * EPS


def test_min_mbar_at_k1_is_recorded(strip):
    """M-bar^1_{i,j} = (u^f - u^0) / (C_H(U^1 nbrs) - C_H(U^0 nbrs)).  At
    column i = 2 it does not depend on the weights (U^1_1 = u^f_1 by Theorem
    exactness); with the upwind weights at M-bar itself (so that U^1 = u^f
    upwind) that column also holds the minimum over X.  The paper prints
    5.6e-3; these readings give 2.1e-2 (a recorded difference: the paper
    does not state the weights used upwind, nor its fine solver's details)."""
    seen = {}

    def exact_upwind(k, i, j, Un, Uo, uo):
        m = strip.Mbar(i, j, Un, Uo, uo)
        seen[(i, j)] = m
        return m if np.isfinite(m) else 0.0

    Us, _ = strip.run(0.0, 1, theta_fn=exact_upwind)
    vals = np.array([v for v in seen.values() if np.isfinite(v)])
    assert np.all(vals > 0)
    col2 = min(seen[(2, j)] for j in range(1, strip.M + 1))
    assert vals.min() == col2
    assert 0.02 < col2 < 0.022
    # with M-bar as the weight every node lands on u^f
    assert np.max(np.abs(Us[1][1:, 1:] - strip.uf[1:, 1:])) <= 64 * EPS


@pytest.mark.parametrize("N,M", [(10, 100), (20, 50), (50, 20)])
def test_estimated_weights_are_stable_on_the_model_problem(N, M):
    """Fig. vartheta's runs (h = 1/1000, H = 1/10, 1/20, 1/50) with the
    weights of eqs. secthetaest and thetaest (gamma = .75, delta = .01,
    x0 = .9): the columns are exact from k = N on (Theorem exactness holds
    for any weights).  At H = 1/10 and 1/20 the error never rises above its
    starting value and its sum over k < N is below that of every fixed
    weight tried (the advantage over a fixed theta the figure shows).  At
    H = 1/50 this reading has a transient at k = 14 that reaches 1.07 times
    the starting error, and the small fixed weights do better (recorded,
    bounded at 1.1 here)."""
    S = ModelStrip(N, M)
    e = np.array(S.errors(S.run_estimate(N + 1)))
    assert np.all(e[N:] <= 16 * EPS)
    assert np.all(e[1:] <= (1.0 if N <= 20 else 1.1) * e[0])
    if N <= 20:
        for th in (0.05, 0.1, 0.25):
            Us, _ = S.run(th, N)
            assert np.sum(e[1:N]) < np.sum(S.errors(Us)[1:N]), th
