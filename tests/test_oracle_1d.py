"""Pins from the one-dimensional example of Sec. 3.1, on the oracle's 1D
method (oracle/dd1d.py).  The paper prints three facts about it
(tests/golden/paper_values.json, "one_dimensional_example"):
  * in the first iteration the corrected U_6 lies below U_7 while the wind
    at X_6 = 0.6 points from the right (W_6 = -1), and the causal sweep
    lifts U^1_6 to U^1_7;
  * iteration 3 reaches the fixed point: U^3 equals the fine values u^3.
The coarse grid (H = 0.1) does not see the bump at x = 0.75, so U^0 puts the
kink of u at 0.5 while u^f has it near 0.625: the first iterations must move
information across it, which exercises the wind convention, the Step 2
inflow test, the choice between the two fine values at a coarse node, the
wind-gated correction and the causal sweep.  h and theta are not stated;
the facts must hold for every h and theta tried.  The same facts decide the
reading of Step 2: inflow nodes that may still decrease in the subinterval
solve reproduce them, inflow nodes held at U stall off u^f."""
import json
import os

import numpy as np
import pytest

from oracle import dd1d

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def _golden():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        return json.load(f)["one_dimensional_example"]


def _run(M, theta, inflow_fixed=False, max_iter=8):
    g = _golden()
    N = round(1 / g["H"])

    def r(x):
        return 1 + g["bump_height"] * np.exp(-((x - g["bump_centre"]) ** 2) / (2 * g["bump_width"] ** 2))
    return dd1d.dd1(r, N, M, theta, max_iter=max_iter, inflow_fixed=inflow_fixed), N


def test_local_solve_and_fsm_closed_forms():
    """eq. 1dgod and the 1D FSM: constant r with u(0) = u(1) = 0 gives the
    tent r min(x, 1 - x) exactly (sums of r h in order) and winds pointing
    away from the sources.  The middle node keeps the wind of the sweep that
    set its value (the first, from the left): the later tie offers the same
    value, which the strict minimum does not take."""
    n = 21
    u = np.full(n, np.inf)
    w = np.zeros(n, dtype=int)
    fx = np.zeros(n, dtype=bool)
    u[0] = u[-1] = 0.0
    fx[0] = fx[-1] = True
    rd = [0.25] * n
    dd1d.fsm1(u, w, fx, rd)
    ref = np.zeros(n)
    for m in range(1, n // 2 + 1):
        ref[m] = ref[m - 1] + 0.25
    for m in range(n - 2, n // 2 - 1, -1):
        ref[m] = ref[m + 1] + 0.25
    assert np.array_equal(u, ref)
    assert list(w[1:10]) == [1] * 9 and list(w[11:20]) == [-1] * 9 and w[10] == 1
    assert dd1d.godunov1(2.0, 2.0, 0.5) == (2.5, -1)


@pytest.mark.parametrize("M", [50, 100, 400])
@pytest.mark.parametrize("theta", [0.1, 0.5, 1.0])
def test_causal_sweep_event_at_k1(M, theta):
    """k = 1: the corrected U_6 is below U_7 with W_6 = -1, and the causal
    sweep lifts it to exactly U_7's value."""
    R, N = _run(M, theta, max_iter=1)
    pre, U1, W1 = R["Upre"][0], R["U"][1], R["W"][1]
    assert pre[6] < pre[7]
    assert W1[6] == -1
    assert U1[6] == U1[7] == pre[7]
    assert U1[6] > pre[6]


@pytest.mark.parametrize("M", [50, 100, 400])
@pytest.mark.parametrize("theta", [0.1, 0.5, 1.0])
def test_converges_at_k3(M, theta):
    """U^3 = u^f at every coarse node (to a few ulp), U^2 is still off by a
    visible amount, and U^3 = u^3 (the fine values at the coarse nodes)."""
    R, N = _run(M, theta, max_iter=4)
    uf = R["uf"][::M]
    err = [np.max(np.abs(U - uf)) for U in R["U"]]
    g = _golden()
    k = g["iterations"]
    assert err[k] <= 32 * EPS, err
    assert all(e > 1e-3 for e in err[:k]), err
    assert np.max(np.abs(R["uk"][k] - R["U"][k])) <= 32 * EPS


@pytest.mark.parametrize("theta", [0.1, 1.0])
def test_inflow_held_at_U_stalls_off_the_fine_solution(theta):
    """The literal reading of Step 2 (an inflow end node held at U) settles
    (residual 0) on a state that is not u^f: the reading the method uses,
    and the paper's k = 3, needs the inflow value to be an upper bound the
    subinterval solve may lower."""
    R, N = _run(100, theta, inflow_fixed=True, max_iter=12)
    uf = R["uf"][::100]
    assert R["resid"][-1] == 0.0
    assert np.max(np.abs(R["U"][-1] - uf)) > 1e-2
