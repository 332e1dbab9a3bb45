"""Pins for two rules of Sec. 3.2 that the fixed point u^f does not fix: the
causal sweep (Alg. causalsweep2D) and the reconciliation of the fine values
at a coarse node (Alg. fineupdate), on hand-built states whose outcome
follows from the printed rules by hand.

Alg. causalsweep2D at a vertically shifted node X = (i, j_m): if the flow
comes from +y (W . (0, -1) > 0) and U(X) < U(X + h e_y), then U(X) = U(X +
h e_y); if it comes from -y and U(X) < U(X - h e_y), U(X) = U(X - h e_y).
The neighbours are the fine-spacing ones (they lie on other shifted
lattices), and only coarse nodes take part; a horizontally shifted node
does the same along x, a corner along both.

Alg. fineupdate at a vertically shifted node between subdomains Omega_{i-1}
(minus side) and Omega_i (plus side), n^1 = (-1, 0), n^2 = (1, 0): if both
fine winds and W^k have w . n^1 >= 0 the node takes Omega_i's value, else
if all have w . n^2 >= 0 Omega_{i-1}'s, else the smaller (ties to
Omega_{i-1}'s); the wind comes with the value.  Winds are flow directions:
w_x = -1 means the upwind neighbour lies on the plus side."""
import numpy as np
import pytest

import oracle

n = (17, 17)
M = 4
N = n[0] * n[1]


def li(i, j):
    return i + n[0] * j


def state(values=(), winds=(), gamma=()):
    """Skeleton U = 0 at every coarse node (NaN elsewhere), winds 0, plus the
    given values / winds (axis components) / Gamma nodes."""
    U = np.full(N, np.nan)
    for j in range(n[1]):
        for i in range(n[0]):
            if i % M == 0 or j % M == 0:
                U[li(i, j)] = 0.0
    W = np.zeros((2, N), dtype=np.int8)
    isg = np.zeros(N, dtype=np.uint8)
    for (i, j), v in values:
        U[li(i, j)] = v
    for (i, j), (wx, wy) in winds:
        W[0, li(i, j)], W[1, li(i, j)] = wx, wy
    for (i, j) in gamma:
        isg[li(i, j)] = 1
    return U, W, isg


def run(U, W, isg):
    return oracle.causal(n, M, U, W, isg)


def changed(U0, U1):
    return sorted(int(x) for x in np.nonzero(~((U0 == U1) | (np.isnan(U0) & np.isnan(U1))))[0])


def test_vertical_node_flow_from_plus_y_is_raised_to_its_upper_neighbour():
    U, W, g = state([((4, 5), 1.0), ((4, 6), 2.0), ((4, 4), 3.0)], [((4, 5), (0, -1))])
    V = run(U, W, g)
    assert V[li(4, 5)] == 2.0
    assert changed(U, V) == [li(4, 5)]


def test_vertical_node_flow_from_minus_y_is_raised_to_its_lower_neighbour():
    U, W, g = state([((4, 5), 1.0), ((4, 6), 2.0), ((4, 4), 3.0)], [((4, 5), (0, 1))])
    V = run(U, W, g)
    assert V[li(4, 5)] == 3.0
    assert changed(U, V) == [li(4, 5)]


@pytest.mark.parametrize("val,wind", [(2.5, (0, -1)),    # already above the upwind neighbour
                                      (1.0, (0, 0)),     # no y component
                                      (1.0, (1, 0)),     # x: the fine x neighbours are not coarse nodes
                                      (1.0, (-1, 0))])
def test_vertical_node_left_alone(val, wind):
    U, W, g = state([((4, 5), val), ((4, 6), 2.0), ((4, 4), 3.0), ((3, 5), np.nan), ((5, 5), np.nan)],
                    [((4, 5), wind)])
    V = run(U, W, g)
    assert changed(U, V) == []


@pytest.mark.parametrize("wy", [-1, 1])
def test_a_chain_along_the_flow_takes_the_upwind_value_in_one_causal_sweep(wy):
    # nodes (4, 5..7) (flow from +y) or (4, 1..3) (flow from -y), increasing
    # away from the corner that holds 5
    js = [5, 6, 7] if wy < 0 else [3, 2, 1]
    corner = (4, 8) if wy < 0 else (4, 0)
    vals = [((4, j), float(k + 1)) for k, j in enumerate(js)] + [(corner, 5.0)]
    U, W, g = state(vals, [((4, j), (0, wy)) for j in js])
    V = run(U, W, g)
    assert all(V[li(4, j)] == 5.0 for j in js)


def test_horizontal_node_uses_x():
    U, W, g = state([((5, 4), 1.0), ((6, 4), 2.0), ((4, 4), 0.5)], [((5, 4), (-1, 1))])
    V = run(U, W, g)
    assert V[li(5, 4)] == 2.0     # x: flow from +x, raised to U(6, 4); y neighbours are not coarse
    U, W, g = state([((5, 4), 1.0), ((6, 4), 2.0), ((4, 4), 1.5)], [((5, 4), (1, 0))])
    assert run(U, W, g)[li(5, 4)] == 1.5


def test_corner_applies_x_then_y():
    U, W, g = state([((4, 4), 1.0), ((5, 4), 2.0), ((4, 5), 3.0)], [((4, 4), (-1, -1))])
    assert run(U, W, g)[li(4, 4)] == 3.0
    U, W, g = state([((4, 4), 1.0), ((5, 4), 2.0), ((4, 3), 3.0)], [((4, 4), (-1, 1))])
    assert run(U, W, g)[li(4, 4)] == 3.0


def test_gamma_and_domain_edges():
    # a Gamma node keeps its value; a node on the right edge has no x+1 neighbour
    U, W, g = state([((4, 5), 1.0), ((4, 6), 2.0), ((16, 5), 1.0)], [((4, 5), (0, -1)), ((16, 5), (-1, 0))],
                    gamma=[(4, 5)])
    assert changed(U, run(U, W, g)) == []


# ---------------------------------------------------------------------------
# reconciliation (Alg. fineupdate, per axis)
# ---------------------------------------------------------------------------

def rec2(uL, wL, uR, wR, Wk):
    return oracle.reconcile([uL, uR], [wL, wR], [[0, 0], [1, 0]], [1, 0], Wk)


def test_flow_towards_minus_x_takes_the_plus_side_value():
    u, w = rec2(1.0, (-1, 0), 2.0, (-1, 1), (-1, 0))
    assert u == 2.0 and list(w) == [-1, 1]


def test_flow_towards_plus_x_takes_the_minus_side_value():
    u, w = rec2(3.0, (1, 0), 2.0, (1, -1), (1, 1))
    assert u == 3.0 and list(w) == [1, 0]


def test_disagreeing_winds_take_the_smaller_ties_to_the_minus_side():
    assert rec2(3.0, (1, 0), 2.0, (-1, 0), (1, 0)) == (2.0, pytest.approx([-1, 0]))
    u, w = rec2(2.0, (1, 1), 2.0, (-1, 0), (-1, 0))
    assert u == 2.0 and list(w) == [1, 1]


def test_no_x_component_takes_the_first_branch():
    # every w . n^1 = 0 >= 0: the plus side, even when it is larger
    u, w = rec2(1.0, (0, 1), 4.0, (0, -1), (0, 1))
    assert u == 4.0 and list(w) == [0, -1]


def test_an_unreached_candidate_is_set_aside():
    # the printed rule would take the plus side's +inf; a candidate the
    # subdomain never reached carries no information, the finite one is kept
    u, w = rec2(1.0, (-1, 0), np.inf, (0, 0), (-1, 0))
    assert u == 1.0 and list(w) == [-1, 0]
    u, _ = rec2(np.inf, (0, 0), np.inf, (0, 0), (0, 0))
    assert u == np.inf


def test_corner_node_per_axis():
    # candidates in lexicographic tile order, x slowest: (x-,y-), (x-,y+), (x+,y-), (x+,y+)
    sides = [[0, 0], [0, 1], [1, 0], [1, 1]]
    vals = [4.0, 3.0, 2.0, 1.0]
    # all flow from -x and -y: the (x-, y-) subdomain's value
    u, w = oracle.reconcile(vals, [(1, 1)] * 4, sides, [1, 1], (1, 1))
    assert u == 4.0
    # flow from +x everywhere, y mixed: the plus side in x, both in y -> smaller of (x+,y-), (x+,y+)
    u, w = oracle.reconcile(vals, [(-1, 1), (-1, -1), (-1, 1), (-1, -1)], sides, [1, 1], (-1, 0))
    assert u == 1.0 and list(w) == [-1, -1]
