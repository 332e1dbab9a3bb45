"""Pins of the oracle's homogenised coarse solver (Sec. 5.3, the squares
medium): on a lattice it is the upwind scheme of max(|u_x|, |u_y|) = r, whose
solution from a point is r times the L1 distance.

- constant slowness, one source: after Step 1 every skeleton node holds the
  smallest of (Euclidean value at a near lattice node) + r * (L1 distance to
  it), computed here by brute force over the near nodes, in 2D and 3D; the
  Godunov coarse solver does not give that on the diagonals;
- the DD iteration with either coarse solver converges to the fine solution
  u^f (the fixed point of Sec. 3 does not depend on the coarse solver);
- on the squares medium the homogenised solver gives smaller relative L1
  errors than C_H over the iterations, as the paper reports for it."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1805_04198_amd import workloads as W


def near_l1_closed_form(n, h, r, src, M, U):
    """Brute force: for every skeleton node X (U not NaN), the minimum over
    the nodes Y of X's lattice (Y = X + M*k) within max-norm distance < M
    of the source of r*h*|Y - src|_2 + r*M*h*|k|_1."""
    d = len(n)
    out = np.full_like(U, np.nan)
    idx = np.nonzero(~np.isnan(U))[0]
    strides = [int(np.prod(n[:a])) for a in range(d)]
    for X in idx:
        c = [(X // strides[a]) % n[a] for a in range(d)]
        best = np.inf
        ranges = []
        for a in range(d):
            ks = [k for k in range(-(n[a] // M) - 1, n[a] // M + 2)
                  if abs(c[a] + k * M - src[a]) < M and 0 <= c[a] + k * M < n[a]]
            ranges.append(ks)
        for ks in itertools.product(*ranges):
            y = [c[a] + ks[a] * M for a in range(d)]
            d2 = sum((y[a] - src[a]) ** 2 for a in range(d))
            v = r * (h * np.sqrt(float(d2))) + r * (M * h) * sum(abs(k) for k in ks)
            best = min(best, v)
        out[X] = best
    return out


@pytest.mark.parametrize("n,S,M,src", [((65, 49), 16, 8, (24, 21)), ((33, 25), 8, 4, (16, 8)),
                                       ((17, 17, 9), 8, 4, (8, 5, 4))])
def test_step1_is_l1_distance_from_near_nodes(n, S, M, src):
    r = 1.5
    h = 1.0 / (n[0] - 1)
    rr = np.full(n[::-1], r)
    g = W.linear_index(n, *src)
    O = oracle.dd(n, h, rr, np.array([g]), np.zeros(1), S, M, max_iter=0, coarse_solver="l1",
                  max_coarse_sweeps=1000)
    U = O["U"]
    ref = near_l1_closed_form(n, h, r, src, M, U)
    m = ~np.isnan(U)
    assert m.sum() > 0
    assert np.allclose(U[m], ref[m], rtol=1e-13, atol=0), np.max(np.abs(U[m] - ref[m]))
    # the Godunov coarse solver is not the L1 distance off the lattice axes
    G = oracle.dd(n, h, rr, np.array([g]), np.zeros(1), S, M, max_iter=0, max_coarse_sweeps=1000)["U"]
    assert np.max(np.abs(G[m] - ref[m])) > 0.1 * r * M * h


def small_squares():
    # h = 1/224, eps = 8h, H = 16h = 1/14: coarse nodes on the r = 1 lines
    return W.squares(n_side=225, period=8, S=32, M=16)


def test_squares_medium_definition():
    p = W.squares()
    assert p.n == (449, 449) and abs(p.h - 1 / 448) < 1e-15 and p.M * p.h == pytest.approx(1 / 14)
    i = np.arange(449)
    on = (i % 8) == 0
    assert np.array_equal(p.r == 1.0, on[None, :] | on[:, None])
    assert set(np.unique(p.r)) == {1.0, 2.0}
    assert p.gamma_idx[0] == W.linear_index(p.n, 224, 224)
    # every coarse-lattice node (any shift that is a multiple of the period) has r = 1
    assert np.all(p.r[::p.M, ::p.M] == 1.0)


@pytest.mark.parametrize("cs", ["godunov", "l1"])
def test_converges_to_fine_solution(cs):
    p = small_squares()
    uf, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val)
    R = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=0.25, tol=1e-13, max_iter=200,
                  coarse_solver=cs)
    assert R["converged"]
    assert np.max(np.abs(R["u"] - uf)) <= 1e-12


def test_homogenised_solver_has_smaller_errors_on_squares():
    p = small_squares()
    uf, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val)
    errs = {}
    for cs in ("godunov", "l1"):
        e = []
        for k in (0, 1, 2, 4, 6):
            R = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=0.25, tol=0.0, max_iter=k,
                          coarse_solver=cs)
            m = np.isfinite(R["U"])
            e.append(np.sum(np.abs(R["U"][m] - uf[m])) / np.sum(np.abs(uf[m])))
        errs[cs] = np.array(e)
    assert np.all(errs["l1"] < errs["godunov"]), errs
    # the Godunov solver's error on U^0 is the diamond-versus-circle gap
    assert errs["godunov"][0] > 3 * errs["l1"][0], errs


def test_coarse_solver_argument():
    p = W.random_problem(1, (33, 33), 16, 8)
    with pytest.raises(KeyError):
        oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, max_iter=1, coarse_solver="max")
