"""The one-dimensional method of Sec. 3.1, written out on its own.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): it exists to pin, with
the facts the paper prints for its 1D example, the rules the 2D/3D method
shares with it: the wind convention, the Step 2 inflow test, the choice
between the two fine values at a coarse node, the wind-gated weighted
correction and the causal sweep.  Plain Python loops (the 1D problems are
small).

Grids (Sec. 3.1): coarse nodes X_i = iH, i = 0..N, H = 1/N; subinterval i
holds the fine nodes iH + mh, m = 0..M, h = H/M.  Boundary data u(0) = u(1)
= g at X_0 and X_N.  Winds take the flow direction: +1 when the value came
from the left neighbour (the characteristic arrives from the left), -1 from
the right, as Step 1 defines them (its Step 4 names the opposite signs for
W~, which would make the correction's test W^k = w^k = W~ compare opposite
conventions; the flow direction is taken throughout).  Ties between the two
neighbours select the right one (the comparison is strict).
"""
from __future__ import annotations

import numpy as np

INF = float("inf")


def godunov1(left: float, right: float, rd: float):
    """eq. 1dgod: min(left, right) + r Delta, and the flow-direction wind of
    the neighbour used (+1 left, -1 right; ties go right)."""
    if left < right:
        return left + rd, 1
    return right + rd, -1


def fsm1(u, w, fixed, rd, max_sweeps=10000):
    """FSM on a 1D grid (Sec. 1.1): Gauss-Seidel sweeps left to right, then
    right to left, and so on, u = min(u, u~) at every free node, one-sided
    at the ends (a missing neighbour is +inf), until a sweep changes
    nothing.  u, w are updated in place; returns the number of sweeps."""
    n = len(u)
    s = 0
    while s < max_sweeps:
        order = range(n) if s % 2 == 0 else range(n - 1, -1, -1)
        changed = False
        for m in order:
            if fixed[m]:
                continue
            left = u[m - 1] if m > 0 else INF
            right = u[m + 1] if m < n - 1 else INF
            ut, wt = godunov1(left, right, rd[m])
            if ut < u[m]:
                u[m] = ut
                w[m] = wt
                changed = True
        s += 1
        if not changed:
            break
    return s


def coarse_fsm(N, H, r_coarse, g0, gN):
    """Step 1: FSM on the coarse grid with Gamma = {X_0, X_N}: U^0, W^0."""
    U = np.full(N + 1, INF)
    W = np.zeros(N + 1, dtype=int)
    fixed = np.zeros(N + 1, dtype=bool)
    U[0], U[N] = g0, gN
    fixed[0] = fixed[N] = True
    fsm1(U, W, fixed, [r * H for r in r_coarse])
    return U, W


def fine_solve(i, U, W, N, M, h, r_fine, g0, gN, inflow_fixed):
    """Steps 2 and 3 on subinterval i: an end node that is X_0 or X_N keeps
    g; an end node where the coarse wind points into the subinterval
    (W_i = +1 at the left end, W_{i+1} = -1 at the right end) takes U with
    its wind W, held fixed if inflow_fixed else free to decrease (the
    reading of the 2D/3D method); every other node starts at +inf.  Returns
    the fine values and winds of the subinterval's M + 1 nodes."""
    u = np.full(M + 1, INF)
    w = np.zeros(M + 1, dtype=int)
    fixed = np.zeros(M + 1, dtype=bool)
    rd = [r_fine[i * M + m] * h for m in range(M + 1)]
    if i == 0:
        u[0], fixed[0] = g0, True
    elif W[i] == 1:
        u[0], w[0], fixed[0] = U[i], 1, inflow_fixed
    if i == N - 1:
        u[M], fixed[M] = gN, True
    elif W[i + 1] == -1:
        u[M], w[M], fixed[M] = U[i + 1], -1, inflow_fixed
    fsm1(u, w, fixed, rd)
    return u, w


def choose_fine(uL, wL, uR, wR):
    """Step 3's choice at an interior coarse node X_i between the value of
    subinterval i-1 (its right end: uL, wL) and of subinterval i (its left
    end: uR, wR): both winds +1 (flow left to right) take the left
    subinterval's, both -1 the right one's, otherwise the smaller (ties to
    the left one); the wind goes with the value."""
    if wL == 1 and wR == 1:
        return uL, wL
    if wL == -1 and wR == -1:
        return uR, wR
    return (uL, wL) if uL <= uR else (uR, wR)


def dd1(r, N, M, theta, max_iter=50, tol=0.0, g0=0.0, gN=0.0, inflow_fixed=False, max_coarse_sweeps=1000):
    """The 1D method of Sec. 3.1 on (0, 1) with u(0) = g0, u(1) = gN.
    r: slowness as a function of x (vectorised).  Returns a dict with the
    coarse iterates U^k, W^k (k = 0, 1, ...), the pre-causal-sweep values of
    every Step 4, the fine values u^k at the coarse nodes and their winds,
    the patched fine solutions, and the overall fine solution u^f."""
    H = 1.0 / N
    h = H / M
    xf = np.arange(N * M + 1) * h
    rf = np.asarray(r(xf), dtype=float)
    rc = rf[::M]
    U, W = coarse_fsm(N, H, rc, g0, gN)
    hist = {"U": [U.copy()], "W": [W.copy()], "Upre": [], "uk": [], "wk": [], "ufine": [], "resid": []}
    for k in range(max_iter):
        # Steps 2-3: every subinterval, then the value at each coarse node
        fine = [fine_solve(i, U, W, N, M, h, rf, g0, gN, inflow_fixed) for i in range(N)]
        uk = np.zeros(N + 1)
        wk = np.zeros(N + 1, dtype=int)
        uk[0], uk[N] = g0, gN
        for i in range(1, N):
            uk[i], wk[i] = choose_fine(fine[i - 1][0][M], fine[i - 1][1][M], fine[i][0][0], fine[i][1][0])
        ufine = np.concatenate([fine[i][0][:M] for i in range(N)] + [[gN]])
        ufine[0::M] = uk
        # Step 4: C^k once from U^k, then FSM-style sweeps with the weighted
        # update from U = +inf (X_0, X_N fixed), until a sweep changes nothing
        Ck = np.full(N + 1, np.nan)
        for i in range(1, N):
            Ck[i] = godunov1(U[i - 1], U[i + 1], rc[i] * H)[0]
        Un = np.full(N + 1, INF)
        Wn = wk.copy()
        Un[0], Un[N] = g0, gN
        for s in range(max_coarse_sweeps):
            order = range(1, N) if s % 2 == 0 else range(N - 1, 0, -1)
            changed = False
            for i in order:
                Ut, Wt = godunov1(Un[i - 1], Un[i + 1], rc[i] * H)
                if W[i] == wk[i] == Wt and np.isfinite(Ut) and np.isfinite(Ck[i]):
                    v = theta * Ut + uk[i] - theta * Ck[i]
                else:
                    v = uk[i]
                if v != Un[i]:
                    Un[i] = v
                    changed = True
            if not changed:
                break
        hist["Upre"].append(Un.copy())
        # the causal sweep, left to right and then right to left
        for order in (range(1, N), range(N - 1, 0, -1)):
            for i in order:
                if Wn[i] == 1 and Un[i] < Un[i - 1]:
                    Un[i] = Un[i - 1]
                if Wn[i] == -1 and Un[i] < Un[i + 1]:
                    Un[i] = Un[i + 1]
        d = np.abs(Un - U)
        d[np.isinf(Un) & np.isinf(U)] = 0.0
        U, W = Un, Wn
        hist["U"].append(U.copy())
        hist["W"].append(W.copy())
        hist["uk"].append(uk)
        hist["wk"].append(wk)
        hist["ufine"].append(ufine)
        hist["resid"].append(float(np.max(d)))
        if hist["resid"][-1] <= tol:
            break
    # the overall fine solution on the whole fine grid
    uf = np.full(N * M + 1, INF)
    wf = np.zeros(N * M + 1, dtype=int)
    fx = np.zeros(N * M + 1, dtype=bool)
    uf[0], uf[-1] = g0, gN
    fx[0] = fx[-1] = True
    fsm1(uf, wf, fx, rf * h)
    hist["uf"] = uf
    hist["x_coarse"] = xf[::M]
    return hist
