"""Sec. 4's model problem, evaluated as the paper writes it (eq. modelprob
with the boundary conditions eqs. modelBC1 and modelBC2).

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).

Omega = [0, 1] x [0, H], r = 1, Gamma = the bottom edge and the left edge,
u = sqrt(x^2 + y^2) on Gamma, H = 1/N, h = H/M.  The coarse nodes are
X_{i,j} = (iH, jh), i = 0..N, j = 0..M (every fine row of each vertical
coarse line).  The coarse solver looks only left and down:
    C_H(U_{i-1,j}, U_{i,j-M}) = the two-sided Godunov value of a = U_{i-1,j}
                                and b = U_{i,0} (one-sided min + H when
                                |a - b| >= H) for j = M,
                              = U_{i-1,j} + H for j < M (no node below),
U^0_{i,j} = C_H(U^0_{i-1,j}, U^0_{i,j-M}), and for k >= 0
    U^{k+1}_{i,j} = theta^{k+1}_{i,j} [C_H(U^{k+1}_{i-1,j}, U^{k+1}_{i,j-M})
                    - C_H(U^k_{i-1,j}, U^k_{i,j-M})] + u^k_{i,j}
with U_{0,j} = u^f_{0,j} and U_{i,0} = u^f_{i,0} at every iteration.  u^k_{i,j}
is the fine solution at (iH, jh) of the subdomain [(i-1)H, iH] x [0, H],
solved by FSM with its bottom row on Gamma and its left column held at
U^k_{i-1,j} (the boundary values the proof of Theorem exactness uses: the
characteristics all run up and to the right, so the left column is inflow
and the other two sides are outflow, solved one-sidedly).  The correction
is applied at every node: the winds always agree here.
"""
from __future__ import annotations

import math

import numpy as np

from . import fsm as _fsm  # the oracle FSM of Sec. 1.1
from . import theta_damped as _theta_damped  # eq. thetaest


def c_h(a: float, b: float, H: float) -> float:
    """The coarse Godunov value (Sec. 3.2's C_H with r = 1): two-sided when
    |a - b| < H, else min(a, b) + H."""
    d = a - b
    if abs(d) < H:
        t = H * H
        t = t + t
        t = t - d * d
        return ((a + b) + math.sqrt(t)) * 0.5
    return (a if a < b else b) + H


class ModelStrip:
    def __init__(self, N: int, M: int):
        self.N, self.M = N, M
        self.H = 1.0 / N
        self.h = self.H / M
        self.n = (N * M + 1, M + 1)
        nodes, vals = [], []
        for i in range(self.n[0]):
            nodes.append(i)                      # bottom row j = 0
            vals.append(i * self.h)
        for j in range(1, self.n[1]):
            nodes.append(self.n[0] * j)          # left column i = 0
            vals.append(j * self.h)
        order = np.argsort(nodes)
        self.gidx = np.asarray(nodes, dtype=np.int64)[order]
        self.gval = np.asarray(vals, dtype=np.float64)[order]
        uf, _ = _fsm(self.n, self.h, np.ones(self.n[::-1]), self.gidx, self.gval)
        uf = uf.reshape(self.n[::-1])
        # u^f at the coarse nodes: [i, j]
        self.uf = np.array([[uf[j, i * M] for j in range(M + 1)] for i in range(N + 1)])
        self.uf_grid = uf

    def ch(self, U, i, j):
        """C_H(U_{i-1,j}, U_{i,j-M}) of the model problem."""
        if j == self.M:
            return c_h(U[i - 1, j], U[i, 0], self.H)
        return U[i - 1, j] + self.H

    def coarse_init(self):
        U = np.zeros((self.N + 1, self.M + 1))
        U[0, :] = self.uf[0, :]
        U[:, 0] = self.uf[:, 0]
        for i in range(1, self.N + 1):
            for j in range(1, self.M + 1):
                U[i, j] = self.ch(U, i, j)
        return U

    def fine(self, U):
        """u^k_{i,j}, i = 1..N: the subdomain solves with the left column
        held at U_{i-1, 1..M} and the bottom row on Gamma."""
        M, h = self.M, self.h
        u = np.zeros((self.N + 1, M + 1))
        u[0, :] = self.uf[0, :]
        n = (M + 1, M + 1)
        for i in range(1, self.N + 1):
            x0 = (i - 1) * M
            nodes = list(range(M + 1)) + [n[0] * j for j in range(1, M + 1)]
            vals = [(x0 + l) * h for l in range(M + 1)] + [U[i - 1, j] for j in range(1, M + 1)]
            order = np.argsort(nodes)
            us, _ = _fsm(n, h, np.ones((M + 1, M + 1)), np.asarray(nodes, np.int64)[order],
                         np.asarray(vals)[order])
            u[i, :] = us.reshape(M + 1, M + 1)[:, M]
        return u

    def run(self, theta, kmax, theta_fn=None):
        """Iterates U^0..U^kmax and u^0..u^{kmax-1}.  theta: a constant, or
        theta_fn(k, i, j, U_new, U_old, u_old) -> theta^{k}_{i,j} evaluated
        when U^k_{i,j} is formed (the upwind values U^k_{i-1,.} are final by
        then)."""
        Us = [self.coarse_init()]
        us = []
        for k in range(kmax):
            Uo = Us[-1]
            uo = self.fine(Uo)
            us.append(uo)
            Un = np.zeros_like(Uo)
            Un[0, :] = self.uf[0, :]
            Un[:, 0] = self.uf[:, 0]
            for i in range(1, self.N + 1):
                for j in range(1, self.M + 1):
                    th = theta if theta_fn is None else theta_fn(k + 1, i, j, Un, Uo, uo)
                    Un[i, j] = th * (self.ch(Un, i, j) - self.ch(Uo, i, j)) + uo[i, j]
            Us.append(Un)
        return Us, us

    def Mbar(self, i, j, Unew, Uold, uold):
        """M-bar^k_{i,j} = (u^f - u^{k-1}) / (C_H(U^k nbrs) - C_H(U^{k-1}
        nbrs)) (Sec. 4.1, the bound of Theorem choosetheta), NaN when the
        denominator is 0."""
        den = self.ch(Unew, i, j) - self.ch(Uold, i, j)
        if den == 0.0:
            return float("nan")
        return (self.uf[i, j] - uold[i, j]) / den

    def errors(self, Us):
        return [float(np.max(np.abs(U[1:, 1:] - self.uf[1:, 1:]))) for U in Us]

    def run_estimate(self, kmax, theta0=0.1, omega=(1.0, 1.0, 1.0), gamma=0.75, delta=0.01, x0=0.9):
        """The iteration with the weights of Sec. 4.2: theta^k_{i,j} from
        eq. secthetaest, (u^{k-1} - u^{k-2}) over the omega-weighted mean of
        the increments of C_H at the node, s = 0 being the current one
        (C_H(U^k nbrs) - C_H(U^{k-1} nbrs)) and s = 1, 2 the two before,
        then damped by eq. thetaest; theta0 where the history is too short
        or the denominator is 0 (the reading of the DD solver).  Returns
        the iterates U^0..U^kmax."""
        def c_all(U):
            C = np.full_like(U, np.nan)
            for i in range(1, self.N + 1):
                for j in range(1, self.M + 1):
                    C[i, j] = self.ch(U, i, j)
            return C

        Us = [self.coarse_init()]
        us, Cs = [], [c_all(Us[0])]
        wsum = (omega[0] + omega[1]) + omega[2]
        for _ in range(kmax):
            Uo = Us[-1]
            uo = self.fine(Uo)
            us.append(uo)
            Un = np.zeros_like(Uo)
            Un[0, :] = self.uf[0, :]
            Un[:, 0] = self.uf[:, 0]
            for i in range(1, self.N + 1):
                for j in range(1, self.M + 1):
                    cnew, cold = self.ch(Un, i, j), self.ch(Uo, i, j)
                    th = theta0
                    if len(us) >= 2 and len(Cs) >= 3:
                        num = us[-1][i, j] - us[-2][i, j]
                        den = (omega[0] * (cnew - cold) + omega[1] * (Cs[-1][i, j] - Cs[-2][i, j])
                               + omega[2] * (Cs[-2][i, j] - Cs[-3][i, j])) / wsum
                        if den != 0.0 and math.isfinite(den) and math.isfinite(num):
                            th = _theta_damped(num / den, gamma, delta, x0)
                    Un[i, j] = th * (cnew - cold) + uo[i, j]
            Us.append(Un)
            Cs.append(c_all(Un))
        return Us
