"""Autotuner for batched DD solves: per problem size, the subdomain side S,
the coarse spacing M = H/h and the weight theta that give the shortest
time to solution.

For every distinct grid shape in a batch it times eik_dd_solve on the first
problem of that shape for each admissible candidate (S from `sides`, M from
`spacings` with S % M == 0, lattices of at most 65 nodes per axis, theta
from `thetas`), skips candidates that do not reach the tolerance within
`max_iter` iterations, and keeps the fastest.  The choice changes the
iterates (another partition or weight), not the target: every accepted run
has converged to the same tolerance.  Timing uses the library's device time
of the solve after one warm-up call per candidate."""
from __future__ import annotations

import paper_1805_04198_amd as E

SIDES = (32, 64)
SPACINGS = (16, 32, 64)
THETAS = (0.1, 0.25)
MAX_NODES = 65


def candidates(n, sides=SIDES, spacings=SPACINGS, thetas=THETAS):
    out = []
    for S in sides:
        if any((m - 1) % S for m in n) or S + 1 > MAX_NODES:
            continue
        for M in spacings:
            if M > S or S % M or any((m - 1) // M + 1 > MAX_NODES for m in n):
                continue
            for th in thetas:
                out.append((S, M, th))
    return out


def tune(rs, gammas, hs, tol=1e-6, max_iter=300, sides=SIDES, spacings=SPACINGS, thetas=THETAS):
    """rs, gammas, hs as for dd_solve_batch.  Returns ({shape: (S, M,
    theta)}, table of (shape, S, M, theta, converged, iterations, ms))."""
    best, table = {}, []
    seen = {}
    for i, r in enumerate(rs):
        shape = tuple(r.shape)
        if shape not in seen:
            seen[shape] = i
    for shape, i in seen.items():
        n = shape[::-1]
        pick = None
        for S, M, th in candidates(n, sides, spacings, thetas):
            kw = dict(theta=th, tol=tol, max_iter=max_iter)
            E.dd_solve(rs[i], gammas[i][0], gammas[i][1], hs[i], S, M, **kw)
            R = E.dd_solve(rs[i], gammas[i][0], gammas[i][1], hs[i], S, M, **kw)
            table.append((shape, S, M, th, R["converged"], R["iterations"], R["ms_total"]))
            if R["converged"] and (pick is None or R["ms_total"] < pick[1]):
                pick = ((S, M, th), R["ms_total"])
        if pick is None:
            raise RuntimeError(f"no candidate converged for grid {n}")
        best[shape] = pick[0]
    return best, table


def apply(rs, best):
    """Per-problem S, M, theta lists from a tuning result."""
    S, M, th = zip(*[best[tuple(r.shape)] for r in rs])
    return list(S), list(M), list(th)
