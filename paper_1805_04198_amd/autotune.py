"""Autotuner for batched DD solves.

Two searches, both timed with the library's own device time after one
warm-up call per candidate:

  * per problem size, the partition: subdomain side S and coarse spacing
    M = H/h (S from `sides`, M from `spacings` with S % M == 0 and lattices
    of at most 65 nodes per axis), timed as one batched solve of up to
    `per_shape` problems of that size (a small batch, as the problems will
    run: a partition with more subdomains fills the device better alone but
    costs more iterations and work once the device is full), at the
    caller's weight theta.  Another partition changes the iterates but not
    the target: candidates that do not reach the tolerance within
    `max_iter` iterations are skipped, so every accepted run has converged
    to the same tolerance.  The weight is not searched: it changes what the
    iteration computes, and large weights make it unstable (Sec. 4), so it
    stays the caller's choice.
  * for the whole batch, the launch schedule of Steps 3 and 4: one block
    per subdomain / lattice box ("stream") or resident grids whose blocks take
    the boxes from a counter ("persistent"), with as many blocks per compute
    unit as fit or fewer (`PERSISTENT_BLOCKS`; fewer blocks take more boxes
    each).  The schedule changes nothing in the results (each box is
    computed the same way), only the time.
"""
from __future__ import annotations

import paper_1805_04198_amd as E

SIDES = (32, 64)
SPACINGS = (16, 32, 64)
LAUNCHES = ("stream", "persistent")
PERSISTENT_BLOCKS = (0, 1, 2)  # resident blocks per compute unit; 0 = as many as fit
MAX_NODES = 65


def candidates(n, sides=SIDES, spacings=SPACINGS):
    out = []
    for S in sides:
        if any((m - 1) % S for m in n) or S + 1 > MAX_NODES:
            continue
        for M in spacings:
            if M > S or S % M or any((m - 1) // M + 1 > MAX_NODES for m in n):
                continue
            out.append((S, M))
    return out


def tune(rs, gammas, hs, theta=0.1, tol=1e-6, max_iter=300, sides=SIDES, spacings=SPACINGS, per_shape=4):
    """rs, gammas, hs as for dd_solve_batch.  Returns ({shape: (S, M)},
    table of (shape, S, M, converged, iterations, ms)); iterations: the
    slowest problem of the shape's sample."""
    best, table = {}, []
    seen = {}
    for i, r in enumerate(rs):
        seen.setdefault(tuple(r.shape), []).append(i)
    for shape, idx in seen.items():
        n = shape[::-1]
        idx = idx[:per_shape]
        sr = [rs[i] for i in idx]
        sg = [gammas[i] for i in idx]
        sh = [hs[i] for i in idx]
        pick = None
        for S, M in candidates(n, sides, spacings):
            kw = dict(theta=theta, tol=tol, max_iter=max_iter)
            E.dd_solve_batch(sr, sg, sh, S, M, **kw)
            B = E.dd_solve_batch(sr, sg, sh, S, M, **kw)
            conv = all(b["converged"] for b in B)
            ms = B[0]["ms_total"]
            table.append((shape, S, M, conv, max(b["iterations"] for b in B), ms))
            if conv and (pick is None or ms < pick[1]):
                pick = ((S, M), ms)
        if pick is None:
            raise RuntimeError(f"no candidate converged for grid {n}")
        best[shape] = pick[0]
    return best, table


def launch_candidates(launches=LAUNCHES, blocks=PERSISTENT_BLOCKS):
    """(launch, persistent_blocks) pairs to time: the stream schedule once,
    the persistent one per grid size."""
    out = []
    for lm in launches:
        for b in (blocks if lm == "persistent" else (0,)):
            out.append((lm, b))
    return out


def tune_launch(rs, gammas, hs, S, M, theta=0.1, tol=1e-6, max_iter=600, launches=LAUNCHES,
                blocks=PERSISTENT_BLOCKS):
    """The fastest launch schedule of the whole batch with partitions S, M
    (lists).  Returns ((launch, persistent_blocks), {"launch/blocks": ms})."""
    times = {}
    for lm, b in launch_candidates(launches, blocks):
        kw = dict(theta=theta, tol=tol, max_iter=max_iter, launch=lm, persistent_blocks=b)
        E.dd_solve_batch(rs, gammas, hs, S, M, **kw)
        B = E.dd_solve_batch(rs, gammas, hs, S, M, **kw)
        times[(lm, b)] = B[0]["ms_total"]
    best = min(times, key=times.get)
    return best, {f"{lm}/{b}": t for (lm, b), t in times.items()}


def apply(rs, best):
    """Per-problem S, M lists from a tuning result."""
    S, M = zip(*[best[tuple(r.shape)] for r in rs])
    return list(S), list(M)
