"""Seeded synthetic inputs for the Eikonal domain-decomposition solver.

This module only *generates inputs*: slowness fields r_eps sampled on the
nodes of a uniform grid on [0,1]^d, the boundary set Gamma (linear node
indices, sorted and unique) with its data g, and the partition parameters.
It contains none of the solver's arithmetic, so both the CPU oracle's tests
and the GPU path draw from it.

Layout: x is the fastest axis.  A 2D field has numpy shape (n1, n0) and node
(i, j) sits at linear index i + n0*j; a 3D field has shape (n2, n1, n0) and
node (i, j, k) sits at i + n0*(j + n1*k).

Every field is produced in float64 with numpy's default_rng(seed); an fp32
run uses the float32 rounding of the same field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One boundary value problem |grad u| = r on [0,1]^d, u = g on Gamma,
    with its two-scale partition (Section 3.2 of the paper: subdomain side S
    and coarse spacing M = H/h, both in fine cells)."""

    name: str
    n: tuple                   # nodes per axis (x first)
    h: float                   # fine spacing
    r: np.ndarray              # float64 slowness, shape n[::-1]
    gamma_idx: np.ndarray      # int64, sorted unique linear indices
    gamma_val: np.ndarray      # float64 boundary data g
    S: int = 0                 # subdomain side in fine cells
    M: int = 0                 # coarse spacing H/h in fine cells
    theta: float = 0.5         # parareal weight
    tol: float = 1e-12         # stop when max|U^{k+1}-U^k| < tol

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def r_as(self, dtype) -> np.ndarray:
        return np.ascontiguousarray(self.r.astype(dtype))

    def g_as(self, dtype) -> np.ndarray:
        return np.ascontiguousarray(self.gamma_val.astype(dtype))


def _coords(n, h):
    """Node coordinates as float64 arrays broadcast to the field shape."""
    axes = [np.arange(m, dtype=np.float64) * h for m in n]
    # meshgrid with indexing='ij' over reversed axes gives shape n[::-1]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    return grids[::-1]  # x, y[, z]


def linear_index(n, *ijk) -> int:
    idx = 0
    stride = 1
    for a, c in enumerate(ijk):
        idx += int(c) * stride
        stride *= int(n[a])
    return idx


def _gamma(n, nodes, vals):
    idx = np.array([linear_index(n, *c) for c in nodes], dtype=np.int64)
    val = np.asarray(vals, dtype=np.float64)
    order = np.argsort(idx, kind="stable")
    idx, val = idx[order], val[order]
    keep = np.ones(len(idx), dtype=bool)
    keep[1:] = idx[1:] != idx[:-1]
    return idx[keep], val[keep]


# ---------------------------------------------------------------------------
# the workloads the solver is measured and checked on
# ---------------------------------------------------------------------------

def config1() -> Problem:
    """129^2, h = 1/128, 4x4 subdomains (S = 32), H = 1/16 (M = 8).
    r = 1 + 0.5 sin(2 pi x / eps) sin(2 pi y / eps), eps = 1/16; point source
    g = 0 at node (64, 64) = (0.5, 0.5); theta = 0.5; fp64 to 1e-12."""
    n = (129, 129)
    h = 1.0 / 128
    x, y = _coords(n, h)
    eps = 1.0 / 16
    r = 1.0 + 0.5 * np.sin(2 * np.pi * x / eps) * np.sin(2 * np.pi * y / eps)
    gi, gv = _gamma(n, [(64, 64)], [0.0])
    return Problem("c1_129sq_S32_M8", n, h, r, gi, gv, S=32, M=8, theta=0.5, tol=1e-12)


def config2_slowness(n, h, seed=2):
    """r0 + a_eps on a 2D grid: r0 = 1 + 0.3 exp(-|x-(0.3,0.7)|^2/0.05) plus
    32 seeded random Fourier modes (wavenumber in [32,128], direction and
    phase uniform, amplitude N(0, 0.02)), floored at 0.2."""
    x, y = _coords(n, h)
    rng = np.random.default_rng(seed)
    kmag = rng.uniform(32.0, 128.0, 32)
    ang = rng.uniform(0.0, 2 * np.pi, 32)
    phi = rng.uniform(0.0, 2 * np.pi, 32)
    amp = rng.normal(0.0, 0.02, 32)
    r0 = 1.0 + 0.3 * np.exp(-((x - 0.3) ** 2 + (y - 0.7) ** 2) / 0.05)
    a = np.zeros_like(x)
    for m in range(32):
        a += amp[m] * np.cos(2 * np.pi * kmag[m] * (x * np.cos(ang[m]) + y * np.sin(ang[m])) + phi[m])
    return np.maximum(r0 + a, 0.2)


def config2(n_side: int = 1025, S: int = 64, M: int = 16) -> Problem:
    """1025^2, h = 1/1024, 16x16 subdomains (S = 64), H = 1/64 (M = 16);
    multiscale random-Fourier slowness; source = the whole left edge x = 0
    with g = 0; theta = 0.5."""
    n = (n_side, n_side)
    h = 1.0 / (n_side - 1)
    r = config2_slowness(n, h)
    nodes = [(0, j) for j in range(n_side)]
    gi, gv = _gamma(n, nodes, np.zeros(n_side))
    return Problem(f"c2_{n_side}sq_S{S}_M{M}", n, h, r, gi, gv, S=S, M=M, theta=0.5, tol=1e-12)


def config3(n_side: int = 257, S: int = 32, M: int = 8) -> Problem:
    """257^3, h = 1/256, 8^3 subdomains (S = 32), H = 1/32 (M = 8).
    r = (1 + 0.4 prod_i sin(2 pi x_i / eps)) * exp(0.1 z_b), eps = 1/32, with
    z_b a seeded N(0,1) draw per checkerboard block of side 1/16 (16 fine
    cells at n = 257).  Sources: node (64,64,64) with g = 0, and the off-node
    point (0.75, 0.6, 0.5) represented by its two nearest nodes along y with
    g = r(x0) * distance (the paper fixes values "on or near" the boundary)."""
    n = (n_side, n_side, n_side)
    h = 1.0 / (n_side - 1)
    x, y, z = _coords(n, h)
    eps = 1.0 / 32
    rng = np.random.default_rng(3)
    nb = 16
    zb = rng.normal(0.0, 1.0, (nb, nb, nb))  # [bx][by][bz]
    cell = max(1, (n_side - 1) // 16)
    bi = np.minimum(np.arange(n_side) // cell, nb - 1)
    # field shape is (nz, ny, nx): index zb[bx, by, bz]
    blk = zb[bi[None, None, :], bi[None, :, None], bi[:, None, None]]
    r = (1.0 + 0.4 * np.sin(2 * np.pi * x / eps) * np.sin(2 * np.pi * y / eps)
         * np.sin(2 * np.pi * z / eps)) * np.exp(0.1 * blk)
    x0 = (0.75, 0.6, 0.5)
    i0 = int(round(x0[0] * (n_side - 1)))
    k0 = int(round(x0[2] * (n_side - 1)))
    yf = x0[1] * (n_side - 1)
    jlo = int(math.floor(yf))
    bxi = min(int(x0[0] * (n_side - 1)) // cell, nb - 1)
    byi = min(int(x0[1] * (n_side - 1)) // cell, nb - 1)
    bzi = min(int(x0[2] * (n_side - 1)) // cell, nb - 1)
    r_x0 = (1.0 + 0.4 * math.sin(2 * math.pi * x0[0] / eps) * math.sin(2 * math.pi * x0[1] / eps)
            * math.sin(2 * math.pi * x0[2] / eps)) * math.exp(0.1 * zb[bxi, byi, bzi])
    c = n_side // 4
    nodes = [(c, c, c), (i0, jlo, k0), (i0, jlo + 1, k0)]
    vals = [0.0, r_x0 * (yf - jlo) * h, r_x0 * (jlo + 1 - yf) * h]
    gi, gv = _gamma(n, nodes, vals)
    return Problem(f"c3_{n_side}cube_S{S}_M{M}", n, h, r, gi, gv, S=S, M=M, theta=0.5, tol=1e-12)


# ---------------------------------------------------------------------------
# small seeded cases for parity tests
# ---------------------------------------------------------------------------

def random_media(n, h, seed, kind="fourier"):
    """A smooth positive random medium on the grid (float64)."""
    rng = np.random.default_rng(seed)
    xs = _coords(n, h)
    if kind == "const":
        return np.full(tuple(n[::-1]), float(rng.uniform(0.5, 2.0)))
    if kind == "blocks":
        nb = int(rng.integers(2, 6))
        vals = rng.choice([1.0, 2.0], size=(nb,) * len(n))
        idx = [np.minimum((c * nb).astype(np.int64), nb - 1) for c in xs]
        return vals[tuple(idx)]
    r = np.ones(tuple(n[::-1]))
    for _ in range(6):
        k = rng.uniform(1.0, 8.0, len(n))
        ph = rng.uniform(0, 2 * np.pi)
        amp = rng.uniform(0.05, 0.2)
        arg = sum(k[a] * 2 * np.pi * xs[a] for a in range(len(n))) + ph
        r = r + amp * np.sin(arg)
    return np.maximum(r, 0.2)


def random_problem(seed: int, n, S: int, M: int, n_src: int = 1,
                   kind: str = "fourier", edge: Optional[int] = None,
                   theta: float = 0.5) -> Problem:
    """A seeded small problem: random smooth (or blocky / constant) medium,
    n_src random node sources with g = 0, or a whole domain edge when
    `edge` is given (axis index; the x_axis = 0 face)."""
    n = tuple(int(v) for v in n)
    h = 1.0 / (n[0] - 1)
    r = random_media(n, h, seed, kind)
    rng = np.random.default_rng(seed + 1000)
    if edge is not None:
        grid = np.indices(n[::-1]).reshape(len(n), -1)[::-1].T  # (i, j[, k])
        nodes = [tuple(c) for c in grid if c[edge] == 0]
        vals = np.zeros(len(nodes))
    else:
        nodes = [tuple(int(rng.integers(0, m)) for m in n) for _ in range(n_src)]
        vals = rng.uniform(0.0, 0.05, n_src)
    gi, gv = _gamma(n, nodes, vals)
    return Problem(f"rand{seed}", n, h, r, gi, gv, S=S, M=M, theta=theta, tol=1e-12)


def barriers(n_side: int = 129, S: int = 64, M: int = 16, contrast: float = 100.0,
             spacing: int = 4) -> Problem:
    """A 100:1-contrast medium of thin slow walls: r = 1, except on the rows
    j = spacing, 2 spacing, ... (one node thick), where r = contrast.  Each
    wall has a gap of `spacing` nodes in every block of S columns: at the
    block's left end on even walls, at its right end on odd ones.  Crossing
    a wall costs contrast * h, going round it at most S * h, so inside every
    subdomain the first arrival snakes between the walls, and the sweeps
    must change x direction once per wall.  Source: node (0, 0), g = 0.  No
    randomness."""
    n = (n_side, n_side)
    h = 1.0 / (n_side - 1)
    r = np.ones((n_side, n_side))
    col = np.arange(n_side) % S
    for k, j in enumerate(range(spacing, n_side - 1, spacing)):
        gap = col < spacing if k % 2 == 0 else col >= S - spacing
        r[j, :] = np.where(gap, 1.0, contrast)
    gi, gv = _gamma(n, [(0, 0)], [0.0])
    return Problem(f"walls_{n_side}", n, h, r, gi, gv, S=S, M=M)


def model_strip(N: int, M: int) -> Problem:
    """The model problem of Section 4: Omega = [0,1] x [0,H], r = 1,
    Gamma = bottom and left edges, g = sqrt(x^2 + y^2); H = 1/N, h = 1/(NM).
    The subdomains are the coarse cells (S = M)."""
    n = (N * M + 1, M + 1)
    h = 1.0 / (N * M)
    r = np.ones((n[1], n[0]))
    nodes, vals = [], []
    for i in range(n[0]):
        nodes.append((i, 0))
        vals.append(i * h)
    for j in range(1, n[1]):
        nodes.append((0, j))
        vals.append(j * h)
    gi, gv = _gamma(n, nodes, vals)
    return Problem(f"strip_N{N}_M{M}", n, h, r, gi, gv, S=M, M=M)


def squares(n_side: int = 449, period: int = 8, S: int = 32, M: int = 32) -> Problem:
    """The squares medium of Sec. 5.3: r = 1 on the lines x = 0 or y = 0
    modulo the period eps, 2 elsewhere; source (0.5, 0.5), g = 0.  The paper
    uses h = 1/1400, eps = 7h, H = 1/14 and says r is 1 at every coarse node;
    here h = 1/(n-1), eps = period * h with H = M h a multiple of eps, so
    that the coarse nodes lie on the lines as stated (defaults: h = 1/448,
    eps = 8h = 1/56, H = 32h = 1/14)."""
    n = (n_side, n_side)
    h = 1.0 / (n_side - 1)
    i = np.arange(n_side)
    on = (i % period) == 0
    r = np.where(on[None, :] | on[:, None], 1.0, 2.0)
    c = (n_side - 1) // 2
    gi, gv = _gamma(n, [(c, c)], [0.0])
    return Problem(f"squares_{n_side}_eps{period}h", n, h, r, gi, gv, S=S, M=M, theta=0.25, tol=1e-12)


def config4(n_prob: int = 64, seed: int = 4, sizes=(257, 513, 1025, 2049)) -> list:
    """Batching workload: n_prob independent 2D problems, side lengths drawn
    uniformly from `sizes`, subdomains of 64^2 cells (S = 64).  Each problem
    has its own medium, the config-2 recipe with r0 = 1 and the wavenumber
    band [1/eps, 4/eps], eps drawn from {1/32, 1/64} (32 modes, phase and
    direction uniform, amplitude N(0, 0.02), floored at 0.2), and one random
    interior source node with g = 0.  H is not stated: M = 16 where the
    coarse lattices then have <= 65 nodes per axis (n <= 1025), else
    M = (n-1)/64 (M = 32 at n = 2049).  Per-problem generators come from
    SeedSequence(seed).spawn."""
    children = np.random.SeedSequence(seed).spawn(n_prob)
    out = []
    for i, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n_side = int(rng.choice(sizes))
        eps = float(rng.choice([1.0 / 32, 1.0 / 64]))
        n = (n_side, n_side)
        h = 1.0 / (n_side - 1)
        kmag = rng.uniform(1.0 / eps, 4.0 / eps, 32)
        ang = rng.uniform(0.0, 2 * np.pi, 32)
        phi = rng.uniform(0.0, 2 * np.pi, 32)
        amp = rng.normal(0.0, 0.02, 32)
        # sum_k amp_k cos(2 pi k (x cos a + y sin a) + phi), each mode split
        # into x and y factors: cos(X + Y) = cos X cos Y - sin X sin Y
        t = np.arange(n_side, dtype=np.float64) * h
        X = 2 * np.pi * np.outer(t, kmag * np.cos(ang))             # (nx, 32)
        Y = 2 * np.pi * np.outer(t, kmag * np.sin(ang)) + phi        # (ny, 32)
        a = (np.cos(Y) * amp) @ np.cos(X).T - (np.sin(Y) * amp) @ np.sin(X).T   # (ny, nx)
        r = np.maximum(1.0 + a, 0.2)
        src = (int(rng.integers(1, n_side - 1)), int(rng.integers(1, n_side - 1)))
        gi, gv = _gamma(n, [src], [0.0])
        M = 16 if (n_side - 1) // 16 + 1 <= 65 else (n_side - 1) // 64
        out.append(Problem(f"c4_{i}_{n_side}sq_eps{int(round(1 / eps))}", n, h, r, gi, gv, S=64, M=M,
                           theta=0.25, tol=1e-6))
    return out


@dataclasses.dataclass
class GradProblem:
    """The travel-time gradient workload: one slowness, many point sources,
    receivers, and the perturbed slowness the target times come from."""

    name: str
    n: tuple
    h: float
    r: np.ndarray              # slowness, shape n[::-1]
    r_perturbed: np.ndarray    # slowness of the synthetic observations
    sources: list              # node indices (g = 0 at each, one problem per source)
    receivers: np.ndarray      # node indices
    targets: np.ndarray        # (len(sources), len(receivers)) stand-in targets, see config5_problem


def config5_problem(n_side: int = 1025, n_src: int = 32, n_bumps: int = 8, seed: int = 5) -> GradProblem:
    """Differentiation workload: 1025^2, the config-1 slowness (eps = 1/16),
    32 distinct seeded top-edge sources, receivers at i = 2 + 4m on the
    bottom edge (256 at n = 1025), and a perturbed slowness r + sum of
    n_bumps Gaussian bumps 0.05 exp(-|x - c|^2 / (2 0.05^2)), centres
    uniform in [0.1, 0.9]^2.  The observations are meant to be the travel
    times through r_perturbed (the benchmark solves for them on the GPU);
    `targets` holds a stand-in that needs no solver: straight-ray times
    |x_r - x_s| times the mean of r_perturbed."""
    n = (n_side, n_side)
    h = 1.0 / (n_side - 1)
    x, y = _coords(n, h)
    eps = 1.0 / 16
    r = 1.0 + 0.5 * np.sin(2 * np.pi * x / eps) * np.sin(2 * np.pi * y / eps)
    rng = np.random.default_rng(seed)
    cols = np.sort(rng.choice(n_side, n_src, replace=False))
    centres = rng.uniform(0.1, 0.9, (n_bumps, 2))
    rp = r.copy()
    for cx, cy in centres:
        rp = rp + 0.05 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.05 ** 2))
    sources = [linear_index(n, int(i), n_side - 1) for i in cols]
    ri = np.arange(2, n_side - 1, 4)[:256]
    receivers = np.array([linear_index(n, int(i), 0) for i in ri], dtype=np.int64)
    mean_r = float(np.mean(rp))
    targets = np.array([[mean_r * h * float(np.hypot(ri_ - si, n_side - 1)) for ri_ in ri] for si in cols])
    return GradProblem(f"c5_{n_side}sq_{n_src}src", n, h, r, rp, sources, receivers, targets)


CONFIGS = {"c1": config1, "c2": config2, "c3": config3}
