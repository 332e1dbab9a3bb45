"""GPU parity (bitwise with the oracle in the same precision) on degenerate
placements of Gamma: none at all, point sources exactly on subdomain corners
and interfaces (where up to four subdomains reconcile a node and the Step 2
inflow test sees Gamma on the boundary), a whole interface line, and a whole
coarse lattice line, in 2D and 3D; iterates and converged results.  Also a
100:1-contrast medium of thin walls (many sweeps, the sweep cap) and the
fp32 input domain."""
import numpy as np
import pytest

import oracle
from paper_1805_04198_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1805_04198_amd as E  # noqa: E402


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def gpu_inputs(p, dtype):
    return dev(p.r, dtype), torch.from_numpy(p.gamma_idx.astype(np.int64)).cuda(), dev(p.gamma_val, dtype)


def same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


def run(n, h, r, gidx, gval, S, M, dtype, theta, max_iter, tol):
    gidx = np.asarray(gidx, np.int64)
    gval = np.asarray(gval, np.float64)
    G = E.dd_solve(dev(r, dtype), torch.from_numpy(gidx).cuda(), dev(gval, dtype), h, S, M, theta=theta, tol=tol,
                   max_iter=max_iter)
    O = oracle.dd(n, h, r, gidx, gval, S, M, theta=theta, tol=tol, max_iter=max_iter, dtype=dtype)
    d = len(n)
    U = G["U"].cpu().numpy().reshape(-1)
    assert same(U, O["U"])
    assert same(E.decode_winds(G["W"].cpu().numpy(), d), O["W"])
    if O["iterations"] > 0:
        assert same(G["u"].cpu().numpy().reshape(-1), O["u"])
    assert G["iterations"] == O["iterations"] and G["converged"] == O["converged"]
    assert G["fine_updates"] == O["fine_updates"] and G["coarse_updates"] == O["coarse_updates"]
    return G, O


def sources_2d(n, S, M, kind):
    li = lambda i, j: W.linear_index(n, i, j)
    if kind == "none":
        return [], []
    if kind == "corners":   # subdomain corners (shared by four subdomains)
        pts = [li(S, S), li(2 * S, S), li(0, 0), li(n[0] - 1, n[1] - 1)]
    elif kind == "interfaces":   # on interface lines, off the corners and off the lattice
        pts = [li(S, 3), li(S + 5, S), li(2 * S, n[1] - 2)]
    elif kind == "line":   # a whole interface line
        pts = [li(S, j) for j in range(n[1])]
    else:   # a whole line of the main coarse lattice, inside a subdomain
        pts = [li(i, M) for i in range(n[0])]
    pts = sorted(set(pts))
    vals = np.random.default_rng(len(pts)).uniform(0.0, 0.02, len(pts))
    return pts, vals


KINDS = ["none", "corners", "interfaces", "line", "lattice_line"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind", KINDS)
def test_gamma_placements_2d(kind, dtype):
    n, S, M = (97, 65), 32, 8
    p = W.random_problem(43, n, S, M, kind="fourier")
    gidx, gval = sources_2d(n, S, M, kind)
    print(f"2D gamma={kind} dtype={np.dtype(dtype).name}", flush=True)
    run(n, p.h, p.r, gidx, gval, S, M, dtype, 0.25, 3, 0.0)
    tol = 1e-12 if dtype == np.float64 else 1e-6
    G, O = run(n, p.h, p.r, gidx, gval, S, M, dtype, 0.25, 300, tol)
    assert O["converged"]
    if kind == "none":
        assert O["iterations"] == 1 and np.all(np.isinf(O["u"]))


@pytest.mark.parametrize("kind", ["none", "corners", "line"])
def test_gamma_placements_3d(kind):
    n, S, M = (17, 25, 17), 8, 4
    p = W.random_problem(44, n, S, M, kind="blocks")
    li = lambda i, j, k: W.linear_index(n, i, j, k)
    if kind == "none":
        gidx, gval = [], []
    elif kind == "corners":
        gidx = sorted({li(8, 8, 8), li(0, 16, 8), li(16, 24, 16)})
        gval = [0.0, 0.01, 0.02]
    else:
        gidx = sorted(li(8, j, 4) for j in range(n[1]))
        gval = np.zeros(len(gidx))
    print(f"3D gamma={kind}", flush=True)
    run(n, p.h, p.r, gidx, gval, S, M, np.float64, 0.3, 2, 0.0)
    G, O = run(n, p.h, p.r, gidx, gval, S, M, np.float64, 0.3, 200, 1e-12)
    assert O["converged"]


# ---------------------------------------------------------------------------
# high contrast: thin walls 100 times slower than the background
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,theta,tol,max_fine", [
    (np.float64, 0.25, 1e-12, 256),   # to convergence (38 iterations)
    (np.float32, 0.25, 1e-6, 256),    # to convergence (24 iterations)
    (np.float64, 0.25, 0.0, 16),      # every subdomain reaches the sweep cap
])
def test_walls_100_to_1_bitwise(dtype, theta, tol, max_fine):
    """100:1 walls with alternating gaps (workloads.barriers): the first
    arrival snakes through every subdomain, so the subdomain sweeps change x
    direction once per wall (about 30 sweeps per subdomain and iteration).
    Bitwise against the oracle in the run's precision, to convergence, and
    with a sweep cap of 16 that every subdomain hits."""
    p = W.barriers(129, 64, 16)
    max_iter = 400 if tol > 0 else 3
    print(f"walls dtype={np.dtype(dtype).name} theta={theta} tol={tol} max_fine={max_fine}", flush=True)
    r, gi, gv = gpu_inputs(p, dtype)
    G = E.dd_solve(r, gi, gv, p.h, p.S, p.M, theta=theta, tol=tol, max_iter=max_iter,
                   max_fine_sweeps=max_fine)
    O = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=theta, tol=tol,
                  max_iter=max_iter, max_fine_sweeps=max_fine, dtype=dtype)
    assert G["iterations"] == O["iterations"]
    assert G["fine_updates"] == O["fine_updates"] and G["coarse_updates"] == O["coarse_updates"]
    u = G["u"].cpu().numpy().reshape(-1)
    assert np.array_equal(u, O["u"], equal_nan=True)
    if max_fine == 16:
        tiles = ((p.n[0] - 1) // p.S) ** 2
        assert O["fine_updates"] >= max_iter * tiles * 16 * ((p.S + 1) ** 2 - 1)
    if tol > 0:
        assert G["converged"]
        uf, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val)
        bound = (1e-10 if dtype == np.float64 else 2e-5) * np.max(uf)
        assert np.max(np.abs(u.astype(np.float64) - uf)) <= bound


def test_fp32_slowness_below_the_square_root_domain_is_rejected():
    """fp32 runs need r h >= 2^-40 (the exact fp32 square root of the local
    solve is built for arguments >= 2^-96); smaller r is refused, fp64 runs
    take it."""
    p = W.random_problem(30, (33, 33), 8, 4)
    tiny = p.r * 1e-12  # r h ~ 3e-14 < 2^-40 ~ 9.1e-13
    for fn in ("dd", "solve"):
        _, gi, gv32 = gpu_inputs(p, np.float32)
        r32 = dev(tiny, np.float32)
        with pytest.raises(E.EikError) as ei:
            if fn == "dd":
                E.dd_solve(r32, gi, gv32, p.h, 8, 4, max_iter=1)
            else:
                E.solve(r32, gi, gv32, p.h)
        assert ei.value.status == E.EIK_ERR_UNSUPPORTED
    r64 = dev(tiny, np.float64)
    _, gi, gv64 = gpu_inputs(p, np.float64)
    E.dd_solve(r64, gi, gv64, p.h, 8, 4, max_iter=1)
