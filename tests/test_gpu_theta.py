"""GPU parity of the Step 4 weight rules (estimated, reference, field):
every iterate bit-identical to the oracle in the same precision, in 2D and
3D, over enough iterations for the estimate to use its history (C^{k-2}
exists from the third iteration on)."""
import numpy as np
import pytest

import oracle
from paper_1805_04198_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1805_04198_amd as E  # noqa: E402


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


def show_diff(name, g, o):
    g = np.asarray(g).reshape(-1)
    o = np.asarray(o).reshape(-1)
    if g.dtype.kind == "f":
        bad = np.nonzero(~((g == o) | (np.isnan(g) & np.isnan(o))))[0]
    else:
        bad = np.nonzero(g != o)[0]
    return f"{name}: {len(bad)} mismatches, first {bad[:5]} gpu={g[bad[:5]]} oracle={o[bad[:5]]}"


def theta_ref_for(p, mode, dtype):
    if mode == "reference":
        uf, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, dtype=dtype)
        return uf
    if mode == "field":
        rng = np.random.default_rng(99)
        return rng.uniform(0.0, 0.6, p.r.size).astype(dtype)
    return None


def run_pair(p, dtype, theta, k, mode, tol=0.0):
    ref = theta_ref_for(p, mode, dtype)
    r = dev(p.r, dtype)
    gi = torch.from_numpy(p.gamma_idx.astype(np.int64)).cuda()
    gv = dev(p.gamma_val, dtype)
    G = E.dd_solve(r, gi, gv, p.h, p.S, p.M, theta=theta, tol=tol, max_iter=k, debug=True,
                   theta_mode=mode, theta_ref=None if ref is None else dev(ref, dtype))
    O = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=theta, tol=tol, max_iter=k,
                  dtype=dtype, theta_mode=mode, theta_ref=ref)
    return G, O


def compare(G, O, d):
    U = G["U"].cpu().numpy().reshape(-1)
    assert same(U, O["U"]), show_diff("U", U, O["U"])
    Wg = E.decode_winds(G["W"].cpu().numpy(), d)
    assert same(Wg, O["W"]), show_diff("W", Wg, O["W"])
    if O["iterations"] > 0:
        m = ~np.isnan(O["U"])
        up = G["Upre"].cpu().numpy().reshape(-1)
        assert same(up[m], O["Upre"][m]), show_diff("Upre", up[m], O["Upre"][m])
        u = G["u"].cpu().numpy().reshape(-1)
        assert same(u, O["u"]), show_diff("u", u, O["u"])
    assert G["iterations"] == O["iterations"]
    assert G["coarse_updates"] == O["coarse_updates"]
    assert G["fine_updates"] == O["fine_updates"]


CASES_2D = [
    dict(seed=60, n=(65, 65), S=16, M=8, nsrc=2, kind="fourier", theta=0.3),
    dict(seed=61, n=(129, 65), S=32, M=8, nsrc=1, kind="blocks", theta=0.5),
    dict(seed=62, n=(49, 97), S=16, M=4, nsrc=3, kind="fourier", theta=0.25),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", ["estimate", "reference", "field"])
@pytest.mark.parametrize("ci", range(len(CASES_2D)))
def test_theta_modes_2d_bitwise(ci, mode, dtype):
    c = CASES_2D[ci]
    p = W.random_problem(c["seed"], c["n"], c["S"], c["M"], n_src=c["nsrc"], kind=c["kind"])
    print(f"theta2d case={c} mode={mode} dtype={np.dtype(dtype).name}", flush=True)
    G, O = run_pair(p, dtype, c["theta"], 6, mode)
    compare(G, O, 2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_config1_estimate_to_convergence(dtype):
    p = W.config1()
    tol = 1e-12 if dtype == np.float64 else 1e-6
    print(f"config1 estimate dtype={np.dtype(dtype).name}", flush=True)
    G, O = run_pair(p, dtype, 0.5, 200, "estimate", tol=tol)
    assert G["converged"] and O["converged"]
    compare(G, O, 2)
    uf, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val)
    u = G["u"].cpu().numpy().reshape(-1).astype(np.float64)
    bound = (1e-10 if dtype == np.float64 else 2e-5) * np.max(uf)
    assert np.max(np.abs(u - uf)) <= bound


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_config2_estimate_first_iterations(dtype):
    """65 x 65 lattices: in fp64 Step 4's weight terms do not fit in LDS
    beside the lattice and are kept in global memory."""
    p = W.config2()
    print(f"config2 estimate {np.dtype(dtype).name} 4 iterations", flush=True)
    G, O = run_pair(p, dtype, 0.25, 4, "estimate")
    compare(G, O, 2)


@pytest.mark.parametrize("mode", ["estimate", "reference", "field"])
def test_theta_modes_fp64_65_node_lattices(mode):
    """129^2 with M = 2: 65 x 65 lattices, weight terms in global memory in
    fp64; single solve and the same problem in a batch, bitwise."""
    p = W.random_problem(63, (129, 129), 16, 2, n_src=2, kind="fourier")
    print(f"fp64 65-node lattices mode={mode}", flush=True)
    G, O = run_pair(p, np.float64, 0.3, 6, mode)
    compare(G, O, 2)
    ref = theta_ref_for(p, mode, np.float64)
    r = dev(p.r, np.float64)
    g = (torch.from_numpy(p.gamma_idx).cuda(), dev(p.gamma_val, np.float64))
    q = W.random_problem(64, (65, 65), 16, 8, n_src=1)
    rq = dev(q.r, np.float64)
    gq = (torch.from_numpy(q.gamma_idx).cuda(), dev(q.gamma_val, np.float64))
    refq = theta_ref_for(q, mode, np.float64)
    refs = [None if x is None else dev(x, np.float64) for x in (ref, refq)]
    B = E.dd_solve_batch([r, rq], [g, gq], [p.h, q.h], [16, 16], [2, 8], theta=0.3, tol=0.0, max_iter=6,
                         theta_mode=mode, theta_refs=refs)
    u = B[0]["u"].cpu().numpy().reshape(-1)
    assert same(u, O["u"]), show_diff("batch u", u, O["u"])
    assert B[0]["coarse_updates"] == O["coarse_updates"]


CASES_3D = [
    dict(seed=70, n=(17, 17, 17), S=8, M=4, nsrc=2, kind="fourier", theta=0.3),
    dict(seed=71, n=(33, 25, 17), S=8, M=4, nsrc=1, kind="blocks", theta=0.5),
]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("mode", ["estimate", "reference", "field"])
@pytest.mark.parametrize("ci", range(len(CASES_3D)))
def test_theta_modes_3d_bitwise(ci, mode, dtype):
    c = CASES_3D[ci]
    p = W.random_problem(c["seed"], c["n"], c["S"], c["M"], n_src=c["nsrc"], kind=c["kind"])
    print(f"theta3d case={c} mode={mode} dtype={np.dtype(dtype).name}", flush=True)
    G, O = run_pair(p, dtype, c["theta"], 5, mode)
    compare(G, O, 3)


def test_theta_mode_argument_errors():
    p = W.random_problem(72, (33, 33), 8, 4)
    r = dev(p.r, np.float64)
    gi = torch.from_numpy(p.gamma_idx).cuda()
    gv = dev(p.gamma_val, np.float64)
    with pytest.raises(E.EikError) as ei:
        E.dd_solve(r, gi, gv, p.h, 8, 4, max_iter=1, theta_mode="reference")
    assert ei.value.status == E.EIK_ERR_ARG
    bad = list(E.THETA_PARAMS)
    bad[0] = 0.0
    with pytest.raises(E.EikError) as ei:
        E.dd_solve(r, gi, gv, p.h, 8, 4, max_iter=1, theta_mode="estimate", theta_params=bad)
    assert ei.value.status == E.EIK_ERR_ARG
