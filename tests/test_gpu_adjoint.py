"""GPU parity of the travel-time gradient (eik_adjoint_batch): dL/dr and the
adjoint fields bit-identical to the oracle's adjoint in the same precision,
on the oracle's own forward solutions; the autograd path; and central
differences of the loss through the GPU forward solve (fp64)."""
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
    return np.array_equal(np.asarray(a), np.asarray(b), equal_nan=True)


def show_diff(name, g, o):
    g = np.asarray(g).reshape(-1)
    o = np.asarray(o).reshape(-1)
    bad = np.nonzero(~((g == o) | (np.isnan(g) & np.isnan(o))))[0]
    return f"{name}: {len(bad)} mismatches, first {bad[:5]} gpu={g[bad[:5]]} oracle={o[bad[:5]]}"


def setup(n, seed, nsrc, nrcv, dtype):
    p = W.random_problem(seed, n, 1, 1, kind="fourier")
    rng = np.random.default_rng(seed + 5)
    srcs = [W.linear_index(n, int(i), n[1] - 1) for i in rng.choice(n[0], nsrc, replace=False)]
    rcvs = np.array([W.linear_index(n, int(i), 0) for i in np.linspace(1, n[0] - 2, nrcv).astype(int)])
    us, ws = [], []
    for s in srcs:
        u, w = oracle.fsm(p.n, p.h, p.r, np.array([s]), np.zeros(1), dtype=dtype)
        us.append(u)
        ws.append(w)
    us = np.array(us)
    target = rng.uniform(0.2, 0.8, (nsrc, nrcv)).astype(dtype)
    seed_ = np.zeros_like(us)
    for b in range(nsrc):
        seed_[b, rcvs] = 2 * (us[b, rcvs] - target[b])
    return p, srcs, rcvs, us, np.array(ws), seed_, target


def encode(ws):
    """axis components (nb, 2, N) -> wind codes (nb, N)"""
    wx, wy = ws[:, 0].astype(np.int16), ws[:, 1].astype(np.int16)
    return ((wx & 3) | ((wy & 3) << 2)).astype(np.int8)


CASES = [
    dict(n=(41, 33), seed=1, nsrc=3, nrcv=8),
    dict(n=(70, 45), seed=2, nsrc=4, nrcv=12),       # ragged boxes
    dict(n=(131, 97), seed=3, nsrc=5, nrcv=20),      # several boxes per axis
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("saved_winds", [True, False])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_adjoint_batch_bitwise(ci, saved_winds, dtype):
    c = CASES[ci]
    print(f"adjoint case={c} saved={saved_winds} dtype={np.dtype(dtype).name}", flush=True)
    p, srcs, rcvs, us, ws, seed_, _ = setup(c["n"], c["seed"], c["nsrc"], c["nrcv"], dtype)
    go, lo, _ = oracle.adjoint(p.n, p.h, p.r, [np.array([s]) for s in srcs], us, seed_,
                               winds=ws if saved_winds else None, dtype=dtype)
    shape = (len(srcs),) + p.r.shape
    r = dev(p.r, dtype)
    gams = [(torch.tensor([s], dtype=torch.int64).cuda(), torch.zeros(1, dtype=r.dtype).cuda()) for s in srcs]
    wind = dev(encode(ws), np.int8).reshape(shape) if saved_winds else None
    grad, lam, info = E.adjoint(r, gams, dev(us, dtype).reshape(shape), dev(seed_, dtype).reshape(shape), p.h,
                                wind=wind, with_lambda=True)
    assert info["converged"]
    g = grad.cpu().numpy().reshape(-1)
    assert same(g, go), show_diff("grad", g, go)
    lg = lam.cpu().numpy().reshape(len(srcs), -1)
    assert same(lg, lo), show_diff("lambda", lg, lo)


def test_autograd_travel_times_matches_adjoint_and_central_differences():
    n = (49, 41)
    p = W.random_problem(11, n, 1, 1, kind="fourier")
    srcs = [W.linear_index(n, i, n[1] - 1) for i in (5, 24, 40)]
    rcvs = torch.tensor([W.linear_index(n, i, 0) for i in range(2, 47, 4)]).cuda()
    rng = np.random.default_rng(3)
    target = torch.from_numpy(rng.uniform(0.3, 0.9, (3, len(rcvs)))).cuda()
    print("autograd fp64 49x41", flush=True)

    def loss_of(rt):
        U = E.travel_times(rt, p.h, srcs)
        return ((U.reshape(3, -1)[:, rcvs] - target) ** 2).sum()

    r = dev(p.r, np.float64).requires_grad_(True)
    L = loss_of(r)
    L.backward()
    g = r.grad.detach().cpu().numpy().reshape(-1)
    # the same gradient from the oracle on the oracle's solutions
    us = np.array([oracle.fsm(p.n, p.h, p.r, np.array([s]), np.zeros(1))[0] for s in srcs])
    seed_ = np.zeros_like(us)
    rc = rcvs.cpu().numpy()
    for b in range(3):
        seed_[b, rc] = 2 * (us[b, rc] - target[b].cpu().numpy())
    go, _, _ = oracle.adjoint(p.n, p.h, p.r, [np.array([s]) for s in srcs], us, seed_)
    assert same(g, go), show_diff("grad", g, go)
    # central differences through the GPU forward solve on 20 cells
    cells = np.random.default_rng(4).choice(p.r.size, 20, replace=False)
    hits = 0
    with torch.no_grad():
        for cidx in cells:
            rr = dev(p.r, np.float64).reshape(-1)
            eps = 1e-6 * float(rr[cidx])
            rr[cidx] += eps
            lp = float(loss_of(rr.reshape(p.r.shape)))
            rr[cidx] -= 2 * eps
            lm = float(loss_of(rr.reshape(p.r.shape)))
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[cidx]) <= 1e-5 * max(abs(fd), abs(g[cidx])) + 1e-9, (cidx, fd, g[cidx])
            hits += abs(g[cidx]) > 1e-6
    assert hits >= 3


def test_config5_full_size_two_sources_fp32():
    """1025^2, config-1 slowness, two of the top-edge sources, all 256
    receivers: gradient bit-identical to the oracle's fp32 adjoint."""
    p = W.config5_problem()
    srcs = p.sources[:2]
    print("config5 full size 2 sources fp32", flush=True)
    us, ws = [], []
    for s in srcs:
        u, w = oracle.fsm(p.n, p.h, p.r, np.array([s]), np.zeros(1), dtype=np.float32)
        us.append(u)
        ws.append(w)
    us = np.array(us)
    seed_ = np.zeros_like(us)
    for b in range(2):
        seed_[b, p.receivers] = 2 * (us[b, p.receivers] - p.targets[b].astype(np.float32))
    go, _, _ = oracle.adjoint(p.n, p.h, p.r, [np.array([s]) for s in srcs], us, seed_, winds=np.array(ws),
                              dtype=np.float32)
    shape = (2,) + p.r.shape
    r = dev(p.r, np.float32)
    gams = [(torch.tensor([s], dtype=torch.int64).cuda(), torch.zeros(1, dtype=r.dtype).cuda()) for s in srcs]
    grad, _, info = E.adjoint(r, gams, dev(us, np.float32).reshape(shape), dev(seed_, np.float32).reshape(shape),
                              p.h, wind=dev(encode(np.array(ws)), np.int8).reshape(shape))
    g = grad.cpu().numpy().reshape(-1)
    assert same(g, go), show_diff("grad", g, go)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_solve_batch_equals_single_solves(dtype):
    n = (131, 70)
    p = W.random_problem(13, n, 1, 1, kind="blocks")
    r = dev(p.r, dtype)
    srcs = [W.linear_index(n, i, j) for i, j in ((3, 69), (64, 0), (130, 35), (70, 40), (0, 0))]
    gams = [(torch.tensor([s]).cuda(), torch.zeros(1, dtype=r.dtype).cuda()) for s in srcs]
    print(f"solve_batch dtype={np.dtype(dtype).name}", flush=True)
    U, Wd, info = E.solve_batch(r, gams, p.h, with_wind=True)
    for b, (gi, gv) in enumerate(gams):
        u, w, i1 = E.solve(r, gi, gv, p.h, with_wind=True)
        assert torch.equal(U[b], u) and torch.equal(Wd[b], w), b
        assert info[b]["sweeps"] == i1["sweeps"]


@pytest.mark.parametrize("n", [(9, 9), (9, 9, 9)])
def test_adjoint_errors(n):
    p = W.random_problem(12, n, 1, 1)
    r = dev(p.r, np.float64)
    gams = [(torch.tensor([0]).cuda(), torch.zeros(1, dtype=r.dtype).cuda())]
    u, _, _ = E.solve(r, gams[0][0], gams[0][1], p.h)
    u = u.reshape((1,) + p.r.shape)
    seed_ = torch.ones_like(u)
    with pytest.raises(E.EikError) as ei:
        E.adjoint(r, gams, u, seed_, p.h, max_sweeps=0)
    assert ei.value.status == E.EIK_ERR_ARG
    # the first sweep changes every free lambda, so a cap of one sweep is
    # reported (the outputs are written, the status says the cap was hit)
    _, _, info = E.adjoint(r, gams, u, seed_, p.h, max_sweeps=1)
    assert info["status"] == E.EIK_ERR_NOCONV and not info["converged"]
    _, _, info = E.adjoint(r, gams, u, seed_, p.h)
    assert info["status"] == E.EIK_OK and info["converged"]
