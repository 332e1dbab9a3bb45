"""The DD iteration replayed from HIP graphs (launch="graph") against stream
launches and the oracle: the same kernels on the same arguments, so every
output, count and residual must be bit-identical.  Covers a first capture,
a replay of the cached graphs by a second call with the same arguments, a
different problem (captured again), a run that stops inside a replayed
block, and max_iter cutting the last block short."""
import numpy as np
import pytest

import oracle
from paper_1805_04198_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1805_04198_amd as E  # noqa: E402


def inputs(p, dtype):
    r = torch.from_numpy(p.r.astype(dtype)).cuda()
    gi = torch.from_numpy(p.gamma_idx.astype(np.int64)).cuda()
    gv = torch.from_numpy(p.gamma_val.astype(dtype)).cuda()
    return r, gi, gv


KEYS = ("iterations", "converged", "fine_updates", "coarse_updates", "residuals")


def check_same(a, b):
    for k in ("u", "U", "W"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True), k
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_graph_replay_equals_stream_launches(dtype):
    p = W.config2(257, 32, 8)
    r, gi, gv = inputs(p, dtype)
    kw = dict(theta=0.1, tol=1e-6 if dtype == np.float32 else 1e-12, max_iter=200)
    ref = E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw)
    assert ref["converged"] and ref["iterations"] > 8
    first = E.dd_solve(r, gi, gv, p.h, p.S, p.M, launch="graph", **kw)
    again = E.dd_solve(r, gi, gv, p.h, p.S, p.M, launch="graph", **kw)
    check_same(ref, first)
    check_same(ref, again)
    # another problem on the same workspace: the cached graphs do not match
    q = W.random_problem(7, (257, 257), 32, 8, n_src=2)
    r2, gi2, gv2 = inputs(q, dtype)
    ref2 = E.dd_solve(r2, gi2, gv2, q.h, q.S, q.M, **kw)
    g2 = E.dd_solve(r2, gi2, gv2, q.h, q.S, q.M, launch="graph", **kw)
    check_same(ref2, g2)


@pytest.mark.parametrize("max_iter", [9, 10, 13])
def test_graph_with_short_last_block_against_oracle(max_iter):
    p = W.random_problem(8, (129, 129), 32, 8, n_src=1)
    r, gi, gv = inputs(p, np.float64)
    G = E.dd_solve(r, gi, gv, p.h, p.S, p.M, theta=0.3, tol=0.0, max_iter=max_iter, launch="graph")
    O = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=0.3, tol=0.0, max_iter=max_iter)
    assert G["iterations"] == O["iterations"] == max_iter
    assert np.array_equal(G["u"].cpu().numpy().reshape(-1), O["u"], equal_nan=True)
    assert np.array_equal(G["U"].cpu().numpy().reshape(-1), O["U"], equal_nan=True)
    assert G["fine_updates"] == O["fine_updates"] and G["coarse_updates"] == O["coarse_updates"]
