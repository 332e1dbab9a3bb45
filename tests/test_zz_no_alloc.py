"""The allocation-free entry point (eik_dd_solve_noalloc) against
eik_dd_solve: the same kernels on a fixed scratch array, so outputs,
iteration counts and update counters must be bitwise equal.  Two calls in a
row, the second on a smaller problem, so that the second reuses scratch the
first left behind."""
import numpy as np
import pytest

from paper_1805_04198_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1805_04198_amd as E  # noqa: E402


def _inputs(p, dtype):
    r = torch.from_numpy(np.ascontiguousarray(p.r, dtype=dtype)).cuda()
    gi = torch.from_numpy(p.gamma_idx.astype(np.int64)).cuda()
    gv = torch.from_numpy(np.ascontiguousarray(p.gamma_val, dtype=dtype)).cuda()
    return r, gi, gv


def _check_same(a, b):
    for k in ("u", "U", "W"):
        assert torch.equal(torch.nan_to_num(a[k], nan=-7.0), torch.nan_to_num(b[k], nan=-7.0)), k
    for k in ("iterations", "converged", "fine_updates", "coarse_updates", "residuals"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_matches_dd_solve_twice(dtype):
    big = W.config2(257, 32, 8)
    small = W.random_problem(11, (97, 65), 32, 8, n_src=2, kind="blocks")
    tol = 1e-6 if dtype == np.float32 else 1e-12
    for p in (big, small):
        r, gi, gv = _inputs(p, dtype)
        kw = dict(theta=0.2, tol=tol, max_iter=200)
        ref = E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw)
        got = E.dd_solve(r, gi, gv, p.h, p.S, p.M, noalloc=True, **kw)
        _check_same(got, ref)
        assert got["ms_total"] == 0.0


def test_noalloc_rejects_a_problem_beyond_its_scratch():
    # 2049^2 in fp64 needs about 330 MB of scratch
    n = 2049
    r = torch.ones((n, n), dtype=torch.float64, device="cuda")
    gi = torch.zeros(1, dtype=torch.int64, device="cuda")
    gv = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EikError) as ex:
        E.dd_solve(r, gi, gv, 1.0 / (n - 1), 64, 32, theta=0.1, max_iter=1, noalloc=True)
    assert ex.value.status == E.EIK_ERR_UNSUPPORTED
    assert "scratch" in str(ex.value)


def test_noalloc_varying_weight_on_65_node_lattices_fp64():
    """fp64 with the estimated weight on 65-node lattices keeps Step 4's
    weight terms in global memory: in the allocation-free call they come
    from the same scratch array; twice, the second problem smaller."""
    big = W.random_problem(12, (129, 129), 16, 2, n_src=2, kind="fourier")
    small = W.random_problem(13, (65, 129), 16, 2, n_src=1, kind="blocks")
    for p in (big, small):
        r, gi, gv = _inputs(p, np.float64)
        kw = dict(theta=0.3, tol=1e-12, max_iter=8, theta_mode="estimate")
        ref = E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw)
        got = E.dd_solve(r, gi, gv, p.h, p.S, p.M, noalloc=True, **kw)
        _check_same(got, ref)
