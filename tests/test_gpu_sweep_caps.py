"""GPU parity (bitwise with the oracle in the same precision) of the box
sweeps that two waves of a block share: odd and even caps on the number of
subdomain and lattice sweeps (so the sweep that ends the sweeping falls on
either wave, and a capped run stops on either), subdomain boxes of 65 rows
(row 64 runs late on lane 0), 64 and 63 rows, and rectangular lattices."""
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
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


CASES = [
    dict(seed=51, n=(129, 129), S=64, M=16, kind="fourier"),  # 65-row boxes
    dict(seed=52, n=(127, 127), S=63, M=9, kind="blocks"),    # 64-row subdomains
    dict(seed=53, n=(125, 125), S=62, M=31, kind="fourier"),  # 63-row subdomains, 5-node lattices
    dict(seed=54, n=(129, 65), S=32, M=8, kind="blocks"),     # rectangular lattices
]
CAPS = [(1, 1), (2, 3), (3, 2), (5, 7), (256, 32)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("caps", CAPS)
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_sweep_caps_bitwise(ci, caps, dtype):
    c = CASES[ci]
    fine, coarse = caps
    p = W.random_problem(c["seed"], c["n"], c["S"], c["M"], n_src=2, kind=c["kind"])
    print(f"case={c} caps={caps} dtype={np.dtype(dtype).name}", flush=True)
    G = E.dd_solve(dev(p.r, dtype), torch.from_numpy(p.gamma_idx).cuda(), dev(p.gamma_val, dtype), p.h, p.S,
                   p.M, theta=0.3, tol=0.0, max_iter=3, max_fine_sweeps=fine, max_coarse_sweeps=coarse)
    O = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=0.3, tol=0.0, max_iter=3,
                  dtype=dtype, max_fine_sweeps=fine, max_coarse_sweeps=coarse)
    assert same(G["U"].cpu().numpy().reshape(-1), O["U"])
    assert same(E.decode_winds(G["W"].cpu().numpy(), 2), O["W"])
    assert same(G["u"].cpu().numpy().reshape(-1), O["u"])
    assert G["fine_updates"] == O["fine_updates"] and G["coarse_updates"] == O["coarse_updates"]
