"""Host-side logic that needs no GPU: the autotuner's candidate rules and
the batching / differentiation workload generators."""
import numpy as np

from paper_1805_04198_amd import autotune
from paper_1805_04198_amd import workloads as W


def test_autotune_candidates_respect_the_solver_limits():
    for n in [(257, 257), (513, 513), (1025, 1025), (2049, 2049), (97, 161)]:
        cands = autotune.candidates(n)
        assert cands, n
        for S, M in cands:
            assert all((m - 1) % S == 0 for m in n) and S + 1 <= 65
            assert S % M == 0 and M <= S
            assert all((m - 1) // M + 1 <= 65 for m in n)
    # 2049: M = 16 would give 129-node lattices
    assert all(M >= 32 for _, M in autotune.candidates((2049, 2049)))
    assert autotune.candidates((100, 100)) == []
    # the weight is the caller's, never searched; the launch schedules are
    # the two the batch API offers
    assert not hasattr(autotune, "THETAS")
    assert set(autotune.LAUNCHES) == {"stream", "persistent"}
    # the launch search: the stream schedule once, the persistent one per
    # grid size (0 = as many resident blocks as fit)
    lc = autotune.launch_candidates()
    assert lc[0] == ("stream", 0) and len(lc) == len(set(lc))
    assert {b for lm, b in lc if lm == "persistent"} == set(autotune.PERSISTENT_BLOCKS)
    assert all(b >= 0 for _, b in lc)


def test_options_struct_matches_the_header():
    """The binding's eik_dd_opts mirrors include/eik.h field for field."""
    import ctypes
    import os
    import re
    import paper_1805_04198_amd as E
    hdr = open(os.path.join(os.path.dirname(E.__file__), "..", "include", "eik.h")).read()
    body = hdr[hdr.index("typedef struct {", hdr.index("eik_dd_debug;")):hdr.index("} eik_dd_opts;")]
    names = re.findall(r"\b(\w+)(?:\[\d+\])?;", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert [f[0] for f in E.DDOpts._fields_] == names
    assert ctypes.sizeof(E.DDOpts) % 8 == 0


def test_config4_generator():
    P = W.config4(n_prob=12)
    assert len(P) == 12
    for p in P:
        assert p.n[0] == p.n[1] and p.n[0] in (257, 513, 1025, 2049)
        assert p.S == 64 and (p.n[0] - 1) % p.S == 0 and p.S % p.M == 0
        assert (p.n[0] - 1) // p.M + 1 <= 65
        assert p.r.shape == p.n[::-1] and np.all(p.r >= 0.2) and np.all(np.isfinite(p.r))
        assert len(p.gamma_idx) == 1 and np.all(p.gamma_val == 0)
        i, j = p.gamma_idx[0] % p.n[0], p.gamma_idx[0] // p.n[0]
        assert 0 < i < p.n[0] - 1 and 0 < j < p.n[1] - 1
    # same seed, same problems
    Q = W.config4(n_prob=12)
    assert all(np.array_equal(a.r, b.r) and np.array_equal(a.gamma_idx, b.gamma_idx) for a, b in zip(P, Q))


def test_config4_medium_matches_its_definition():
    """The separable evaluation equals the direct sum of cosines."""
    p = W.config4(n_prob=1, sizes=(65,))[0]
    rng = np.random.default_rng(np.random.SeedSequence(4).spawn(1)[0])
    n_side = int(rng.choice((65,)))
    eps = float(rng.choice([1.0 / 32, 1.0 / 64]))
    kmag = rng.uniform(1 / eps, 4 / eps, 32)
    ang = rng.uniform(0, 2 * np.pi, 32)
    phi = rng.uniform(0, 2 * np.pi, 32)
    amp = rng.normal(0, 0.02, 32)
    t = np.arange(n_side) / (n_side - 1)
    y, x = np.meshgrid(t, t, indexing="ij")
    a = sum(amp[k] * np.cos(2 * np.pi * kmag[k] * (x * np.cos(ang[k]) + y * np.sin(ang[k])) + phi[k])
            for k in range(32))
    assert np.allclose(p.r, np.maximum(1 + a, 0.2), rtol=0, atol=1e-12)


def test_config5_generator():
    p = W.config5_problem(n_side=257, n_src=8)
    assert len(set(p.sources)) == 8
    assert all(s // p.n[0] == p.n[1] - 1 for s in p.sources)      # top edge
    assert np.all(p.receivers // p.n[0] == 0)                      # bottom edge
    assert np.array_equal(p.receivers % p.n[0], np.arange(2, 255, 4)[: len(p.receivers)])
    assert np.all(p.r_perturbed >= p.r) and np.max(p.r_perturbed - p.r) <= 0.05 * 8
    assert p.targets.shape == (8, len(p.receivers)) and np.all(p.targets > 0)
