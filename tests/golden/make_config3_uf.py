"""Writes tests/golden/config3_uf_samples.json: the fp64 oracle's overall
fine solution u^f (eikref_fsm, Sec. 1.1) of the 3D 257^3 workload at 2048
seeded sample nodes, the nodes of its largest value, its maximum, its
sweep count and the sum of all its values.  Calls only the oracle and the
seeded input generator.

    python tests/golden/make_config3_uf.py

The full solve takes about four minutes on one core; it is resumed every
eight sweeps (one cycle of the 2^3 orders, which resumes exactly) to report
progress."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1805_04198_amd import workloads as W  # noqa: E402

N_SAMPLES = 2048
SEED = 33


def main():
    p = W.config3()
    t0 = time.time()
    u = None
    sweeps = 0
    while True:
        u, _, info = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, max_sweeps=8, with_info=True,
                                u_init=u)
        sweeps += info["sweeps"]
        print(f"oracle u^f 257^3: {sweeps} sweeps, {time.time() - t0:.0f} s", flush=True)
        if info["converged"]:
            break
    idx = np.sort(np.random.default_rng(SEED).choice(u.size, N_SAMPLES, replace=False))
    imax = int(np.argmax(u))
    out = {
        "cite": "overall fine solution u^f (FSM of Sec. 1.1, run until a sweep changes nothing) of the 3D "
                "workload: 257^3, h = 1/256, sin-product x lognormal-block slowness (seed 3), two sources; "
                "computed by the fp64 oracle (eikref_fsm) with this script",
        "workload": "config3",
        "sweeps": sweeps,
        "max": float(u[imax]),
        "argmax": imax,
        "sum": float(np.sum(u)),
        "sample_seed": SEED,
        "idx": [int(i) for i in idx],
        "u": [float(u[i]).hex() for i in idx],
    }
    with open(os.path.join(HERE, "config3_uf_samples.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {len(idx)} samples, max {u[imax]!r}", flush=True)


if __name__ == "__main__":
    main()
