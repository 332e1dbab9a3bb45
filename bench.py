"""Benchmark: the two-scale DD Eikonal solve on MI355X.

One step = one eik_dd_solve to convergence on the config-2 workload (2D
1025^2, h = 1/1024, 16x16 subdomains S = 64, H = 1/64 (M = 16), seeded
random-Fourier multiscale slowness, source = left edge), i.e. one pass of the
whole hot path: Step 1, then Steps 2-4 and the causal sweep every iteration
until max|U^{k+1}-U^k| < tol.  Inputs are resident in HBM before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]

Prints one JSON line.  value = fine-grid Godunov updates per second over the
whole solve (Step 3 local solves of the serial FSM / wall time of the
solves); ms_per_step is the DD time-to-solution.  The line also carries a
"config3" block: the 3D 257^3 workload's time to solution, its error against
the fp64 u^f, its kernel roofline and its oracle baseline (--no-config3
leaves it out).  The roofline object describes the dominant kernel
(the Step 4 lattice correction or the Step 3 subdomain sweep, whichever takes
longer per launch), timed with HIP events on the stream it runs on, inside
the library; its traffic comes from the committed rocprofv3 counter summary
while the kernel sources are unchanged.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point operations of one local solve (eq. godonuv in
# closed form, two-sided branch): 2 neighbour-minimum compares, a - b,
# |a - b| < r h, (rh)^2, doubling, (a-b)^2, subtraction, a + b, sqrt, add,
# halving, and the FSM minimum compare.
OPS_PER_UPDATE = 13
# Step 4 adds the weighted correction u^k + theta (U~ - C^k) (3 ops) and the
# two wind-agreement / finiteness tests (2 ops) to the local solve.
OPS_PER_CORRECTION = 18
# Non-FMA vector issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3 T lane-ops/s (the published 157.3 TFLOP/s fp32 counts an FMA as two
# flops and packed fp32 as two lanes; 78.6 TFLOP/s fp64 counts the FMA).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Instructions on the dependency path that carries a lane's value from one
# anti-diagonal step to the next, counted in the library's gfx950 ISA of the
# fp32 step loops (DPP receive, neighbour minimum, local solve with the
# correctly rounded square root, the minimum / weighted assignment, the
# lane's carried value); each costs at least one dependent-issue latency.
CHAIN_INSTS = {"k_tile": 21, "k_lattice_correct": 24}
# 3D local solve: 3 neighbour minima (6 compares), a 3-element sort (3
# compares), the one-, two- and three-sided roots (~12 ops and 2 sqrt, one
# division), the FSM minimum compare: about 25 algorithmic ops per update
OPS3_PER_UPDATE = 25


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--theta", type=float, default=0.1)
    ap.add_argument("--n", type=int, default=1025)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config3", action="store_true",
                    help="leave out the 3D 257^3 block of the default (config 2) line")
    ap.add_argument("--workload", choices=["config2", "config3", "config4", "config5", "squares"], default="config2",
                    help="config2 (default): the headline 2D DD solve; config3: 3D 257^3; config4: 64 "
                         "problems in one batched solve; config5: batched travel-time gradient")
    ap.add_argument("--launch", choices=["stream", "graph"], default="graph",
                    help="config2: replay the DD iterations' kernels from HIP graphs (default) or "
                         "launch them on the stream (same kernels and results); the per-kernel "
                         "times always come from stream-launched solves")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (3 times), the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings")
    return ap.parse_args()


def measured_traffic(kernel_prefix, dtype):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/hbm_traffic_config2_<dtype>.md), or None when there is
    none or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_config2_{dtype}.md")
    if not os.path.exists(path):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1805_04198_amd", "csrc", f), "rb").read()
                   for f in ("kernels2d.hpp", "eik.hip"))
    h = hashlib.sha256(src).hexdigest()[:16]
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "traffic" and parts[1].startswith(kernel_prefix):
            kv = dict(x.split("=") for x in parts[2:])
            if kv["source_sha256_16"] != h:
                return None
            return {"bytes": int(kv["read_bytes"]) + int(kv["write_bytes"]),
                    "read_bytes": int(kv["read_bytes"]), "write_bytes": int(kv["write_bytes"])}
    return None


def measured_pmc(kernel_prefix, dtype):
    """Per-dispatch SQ counters of a kernel from the committed rocprofv3
    summary (profiles/pmc_config2_<dtype>.md), or None when there is none or
    the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_config2_{dtype}.md")
    if not os.path.exists(path):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1805_04198_amd", "csrc", f), "rb").read()
                   for f in ("kernels2d.hpp", "eik.hip"))
    h = hashlib.sha256(src).hexdigest()[:16]
    for line in open(path):
        parts = line.split()
        if len(parts) > 2 and parts[0] == "pmc" and parts[1].startswith(kernel_prefix):
            kv = dict(x.split("=") for x in parts[2:])
            if kv.pop("source_sha256_16") != h:
                return None
            return {k: float(v) for k, v in kv.items()}
    return None


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024  # 256 MiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}), flush=True)


def host_info():
    """The host CPU model, the logical CPUs the OS reports and the CPUs this
    process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def oracle_threads():
    # the GPU machine's CPU share is 16 cores per GPU, whatever the OS reports
    return max(1, min(16, host_info()["cpus_allowed"] or 1))


def cpu_baseline(p, theta, tol, dtype, max_iter=400):
    """The oracle as it stands, on the same workload and in the same
    precision as the GPU run (so its iterates and update counts are the
    GPU's, bit for bit): the whole solve to convergence, serial and with the
    OpenMP build (subdomains and lattices in parallel, causal sweep serial)
    on the host's cores."""
    import numpy as np

    import oracle
    args = (p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M)
    kw = dict(theta=theta, tol=tol, max_iter=max_iter, dtype=dtype)
    nt = oracle_threads()
    t0 = time.perf_counter()
    Rm = oracle.dd(*args, threads=nt, **kw)
    t_omp = time.perf_counter() - t0
    t0 = time.perf_counter()
    Rs = oracle.dd(*args, **kw)
    t_ser = time.perf_counter() - t0
    same = bool(np.array_equal(Rm["u"], Rs["u"]) and Rm["iterations"] == Rs["iterations"])
    prec = "fp32" if np.dtype(dtype) == np.float32 else "fp64"
    return {"value": Rm["fine_updates"] / t_omp, "unit": "updates/s", "cores": nt, "kind": "oracle",
            "sample": f"{p.name}: the whole solve to convergence ({Rm['iterations']} DD iterations, "
                      f"{Rm['fine_updates']} fine updates), {prec} oracle, OpenMP build on {nt} threads",
            "time_to_solution_s": t_omp, "iterations": Rm["iterations"],
            "serial": {"value": Rs["fine_updates"] / t_ser, "unit": "updates/s", "cores": 1,
                       "time_to_solution_s": t_ser},
            "omp_equals_serial": same, **host_info()}


def common(a, metric, value, unit, ms, dtype, workload, extra):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": {"workload": workload, "global_batch": 1, "seq_len": None,
                                            "parallelism": "none"}}
    line.update(extra)
    print(json.dumps(line), flush=True)


def config3_block(a, cpu=True):
    """3D 257^3, S = 32, M = 8, fp32, theta = 0.1, tol 1e-6 (the weight is
    not stated for this workload; 0.25 stalls in an fp32 limit cycle):
    time to solution, the error against the fp64 u^f (eik_solve in fp64,
    checked bit for bit against the fp64 oracle's u^f at the stored sample
    nodes of tests/golden/config3_uf_samples.json), the subdomain kernel's
    roofline, and the oracle on a bounded sample of the same solve."""
    import json

    import numpy as np
    import torch

    import paper_1805_04198_amd as E
    from paper_1805_04198_amd import workloads as W
    p = W.config3()
    r = torch.from_numpy(p.r.astype(np.float32)).cuda()
    gi = torch.from_numpy(p.gamma_idx).cuda()
    gv = torch.from_numpy(p.gamma_val.astype(np.float32)).cuda()
    kw = dict(theta=0.1, tol=1e-6, max_iter=400)
    steps = max(1, min(a.steps, 3))
    for _ in range(max(1, min(a.warmup, 1))):
        E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    last = outs[-1]
    fine = sum(o["fine_updates"] for o in outs)
    # the fp64 problem (r and g in fp64, not the fp32 run's fl32(r))
    uf_t, _, _ = E.solve(torch.from_numpy(p.r).cuda(), gi, torch.from_numpy(p.gamma_val).cuda(), p.h)
    uf = uf_t.cpu().numpy().reshape(-1)
    u = last["u"].double().cpu().numpy().reshape(-1)
    gold_path = os.path.join(ROOT, "tests", "golden", "config3_uf_samples.json")
    with open(gold_path) as f:
        gold = json.load(f)
    idx = np.array(gold["idx"], dtype=np.int64)
    uo = np.array([float.fromhex(x) for x in gold["u"]])
    it = last["iterations"]
    upl = last["fine_updates"] / it
    msl = last["ms_fine"] / it
    ach = upl * OPS3_PER_UPDATE / (msl * 1e-3) / 1e12
    out = {"workload": "3D 257^3, h=1/256, 8^3 subdomains (S=32), H=1/32 (M=8), sin-product x lognormal block "
                       "slowness (seed 3), two sources, theta=0.1, tol=1e-6, fp32",
           "time_to_solution_ms": wall * 1e3 / steps, "steps": steps, "updates_per_s": fine / wall,
           "iterations": it, "converged": last["converged"], "fine_updates_per_solve": last["fine_updates"],
           "rel_err_vs_fp64_uf": float(np.max(np.abs(u - uf)) / np.max(uf)),
           "rel_err_vs_fp64_oracle_uf_samples": float(np.max(np.abs(u[idx] - uo)) / gold["max"]),
           "fp64_uf_equals_oracle_at_samples": bool(np.array_equal(uf[idx], uo)
                                                    and float(np.max(uf)) == gold["max"]),
           "gate": 2e-5,
           "ms_fine_per_solve": last["ms_fine"], "ms_correct_per_solve": last["ms_correct"],
           "ms_causal_per_solve": last["ms_causal"],
           "roofline": {"bound": "alu", "kernel": "k_tile3 (Step 3 subdomain FSM, 33^3 boxes)", "achieved": ach,
                        "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s", "frac": ach / ALU_PEAK_TOPS, "traffic": None,
                        "per_launch": {"updates": upl, "ms": msl, "ops_per_update": OPS3_PER_UPDATE}}}
    if cpu:
        import oracle
        nt = oracle_threads()
        t0 = time.perf_counter()
        R = oracle.dd(p.n, p.h, p.r, p.gamma_idx, p.gamma_val, p.S, p.M, theta=0.1, tol=0.0, max_iter=1,
                      dtype=np.float32, threads=nt)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": R["fine_updates"] / dt, "unit": "updates/s", "cores": nt, "kind": "oracle",
                               "sample": f"3D 257^3: Step 1 + the first DD iteration, fp32 oracle, OpenMP build "
                                         f"on {nt} threads, {R['fine_updates']} fine updates in {dt:.1f} s",
                               **host_info()}
    return out


def bench_config3(a):
    blk = config3_block(a, cpu=not a.no_cpu_baseline)
    extra = {k: v for k, v in blk.items() if k not in ("workload", "time_to_solution_ms", "updates_per_s", "steps")}
    common(a, "fine-grid Godunov updates/s + DD time-to-solution at stated error vs FP64 oracle",
           blk["updates_per_s"], "updates/s", blk["time_to_solution_ms"], "f32",
           "config 3: " + blk["workload"], extra)


def bench_config4(a):
    """64 independent 2D problems (257^2..2049^2): the partition S, M
    autotuned per size and the launch schedule of Steps 3 and 4 for the whole
    batch, at the given weight (not tuned), one batched solve; compared with
    the same problems solved one by one with the same parameters (identical
    results)."""
    import numpy as np
    import torch

    import paper_1805_04198_amd as E
    from paper_1805_04198_amd import autotune
    from paper_1805_04198_amd import workloads as W
    P = W.config4()
    rs = [torch.from_numpy(p.r.astype(np.float32)).cuda() for p in P]
    gams = [(torch.from_numpy(p.gamma_idx).cuda(), torch.from_numpy(p.gamma_val.astype(np.float32)).cuda())
            for p in P]
    hs = [p.h for p in P]
    th = a.theta
    t0 = time.perf_counter()
    best, table = autotune.tune(rs, gams, hs, theta=th, tol=1e-6, max_iter=300)
    S, M = autotune.apply(rs, best)
    (launch, pblocks), launch_ms = autotune.tune_launch(rs, gams, hs, S, M, theta=th, tol=1e-6, max_iter=600)
    t_tune = time.perf_counter() - t0
    kw = dict(theta=th, tol=1e-6, max_iter=600)
    for _ in range(a.warmup):
        E.dd_solve_batch(rs, gams, hs, S, M, launch=launch, persistent_blocks=pblocks, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        B = E.dd_solve_batch(rs, gams, hs, S, M, launch=launch, persistent_blocks=pblocks, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fine = sum(b["fine_updates"] for b in B)
    t0 = time.perf_counter()
    same = 0
    for i in range(len(P)):
        R = E.dd_solve(rs[i], gams[i][0], gams[i][1], hs[i], S[i], M[i], **kw)
        same += int(R["iterations"] == B[i]["iterations"] and torch.equal(R["u"], B[i]["u"]))
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    extra = {"problems": len(P), "converged": sum(b["converged"] for b in B), "identical_to_single": same,
             "fine_updates_per_batch": fine, "ms_single_solves_total": t_single * 1e3,
             "speedup_vs_single_solves": t_single / (wall / a.steps), "autotune_s": t_tune,
             "theta": th, "launch": launch, "persistent_blocks": pblocks, "launch_ms": launch_ms,
             "tuned": {f"{k[1]}x{k[0]}": {"S": v[0], "M": v[1]} for k, v in best.items()},
             "tuning_table": [{"shape": f"{t[0][1]}x{t[0][0]}", "S": t[1], "M": t[2], "converged": t[3],
                               "iterations": t[4], "ms": t[5]} for t in table],
             "max_iterations": max(b["iterations"] for b in B)}
    common(a, "fine-grid Godunov updates/s + DD time-to-solution at stated error vs FP64 oracle", fine / wall,
           "updates/s", wall * 1e3 / a.steps, "f32",
           f"config 4: 64 independent 2D problems, sides {{257,513,1025,2049}} (seed 4), partition (S, M) "
           f"autotuned per size, launch schedule autotuned, theta={th}, random-Fourier media, random point "
           f"sources, tol=1e-6, one batched solve", extra)


def bench_config5(a):
    """Travel-time gradient: 1025^2, 32 top-edge sources, 256 receivers,
    targets solved through the perturbed slowness; one step = forward solves
    of all sources + the batched adjoint (fp32).  Central differences of the
    loss (fp64 forward solves) on 20 random cells check the gradient."""
    import numpy as np
    import torch

    import paper_1805_04198_amd as E
    from paper_1805_04198_amd import workloads as W
    p = W.config5_problem()
    r = torch.from_numpy(p.r.astype(np.float32)).cuda()
    rcv = torch.from_numpy(p.receivers).cuda()
    with torch.no_grad():
        rp = torch.from_numpy(p.r_perturbed.astype(np.float32)).cuda()
        target = E.travel_times(rp, p.h, p.sources).reshape(len(p.sources), -1)[:, rcv]

    def step(rr):
        rr = rr.detach().requires_grad_(True)
        U = E.travel_times(rr, p.h, p.sources)
        loss = ((U.reshape(len(p.sources), -1)[:, rcv] - target) ** 2).sum()
        loss.backward()
        return float(loss), rr.grad

    for _ in range(a.warmup):
        step(r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        loss, g = step(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # central differences in fp64 on 20 random cells
    r64 = torch.from_numpy(p.r).cuda()
    t64 = target.double()
    cells = np.random.default_rng(5).choice(p.r.size, 20, replace=False)
    worst = 0.0

    def loss64(rr):
        with torch.no_grad():
            U = E.travel_times(rr, p.h, p.sources)
            return float(((U.reshape(len(p.sources), -1)[:, rcv] - t64) ** 2).sum())

    rr64 = r64.clone().requires_grad_(True)
    U = E.travel_times(rr64, p.h, p.sources)
    L = ((U.reshape(len(p.sources), -1)[:, rcv] - t64) ** 2).sum()
    L.backward()
    gd = rr64.grad.reshape(-1).cpu().numpy()
    g32 = g.reshape(-1).double().cpu().numpy()
    fd_rows = []
    for c in cells:
        eps = 1e-6 * float(p.r.reshape(-1)[c])
        rr = r64.clone().reshape(-1)
        rr[c] += eps
        lp = loss64(rr.reshape(p.r.shape))
        rr[c] -= 2 * eps
        lm = loss64(rr.reshape(p.r.shape))
        fd = (lp - lm) / (2 * eps)
        print(f"bench.py: fd cell {len(fd_rows) + 1}/20", file=sys.stderr, flush=True)
        scale = max(abs(fd), abs(gd[c]), 1e-12)
        rel = abs(fd - gd[c]) / scale if scale > 1e-9 else 0.0
        worst = max(worst, rel)
        fd_rows.append((int(c), fd, float(gd[c]), float(g32[c]), rel))
    rels = np.array([x[4] for x in fd_rows])
    extra = {"sources": len(p.sources), "receivers": len(p.receivers), "loss": loss,
             "fd_check_fp64": {"cells": len(fd_rows), "within_1e-4": int(np.sum(rels <= 1e-4)),
                               # central differences resolve about 1e-9 absolute here
                               # (loss rounding / step); smaller gradients are below it
                               "pass_rel1e-4_abs1e-9": int(sum(abs(x[1] - x[2]) <= 1e-4 * abs(x[2]) + 1e-9
                                                               for x in fd_rows)),
                               "median_rel_err": float(np.median(rels)), "max_rel_err": worst},
             "fd_cells": fd_rows,
             "fp32_vs_fp64_grad_max_rel": float(np.max(np.abs(g32 - gd)) / max(np.max(np.abs(gd)), 1e-30))}
    common(a, "gradient evaluations/s (32 forward FSM solves + batched adjoint)", a.steps / wall, "gradients/s",
           wall * 1e3 / a.steps, "f32",
           "config 5: 2D 1025^2, config-1 slowness, 32 top-edge sources, 256 bottom-edge receivers, targets "
           "through r + 8 Gaussian bumps (seed 5)", extra)


def bench_squares(a):
    """The squares medium of Sec. 5.3 (r = 1 on the lines of period eps = 8h,
    2 elsewhere; source at the centre) on 897^2 (h = 1/896, H = 64h = 1/14,
    S = 64): time to solution with the homogenised coarse solver (timed) and
    with C_H, fp32, tol 1e-6, for theta = 0.1 and 0.25, and the relative L1
    error of U^k against the fine solution u^f over the first iterations
    (Fig. b5's comparison)."""
    import numpy as np
    import torch

    import paper_1805_04198_amd as E
    from paper_1805_04198_amd import workloads as W
    p = W.squares(n_side=897, period=8, S=64, M=64)
    r = torch.from_numpy(p.r.astype(np.float32)).cuda()
    gi = torch.from_numpy(p.gamma_idx).cuda()
    gv = torch.from_numpy(p.gamma_val.astype(np.float32)).cuda()
    theta = 0.25

    def solve(cs, th, **kw):
        kw.setdefault("tol", 1e-6)
        kw.setdefault("max_iter", 400)
        return E.dd_solve(r, gi, gv, p.h, p.S, p.M, theta=th, coarse_solver=cs, **kw)

    for _ in range(a.warmup):
        solve("l1", theta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [solve("l1", theta) for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fine = sum(o["fine_updates"] for o in outs)
    # the fine solution u^f in fp64 (eik_solve) for the error curves
    uf, _, _ = E.solve(r.double(), gi, gv.double(), p.h)
    ufn = uf.cpu().numpy().reshape(-1)
    runs = {}
    for cs in ("l1", "godunov"):
        for th in (0.1, 0.25):
            R = solve(cs, th)
            u = R["u"].double().cpu().numpy().reshape(-1)
            curve = []
            for k in (0, 1, 2, 4, 8, 16):
                U = solve(cs, th, tol=0.0, max_iter=k)["U"].double().cpu().numpy().reshape(-1)
                m = np.isfinite(U)
                curve.append(float(np.sum(np.abs(U[m] - ufn[m])) / np.sum(np.abs(ufn[m]))))
            runs[f"{cs}_theta{th}"] = {"iterations": R["iterations"], "converged": R["converged"],
                                       "ms_to_solution": R["ms_total"],
                                       "max_rel_err_u_vs_uf": float(np.max(np.abs(u - ufn)) / np.max(ufn)),
                                       "rel_L1_err_U_k_0_1_2_4_8_16": curve}
    extra = {"coarse_solver": "l1 (homogenised, timed)", "theta": theta, "iterations": outs[-1]["iterations"],
             "converged": outs[-1]["converged"], "runs": runs}
    common(a, "fine-grid Godunov updates/s + DD time-to-solution at stated error vs FP64 oracle", fine / wall,
           "updates/s", wall * 1e3 / a.steps, "f32",
           "squares medium (Sec. 5.3): 2D 897x897, h=1/896, eps=8h, H=64h=1/14, S=64, centre source, "
           "homogenised coarse solver, theta=0.25, tol=1e-6", extra)


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return
    if a.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (got --gpus {a.gpus}); the DD "
              "path would shard subdomains across GPUs with one skeleton exchange per "
              "iteration, which is not built.", file=sys.stderr)
        sys.exit(2)
    if a.workload != "config2":
        {"config3": bench_config3, "config4": bench_config4, "config5": bench_config5,
         "squares": bench_squares}[a.workload](a)
        return
    import numpy as np
    import torch

    import paper_1805_04198_amd as E
    from paper_1805_04198_amd import workloads as W

    dt = np.float32 if a.dtype == "f32" else np.float64
    tdt = torch.float32 if a.dtype == "f32" else torch.float64
    tol = 1e-6 if a.dtype == "f32" else 1e-12
    p = W.config2(a.n)
    dev = torch.device("cuda:0")
    r = torch.from_numpy(p.r.astype(dt)).to(dev)
    gi = torch.from_numpy(p.gamma_idx).to(dev)
    gv = torch.from_numpy(p.gamma_val.astype(dt)).to(dev)
    kw = dict(theta=a.theta, tol=tol, max_iter=400, launch=a.launch)

    for _ in range(a.warmup):
        E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for _ in range(a.steps):
        outs.append(E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kw))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    last = outs[-1]
    fine = sum(o["fine_updates"] for o in outs)
    ms_step = wall * 1e3 / a.steps
    value = fine / wall
    # per-kernel device times (HIP events around each phase, on the stream
    # the kernels run on) from stream-launched solves after the timed region:
    # graph replays carry no phase events
    if a.launch == "stream":
        tims = outs
    else:
        kws = dict(kw, launch="stream")
        tims = [E.dd_solve(r, gi, gv, p.h, p.S, p.M, **kws) for _ in range(2)]
    iters = sum(o["iterations"] for o in tims)
    fine_t = sum(o["fine_updates"] for o in tims)
    # Step 1 alone, to split the coarse update count into Step 1 and Step 4
    init = E.dd_solve(r, gi, gv, p.h, p.S, p.M, theta=a.theta, tol=tol, max_iter=0)
    corr_updates = sum(o["coarse_updates"] - init["coarse_updates"] for o in tims)

    ceil = measured_ceilings()

    def kernel_line(name, sym, updates, ms, ops, q):
        upl = updates / iters
        msl = ms / iters
        ach = upl * ops / (msl * 1e-3) / 1e12
        kname = f"eik::{sym}<{'float' if a.dtype == 'f32' else 'double'}>"
        tr = measured_traffic(kname, a.dtype)
        line = {"bound": "alu", "kernel": name, "achieved": ach, "peak": ALU_PEAK_TOPS,
                "unit": "TFLOP/s", "frac": ach / ALU_PEAK_TOPS,
                "traffic": None if tr is None else tr["bytes"],
                "traffic_detail": tr,
                "per_launch": {"updates": upl, "ms": msl, "ops_per_update": ops}}
        # the dependent-step time of the boxes' leading waves (clock64 ticks
        # per anti-diagonal step, measured in the kernels of these solves)
        # against the latency of the step's dependency path
        steps = sum(o["lead_steps"][q] for o in tims)
        ticks = sum(o["lead_ticks"][q] for o in tims)
        if steps > 0:
            cps = ticks / steps
            line["cycles_per_step"] = cps
            if ceil and a.dtype == "f32":
                chain = CHAIN_INSTS[sym] * ceil["dependent_add_cycles"]
                line["chain_cycles_per_step"] = chain
                line["critical_path_frac"] = chain / cps
        pmc = measured_pmc(kname, a.dtype)
        line["pmc"] = pmc
        if pmc is not None and pmc.get("GRBM_GUI_ACTIVE"):
            # AMD's VALU-busy measure: VALU issue cycles (4 per wave64
            # instruction) over the dispatch's cycles on all 1024 SIMDs
            line["valu_util"] = pmc["SQ_ACTIVE_INST_VALU"] * 4 / (1024 * pmc["GRBM_GUI_ACTIVE"])
            if "lds_bytes" in pmc:
                line["lds_bytes_per_s"] = pmc["lds_bytes"] / (msl * 1e-3)
        return line

    k_fine = kernel_line("k_tile (Step 3 subdomain FSM)", "k_tile", fine_t,
                         sum(o["ms_fine"] for o in tims), OPS_PER_UPDATE, 0)
    k_corr = kernel_line("k_lattice_correct (Step 4 weighted correction sweeps)",
                         "k_lattice_correct", corr_updates,
                         sum(o["ms_correct"] for o in tims), OPS_PER_CORRECTION, 1)
    dominant, other = (k_corr, k_fine) if k_corr["per_launch"]["ms"] > k_fine["per_launch"]["ms"] \
        else (k_fine, k_corr)

    # error against the fp64 oracle's overall fine solution u^f of the fp64
    # problem (the fixed point the iteration converges to), from eik_solve in
    # fp64, which the parity tests hold bit-identical to the oracle's
    uf_t, _, _ = E.solve(torch.from_numpy(p.r.astype(np.float64)).to(dev), gi,
                         torch.from_numpy(p.gamma_val.astype(np.float64)).to(dev), p.h)
    uf = uf_t.cpu().numpy().reshape(-1)
    u = last["u"].double().cpu().numpy().reshape(-1)
    err = float(np.max(np.abs(u - uf)) / np.max(uf))

    line = {
        "metric": "fine-grid Godunov updates/s + DD time-to-solution at stated error vs FP64 oracle",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.dtype,
        "data": "synthetic",
        "config": {"workload": f"config 2: 2D {p.n[0]}x{p.n[1]}, h=1/{p.n[0]-1}, {p.n[0]//p.S}x{p.n[1]//p.S} "
                               f"subdomains (S={p.S}), H=1/{(p.n[0]-1)//p.M} (M={p.M}), random-Fourier "
                               f"multiscale slowness (seed 2), left-edge source, theta={a.theta}, tol={tol}",
                   "global_batch": 1, "seq_len": None, "parallelism": "none"},
        "time_to_solution_ms": ms_step,
        "iterations": last["iterations"],
        "converged": last["converged"],
        "fine_updates_per_solve": last["fine_updates"],
        "coarse_updates_per_solve": last["coarse_updates"],
        "updates_counted_as": "local solves of the serial FSM on every subdomain (free nodes x sweeps, equal "
                              "to the oracle's count); the GPU sweeps skip the anti-diagonals that cannot "
                              "change, so updates/s is serial-equivalent work per second of wall time",
        "rel_err_vs_fp64_uf": err,
        "gate": 2e-5 if a.dtype == "f32" else 1e-10,
        "launch": a.launch,
        "ms_fine_per_solve": tims[-1]["ms_fine"],
        "ms_coarse_per_solve": tims[-1]["ms_coarse"],
        "ms_correct_per_solve": tims[-1]["ms_correct"],
        "ms_causal_per_solve": tims[-1]["ms_causal"],
        "phase_times_from": "stream-launched solves" if a.launch == "graph" else "the timed solves",
        "roofline": dominant,
        "roofline_secondary": other,
    }
    line["measured_ceilings"] = ceil
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, a.theta, tol, dt)
        # the oracle's own u^f (fp64, serial), the error reference of the metric
        import oracle
        uf_o, _ = oracle.fsm(p.n, p.h, p.r, p.gamma_idx, p.gamma_val)
        line["rel_err_vs_fp64_oracle_uf"] = float(np.max(np.abs(u - uf_o)) / np.max(uf_o))
    if not a.no_config3:
        line["config3"] = config3_block(a, cpu=not a.no_cpu_baseline)
    print(json.dumps(line), flush=True)


def measured_ceilings():
    """The GPU's measured ceilings (libeik_ceilings.so and a device copy):
    non-FMA VALU adds/s with every SIMD busy, cycles per dependent fp32 add
    in a lone wave, LDS read bytes/s, the shader clock during that run, and
    HBM bytes/s of a 1 GiB device-to-device copy (read + write)."""
    import ctypes

    import torch
    path = os.path.join(ROOT, "paper_1805_04198_amd", "_lib", "libeik_ceilings.so")
    if not os.path.exists(path):
        return None
    L = ctypes.CDLL(path)
    L.ceil_measure.restype = ctypes.c_int
    L.ceil_measure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    blocks, iters = 8192, 4096
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda:0")
    lat = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    out = (ctypes.c_double * 4)()
    torch.cuda.synchronize()
    if L.ceil_measure(blocks, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(lat.data_ptr()), out,
                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) != 0:
        return None
    n = 256 * 1024 * 1024  # 1 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    best = None
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return {"valu_adds_per_s": out[0], "dependent_add_cycles": out[1], "lds_read_bytes_per_s": out[2],
            "shader_clock_hz": out[3], "hbm_copy_bytes_per_s": 2.0 * 4 * n / (best * 1e-3),
            "published": {"valu_non_fma_ops_per_s": ALU_PEAK_TOPS * 1e12, "hbm_bytes_per_s": 8.0e12}}


if __name__ == "__main__":
    main()
