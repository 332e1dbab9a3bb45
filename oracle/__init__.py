"""CPU oracle for the two-scale domain-decomposition Eikonal solver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The oracle is a plain
serial C implementation (eikref.c) of what the method computes, written from
Martin & Tsai, arXiv 1805.04198, Sec. 1.1 (FSM, FMM) and Sec. 3.2 (the DD
iteration).  It shares no code with the GPU library.

Functions take numpy arrays (host memory) and return numpy arrays.  Winds
are returned per axis: array of shape (d, N), int8, +1 = flow from the minus
side (the upwind neighbour lies at the smaller index).

Two small Python modules hold the paper's worked examples, used only as
pins: dd1d.py (the one-dimensional method of Sec. 3.1) and model_problem.py
(the model problem of Sec. 4 as eq. modelprob writes it).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eikref.c")
_LIB = os.path.join(_HERE, "libeikref.so")
# the same source built with OpenMP over subdomains and lattices (Steps 1, 3
# and 4 of Sec. 3.2; the causal sweep stays serial): the all-core CPU
# baseline, bitwise equal to the serial build
_LIB_OMP = os.path.join(_HERE, "libeikref_omp.so")

STATUS = {0: "OK", -1: "ARG", -2: "SHAPE", -3: "NOCONV", -7: "NOMEM"}


def build(force: bool = True) -> str:
    """Compile eikref.c twice (double and float) into libeikref.so, and the
    same again with OpenMP into libeikref_omp.so."""
    if not force and all(os.path.exists(x) and os.path.getmtime(x) >= os.path.getmtime(_SRC)
                         for x in (_LIB, _LIB_OMP)):
        return _LIB
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-std=c99", "-Wall",
             "-Wno-unused-function"]
    for out, extra, link in ((_LIB, ["-Wno-unknown-pragmas"], []), (_LIB_OMP, ["-fopenmp"], ["-fopenmp"])):
        objs = []
        for tag, defs in (("f64", ["-DREAL=double", "-DSFX=_f64"]),
                          ("f32", ["-DREAL=float", "-DSFX=_f32", "-DORACLE_FLOAT"])):
            obj = out[:-3] + f"_{tag}.o"
            subprocess.check_call(["gcc", *flags, *extra, *defs, "-c", _SRC, "-o", obj])
            objs.append(obj)
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-shared", *link, "-o", tmp, *objs, "-lm"])
        os.replace(tmp, out)
        for o in objs:
            os.remove(o)
    return _LIB


_lib = None
_lib_omp = None


def lib(omp: bool = False):
    """The serial oracle library, or (omp=True) its OpenMP build."""
    global _lib, _lib_omp
    if (_lib_omp if omp else _lib) is None:
        path = _LIB_OMP if omp else _LIB
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        vp = ctypes.c_void_p
        for sfx in ("_f64", "_f32"):
            f = getattr(L, "eikref_fsm" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_double, vp, ctypes.c_int64, i64p, vp,
                          ctypes.c_int, vp, vp, i64p, vp]
            f = getattr(L, "eikref_fmm" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_double, vp, ctypes.c_int64, i64p, vp, vp]
            f = getattr(L, "eikref_dd" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_double, vp, ctypes.c_int64, i64p, vp,
                          ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp,
                          vp, i64p, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                          ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp, ctypes.c_int,
                          ctypes.c_int]
            f = getattr(L, "eikref_causal" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_int, vp, vp, vp]
            f = getattr(L, "eikref_reconcile" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp]
            if omp:
                f = getattr(L, "eikref_set_threads" + sfx)
                f.restype = ctypes.c_int
                f.argtypes = [ctypes.c_int]
            f = getattr(L, "eikref_adjoint" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_double, vp, ctypes.c_int, i64p, vp, vp, vp, vp,
                          vp, vp, i64p]
            f = getattr(L, "eikref_exp_cw" + sfx)
            f.restype = ctypes.c_double
            f.argtypes = [ctypes.c_double]
            f = getattr(L, "eikref_theta_damped" + sfx)
            f.restype = ctypes.c_double
            f.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
            f = getattr(L, "eikref_local" + sfx)
            f.restype = ctypes.c_int
            rt = ctypes.c_float if sfx == "_f32" else ctypes.c_double
            f.argtypes = [ctypes.c_int, vp, vp, rt, ctypes.c_int, vp, vp]
        if omp:
            _lib_omp = L
        else:
            _lib = L
    return _lib_omp if omp else _lib


def _sfx(dtype) -> str:
    return "_f32" if np.dtype(dtype) == np.float32 else "_f64"


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _prep(n, r, gidx, gval, dtype):
    n64 = np.zeros(3, dtype=np.int64)
    n64[: len(n)] = n
    r = np.ascontiguousarray(np.asarray(r, dtype=dtype).reshape(-1))
    gidx = np.ascontiguousarray(np.asarray(gidx, dtype=np.int64))
    gval = np.ascontiguousarray(np.asarray(gval, dtype=dtype))
    return n64, r, gidx, gval


def fsm(n, h, r, gidx, gval, dtype=np.float64, max_sweeps=10000, with_info=False, u_init=None):
    """u^f: FSM on the whole grid (Sec. 1.1).  Returns u, winds (d, N).
    u_init: resume from these values (whole cycles of 2^d sweeps resume
    exactly; see eikref_fsm)."""
    d = len(n)
    n64, r, gidx, gval = _prep(n, r, gidx, gval, dtype)
    N = int(np.prod(n))
    u = np.empty(N, dtype=dtype)
    w = np.zeros(d * N, dtype=np.int8)
    info = np.zeros(3, dtype=np.int64)
    ui = None if u_init is None else np.ascontiguousarray(np.asarray(u_init, dtype=dtype).reshape(-1))
    st = getattr(lib(), "eikref_fsm" + _sfx(dtype))(d, _i64(n64), float(h), _p(r), len(gidx),
                                                    _i64(gidx), _p(gval), int(max_sweeps),
                                                    _p(u), _p(w), _i64(info), _p(ui))
    if st not in (0, -3):
        raise ValueError(f"eikref_fsm: {STATUS.get(st, st)}")
    out = (u, w.reshape(d, N))
    if with_info:
        return out + ({"sweeps": int(info[0]), "updates": int(info[1]), "converged": bool(info[2])},)
    return out


def fmm(n, h, r, gidx, gval, dtype=np.float64):
    """Fast marching on the same discrete system (an independent solver)."""
    d = len(n)
    n64, r, gidx, gval = _prep(n, r, gidx, gval, dtype)
    N = int(np.prod(n))
    u = np.empty(N, dtype=dtype)
    st = getattr(lib(), "eikref_fmm" + _sfx(dtype))(d, _i64(n64), float(h), _p(r), len(gidx),
                                                    _i64(gidx), _p(gval), _p(u))
    if st != 0:
        raise ValueError(f"eikref_fmm: {STATUS.get(st, st)}")
    return u


THETA_MODES = {"constant": 0, "estimate": 1, "reference": 2, "field": 3}
# gamma, delta, x0 of eq. thetaest (Sec. 4.2 figure) and the omega weights
# of eq. secthetaest (unstated in the paper: equal weights), margin of the
# reference weight M-bar - 0.001 (Sec. 5.3)
THETA_PARAMS = (0.75, 0.01, 0.9, 1.0, 1.0, 1.0, 0.001)


def dd(n, h, r, gidx, gval, S, M, theta=0.5, tol=1e-12, max_iter=None, dtype=np.float64,
       max_fine_sweeps=256, max_coarse_sweeps=32, U_init=None, W_init=None, hist_cap=4096,
       theta_mode="constant", theta_params=THETA_PARAMS, theta_ref=None, coarse_solver="godunov",
       threads=None, inflow_fixed=False):
    """The DD iteration of Sec. 3.2.  Returns a dict with the patched fine
    solution u, coarse values U (NaN off the skeleton), coarse winds W (d, N),
    the last iteration's reconciled fine values uk / winds wk, the last
    corrected U before its causal sweep (Upre), and the counters.
    theta_mode selects the Step 4 weight (see theta_node in eikref.c):
    "constant", "estimate" (eqs. secthetaest, thetaest), "reference"
    (M-bar minus a margin, theta_ref = u^f) or "field" (theta_ref = theta
    per node).  coarse_solver: "godunov" (C_H of Sec. 3.2) or "l1" (the
    homogenised coarse solver of the squares medium, Sec. 5.3).
    threads: run the OpenMP build with that many threads (subdomains and
    lattices in parallel; bitwise the serial result).  inflow_fixed: the
    test-only literal reading of Step 2 (inflow nodes held at U)."""
    d = len(n)
    n64, r, gidx, gval = _prep(n, r, gidx, gval, dtype)
    N = int(np.prod(n))
    if max_iter is None:
        max_iter = 4 * (int(n[0]) - 1) // M + 16
    u = np.empty(N, dtype=dtype)
    U = np.empty(N, dtype=dtype)
    W = np.zeros(d * N, dtype=np.int8)
    uk = np.empty(N, dtype=dtype)
    wk = np.zeros(d * N, dtype=np.int8)
    Upre = np.full(N, np.nan, dtype=dtype)
    info = np.zeros(5, dtype=np.int64)
    hist = np.zeros(max(1, hist_cap), dtype=np.float64)
    Ui = None if U_init is None else np.ascontiguousarray(np.asarray(U_init, dtype=dtype).reshape(-1))
    Wi = None if W_init is None else np.ascontiguousarray(np.asarray(W_init, dtype=np.int8).reshape(-1))
    mode = THETA_MODES[theta_mode]
    tpar = np.ascontiguousarray(np.asarray(theta_params, dtype=np.float64))
    assert tpar.shape == (7,)
    tref = None if theta_ref is None else np.ascontiguousarray(np.asarray(theta_ref, dtype=dtype).reshape(-1))
    L = lib(omp=threads is not None)
    if threads is not None:
        getattr(L, "eikref_set_threads" + _sfx(dtype))(int(threads))
    st = getattr(L, "eikref_dd" + _sfx(dtype))(
        d, _i64(n64), float(h), _p(r), len(gidx), _i64(gidx), _p(gval), int(S), int(M),
        float(theta), float(tol), int(max_iter), int(max_fine_sweeps), int(max_coarse_sweeps),
        _p(Ui), _p(Wi), _p(u), _p(U), _p(W), _p(uk), _p(wk), _p(Upre), _i64(info),
        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(hist_cap), int(mode),
        tpar.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _p(tref),
        {"godunov": 0, "l1": 1}[coarse_solver], int(bool(inflow_fixed)))
    if st not in (0, -3):
        raise ValueError(f"eikref_dd: {STATUS.get(st, st)}")
    it = int(info[0])
    return {"u": u, "U": U, "W": W.reshape(d, N), "uk": uk, "wk": wk.reshape(d, N),
            "Upre": Upre, "iterations": it, "converged": bool(info[1]),
            "fine_updates": int(info[2]), "coarse_updates": int(info[3]),
            "status": int(info[4]), "residuals": hist[: min(it, hist_cap)].copy()}


def adjoint(n, h, r, gammas, u, seed, winds=None, dtype=np.float64):
    """Travel-time gradient by the discrete adjoint of the converged upwind
    system (see eikref_adjoint): a batch of problems on one slowness.
    gammas: list of Gamma index arrays, one per problem; u, seed: (nb, N);
    winds: (nb, d, N) axis components or None (recomputed from u).
    Returns (dL/dr (N,), lambda (nb, N), passes)."""
    d = len(n)
    nb = len(gammas)
    n64 = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
    N = int(np.prod(n))
    r = np.ascontiguousarray(np.asarray(r, dtype=dtype).reshape(-1))
    u = np.ascontiguousarray(np.asarray(u, dtype=dtype).reshape(nb, N))
    seed = np.ascontiguousarray(np.asarray(seed, dtype=dtype).reshape(nb, N))
    gl = [np.ascontiguousarray(np.asarray(g, dtype=np.int64)) for g in gammas]
    gcount = np.array([len(g) for g in gl], dtype=np.int64)
    ptrs = (ctypes.c_void_p * nb)(*[g.ctypes.data for g in gl])
    w = None if winds is None else np.ascontiguousarray(np.asarray(winds, dtype=np.int8).reshape(nb, d, N))
    lam = np.empty((nb, N), dtype=dtype)
    grad = np.empty(N, dtype=dtype)
    info = np.zeros(1, dtype=np.int64)
    st = getattr(lib(), "eikref_adjoint" + _sfx(dtype))(
        d, _i64(n64), float(h), _p(r), nb, _i64(gcount), ctypes.cast(ptrs, ctypes.c_void_p), _p(u), _p(w),
        _p(seed), _p(lam), _p(grad), _i64(info))
    if st != 0:
        raise ValueError(f"eikref_adjoint: {STATUS.get(st, st)}")
    return grad, lam, int(info[0])


def causal(n, M, U, W, isg, dtype=np.float64):
    """The causal sweep alone (Alg. causalsweep2D; see eikref_causal) on a
    full-grid U (returned, a copy), winds W (d, N) and Gamma flags (N,)."""
    d = len(n)
    n64 = np.zeros(3, dtype=np.int64)
    n64[:d] = n
    U = np.array(np.asarray(U, dtype=dtype).reshape(-1), copy=True)
    W = np.ascontiguousarray(np.asarray(W, dtype=np.int8).reshape(-1))
    isg = np.ascontiguousarray(np.asarray(isg, dtype=np.uint8).reshape(-1))
    st = getattr(lib(), "eikref_causal" + _sfx(dtype))(d, _i64(n64), int(M), _p(U), _p(W), _p(isg))
    if st != 0:
        raise ValueError("eikref_causal")
    return U


def reconcile(values, winds, sides, iface, Wk, dtype=np.float64):
    """The reconciliation at one node (Alg. fineupdate per axis; see
    reconcile_node in eikref.c): candidate values (nc,), winds (nc, d),
    sides (nc, d) with 0 = minus, 1 = plus; interface axes (d,); coarse wind
    W^k (d,).  Returns (u^k, w^k)."""
    nc = len(values)
    d = len(iface)
    cu = np.ascontiguousarray(np.asarray(values, dtype=dtype))
    cw = np.zeros((nc, 3), dtype=np.int8)
    cw[:, :d] = winds
    cs = np.zeros((nc, 3), dtype=np.int32)
    cs[:, :d] = sides
    fa = np.zeros(3, dtype=np.int32)
    fa[:d] = iface
    wk3 = np.zeros(3, dtype=np.int8)
    wk3[:d] = Wk
    uk = np.zeros(1, dtype=dtype)
    wk = np.zeros(3, dtype=np.int8)
    st = getattr(lib(), "eikref_reconcile" + _sfx(dtype))(d, nc, _p(cu), _p(cw), _p(cs), _p(fa), _p(wk3),
                                                         _p(uk), _p(wk))
    if st != 0:
        raise ValueError("eikref_reconcile")
    return uk[0], wk[:d].copy()


def exp_cw(x):
    """The oracle's fixed-sequence e^x (Cody-Waite reduction + Taylor)."""
    return lib().eikref_exp_cw_f64(float(x))


def theta_damped(tb, gamma=0.75, delta=0.01, x0=0.9):
    """eq. thetaest applied to an estimate tb."""
    return lib().eikref_theta_damped_f64(float(tb), float(gamma), float(delta), float(x0))


def local(m, ws, rd, rule=0, dtype=np.float64):
    """The local solve alone (eq. godonuv in the closed form of C_H, with
    the fine (rule 0, Alg. fineupdate2D) or coarse (rule 1, Alg. update2D)
    wind rule).  m: per-axis neighbour minima, ws: their wind signs."""
    d = len(m)
    mm = np.full(3, np.inf, dtype=dtype)
    mm[:d] = m
    w = np.zeros(3, dtype=np.int8)
    w[:d] = ws
    wt = np.zeros(3, dtype=np.int8)
    out = np.zeros(1, dtype=dtype)
    st = getattr(lib(), "eikref_local" + _sfx(dtype))(d, _p(mm), _p(w), rd, int(rule), _p(wt), _p(out))
    if st != 0:
        raise ValueError("eikref_local")
    return out[0], wt[:d].copy()


def speedup_bound(N: int, M: int, d: int, iterations: int) -> float:
    """Sec. 4.3 (complexity and speed up): the number of DD iterations k
    below which the method, with one processor per coarse grid and per
    subdomain, takes fewer flops than serial FSM on the fine grid.  FSM with
    `iterations` iterations of 2^d sweeps on (n+1)^d nodes costs
    A(n, d) = iterations * 2^d * (n+1)^d (unit cost per node update); one DD
    iteration costs A(N, d) + A(M, d) + 2^d M (N+1)^2 (the causal-sweep term
    as the paper writes it); the bound is A(NM, d) over that."""
    def A(n):
        return iterations * 2 ** d * (n + 1) ** d
    return A(N * M) / (A(N) + A(M) + 2 ** d * M * (N + 1) ** 2)


def solve_problem(p, dtype=np.float64, **kw):
    """Convenience: run dd() on a workloads.Problem."""
    return dd(p.n, p.h, p.r_as(np.float64), p.gamma_idx, p.gamma_val.astype(np.float64),
              p.S, p.M, theta=kw.pop("theta", p.theta), tol=kw.pop("tol", p.tol), dtype=dtype,
              **kw)
