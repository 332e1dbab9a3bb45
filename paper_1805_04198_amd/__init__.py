"""MI355X-native two-scale domain-decomposition Eikonal solver.

Python binding of libeik.so (HIP, gfx950): argument marshalling only.  Every
step of the solve runs in the library's kernels; PyTorch provides device
memory and the current stream.  Importing the package does not load the
library; the first call does, and raises if it is missing (build it with
``python -m paper_1805_04198_amd.build`` or ``__graft_entry__.build()``).

Method: Martin & Tsai, arXiv 1805.04198 (Sec. 1.1 FSM, Sec. 3.2 DD).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libeik.so")

EIK_OK, EIK_ERR_ARG, EIK_ERR_SHAPE, EIK_ERR_NOCONV = 0, -1, -2, -3
EIK_ERR_HIP, EIK_ERR_UNSUPPORTED, EIK_ERR_NONFINITE = -4, -5, -6
EIK_ERR_INTERNAL = -7
EIK_F32, EIK_F64 = 0, 1
STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_SHAPE", -3: "ERR_NOCONV", -4: "ERR_HIP",
                -5: "ERR_UNSUPPORTED", -6: "ERR_NONFINITE",
                -7: "ERR_INTERNAL"}

# exported symbols of include/eik.h
SYMBOLS = ("eik_solve", "eik_solve_batch", "eik_dd_solve", "eik_dd_solve_batch", "eik_dd_solve_noalloc",
           "eik_adjoint", "eik_adjoint_batch", "eik_last_error", "eik_release", "eik_version")


class EikError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double)]


class Gamma(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("idx", ctypes.c_void_p), ("g", ctypes.c_void_p)]


class DDDebug(ctypes.Structure):
    _fields_ = [("uk", ctypes.c_void_p), ("wk", ctypes.c_void_p), ("U_pre_causal", ctypes.c_void_p)]


class DDOpts(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("M", ctypes.c_int32), ("theta", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_fine_sweeps", ctypes.c_int32), ("max_coarse_sweeps", ctypes.c_int32),
                ("theta_mode", ctypes.c_int32), ("U_init", ctypes.c_void_p),
                ("W_init", ctypes.c_void_p), ("debug", ctypes.POINTER(DDDebug)),
                ("theta_ref", ctypes.c_void_p), ("theta_params", ctypes.c_double * 7),
                ("coarse_solver", ctypes.c_int32), ("launch_mode", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32)]


THETA_MODES = {"constant": 0, "estimate": 1, "reference": 2, "field": 3}
# coarse solver of Steps 1 and 4: C_H, or the homogenised solver of Sec. 5.3
COARSE_SOLVERS = {"godunov": 0, "l1": 1}
# how the DD iterations' kernels are issued: stream launches, HIP graph
# replays (single 2D solves), persistent Step 3/4 grids (batches)
LAUNCH_MODES = {"stream": 0, "graph": 1, "persistent": 2}
# gamma, delta, x0 of eq. thetaest (the paper's values), equal omegas for
# eq. secthetaest (not stated in the paper), margin 0.001 of the reference
# weight
THETA_PARAMS = (0.75, 0.01, 0.9, 1.0, 1.0, 1.0, 0.001)


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("fine_updates", ctypes.c_int64), ("coarse_updates", ctypes.c_int64),
                ("sweeps", ctypes.c_int64), ("final_residual", ctypes.c_double),
                ("residual_history", ctypes.POINTER(ctypes.c_double)),
                ("history_cap", ctypes.c_int32), ("ms_total", ctypes.c_float),
                ("ms_fine", ctypes.c_float), ("ms_coarse", ctypes.c_float),
                ("ms_correct", ctypes.c_float), ("ms_causal", ctypes.c_float),
                ("lead_steps", ctypes.c_int64 * 2), ("lead_ticks", ctypes.c_int64 * 2)]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libeik.so (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # torch provides the device memory and streams; load its HIP runtime first
    # so that the library binds to the same runtime instance
    _torch()
    if not os.path.exists(p):
        raise RuntimeError(f"libeik.so not found at {p}: build it with "
                           "`python -m paper_1805_04198_amd.build`")
    L = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    L.eik_solve.restype = ctypes.c_int32
    L.eik_solve.argtypes = [ctypes.POINTER(Grid), vp, ctypes.POINTER(Gamma), ctypes.c_int32, vp,
                            vp, ctypes.POINTER(Stats), vp]
    L.eik_dd_solve.restype = ctypes.c_int32
    L.eik_dd_solve.argtypes = [ctypes.POINTER(Grid), vp, ctypes.POINTER(Gamma),
                               ctypes.POINTER(DDOpts), vp, vp, vp, ctypes.POINTER(Stats), vp]
    L.eik_dd_solve_noalloc.restype = ctypes.c_int32
    L.eik_dd_solve_noalloc.argtypes = L.eik_dd_solve.argtypes
    L.eik_solve_batch.restype = ctypes.c_int32
    L.eik_solve_batch.argtypes = [ctypes.POINTER(Grid), vp, ctypes.c_int32, ctypes.POINTER(Gamma), ctypes.c_int32,
                                  vp, vp, ctypes.POINTER(Stats), vp]
    L.eik_dd_solve_batch.restype = ctypes.c_int32
    L.eik_dd_solve_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Grid), vp, ctypes.POINTER(Gamma),
                                     ctypes.POINTER(DDOpts), vp, vp, vp, ctypes.POINTER(Stats), vp]
    L.eik_adjoint.restype = ctypes.c_int32
    L.eik_adjoint.argtypes = [ctypes.POINTER(Grid), vp, ctypes.POINTER(Gamma), vp, vp, vp, vp, vp]
    L.eik_adjoint_batch.restype = ctypes.c_int32
    L.eik_adjoint_batch.argtypes = [ctypes.POINTER(Grid), vp, ctypes.c_int32, ctypes.POINTER(Gamma), vp, vp,
                                    vp, vp, vp, ctypes.c_int32, ctypes.POINTER(Stats), vp]
    L.eik_last_error.restype = ctypes.c_char_p
    L.eik_release.restype = ctypes.c_int32
    L.eik_version.restype = ctypes.c_char_p
    if path is None:
        _lib = L
    return L


def _torch():
    import torch
    return torch


def _check(L, st):
    if st != EIK_OK and st != EIK_ERR_NOCONV:
        raise EikError(st, L.eik_last_error().decode())
    return st


def _grid(r, h):
    torch = _torch()
    if not r.is_cuda:
        raise ValueError("r must be a device tensor")
    if r.dtype not in (torch.float32, torch.float64):
        raise ValueError("r must be float32 or float64")
    g = Grid()
    g.dim = r.dim()
    g.dtype = EIK_F32 if r.dtype == torch.float32 else EIK_F64
    shape = list(r.shape)[::-1]  # x fastest
    for a in range(3):
        g.n[a] = shape[a] if a < len(shape) else 1
    g.h = float(h)
    return g


def _gamma(idx, val, r):
    torch = _torch()
    gm = Gamma()
    idx = idx.to(device=r.device, dtype=torch.int64).contiguous()
    val = val.to(device=r.device, dtype=r.dtype).contiguous()
    gm.count = idx.numel()
    gm.idx = idx.data_ptr() if idx.numel() else None
    gm.g = val.data_ptr() if val.numel() else None
    return gm, (idx, val)


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def solve(r, gamma_idx, gamma_val, h, max_sweeps: int = 100000, with_wind: bool = False):
    """eik_solve: FSM on the whole fine grid (the overall fine solution u^f).
    Returns (u, wind codes or None, stats dict)."""
    torch = _torch()
    L = load_library()
    r = r.contiguous()
    g = _grid(r, h)
    gm, keep = _gamma(gamma_idx, gamma_val, r)
    u = torch.empty_like(r)
    w = torch.empty(r.shape, dtype=torch.int8, device=r.device) if with_wind else None
    st = Stats()
    status = L.eik_solve(ctypes.byref(g), r.data_ptr(), ctypes.byref(gm), int(max_sweeps),
                         u.data_ptr(), w.data_ptr() if w is not None else None, ctypes.byref(st),
                         _stream())
    _check(L, status)
    info = {"status": status, "converged": bool(st.converged), "sweeps": int(st.sweeps),
            "updates": int(st.fine_updates), "ms": float(st.ms_total)}
    return u, w, info


def dd_solve(r, gamma_idx, gamma_val, h, S: int, M: int, theta: float = 0.5, tol: float = 1e-12,
             max_iter: Optional[int] = None, max_fine_sweeps: int = 256,
             max_coarse_sweeps: int = 32, U_init=None, W_init=None, debug: bool = False,
             history_cap: int = 4096, theta_mode: str = "constant", theta_params=THETA_PARAMS,
             theta_ref=None, coarse_solver: str = "godunov", noalloc: bool = False,
             launch: str = "stream"):
    """eik_dd_solve: the two-scale DD iteration (Sec. 3.2).  Returns a dict
    with the patched fine solution u, coarse values U (NaN off the skeleton),
    coarse wind codes W, counters and timings; with debug=True also the last
    iteration's u^k, w^k and pre-causal-sweep U.  coarse_solver: "godunov"
    (C_H) or "l1" (the homogenised solver of the squares medium, Sec. 5.3).
    noalloc=True calls eik_dd_solve_noalloc (the library's fixed scratch
    array instead of its workspace; timings are 0).  launch: "stream" or
    "graph" (2D: whole blocks of launched-ahead iterations replayed from a
    HIP graph; same kernels and results, phase timings cover only the
    stream-launched iterations)."""
    torch = _torch()
    L = load_library()
    r = r.contiguous()
    g = _grid(r, h)
    gm, keep = _gamma(gamma_idx, gamma_val, r)
    if max_iter is None:
        max_iter = 4 * (int(g.n[0]) - 1) // M + 16
    u = torch.empty_like(r)
    U = torch.empty_like(r)
    W = torch.empty(r.shape, dtype=torch.int8, device=r.device)
    o = DDOpts()
    o.S, o.M, o.theta, o.tol = int(S), int(M), float(theta), float(tol)
    o.max_iter, o.max_fine_sweeps, o.max_coarse_sweeps = int(max_iter), int(max_fine_sweeps), int(max_coarse_sweeps)
    o.theta_mode = THETA_MODES[theta_mode]
    o.coarse_solver = COARSE_SOLVERS[coarse_solver]
    o.launch_mode = LAUNCH_MODES[launch]
    for q, v in enumerate(theta_params):
        o.theta_params[q] = float(v)
    if theta_ref is not None:
        theta_ref = theta_ref.to(device=r.device, dtype=r.dtype).contiguous()
        o.theta_ref = theta_ref.data_ptr()
    if U_init is not None:
        U_init = U_init.to(device=r.device, dtype=r.dtype).contiguous()
        W_init = W_init.to(device=r.device, dtype=torch.int8).contiguous()
        o.U_init, o.W_init = U_init.data_ptr(), W_init.data_ptr()
    dbg = None
    if debug:
        dbg_t = {"uk": torch.empty_like(r), "wk": torch.empty(r.shape, dtype=torch.int8, device=r.device),
                 "Upre": torch.empty_like(r)}
        dbg = DDDebug(dbg_t["uk"].data_ptr(), dbg_t["wk"].data_ptr(), dbg_t["Upre"].data_ptr())
        o.debug = ctypes.pointer(dbg)
    hist = (ctypes.c_double * max(1, history_cap))()
    st = Stats()
    st.residual_history = hist
    st.history_cap = history_cap
    fn = L.eik_dd_solve_noalloc if noalloc else L.eik_dd_solve
    status = fn(ctypes.byref(g), r.data_ptr(), ctypes.byref(gm), ctypes.byref(o),
                u.data_ptr(), U.data_ptr(), W.data_ptr(), ctypes.byref(st), _stream())
    _check(L, status)
    it = int(st.iterations)
    out = {"u": u, "U": U, "W": W, "status": status, "iterations": it,
           "converged": bool(st.converged), "fine_updates": int(st.fine_updates),
           "coarse_updates": int(st.coarse_updates), "residuals": list(hist[: min(it, history_cap)]),
           "ms_total": float(st.ms_total), "ms_fine": float(st.ms_fine),
           "ms_coarse": float(st.ms_coarse), "ms_correct": float(st.ms_correct),
           "ms_causal": float(st.ms_causal),
           "lead_steps": [int(st.lead_steps[0]), int(st.lead_steps[1])],
           "lead_ticks": [int(st.lead_ticks[0]), int(st.lead_ticks[1])]}
    if debug:
        out.update(dbg_t)
    return out


def solve_batch(r, gammas, h, max_sweeps: int = 100000, with_wind: bool = False):
    """eik_solve_batch: the whole-grid FSM for several boundary sets (e.g.
    one source each) on one slowness.  gammas: list of (idx, val).  Returns
    (u (nb, *r.shape), wind codes or None, list of stats dicts)."""
    torch = _torch()
    L = load_library()
    r = r.contiguous()
    g = _grid(r, h)
    nb = len(gammas)
    gms = (Gamma * nb)()
    keep = []
    for b, (gi, gv) in enumerate(gammas):
        gm, k = _gamma(gi, gv, r)
        gms[b] = gm
        keep.append(k)
    u = torch.empty((nb,) + tuple(r.shape), dtype=r.dtype, device=r.device)
    w = torch.empty(u.shape, dtype=torch.int8, device=r.device) if with_wind else None
    st = (Stats * nb)()
    status = L.eik_solve_batch(ctypes.byref(g), r.data_ptr(), nb, gms, int(max_sweeps), u.data_ptr(),
                               w.data_ptr() if w is not None else None, st, _stream())
    _check(L, status)
    info = [{"status": status, "converged": bool(x.converged), "sweeps": int(x.sweeps),
             "updates": int(x.fine_updates), "ms": float(x.ms_total)} for x in st]
    return u, w, info


def dd_solve_batch(rs, gammas, hs, S, M, theta=0.25, tol=1e-6, max_iter=None, max_fine_sweeps: int = 256,
                   max_coarse_sweeps: int = 32, theta_mode="constant", theta_params=THETA_PARAMS,
                   theta_refs=None, history_cap: int = 4096, coarse_solver="godunov", launch: str = "stream",
                   persistent_blocks: int = 0):
    """eik_dd_solve_batch: the DD iteration on independent problems at once
    (2D: every DD step is one launch over all problems that have not
    converged; 3D: the problems one after another).  rs: list of device
    slowness tensors (one dtype, all 2D or all 3D); gammas:
    list of (idx, val); hs: list of spacings; S, M, theta, tol, max_iter,
    theta_mode, coarse_solver: one value for all or a list.  launch: "stream" (one
    block per subdomain / lattice) or "persistent" (resident grids that take
    the boxes from a counter; same results), with persistent_blocks resident
    blocks per compute unit (0: as many as fit).  Returns a list of result
    dicts as dd_solve, plus the batch's device time in each."""
    torch = _torch()
    L = load_library()
    P = len(rs)
    per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * P
    hs, Ss, Ms, thetas, tols = per(hs), per(S), per(M), per(theta), per(tol)
    iters, modes, solvers = per(max_iter), per(theta_mode), per(coarse_solver)
    refs = per(theta_refs) if theta_refs is not None else [None] * P
    grids = (Grid * P)()
    gms = (Gamma * P)()
    opts = (DDOpts * P)()
    stats = (Stats * P)()
    rptr = (ctypes.c_void_p * P)()
    uptr = (ctypes.c_void_p * P)()
    Uptr = (ctypes.c_void_p * P)()
    Wptr = (ctypes.c_void_p * P)()
    keep, outs, hists = [], [], []
    for p in range(P):
        r = rs[p].contiguous()
        keep.append(r)
        grids[p] = _grid(r, hs[p])
        gm, k = _gamma(gammas[p][0], gammas[p][1], r)
        gms[p] = gm
        keep.append(k)
        mi = iters[p] if iters[p] is not None else 4 * (int(grids[p].n[0]) - 1) // Ms[p] + 16
        o = opts[p]
        o.S, o.M, o.theta, o.tol = int(Ss[p]), int(Ms[p]), float(thetas[p]), float(tols[p])
        o.max_iter, o.max_fine_sweeps, o.max_coarse_sweeps = int(mi), int(max_fine_sweeps), int(max_coarse_sweeps)
        o.theta_mode = THETA_MODES[modes[p]]
        o.coarse_solver = COARSE_SOLVERS[solvers[p]]
        o.launch_mode = LAUNCH_MODES[launch]
        o.persistent_blocks = int(persistent_blocks)
        for q_, v in enumerate(theta_params):
            o.theta_params[q_] = float(v)
        if refs[p] is not None:
            tr = refs[p].to(device=r.device, dtype=r.dtype).contiguous()
            keep.append(tr)
            o.theta_ref = tr.data_ptr()
        u = torch.empty_like(r)
        U = torch.empty_like(r)
        W = torch.empty(r.shape, dtype=torch.int8, device=r.device)
        outs.append((u, U, W))
        rptr[p], uptr[p], Uptr[p], Wptr[p] = r.data_ptr(), u.data_ptr(), U.data_ptr(), W.data_ptr()
        h = (ctypes.c_double * max(1, history_cap))()
        hists.append(h)
        stats[p].residual_history = h
        stats[p].history_cap = history_cap
    status = L.eik_dd_solve_batch(P, grids, rptr, gms, opts, uptr, Uptr, Wptr, stats, _stream())
    _check(L, status)
    res = []
    for p in range(P):
        st = stats[p]
        it = int(st.iterations)
        u, U, W = outs[p]
        res.append({"u": u, "U": U, "W": W, "status": status, "iterations": it,
                    "converged": bool(st.converged), "fine_updates": int(st.fine_updates),
                    "coarse_updates": int(st.coarse_updates),
                    "residuals": list(hists[p][: min(it, history_cap)]), "ms_total": float(st.ms_total),
                    "ms_fine": float(st.ms_fine), "ms_correct": float(st.ms_correct),
                    "ms_causal": float(st.ms_causal)})
    return res


def adjoint(r, gammas, u, dL_du, h, wind=None, max_sweeps: int = 100000, with_lambda: bool = False):
    """eik_adjoint_batch: dL/dr for a batch of converged solutions on one
    slowness.  gammas: list of (idx, val) device tensors, one per problem;
    u, dL_du: (nb, *r.shape) device tensors of r's dtype; wind: (nb,
    *r.shape) int8 codes from eik_solve or None.  Returns (dL/dr, lambda or
    None, stats dict)."""
    torch = _torch()
    L = load_library()
    r = r.contiguous()
    g = _grid(r, h)
    nb = len(gammas)
    u = u.to(dtype=r.dtype).contiguous()
    dL_du = dL_du.to(dtype=r.dtype).contiguous()
    if u.shape != (nb,) + tuple(r.shape) or dL_du.shape != u.shape:
        raise ValueError("u and dL_du must have shape (nb, *r.shape)")
    gms = (Gamma * nb)()
    keep = []
    for b, (gi, gv) in enumerate(gammas):
        gm, k = _gamma(gi, gv, r)
        gms[b] = gm
        keep.append(k)
    if wind is not None:
        wind = wind.to(dtype=torch.int8).contiguous()
        if wind.shape != u.shape:
            raise ValueError("wind must have shape (nb, *r.shape)")
    grad = torch.empty_like(r)
    lam = torch.empty_like(u) if with_lambda else None
    st = Stats()
    status = L.eik_adjoint_batch(ctypes.byref(g), r.data_ptr(), nb, gms, u.data_ptr(),
                                 wind.data_ptr() if wind is not None else None, dL_du.data_ptr(),
                                 grad.data_ptr(), lam.data_ptr() if lam is not None else None,
                                 int(max_sweeps), ctypes.byref(st), _stream())
    _check(L, status)
    return grad, lam, {"status": status, "sweeps": int(st.sweeps), "converged": bool(st.converged),
                       "ms": float(st.ms_total)}


def _travel_times_function():
    torch = _torch()

    class TravelTimes(torch.autograd.Function):
        """u_b = the converged fine travel times (eik_solve_batch) from point
        source b (g = 0 there), stacked; the backward pass is the batched
        adjoint."""

        @staticmethod
        def forward(ctx, r, h, sources):
            gams = [(torch.tensor([int(s_)], dtype=torch.int64, device=r.device),
                     torch.zeros(1, dtype=r.dtype, device=r.device)) for s_ in sources]
            U, Wd, _ = solve_batch(r, gams, h, with_wind=True)
            ctx.save_for_backward(r, U, Wd)
            ctx.h = h
            ctx.gams = gams
            return U

        @staticmethod
        def backward(ctx, dU):
            r, U, Wd = ctx.saved_tensors
            grad, _, _ = adjoint(r, ctx.gams, U, dU, ctx.h, wind=Wd)
            return grad, None, None

    return TravelTimes


def travel_times(r, h, sources):
    """Differentiable travel times from point sources (node indices) on the
    slowness r: returns (len(sources), *r.shape); backward gives dL/dr by the
    batched adjoint (eik_adjoint_batch)."""
    return _travel_times_function().apply(r, h, list(sources))


def decode_winds(codes, d: int):
    """Wind codes (2 bits per axis, see include/eik.h) -> per-axis int8
    components in {-1, 0, +1}, shape (d, N)."""
    import numpy as np
    c = np.asarray(codes).astype(np.uint8).reshape(-1)
    out = np.zeros((d, c.size), dtype=np.int8)
    for a in range(d):
        f = (c >> (2 * a)) & 3
        out[a] = np.where(f == 3, -1, f).astype(np.int8)
    return out
