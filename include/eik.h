/*
 * eik.h -- C ABI of the MI355X (gfx950) two-scale domain-decomposition
 * Eikonal solver (Martin & Tsai, "A multiscale domain decomposition
 * algorithm for boundary value problems for Eikonal equations",
 * arXiv 1805.04198).
 *
 * Problem (Sec. 1, eq. eikonal; Sec. 3.2, eqs. 2Deq/2Dbc):
 *     |grad u(x)| = r(x) in Omega = [0,1]^d,   u = g on Gamma,
 * discretised on a uniform grid by the Godunov upwind scheme (Sec. 1.1,
 * eq. godonuv).  r is the slowness r_eps = r0 + a_eps sampled at the nodes.
 *
 * Conventions shared by every entry point
 *   - Layout: node (i,j[,k]) lives at linear index i + n0*(j + n1*k); x is the
 *     fastest axis.  All arrays are DEVICE pointers owned by the caller; the
 *     library never frees them and keeps no reference after the call returns.
 *   - Calls are ordered on the given HIP stream (NULL = the null stream).  An
 *     entry point returns after its work is complete (it synchronises that
 *     stream), so outputs and the host-side stats are ready on return.
 *   - Winds (the paper's w and W, Secs. 3.1-3.2) are int8 codes, two bits per
 *     axis: bits 0-1 = x, 2-3 = y, 4-5 = z; each field 0 = no component,
 *     1 = +1, 3 = -1.  A +1 component means the flow arrives from the minus
 *     side (the upwind neighbour has the smaller index).
 *   - Every call returns an eik_status.  Nothing throws.  On an error the
 *     outputs are unspecified unless stated otherwise; eik_last_error()
 *     returns a message for the calling thread.
 *   - Workspace is allocated by the library on first use on a device and
 *     reused (grown when a larger problem arrives) until eik_release().
 *     Calls that overlap on one device from different host threads are
 *     serialised by the library.
 */
#ifndef EIK_H
#define EIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t eik_status;
#define EIK_OK 0
#define EIK_ERR_ARG (-1)          /* bad argument: r <= 0 or not finite, Gamma unsorted or out of range, theta outside [0,1], NULL pointer */
#define EIK_ERR_SHAPE (-2)        /* (n-1) % S != 0, S % M != 0, M < 2, extents too small */
#define EIK_ERR_NOCONV (-3)       /* max_iter reached without max|U^{k+1}-U^k| < tol; outputs and stats ARE written */
#define EIK_ERR_HIP (-4)          /* a HIP runtime call failed */
#define EIK_ERR_UNSUPPORTED (-5)  /* valid problem outside what this library implements (see eik_last_error) */
#define EIK_ERR_NONFINITE (-6)    /* the residual became NaN */
#define EIK_ERR_INTERNAL (-7)     /* an internal bound was exceeded (a wait between the two waves of a 2D box sweep
                                     gave up); outputs unspecified */

typedef enum { EIK_F32 = 0, EIK_F64 = 1 } eik_dtype;

/* The grid: d = 2 (or 3), n[a] nodes along axis a (n[a] >= 2; unused axes
 * ignored), spacing h > 0, and the element type of every real array passed
 * with it. */
typedef struct {
    int32_t dim;
    int32_t dtype; /* eik_dtype */
    int64_t n[3];
    double h;
} eik_grid;

/* The boundary set Gamma (Sec. 1.1, "Initialization"): `count` node indices
 * (device, int64, strictly increasing, each in [0, N)) and their values g
 * (device, grid dtype, finite).  count may be 0. */
typedef struct {
    int64_t count;
    const int64_t* idx;
    const void* g;
} eik_gamma;

/* Optional per-iteration snapshots for debugging and parity tests: full-grid
 * device arrays (NaN / 0 off the coarse skeleton) of the LAST iteration's
 * reconciled fine values u^k and winds w^k (Sec. 3.2, Alg. fineupdate) and
 * of its corrected coarse values before the causal sweep (Alg.
 * 2Dweightedupdate).  Any member may be NULL. */
typedef struct {
    void* uk;
    int8_t* wk;
    void* U_pre_causal;
} eik_dd_debug;

/* Weight of the Step 4 correction U = u^k + theta (U~ - C^k) at a node
 * (Sec. 3.2 lets theta vary per node and iteration; Sec. 4.2 estimates it):
 *   EIK_THETA_CONSTANT   opts->theta everywhere.
 *   EIK_THETA_ESTIMATE   eq. secthetaest: t = (u^k - u^{k-1}) / (omega-weighted
 *                        mean of the increments C_H(U^{k+1-s}) - C_H(U^{k-s}),
 *                        s = 0, 1, 2; the s = 0 one is U~ - C^k), evaluated as
 *                        num / ((w0 d0 + (w1 d1 + w2 d2)) / ((w0 + w1) + w2)),
 *                        then eq. thetaest: [s t + (1 - s) delta t]^+ with
 *                        s = 1 / (1 + e^{(t - x0)/gamma}).  opts->theta is used
 *                        until C^{k-2} exists (the first two iterations of a
 *                        call, also after a resume) and where a term is not
 *                        finite or the denominator is 0.
 *   EIK_THETA_REFERENCE  M-bar of Sec. 4.2 minus a margin: (u_ref - u^k) /
 *                        (U~ - C^k) - margin, clamped at 0 (Sec. 5.3 uses
 *                        u_ref = u^f and margin 0.001); opts->theta where not
 *                        defined.
 *   EIK_THETA_FIELD      theta_ref holds theta per node.
 * The weight is computed in double from the grid-dtype values; e^x there is
 * a fixed sequence of double operations (Cody-Waite reduction, Taylor series
 * to degree 13), so results do not depend on the math library.  Only
 * the node where the correction applies uses it. */
#define EIK_THETA_CONSTANT 0
#define EIK_THETA_ESTIMATE 1
#define EIK_THETA_REFERENCE 2
#define EIK_THETA_FIELD 3

/* Coarse solver of Steps 1 and 4 (Sec. 3.2 uses C_H; Sec. 5.3 replaces it,
 * on the squares medium, by a solver of the homogenised equation eq. homog):
 *   EIK_COARSE_GODUNOV  C_H: the Godunov scheme of |grad U| = r on the lattice.
 *   EIK_COARSE_L1       the homogenised solver of a medium whose optimal paths
 *                       run along the axes (travel cost r (|a1| + |a2| (+ |a3|))
 *                       per unit length in direction a): the upwind scheme of
 *                       max_a |dU/dx_a| = r, i.e. the smallest neighbour plus
 *                       r*H, which makes U r times the lattice L1 distance.
 *                       r is the slowness at the coarse node (1 on every node of
 *                       the squares medium).  The fine solver is unchanged.
 * The choice changes the iterates, not the fixed point: a converged run gives
 * the fine solution u^f either way. */
#define EIK_COARSE_GODUNOV 0
#define EIK_COARSE_L1 1

/* How the DD iteration issues its kernels; the kernels and the results are
 * the same in every mode.  A mode that does not apply to a call is taken as
 * EIK_LAUNCH_STREAM.
 *   EIK_LAUNCH_STREAM      every kernel launched on the stream; the
 *                          subdomain and lattice kernels with one block per
 *                          box.  eik_dd_solve (d = 2) launches several
 *                          iterations ahead of its check of the stopping rule
 *                          (an iteration after the one that stopped returns
 *                          at once and changes nothing).
 *   EIK_LAUNCH_GRAPH       eik_dd_solve, d = 2: each whole block of launched-
 *                          ahead iterations after the first is replayed from
 *                          a HIP graph, captured once and kept per device
 *                          for the next call with the same arguments and
 *                          workspace (else captured again).  The debug
 *                          snapshots, EIK_THETA_ESTIMATE and
 *                          eik_dd_solve_noalloc use stream launches;
 *                          ms_fine, ms_correct and ms_causal cover only the
 *                          stream-launched iterations.
 *   EIK_LAUNCH_PERSISTENT  eik_dd_solve_batch (from the first problem's
 *                          options): Steps 3 and 4 run on a grid of the
 *                          blocks that are resident at once (at most
 *                          persistent_blocks per compute unit when that is
 *                          set), each taking the (problem, box) items in
 *                          order from a counter. */
#define EIK_LAUNCH_STREAM 0
#define EIK_LAUNCH_GRAPH 1
#define EIK_LAUNCH_PERSISTENT 2

/* Options of the domain-decomposition iteration (Sec. 3.2). */
typedef struct {
    int32_t S;          /* subdomain side in fine cells; (n[a]-1) % S == 0 */
    int32_t M;          /* coarse spacing H/h in fine cells; S % M == 0, M >= 2 */
    double theta;       /* parareal weight theta in [0,1] (Sec. 2, eq. wtdparasimp) */
    double tol;         /* stop when max |U^{k+1} - U^k| over the coarse nodes < tol (or == 0) */
    int32_t max_iter;   /* cap on DD iterations (0: only Step 1) */
    int32_t max_fine_sweeps;   /* cap on FSM sweeps per subdomain per iteration (>= 1) */
    int32_t max_coarse_sweeps; /* cap on sweeps per coarse lattice in Steps 1 and 4 (>= 1) */
    int32_t theta_mode;        /* EIK_THETA_*; 0 = constant */
    const void* U_init;        /* optional resume state (device, full grid, grid dtype): U^k ... */
    const int8_t* W_init;      /* ... and W^k codes; both NULL = run Step 1 */
    const eik_dd_debug* debug; /* optional snapshots, NULL = none */
    const void* theta_ref;     /* device, N, grid dtype: u_ref (REFERENCE) or theta (FIELD); else unused */
    double theta_params[7];    /* gamma, delta, x0, omega0, omega1, omega2, margin (ESTIMATE and
                                * REFERENCE; the paper's values are 0.75, 0.01, 0.9, -, -, -, 0.001;
                                * the omegas are not stated there) */
    int32_t coarse_solver;     /* EIK_COARSE_*; 0 = C_H */
    int32_t launch_mode;       /* EIK_LAUNCH_*; 0 = stream launches, one block per box */
    int32_t persistent_blocks; /* EIK_LAUNCH_PERSISTENT: resident blocks per compute unit for
                                * Steps 3 and 4, capped at what fits (0 = as many as fit); each
                                * block takes boxes until none is left, so fewer blocks means
                                * more boxes per block.  >= 0 */
} eik_dd_opts;

/* Host-side statistics.  residual_history (host, may be NULL) receives
 * max|U^{k+1}-U^k| of up to history_cap iterations. */
typedef struct {
    int32_t iterations;      /* DD iterations run */
    int32_t converged;       /* 1 if the residual went below tol */
    int64_t fine_updates;    /* local solves evaluated in Step 3: sum over subdomains of (non-Gamma nodes) x (sweeps) */
    int64_t coarse_updates;  /* the same for the coarse lattices in Steps 1 and 4 */
    int64_t sweeps;          /* eik_solve: sweeps run */
    double final_residual;
    double* residual_history;
    int32_t history_cap;
    float ms_total;          /* device time of the whole call */
    float ms_fine;           /* device time in Step 3 (subdomain FSM) */
    float ms_coarse;         /* device time in everything else (Steps 1, 2, 4, causal sweeps, residuals) */
    float ms_correct;        /* device time of the Step 4 lattice sweeps (incl. the reconciliation) */
    float ms_causal;         /* device time of the causal sweeps after Step 4 and the residuals */
    /* eik_dd_solve with d = 2 (eik_dd_solve_noalloc too) writes these; other
     * calls leave them as they are.  The leading wave of every subdomain box
     * [0] (Step 3) and lattice box [1] (Step 4): anti-diagonal steps it ran
     * and clock64 ticks it spent in them, summed over boxes and iterations
     * (ticks / steps = the time of one dependent step). */
    int64_t lead_steps[2];
    int64_t lead_ticks[2];
} eik_stats;

/* eik_solve -- the fast sweeping method on the whole fine grid (Sec. 1.1:
 * Gamma nodes fixed at g, all others start at +inf; Gauss-Seidel sweeps in
 * the 2^d orderings of the paper's loop nest with u = min(u, u~), eq.
 * FSMupdate), stopped after the first sweep that changes no value or after
 * max_sweeps.  This is the "overall fine solution" u^f of Secs. 4-5.
 *   r        device, N elements of grid dtype, > 0 and finite
 *   u_out    device, N elements of grid dtype (must not alias r)
 *   wind_out device, N int8 wind codes, or NULL
 *   stats    host, or NULL (fields iterations/converged/sweeps/ms_total)
 * Returns EIK_ERR_NOCONV (outputs written) if max_sweeps was reached. */
eik_status eik_solve(const eik_grid* grid, const void* r, const eik_gamma* gamma,
                     int32_t max_sweeps, void* u_out, int8_t* wind_out, eik_stats* stats,
                     void* hip_stream);

/* eik_dd_solve -- the two-scale DD iteration of Sec. 3.2:
 *   Step 1  FSM on every shifted coarse lattice with Alg. update2D, then the
 *           causal sweep (Alg. causalsweep2D) -> U^0, W^0 (skipped when
 *           opts->U_init / W_init are given);
 *   Step 2  subdomain boundary data from (U^k, W^k) (inflow test W . n > 0);
 *   Step 3  FSM on every subdomain with Alg. fineupdate2D, then the
 *           reconciliation of Alg. fineupdate at the coarse nodes -> u^k, w^k;
 *   Step 4  Alg. 2Dweightedupdate sweeps on every lattice, then the causal
 *           sweep -> U^{k+1}, W^{k+1};
 * repeated until max|U^{k+1} - U^k| < tol.
 *   r      device, N elements, > 0 and finite
 *   u_out  device, N: the subdomain solutions of the last Step 3 patched
 *          together (coarse nodes take u^k); NaN if max_iter == 0
 *   U_out  device, N or NULL: U of the last iterate, NaN off the skeleton
 *   W_out  device, N int8 codes or NULL: W of the last iterate
 * Resume: passing (U_out, W_out) of a run as opts->U_init/W_init continues
 * it exactly (the iteration reads nothing else).
 * Limits: d = 2 with subdomain side S+1 <= 65 nodes and lattice extents
 * (n-1)/M + 1 <= 65; d = 3 with S+1 <= 34 and (n-1)/M + 1 <= 34 and the box
 * in 160 KB of LDS ((S+1)^3 values of the grid dtype); with a non-constant
 * theta_mode on 65-node lattices in fp64, Step 4 keeps its per-node weight
 * terms in global memory (they do not fit in LDS beside the lattice). */
eik_status eik_dd_solve(const eik_grid* grid, const void* r, const eik_gamma* gamma,
                        const eik_dd_opts* opts, void* u_out, void* U_out, int8_t* W_out,
                        eik_stats* stats, void* hip_stream);

/* eik_dd_solve_noalloc -- eik_dd_solve for callers that cannot allocate
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, same iteration and kernels, and
 * bitwise the same outputs and counters as eik_dd_solve; it calls no
 * hipMalloc, hipFree, hipHostMalloc or event creation.  Its scratch (every
 * buffer eik_dd_solve takes from its workspace) is carved from one fixed
 * array of EIK_NOALLOC_SCRATCH_BYTES in device memory, one copy per device,
 * which the library holds until the process ends; its device address is
 * looked up on the first call on each device.
 *   - Limit: the problem's scratch must fit in EIK_NOALLOC_SCRATCH_BYTES,
 *     else EIK_ERR_UNSUPPORTED (the message gives the size needed).  About
 *     50 bytes per node in fp32 and 78 in fp64 (a 1025^2 grid needs 52.5 MB
 *     in fp32, 82 MB in fp64), 4 values of the grid dtype more per node
 *     with EIK_THETA_ESTIMATE, plus the subdomain edge buffers.
 *   - d = 2 only (d = 3 gives EIK_ERR_UNSUPPORTED).
 *   - stats: the ms_* fields are 0 (no events); everything else as
 *     eik_dd_solve.
 *   - Every call on a device shares that device's array, which keeps the
 *     last call's contents; each call clears what must start at zero.  Calls
 *     that overlapped on one device would race on the array; within a
 *     process the library prevents that by serialising the calls on a
 *     device (the same lock as the other entry points), and each call
 *     synchronises its stream before returning. */
#define EIK_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
eik_status eik_dd_solve_noalloc(const eik_grid* grid, const void* r, const eik_gamma* gamma,
                                const eik_dd_opts* opts, void* u_out, void* U_out, int8_t* W_out,
                                eik_stats* stats, void* hip_stream);

/* eik_solve_batch -- eik_solve for nb problems on one grid and slowness,
 * each with its own Gamma (e.g. one point source each): every launch of a
 * sweep covers one box diagonal of all problems that have not yet had a
 * sweep without change.  Problem b's u and winds are exactly those of its
 * own eik_solve (a problem whose sweep changed nothing is stationary and is
 * not swept again).
 *   gammas    host array of nb boundary sets
 *   u_out     device, nb x N (problem b at offset b*N)
 *   wind_out  device, nb x N codes, or NULL
 *   stats     host array of nb entries or NULL (sweeps per problem; device
 *             time of the whole call)
 * d = 2: the problems' sweeps share launches; d = 3: the problems are solved
 * one after another on the stream, each as by its own eik_solve. */
eik_status eik_solve_batch(const eik_grid* grid, const void* r, int32_t nb, const eik_gamma* gammas,
                           int32_t max_sweeps, void* u_out, int8_t* wind_out, eik_stats* stats,
                           void* hip_stream);

/* eik_dd_solve_batch -- eik_dd_solve on nprob independent problems at once
 * (one dtype; the subdomains of Sec. 3.2 and the problems are all
 * independent work).  d = 2: every DD step is one launch over the
 * subdomains, lattices and causal-sweep segments of all problems that have
 * not yet converged, and one readback per iteration serves all residuals.
 * d = 3 (every problem 3D; mixing 2D and 3D gives EIK_ERR_UNSUPPORTED): the
 * problems run one after another on the stream.  Problem
 * p stops like its own eik_dd_solve would (its tol / max_iter), and its
 * outputs are exactly those of eik_dd_solve(grids[p], r[p], &gammas[p],
 * &opts[p], u_out[p], U_out[p], W_out[p]).
 *   grids, gammas, opts, stats  host arrays of nprob entries (opts[p].debug
 *                               must be NULL); stats may be NULL; the
 *                               device-time fields of every entry hold the
 *                               batch's totals
 *   r, u_out                    host arrays of nprob device pointers
 *   U_out, W_out                host arrays of nprob device pointers (entries
 *                               may be NULL) or NULL
 * Returns EIK_ERR_NOCONV if any problem reached its max_iter (all outputs
 * written). */
eik_status eik_dd_solve_batch(int32_t nprob, const eik_grid* grids, const void* const* r,
                              const eik_gamma* gammas, const eik_dd_opts* opts, void* const* u_out,
                              void* const* U_out, int8_t* const* W_out, eik_stats* stats, void* hip_stream);

/* eik_adjoint_batch -- gradient of a loss L of converged travel times with
 * respect to the slowness, for nb problems on one grid and slowness (e.g.
 * one per source), by the discrete adjoint of the upwind scheme (eq.
 * godonuv).  Not a step of the paper's method.  At a free node x whose
 * converged update used the axes A (the nonzero components of its fine wind,
 * Alg. fineupdate2D) with upwind neighbours u_a:
 *     S = sum_{a in A} (u - u_a),  c_a = (u - u_a)/S,  q = (r h) h / S,
 * so du = sum_a c_a du_a + q dr.  The adjoint field lambda solves
 * lambda(y) = dL/du(y) + sum of c(x -> y) lambda(x) over the neighbours x
 * that use y (terms in the order x-, x+, y- of y, y+ of y), found by
 * Gauss-Seidel sweeps of the whole grid in the paper's four orders until a
 * sweep changes nothing; dL/dr = sum over the batch, in order, of lambda q.
 * Gamma nodes and unreached nodes (u = +inf) carry no equation.
 *   gammas     host array of nb boundary sets (device pointers inside)
 *   u          device, nb x N, grid dtype: converged solutions (eik_solve)
 *   wind       device, nb x N wind codes from the same solves, or NULL:
 *              recomputed from u with the fine rule
 *   dL_du      device, nb x N, grid dtype
 *   dL_dr_out  device, N, grid dtype (overwritten)
 *   lambda_out device, nb x N, or NULL
 *   stats      host or NULL: sweeps, ms_total
 * d = 3: three axes, six terms in the order x-, x+, y-, y+, z-, z+, and
 * Gauss-Seidel sweeps in the eight orders of eik_solve in 3D.
 * Returns EIK_ERR_NOCONV if max_sweeps was reached. */
eik_status eik_adjoint_batch(const eik_grid* grid, const void* r, int32_t nb, const eik_gamma* gammas,
                             const void* u, const int8_t* wind, const void* dL_du, void* dL_dr_out,
                             void* lambda_out, int32_t max_sweeps, eik_stats* stats, void* hip_stream);

/* eik_adjoint -- eik_adjoint_batch for one problem (nb = 1, no lambda, no
 * stats, sweep cap 100000). */
eik_status eik_adjoint(const eik_grid* grid, const void* r, const eik_gamma* gamma,
                       const void* u, const int8_t* wind, const void* dL_du, void* dL_dr_out,
                       void* hip_stream);

/* Message for the last non-OK status returned to the calling thread. */
const char* eik_last_error(void);

/* Frees the workspace held on every device.  Returns EIK_OK. */
eik_status eik_release(void);

/* Library version string. */
const char* eik_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIK_H */
