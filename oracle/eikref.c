/*
 * eikref.c -- CPU ORACLE for the two-scale domain-decomposition Eikonal
 * solver of Martin & Tsai (arXiv 1805.04198).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library: every step below is written out
 * again, serially and plainly, from the paper.
 *
 * It is compiled twice: with REAL=double (the oracle proper) and with
 * REAL=float (so that an fp32 kernel's discrete decisions -- winds, branch
 * choices, stopping -- can be compared in the kernel's own precision).
 * Build with -O2 -ffp-contract=off and without fast-math: every expression
 * below is evaluated exactly as written, in REAL precision.
 *
 * Grid: d = 2 or 3 axes, n[a] nodes per axis, node (i,j,k) at linear index
 * i + n0*(j + n1*k) (x fastest).  Winds are stored per axis as signed chars,
 * array [a*N + node], with the flow-direction convention: component +1
 * means the upwind neighbour lies on the minus side of that axis.
 *
 * Function map (paper section / algorithm):
 *   local_solve      -- Godunov upwind scheme (eq. godonuv, Sec. 1.1) in the
 *                       closed form of the coarse solver C_H (Sec. 3.2), with
 *                       the wind rules of Alg. fineupdate2D (fine) and
 *                       Alg. update2D (coarse); 3D by the sorted cascade.
 *                       Rule 2 is the homogenised coarse solver of the
 *                       squares medium (Sec. 5.3, eq. homog): smallest
 *                       neighbour plus r*H, i.e. r times the lattice L1
 *                       distance, used in place of C_H in Steps 1 and 4
 *                       when eikref_dd is given coarse_solver = 1.
 *   fsm_run          -- fast sweeping method (Sec. 1.1: initialisation, the
 *                       2^d orderings, eq. FSMupdate).
 *   eikref_fsm       -- FSM on the whole fine grid: the "overall fine
 *                       solution" u^f.
 *   eikref_fmm       -- fast marching (Sec. 1.1), an independent solver of
 *                       the same discrete system, used only to pin eikref_fsm.
 *   eikref_dd        -- the domain-decomposition iteration of Sec. 3.2:
 *                       Step 1 (coarse FSM on every shifted lattice with
 *                       Alg. update2D, then Alg. causalsweep2D), Step 2
 *                       (subdomain boundary data g), Step 3 (subdomain FSM with
 *                       Alg. fineupdate2D, then Alg. fineupdate), Step 4
 *                       (Alg. 2Dweightedupdate sweeps, then the causal sweep),
 *                       repeated until max|U^{k+1}-U^k| < tol.
 *   theta_node       -- the weight of the Step 4 correction at one node:
 *                       constant, the estimate of eqs. secthetaest and
 *                       thetaest (Sec. 4.2), the reference weight M-bar
 *                       minus a margin (Sec. 5.3), or a caller field.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
#ifndef SFX
#define SFX _f64
#endif
#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define NAME(x) CAT(x, SFX)

typedef REAL real;
#define RINF ((real)INFINITY)

#if defined(ORACLE_FLOAT)
#define RSQRT_(x) sqrtf(x)
#define RABS_(x) fabsf(x)
#else
#define RSQRT_(x) sqrt(x)
#define RABS_(x) fabs(x)
#endif

enum { OK = 0, ERR_ARG = -1, ERR_SHAPE = -2, ERR_NOCONV = -3, ERR_NOMEM = -7 };

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int d;
    int64_t L[3];   /* extent per axis (1 for unused axes) */
    int64_t st[3];  /* strides */
    int64_t cnt;
} box;

static void box_init(box* B, int d, const int64_t* L) {
    B->d = d;
    for (int a = 0; a < 3; a++) B->L[a] = (a < d) ? L[a] : 1;
    B->st[0] = 1;
    B->st[1] = B->L[0];
    B->st[2] = B->L[0] * B->L[1];
    B->cnt = B->L[0] * B->L[1] * B->L[2];
}

static void box_coords(const box* B, int64_t idx, int64_t c[3]) {
    c[0] = idx % B->L[0];
    idx /= B->L[0];
    c[1] = idx % B->L[1];
    c[2] = idx / B->L[1];
}

/* Sweep direction number dir in [0, 2^d): the paper's loop nest takes
 * s1 in {-1,+1} outermost, then s2 (then s3), so bit (d-1-a) of dir gives
 * the sign of axis a. */
static int dir_sign(int d, int dir, int a) { return ((dir >> (d - 1 - a)) & 1) ? 1 : -1; }

/* ------------------------------------------------------------------ */
/* local solve (eq. godonuv; closed form of C_H in Sec. 3.2)           */
/* ------------------------------------------------------------------ */

/* m[a]  : the smaller of the two neighbours along axis a (+inf if none)
 * ws[a] : wind sign of that choice (+1: minus-side neighbour, -1: plus side;
 *         ties take the plus side, as the strict '<' in the algorithms)
 * rd    : r * Delta (Delta = h on the fine grid, H on a coarse lattice)
 * rule  : 0 = fine wind rule (Alg. fineupdate2D), 1 = coarse (Alg. update2D),
 *         2 = the homogenised coarse solver of the squares medium (coarse winds)
 * wt    : output wind of the candidate value */
static real local_solve(int d, const real* m, const signed char* ws, real rd, int rule,
                        signed char* wt) {
    if (rule == 2) {
        /* the homogenised coarse solver of the squares medium (Sec. 5.3):
         * optimal paths run along grid lines, so the effective metric is the
         * L1 distance and its upwind scheme, max(|u_x|, |u_y|) = r, gives
         * the smallest neighbour plus r Delta; winds by the coarse rule */
        real mn = m[0];
        for (int a = 1; a < d; a++)
            if (m[a] < mn) mn = m[a];
        real ut = mn + rd;
        for (int a = 0; a < 3; a++) wt[a] = 0;
        if (d == 2) {
            if (ut < m[1]) {
                wt[0] = ws[0];
            } else if (ut < m[0]) {
                wt[1] = ws[1];
            } else {
                wt[0] = ws[0];
                wt[1] = ws[1];
            }
        } else {
            for (int a = 0; a < 3; a++) wt[a] = (ut < m[a]) ? 0 : ws[a];
        }
        return ut;
    }
    if (d == 2) {
        real a = m[0], b = m[1];
        real dd = a - b;
        real ut;
        int two = RABS_(dd) < rd;
        if (two) {
            real t = rd * rd;
            t = t + t;
            t = t - dd * dd;
            ut = ((a + b) + RSQRT_(t)) * (real)0.5;
        } else {
            ut = (a < b) ? (a + rd) : (b + rd);
        }
        if (rule == 0) {
            /* Alg. fineupdate2D: two-sided -> both axes; one-sided -> the
             * axis of the smaller neighbour */
            if (two) {
                wt[0] = ws[0];
                wt[1] = ws[1];
            } else if (a < b) {
                wt[0] = ws[0];
                wt[1] = 0;
            } else {
                wt[0] = 0;
                wt[1] = ws[1];
            }
        } else {
            /* Alg. update2D: U~ < b -> x only; else U~ < a -> y only; else both */
            if (ut < b) {
                wt[0] = ws[0];
                wt[1] = 0;
            } else if (ut < a) {
                wt[0] = 0;
                wt[1] = ws[1];
            } else {
                wt[0] = ws[0];
                wt[1] = ws[1];
            }
        }
        return ut;
    }
    /* d == 3: sort the three axis minima ascending (stable in axis order),
     * take the one-sided value, then the two-, then the three-sided root of
     * sum_a ((u - m_a)^+)^2 = rd^2 as long as the next neighbour is below. */
    int p[3] = {0, 1, 2};
    for (int x = 1; x < 3; x++)
        for (int y = x; y > 0 && m[p[y]] < m[p[y - 1]]; y--) {
            int t = p[y];
            p[y] = p[y - 1];
            p[y - 1] = t;
        }
    real a1 = m[p[0]], a2 = m[p[1]], a3 = m[p[2]];
    real ut;
    int used;
    real d12 = a1 - a2;
    if (!(RABS_(d12) < rd)) {
        ut = a1 + rd;
        used = 1;
    } else {
        real t = rd * rd;
        t = t + t;
        t = t - d12 * d12;
        real u2 = ((a1 + a2) + RSQRT_(t)) * (real)0.5;
        if (!(a3 < u2)) {
            ut = u2;
            used = 2;
        } else {
            real d13 = a1 - a3, d23 = a2 - a3;
            real q = rd * rd;
            q = (q + q) + q;
            q = q - ((d12 * d12 + d13 * d13) + d23 * d23);
            if (q < (real)0) q = (real)0;
            ut = (((a1 + a2) + a3) + RSQRT_(q)) / (real)3;
            used = 3;
        }
    }
    for (int a = 0; a < 3; a++) wt[a] = 0;
    if (rule == 0) {
        for (int x = 0; x < used; x++) wt[p[x]] = ws[p[x]];
    } else {
        /* coarse rule in 3D: an axis contributes unless U~ lies below its
         * neighbour minimum (the 2D Alg. update2D tests, taken per axis) */
        for (int a = 0; a < 3; a++) wt[a] = (ut < m[a]) ? 0 : ws[a];
    }
    return ut;
}

/* neighbour minima of node idx in box B along each axis */
static void gather(const box* B, const real* u, int64_t idx, real* m, signed char* ws) {
    int64_t c[3];
    box_coords(B, idx, c);
    for (int a = 0; a < B->d; a++) {
        real lo = (c[a] > 0) ? u[idx - B->st[a]] : RINF;
        real hi = (c[a] < B->L[a] - 1) ? u[idx + B->st[a]] : RINF;
        if (lo < hi) {
            m[a] = lo;
            ws[a] = 1;
        } else {
            m[a] = hi;
            ws[a] = -1;
        }
    }
    for (int a = B->d; a < 3; a++) {
        m[a] = RINF;
        ws[a] = 0;
    }
}

/* ------------------------------------------------------------------ */
/* fast sweeping (Sec. 1.1)                                            */
/* ------------------------------------------------------------------ */

/* visit every node of box B in the lexicographic order of sweep dir
 * (axis 0 outermost) and call fn on it */
typedef int (*node_fn)(const box* B, int64_t idx, void* ctx);

static int64_t sweep_box(const box* B, int dir, node_fn fn, void* ctx) {
    int64_t changed = 0;
    int s0 = dir_sign(B->d, dir, 0), s1 = dir_sign(B->d, dir, 1);
    int s2 = (B->d == 3) ? dir_sign(B->d, dir, 2) : 1;
    for (int64_t q0 = 0; q0 < B->L[0]; q0++) {
        int64_t i = (s0 > 0) ? q0 : B->L[0] - 1 - q0;
        for (int64_t q1 = 0; q1 < B->L[1]; q1++) {
            int64_t j = (s1 > 0) ? q1 : B->L[1] - 1 - q1;
            for (int64_t q2 = 0; q2 < B->L[2]; q2++) {
                int64_t k = (s2 > 0) ? q2 : B->L[2] - 1 - q2;
                changed += fn(B, i + B->L[0] * (j + B->L[1] * k), ctx);
            }
        }
    }
    return changed;
}

/* Sweep in the 2^d orders in turn until a whole sweep changes nothing.  A
 * sweep that changes nothing has evaluated every node on the final state,
 * so the state is then stationary for every ordering.  Returns 1 if that
 * happened within max_sweeps, and the number of sweeps run. */
static int run_sweeps(const box* B, int max_sweeps, node_fn fn, void* ctx, int64_t* nsweeps) {
    int nd = 1 << B->d;
    int64_t s = 0;
    int conv = 0;
    while (s < max_sweeps) {
        int64_t ch = sweep_box(B, (int)(s % nd), fn, ctx);
        s++;
        if (ch == 0) {
            conv = 1;
            break;
        }
    }
    *nsweeps = s;
    return conv;
}

typedef struct {
    real* u;
    signed char* w;        /* [a*cnt + idx] */
    const unsigned char* fixed;
    const real* rd;        /* r*Delta per node */
    int rule;
} fsm_ctx;

/* eq. FSMupdate: u_new = min(u_curr, u~), wind recorded with the value */
static int fsm_node(const box* B, int64_t idx, void* vctx) {
    fsm_ctx* C = (fsm_ctx*)vctx;
    if (C->fixed[idx]) return 0;
    real m[3];
    signed char ws[3], wt[3];
    gather(B, C->u, idx, m, ws);
    real ut = local_solve(B->d, m, ws, C->rd[idx], C->rule, wt);
    if (ut < C->u[idx]) {
        C->u[idx] = ut;
        for (int a = 0; a < B->d; a++) C->w[a * B->cnt + idx] = wt[a];
        return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* argument checks                                                     */
/* ------------------------------------------------------------------ */

static int check_problem(int d, const int64_t* n, double h, const real* r, int64_t ng,
                         const int64_t* gidx, const real* gval, int64_t* Nout) {
    if (d != 2 && d != 3) return ERR_ARG;
    if (!(h > 0) || !isfinite(h)) return ERR_ARG;
    int64_t N = 1;
    for (int a = 0; a < d; a++) {
        if (n[a] < 2) return ERR_SHAPE;
        N *= n[a];
    }
    for (int64_t x = 0; x < N; x++)
        if (!(r[x] > 0) || !isfinite((double)r[x])) return ERR_ARG;
    if (ng < 0) return ERR_ARG;
    for (int64_t g = 0; g < ng; g++) {
        if (gidx[g] < 0 || gidx[g] >= N) return ERR_ARG;
        if (g > 0 && gidx[g] <= gidx[g - 1]) return ERR_ARG;
        if (!isfinite((double)gval[g])) return ERR_ARG;
    }
    *Nout = N;
    return OK;
}

/* ------------------------------------------------------------------ */
/* FSM on the whole fine grid: u^f                                     */
/* ------------------------------------------------------------------ */

/* info[0] = sweeps run, info[1] = local solves evaluated (free nodes x
 * sweeps), info[2] = 1 if stationary.  w may be NULL. */
/* u_init (may be NULL): start from these values instead of +inf (Gamma
 * nodes still take g).  A run cut into pieces of whole cycles of 2^d sweeps,
 * each resumed from the last one's u, visits the same directions on the same
 * values as one uninterrupted run (the min update does not read the winds),
 * so its values and total sweep count are the same; the winds then record
 * only the updates after the last resume. */
int NAME(eikref_fsm)(int d, const int64_t* n, double h, const real* r, int64_t ng,
                     const int64_t* gidx, const real* gval, int max_sweeps, real* u,
                     signed char* w, int64_t* info, const real* u_init) {
    int64_t N;
    int st = check_problem(d, n, h, r, ng, gidx, gval, &N);
    if (st != OK) return st;
    box B;
    box_init(&B, d, n);
    real hT = (real)h;
    unsigned char* fixed = (unsigned char*)calloc((size_t)N, 1);
    real* rd = (real*)malloc(sizeof(real) * (size_t)N);
    signed char* ww = (signed char*)calloc((size_t)(d * N), 1);
    if (!fixed || !rd || !ww) {
        free(fixed);
        free(rd);
        free(ww);
        return ERR_NOMEM;
    }
    for (int64_t x = 0; x < N; x++) {
        u[x] = u_init ? u_init[x] : RINF;
        rd[x] = r[x] * hT;
    }
    /* initialisation: boundary data fixed, all else a large value (+inf) */
    for (int64_t g = 0; g < ng; g++) {
        fixed[gidx[g]] = 1;
        u[gidx[g]] = gval[g];
    }
    fsm_ctx C = {u, ww, fixed, rd, 0};
    int64_t ns = 0;
    int conv = run_sweeps(&B, max_sweeps, fsm_node, &C, &ns);
    if (info) {
        info[0] = ns;
        info[1] = (N - ng) * ns;
        info[2] = conv;
    }
    if (w) memcpy(w, ww, (size_t)(d * N));
    free(fixed);
    free(rd);
    free(ww);
    return conv ? OK : ERR_NOCONV;
}

/* ------------------------------------------------------------------ */
/* fast marching on the same discrete system (independent check)       */
/* ------------------------------------------------------------------ */

typedef struct {
    real* key;
    int64_t* node;
    int64_t* pos;  /* heap position per grid node, -1 if absent */
    int64_t size;
} heap;

static void heap_swap(heap* Hp, int64_t a, int64_t b) {
    real k = Hp->key[a];
    Hp->key[a] = Hp->key[b];
    Hp->key[b] = k;
    int64_t t = Hp->node[a];
    Hp->node[a] = Hp->node[b];
    Hp->node[b] = t;
    Hp->pos[Hp->node[a]] = a;
    Hp->pos[Hp->node[b]] = b;
}

static void heap_up(heap* Hp, int64_t x) {
    while (x > 0) {
        int64_t p = (x - 1) / 2;
        if (Hp->key[x] < Hp->key[p]) {
            heap_swap(Hp, x, p);
            x = p;
        } else
            break;
    }
}

static void heap_down(heap* Hp, int64_t x) {
    for (;;) {
        int64_t l = 2 * x + 1, r = l + 1, m = x;
        if (l < Hp->size && Hp->key[l] < Hp->key[m]) m = l;
        if (r < Hp->size && Hp->key[r] < Hp->key[m]) m = r;
        if (m == x) break;
        heap_swap(Hp, x, m);
        x = m;
    }
}

static void heap_push_or_decrease(heap* Hp, int64_t node, real key) {
    int64_t p = Hp->pos[node];
    if (p < 0) {
        p = Hp->size++;
        Hp->key[p] = key;
        Hp->node[p] = node;
        Hp->pos[node] = p;
        heap_up(Hp, p);
    } else if (key < Hp->key[p]) {
        Hp->key[p] = key;
        heap_up(Hp, p);
    }
}

static int64_t heap_pop(heap* Hp) {
    int64_t node = Hp->node[0];
    Hp->pos[node] = -1;
    Hp->size--;
    if (Hp->size > 0) {
        Hp->key[0] = Hp->key[Hp->size];
        Hp->node[0] = Hp->node[Hp->size];
        Hp->pos[Hp->node[0]] = 0;
        heap_down(Hp, 0);
    }
    return node;
}

/* Nodes are accepted in increasing value order; a trial node's value is
 * the local solve over its accepted neighbours only. */
int NAME(eikref_fmm)(int d, const int64_t* n, double h, const real* r, int64_t ng,
                     const int64_t* gidx, const real* gval, real* u) {
    int64_t N;
    int st = check_problem(d, n, h, r, ng, gidx, gval, &N);
    if (st != OK) return st;
    box B;
    box_init(&B, d, n);
    real hT = (real)h;
    unsigned char* acc = (unsigned char*)calloc((size_t)N, 1);
    unsigned char* fixed = (unsigned char*)calloc((size_t)N, 1);
    real* known = (real*)malloc(sizeof(real) * (size_t)N);
    heap Hp;
    Hp.key = (real*)malloc(sizeof(real) * (size_t)N);
    Hp.node = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    Hp.pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    Hp.size = 0;
    if (!acc || !fixed || !known || !Hp.key || !Hp.node || !Hp.pos) {
        free(acc); free(fixed); free(known); free(Hp.key); free(Hp.node); free(Hp.pos);
        return ERR_NOMEM;
    }
    for (int64_t x = 0; x < N; x++) {
        u[x] = RINF;
        known[x] = RINF;
        Hp.pos[x] = -1;
    }
    for (int64_t g = 0; g < ng; g++) {
        fixed[gidx[g]] = 1;
        u[gidx[g]] = gval[g];
        heap_push_or_decrease(&Hp, gidx[g], gval[g]);
    }
    while (Hp.size > 0) {
        int64_t x = heap_pop(&Hp);
        acc[x] = 1;
        known[x] = u[x];
        int64_t c[3];
        box_coords(&B, x, c);
        for (int a = 0; a < d; a++) {
            for (int sg = -1; sg <= 1; sg += 2) {
                int64_t cc = c[a] + sg;
                if (cc < 0 || cc >= B.L[a]) continue;
                int64_t y = x + sg * B.st[a];
                if (acc[y] || fixed[y]) continue;
                real m[3];
                signed char ws[3], wt[3];
                gather(&B, known, y, m, ws);
                real ut = local_solve(d, m, ws, r[y] * hT, 0, wt);
                if (ut < u[y]) {
                    u[y] = ut;
                    heap_push_or_decrease(&Hp, y, ut);
                }
            }
        }
    }
    free(acc); free(fixed); free(known); free(Hp.key); free(Hp.node); free(Hp.pos);
    return OK;
}

/* ------------------------------------------------------------------ */
/* the domain-decomposition iteration (Sec. 3.2)                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int d;
    int64_t n[3], st[3], N;
    int S, M;
    int64_t P[3];   /* subdomains per axis */
    real hT, HT, thetaT;
    const real* r;
    unsigned char* isg;   /* Gamma flag per node */
    real* gv;             /* Gamma data per node */
    /* weight of the Step 4 correction (theta_node) */
    int crule;            /* coarse solver: 1 = C_H (Sec. 3.2), 2 = homogenised (Sec. 5.3) */
    int theta_mode;       /* 0 constant, 1 estimate, 2 reference, 3 field */
    int inflow_fixed;     /* test-only reading of Step 2: inflow nodes held at U (see tile_solve) */
    double tpar[7];       /* gamma, delta, x0, omega0, omega1, omega2, margin */
    const real* tref;     /* mode 2: u^f per node; mode 3: theta per node */
    const real* ukm1;     /* u^{k-1} per node, or NULL before there is one */
    const real* ckm1;     /* C^{k-1} per node, or NULL */
    const real* ckm2;     /* C^{k-2} per node, or NULL */
} ddp;

static void node_coords(const ddp* D, int64_t x, int64_t c[3]) {
    c[0] = x % D->n[0];
    x /= D->n[0];
    c[1] = x % D->n[1];
    c[2] = x / D->n[1];
    if (D->d == 2) c[2] = 0;
}

static int64_t node_index(const ddp* D, const int64_t c[3]) {
    return c[0] + D->n[0] * (c[1] + D->n[1] * (D->d == 3 ? c[2] : 0));
}

/* a coarse node lies on a coarse grid line/plane: some index = 0 mod M */
static int is_coarse(const ddp* D, const int64_t c[3]) {
    for (int a = 0; a < D->d; a++)
        if (c[a] % D->M == 0) return 1;
    return 0;
}

/* axis a is an interface axis of the node: the node lies on a subdomain
 * boundary plane that is not the domain boundary */
static int is_iface_axis(const ddp* D, const int64_t c[3], int a) {
    return (c[a] % D->S == 0) && c[a] > 0 && c[a] < D->n[a] - 1;
}

/* ---- one coarse lattice as a dense box ---- */
typedef struct {
    int64_t off[3];   /* offsets in [0, M) */
    box B;
} lattice;

/* number of lattices = offsets in [0,M)^d with at least one zero */
static int64_t lattice_list(const ddp* D, lattice** out) {
    int64_t M = D->M;
    int64_t tot = (D->d == 2) ? M * M : M * M * M;
    lattice* L = (lattice*)malloc(sizeof(lattice) * (size_t)tot);
    int64_t cnt = 0;
    for (int64_t o0 = 0; o0 < M; o0++)
        for (int64_t o1 = 0; o1 < M; o1++)
            for (int64_t o2 = 0; o2 < (D->d == 3 ? M : 1); o2++) {
                int64_t o[3] = {o0, o1, o2};
                int z = 0;
                for (int a = 0; a < D->d; a++) z |= (o[a] == 0);
                if (!z) continue;
                lattice* l = &L[cnt++];
                int64_t ext[3];
                for (int a = 0; a < 3; a++) {
                    l->off[a] = o[a];
                    ext[a] = (a < D->d) ? (D->n[a] - 1 - o[a]) / M + 1 : 1;
                }
                box_init(&l->B, D->d, ext);
            }
    *out = L;
    return cnt;
}

static int64_t lattice_global(const ddp* D, const lattice* l, int64_t li) {
    int64_t p[3], c[3];
    box_coords(&l->B, li, p);
    for (int a = 0; a < 3; a++) c[a] = l->off[a] + p[a] * D->M;
    return node_index(D, c);
}

/* ---- Step 1: coarse initialisation on every lattice ---- */
static int64_t step1_init(const ddp* D, real* U, signed char* W, int max_sweeps,
                          int64_t ng, const int64_t* gidx, const real* gval) {
    lattice* L;
    int64_t nl = lattice_list(D, &L);
    int64_t upd = 0;
    int d = D->d;
    /* the lattices are independent (Step 1 of Sec. 3.2) */
#pragma omp parallel for schedule(dynamic) reduction(+ : upd)
    for (int64_t q = 0; q < nl; q++) {
        lattice* l = &L[q];
        int64_t cnt = l->B.cnt;
        real* u = (real*)malloc(sizeof(real) * (size_t)cnt);
        real* rd = (real*)malloc(sizeof(real) * (size_t)cnt);
        signed char* w = (signed char*)calloc((size_t)(d * cnt), 1);
        unsigned char* fixed = (unsigned char*)calloc((size_t)cnt, 1);
        int64_t nfree = 0;
        for (int64_t li = 0; li < cnt; li++) {
            int64_t X = lattice_global(D, l, li);
            int64_t c[3];
            node_coords(D, X, c);
            rd[li] = D->r[X] * D->HT;
            u[li] = RINF;
            /* Initialisation "on or near" the boundary: lattice nodes within
             * max-norm distance < H of a Gamma node start at the smallest
             * g + r*|X - x_g| (wind: direction from x_g to X); Gamma nodes
             * themselves are included at distance 0. */
            real best = RINF;
            int64_t bestg = -1;
            if (D->isg[X]) {
                /* a Gamma node keeps its own boundary value, wind 0 */
                fixed[li] = 1;
                u[li] = D->gv[X];
                continue;
            }
            for (int64_t g = 0; g < ng; g++) {
                int64_t cg[3];
                node_coords(D, gidx[g], cg);
                int near = 1;
                int64_t d2 = 0;
                for (int a = 0; a < d; a++) {
                    int64_t df = c[a] - cg[a];
                    if (df <= -D->M || df >= D->M) near = 0;
                    d2 += df * df;
                }
                if (!near) continue;
                real sq = RSQRT_((real)d2);
                real dist = D->hT * sq;
                real v = gval[g] + D->r[X] * dist;
                if (v < best) {
                    best = v;
                    bestg = g;
                }
            }
            if (bestg >= 0) {
                fixed[li] = 1;
                u[li] = best;
                int64_t cg[3];
                node_coords(D, gidx[bestg], cg);
                for (int a = 0; a < d; a++) {
                    int64_t df = c[a] - cg[a];
                    w[a * cnt + li] = (signed char)((df > 0) - (df < 0));
                }
            } else {
                nfree++;
            }
        }
        fsm_ctx C = {u, w, fixed, rd, D->crule};
        int64_t ns = 0;
        run_sweeps(&l->B, max_sweeps, fsm_node, &C, &ns);
        upd += nfree * ns;
        for (int64_t li = 0; li < cnt; li++) {
            int64_t X = lattice_global(D, l, li);
            U[X] = u[li];
            for (int a = 0; a < d; a++) W[a * D->N + X] = w[a * cnt + li];
        }
        free(u);
        free(rd);
        free(w);
        free(fixed);
    }
    free(L);
    return upd;
}

/* ---- causal sweep (Alg. causalsweep2D) ----
 * The 2^d directions once each, every coarse node in lexicographic fine-index
 * order.  At a non-Gamma coarse node X and for each axis e (x, y, z in turn):
 *   if W_e(X) < 0 (flow from the plus side) and U(X) < U(X+e): U(X) = U(X+e)
 *   if W_e(X) > 0 (flow from the minus side) and U(X) < U(X-e): U(X) = U(X-e)
 * where each comparison needs that fine neighbour to be a coarse node. */
static void causal_sweep(const ddp* D, real* U, const signed char* W) {
    box B;
    box_init(&B, D->d, D->n);
    int nd = 1 << D->d;
    for (int dir = 0; dir < nd; dir++) {
        int s0 = dir_sign(D->d, dir, 0), s1 = dir_sign(D->d, dir, 1);
        int s2 = (D->d == 3) ? dir_sign(D->d, dir, 2) : 1;
        for (int64_t q0 = 0; q0 < B.L[0]; q0++) {
            int64_t i = (s0 > 0) ? q0 : B.L[0] - 1 - q0;
            for (int64_t q1 = 0; q1 < B.L[1]; q1++) {
                int64_t j = (s1 > 0) ? q1 : B.L[1] - 1 - q1;
                for (int64_t q2 = 0; q2 < B.L[2]; q2++) {
                    int64_t k = (s2 > 0) ? q2 : B.L[2] - 1 - q2;
                    int64_t c[3] = {i, j, k};
                    if (!is_coarse(D, c)) continue;
                    int64_t X = node_index(D, c);
                    if (D->isg[X]) continue;
                    for (int e = 0; e < D->d; e++) {
                        int we = W[e * D->N + X];
                        if (we < 0 && c[e] + 1 < D->n[e]) {
                            int64_t cn[3] = {c[0], c[1], c[2]};
                            cn[e] += 1;
                            if (is_coarse(D, cn)) {
                                int64_t Y = X + D->st[e];
                                if (U[X] < U[Y]) U[X] = U[Y];
                            }
                        }
                        if (we > 0 && c[e] > 0) {
                            int64_t cn[3] = {c[0], c[1], c[2]};
                            cn[e] -= 1;
                            if (is_coarse(D, cn)) {
                                int64_t Y = X - D->st[e];
                                if (U[X] < U[Y]) U[X] = U[Y];
                            }
                        }
                    }
                }
            }
        }
    }
}

/* ---- Steps 2 and 3 on one subdomain ----
 * Step 2: nodes of the subdomain that are Gamma nodes are fixed at g (wind 0);
 * a boundary node of the subdomain lying on an interface (a subdomain
 * boundary that is not the domain boundary) is an inflow node if
 * W . n_in > 0 for an inward normal n_in of the subdomain there (a corner has
 * one normal per interface axis): it starts at U with its wind W and, like
 * every other non-Gamma node, takes the FSM minimum (the reading that the
 * boundary value is an upper bound, as u <= g in the exit-time form of the
 * value function, Sec. 1.1); every other node starts at +inf (boundary data
 * "infinity").  With D->inflow_fixed (a test-only flag) inflow nodes are held
 * at U instead, the literal reading of the subdomain problem's u = g.
 * Step 3: FSM on the subdomain grid with one-sided differences at its
 * boundary. */
static int64_t tile_solve(const ddp* D, const int64_t T[3], const real* U, const signed char* W,
                          real* tu, signed char* tw, int max_sweeps) {
    int d = D->d;
    int64_t ext[3] = {D->S + 1, D->S + 1, D->S + 1};
    box B;
    box_init(&B, d, ext);
    int64_t cnt = B.cnt;
    real* rd = (real*)malloc(sizeof(real) * (size_t)cnt);
    unsigned char* fixed = (unsigned char*)calloc((size_t)cnt, 1);
    int64_t nfree = 0;
    for (int64_t li = 0; li < cnt; li++) {
        int64_t lc[3], c[3];
        box_coords(&B, li, lc);
        for (int a = 0; a < 3; a++) c[a] = (a < d) ? T[a] * D->S + lc[a] : 0;
        int64_t X = node_index(D, c);
        rd[li] = D->r[X] * D->hT;
        tu[li] = RINF;
        for (int a = 0; a < d; a++) tw[a * cnt + li] = 0;
        if (D->isg[X]) {
            fixed[li] = 1;
            tu[li] = D->gv[X];
            continue;
        }
        int inflow = 0;
        for (int a = 0; a < d; a++) {
            if (!is_iface_axis(D, c, a)) continue;
            int we = W[a * D->N + X];
            if (lc[a] == 0 && we > 0) inflow = 1;          /* inward normal +e_a */
            if (lc[a] == D->S && we < 0) inflow = 1;       /* inward normal -e_a */
        }
        if (inflow) {
            tu[li] = U[X];
            for (int a = 0; a < d; a++) tw[a * cnt + li] = W[a * D->N + X];
            if (D->inflow_fixed) {
                /* the literal reading ("u = g on the boundary"): held at U */
                fixed[li] = 1;
                continue;
            }
        }
        nfree++;
    }
    fsm_ctx C = {tu, tw, fixed, rd, 0};
    int64_t ns = 0;
    run_sweeps(&B, max_sweeps, fsm_node, &C, &ns);
    free(rd);
    free(fixed);
    return nfree * ns;
}

/* ---- reconciliation at a node (Alg. fineupdate, one axis at a time) ----
 * Candidates: the subdomains containing X, ordered lexicographically with x
 * slowest and the minus side first.  Candidates at +inf are set aside unless
 * all are.  For each interface axis e: if every remaining candidate's fine
 * wind and the coarse wind W^k satisfy w . (-e) >= 0, the plus-side
 * subdomains are kept; otherwise if all satisfy w . e >= 0 the minus side is
 * kept; otherwise both.  u^k is the smallest kept value (first candidate on
 * ties), w^k its wind.  If no candidate survives the side filter, the
 * smallest finite one is taken. */
typedef struct {
    real u;
    signed char w[3];
    int side[3];  /* 0 = minus, 1 = plus (only for interface axes) */
} cand;

static void reconcile_node(int d, const cand* cs, int nc, const int* iface, const signed char* Wk,
                           real* uk, signed char* wk) {
    int fin[8], nf = 0;
    for (int x = 0; x < nc; x++)
        if (cs[x].u < RINF) fin[nf++] = x;
    if (nf == 0) {
        for (int x = 0; x < nc; x++) fin[nf++] = x;
    }
    int allow[3][2];
    for (int e = 0; e < 3; e++) allow[e][0] = allow[e][1] = 1;
    for (int e = 0; e < d; e++) {
        if (!iface[e]) continue;
        int le = (Wk[e] <= 0), ge = (Wk[e] >= 0);
        for (int y = 0; y < nf; y++) {
            int we = cs[fin[y]].w[e];
            le = le && (we <= 0);
            ge = ge && (we >= 0);
        }
        if (le) {
            allow[e][0] = 0;  /* keep plus side */
        } else if (ge) {
            allow[e][1] = 0;  /* keep minus side */
        }
    }
    int best = -1;
    for (int y = 0; y < nf; y++) {
        const cand* c = &cs[fin[y]];
        int ok = 1;
        for (int e = 0; e < d; e++)
            if (iface[e] && !allow[e][c->side[e]]) ok = 0;
        if (!ok) continue;
        if (best < 0 || c->u < cs[best].u) best = fin[y];
    }
    if (best < 0) {
        for (int y = 0; y < nf; y++)
            if (best < 0 || cs[fin[y]].u < cs[best].u) best = fin[y];
    }
    *uk = cs[best].u;
    for (int e = 0; e < d; e++) wk[e] = cs[best].w[e];
}

/* ---- the weight theta of the Step 4 correction ----
 *
 * exp_cw: e^x in double by Cody and Waite's range reduction (x = n ln2 + r,
 * |r| <= ln2/2, with ln2 split into a high part exact in 32 bits and a low
 * correction, the split used by fdlibm) and the Taylor series of e^r to
 * r^13 in Horner form.  The logistic damping below needs e^x only to a few
 * ulp; the point of writing it out is that every step is a fixed sequence
 * of IEEE double operations.  Arguments below -700 give 0 (then 1 + e^x
 * rounds to 1 anyway), arguments from 709.78 on give +inf. */
static double exp_cw(double x) {
    if (x != x) return x;
    if (x >= 709.78) return INFINITY;
    if (x < -700.0) return 0.0;
    const double inv_ln2 = 0x1.71547652b82fep0;
    const double ln2_hi = 0x1.62e42feep-1;
    const double ln2_lo = 0x1.a39ef35793c76p-33;
    double n = floor(x * inv_ln2 + 0.5);
    double r = (x - n * ln2_hi) - n * ln2_lo;
    double p = 1.0 / 6227020800.0;       /* 1/13! */
    p = p * r + 1.0 / 479001600.0;       /* 1/12! */
    p = p * r + 1.0 / 39916800.0;        /* 1/11! */
    p = p * r + 1.0 / 3628800.0;         /* 1/10! */
    p = p * r + 1.0 / 362880.0;          /* 1/9! */
    p = p * r + 1.0 / 40320.0;           /* 1/8! */
    p = p * r + 1.0 / 5040.0;            /* 1/7! */
    p = p * r + 1.0 / 720.0;             /* 1/6! */
    p = p * r + 1.0 / 120.0;             /* 1/5! */
    p = p * r + 1.0 / 24.0;              /* 1/4! */
    p = p * r + 1.0 / 6.0;               /* 1/3! */
    p = p * r + 0.5;                     /* 1/2! */
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)n);
}

/* the damped weight of eq. thetaest: [s(t) t + (1 - s(t)) delta t]^+ with
 * the logistic s(t) = 1 / (1 + e^{(t - x0)/gamma}) */
static double theta_damped(double tb, double gamma, double delta, double x0) {
    double e = exp_cw((tb - x0) / gamma);
    double sg = 1.0 / (1.0 + e);
    double th = sg * tb + (1.0 - sg) * (delta * tb);
    return th > 0.0 ? th : 0.0;
}

/* Weight at coarse node X given the current lattice candidate Ut (U~, the
 * coarse solver on the current neighbours, i.e. C_H(nbrs(U^{k+1}))) and
 * C^k = C_H(nbrs(U^k)).  All in double from the working-precision values.
 *  mode 0: the constant theta.
 *  mode 1: eq. secthetaest with the estimate's numerator u^k - u^{k-1} and
 *          the omega-weighted mean of the last three coarse increments
 *          C_H(U^{k+1-s}) - C_H(U^{k-s}), s = 0, 1, 2 (the s = 0 increment
 *          is U~ - C^k, the others come from earlier iterations), then
 *          eq. thetaest.  Evaluated as t = num / ((w0 d0 + (w1 d1 + w2 d2))
 *          / (w0 + w1 + w2)).  Until C^{k-2} exists, or when a term is not
 *          finite or the denominator is 0, the constant theta is used.
 *  mode 2: M-bar of Sec. 4.2 at this iteration, (u^f - u^k) / (U~ - C^k),
 *          minus a margin (the paper uses 0.001), clamped at 0; the
 *          constant theta where it is not defined.
 *  mode 3: a caller-supplied theta per node. */
static double theta_node(const ddp* D, int64_t X, real Ut, real Ck, real ukX, double theta) {
    const double* q = D->tpar;
    if (D->theta_mode == 1) {
        if (!D->ukm1 || !D->ckm1 || !D->ckm2) return theta;
        double num = (double)ukX - (double)D->ukm1[X];
        double d1 = (double)Ck - (double)D->ckm1[X];
        double d2 = (double)D->ckm1[X] - (double)D->ckm2[X];
        double hs = q[4] * d1 + q[5] * d2;
        if (!isfinite(num) || !isfinite(hs)) return theta;
        double d0 = (double)Ut - (double)Ck;
        double den = (q[3] * d0 + hs) / ((q[3] + q[4]) + q[5]);
        if (!isfinite(den) || den == 0.0) return theta;
        return theta_damped(num / den, q[0], q[1], q[2]);
    }
    if (D->theta_mode == 2) {
        double num = (double)D->tref[X] - (double)ukX;
        double den = (double)Ut - (double)Ck;
        if (!isfinite(num) || !isfinite(den) || den == 0.0) return theta;
        double th = num / den - q[6];
        return th > 0.0 ? th : 0.0;
    }
    if (D->theta_mode == 3) return (double)D->tref[X];
    return theta;
}

/* exported for the tests of the weight rule */
double NAME(eikref_exp_cw)(double x) { return exp_cw(x); }
double NAME(eikref_theta_damped)(double tb, double gamma, double delta, double x0) {
    return theta_damped(tb, gamma, delta, x0);
}

/* ---- Step 4 on one lattice (Alg. 2Dweightedupdate) ---- */
typedef struct {
    const ddp* D;
    const lattice* l;
    real* u;                /* current U on the lattice */
    const real* Uk;         /* U^k */
    const real* uk;         /* reconciled fine values u^k */
    const real* Ck;         /* C_H(nbrs^H(U^k)) */
    const signed char* wk;  /* [a*cnt+li] */
    const signed char* Wk;
    const real* rd;
    const unsigned char* fixed;
    const unsigned char* normal;  /* bit a set: axis a is a normal of the node's coarse line */
} corr_ctx;

static int corr_node(const box* B, int64_t li, void* vctx) {
    corr_ctx* C = (corr_ctx*)vctx;
    if (C->fixed[li]) return 0;
    int d = B->d;
    real m[3];
    signed char ws[3], wt[3];
    gather(B, C->u, li, m, ws);
    real Ut = local_solve(d, m, ws, C->rd[li], C->D->crule, wt);
    int cond = 1;
    for (int e = 0; e < d; e++) {
        if (!((C->normal[li] >> e) & 1)) continue;
        int a = C->wk[e * B->cnt + li], b = C->Wk[e * B->cnt + li], t = wt[e];
        int le = (a <= 0) && (b <= 0) && (t <= 0);
        int ge = (a >= 0) && (b >= 0) && (t >= 0);
        if (!(le || ge)) cond = 0;
    }
    real v;
    if (cond && isfinite((double)Ut) && isfinite((double)C->Ck[li])) {
        real th = C->D->thetaT;
        if (C->D->theta_mode != 0)
            th = (real)theta_node(C->D, lattice_global(C->D, C->l, li), Ut, C->Ck[li], C->uk[li],
                                  (double)C->D->thetaT);
        v = C->uk[li] + th * (Ut - C->Ck[li]);
    } else {
        v = C->uk[li];
    }
    if (v != C->u[li]) {
        C->u[li] = v;
        return 1;
    }
    return 0;
}

static int64_t step4_correct(const ddp* D, const real* Uk, const signed char* Wk, const real* ukg,
                             const signed char* wkg, real* Un, signed char* Wn, int max_sweeps,
                             real* Ck_out) {
    lattice* L;
    int64_t nl = lattice_list(D, &L);
    int d = D->d;
    int64_t upd = 0;
    /* the lattices are independent (Step 4 of Sec. 3.2) */
#pragma omp parallel for schedule(dynamic) reduction(+ : upd)
    for (int64_t q = 0; q < nl; q++) {
        lattice* l = &L[q];
        int64_t cnt = l->B.cnt;
        real* u = (real*)malloc(sizeof(real) * cnt);
        real* lUk = (real*)malloc(sizeof(real) * cnt);
        real* luk = (real*)malloc(sizeof(real) * cnt);
        real* lCk = (real*)malloc(sizeof(real) * cnt);
        real* rd = (real*)malloc(sizeof(real) * cnt);
        signed char* lwk = (signed char*)malloc((size_t)(d * cnt));
        signed char* lWk = (signed char*)malloc((size_t)(d * cnt));
        unsigned char* fixed = (unsigned char*)calloc((size_t)cnt, 1);
        unsigned char* normal = (unsigned char*)calloc((size_t)cnt, 1);
        int64_t nfree = 0;
        for (int64_t li = 0; li < cnt; li++) {
            int64_t X = lattice_global(D, l, li);
            int64_t c[3];
            node_coords(D, X, c);
            lUk[li] = Uk[X];
            luk[li] = ukg[X];
            rd[li] = D->r[X] * D->HT;
            for (int a = 0; a < d; a++) {
                lwk[a * cnt + li] = wkg[a * D->N + X];
                lWk[a * cnt + li] = Wk[a * D->N + X];
                if (c[a] % D->M == 0) normal[li] |= (unsigned char)(1 << a);
            }
            if (D->isg[X]) {
                fixed[li] = 1;
                u[li] = D->gv[X];
            } else {
                u[li] = RINF;
                nfree++;
            }
        }
        /* C^k = C_H(nbrs^H(U^k)) at every node, evaluated once (Jacobi) */
        for (int64_t li = 0; li < cnt; li++) {
            real m[3];
            signed char ws[3], wt[3];
            gather(&l->B, lUk, li, m, ws);
            lCk[li] = local_solve(d, m, ws, rd[li], D->crule, wt);
            if (Ck_out) Ck_out[lattice_global(D, l, li)] = lCk[li];
        }
        corr_ctx C = {D, l, u, lUk, luk, lCk, lwk, lWk, rd, fixed, normal};
        int64_t ns = 0;
        run_sweeps(&l->B, max_sweeps, corr_node, &C, &ns);
        upd += nfree * ns;
        for (int64_t li = 0; li < cnt; li++) {
            int64_t X = lattice_global(D, l, li);
            Un[X] = u[li];
            for (int a = 0; a < d; a++) Wn[a * D->N + X] = fixed[li] ? 0 : lwk[a * cnt + li];
        }
        free(u); free(lUk); free(luk); free(lCk); free(rd); free(lwk); free(lWk);
        free(fixed); free(normal);
    }
    free(L);
    return upd;
}

/* info: [0] iterations, [1] converged, [2] fine updates (Step 3 local solves),
 *       [3] coarse updates (Steps 1 and 4 local solves), [4] status
 * hist: max|U^{k+1}-U^k| per iteration (up to hist_cap entries) */
int NAME(eikref_dd)(int d, const int64_t* n, double h, const real* r, int64_t ng,
                    const int64_t* gidx, const real* gval, int S, int M, double theta,
                    double tol, int max_iter, int max_fine_sweeps, int max_coarse_sweeps,
                    const real* U_init, const signed char* W_init, real* u_out, real* U_out,
                    signed char* W_out, real* uk_out, signed char* wk_out, real* Upre_out,
                    int64_t* info, double* hist, int hist_cap, int theta_mode, const double* tpar,
                    const real* tref, int coarse_solver, int inflow_fixed) {
    int64_t N;
    int st = check_problem(d, n, h, r, ng, gidx, gval, &N);
    if (st != OK) return st;
    if (M < 2 || S < M || S % M != 0) return ERR_SHAPE;
    if (!(theta >= 0.0 && theta <= 1.0)) return ERR_ARG;
    if (max_iter < 0 || max_fine_sweeps < 1 || max_coarse_sweeps < 1) return ERR_ARG;
    if (theta_mode < 0 || theta_mode > 3) return ERR_ARG;
    if (theta_mode != 0 && !tpar) return ERR_ARG;
    if ((theta_mode == 2 || theta_mode == 3) && !tref) return ERR_ARG;
    if (coarse_solver != 0 && coarse_solver != 1) return ERR_ARG;
    ddp D;
    memset(&D, 0, sizeof(D));
    D.d = d;
    D.N = N;
    D.S = S;
    D.M = M;
    for (int a = 0; a < 3; a++) {
        D.n[a] = (a < d) ? n[a] : 1;
        if (a < d && (n[a] - 1) % S != 0) return ERR_SHAPE;
        D.P[a] = (a < d) ? (n[a] - 1) / S : 1;
    }
    D.st[0] = 1;
    D.st[1] = D.n[0];
    D.st[2] = D.n[0] * D.n[1];
    D.hT = (real)h;
    D.HT = (real)((double)M * h);
    D.thetaT = (real)theta;
    D.theta_mode = theta_mode;
    D.inflow_fixed = inflow_fixed;
    D.crule = coarse_solver ? 2 : 1;
    for (int q = 0; q < 7; q++) D.tpar[q] = tpar ? tpar[q] : 0.0;
    D.tref = tref;
    D.r = r;
    D.isg = (unsigned char*)calloc((size_t)N, 1);
    D.gv = (real*)calloc((size_t)N, sizeof(real));
    for (int64_t g = 0; g < ng; g++) {
        D.isg[gidx[g]] = 1;
        D.gv[gidx[g]] = gval[g];
    }

    real* U = (real*)malloc(sizeof(real) * N);
    real* Un = (real*)malloc(sizeof(real) * N);
    real* uk = (real*)malloc(sizeof(real) * N);
    signed char* W = (signed char*)calloc((size_t)(d * N), 1);
    signed char* Wn = (signed char*)calloc((size_t)(d * N), 1);
    signed char* wk = (signed char*)calloc((size_t)(d * N), 1);
    /* history for the estimated weight: u^{k-1}, C^k, C^{k-1}, C^{k-2} */
    real* hu = (real*)malloc(sizeof(real) * N);
    real* hc[3];
    for (int q = 0; q < 3; q++) hc[q] = (real*)malloc(sizeof(real) * N);
    int64_t ntile = D.P[0] * D.P[1] * D.P[2];
    int64_t V = 1;
    for (int a = 0; a < d; a++) V *= (S + 1);
    real* tu = (real*)malloc(sizeof(real) * (size_t)(ntile * V));
    signed char* tw = (signed char*)malloc((size_t)(ntile * V * d));
    for (int64_t x = 0; x < N; x++) {
        U[x] = (real)NAN;
        uk[x] = (real)NAN;
        u_out[x] = (real)NAN;
    }

    int64_t coarse_upd = 0, fine_upd = 0;
    if (U_init) {
        for (int64_t x = 0; x < N; x++) {
            int64_t c[3];
            node_coords(&D, x, c);
            if (is_coarse(&D, c)) U[x] = U_init[x];
        }
        if (W_init) memcpy(W, W_init, (size_t)(d * N));
    } else {
        coarse_upd += step1_init(&D, U, W, max_coarse_sweeps, ng, gidx, gval);
        causal_sweep(&D, U, W);
    }

    int it = 0, conv = 0;
    for (int k = 0; k < max_iter; k++) {
        /* Steps 2-3: every subdomain independently */
#pragma omp parallel for schedule(dynamic) reduction(+ : fine_upd)
        for (int64_t t = 0; t < ntile; t++) {
            int64_t T[3] = {t % D.P[0], (t / D.P[0]) % D.P[1], t / (D.P[0] * D.P[1])};
            fine_upd += tile_solve(&D, T, U, W, tu + t * V, tw + t * V * d, max_fine_sweeps);
        }
        /* reconciliation at coarse nodes and the patched fine solution */
        for (int64_t X = 0; X < N; X++) {
            int64_t c[3];
            node_coords(&D, X, c);
            int iface[3] = {0, 0, 0};
            int64_t tl[3][2];
            int ns[3];
            for (int a = 0; a < 3; a++) {
                if (a >= d) {
                    tl[a][0] = 0;
                    ns[a] = 1;
                    continue;
                }
                if (is_iface_axis(&D, c, a)) {
                    iface[a] = 1;
                    tl[a][0] = c[a] / S - 1;
                    tl[a][1] = c[a] / S;
                    ns[a] = 2;
                } else {
                    int64_t tt = c[a] / S;
                    if (tt >= D.P[a]) tt = D.P[a] - 1;
                    tl[a][0] = tt;
                    ns[a] = 1;
                }
            }
            cand cs[8];
            int nc = 0;
            for (int x0 = 0; x0 < ns[0]; x0++)
                for (int x1 = 0; x1 < ns[1]; x1++)
                    for (int x2 = 0; x2 < ns[2]; x2++) {
                        int sd[3] = {x0, x1, x2};
                        int64_t T[3], lc[3];
                        for (int a = 0; a < 3; a++) {
                            T[a] = tl[a][sd[a]];
                            lc[a] = (a < d) ? c[a] - T[a] * S : 0;
                        }
                        int64_t t = T[0] + D.P[0] * (T[1] + D.P[1] * T[2]);
                        int64_t li = lc[0] + (S + 1) * (lc[1] + (S + 1) * lc[2]);
                        cand* cc = &cs[nc++];
                        cc->u = tu[t * V + li];
                        for (int a = 0; a < 3; a++) {
                            cc->w[a] = (a < d) ? tw[t * V * d + a * V + li] : 0;
                            cc->side[a] = sd[a];
                        }
                    }
            real v;
            signed char wv[3] = {0, 0, 0};
            if (nc == 1) {
                v = cs[0].u;
                for (int a = 0; a < d; a++) wv[a] = cs[0].w[a];
            } else {
                signed char Wx[3] = {0, 0, 0};
                for (int a = 0; a < d; a++) Wx[a] = W[a * N + X];
                reconcile_node(d, cs, nc, iface, Wx, &v, wv);
            }
            u_out[X] = v;
            if (is_coarse(&D, c)) {
                uk[X] = v;
                for (int a = 0; a < d; a++) wk[a * N + X] = wv[a];
            }
        }
        /* Step 4: weighted correction on every lattice, then causal sweep */
        for (int64_t x = 0; x < N; x++) Un[x] = (real)NAN;
        /* C^k goes to hc[k % 3]; C^{k-1} and C^{k-2} are the other two */
        D.ckm1 = (k >= 1) ? hc[(k + 2) % 3] : NULL;
        D.ckm2 = (k >= 2) ? hc[(k + 1) % 3] : NULL;
        D.ukm1 = (k >= 1) ? hu : NULL;
        coarse_upd += step4_correct(&D, U, W, uk, wk, Un, Wn, max_coarse_sweeps, hc[k % 3]);
        memcpy(hu, uk, sizeof(real) * N);
        if (Upre_out) memcpy(Upre_out, Un, sizeof(real) * N);
        causal_sweep(&D, Un, Wn);
        /* max|U^{k+1} - U^k| over coarse nodes, |inf - inf| = 0 */
        double delta = 0.0;
        for (int64_t X = 0; X < N; X++) {
            int64_t c[3];
            node_coords(&D, X, c);
            if (!is_coarse(&D, c)) continue;
            double a = (double)Un[X], b = (double)U[X];
            double df;
            if (isinf(a) && isinf(b))
                df = 0.0;
            else
                df = fabs(a - b);
            if (df > delta || isnan(df)) delta = isnan(df) ? INFINITY : df;
        }
        if (hist && k < hist_cap) hist[k] = delta;
        real* tU = U;
        U = Un;
        Un = tU;
        signed char* tW = W;
        W = Wn;
        Wn = tW;
        it = k + 1;
        if (delta < tol || delta == 0.0) {
            conv = 1;
            break;
        }
    }

    if (U_out) {
        for (int64_t x = 0; x < N; x++) {
            int64_t c[3];
            node_coords(&D, x, c);
            U_out[x] = is_coarse(&D, c) ? U[x] : (real)NAN;
        }
    }
    if (W_out) memcpy(W_out, W, (size_t)(d * N));
    if (uk_out) memcpy(uk_out, uk, sizeof(real) * N);
    if (wk_out) memcpy(wk_out, wk, (size_t)(d * N));
    if (info) {
        info[0] = it;
        info[1] = conv;
        info[2] = fine_upd;
        info[3] = coarse_upd;
        info[4] = (max_iter == 0 || conv) ? OK : ERR_NOCONV;
    }
    free(D.isg); free(D.gv); free(U); free(Un); free(uk); free(W); free(Wn); free(wk);
    free(hu); free(hc[0]); free(hc[1]); free(hc[2]);
    free(tu); free(tw);
    return (max_iter == 0 || conv) ? OK : ERR_NOCONV;
}

/* Test hook: the causal sweep alone (Alg. causalsweep2D, 3D by the same
 * rule per axis) on a full-grid U (in place), winds W [a*N + X] and Gamma
 * flags isg; U is read only at coarse nodes (some index = 0 mod M). */
int NAME(eikref_causal)(int d, const int64_t* n, int M, real* U, const signed char* W,
                        const unsigned char* isg) {
    if ((d != 2 && d != 3) || M < 1) return ERR_ARG;
    ddp D;
    memset(&D, 0, sizeof(D));
    D.d = d;
    D.M = M;
    D.N = 1;
    for (int a = 0; a < 3; a++) {
        D.n[a] = (a < d) ? n[a] : 1;
        D.N *= D.n[a];
    }
    D.st[0] = 1;
    D.st[1] = D.n[0];
    D.st[2] = D.n[0] * D.n[1];
    D.isg = (unsigned char*)isg;
    causal_sweep(&D, U, W);
    return OK;
}

/* Test hook: the reconciliation at one node (Alg. fineupdate, per axis):
 * nc candidates with values cu[nc], winds cw[nc][3] and sides cside[nc][3]
 * (0 minus, 1 plus), interface axes iface[3], coarse wind Wk[3]. */
int NAME(eikref_reconcile)(int d, int nc, const real* cu, const signed char* cw, const int* cside,
                           const int* iface, const signed char* Wk, real* uk, signed char* wk) {
    if ((d != 2 && d != 3) || nc < 1 || nc > 8) return ERR_ARG;
    cand cs[8];
    for (int x = 0; x < nc; x++) {
        cs[x].u = cu[x];
        for (int a = 0; a < 3; a++) {
            cs[x].w[a] = cw[3 * x + a];
            cs[x].side[a] = cside[3 * x + a];
        }
    }
    reconcile_node(d, cs, nc, iface, Wk, uk, wk);
    return OK;
}

#ifdef _OPENMP
#include <omp.h>
/* OpenMP build only: threads for the subdomain and lattice loops. */
int NAME(eikref_set_threads)(int n) {
    omp_set_num_threads(n);
    return omp_get_max_threads();
}
#endif

/* Test hook: the local solve alone.  m, ws, wt have 3 entries (unused axes
 * ignored); returns u~ in *out. */
int NAME(eikref_local)(int d, const real* m, const signed char* ws, real rd, int rule,
                       signed char* wt, real* out) {
    if (d != 2 && d != 3) return ERR_ARG;
    real mm[3] = {RINF, RINF, RINF};
    signed char ww[3] = {0, 0, 0};
    for (int a = 0; a < d; a++) {
        mm[a] = m[a];
        ww[a] = ws[a];
    }
    *out = local_solve(d, mm, ww, rd, rule, wt);
    return OK;
}

/* ------------------------------------------------------------------ */
/* Travel-time gradient: the adjoint of the converged Godunov system   */
/* ------------------------------------------------------------------ */

/* Not a step of the paper's method: the gradient of a loss of converged
 * travel times with respect to the slowness, by the discrete adjoint of the
 * upwind scheme (eq. godonuv).  At a free node x whose update used the axes
 * A (the nonzero components of its fine wind, Alg. fineupdate2D), the local
 * equation is sum_{a in A} (u - u_a)^2 = (r h)^2, u_a the upwind neighbour
 * x - w_a e_a.  Differentiating:
 *     du = sum_a c_a du_a + q dr,   S = sum_{a in A} (u - u_a),
 *     c_a = (u - u_a) / S,   q = (r h) h / S
 * (one axis: c = 1, q = h up to rounding).  Gamma nodes and unreached nodes
 * carry no equation.  For a loss L with seed s = dL/du the adjoint field
 * solves lambda(y) = s(y) + sum over downwind nodes x that use y of
 * c(x -> y) lambda(x), and dL/dr(x) = lambda(x) q(x).  The system is
 * triangular in the order of decreasing u (an upwind neighbour has a
 * strictly smaller value), so it is solved by passes over the nodes in that
 * order until a pass changes nothing.
 *
 * Each node evaluates lambda(y) = s(y) + acc with acc summed in the fixed
 * order of the terms  pm_0 lambda(y - e_0), pp_0 lambda(y + e_0), pm_1 ...,
 * pp_1 ... (pm_a: coefficient of the node y - e_a towards y, pp_a: of
 * y + e_a; a term is exactly 0 where the coefficient is 0, i.e. where that
 * neighbour does not use y or does not exist), starting from acc = the
 * first term.
 *
 * Batch of nb problems on one grid and slowness (e.g. one per source): u,
 * seed, lambda are nb stacked N-arrays, gammas[b] the boundary set of
 * problem b; grad = sum over b in order of lambda_b q_b.  w (nb stacked
 * d*N arrays of axis components, as from eikref_fsm) may be NULL: the winds
 * are then recomputed from u with the fine rule.  info[0] = passes of the
 * slowest problem. */
typedef struct {
    real u;
    int64_t x;
} ukey;

static int cmp_desc(const void* A, const void* B) {
    const ukey* a = (const ukey*)A;
    const ukey* b = (const ukey*)B;
    if (a->u > b->u) return -1;
    if (a->u < b->u) return 1;
    return (a->x < b->x) ? -1 : (a->x > b->x);
}

int NAME(eikref_adjoint)(int d, const int64_t* n, double h, const real* r, int nb,
                         const int64_t* gcount, const int64_t* const* gidx, const real* u,
                         const signed char* w, const real* seed, real* lam, real* grad,
                         int64_t* info) {
    if (d != 2 && d != 3) return ERR_ARG;
    if (nb < 1) return ERR_ARG;
    box B;
    box_init(&B, d, n);
    const int64_t N = B.cnt;
    real hT = (real)h;
    real* c = (real*)malloc(sizeof(real) * (size_t)(d * N));   /* c_a(x) */
    signed char* wd = (signed char*)malloc((size_t)(d * N));  /* used winds */
    real* q = (real*)malloc(sizeof(real) * (size_t)N);
    unsigned char* fix = (unsigned char*)malloc((size_t)N);
    ukey* ord = (ukey*)malloc(sizeof(ukey) * (size_t)N);
    for (int64_t x = 0; x < N; x++) grad[x] = (real)0;
    int64_t maxpass = 0;
    for (int b = 0; b < nb; b++) {
        const real* ub = u + (int64_t)b * N;
        const real* sb = seed + (int64_t)b * N;
        real* lb = lam + (int64_t)b * N;
        memset(fix, 0, (size_t)N);
        for (int64_t g = 0; g < gcount[b]; g++) {
            int64_t X = gidx[b][g];
            if (X < 0 || X >= N) {
                free(c); free(wd); free(q); free(fix); free(ord);
                return ERR_ARG;
            }
            fix[X] = 1;
        }
        /* coefficients of every node's own equation */
        for (int64_t x = 0; x < N; x++) {
            q[x] = (real)0;
            for (int a = 0; a < d; a++) {
                c[a * N + x] = (real)0;
                wd[a * N + x] = 0;
            }
            if (fix[x] || !(ub[x] < RINF)) continue;
            signed char wt[3] = {0, 0, 0};
            if (w) {
                for (int a = 0; a < d; a++) wt[a] = w[(int64_t)b * d * N + a * N + x];
            } else {
                real m[3];
                signed char ws[3];
                gather(&B, ub, x, m, ws);
                local_solve(d, m, ws, r[x] * hT, 0, wt);
            }
            int64_t cx[3];
            box_coords(&B, x, cx);
            real S = (real)0;
            int first = 1;
            for (int a = 0; a < d; a++) {
                if (wt[a] == 0) continue;
                real ua = ub[x - wt[a] * B.st[a]];
                S = first ? (ub[x] - ua) : (S + (ub[x] - ua));
                first = 0;
            }
            if (first || !(S > (real)0)) continue;
            for (int a = 0; a < d; a++) {
                if (wt[a] == 0) continue;
                real ua = ub[x - wt[a] * B.st[a]];
                c[a * N + x] = (ub[x] - ua) / S;
                wd[a * N + x] = wt[a];
            }
            q[x] = ((r[x] * hT) * hT) / S;
        }
        /* passes in the order of decreasing u until nothing changes */
        for (int64_t x = 0; x < N; x++) {
            ord[x].u = ub[x];
            ord[x].x = x;
            lb[x] = (real)0;
        }
        qsort(ord, (size_t)N, sizeof(ukey), cmp_desc);
        int64_t pass = 0;
        for (;;) {
            int64_t changed = 0;
            for (int64_t k = 0; k < N; k++) {
                int64_t y = ord[k].x;
                int64_t cy[3];
                box_coords(&B, y, cy);
                real acc = (real)0;
                for (int a = 0; a < d; a++) {
                    /* a term is c * lambda where the neighbour uses y, else 0 */
                    real tm = (real)0, tp = (real)0;
                    if (cy[a] > 0) {
                        int64_t xm = y - B.st[a];
                        real pm = (wd[a * N + xm] == -1) ? c[a * N + xm] : (real)0;
                        if (pm != (real)0) tm = pm * lb[xm];
                    }
                    if (cy[a] < B.L[a] - 1) {
                        int64_t xp = y + B.st[a];
                        real pp = (wd[a * N + xp] == 1) ? c[a * N + xp] : (real)0;
                        if (pp != (real)0) tp = pp * lb[xp];
                    }
                    acc = (a == 0) ? tm : acc + tm;
                    acc = acc + tp;
                }
                real v = sb[y] + acc;
                if (v != lb[y]) {
                    lb[y] = v;
                    changed++;
                }
            }
            pass++;
            if (!changed) break;
        }
        if (pass > maxpass) maxpass = pass;
        for (int64_t x = 0; x < N; x++) grad[x] = grad[x] + lb[x] * q[x];
    }
    if (info) info[0] = maxpass;
    free(c); free(wd); free(q); free(fix); free(ord);
    return OK;
}
