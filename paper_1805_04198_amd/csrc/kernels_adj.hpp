// Device code of the travel-time gradient (2D and 3D): the adjoint of the
// converged upwind system (eq. godonuv) for a batch of problems that share
// the grid and the slowness (one per source).
//
// At a free node x with used axes A (the nonzero components of its fine
// wind) and upwind neighbours u_a = u(x - w_a e_a):
//     S = sum_{a in A} (u - u_a)   (axis order),
//     c_a = (u - u_a) / S,   q = (r h) h / S,
// and the adjoint field solves  lambda(y) = s(y) + sum of the terms
// pm_0 lambda(y - e_0), pp_0 lambda(y + e_0), pm_1 lambda(y - e_1),
// pp_1 lambda(y + e_1) (, pm_2, pp_2 in 3D)  (in that order; pm_a is c_a of the node y - e_a if
// that node uses y, pp_a the same for y + e_a; a term is exactly 0 where its
// coefficient is 0).  The gradient is dL/dr = sum over the batch (in order)
// of lambda_b q_b.  The system is triangular in decreasing u; it is solved
// by Gauss-Seidel sweeps of the whole grid (box wavefront, as the forward
// FSM) until a sweep changes nothing, which gives its unique solution with
// every node evaluated by the same expression.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels2d.hpp"
#include "kernels3d.hpp"

namespace eik {

template <typename T>
struct ADJ2 {
  int n0, n1;
  int nb;             // problems in the batch
  int B, BX, BY;      // sweep boxes
  T hT;
  const T* r;
  const T* u;         // [nb][N]
  const int8_t* w;    // [nb][N] wind codes, or NULL: recomputed from u
  const T* seed;      // [nb][N] dL/du
  uint8_t* fixed;     // [nb][N] Gamma flags
  T* c;               // [nb][2][N] c_a of each node's own equation
  uint8_t* wd;        // [nb][N] used wind codes
  T* q;               // [nb][N] du/dr
  T* pc;              // [nb][4][N] pm_0, pp_0, pm_1, pp_1
  T* lam;             // [nb][N]
  T* grad;            // [N]
  unsigned int* changed;
  int* eval_at;       // [nb][box] as in GS2 (box_needed)
  int* chg_at;
};

template <typename T>
__global__ void k_adj_mark(uint8_t* fixed, const int64_t* gidx, int64_t ng) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < ng) fixed[gidx[t]] = 1;
}

// the coefficients of node x's own equation (problem blockIdx.y)
template <typename T>
__global__ void k_adj_coef(ADJ2<T> A) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int64_t o = (int64_t)blockIdx.y * N;
  const T* u = A.u + o;
  const T inf = pinf<T>();
  T c0 = T(0), c1 = T(0), qv = T(0);
  uint8_t code = 0;
  const T ux = u[x];
  if (!A.fixed[o + x] && ux < inf) {
    const int i = (int)(x % A.n0), j = (int)(x / A.n0);
    int wx, wy;
    if (A.w) {
      const uint8_t cw = (uint8_t)A.w[o + x];
      wx = wx_of(cw);
      wy = wy_of(cw);
    } else {
      // fine wind rule (Alg. fineupdate2D) on the final values
      const T xm = i > 0 ? u[x - 1] : inf, xp = i < A.n0 - 1 ? u[x + 1] : inf;
      const T ym = j > 0 ? u[x - A.n0] : inf, yp = j < A.n1 - 1 ? u[x + A.n0] : inf;
      T a, b;
      int sa, sb;
      pick(xm, xp, a, sa);
      pick(ym, yp, b, sb);
      const T rd = A.r[x] * A.hT;
      const bool two = dabs(a - b) < rd;
      wx = (two || a < b) ? sa : 0;
      wy = (two || !(a < b)) ? sb : 0;
    }
    T S = T(0);
    bool first = true;
    T ua = T(0), ub = T(0);
    if (wx != 0) {
      ua = u[x - wx];
      S = ux - ua;
      first = false;
    }
    if (wy != 0) {
      ub = u[x - (int64_t)wy * A.n0];
      S = first ? (ux - ub) : (S + (ux - ub));
      first = false;
    }
    if (!first && S > T(0)) {
      if (wx != 0) c0 = (ux - ua) / S;
      if (wy != 0) c1 = (ux - ub) / S;
      qv = ((A.r[x] * A.hT) * A.hT) / S;
      code = wenc(wx, wy);
    }
  }
  A.c[(o * 2) + x] = c0;
  A.c[(o * 2) + N + x] = c1;
  A.q[o + x] = qv;
  A.wd[o + x] = code;
}

// pull coefficients of node y: the coefficients of its neighbours that use it
template <typename T>
__global__ void k_adj_pull(ADJ2<T> A) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t y = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (y >= N) return;
  const int64_t o = (int64_t)blockIdx.y * N;
  const int i = (int)(y % A.n0), j = (int)(y / A.n0);
  const uint8_t* wd = A.wd + o;
  const T* c0 = A.c + o * 2;
  const T* c1 = c0 + N;
  T* pc = A.pc + o * 4;
  pc[y] = (i > 0 && wx_of(wd[y - 1]) == -1) ? c0[y - 1] : T(0);
  pc[N + y] = (i < A.n0 - 1 && wx_of(wd[y + 1]) == 1) ? c0[y + 1] : T(0);
  pc[2 * N + y] = (j > 0 && wy_of(wd[y - A.n0]) == -1) ? c1[y - A.n0] : T(0);
  pc[3 * N + y] = (j < A.n1 - 1 && wy_of(wd[y + A.n0]) == 1) ? c1[y + A.n0] : T(0);
}

template <typename T>
struct PreAdj {
  T self, xn, yn, hx, hy, s, pxm, pxp, pym, pyp;
};

// lambda(y) = s(y) + terms (see above); direct assignment
template <typename T>
struct AdjRule {
  using real = T;
  using Pre = PreAdj<T>;
  static constexpr bool kHalo = true;
  T* u;  // lambda
  const T* s;
  const T* pxm;
  const T* pxp;
  const T* pym;
  const T* pyp;
  int SP;
  __device__ __forceinline__ T value(int x) const { return u[x]; }
  template <int SX, int SY>
  __device__ __forceinline__ Pre load(int x) const {
    Pre p;
    p.self = u[x];
    p.xn = u[x + SX];
    p.yn = u[x + SY * SP];
    p.hx = u[x - SX];
    p.hy = u[x - SY * SP];
    p.s = s[x];
    p.pxm = pxm[x];
    p.pxp = pxp[x];
    p.pym = pym[x];
    p.pyp = pyp[x];
    return p;
  }
  template <int SX, int SY>
  __device__ __forceinline__ T compute(T xm, T xp, T ym, T yp, const Pre& p, int x, bool act, bool& ch) const {
    const T tm0 = p.pxm != T(0) ? p.pxm * xm : T(0);
    const T tp0 = p.pxp != T(0) ? p.pxp * xp : T(0);
    const T tm1 = p.pym != T(0) ? p.pym * ym : T(0);
    const T tp1 = p.pyp != T(0) ? p.pyp * yp : T(0);
    T acc = tm0;
    acc = acc + tp0;
    acc = acc + tm1;
    acc = acc + tp1;
    const T v = p.s + acc;
    ch = act && (v != p.self);
    u[ch ? x : dummy_slot()] = v;
    return act ? v : p.self;
  }
};

// One directional sweep of the boxes on box-diagonal diag (sweep order),
// problem blockIdx.y.  Halo values come from global memory (upwind boxes
// finished, downwind boxes untouched); outside the grid they are 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_sweep(ADJ2<T> A, GridLaunch2 L) {
  extern __shared__ __align__(16) unsigned char smem[];
  // one or two sweeps per launch, as k_grid_sweep
  const int g = (L.n > 1 && (int)blockIdx.x >= L.start[1]) ? 1 : 0;
  const int dir = L.dir[g], diag = L.diag[g], t = L.t[g];
  A.changed += L.chg_off[g];
  const int sx = (dir & 2) ? 1 : -1, sy = (dir & 1) ? 1 : -1;
  const int q0 = max(0, diag - (A.BY - 1));
  const int Iq = q0 + (int)blockIdx.x - L.start[g];
  const int Jq = diag - Iq;
  if (Iq >= A.BX || Jq < 0) return;
  const int I = sx > 0 ? Iq : A.BX - 1 - Iq;
  const int J = sy > 0 ? Jq : A.BY - 1 - Jq;
  // lambda(y) is a function of its neighbours only, so the stationary-box
  // test of the forward sweeps applies unchanged
  int* eval_at = A.eval_at + blockIdx.y * A.BX * A.BY;
  int* chg_at = A.chg_at + blockIdx.y * A.BX * A.BY;
  if (!box_needed(eval_at, chg_at, I, J, A.BX, A.BY)) return;
  const int bi = I * A.B, bj = J * A.B;
  const int L0 = min(A.B, A.n0 - bi), L1 = min(A.B, A.n1 - bj);
  const int SP = halo_stride(L0);
  const int cnt = halo_count(L0, L1);
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t o = (int64_t)blockIdx.y * N;
  T* lamg = A.lam + o;
  const T* pcg = A.pc + o * 4;
  unsigned char* lc = smem;
  T* lam = carve<T>(lc, cnt);
  T* sd = carve<T>(lc, cnt);
  T* pxm = carve<T>(lc, cnt);
  T* pxp = carve<T>(lc, cnt);
  T* pym = carve<T>(lc, cnt);
  T* pyp = carve<T>(lc, cnt);
  for (int k = threadIdx.x; k < cnt; k += kBlock) {
    const int hi = k % SP - 1, hj = k / SP - 1;
    const int xi = bi + hi, yi = bj + hj;
    const bool inside = hi >= 0 && hi < L0 && hj >= 0 && hj < L1;
    T v = T(0), sv = T(0), a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    if (inside) {
      const int64_t X = xi + (int64_t)A.n0 * yi;
      v = lamg[X];
      sv = A.seed[o + X];
      a0 = pcg[X];
      a1 = pcg[N + X];
      a2 = pcg[2 * N + X];
      a3 = pcg[3 * N + X];
    } else if (hi >= -1 && hi <= L0 && hj >= -1 && hj <= L1 && xi >= 0 && xi < A.n0 && yi >= 0 &&
               yi < A.n1) {
      v = lamg[xi + (int64_t)A.n0 * yi];
    }
    lam[k] = v;
    sd[k] = sv;
    pxm[k] = a0;
    pxp[k] = a1;
    pym[k] = a2;
    pyp[k] = a3;
  }
  __syncthreads();
  __shared__ int sh_ch;
  if (threadIdx.x == 0) sh_ch = 0;
  __syncthreads();
  if (threadIdx.x < kWave) {
    AdjRule<T> R{lam, sd, pxm, pxp, pym, pyp, SP};
    const bool ch = sweep_any(R, L0, L1, SP, dir);
    if (__any(ch) && threadIdx.x == 0) sh_ch = 1;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int li = k % L0, lj = k / L0;
    lamg[(bi + li) + (int64_t)A.n0 * (bj + lj)] = lam[(lj + 1) * SP + (li + 1)];
  }
  if (threadIdx.x == 0) {
    eval_at[I + A.BX * J] = t;
    if (sh_ch) {
      chg_at[I + A.BX * J] = t;
      atomicOr(A.changed, 1u);
    }
  }
}

// dL/dr = sum over the batch, in order, of lambda_b q_b
template <typename T>
__global__ void k_adj_grad(ADJ2<T> A) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= N) return;
  T acc = T(0);
  for (int b = 0; b < A.nb; ++b) acc = acc + A.lam[(int64_t)b * N + x] * A.q[(int64_t)b * N + x];
  A.grad[x] = acc;
}

// ---------------------------------------------------------------------------
// 3D: the same equations with three axes; the whole grid is swept in boxes
// of side B held in LDS (as eik_solve in 3D), eight orders.
// ---------------------------------------------------------------------------

template <typename T>
struct ADJ3 {
  int n[3];
  int nb;             // problems in the batch
  int B;              // sweep box side
  int nbx[3];         // boxes per axis
  T hT;
  const T* r;
  const T* u;         // [nb][N]
  const int8_t* w;    // [nb][N] wind codes (2 bits per axis), or NULL: recomputed from u
  const T* seed;      // [nb][N] dL/du
  uint8_t* fixed;     // [nb][N] Gamma flags
  T* c;               // [nb][3][N] c_a of each node's own equation
  uint8_t* wd;        // [nb][N] used wind codes
  T* q;               // [nb][N] du/dr
  T* pc;              // [nb][6][N] pm_0, pp_0, pm_1, pp_1, pm_2, pp_2
  T* lam;             // [nb][N]
  T* grad;            // [N]
  unsigned int* changed;
  int* eval_at;       // [nb][box] as in GS3 (box_needed3)
  int* chg_at;
};

// the coefficients of node x's own equation (problem blockIdx.y)
template <typename T>
__global__ void k_adj_coef3(ADJ3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int64_t o = (int64_t)blockIdx.y * N;
  const T* u = A.u + o;
  const T inf = pinf<T>();
  T ca[3] = {T(0), T(0), T(0)};
  T qv = T(0);
  uint8_t code = 0;
  const T ux = u[x];
  const int64_t st[3] = {1, A.n[0], (int64_t)A.n[0] * A.n[1]};
  if (!A.fixed[o + x] && ux < inf) {
    const int c[3] = {(int)(x % A.n[0]), (int)((x / A.n[0]) % A.n[1]), (int)(x / st[2])};
    int wt[3];
    if (A.w) {
      const uint8_t cw = (uint8_t)A.w[o + x];
      for (int a = 0; a < 3; ++a) wt[a] = w_of(cw, a);
    } else {
      // fine wind rule (the used axes of the local solve) on the final values
      T m[3];
      int ws[3];
      for (int a = 0; a < 3; ++a) {
        const T lo = c[a] > 0 ? u[x - st[a]] : inf;
        const T hi = c[a] < A.n[a] - 1 ? u[x + st[a]] : inf;
        const bool lt = lo < hi;
        m[a] = lt ? lo : hi;
        ws[a] = lt ? 1 : -1;
      }
      uint8_t cw;
      (void)godunov3<T, false>(m, ws, A.r[x] * A.hT, cw);
      for (int a = 0; a < 3; ++a) wt[a] = w_of(cw, a);
    }
    // S in axis order, starting from the first used axis
    T S = T(0), ua[3] = {T(0), T(0), T(0)};
    bool first = true;
    for (int a = 0; a < 3; ++a) {
      if (wt[a] == 0) continue;
      ua[a] = u[x - wt[a] * st[a]];
      S = first ? (ux - ua[a]) : (S + (ux - ua[a]));
      first = false;
    }
    if (!first && S > T(0)) {
      for (int a = 0; a < 3; ++a)
        if (wt[a] != 0) ca[a] = (ux - ua[a]) / S;
      qv = ((A.r[x] * A.hT) * A.hT) / S;
      code = wenc3(wt[0], wt[1], wt[2]);
    }
  }
  for (int a = 0; a < 3; ++a) A.c[o * 3 + a * N + x] = ca[a];
  A.q[o + x] = qv;
  A.wd[o + x] = code;
}

// pull coefficients of node y: the coefficients of its neighbours that use it
template <typename T>
__global__ void k_adj_pull3(ADJ3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t y = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (y >= N) return;
  const int64_t o = (int64_t)blockIdx.y * N;
  const int64_t st[3] = {1, A.n[0], (int64_t)A.n[0] * A.n[1]};
  const int c[3] = {(int)(y % A.n[0]), (int)((y / A.n[0]) % A.n[1]), (int)(y / st[2])};
  const uint8_t* wd = A.wd + o;
  const T* ca = A.c + o * 3;
  T* pc = A.pc + o * 6;
  for (int a = 0; a < 3; ++a) {
    const T* cc = ca + a * N;
    // y - e_a uses y when its wind along a is -1; y + e_a when it is +1
    pc[(2 * a) * N + y] = (c[a] > 0 && w_of(wd[y - st[a]], a) == -1) ? cc[y - st[a]] : T(0);
    pc[(2 * a + 1) * N + y] = (c[a] < A.n[a] - 1 && w_of(wd[y + st[a]], a) == 1) ? cc[y + st[a]] : T(0);
  }
}

// One directional sweep of the boxes of a whole-grid launch (grid_box3),
// problem blockIdx.y: lambda(y) = s(y) + the six terms in order, direct
// assignment.  Neighbours outside the box come from global memory (upwind
// boxes finished, downwind boxes untouched); a term whose coefficient is 0
// reads nothing (outside the grid every coefficient is 0).
template <typename T>
__global__ __launch_bounds__(kBlock3) void k_adj_sweep3(ADJ3<T> A, GridLaunch3 GL) {
  extern __shared__ __align__(16) unsigned char smem[];
  int g, Tb[3];
  if (!grid_box3(GL, A.nbx, (int)blockIdx.x, g, Tb)) return;
  const int dir = GL.dir[g], t = GL.t[g];
  unsigned int* changed = A.changed + GL.chg_off[g];
  const int nbox = A.nbx[0] * A.nbx[1] * A.nbx[2];
  // lambda(y) is a function of its neighbours only, so the stationary-box
  // test of the forward sweeps applies unchanged
  int* eval_at = A.eval_at + (int64_t)blockIdx.y * nbox;
  int* chg_at = A.chg_at + (int64_t)blockIdx.y * nbox;
  if (!box_needed3(eval_at, chg_at, Tb, A.nbx)) return;
  int o3[3], L[3];
  for (int a = 0; a < 3; ++a) {
    o3[a] = Tb[a] * A.B;
    L[a] = min(A.B, A.n[a] - o3[a]);
  }
  const int cnt = L[0] * L[1] * L[2];
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t o = (int64_t)blockIdx.y * N;
  T* lamg = A.lam + o;
  T* lam = (T*)smem;
  const int64_t base = idx3(A.n, o3[0], o3[1], o3[2]);
  const int64_t gs1 = A.n[0], gs2 = (int64_t)A.n[0] * A.n[1];
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    lam[x] = lamg[base + p0 + p1 * gs1 + p2 * gs2];
  }
  __syncthreads();
  struct Rule {
    T* u;  // lambda of the box
    int L0, L1, L2;
    const T* lamg;
    const T* s;
    const T* pc;
    int64_t N, base, gs1, gs2;
    struct In {
      T s, p[6];  // seed; pm_0, pp_0, pm_1, pp_1, pm_2, pp_2
    };
    __device__ In load(int i, int j, int k) const {
      const int64_t X = base + i + j * gs1 + k * gs2;
      In in;
      in.s = s[X];
#pragma unroll
      for (int e = 0; e < 6; ++e) in.p[e] = pc[e * N + X];
      return in;
    }
    __device__ bool update(int i, int j, int k, const In& in) const {
      const int64_t X = base + i + j * gs1 + k * gs2;
      const int x = i + L0 * (j + L1 * k);
      const int c[3] = {i, j, k};
      const int L[3] = {L0, L1, L2};
      const int st[3] = {1, L0, L0 * L1};
      const int64_t gst[3] = {1, gs1, gs2};
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T pm = in.p[2 * a], pp = in.p[2 * a + 1];
        T tm = T(0), tp = T(0);
        if (pm != T(0)) tm = pm * (c[a] > 0 ? u[x - st[a]] : lamg[X - gst[a]]);
        if (pp != T(0)) tp = pp * (c[a] < L[a] - 1 ? u[x + st[a]] : lamg[X + gst[a]]);
        acc = a == 0 ? tm : acc + tm;
        acc = acc + tp;
      }
      const T v = in.s + acc;
      if (v != u[x]) {
        u[x] = v;
        return true;
      }
      return false;
    }
  } R{lam, L[0], L[1], L[2], lamg, A.seed + o, A.pc + o * 6, N, base, gs1, gs2};
  Range3 P{0, L[0] + L[1] + L[2] - 3};
  const bool ch = sweep3(R, L[0], L[1], L[2], dir, dir, P);
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    lamg[base + p0 + p1 * gs1 + p2 * gs2] = lam[x];
  }
  if (threadIdx.x == 0) {
    const int bidx = Tb[0] + A.nbx[0] * (Tb[1] + A.nbx[1] * Tb[2]);
    eval_at[bidx] = t;
    if (ch) {
      chg_at[bidx] = t;
      atomicOr(changed, 1u);
    }
  }
}

// dL/dr = sum over the batch, in order, of lambda_b q_b
template <typename T>
__global__ void k_adj_grad3(ADJ3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= N) return;
  T acc = T(0);
  for (int b = 0; b < A.nb; ++b) acc = acc + A.lam[(int64_t)b * N + x] * A.q[(int64_t)b * N + x];
  A.grad[x] = acc;
}

// LDS bytes of k_adj_sweep for boxes of side B
__host__ __device__ inline size_t adj_box_bytes(int B, size_t szT) {
  return box_bytes(halo_count(B, B), 6, 0, szT);
}

}  // namespace eik
