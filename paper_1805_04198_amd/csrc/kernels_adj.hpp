// Device code of the travel-time gradient (2D): the adjoint of the
// converged upwind system (eq. godonuv) for a batch of problems that share
// the grid and the slowness (one per source).
//
// At a free node x with used axes A (the nonzero components of its fine
// wind) and upwind neighbours u_a = u(x - w_a e_a):
//     S = sum_{a in A} (u - u_a)   (axis order),
//     c_a = (u - u_a) / S,   q = (r h) h / S,
// and the adjoint field solves  lambda(y) = s(y) + sum of the terms
// pm_0 lambda(y - e_0), pp_0 lambda(y + e_0), pm_1 lambda(y - e_1),
// pp_1 lambda(y + e_1)  (in that order; pm_a is c_a of the node y - e_a if
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

// LDS bytes of k_adj_sweep for boxes of side B
__host__ __device__ inline size_t adj_box_bytes(int B, size_t szT) {
  return box_bytes(halo_count(B, B), 6, 0, szT);
}

}  // namespace eik
