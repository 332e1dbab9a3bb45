// Device code of the 3D domain-decomposition Eikonal solver for gfx950.
//
// The paper writes the method in 2D and states that it generalises (Sec. 3,
// Sec. 1.1: 2^d sweeps); this file carries every step to d = 3 with the same
// per-axis rules as the CPU reference:
//   local solve  : the minima of the three axes sorted ascending (stable in
//                  axis order); one-sided u = a1 + rd, then the two-sided root
//                  if a2 is below it, then the three-sided root if a3 is below
//                  the two-sided one (t3 = 3 rd^2 - sum of squared pairwise
//                  differences, clamped at 0; u = ((a1+a2)+a3 + sqrt t3) / 3)
//   fine wind    : the axes used by the final root (Alg. fineupdate2D)
//   coarse wind  : an axis enters unless U~ lies below its neighbour minimum
//                  (the tests of Alg. update2D taken per axis)
// Layout: node (i, j, k) at i + n0*(j + n1*k).
//
// A box (subdomain or lattice, <= 34 nodes per axis in fp32) is swept by one
// workgroup with its values in LDS: thread p owns x-pencils (j, k); at step t
// of a sweep pencil (j, k) (in sweep order) updates node i = t - j - k, so the
// nodes of hyperplane t are updated between two barriers.  A node reads only
// hyperplanes t-1 (updated) and t+1 (not yet updated), so the result is the
// paper's lexicographic Gauss-Seidel sweep value for value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels2d.hpp"

namespace eik {

constexpr int kBlock3 = 1024;
// nodes per axis of a 3D box held in LDS (fp32); sweep3 relies on kMaxL3^2 <=
// 2 * kBlock3 (at most two pencils per thread)
constexpr int kMaxL3 = 34;
static_assert(kMaxL3 * kMaxL3 <= 2 * kBlock3, "sweep3 gives each thread at most two pencils");


__device__ __forceinline__ int w_of(uint8_t c, int a) { int v = (c >> (2 * a)) & 3; return v == 3 ? -1 : v; }
__device__ __forceinline__ uint8_t wenc3(int wx, int wy, int wz) {
  return (uint8_t)((wx & 3) | ((wy & 3) << 2) | ((wz & 3) << 4));
}

// x / 3 rounded to nearest.  fp32: the product with RN(1/3) corrected once
// by its exact remainder (Markstein's correction step: r = x - 3 q0 by one
// fused multiply-add, then q0 + r RN(1/3) by another); checked against the
// IEEE quotient for every finite float, where it differs only at x = -0
// (it gives +0), which is passed through.  fp64: the IEEE quotient.
__device__ __forceinline__ float div3(float x) {
  const float third = 0x1.555556p-2f;  // RN(1/3)
  const float q0 = x * third;
  const float r = __builtin_fmaf(-q0, 3.0f, x);
  const float q = __builtin_fmaf(r, third, q0);
  return x == 0.0f ? x : q;
}
__device__ __forceinline__ double div3(double x) { return x / 3.0; }

// 3D local solve.  m: per-axis neighbour minima; ws: their wind signs.
// Coarse = false: fine wind, true: coarse wind.  homog (coarse only): the
// homogenised solver of the squares medium (Sec. 5.3), the smallest
// neighbour plus r*H, in place of C_H.  Returns u~ and the wind code.
template <typename T, bool Coarse>
__device__ __forceinline__ T godunov3(const T (&m)[3], const int (&ws)[3], T rd, uint8_t& code,
                                      bool homog = false) {
  // a1 <= a2 <= a3: the neighbour minima in increasing order (min, median,
  // max; exact)
  const bool l01 = m[0] < m[1];
  const T lo01 = l01 ? m[0] : m[1], hi01 = l01 ? m[1] : m[0];
  const T a1 = lo01 < m[2] ? lo01 : m[2];
  const T a3 = hi01 < m[2] ? m[2] : hi01;
  const T a2 = hi01 < m[2] ? hi01 : (lo01 < m[2] ? m[2] : lo01);
  // the one-, two- and three-term candidates are all evaluated and the
  // cascade's choice selected (no branches; a lane whose choice does not
  // need a square root takes the root of 1 there)
  const T d12 = a1 - a2;
  const bool one = (Coarse && homog) || !(dabs(d12) < rd);
  T t = rd * rd;
  t = t + t;
  t = t - d12 * d12;
  const T u2 = ((a1 + a2) + dsqrt(one ? T(1) : t)) * T(0.5);
  const bool two = !one && !(a3 < u2);
  const T d13 = a1 - a3, d23 = a2 - a3;
  T q = rd * rd;
  q = (q + q) + q;
  q = q - ((d12 * d12 + d13 * d13) + d23 * d23);
  if (q < T(0)) q = T(0);
  const T u3 = div3(((a1 + a2) + a3) + dsqrt((one || two) ? T(1) : q));
  const T ut = one ? a1 + rd : (two ? u2 : u3);
  const int used = one ? 1 : (two ? 2 : 3);
  int w0, w1, w2;
  if (!Coarse) {
    // the axes of the used terms: those whose rank in the stable ascending
    // order of the minima (ties: lower axis first) is below `used`
    const int r0 = (m[1] < m[0] ? 1 : 0) + (m[2] < m[0] ? 1 : 0);
    const int r1 = (m[0] <= m[1] ? 1 : 0) + (m[2] < m[1] ? 1 : 0);
    const int r2 = (m[0] <= m[2] ? 1 : 0) + (m[1] <= m[2] ? 1 : 0);
    w0 = r0 < used ? ws[0] : 0;
    w1 = r1 < used ? ws[1] : 0;
    w2 = r2 < used ? ws[2] : 0;
  } else {
    w0 = (ut < m[0]) ? 0 : ws[0];
    w1 = (ut < m[1]) ? 0 : ws[1];
    w2 = (ut < m[2]) ? 0 : ws[2];
  }
  code = wenc3(w0, w1, w2);
  return ut;
}

// ---------------------------------------------------------------------------
// arguments
// ---------------------------------------------------------------------------

template <typename T>
struct DD3 {
  int n[3];          // nodes per axis
  int S, M;          // subdomain side, coarse spacing (fine cells)
  int P[3];          // subdomains per axis
  int NC[3];         // coarse cells per axis ((n-1)/M)
  int nlat;          // lattices: offsets in [0,M)^3 with a zero component
  T hT, HT, theta;
  int max_fine_sweeps, max_coarse_sweeps;
  const T* r;
  const T* gfull;     // Gamma value per node, NaN if not Gamma
  const int64_t* gidx;
  const T* gval;
  int64_t ng;
  T* rdh;             // r*h, NaN at Gamma nodes
  T* rdH;             // r*H, NaN at Gamma nodes
  T* U;
  uint8_t* W;
  T* Un;
  uint8_t* Wn;
  T* uk;
  uint8_t* wk;
  T* ck;              // C^k (full grid, coarse nodes used)
  uint16_t* mk;       // Step 4 condition masks
  T* u_out;
  T* face_u;          // [tile][6][(S+1)^2]
  uint8_t* face_w;
  uint8_t* tile_w;    // [tile][(S+1)^3] winds of the subdomain sweep
  const int* tile_order;  // block b sweeps subdomain tile_order[b] (NULL: b)
  int* tile_time;         // [tile] duration of the subdomain's last block, 10 ns units (NULL: not kept)
  T* cvals;           // causal sweep scratch: V per coarse node (full grid)
  unsigned long long* near_key;
  long long* near_win;
  unsigned long long* counters;  // [0] fine updates, [1] coarse updates, [2] residual bits
  // Step 4 weight (theta_at): parameters, u_ref or theta per node, and the
  // history u^{k-1}, C^{k-1}, C^{k-2} (NULL until it exists)
  ThetaPar tq;
  const T* tref;
  const T* ukm1;
  const T* ckm1;
  const T* ckm2;
  // coarse solver of Steps 1 and 4: 0 = C_H, 1 = the homogenised solver
  int coarse_homog;
  // Step 4 (constant weight), or NULL: each lattice's read-only operands in
  // lattice-major records (lattice q at rec + q rec_stride), gathered once
  // per launch so that every sweep reads them contiguously
  void* rec;
  int rec_stride;
};

// Step 4's read-only operands of a lattice node in one record
template <typename T>
struct alignas(4 * sizeof(T)) Corr3Rec {
  T rd;    // r*H, NaN at Gamma nodes
  T ukx;   // u^k
  T ckx;   // C^k
  unsigned mask;
};

__device__ __forceinline__ int64_t idx3(const int (&n)[3], int i, int j, int k) {
  return (int64_t)i + (int64_t)n[0] * ((int64_t)j + (int64_t)n[1] * k);
}

__device__ __forceinline__ bool coarse3(int i, int j, int k, int M) {
  return (i % M == 0) || (j % M == 0) || (k % M == 0);
}

// lattice q -> offset: first all with o0 = 0 (M^2), then o0 > 0 and o1 = 0
// (M(M-1)), then o0 > 0, o1 > 0, o2 = 0 ((M-1)^2)
__device__ __forceinline__ void lattice_offset3(int q, int M, int& o0, int& o1, int& o2) {
  if (q < M * M) { o0 = 0; o1 = q % M; o2 = q / M; return; }
  q -= M * M;
  if (q < (M - 1) * M) { o0 = 1 + q % (M - 1); o1 = 0; o2 = q / (M - 1); return; }
  q -= (M - 1) * M;
  o0 = 1 + q % (M - 1);
  o1 = 1 + q / (M - 1);
  o2 = 0;
}

// ---------------------------------------------------------------------------
// the 3D box sweep engine
// ---------------------------------------------------------------------------

// The hyperplanes [t0, tmax] of a sweep that hold every node that may
// change in it without an upwind change inside it (t0 > tmax: none).
struct Range3 {
  int t0, tmax;
};

// One directional sweep over an L0 x L1 x L2 box in LDS (index i + L0*(j +
// L1*k)); returns true (block-wide) if any value changed.  A thread owns at
// most two pencils (L1*L2 <= 2*blockDim); the read-only inputs of the node a
// pencil reaches at step t+1 (Rule::load) are fetched before the update of
// step t, so their global-memory latency overlaps a step.
//
// Restricted to what can change: P holds the hyperplanes with every node
// that may change in this sweep without an upwind change inside it (a node
// whose neighbours kept their values since its last evaluation computes the
// same value again).  The sweep starts at P.t0 and, from P.tmax on, stops
// after the first hyperplane without a change (a node past P changes only if
// an upwind neighbour, one hyperplane earlier, changed).  On return P holds
// the same for the next sweep, in direction ndir: the hyperplanes of that
// sweep within one of a node this sweep changed (the nodes next to a change
// lie there); empty if nothing changed.
template <typename Rule>
__device__ bool sweep3(Rule& R, int L0, int L1, int L2, int dir, int ndir, Range3& P) {
  using In = typename Rule::In;
  __shared__ int sh_rng[2];
  const int sx = (dir & 4) ? 1 : -1, sy = (dir & 2) ? 1 : -1, sz = (dir & 1) ? 1 : -1;
  const int nsteps = L0 + L1 + L2 - 2;
  const int t0 = P.t0, tmax = P.tmax;
  // hyperplane of box node (i, j, k) in the next sweep
  const int nsx = (ndir & 4) ? 1 : -1, nsy = (ndir & 2) ? 1 : -1, nsz = (ndir & 1) ? 1 : -1;
  auto next_plane = [&](int i, int j, int k) {
    return (nsx > 0 ? i : L0 - 1 - i) + (nsy > 0 ? j : L1 - 1 - j) + (nsz > 0 ? k : L2 - 1 - k);
  };
  if (threadIdx.x == 0) {
    sh_rng[0] = 0x7fffffff;
    sh_rng[1] = -1;
  }
  __syncthreads();
  const int np = L1 * L2;
  // Pencils (j, k) in sweep coordinates are numbered by anti-diagonal
  // s = j + k (then by j): the pencils that hold a node of hyperplane t are
  // those with t - L0 < s <= t, a contiguous run of threads, so the waves
  // outside it skip the step as a whole.
  int jq[2], kq[2], jj[2], kk[2];
  bool has[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int p = threadIdx.x + q * blockDim.x;
    has[q] = p < np;
    int d = 0, sd = 0, len = 1;
    for (;;) {  // the anti-diagonal sd that holds pencil number p
      len = min(sd, L1 - 1) - max(0, sd - (L2 - 1)) + 1;
      if (!has[q] || p < d + len) break;
      d += len;
      ++sd;
    }
    jq[q] = has[q] ? max(0, sd - (L2 - 1)) + (p - d) : 0;
    kq[q] = has[q] ? sd - jq[q] : 0;
    jj[q] = sy > 0 ? jq[q] : L1 - 1 - jq[q];
    kk[q] = sz > 0 ? kq[q] : L2 - 1 - kq[q];
  }
  // The read-only operands (global memory) of hyperplane t + kAhead are
  // requested while hyperplane t is updated: a ring of kAhead register sets,
  // the loop unrolled kAhead times so that every slot is a fixed register
  // (two sets where the operands are large, to stay clear of spills).
  constexpr int kAhead = sizeof(In) <= 32 ? 3 : 2;
  In buf[2][kAhead];
  auto fetch = [&](int t, int q, In& dst) {
    const int iq = t - jq[q] - kq[q];
    if (has[q] && iq >= 0 && iq < L0) dst = R.load(sx > 0 ? iq : L0 - 1 - iq, jj[q], kk[q]);
  };
#pragma unroll
  for (int r = 0; r < kAhead; ++r) {
#pragma unroll
    for (int q = 0; q < 2; ++q) fetch(t0 + r, q, buf[q][r]);
  }
  // next-sweep hyperplanes of the nodes this thread changed
  int hmin = 0x7fffffff, hmax = -1;
  bool done = false;
  for (int tb = t0; tb < nsteps && !done; tb += kAhead) {
#pragma unroll
    for (int r = 0; r < kAhead; ++r) {
      const int t = tb + r;
      if (t < nsteps && !done) {  // the same in every thread
        In cur[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          cur[q] = buf[q][r];
          fetch(t + kAhead, q, buf[q][r]);
        }
        int stepch = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int iq = t - jq[q] - kq[q];
          if (has[q] && iq >= 0 && iq < L0) {
            const int i = sx > 0 ? iq : L0 - 1 - iq;
            if (R.update(i, jj[q], kk[q], cur[q])) {
              stepch = 1;
              const int h = next_plane(i, jj[q], kk[q]);
              hmin = min(hmin, h);
              hmax = max(hmax, h);
            }
          }
        }
        if (t >= tmax) {
          if (!__syncthreads_or(stepch)) done = true;
        } else {
          __syncthreads();
        }
      }
    }
  }
  if (hmax >= 0) {
    atomicMin(&sh_rng[0], hmin);
    atomicMax(&sh_rng[1], hmax);
  }
  __syncthreads();
  const bool any = sh_rng[1] >= 0;
  P.t0 = any ? max(sh_rng[0] - 1, 0) : 1;
  P.tmax = any ? min(sh_rng[1] + 1, nsteps - 1) : 0;
  __syncthreads();  // every thread has read sh_rng before the next sweep resets it
  return any;
}

// 2^d orders of the loop nest (x outermost, z innermost) until a sweep
// changes nothing, at most max_sweeps; every node starts out as possibly
// changing, then each sweep covers what can change (sweep3), which gives the
// full sweeps' values, winds and sweep count.
template <typename Rule>
__device__ int fsm3(Rule& R, int L0, int L1, int L2, int max_sweeps) {
  int s = 0;
  Range3 P{0, L0 + L1 + L2 - 3};
  while (s < max_sweeps) {
    const bool ch = sweep3(R, L0, L1, L2, s & 7, (s + 1) & 7, P);
    ++s;
    if (!ch) break;
  }
  return s;
}

// neighbour minima of box node x=(i,j,k); missing neighbours are +inf.  Both
// reads of an axis always happen (the node itself stands in for a neighbour
// outside the box) and a missing one is then replaced by +inf: selects, not
// branches around the reads.
template <typename T>
__device__ __forceinline__ void gather3(const T* u, int L0, int L1, int L2, int i, int j, int k, T (&m)[3],
                                        int (&ws)[3]) {
  const T inf = pinf<T>();
  const int x = i + L0 * (j + L1 * k);
  const int st[3] = {1, L0, L0 * L1};
  const int c[3] = {i, j, k};
  const int L[3] = {L0, L1, L2};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool hl = c[a] > 0, hh = c[a] < L[a] - 1;
    const T lo0 = u[hl ? x - st[a] : x];
    const T hi0 = u[hh ? x + st[a] : x];
    const T lo = hl ? lo0 : inf;
    const T hi = hh ? hi0 : inf;
    const bool lt = lo < hi;
    m[a] = lt ? lo : hi;
    ws[a] = lt ? 1 : -1;
  }
}

// Minimum-update rule (fine, Alg. fineupdate2D generalised; or Step 1 coarse,
// Alg. update2D generalised).  rd: global r*Delta at the node (NaN = fixed);
// wind codes go to a global per-box array when a value is lowered.
template <typename T, bool Coarse>
struct MinRule3 {
  T* u;
  int L0, L1, L2;
  const T* rd_g;       // global array of r*Delta
  uint8_t* w_g;        // global wind array of the box nodes
  int64_t base;        // global index of box node (0,0,0)
  int gs[3];           // global strides of the box axes
  int64_t wbase;       // index of box node (0,0,0) in w_g
  int ws_[3];          // strides of the box axes in w_g
  struct In {
    T rd;
  };
  __device__ __forceinline__ In load(int i, int j, int k) const {
    return In{rd_g[base + (int64_t)i * gs[0] + (int64_t)j * gs[1] + (int64_t)k * gs[2]]};
  }
  __device__ __forceinline__ bool update(int i, int j, int k, const In& in) const {
    const T rd = in.rd;
    if (disnan(rd)) return false;
    T m[3];
    int ws[3];
    gather3(u, L0, L1, L2, i, j, k, m, ws);
    uint8_t code;
    const T ut = godunov3<T, Coarse>(m, ws, rd, code);
    const int x = i + L0 * (j + L1 * k);
    if (ut < u[x]) {
      u[x] = ut;
      w_g[wbase + (int64_t)i * ws_[0] + (int64_t)j * ws_[1] + (int64_t)k * ws_[2]] = code;
      return true;
    }
    return false;
  }
};

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

// r*h and r*H with NaN at Gamma nodes
template <typename T>
__global__ void k_rd3(DD3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const bool g = !disnan(A.gfull[t]);
  const T nan = T(__builtin_nan(""));
  A.rdh[t] = g ? nan : A.r[t] * A.hT;
  A.rdH[t] = g ? nan : A.r[t] * A.HT;
}

template <typename T>
__device__ __forceinline__ bool near_candidate3(const DD3<T>& A, int64_t gi, int off, int64_t& X, T& v) {
  const int W2 = 2 * A.M - 1;
  const int dx = off % W2 - (A.M - 1), dy = (off / W2) % W2 - (A.M - 1), dz = off / (W2 * W2) - (A.M - 1);
  const int64_t g = A.gidx[gi];
  const int gx = (int)(g % A.n[0]), gy = (int)((g / A.n[0]) % A.n[1]), gz = (int)(g / ((int64_t)A.n[0] * A.n[1]));
  const int xi = gx + dx, yi = gy + dy, zi = gz + dz;
  if (xi < 0 || xi >= A.n[0] || yi < 0 || yi >= A.n[1] || zi < 0 || zi >= A.n[2]) return false;
  if (!coarse3(xi, yi, zi, A.M)) return false;
  X = idx3(A.n, xi, yi, zi);
  const int d2 = dx * dx + dy * dy + dz * dz;
  const T sq = dsqrt((T)d2);
  const T dist = A.hT * sq;
  v = A.gval[gi] + A.r[X] * dist;
  return true;
}

template <typename T>
__global__ void k_near3_a(DD3<T> A) {
  const int W2 = 2 * A.M - 1, W3 = W2 * W2 * W2;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A.ng * W3) return;
  int64_t X;
  T v;
  if (near_candidate3(A, t / W3, (int)(t % W3), X, v)) atomicMin(&A.near_key[X], okey(v));
}

template <typename T>
__global__ void k_near3_b(DD3<T> A) {
  const int W2 = 2 * A.M - 1, W3 = W2 * W2 * W2;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A.ng * W3) return;
  int64_t X;
  T v;
  const int64_t gi = t / W3;
  if (near_candidate3(A, gi, (int)(t % W3), X, v))
    if (okey(v) == A.near_key[X]) atomicMin(&A.near_win[X], (long long)gi);
}

// ---------------------------------------------------------------------------
// Step 1 on every lattice
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock3) void k_lattice_init3(DD3<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  int o[3];
  lattice_offset3(blockIdx.x, A.M, o[0], o[1], o[2]);
  int L[3];
  for (int a = 0; a < 3; ++a) L[a] = (A.n[a] - 1 - o[a]) / A.M + 1;
  const int cnt = L[0] * L[1] * L[2];
  T* u = (T*)smem;
  __shared__ int sh_free;
  if (threadIdx.x == 0) sh_free = 0;
  const int64_t base = idx3(A.n, o[0], o[1], o[2]);
  const int gs[3] = {A.M, A.M * A.n[0], A.M * A.n[0] * A.n[1]};
  int nfree = 0;
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    const int xi = o[0] + p0 * A.M, yi = o[1] + p1 * A.M, zi = o[2] + p2 * A.M;
    const int64_t X = idx3(A.n, xi, yi, zi);
    const T g = A.gfull[X];
    if (!disnan(g)) {
      u[x] = g;
      A.W[X] = 0;
    } else if (A.near_win[X] != 0x7fffffffffffffffll) {
      u[x] = (T)okey_dec(A.near_key[X]);
      const int64_t gg = A.gidx[A.near_win[X]];
      const int gx = (int)(gg % A.n[0]), gy = (int)((gg / A.n[0]) % A.n[1]),
                gz = (int)(gg / ((int64_t)A.n[0] * A.n[1]));
      const int dx = xi - gx, dy = yi - gy, dz = zi - gz;
      A.W[X] = wenc3((dx > 0) - (dx < 0), (dy > 0) - (dy < 0), (dz > 0) - (dz < 0));
    } else {
      u[x] = pinf<T>();
      A.W[X] = 0;
      ++nfree;
    }
  }
  __syncthreads();
  // nodes fixed by Gamma or by the near-Gamma initialisation are not updated
  struct Rule {
    T* u;
    int L0, L1, L2;
    const T* gfull;
    const long long* near_win;
    const T* rdH;
    uint8_t* W;
    bool homog;
    int64_t base;
    int gs0, gs1, gs2;
    struct In {
      T rd;  // NaN: the node is fixed
    };
    __device__ In load(int i, int j, int k) const {
      const int64_t X = base + (int64_t)i * gs0 + (int64_t)j * gs1 + (int64_t)k * gs2;
      const bool fixed = !disnan(gfull[X]) || near_win[X] != 0x7fffffffffffffffll;
      return In{fixed ? T(__builtin_nan("")) : rdH[X]};
    }
    __device__ bool update(int i, int j, int k, const In& in) const {
      const int64_t X = base + (int64_t)i * gs0 + (int64_t)j * gs1 + (int64_t)k * gs2;
      if (disnan(in.rd)) return false;
      T m[3];
      int ws[3];
      gather3(u, L0, L1, L2, i, j, k, m, ws);
      uint8_t code;
      const T ut = godunov3<T, true>(m, ws, in.rd, code, homog);
      const int x = i + L0 * (j + L1 * k);
      if (ut < u[x]) {
        u[x] = ut;
        W[X] = code;
        return true;
      }
      return false;
    }
  } R{u, L[0], L[1], L[2], A.gfull, A.near_win, A.rdH, A.W, A.coarse_homog != 0, base, gs[0], gs[1], gs[2]};
  const int ns = fsm3(R, L[0], L[1], L[2], A.max_coarse_sweeps);
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    A.U[base + (int64_t)p0 * gs[0] + (int64_t)p1 * gs[1] + (int64_t)p2 * gs[2]] = u[x];
  }
  for (int of = 32; of > 0; of >>= 1) nfree += __shfl_xor(nfree, of);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[1], (unsigned long long)sh_free * (unsigned long long)ns);
}

// ---------------------------------------------------------------------------
// Steps 2 and 3
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool iface3(int c, int S, int n) { return (c % S == 0) && c > 0 && c < n - 1; }

template <typename T>
__global__ __launch_bounds__(kBlock3) void k_tile3(DD3<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = A.S + 1;
  const long long t_start = (long long)wall_clock64();  // constant 100 MHz clock
  const int tile = A.tile_order ? A.tile_order[blockIdx.x] : (int)blockIdx.x;
  const int T0 = tile % A.P[0], T1 = (tile / A.P[0]) % A.P[1], T2 = tile / (A.P[0] * A.P[1]);
  const int b0 = T0 * A.S, b1 = T1 * A.S, b2 = T2 * A.S;
  const int cnt = L * L * L;
  T* u = (T*)smem;
  __shared__ int sh_free;
  if (threadIdx.x == 0) sh_free = 0;
  uint8_t* tw = A.tile_w + (int64_t)tile * cnt;
  int nfree = 0;
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int li = x % L, lj = (x / L) % L, lk = x / (L * L);
    const int c[3] = {b0 + li, b1 + lj, b2 + lk};
    const int lc[3] = {li, lj, lk};
    const int64_t X = idx3(A.n, c[0], c[1], c[2]);
    const T g = A.gfull[X];
    T v = pinf<T>();
    uint8_t wc = 0;
    if (!disnan(g)) {
      v = g;
    } else {
      ++nfree;
      bool inflow = false;
      uint8_t Wc = 0;
      bool onif = false;
      for (int a = 0; a < 3; ++a) onif = onif || ((lc[a] == 0 || lc[a] == A.S) && iface3(c[a], A.S, A.n[a]));
      if (onif) {
        Wc = A.W[X];
        for (int a = 0; a < 3; ++a) {
          if (!iface3(c[a], A.S, A.n[a])) continue;
          const int we = w_of(Wc, a);
          if ((lc[a] == 0 && we > 0) || (lc[a] == A.S && we < 0)) inflow = true;
        }
      }
      if (inflow) {
        v = A.U[X];
        wc = Wc;
      }
    }
    u[x] = v;
    tw[x] = wc;
  }
  __syncthreads();
  MinRule3<T, false> R;
  R.u = u; R.L0 = L; R.L1 = L; R.L2 = L;
  R.rd_g = A.rdh;
  R.w_g = tw;
  R.base = idx3(A.n, b0, b1, b2);
  R.gs[0] = 1; R.gs[1] = A.n[0]; R.gs[2] = A.n[0] * A.n[1];
  R.wbase = 0;
  R.ws_[0] = 1; R.ws_[1] = L; R.ws_[2] = L * L;
  const int ns = fsm3(R, L, L, L, A.max_fine_sweeps);
  const int F = L * L;
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int li = x % L, lj = (x / L) % L, lk = x / (L * L);
    const int c[3] = {b0 + li, b1 + lj, b2 + lk};
    const int lc[3] = {li, lj, lk};
    const int64_t X = idx3(A.n, c[0], c[1], c[2]);
    const T v = u[x];
    const uint8_t wc = tw[x];
    bool onif = false;
    for (int a = 0; a < 3; ++a) onif = onif || ((lc[a] == 0 || lc[a] == A.S) && iface3(c[a], A.S, A.n[a]));
    if (!onif) {
      A.u_out[X] = v;
      if (coarse3(c[0], c[1], c[2], A.M)) {
        A.uk[X] = v;
        A.wk[X] = wc;
      }
    }
    // faces: 0/1 = x low/high (index lj + L*lk), 2/3 = y (li + L*lk), 4/5 = z (li + L*lj)
    const int64_t fb = (int64_t)tile * 6 * F;
    if (li == 0) { A.face_u[fb + 0 * F + lj + L * lk] = v; A.face_w[fb + 0 * F + lj + L * lk] = wc; }
    if (li == A.S) { A.face_u[fb + 1 * F + lj + L * lk] = v; A.face_w[fb + 1 * F + lj + L * lk] = wc; }
    if (lj == 0) { A.face_u[fb + 2 * F + li + L * lk] = v; A.face_w[fb + 2 * F + li + L * lk] = wc; }
    if (lj == A.S) { A.face_u[fb + 3 * F + li + L * lk] = v; A.face_w[fb + 3 * F + li + L * lk] = wc; }
    if (lk == 0) { A.face_u[fb + 4 * F + li + L * lj] = v; A.face_w[fb + 4 * F + li + L * lj] = wc; }
    if (lk == A.S) { A.face_u[fb + 5 * F + li + L * lj] = v; A.face_w[fb + 5 * F + li + L * lj] = wc; }
  }
  for (int of = 32; of > 0; of >>= 1) nfree += __shfl_xor(nfree, of);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[0], (unsigned long long)sh_free * (unsigned long long)ns);
  if (threadIdx.x == 0 && A.tile_time) A.tile_time[tile] = (int)((long long)wall_clock64() - t_start);
}

// Reconciliation at every interface node (up to 8 candidates: the subdomains
// containing the node, x slowest, minus side first).
template <typename T>
__global__ void k_reconcile3(DD3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int c[3] = {(int)(t % A.n[0]), (int)((t / A.n[0]) % A.n[1]), (int)(t / ((int64_t)A.n[0] * A.n[1]))};
  bool ifa[3];
  bool any = false;
  for (int a = 0; a < 3; ++a) { ifa[a] = iface3(c[a], A.S, A.n[a]); any = any || ifa[a]; }
  if (!any) return;
  const int L = A.S + 1, F = L * L;
  int tl[3][2], ns[3];
  for (int a = 0; a < 3; ++a) {
    if (ifa[a]) { tl[a][0] = c[a] / A.S - 1; tl[a][1] = c[a] / A.S; ns[a] = 2; }
    else { tl[a][0] = min(c[a] / A.S, A.P[a] - 1); tl[a][1] = tl[a][0]; ns[a] = 1; }
  }
  T cu[8];
  uint8_t cw[8];
  int sd[8][3];
  int nc = 0;
  for (int x0 = 0; x0 < ns[0]; ++x0)
    for (int x1 = 0; x1 < ns[1]; ++x1)
      for (int x2 = 0; x2 < ns[2]; ++x2) {
        const int T0 = tl[0][x0], T1 = tl[1][x1], T2 = tl[2][x2];
        const int tile = T0 + A.P[0] * (T1 + A.P[1] * T2);
        const int l0 = c[0] - T0 * A.S, l1 = c[1] - T1 * A.S, l2 = c[2] - T2 * A.S;
        int f, q;
        if (l0 == 0) { f = 0; q = l1 + L * l2; }
        else if (l0 == A.S) { f = 1; q = l1 + L * l2; }
        else if (l1 == 0) { f = 2; q = l0 + L * l2; }
        else if (l1 == A.S) { f = 3; q = l0 + L * l2; }
        else if (l2 == 0) { f = 4; q = l0 + L * l1; }
        else { f = 5; q = l0 + L * l1; }
        const int64_t e = ((int64_t)tile * 6 + f) * F + q;
        cu[nc] = A.face_u[e];
        cw[nc] = A.face_w[e];
        sd[nc][0] = x0; sd[nc][1] = x1; sd[nc][2] = x2;
        ++nc;
      }
  const uint8_t Wk = A.W[t];
  const T inf = pinf<T>();
  bool keep[8];
  int nf = 0;
  for (int q = 0; q < nc; ++q) { keep[q] = cu[q] < inf; nf += keep[q]; }
  if (nf == 0)
    for (int q = 0; q < nc; ++q) keep[q] = true;
  int allow[3] = {3, 3, 3};
  for (int a = 0; a < 3; ++a) {
    if (!ifa[a]) continue;
    bool le = w_of(Wk, a) <= 0, ge = w_of(Wk, a) >= 0;
    for (int q = 0; q < nc; ++q)
      if (keep[q]) { le = le && w_of(cw[q], a) <= 0; ge = ge && w_of(cw[q], a) >= 0; }
    if (le) allow[a] = 2; else if (ge) allow[a] = 1;
  }
  int best = -1;
  for (int q = 0; q < nc; ++q) {
    if (!keep[q]) continue;
    bool ok = true;
    for (int a = 0; a < 3; ++a)
      if (ifa[a] && !((allow[a] >> sd[q][a]) & 1)) ok = false;
    if (!ok) continue;
    if (best < 0 || cu[q] < cu[best]) best = q;
  }
  if (best < 0)
    for (int q = 0; q < nc; ++q)
      if (keep[q] && (best < 0 || cu[q] < cu[best])) best = q;
  A.u_out[t] = cu[best];
  if (coarse3(c[0], c[1], c[2], A.M)) {
    A.uk[t] = cu[best];
    A.wk[t] = cw[best];
  }
}

// ---------------------------------------------------------------------------
// Step 4
// ---------------------------------------------------------------------------

// C^k = C_H(nbrs^H(U^k)) at every coarse node and the condition mask:
// bits 3a..3a+2 = allowed values -1, 0, +1 of component a of W~ (all three
// when a is not a normal axis of the node), bit 9 = C^k finite.
template <typename T>
__global__ void k_ck3(DD3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int c[3] = {(int)(t % A.n[0]), (int)((t / A.n[0]) % A.n[1]), (int)(t / ((int64_t)A.n[0] * A.n[1]))};
  if (!coarse3(c[0], c[1], c[2], A.M)) return;
  const T inf = pinf<T>();
  const int64_t st[3] = {A.M, (int64_t)A.M * A.n[0], (int64_t)A.M * A.n[0] * A.n[1]};
  T m[3];
  int ws[3];
  for (int a = 0; a < 3; ++a) {
    const T lo = c[a] - A.M >= 0 ? A.U[t - st[a]] : inf;
    const T hi = c[a] + A.M <= A.n[a] - 1 ? A.U[t + st[a]] : inf;
    const bool lt = lo < hi;
    m[a] = lt ? lo : hi;
    ws[a] = lt ? 1 : -1;
  }
  uint8_t code;
  const T rd = A.r[t] * A.HT;
  const T v = godunov3<T, true>(m, ws, rd, code, A.coarse_homog != 0);
  A.ck[t] = v;
  const uint8_t wk = A.wk[t], Wk = A.W[t];
  uint16_t mask = dfinite(v) ? (uint16_t)512 : (uint16_t)0;
  for (int a = 0; a < 3; ++a) {
    int bits = 7;
    if (c[a] % A.M == 0) {
      const int q = w_of(wk, a), r = w_of(Wk, a);
      const bool le = q <= 0 && r <= 0, ge = q >= 0 && r >= 0;
      bits = (le ? 1 : 0) | ((le || ge) ? 2 : 0) | (ge ? 4 : 0);
    }
    mask |= (uint16_t)(bits << (3 * a));
  }
  A.mk[t] = mask;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock3) void k_lattice_correct3(DD3<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  int o[3];
  lattice_offset3(blockIdx.x, A.M, o[0], o[1], o[2]);
  int L[3];
  for (int a = 0; a < 3; ++a) L[a] = (A.n[a] - 1 - o[a]) / A.M + 1;
  const int cnt = L[0] * L[1] * L[2];
  T* u = (T*)smem;
  __shared__ int sh_free;
  if (threadIdx.x == 0) sh_free = 0;
  const int64_t base = idx3(A.n, o[0], o[1], o[2]);
  const int gs[3] = {A.M, A.M * A.n[0], A.M * A.n[0] * A.n[1]};
  int nfree = 0;
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    const int64_t X = base + (int64_t)p0 * gs[0] + (int64_t)p1 * gs[1] + (int64_t)p2 * gs[2];
    const T g = A.gfull[X];
    if (!disnan(g)) u[x] = g; else { u[x] = pinf<T>(); ++nfree; }
  }
  __syncthreads();
  struct Rule {
    T* u;
    int L0, L1, L2;
    const T* gfull;
    const T* rdH;
    const uint16_t* mk;
    const T* uk;
    const T* ck;
    T theta;
    int64_t base;
    int gs0, gs1, gs2;
    const T* tref;
    const T* ukm1;
    const T* ckm1;
    const T* ckm2;
    ThetaPar q;
    bool homog;
    struct In {
      T rd;   // NaN at Gamma nodes
      T ukx, ckx;
      unsigned mask;
      double ta, tb;  // weight terms (theta_at)
    };
    __device__ In load(int i, int j, int k) const {
      const int64_t X = base + (int64_t)i * gs0 + (int64_t)j * gs1 + (int64_t)k * gs2;
      In in{rdH[X], uk[X], ck[X], (unsigned)mk[X], 0.0, 0.0};
      if (MODE == 1) {
        in.ta = __builtin_nan("");
        if (ukm1 && ckm1 && ckm2) {
          const double num = (double)in.ukx - (double)ukm1[X];
          const double d1 = (double)in.ckx - (double)ckm1[X];
          const double d2 = (double)ckm1[X] - (double)ckm2[X];
          const double hs = q.w1 * d1 + q.w2 * d2;
          if (finite_d(num) && finite_d(hs)) { in.ta = num; in.tb = hs; }
        }
      } else if (MODE == 2) {
        in.ta = (double)tref[X] - (double)in.ukx;
      } else if (MODE == 3) {
        in.ta = (double)tref[X];
      }
      return in;
    }
    __device__ bool update(int i, int j, int k, const In& in) const {
      if (disnan(in.rd)) return false;
      T m[3];
      int ws[3];
      gather3(u, L0, L1, L2, i, j, k, m, ws);
      uint8_t code;
      const T ut = godunov3<T, true>(m, ws, in.rd, code, homog);
      const unsigned mask = in.mask;
      bool cond = dfinite(ut) && (mask & 512u);
      for (int a = 0; a < 3; ++a) cond = cond && ((mask >> (3 * a + w_of(code, a) + 1)) & 1u);
      const T ukx = in.ukx;
      T th = theta;
      if (MODE != 0) th = (T)theta_at<MODE>(ut, in.ckx, in.ta, in.tb, (double)theta, q);
      const T v = cond ? ukx + th * (ut - in.ckx) : ukx;
      const int x = i + L0 * (j + L1 * k);
      if (v != u[x]) {
        u[x] = v;
        return true;
      }
      return false;
    }
  } R{u, L[0], L[1], L[2], A.gfull, A.rdH, A.mk, A.uk, A.ck, A.theta, base, gs[0], gs[1], gs[2],
      A.tref, A.ukm1, A.ckm1, A.ckm2, A.tq, A.coarse_homog != 0};
  int ns;
  if (MODE == 0 && A.rec != nullptr) {
    // the operands gathered once (the lattice's nodes are M apart in every
    // axis of the full-grid arrays: a memory sector per 4-byte read), then
    // read by every sweep from contiguous records
    Corr3Rec<T>* rec = reinterpret_cast<Corr3Rec<T>*>(A.rec) + (size_t)blockIdx.x * A.rec_stride;
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
      const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
      const int64_t X = base + (int64_t)p0 * gs[0] + (int64_t)p1 * gs[1] + (int64_t)p2 * gs[2];
      rec[x] = Corr3Rec<T>{A.rdH[X], A.uk[X], A.ck[X], (unsigned)A.mk[X]};
    }
    __syncthreads();
    struct RecRule : Rule {
      const Corr3Rec<T>* rec;
      __device__ typename Rule::In load(int i, int j, int k) const {
        const Corr3Rec<T> q = rec[i + this->L0 * (j + this->L1 * k)];
        return typename Rule::In{q.rd, q.ukx, q.ckx, q.mask, 0.0, 0.0};
      }
    };
    RecRule RR;
    static_cast<Rule&>(RR) = R;
    RR.rec = rec;
    ns = fsm3(RR, L[0], L[1], L[2], A.max_coarse_sweeps);
  } else {
    ns = fsm3(R, L[0], L[1], L[2], A.max_coarse_sweeps);
  }
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    const int64_t X = base + (int64_t)p0 * gs[0] + (int64_t)p1 * gs[1] + (int64_t)p2 * gs[2];
    A.Un[X] = u[x];
    A.Wn[X] = disnan(A.gfull[X]) ? A.wk[X] : (uint8_t)0;
  }
  for (int of = 32; of > 0; of >>= 1) nfree += __shfl_xor(nfree, of);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[1], (unsigned long long)sh_free * (unsigned long long)ns);
}

// ---------------------------------------------------------------------------
// causal sweep: coarse-cell wavefront
//
// Directions that keep the x direction overlap: when a later direction
// reverses the axes in a set R, a cell on anti-diagonal t of the earlier one
// is on t - 2 sum_{a in R} C'_a + sum_{a in R} (CN_a - 1) of the later, so
// the later can run sum_{a in R} (CN_a - 1) + 2 diagonals behind (z reversed:
// CN2 + 1; y and z: CN1 + CN2) in the same launches:
// every cell it takes, and the cells next to it, the earlier one has
// finished, and it writes no cell the earlier one will still read.  So
// directions 4m .. 4m+3 can run interleaved in that order; 4m+3 -> 4m+4
// reverses x as well.  The causal sweep takes its cells in this order in
// one persistent launch (k_causal3p, below); the whole-grid FSM's boxes
// use the same staggering in launches.
//
// The launches of k_grid_sweep3 (the whole-grid FSM, boxes for cells: sweeps
// 4m .. 4m+3 share launches), with each sweep's launch number t and change
// flag (offset into A.changed).
struct GridLaunch3 {
  int n;
  int dir[4], diag[4], t[4], start[5], chg_off[4];
};
//
// Cell (I, J, K) owns the coarse nodes with coordinates in [IM, IM+M) x
// [JM, JM+M) x [KM, KM+M) (its three low faces).  In sweep direction s a node
// X takes V(X) = max(U(X), old U(X + s_e e) for the axes where W_e = -s_e),
// then U_new(X) = max(V(X), U_new(X - s_e e) for the axes where W_e = s_e),
// each comparison only with a coarse fine neighbour.  A link X - s_e e lies
// in the same cell or in an upwind cell, so cells are processed one coarse
// anti-diagonal per launch.  Links into upwind cells read final values and
// are folded into V; the links inside the cell are resolved level by level
// (a'+b'+c' in sweep order) in LDS.  max is exact, so any order that
// respects the links gives the serial sweep's values.
// ---------------------------------------------------------------------------

// owned node q of a cell with extents E -> local coordinates: first the face
// l0 = 0 (E1*E2), then l0 > 0, l1 = 0 ((E0-1)*E2), then l0 > 0, l1 > 0,
// l2 = 0 ((E0-1)*(E1-1))
__device__ __forceinline__ void owned_coords(int q, const int (&E)[3], int (&l)[3]) {
  const int fa = E[1] * E[2], fb = (E[0] - 1) * E[2];
  if (q < fa) { l[0] = 0; l[1] = q % E[1]; l[2] = q / E[1]; return; }
  q -= fa;
  if (q < fb) { l[0] = 1 + q % (E[0] - 1); l[1] = 0; l[2] = q / (E[0] - 1); return; }
  q -= fb;
  l[0] = 1 + q % (E[0] - 1);
  l[1] = 1 + q / (E[0] - 1);
  l[2] = 0;
}

__device__ __forceinline__ int owned_index(const int (&l)[3], const int (&E)[3]) {
  const int fa = E[1] * E[2], fb = (E[0] - 1) * E[2];
  if (l[0] == 0) return l[1] + E[1] * l[2];
  if (l[1] == 0) return fa + (l[0] - 1) + (E[0] - 1) * l[2];
  return fa + fb + (l[0] - 1) + (E[0] - 1) * (l[1] - 1);
}

// cell (Iq, Jq, Kq) of diagonal diag in sweep order: the rem-th of the
// diagonal (false past its end)
__device__ __forceinline__ bool diag_cell(const int (&CN)[3], int diag, int rem, int& Iq, int& Jq, int& Kq) {
  for (int i = max(0, diag - (CN[1] - 1) - (CN[2] - 1)); i <= min(diag, CN[0] - 1); ++i) {
    const int r2 = diag - i;
    const int jlo = max(0, r2 - (CN[2] - 1)), jhi = min(r2, CN[1] - 1);
    const int cntj = jhi - jlo + 1;
    if (cntj <= 0) continue;
    if (rem < cntj) { Iq = i; Jq = jlo + rem; Kq = r2 - Jq; return true; }
    rem -= cntj;
  }
  return false;
}

// U as the causal sweep reads and writes it: plain accesses, or (COH) accesses
// coherent across the whole device (no copy in a cache that another
// compute die cannot see), for the persistent sweep, whose blocks hand
// values to each other without kernel boundaries.
template <bool COH, typename T>
__device__ __forceinline__ T uld(const T* p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}
template <bool COH, typename T>
__device__ __forceinline__ void ust(T* p, T v) {
  if constexpr (COH) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}

// The causal-sweep update of one cell (C: its actual coordinates) in
// direction dir, by the whole block (every thread calls it).
template <bool COH = false, typename T>
__device__ __forceinline__ void causal3_cell(const DD3<T>& A, T* U, const uint8_t* W, int dir, const int (&C)[3]) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s[3] = {(dir & 4) ? 1 : -1, (dir & 2) ? 1 : -1, (dir & 1) ? 1 : -1};
  const int M = A.M;
  int E[3];  // cell extent along each axis (the last cell holds the far boundary plane only)
  for (int a = 0; a < 3; ++a) E[a] = min(M, A.n[a] - C[a] * M);
  const int nown = E[1] * E[2] + (E[0] - 1) * E[2] + (E[0] - 1) * (E[1] - 1);
  const int cap = 3 * M * M;
  T* val = (T*)smem;                                   // value per owned node
  short* pred = (short*)(val + cap);                   // in-cell link per axis, -1 = none
  uint8_t* lvl = (uint8_t*)(pred + 3 * cap);           // level, 255 = not updated (Gamma)
  const int64_t st[3] = {1, A.n[0], (int64_t)A.n[0] * A.n[1]};
  // the thread's first node, kept in registers for the level loop
  T myv = T(0);
  uint8_t mylv = 255;
  short mypr[3] = {-1, -1, -1};
  for (int q = threadIdx.x; q < nown; q += blockDim.x) {
    int l[3];
    owned_coords(q, E, l);
    const int c[3] = {C[0] * M + l[0], C[1] * M + l[1], C[2] * M + l[2]};
    const int64_t X = idx3(A.n, c[0], c[1], c[2]);
    // every value the node may need, requested at once: its own, Gamma,
    // wind, and both fine neighbours along each axis (where they exist)
    T v = uld<COH>(&U[X]);
    const T g = A.gfull[X];
    const uint8_t wc = W[X];
    T nb[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      nb[a][0] = c[a] > 0 ? uld<COH>(&U[X - st[a]]) : T(0);
      nb[a][1] = c[a] < A.n[a] - 1 ? uld<COH>(&U[X + st[a]]) : T(0);
    }
    uint8_t lv = 255;
    short pr[3] = {-1, -1, -1};
    if (disnan(g)) {
      for (int a = 0; a < 3; ++a) {
        const int wa = w_of(wc, a);
        if (wa == 0) continue;
        // old value downwind (W_a = -s_a) or new value upwind (W_a = s_a)
        int cn[3] = {c[0], c[1], c[2]};
        cn[a] -= wa;
        if (cn[a] < 0 || cn[a] >= A.n[a] || !coarse3(cn[0], cn[1], cn[2], M)) continue;
        const int la = l[a] - wa;
        if (wa == s[a] && la >= 0 && la < E[a]) {
          int ll[3] = {l[0], l[1], l[2]};
          ll[a] = la;
          pr[a] = (short)owned_index(ll, E);
        } else {
          v = vmax(v, nb[a][wa > 0 ? 0 : 1]);  // U[X - wa * st[a]]
        }
      }
      int lq = 0;
      for (int a = 0; a < 3; ++a) lq += s[a] > 0 ? l[a] : E[a] - 1 - l[a];
      lv = (uint8_t)lq;
    }
    val[q] = v;
    lvl[q] = lv;
    for (int a = 0; a < 3; ++a) pred[3 * q + a] = pr[a];
    if (q == (int)threadIdx.x) {
      myv = v;
      mylv = lv;
      for (int a = 0; a < 3; ++a) mypr[a] = pr[a];
    }
  }
  __syncthreads();
  const int nlev = (E[0] - 1) + (E[1] - 1) + (E[2] - 1);
  // level 0 has no in-cell link
  if (nown <= (int)blockDim.x) {
    // one node per thread: only the predecessors' values come from LDS
    T v = myv;
    for (int lev = 1; lev <= nlev; ++lev) {
      if (mylv == lev) {
        for (int a = 0; a < 3; ++a)
          if (mypr[a] >= 0) v = vmax(v, val[mypr[a]]);
        val[threadIdx.x] = v;
      }
      __syncthreads();
    }
  } else {
    for (int lev = 1; lev <= nlev; ++lev) {
      for (int q = threadIdx.x; q < nown; q += blockDim.x) {
        if (lvl[q] != lev) continue;
        T v = val[q];
        for (int a = 0; a < 3; ++a) {
          const int pq = pred[3 * q + a];
          if (pq >= 0) v = vmax(v, val[pq]);
        }
        val[q] = v;
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < nown; q += blockDim.x) {
    int l[3];
    owned_coords(q, E, l);
    ust<COH>(&U[idx3(A.n, C[0] * M + l[0], C[1] * M + l[1], C[2] * M + l[2])], val[q]);
  }
}

// The causal sweep in one persistent launch: the blocks take the (direction,
// cell) items of the launch schedule above in its order (block b: items b,
// b + gridDim.x, ...) and start an item once the cells it depends on are
// done, instead of waiting for whole launches:
//   - in its own direction, the upwind face neighbour along each axis (its
//     links and old values come from there or from cells before them);
//   - in the previous direction, the cell itself and its six face
//     neighbours (whose nodes it reads and writes; transitively every
//     earlier direction is then done with them too).
// done[dir * ncell + cell] holds the epoch of the sweep that finished the
// cell.  Every item waits only for items earlier in the order, and every
// block is resident (the host launches no more blocks than fit at once), so
// every wait ends; a wait that exceeds its bound sets abort (all later waits
// return at once) and counters[3], which the host reports as an internal
// error.
// abort_flag[0]: set by the first wait that gives up, which also records
// its item, a flag it waited for, the value it last read there, the epoch
// and its block in abort_flag[1..5] (reported by the host).
constexpr int kCausalSpin = 1 << 20;

template <typename T>
__global__ __launch_bounds__(256) void k_causal3p(DD3<T> A, T* U, const uint8_t* W, const int* items, int nitems,
                                                 int* done, int epoch, int* abort_flag) {
  const int CN[3] = {A.NC[0] + 1, A.NC[1] + 1, A.NC[2] + 1};
  const int ncell = CN[0] * CN[1] * CN[2];
  __shared__ int sh_ok;
  for (int it = (int)blockIdx.x; it < nitems; it += (int)gridDim.x) {
    const int code = items[it];
    const int dir = code & 7;
    const int C[3] = {(code >> 3) & 63, (code >> 9) & 63, (code >> 15) & 63};
    const int s[3] = {(dir & 4) ? 1 : -1, (dir & 2) ? 1 : -1, (dir & 1) ? 1 : -1};
    auto cell = [&](int i, int j, int k) { return i + CN[0] * (j + CN[1] * k); };
    if (threadIdx.x < kWave) {
      // the flags this item waits for, one per lane, polled together (one
      // device round trip per poll): lanes 0-2 the upwind face neighbours in
      // its own direction, lane 3 the cell in the previous direction, lanes
      // 4-9 its face neighbours there; -1: none
      const int lane = (int)threadIdx.x;
      int fi = -1;
      int c[3] = {C[0], C[1], C[2]};
      if (lane < 3) {
        c[lane] -= s[lane];
        if (c[lane] >= 0 && c[lane] < CN[lane]) fi = dir * ncell + cell(c[0], c[1], c[2]);
      } else if (dir > 0 && lane == 3) {
        fi = (dir - 1) * ncell + cell(C[0], C[1], C[2]);
      } else if (dir > 0 && lane < 10) {
        const int a = (lane - 4) >> 1;
        c[a] += (lane & 1) ? 1 : -1;
        if (c[a] >= 0 && c[a] < CN[a]) fi = (dir - 1) * ncell + cell(c[0], c[1], c[2]);
      }
      bool ok = true;
      int v = epoch;
      for (int n = 0;; ++n) {
        if (fi >= 0) v = __hip_atomic_load(&done[fi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool mine = fi < 0 || v == epoch;
        if (__all(mine)) break;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = false;
          break;
        }
        if (n >= kCausalSpin) {
          // the first lane still waiting records the item, the flag, the value
          // it last read there, the epoch and the block (reported by the host)
          const unsigned long long w = __ballot(!mine);
          if (lane == (int)__builtin_ctzll(w) && atomicCAS(abort_flag, 0, 1) == 0) {
            abort_flag[1] = it;
            abort_flag[2] = fi;
            abort_flag[3] = v;
            abort_flag[4] = epoch;
            abort_flag[5] = (int)blockIdx.x;
          }
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (lane == 0) {
        if (!ok) atomicOr(&A.counters[3], 1ull);
        sh_ok = ok ? 1 : 0;
      }
    }
    __syncthreads();
    const bool ok = sh_ok != 0;
    // U is read and written device-coherently inside the sweep, so a value
    // is visible everywhere once its store has completed: every wave waits
    // for its stores (a full s_waitcnt), then, after the barrier, thread 0
    // sets the flag (also device-coherent)
    if (ok) causal3_cell<true>(A, U, W, dir, C);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && ok)
      __hip_atomic_store(&done[dir * ncell + cell(C[0], C[1], C[2])], epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

// LDS bytes of k_causal3 for coarse spacing M
template <typename T>
inline size_t causal3_lds(int M) {
  const size_t cap = (size_t)3 * M * M;
  return cap * sizeof(T) + 3 * cap * sizeof(short) + cap;
}

// max |Un - U| over the coarse nodes: grid-stride loop, block maximum, one
// atomic per block
template <typename T>
__global__ __launch_bounds__(256) void k_residual3(DD3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  double dv = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
    const int c0 = (int)(t % A.n[0]), c1 = (int)((t / A.n[0]) % A.n[1]), c2 = (int)(t / ((int64_t)A.n[0] * A.n[1]));
    if (coarse3(c0, c1, c2, A.M)) {
      const T a = A.Un[t], b = A.U[t];
      double d = 0.0;
      if (!(a == b)) d = dabs((double)a - (double)b);
      if (disnan(d)) d = __builtin_huge_val();
      dv = dv < d ? d : dv;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(dv, o);
    dv = dv < v ? v : dv;
  }
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = dv;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = m < part[q] ? part[q] : m;
    if (m > 0.0) atomicMax(&A.counters[2], (unsigned long long)__double_as_longlong(m));
  }
}

template <typename T>
__global__ void k_skel3(DD3<T> A, const T* src, T* dst) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int c0 = (int)(t % A.n[0]), c1 = (int)((t / A.n[0]) % A.n[1]), c2 = (int)(t / ((int64_t)A.n[0] * A.n[1]));
  dst[t] = coarse3(c0, c1, c2, A.M) ? src[t] : T(__builtin_nan(""));
}

// ---------------------------------------------------------------------------
// eik_solve, d = 3: the fast sweeping method on the whole grid with the
// serial sweep's values.  The grid is cut into boxes of at most B^3 nodes;
// in each directional sweep the boxes are taken one box-diagonal per launch
// in sweep order, each box swept by one workgroup in LDS with the same
// hyperplane engine.  Neighbours across a box face are read from global
// memory: the upwind box finished earlier in this sweep and the downwind box
// has not started, which is what the lexicographic loop nest sees.
// ---------------------------------------------------------------------------

template <typename T>
struct GS3 {
  int n[3];
  int B;           // box side
  int nb[3];       // boxes per axis
  T hT;
  const T* r;
  const T* gfull;  // Gamma value per node, NaN if not Gamma
  T* u;
  uint8_t* w;
  unsigned int* changed;
  int* eval_at;    // [box] launch at which the box was last swept (-1: never)
  int* chg_at;     // [box] launch at which it last changed (-1: never)
};

// the stationary-box test of the 2D whole-grid sweep (box_needed), with six
// face neighbours
__device__ __forceinline__ bool box_needed3(const int* eval_at, const int* chg_at, const int (&T)[3],
                                           const int (&nb)[3]) {
  const int b = T[0] + nb[0] * (T[1] + nb[1] * T[2]);
  const int ev = eval_at[b];
  if (chg_at[b] == ev) return true;
  const int st[3] = {1, nb[0], nb[0] * nb[1]};
  for (int a = 0; a < 3; ++a) {
    if (T[a] > 0 && chg_at[b - st[a]] > ev) return true;
    if (T[a] < nb[a] - 1 && chg_at[b + st[a]] > ev) return true;
  }
  return false;
}

// The box that block b of a whole-grid launch sweeps: the launch holds the
// box diagonals GL.diag[g] of up to four sweeps (blocks [start[g],
// start[g+1]) for sweep g), and a diagonal's boxes are taken by increasing
// first, then second box index in sweep order.  Returns false for a block
// past the last box.
__device__ inline bool grid_box3(const GridLaunch3& GL, const int (&nb)[3], int b, int& g, int (&Tb)[3]) {
  g = 0;
  while (g + 1 < GL.n && b >= GL.start[g + 1]) ++g;
  const int dir = GL.dir[g], diag = GL.diag[g];
  const int s[3] = {(dir & 4) ? 1 : -1, (dir & 2) ? 1 : -1, (dir & 1) ? 1 : -1};
  int rem = b - GL.start[g];
  int Iq = -1, Jq = -1, Kq = -1;
  for (int i = max(0, diag - (nb[1] - 1) - (nb[2] - 1)); i <= min(diag, nb[0] - 1); ++i) {
    const int r2 = diag - i;
    const int jlo = max(0, r2 - (nb[2] - 1)), jhi = min(r2, nb[1] - 1);
    const int cntj = jhi - jlo + 1;
    if (cntj <= 0) continue;
    if (rem < cntj) { Iq = i; Jq = jlo + rem; Kq = r2 - Jq; break; }
    rem -= cntj;
  }
  if (Iq < 0) return false;
  Tb[0] = s[0] > 0 ? Iq : nb[0] - 1 - Iq;
  Tb[1] = s[1] > 0 ? Jq : nb[1] - 1 - Jq;
  Tb[2] = s[2] > 0 ? Kq : nb[2] - 1 - Kq;
  return true;
}

template <typename T>
__global__ void k_grid_init3(GS3<T> A) {
  const int64_t N = (int64_t)A.n[0] * A.n[1] * A.n[2];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const T g = A.gfull[t];
  A.u[t] = disnan(g) ? pinf<T>() : g;
  A.w[t] = 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock3) void k_grid_sweep3(GS3<T> A, GridLaunch3 GL) {
  extern __shared__ __align__(16) unsigned char smem[];
  // blocks [start[g], start[g+1]) take boxes of diagonal diag[g] of sweep g
  // of the launch (as the causal sweep's groups of directions)
  int g, Tb[3];
  if (!grid_box3(GL, A.nb, (int)blockIdx.x, g, Tb)) return;
  const int dir = GL.dir[g], t = GL.t[g];
  A.changed += GL.chg_off[g];
  if (!box_needed3(A.eval_at, A.chg_at, Tb, A.nb)) return;
  int o[3], L[3];
  for (int a = 0; a < 3; ++a) {
    o[a] = Tb[a] * A.B;
    L[a] = min(A.B, A.n[a] - o[a]);
  }
  const int cnt = L[0] * L[1] * L[2];
  T* u = (T*)smem;
  const int64_t base = idx3(A.n, o[0], o[1], o[2]);
  const int64_t gs1 = A.n[0], gs2 = (int64_t)A.n[0] * A.n[1];
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    u[x] = A.u[base + p0 + p1 * gs1 + p2 * gs2];
  }
  __syncthreads();
  struct Rule {
    T* u;
    int L0, L1, L2;
    const T* ug;
    const T* gfull;
    const T* r;
    uint8_t* w;
    T hT;
    int64_t base, gs1, gs2;
    int lo0, lo1, lo2;   // box has a neighbour box on the minus side
    int hi0, hi1, hi2;   // ... on the plus side
    struct In {
      T rd;  // NaN at Gamma nodes
    };
    __device__ In load(int i, int j, int k) const {
      const int64_t X = base + i + j * gs1 + k * gs2;
      return In{disnan(gfull[X]) ? r[X] * hT : T(__builtin_nan(""))};
    }
    __device__ bool update(int i, int j, int k, const In& in) const {
      const int64_t X = base + i + j * gs1 + k * gs2;
      if (disnan(in.rd)) return false;
      const T inf = pinf<T>();
      const int x = i + L0 * (j + L1 * k);
      const int c[3] = {i, j, k};
      const int L[3] = {L0, L1, L2};
      const int st[3] = {1, L0, L0 * L1};
      const int64_t gst[3] = {1, gs1, gs2};
      const int lo_nb[3] = {lo0, lo1, lo2}, hi_nb[3] = {hi0, hi1, hi2};
      T m[3];
      int ws[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T lo = c[a] > 0 ? u[x - st[a]] : (lo_nb[a] ? ug[X - gst[a]] : inf);
        const T hi = c[a] < L[a] - 1 ? u[x + st[a]] : (hi_nb[a] ? ug[X + gst[a]] : inf);
        const bool lt = lo < hi;
        m[a] = lt ? lo : hi;
        ws[a] = lt ? 1 : -1;
      }
      uint8_t code;
      const T ut = godunov3<T, false>(m, ws, in.rd, code);
      if (ut < u[x]) {
        u[x] = ut;
        w[X] = code;
        return true;
      }
      return false;
    }
  } R{u, L[0], L[1], L[2], A.u, A.gfull, A.r, A.w, A.hT, base, gs1, gs2,
      o[0] > 0, o[1] > 0, o[2] > 0,
      o[0] + L[0] < A.n[0], o[1] + L[1] < A.n[1], o[2] + L[2] < A.n[2]};
  Range3 P{0, L[0] + L[1] + L[2] - 3};
  const bool ch = sweep3(R, L[0], L[1], L[2], dir, dir, P);
  for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
    const int p0 = x % L[0], p1 = (x / L[0]) % L[1], p2 = x / (L[0] * L[1]);
    A.u[base + p0 + p1 * gs1 + p2 * gs2] = u[x];
  }
  if (threadIdx.x == 0) {
    const int bidx = Tb[0] + A.nb[0] * (Tb[1] + A.nb[1] * Tb[2]);
    A.eval_at[bidx] = t;
    if (ch) {
      A.chg_at[bidx] = t;
      atomicOr(A.changed, 1u);
    }
  }
}

}  // namespace eik
