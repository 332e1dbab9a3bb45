// Device code of the 2D domain-decomposition Eikonal solver for gfx950.
//
// Method: Martin & Tsai, arXiv 1805.04198, Sec. 3.2.  Every step here has a
// counterpart in the CPU reference that is checked value-by-value against it;
// the arithmetic of the local solve follows one fixed evaluation order (no FMA
// contraction: the library is built with -ffp-contract=off) so that the two
// agree bit for bit:
//     rd = r * Delta;  d = a - b;  t = rd*rd;  t = t + t;  t = t - d*d;
//     two-sided (|d| < rd):  u = ((a + b) + sqrt(t)) * 0.5
//     one-sided          :  u = min(a, b) + rd
//
// Layout: node (i, j) at i + n0*j.  Winds are 2-bit-per-axis codes (see
// include/eik.h).  Subdomains ("tiles") and coarse lattices are swept by one
// 64-lane wave each with the whole grid resident in LDS: lane = row in sweep
// order, and at step t lane j updates column t - j, i.e. the anti-diagonal
// (hyperplane) order, which gives exactly the values of the paper's
// lexicographic Gauss-Seidel sweep because a node only reads neighbours on the
// previous (already updated) and next (not yet updated) anti-diagonals.
// A 65th row (tiles of 64 cells) rides on lane 0 one step late.
//
// LDS grids carry a one-node halo ring: interior node (i, j) of an L0 x L1
// box sits at (j+1)*SP + (i+1).  The ring holds +inf (no neighbour: the
// one-sided rule on a box boundary) or, for the whole-grid sweep, the
// neighbouring values across the box edge; it is never updated.  SP is even,
// so neighbouring lanes (address step SP-1 or SP+1) hit different banks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace eik {

constexpr int kWave = 64;
// Box kernels run one workgroup of kBlock threads: all of them stage the box
// between HBM and LDS, wave 0 alone sweeps it.
constexpr int kBlock = 256;
constexpr int kMaxL = 65;  // nodes per axis of a tile / lattice held in LDS
// Every LDS array of a box is surrounded by kGuard spare elements: reads of
// idle lanes may fall there, and stores that must not land anywhere go to
// the lane's own slot kDummy + lane in the leading guard band (distinct
// addresses, so the discarded stores do not serialise on one bank).
constexpr int kGuard = 72;
constexpr int kDummy = -kGuard;
__device__ __forceinline__ int dummy_slot() { return kDummy + (int)(threadIdx.x & (kWave - 1)); }

template <typename T> __device__ __forceinline__ T pinf();
template <> __device__ __forceinline__ float pinf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double pinf<double>() { return __builtin_huge_val(); }

// Correctly rounded single-precision square root for arguments >= 2^-96
// (the local solve's t = 2(r Delta)^2 - (a-b)^2 is far above that): the
// hardware v_sqrt_f32 result s is within one ulp, and Tuckerman's rounding
// test with the adjacent products decides between pred(s), s and succ(s):
// x - pred(s)*s <= 0 means sqrt(x) lies below the lower midpoint, and
// x - succ(s)*s > 0 that it lies above the upper one (the residuals are
// multiples of ulp^2/2, so no value falls strictly between 0 and the true
// midpoint gap).  Other arguments (negative, NaN: the discarded branch) give
// an unspecified value.
__device__ __forceinline__ float dsqrt(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sm = __builtin_bit_cast(float, __builtin_bit_cast(int, s) - 1);
  const float sp = __builtin_bit_cast(float, __builtin_bit_cast(int, s) + 1);
  const float rm = __builtin_fmaf(-sm, s, x);
  const float rp = __builtin_fmaf(-sp, s, x);
  const float t = (rm <= 0.0f) ? sm : s;
  return (rp > 0.0f) ? sp : t;
}
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ bool disnan(float x) { return x != x; }
__device__ __forceinline__ bool disnan(double x) { return x != x; }
template <typename T> __device__ __forceinline__ bool dfinite(T x) { return dabs(x) < pinf<T>(); }

// e^x in double as a fixed sequence of IEEE operations: x = n ln2 + r with
// Cody and Waite's two-part ln2 (high part exact in 32 bits, as in fdlibm),
// |r| <= ln2/2, and the Taylor series of e^r to r^13 in Horner form.  0
// below -700 (where 1 + e^x rounds to 1), +inf from 709.78 on.
__device__ __forceinline__ double exp_cw(double x) {
  if (x != x) return x;
  if (x >= 709.78) return __builtin_huge_val();
  if (x < -700.0) return 0.0;
  const double n = __builtin_floor(x * 0x1.71547652b82fep0 + 0.5);
  const double r = (x - n * 0x1.62e42feep-1) - n * 0x1.a39ef35793c76p-33;
  double p = 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return __builtin_ldexp(p, (int)n);
}

// Step 4 weight rule (eqs. secthetaest and thetaest, Sec. 4.2; the reference
// weight M-bar - margin of Sec. 5.3): parameters and per-node terms
struct ThetaPar {
  double gamma, delta, x0, w0, w1, w2, margin;
};

// eq. thetaest: [s t + (1 - s) delta t]^+, s = 1 / (1 + e^{(t - x0)/gamma})
__device__ __forceinline__ double theta_damped(double tb, const ThetaPar& q) {
  const double e = exp_cw((tb - q.x0) / q.gamma);
  const double sg = 1.0 / (1.0 + e);
  const double th = sg * tb + (1.0 - sg) * (q.delta * tb);
  return th > 0.0 ? th : 0.0;
}

__device__ __forceinline__ bool finite_d(double x) { return __builtin_fabs(x) < __builtin_huge_val(); }

// Weight at a node in mode MODE (1 estimate, 2 reference, 3 field) from the
// candidate ut, C^k, the node's precomputed terms ta / tb (mode 1: u^k -
// u^{k-1} or NaN when it cannot be used, and w1 d1 + w2 d2; mode 2: u_ref -
// u^k; mode 3: theta) and the constant weight.
template <int MODE, typename T>
__device__ __forceinline__ double theta_at(T ut, T ck, double ta, double tb, double theta, const ThetaPar& q) {
  if (MODE == 1) {
    if (ta != ta) return theta;
    const double d0 = (double)ut - (double)ck;
    const double den = (q.w0 * d0 + tb) / ((q.w0 + q.w1) + q.w2);
    if (!finite_d(den) || den == 0.0) return theta;
    return theta_damped(ta / den, q);
  }
  if (MODE == 2) {
    const double den = (double)ut - (double)ck;
    if (!finite_d(ta) || !finite_d(den) || den == 0.0) return theta;
    const double th = ta / den - q.margin;
    return th > 0.0 ? th : 0.0;
  }
  return ta;
}

// ---- wind codes ----
__device__ __forceinline__ int wx_of(uint8_t c) { int v = c & 3; return v == 3 ? -1 : v; }
__device__ __forceinline__ int wy_of(uint8_t c) { int v = (c >> 2) & 3; return v == 3 ? -1 : v; }
__device__ __forceinline__ uint8_t wenc(int wx, int wy) { return (uint8_t)((wx & 3) | ((wy & 3) << 2)); }

// Local solve of the Godunov scheme (eq. godonuv) in the closed form of the
// coarse solver C_H (Sec. 3.2).  a, b: smaller neighbour per axis.
template <typename T>
__device__ __forceinline__ T godunov2(T a, T b, T rd, bool& two) {
  T d = a - b;
  two = dabs(d) < rd;
  if (two) {
    T t = rd * rd;
    t = t + t;
    t = t - d * d;
    return ((a + b) + dsqrt(t)) * T(0.5);
  }
  return (a < b) ? (a + rd) : (b + rd);
}

// Compiler-level ordering point between sweeps: every LDS write of one sweep
// is issued before any LDS read of the next.  One wave executes its LDS
// instructions in order, so no hardware barrier is needed.
__device__ __forceinline__ void step_fence() {
  __builtin_amdgcn_wave_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// Lane i receives lane i-1's value (lane 0 receives lane 63's): DPP wave_ror:1.
__device__ __forceinline__ int dpp_ror1(int v) {
  // every source lane exists under a rotation, so the old operand is unused
  return __builtin_amdgcn_update_dpp(v, v, 0x13C, 0xF, 0xF, false);
}
__device__ __forceinline__ float dpp_ror1(float v) {
  return __builtin_bit_cast(float, dpp_ror1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double dpp_ror1(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_ror1((int)(b & 0xffffffffll));
  const int hi = dpp_ror1((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// Lane i receives lane i-1's value, lane 0 receives fill: DPP wave_shr:1
// (lane 0 has no source lane and keeps the old operand).
__device__ __forceinline__ int dpp_shr1(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ float dpp_shr1(float v, float fill) {
  return __builtin_bit_cast(float, dpp_shr1(__builtin_bit_cast(int, v), __builtin_bit_cast(int, fill)));
}
__device__ __forceinline__ double dpp_shr1(double v, double fill) {
  const long long b = __builtin_bit_cast(long long, v), f = __builtin_bit_cast(long long, fill);
  const int lo = dpp_shr1((int)(b & 0xffffffffll), (int)(f & 0xffffffffll));
  const int hi = dpp_shr1((int)(b >> 32), (int)(f >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Smaller neighbour per axis with the flow-direction wind sign of its side
// (ties take the plus side, as the strict '<' of the paper's algorithms).
template <typename T>
__device__ __forceinline__ void pick(T m, T p, T& v, int& w) {
  const bool lt = m < p;
  v = lt ? m : p;
  w = lt ? 1 : -1;
}

// Godunov local solve, branch-free: both branches are evaluated with the same
// expressions as above and one is selected (the sqrt of a negative argument
// in the unused branch yields NaN and is discarded).
template <typename T>
__device__ __forceinline__ T godunov2_sel(T a, T b, T rd, bool& two) {
  const T d = a - b;
  two = dabs(d) < rd;
  T t = rd * rd;
  t = t + t;
  t = t - d * d;
  const T u2 = ((a + b) + dsqrt(t)) * T(0.5);
  const T u1 = ((a < b) ? a : b) + rd;
  return two ? u2 : u1;
}

// The homogenised coarse solver of the squares medium (Sec. 5.3, eq. homog),
// read as the upwind scheme of max(|u_x|, |u_y|) = r: the smaller neighbour
// plus r*H, which is the one-sided value of the Godunov solve.
template <typename T>
__device__ __forceinline__ T homog2(T a, T b, T rd) {
  return ((a < b) ? a : b) + rd;
}

// The steps [t0, tmax] of a sweep that reach every node that may change in
// it without an upwind change inside it.
struct Range2 {
  int t0, tmax;
};

// Two waves on one box.  In the loop nest's order of the sweep directions,
// sweeps 4m and 4m+1 (likewise 4m+2 and 4m+3) differ in the y direction only.
// The node in column c, row r of the first sweep's order lies on its
// anti-diagonal c + r and on the second's c + (L1 - 1 - r), so the second
// sweep can run on another wave (another SIMD) L1 + 4 steps behind the first
// (L1 + 5 when row 64 runs late on lane 0):
// it then reads every node after the first sweep has written it for the last
// time and writes none before the first sweep has read it for the last time,
// and computes the values of the two sweeps run one after the other.  Wave 0
// (the leader) runs the even sweeps and publishes its progress; wave 1 (the
// follower) runs the odd ones behind it.  The other transitions (4m+1 to
// 4m+2, 4m+3 to 4m+4) reverse both directions; there the next sweep waits
// for the whole previous one.  All fields live in LDS; each is written by one
// wave only.
constexpr int kPipeDone = 1 << 28;
constexpr int kPipeNoKey = 1 << 29;
constexpr int kPipeSpin = 1 << 22;  // polls after which a wait gives up and sets err
struct PipeSync {
  // leader, per lane: the minimum of (column - row), sweep order, over the
  // nodes the lane changed in the current sweep (from kPipeNoKey on: none),
  // and the steps of the sweep completed (every lane writes the same count;
  // it is read from lane 0's slot; kPipeDone after the sweep's end).  One
  // 8-byte store per lane and step pair publishes both.
  int2 kp[kWave];
  int lsweep;      // leader: index of its current sweep
  int fin;         // follower: 1 + the index of its last completed sweep
  int err;         // a wait gave up
  int ch[2];       // whether the last sweep of the leader [0] / follower [1] changed a node
  int ftmax;       // leader: the follower's last step that reaches a node next to its changes
  Range2 lrng;     // follower: the next leader sweep's steps that reach the nodes next to its changes
  int smax;        // leader: sweeps that still run once a cycle was found (else no limit)
  int lsteps;      // leader: anti-diagonal steps run, and the clock64 ticks spent in them
  long long lcyc;
};

__device__ __forceinline__ void pipe_init(PipeSync& ps) {
  ps.lsweep = -1;
  ps.fin = 0;
  ps.err = 0;
  ps.ch[0] = ps.ch[1] = 0;
  ps.smax = 0x7fffffff;
  ps.lsteps = 0;
  ps.lcyc = 0;
}

// Rules whose sweeps need not settle (Step 4 assigns, it takes no minimum)
// may provide cycle_check(s): called by the leader between sweeps s-1 and s
// (s a multiple of 4, both waves off the box), it returns p > 0 when the
// values equal those after sweep s-1-p (p a multiple of 4: the same
// directions follow, so the run repeats with period p from there on).
template <typename Rule>
struct HasCycleCheck {
  static constexpr bool value = false;
};
__device__ __forceinline__ int lds_load_acq(int* p) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
}
// one lane publishes; the release orders every earlier LDS access of the wave
// before it
__device__ __forceinline__ void lds_store_rel(int* p, int v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & (kWave - 1)) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// The per-step-pair progress signals (the leader's publish in sweep_dir, the
// follower's peek).  The LDS operations of one wave are performed in the
// order they are issued (the LDS counter of s_waitcnt counts them down in
// order, which the compiler's own partial waits rely on), so a store issued
// after the wave's earlier LDS accesses is performed after them, and a load
// issued after a load is performed after it.  Only the compiler must be kept
// from moving memory accesses across these: release / acquire at wavefront
// scope order them for the compiler and need no wait instruction, which
// saves the full LDS wait of a workgroup-scope release or acquire on every
// step pair.
__device__ __forceinline__ int lds_peek(int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// The first step of the follower's sweep that reaches a node next to a change
// of the leader's sweep (key as in PipeSync), and the step count the leader
// must have completed before the follower runs step pair (t, t+1).
__device__ __forceinline__ int follow_t0(int key, int L1) { return max(key + L1 - 2, 0); }
__device__ __forceinline__ int follow_lag(int L1, bool extra) { return L1 + 4 + (extra ? 1 : 0); }
// Follower: wait until the leader has completed `need` steps or ended its
// sweep (then tmax becomes the last step that reaches the nodes next to the
// leader's changes).  Returns the steps known to be complete.
__device__ __forceinline__ int pipe_wait(PipeSync* ps, int need, int& tmax) {
  for (int n = 0;; ++n) {
    const int p = lds_load_acq(&ps->kp[0].y);
    if (p >= kPipeDone) {
      tmax = __builtin_amdgcn_readfirstlane(ps->ftmax);
      return 0x7fffffff;
    }
    if (p >= need) return p;
    if (n >= kPipeSpin) {
      if ((threadIdx.x & (kWave - 1)) == 0) ps->err = 1;
      return 0x7fffffff;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Sweep-order columns of the nodes a lane changed during a sweep (min and
// max over both rows of lane 0 in a 65-row box), and whether lane 0 changed
// a node of row 64.
struct StepSpan {
  int cmin = 0x7fffffff, cmax = -1;
  bool rowB = false;
  int steps = 0;  // steps run (set at the end of the sweep)
};

// One directional Gauss-Seidel sweep (signs SX, SY) over an L0 x L1 box in
// LDS, anti-diagonal order, one lane per row.  Dataflow per step t, lane j
// (row j in sweep order, column i = t - j):
//   upwind-x value : the lane's own result of step t-1 (register)
//   upwind-y value : row j-1's result of step t-1, moved by DPP wave_ror:1
//   self, downwind-x, downwind-y, r*Delta, halo values : LDS, loaded one step
//                    ahead.  None of these locations is written during the
//                    step that loads it (nodes of step t are on anti-diagonal
//                    t; the loads are on t+1 and t+2, or halo), so no LDS
//                    round trip lies on the dependency chain.
// Row 64 (boxes of 65 rows) runs on lane 0 one step late, after row 0 is
// done; it takes its upwind-y value from lane 63's result of two steps back.
// Fixed nodes carry r*Delta = NaN, which makes the candidate NaN and leaves
// them untouched.  The step is branch-free: a lane that is idle or does not
// lower its node stores to a dummy LDS slot, and the address of a lane moves
// by SX every step (reads of idle lanes land in the guard bands around each
// LDS array).
//
// The sweep may start at step t0 > 0 and end early: the caller guarantees
// that no node before step t0 can change (the registers that carry values
// from step to step are then loaded from LDS), and the sweep stops after a
// step pair at or beyond tmax in which no lane changed a value.  span (as
// constructed) receives the steps at which each lane changed values.  Returns
// true in lanes that changed a value.
//
// PIPE selects the two-wave mode (PipeSync): 0 alone, 1 leader (publishes its
// progress and the key of its changes after every step pair), 2 follower
// (waits before every step pair until the leader is far enough ahead, and
// takes tmax from the leader once the leader's sweep has ended; `allowed` is
// the leader progress already known).
template <int SX, int SY, bool EXTRA, int PIPE = 0, typename Rule>
__device__ __forceinline__ bool sweep_dir(Rule& R, int L0, int L1, int SP, int t0, int tmax, StepSpan& span,
                                          PipeSync* ps = nullptr, int allowed = 0) {
  using T = typename Rule::real;
  using Pre = typename Rule::Pre;
  static_assert(PIPE == 0 || !Rule::kHalo, "two-wave sweeps read no halo values");
  const T inf = pinf<T>();
  const int lane = threadIdx.x & (kWave - 1);
  const int nsteps = L0 + L1 - 1 + (EXTRA ? 1 : 0);
  const int jA = min(max(SY > 0 ? lane : L1 - 1 - lane, 0), L1 - 1);
  const int jB = SY > 0 ? kWave : L1 - 1 - kWave;
  // LDS index of the lane's node at step t: x = x0 + SX * t
  const int xA0 = (jA + 1) * SP + 1 + (SX > 0 ? -lane : L0 - 1 + lane);
  const int xB0 = (jB + 1) * SP + 1 + (SX > 0 ? -(kWave + 1) : L0 - 1 + kWave + 1);
  const bool laneB = EXTRA && lane == 0;
  const bool rowA = lane < L1;
  auto x_at = [&](int t) { return ((laneB && t > kWave) ? xB0 : xA0) + SX * t; };
  // the lane's value after step t: its node's value, +inf before its row starts
  auto value_at = [&](int t) -> T {
    const bool useB = laneB && t > kWave;
    const int iq = t - (useB ? kWave + 1 : lane);
    const bool ok = t >= 0 && (useB || rowA) && (unsigned)iq < (unsigned)L0;
    const T v = R.value(ok ? x_at(t) : dummy_slot());
    return ok ? v : inf;
  };
  // t0 and tmax are the same in every lane; keep them in scalar registers
  t0 = __builtin_amdgcn_readfirstlane(t0);
  tmax = __builtin_amdgcn_readfirstlane(tmax);
  T cur = inf, cur_prev = inf;
  if (t0 > 0) {
    cur = value_at(t0 - 1);
    if (EXTRA) cur_prev = value_at(t0 - 2);
  }
  unsigned long long recent = 0;
  int x = x_at(t0);
  Pre pa = R.template load<SX, SY>(x), pb;
  // Lane state that changes only when lane 0 moves from row 0 to row 64
  // (EXTRA): the column offset (column = t - ioff), whether the lane's row is
  // the first one (no upwind-y neighbour: halo), whether it is row 64.
  const bool startB = laneB && t0 > kWave;
  int ioff = startB ? kWave + 1 : lane;
  bool ytop = lane == 0 && !startB;
  bool inB = startB;
  const int xB1 = xB0 + SX * (kWave + 1);
  const int ioffB = laneB ? kWave + 1 : lane;
  // One step; p holds this step's operands, pn receives the next step's.
  // PH: 0 any step; with EXTRA, 1 a step before step kWave (lane 0 on row 0,
  // cur_prev not needed) and 2 a step after step kWave + 1 (lane 0 on row
  // 64), which drop the checks for the switch.
  auto step = [&](auto ph, int t, const Pre& p, Pre& pn) {
    constexpr int PH = decltype(ph)::value;
    bool restart = false;
    if (PH == 0 && EXTRA && t == kWave + 1) {
      // lane 0 starts row 64 at its column 0
      ioff = laneB ? kWave + 1 : ioff;
      ytop = false;
      inB = laneB;
      restart = laneB;
    }
    const int iq = t - (PH == 2 ? ioffB : PH == 1 ? lane : ioff);
    const bool act = (EXTRA || rowA) && (unsigned)iq < (unsigned)L0;
    int x1 = x + SX;
    if (PH == 0 && EXTRA && t == kWave) x1 = laneB ? xB1 : x1;
    pn = R.template load<SX, SY>(x1);
    // keep the loads at the top of the step, a whole step ahead of their use
    __builtin_amdgcn_sched_barrier(0);
    T yprev, xprev;
    if (!Rule::kHalo && (PH == 1 || !EXTRA)) {
      // lane 0 holds the first row (no upwind-y neighbour: the halo, +inf)
      yprev = dpp_shr1(cur, inf);
      xprev = cur;
    } else if (Rule::kHalo) {
      const T ex = (EXTRA && PH != 1 && lane == kWave - 1) ? cur_prev : cur;
      const T from_prev_row = dpp_ror1(ex);
      const bool top = PH == 2 ? false : PH == 1 ? lane == 0 : ytop;
      yprev = top ? p.hy : from_prev_row;
      xprev = (iq == 0) ? p.hx : cur;
    } else {
      const T ex = (EXTRA && PH != 1 && lane == kWave - 1) ? cur_prev : cur;
      const T from_prev_row = dpp_ror1(ex);
      const bool top = PH == 2 ? false : PH == 1 ? lane == 0 : ytop;
      // the halo is +inf: the first row has no upwind-y neighbour, and a
      // lane's cur is +inf until its row starts (the delayed row restarts)
      yprev = top ? inf : from_prev_row;
      xprev = (EXTRA && restart) ? inf : cur;
    }
    const T xm = SX > 0 ? xprev : p.xn, xp = SX > 0 ? p.xn : xprev;
    const T ym = SY > 0 ? yprev : p.yn, yp = SY > 0 ? p.yn : yprev;
    bool ch;
    const T v = R.template compute<SX, SY>(xm, xp, ym, yp, p, x, act, ch);
    if (EXTRA && PH != 1) cur_prev = cur;
    cur = act ? v : cur;
    recent |= __ballot(ch);
    span.cmin = min(span.cmin, ch ? iq : 0x7fffffff);
    span.cmax = max(span.cmax, ch ? iq : -1);
    if (EXTRA && PH != 1) span.rowB = span.rowB || (ch && (PH == 2 ? laneB : inB));
    x = x1;
  };
  using Any = std::integral_constant<int, 0>;
  using RowA = std::integral_constant<int, 1>;
  using RowB = std::integral_constant<int, 2>;
  // Step pairs (t, t+1) from t while t < tend: pre(t) before a pair (true:
  // leave without running it), post() after it (true: leave).  With EXTRA,
  // pairs wholly before step kWave and wholly after step kWave + 1 take the
  // lean steps (t only grows, so the state the full steps keep is not needed
  // after the first lean row-64 pair).  Each phase is a loop of its own, so
  // that the loop bodies carry no per-pair dispatch.  Unrolled by two so that
  // the prefetch buffers alternate without copies; a trailing step past the
  // end is idle in every lane.
  int t = t0;
  auto pairs = [&](int tend, auto&& pre, auto&& post) -> bool {
    auto seg = [&](auto ph, int e) -> bool {
      for (; t < e; t += 2) {
        if (pre(t)) return true;
        step(ph, t, pa, pb);
        step(ph, t + 1, pb, pa);
        if (post()) {
          t += 2;
          return true;
        }
      }
      return false;
    };
    if (EXTRA) {
      if (t < kWave - 1 && seg(RowA{}, min(tend, kWave - 1))) return true;
      if (t < kWave + 2 && seg(Any{}, min(tend, kWave + 2))) return true;
      return seg(RowB{}, tend);
    }
    return seg(Any{}, tend);
  };
  auto no_pre = [](int) { return false; };
  if (PIPE == 2 && allowed < kPipeDone) {
    // while the leader runs: every pair waits until the leader is far enough
    // ahead (the progress for the next pair is read during this one, its wait
    // merges with the steps' own); tmax arrives when the leader ends.  Then
    // as a lone sweep (below).  Pairs this phase ran past tmax without
    // checking for a change are harmless: after a pair past tmax that changes
    // nothing, no later step can change anything either.
    const int lag = follow_lag(L1, EXTRA);
    int seen = 0;
    pairs(
        nsteps,
        [&](int tt) {
          if (tt + lag > allowed) {
            allowed = pipe_wait(ps, tt + lag, tmax);
            if (allowed >= kPipeDone) return true;
          }
          seen = lds_peek(&ps->kp[0].y);
          return false;
        },
        [&]() {
          const int seen_u = __builtin_amdgcn_readfirstlane(seen);
          if (seen_u >= kPipeDone) {
            tmax = __builtin_amdgcn_readfirstlane(ps->ftmax);
            allowed = 0x7fffffff;
            return true;
          }
          if (seen_u > allowed) allowed = seen_u;
          return false;
        });
  }
  // leader: the key of this lane's changes (lane 0 also holds row 64: a
  // smaller key than its own only widens the follower's sweep; no change
  // leaves cmin at INT_MAX, a key above kPipeNoKey) and the completed step
  // count, in one store per lane
  int2* const kp_lane = PIPE == 1 ? &ps->kp[lane] : nullptr;
  auto publish = [&](int done) {
    if constexpr (PIPE == 1) {
      const int k = span.cmin - ((EXTRA && laneB && span.rowB) ? kWave : lane);
      const unsigned long long word = ((unsigned long long)(unsigned)done << 32) | (unsigned)k;  // int2{k, done}
      __hip_atomic_store(reinterpret_cast<unsigned long long*>(kp_lane), word, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
  };
  // up to tmax the steps run unconditionally; after that the sweep ends with
  // the first step pair that changes nothing
  pairs(min(tmax - 1, nsteps), no_pre, [&]() {
    if (PIPE == 1) publish(t + 2);
    return false;
  });
  recent = 0;
  pairs(nsteps, no_pre, [&]() {
    if (PIPE == 1) publish(t + 2);
    if (recent == 0) return true;
    recent = 0;
    return false;
  });
  span.steps = t - t0;
  return span.cmax >= 0;  // a change has a column >= 0
}

// Minimum / maximum over the 64 lanes (all active), returned in every lane:
// a prefix scan within each row of 16 lanes (DPP row_shr 1, 2, 4, 8), then
// row 0's result into row 1 and row 2's into row 3 (row_bcast:15), then the
// first half's into the second (row_bcast:31); lane 63 ends with the result.
// Lanes without a source keep the identity.
template <bool MIN>
__device__ __forceinline__ int wave_reduce(int v) {
  constexpr int id = MIN ? 0x7fffffff : (int)0x80000000;
  auto op = [](int a, int b) { return MIN ? min(a, b) : max(a, b); };
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, kWave - 1);
}
__device__ __forceinline__ int wave_min(int v) { return wave_reduce<true>(v); }
__device__ __forceinline__ int wave_max(int v) { return wave_reduce<false>(v); }

// Sweeps restricted to what can change.  The nodes that may change in a
// sweep without an upwind change inside it are those next to a change of the
// previous sweep (a node whose neighbours kept their values since its last
// evaluation computes the same candidate again and cannot change); they lie
// on the anti-diagonals of the sweep within one of a changed node.  A sweep
// starts at the first such step and, from the last one on, stops after the
// first step pair that changes nothing.  Each lane's span (its smallest and
// largest changed column; the row is the lane's) gives the extreme
// anti-diagonals of its changes in the next sweep's order: in the follower's
// (y reversed) column - row + L1 - 1, in the next leader's (both reversed)
// L0 + L1 - 2 - (column + row).  Row 64 runs one step late, hence the
// margin of one step at the end.  The follower starts from the published
// keys (later changes of the leader lie ahead of it) and takes its last step
// once the leader has ended.
//
// The leader's sweep s over the steps P, with its progress published for the
// follower; at its end the follower's last step and whether it changed
// anything.  Returns that flag (the same in every lane).
template <int SX, int SY, bool EXTRA, typename Rule>
__device__ __forceinline__ bool sweep_lead(Rule& R, int L0, int L1, int SP, const Range2& P, PipeSync* ps, int s) {
  const int lane = threadIdx.x & (kWave - 1);
  const int t0 = P.t0, tmax = P.tmax;
  ps->kp[lane] = make_int2(0x7fffffff, t0);  // steps before t0 change nothing
  lds_store_rel(&ps->lsweep, s);
  StepSpan sp;
  // the clock read is a scalar memory operation, which completes out of
  // order: take its value before the sweep, so that the sweep's LDS waits
  // need not wait for it
  long long c0 = clock64();
  __asm__ __volatile__("" : "+s"(c0));
  const bool lane_ch = sweep_dir<SX, SY, EXTRA, 1>(R, L0, L1, SP, t0, tmax, sp, ps);
  const long long c1 = clock64();
  const bool ch = __any(lane_ch);
  if (lane == 0) {
    ps->lsteps += sp.steps;
    ps->lcyc += c1 - c0;
  }
  // lane 0's row 64 (column - 64) never exceeds its row 0 (column - 0)
  const int kx = wave_max(sp.cmax >= 0 ? sp.cmax - lane : (int)0x80000000);
  if (lane == 0) {
    ps->ftmax = ch ? kx + L1 + (EXTRA ? 1 : 0) : 0;
    ps->ch[0] = ch ? 1 : 0;
  }
  lds_store_rel(&ps->kp[0].y, kPipeDone);
  return ch;
}

// The follower's sweep s from step t0 (tmax: its last step that reaches a
// node next to the leader's changes, or "none yet" while the leader runs);
// publishes the next leader sweep's steps and its own flag, then fin = s + 1.
template <int SX, int SY, bool EXTRA, typename Rule>
__device__ __forceinline__ bool sweep_follow(Rule& R, int L0, int L1, int SP, PipeSync* ps, int s, int t0, int tmax,
                                             int allowed) {
  const int lane = threadIdx.x & (kWave - 1);
  StepSpan sp;
  const bool lane_ch = sweep_dir<SX, SY, EXTRA, 2>(R, L0, L1, SP, t0, tmax, sp, ps, allowed);
  const bool ch = __any(lane_ch);
  // anti-diagonals (column + row) of the changes; lane 0 may hold row 64
  const int dmax = wave_max(sp.cmax >= 0 ? sp.cmax + ((EXTRA && lane == 0 && sp.rowB) ? kWave : lane)
                                         : (int)0x80000000);
  const int dmin = wave_min(sp.cmax >= 0 ? sp.cmin + lane : 0x7fffffff);
  if (lane == 0) {
    ps->lrng.t0 = ch ? max(L0 + L1 - 2 - dmax - 1, 0) : 0;
    ps->lrng.tmax = ch ? L0 + L1 - 2 - dmin + 1 + (EXTRA ? 1 : 0) : 0;
    ps->ch[1] = ch ? 1 : 0;
  }
  lds_store_rel(&ps->fin, s + 1);
  return ch;
}

// One full directional sweep (used by the whole-grid FSM, one sweep per
// launch).
template <int SX, int SY, typename Rule>
__device__ __forceinline__ bool sweep_dir2(Rule& R, int L0, int L1, int SP) {
  StepSpan sp;
  const int n = L0 + L1;
  return (L1 > kWave) ? sweep_dir<SX, SY, true>(R, L0, L1, SP, 0, n, sp)
                      : sweep_dir<SX, SY, false>(R, L0, L1, SP, 0, n, sp);
}

template <typename Rule>
__device__ __forceinline__ bool sweep_any(Rule& R, int L0, int L1, int SP, int dir) {
  switch (dir) {
    case 0: return sweep_dir2<-1, -1>(R, L0, L1, SP);
    case 1: return sweep_dir2<-1, 1>(R, L0, L1, SP);
    case 2: return sweep_dir2<1, -1>(R, L0, L1, SP);
    default: return sweep_dir2<1, 1>(R, L0, L1, SP);
  }
}

// Sweep in the 2^d orders of the paper's loop nest ((-,-), (-,+), (+,-),
// (+,+), x outermost) until a whole sweep changes nothing, at most
// max_sweeps.  Every node starts out as possibly changing; afterwards each
// sweep covers only the steps that can change a value, which gives the full
// sweeps' values, winds and sweep count.  Runs on waves 0 and 1 of the block
// (PipeSync, initialised by pipe_init and a block barrier); returns the
// number of sweeps in wave 0.
//
// With a rule that has cycle_check, a run found periodic (period p from
// sweep s on) runs only the (max_sweeps - s) mod p sweeps that decide the
// state the cap would leave, and still counts max_sweeps: the values equal
// those of the whole run to the cap.
template <bool EXTRA, typename Rule>
__device__ __forceinline__ int fsm_leader(Rule& R, int L0, int L1, int SP, int max_sweeps, PipeSync* ps) {
  Range2 P{0, L0 + L1 - 2 + (EXTRA ? 1 : 0)};
  int smax = max_sweeps;
  for (int s = 0;; s += 2) {
    if (s > 0) {
      // the follower's sweep s-1 has ended: it gives this sweep's steps
      for (int n = 0; lds_load_acq(&ps->fin) < s; ++n) {
        if (n >= kPipeSpin) {
          if ((threadIdx.x & (kWave - 1)) == 0) ps->err = 1;
          return s;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (!__builtin_amdgcn_readfirstlane(ps->ch[1])) return s;
      P.t0 = __builtin_amdgcn_readfirstlane(ps->lrng.t0);
      P.tmax = __builtin_amdgcn_readfirstlane(ps->lrng.tmax);
    }
    if (s >= smax) return max_sweeps;
    if constexpr (HasCycleCheck<Rule>::value) {
      if ((s & 3) == 0 && smax == max_sweeps) {
        const int p = __builtin_amdgcn_readfirstlane(R.cycle_check(s));
        if (p > 0) {
          smax = s + (max_sweeps - s) % p;
          lds_store_rel(&ps->smax, smax);
          if (s >= smax) return max_sweeps;
        }
      }
    }
    const bool ch = (s & 2) ? sweep_lead<1, -1, EXTRA>(R, L0, L1, SP, P, ps, s)
                            : sweep_lead<-1, -1, EXTRA>(R, L0, L1, SP, P, ps, s);
    if (!ch) return s + 1;
    if (s + 1 >= smax) return max_sweeps;
  }
}

template <bool EXTRA, typename Rule>
__device__ __forceinline__ void fsm_follower(Rule& R, int L0, int L1, int SP, int max_sweeps, PipeSync* ps) {
  const int lag = follow_lag(L1, EXTRA);
  for (int s = 1; s < max_sweeps; s += 2) {
    // the leader has begun sweep s-1 (or has ended the run before it, having
    // found a cycle) ...
    for (int n = 0; lds_load_acq(&ps->lsweep) < s - 1; ++n) {
      if (HasCycleCheck<Rule>::value && s - 1 >= lds_load_acq(&ps->smax)) return;
      if (n >= kPipeSpin) {
        if ((threadIdx.x & (kWave - 1)) == 0) ps->err = 1;
        return;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // ... and sweep s is within the run (the end is set before sweep s-1)
    if (HasCycleCheck<Rule>::value && s >= lds_load_acq(&ps->smax)) return;
    // ... and has changed a node and run far enough past this sweep's first
    // step, or has ended
    int t0 = 0, tmax = 0x7fffffff, allowed = 0;
    for (int n = 0;; ++n) {
      const int p = lds_load_acq(&ps->kp[0].y);
      const int key = __builtin_amdgcn_readfirstlane(wave_min(ps->kp[threadIdx.x & (kWave - 1)].x));  // after p
      if (p >= kPipeDone) {
        if (!__builtin_amdgcn_readfirstlane(ps->ch[0])) return;
        t0 = follow_t0(key, L1);
        tmax = __builtin_amdgcn_readfirstlane(ps->ftmax);
        allowed = 0x7fffffff;
        break;
      }
      if (key < kPipeNoKey && p >= follow_t0(key, L1) + lag) {
        t0 = follow_t0(key, L1);
        allowed = p;
        break;
      }
      if (n >= kPipeSpin) {
        if ((threadIdx.x & (kWave - 1)) == 0) ps->err = 1;
        return;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    const bool ch = (s & 2) ? sweep_follow<1, 1, EXTRA>(R, L0, L1, SP, ps, s, t0, tmax, allowed)
                            : sweep_follow<-1, 1, EXTRA>(R, L0, L1, SP, ps, s, t0, tmax, allowed);
    if (!ch) return;
  }
}

// The waves of a block that run wave_fsm2: the leader (wave 0) and the
// follower (wave kFollower).
constexpr int kFollower = 1;
__device__ __forceinline__ bool fsm_wave() {
  const int wv = (int)(threadIdx.x / kWave);
  return wv == 0 || wv == kFollower;
}

template <typename Rule>
__device__ __forceinline__ int wave_fsm2(Rule& R, int L0, int L1, int SP, int max_sweeps, PipeSync* ps) {
  const bool extra = L1 > kWave;
  if (threadIdx.x < kWave)
    return extra ? fsm_leader<true>(R, L0, L1, SP, max_sweeps, ps) : fsm_leader<false>(R, L0, L1, SP, max_sweeps, ps);
  if (extra)
    fsm_follower<true>(R, L0, L1, SP, max_sweeps, ps);
  else
    fsm_follower<false>(R, L0, L1, SP, max_sweeps, ps);
  return 0;
}

// ---------------------------------------------------------------------------
// Per-node rules.  load<SX,SY>(x) fetches the node's old value, its downwind
// neighbours, the halo values that stand in for missing upwind neighbours and
// its parameters; compute() returns the node's new value and performs the
// LDS writes.
// ---------------------------------------------------------------------------

template <typename T>
struct PreFine {
  T self, xn, yn, hx, hy, rd;
};

// Fine update (Alg. fineupdate2D with flow-direction winds; eq. FSMupdate).
// Also the coarse update of Step 1 (Alg. update2D) when Coarse = true.
template <typename T, bool Coarse, bool Halo>
struct MinRule {
  using real = T;
  using Pre = PreFine<T>;
  static constexpr bool kHalo = Halo;
  T* u;
  uint8_t* w;
  const T* rd;
  int SP;
  bool homog;  // coarse only: the homogenised solver in place of C_H
  __device__ __forceinline__ T value(int x) const { return u[x]; }
  template <int SX, int SY>
  __device__ __forceinline__ Pre load(int x) const {
    Pre p;
    p.self = u[x];
    p.xn = u[x + SX];
    p.yn = u[x + SY * SP];
    if (Halo) {
      p.hx = u[x - SX];
      p.hy = u[x - SY * SP];
    }
    p.rd = rd[x];
    return p;
  }
  template <int SX, int SY>
  __device__ __forceinline__ T compute(T xm, T xp, T ym, T yp, const Pre& p, int x, bool act,
                                      bool& ch) const {
    T a, b;
    int wx, wy;
    pick(xm, xp, a, wx);
    pick(ym, yp, b, wy);
    bool two;
    T ut = godunov2_sel(a, b, p.rd, two);
    if (Coarse && homog) ut = homog2(a, b, p.rd);
    ch = act && (ut < p.self);
    // axes that enter the wind: Alg. update2D (coarse) or Alg. fineupdate2D
    bool useX, useY;
    if (Coarse) {
      useX = (ut < b) || !(ut < a);
      useY = !(ut < b);
    } else {
      useX = two || (a < b);
      useY = two || !(a < b);
    }
    const uint8_t c = (uint8_t)((useX ? (wx & 3) : 0) | (useY ? ((wy & 3) << 2) : 0));
    const int xs = ch ? x : dummy_slot();
    u[xs] = ut;
    w[xs] = c;
    return ch ? ut : p.self;
  }
};

// fp32 subdomain boxes in packed records, at one fixed geometry (row stride
// kSPf, kCntf nodes with the halo ring) for every box of up to kMaxL nodes a
// side: a node's value and wind code in one 8-byte record (one LDS store per
// update), its r*Delta and 2 (r*Delta)^2 in another (the local solve's
// t = (rd*rd) + (rd*rd), the same bits as evaluating it there).  With the
// stride and the arrays' offsets known at compile time, every LDS access of
// a step is an immediate offset from the lane's one record address.
constexpr int kSPf = (kMaxL + 3) & ~1;
constexpr int kCntf = kSPf * (kMaxL + 2);
struct alignas(8) UWf {
  float u;
  unsigned w;
};
struct alignas(8) RTf {
  float rd, t2;
};

// Fine update of Alg. fineupdate2D (flow-direction winds; eq. FSMupdate) on
// UWf / RTf records.  The wind code is the same as MinRule's: both axes on
// the two-sided branch, otherwise the axis of the smaller neighbour (x when
// a < b), written as selects.
struct MinRuleF32 {
  using real = float;
  using Pre = PreFine<float>;
  static constexpr bool kHalo = false;
  UWf* uw;
  const RTf* rt;
  __device__ __forceinline__ float value(int x) const { return uw[x].u; }
  template <int SX, int SY>
  __device__ __forceinline__ Pre load(int x) const {
    Pre p;
    p.self = uw[x].u;
    p.xn = uw[x + SX].u;
    p.yn = uw[x + SY * kSPf].u;
    const RTf q = rt[x];
    p.rd = q.rd;
    p.hx = q.t2;  // no halo values in this rule: hx carries 2 (r Delta)^2
    return p;
  }
  template <int SX, int SY>
  __device__ __forceinline__ float compute(float xm, float xp, float ym, float yp, const Pre& p, int x, bool act,
                                          bool& ch) const {
    const bool ltx = xm < xp, lty = ym < yp;
    const float a = ltx ? xm : xp, b = lty ? ym : yp;
    const float d = a - b;
    const bool two = dabs(d) < p.rd;
    float t = p.hx;
    t = t - d * d;
    const float u2 = ((a + b) + dsqrt(t)) * 0.5f;
    const bool ab = a < b;
    const float u1 = (ab ? a : b) + p.rd;
    const float ut = two ? u2 : u1;
    ch = act && (ut < p.self);
    const unsigned cx = ltx ? 1u : 3u, cy = lty ? 4u : 12u;
    const unsigned c = two ? (cx | cy) : (ab ? cx : cy);
    // the store goes to the node's own record or, when nothing changes, to
    // the lane's dummy record: a select of two addresses, the node's being
    // the one the loads use
    UWf* dst = ch ? uw + x : uw + dummy_slot();
    *dst = UWf{ut, c};
    return ch ? ut : p.self;
  }
};

// Step 4's read-only operands of a node in one 16-byte record (fp32): one
// LDS read per step in place of four.  Used for a constant weight when the
// records fit in LDS beside the separate arrays they are filled from.
struct alignas(16) CorrPack {
  float rd, uk, ck;
  unsigned m;
};

template <typename T>
struct PreCorr {
  T self, xn, yn, hx, hy, rd, uk, ck;
  double ta, tb;
  uint8_t m;
};

// Step 4 condition mask of a node (Alg. 2Dweightedupdate): bits 0-2 say
// which values -1, 0, +1 of the x component of W~ let the weighted update
// through (all of w^k, W^k, W~ having x components <= 0, or all >= 0; all
// three values when x is not a normal axis of the node's coarse line),
// bits 3-5 the same for y, bit 6 that C^k is finite.
__device__ __forceinline__ uint8_t corr_mask(uint8_t wk, uint8_t Wk, bool nx, bool ny, bool ck_finite) {
  auto axis = [](int q, int r, bool normal) -> int {
    if (!normal) return 7;
    const bool le = q <= 0 && r <= 0, ge = q >= 0 && r >= 0;
    return (le ? 1 : 0) | ((le || ge) ? 2 : 0) | (ge ? 4 : 0);
  };
  return (uint8_t)(axis(wx_of(wk), wx_of(Wk), nx) | (axis(wy_of(wk), wy_of(Wk), ny) << 3) |
                   (ck_finite ? 64 : 0));
}

// Step 4 (Alg. 2Dweightedupdate): U = u^k + theta*(U~ - C^k) when the winds
// w^k, W^k and W~ agree along every normal axis of the node's coarse line and
// U~, C^k are finite; U = u^k otherwise.  Direct assignment, no minimum.
// Gamma nodes carry u^k = g and r*H = NaN, so they always keep g.  MODE
// selects the weight (0 constant, else theta_at).
template <typename T, int MODE, bool Packed = false>
struct CorrectRule {
  static_assert(!Packed || (sizeof(T) == 4 && MODE == 0), "packed operands: fp32, constant weight");
  using real = T;
  using Pre = PreCorr<T>;
  static constexpr bool kHalo = false;
  T* u;
  const T* uk;
  const T* ck;
  const T* rd;
  const uint8_t* mk;
  T theta;
  int SP;
  const double* ta;  // per-node weight terms (MODE != 0)
  const double* tb;
  ThetaPar q;
  bool homog;        // the homogenised coarse solver in place of C_H
  const CorrPack* pk;  // Packed: rd, uk, ck, mk in one record per node
  __device__ __forceinline__ T value(int x) const { return u[x]; }
  template <int SX, int SY>
  __device__ __forceinline__ Pre load(int x) const {
    Pre p;
    p.self = u[x];
    p.xn = u[x + SX];
    p.yn = u[x + SY * SP];
    if constexpr (Packed) {
      const CorrPack c = pk[x];
      p.rd = c.rd;
      p.uk = c.uk;
      p.ck = c.ck;
      p.m = (uint8_t)c.m;
    } else {
      p.rd = rd[x];
      p.uk = uk[x];
      p.ck = ck[x];
      p.m = mk[x];
    }
    if (MODE != 0) {
      p.ta = ta[x];
      if (MODE == 1) p.tb = tb[x];
    }
    return p;
  }
  template <int SX, int SY>
  __device__ __forceinline__ T compute(T xm, T xp, T ym, T yp, const Pre& p, int x, bool act,
                                      bool& ch) const {
    T a, b;
    int wx, wy;
    pick(xm, xp, a, wx);
    pick(ym, yp, b, wy);
    bool two;
    T ut = godunov2_sel(a, b, p.rd, two);
    if (homog) ut = homog2(a, b, p.rd);
    // W~ of Alg. update2D: U~ < b -> (Wx, 0); else U~ < a -> (0, Wy); else both
    const bool lb = ut < b, la = ut < a;
    const int tx = (!lb && la) ? 0 : wx;
    const int ty = lb ? 0 : wy;
    const unsigned m = p.m;
    const bool cond = ((m >> (tx + 1)) & 1u) && ((m >> (ty + 4)) & 1u) && (m & 64u) && dfinite(ut);
    T th = theta;
    if (MODE != 0) th = (T)theta_at<MODE>(ut, p.ck, p.ta, p.tb, (double)theta, q);
    const T corr = p.uk + th * (ut - p.ck);
    const T v = cond ? corr : p.uk;
    ch = act && (v != p.self);
    u[ch ? x : dummy_slot()] = v;
    return v;
  }
};

// Step 4 in fp32 with a constant weight: one 32-byte record per node at the
// fixed box geometry of the subdomain records (kSPf, kCntf): the value U and
// the condition mask, then r*H, 2 (r*H)^2, u^k and C^k.  Every LDS access of
// a step is an immediate offset from the lane's record address.
struct alignas(32) CorrRecF32 {
  float u;
  unsigned m;
  float pad0, pad1;
  float rd, t2, uk, ck;
};
__host__ __device__ __forceinline__ size_t corr_f32_lds_bytes() {
  return (size_t)(kCntf + 2 * kGuard) * sizeof(CorrRecF32);
}

struct CorrectRuleF32 {
  using real = float;
  using Pre = PreCorr<float>;
  static constexpr bool kHalo = false;
  CorrRecF32* rec;
  float theta;
  bool homog;
  __device__ __forceinline__ float value(int x) const { return rec[x].u; }
  template <int SX, int SY>
  __device__ __forceinline__ Pre load(int x) const {
    Pre p;
    p.self = rec[x].u;
    p.m = (uint8_t)rec[x].m;
    p.xn = rec[x + SX].u;
    p.yn = rec[x + SY * kSPf].u;
    const float4 q = *reinterpret_cast<const float4*>(&rec[x].rd);
    p.rd = q.x;
    p.hx = q.y;  // 2 (r H)^2
    p.uk = q.z;
    p.ck = q.w;
    return p;
  }
  template <int SX, int SY>
  __device__ __forceinline__ float compute(float xm, float xp, float ym, float yp, const Pre& p, int x, bool act,
                                          bool& ch) const {
    const bool ltx = xm < xp, lty = ym < yp;
    const float a = ltx ? xm : xp, b = lty ? ym : yp;
    const int wx = ltx ? 1 : -1, wy = lty ? 1 : -1;
    const float d = a - b;
    const bool two = dabs(d) < p.rd && !homog;
    float t = p.hx;
    t = t - d * d;
    const float u2 = ((a + b) + dsqrt(t)) * 0.5f;
    const float u1 = ((a < b) ? a : b) + p.rd;
    const float ut = two ? u2 : u1;
    // W~ of Alg. update2D and the condition of CorrectRule
    const bool lb = ut < b, la = ut < a;
    const int tx = (!lb && la) ? 0 : wx;
    const int ty = lb ? 0 : wy;
    const unsigned m = p.m;
    const bool cond = ((m >> (tx + 1)) & 1u) && ((m >> (ty + 4)) & 1u) && (m & 64u) && dfinite(ut);
    const float corr = p.uk + theta * (ut - p.ck);
    const float v = cond ? corr : p.uk;
    ch = act && (v != p.self);
    float* dst = ch ? &rec[x].u : &rec[dummy_slot()].u;
    *dst = v;
    return v;
  }
  // The values after s-4 and s-8 sweeps are kept in pad0 and pad1 of every
  // record (bit patterns; every record of the box, its ring and the unused
  // part of the fixed geometry, which never change).  Kept from s = 8 on.
  __device__ int cycle_check(int s) const {
    if (s < 8) return 0;
    const int lane = threadIdx.x & (kWave - 1);
    bool d4 = false, d8 = false;
    for (int x = lane; x < kCntf; x += kWave) {
      const uint4 q = *reinterpret_cast<const uint4*>(&rec[x]);  // u, m, pad0, pad1
      d4 = d4 || q.x != q.z;
      d8 = d8 || q.x != q.w;
      *reinterpret_cast<uint2*>(&rec[x].pad0) = make_uint2(q.x, q.z);
    }
    if (s >= 12 && !__any(d4)) return 4;
    if (s >= 16 && !__any(d8)) return 8;
    return 0;
  }
};
template <>
struct HasCycleCheck<CorrectRuleF32> {
  static constexpr bool value = true;
};

// ---------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------

template <typename T>
struct DD2 {
  int n0, n1;        // nodes per axis
  int S, M;          // subdomain side, coarse spacing (fine cells)
  int P0, P1;        // subdomains per axis
  int NI, NJ;        // coarse cells per axis
  T hT, HT, theta;
  int max_fine_sweeps, max_coarse_sweeps;
  const T* r;
  const T* gfull;      // Gamma value per node, NaN if not a Gamma node
  const uint32_t* gbits;  // Gamma flag per node: bit X % 32 of word X / 32
  const int64_t* gidx; // sorted Gamma indices
  const T* gval;
  int64_t ng;
  T* U;               // coarse values (full grid, skeleton used)
  uint8_t* W;
  T* Un;
  uint8_t* Wn;
  T* uk;
  uint8_t* wk;
  T* u_out;
  T* edge_u;          // [tile][4][S+1]
  uint8_t* edge_w;
  T* cwork;           // causal sweep scratch (full grid)
  uint8_t* cflag;     // causal sweep scratch (full grid)
  T* ncx;             // causal sweep: per corner, its x / y successor's value
  T* ncy;
  T* cU;              // causal sweep: per corner, U, W and the Gamma flag,
  uint8_t* cW;        // gathered by the segment kernel so that the corner
  uint8_t* cG;        // kernel's loads are contiguous
  T* hseg_p;          // NI*(NJ+1) segment end values
  uint8_t* hseg_l;
  T* vseg_p;          // (NI+1)*NJ
  uint8_t* vseg_l;
  unsigned long long* near_key;  // Step 1 nearest-Gamma keys (full grid)
  long long* near_win;
  unsigned long long* counters;  // [0] fine updates, [1] coarse updates, [2] residual bits, [3] nonzero if a two-wave sweep wait gave up
  // or NULL: the leading waves' anti-diagonal steps and the clock64 ticks
  // spent in them, summed over the boxes: [0], [1] Step 3, [2], [3] Step 4
  unsigned long long* sweep_prof;
  // Step 4 weight (ThetaPar, theta_at): mode, parameters, u_ref or theta per
  // node, and the history u^{k-1}, C^{k-1}, C^{k-2} (NULL until it exists);
  // this iteration's C^k goes to ck_out
  int theta_mode;
  // Step 4's weight terms in global memory (2 x tglob_stride doubles per
  // lattice) when they do not fit in LDS; NULL: in LDS
  double* tglob = nullptr;
  int tglob_stride = 0;
  ThetaPar tq;
  const T* tref;
  const T* ukm1;
  const T* ckm1;
  const T* ckm2;
  T* ck_out;
  // coarse solver of Steps 1 and 4: 0 = C_H (Sec. 3.2), 1 = the homogenised
  // solver of the squares medium (Sec. 5.3)
  int coarse_homog;
  // Step 4 reads its operands from CorrPack records (fp32, constant weight,
  // when they fit in LDS)
  int corr_packed;
  // this DD iteration's residual max |U^{k+1} - U^k| (double bits; k_tile
  // zeroes it, the causal sweep of U^{k+1} raises it) ...
  unsigned long long* res_out;
  // ... and the previous iteration's, or NULL: when that one met the
  // stopping rule (< tol or 0) every kernel of this iteration returns at
  // once, so iterations can be launched ahead of the host's check
  const unsigned long long* res_prev;
  double tol;
};

template <typename T>
__device__ __forceinline__ bool dd_stopped(const DD2<T>& A) {
  if (!A.res_prev) return false;
  const double r = __longlong_as_double((long long)*A.res_prev);
  return r < A.tol || r == 0.0;
}

__device__ __forceinline__ bool is_iface(int c, int S, int n) { return (c % S == 0) && c > 0 && c < n - 1; }

// order-preserving map of a real onto unsigned 64-bit keys
__device__ __forceinline__ unsigned long long okey(double v) {
  unsigned long long b = __double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ unsigned long long okey(float v) { return okey((double)v); }
__device__ __forceinline__ double okey_dec(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(b);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_gamma_bits(uint32_t* bits, const int64_t* gidx, int64_t ng) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ng) atomicOr(&bits[gidx[i] >> 5], 1u << (gidx[i] & 31));
}
// the Gamma value of node X (NaN if it is not a Gamma node), read from the
// full-grid values only where the bit mask has the node
template <typename T>
__device__ __forceinline__ T gamma_at(const DD2<T>& A, int X) {
  T g = T(__builtin_nan(""));
  if ((A.gbits[X >> 5] >> (X & 31)) & 1u) g = A.gfull[X];
  return g;
}
template <typename T>
__global__ void k_scatter_gamma(T* gfull, const int64_t* gidx, const T* gval, int64_t ng) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < ng) gfull[gidx[i]] = gval[i];
}

// r > 0 and finite everywhere (bit 0), and r >= rmin (bit 3: the input
// domain of the fp32 square root); Gamma sorted, in range (bit 1), finite
// (bit 2).  bad[0] != 0 on failure.
template <typename T>
__global__ void k_validate(const T* r, int64_t N, const int64_t* gidx, const T* gval, int64_t ng,
                           double rmin, unsigned int* bad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) {
    T v = r[i];
    if (!(v > T(0)) || !dfinite(v)) atomicOr(bad, 1u);
    else if ((double)v < rmin) atomicOr(bad, 8u);
  }
  if (i < ng) {
    int64_t g = gidx[i];
    if (g < 0 || g >= N) atomicOr(bad, 2u);
    if (i > 0 && !(gidx[i - 1] < g)) atomicOr(bad, 2u);
    if (!dfinite(gval[i])) atomicOr(bad, 4u);
  }
}

// Step 1 initialisation near Gamma: every coarse node X within max-norm
// distance < H (M cells) of a Gamma node x_g gets the candidate
// g + r_X * (h * sqrt(|X - x_g|^2 / h^2)); the smallest wins, ties to the
// first Gamma node.  Pass A keeps the smallest value, pass B its first index.
template <typename T>
__device__ __forceinline__ bool near_candidate(const DD2<T>& A, int64_t gi, int off, int& X, T& v) {
  const int W2 = 2 * A.M - 1;
  const int dx = off % W2 - (A.M - 1), dy = off / W2 - (A.M - 1);
  const int64_t g = A.gidx[gi];
  const int gxi = (int)(g % A.n0), gyi = (int)(g / A.n0);
  const int xi = gxi + dx, yi = gyi + dy;
  if (xi < 0 || xi >= A.n0 || yi < 0 || yi >= A.n1) return false;
  if (xi % A.M != 0 && yi % A.M != 0) return false;  // not a coarse node
  X = xi + A.n0 * yi;
  const int d2 = dx * dx + dy * dy;
  T sq = dsqrt((T)d2);
  T dist = A.hT * sq;
  v = A.gval[gi] + A.r[X] * dist;
  return true;
}

template <typename T>
__device__ __forceinline__ void near_a_body(const DD2<T>& A, int bx) {
  const int W2 = 2 * A.M - 1;
  int64_t t = bx * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A.ng * W2 * W2) return;
  int X;
  T v;
  if (near_candidate(A, t / (W2 * W2), (int)(t % (W2 * W2)), X, v)) atomicMin(&A.near_key[X], okey(v));
}
template <typename T>
__global__ void k_near_a(DD2<T> A) { near_a_body(A, (int)blockIdx.x); }
template <typename T>
__global__ void k_near_a_b(const DD2<T>* descs, const int2* work) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  near_a_body(A, w.y);
}


template <typename T>
__device__ __forceinline__ void near_b_body(const DD2<T>& A, int bx) {
  const int W2 = 2 * A.M - 1;
  int64_t t = bx * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A.ng * W2 * W2) return;
  int X;
  T v;
  const int64_t gi = t / (W2 * W2);
  if (near_candidate(A, gi, (int)(t % (W2 * W2)), X, v))
    if (okey(v) == A.near_key[X]) atomicMin(&A.near_win[X], (long long)gi);
}
template <typename T>
__global__ void k_near_b(DD2<T> A) { near_b_body(A, (int)blockIdx.x); }
template <typename T>
__global__ void k_near_b_b(const DD2<T>* descs, const int2* work) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  near_b_body(A, w.y);
}


// ---------------------------------------------------------------------------
// LDS boxes
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ int halo_stride(int L0) { return (L0 + 3) & ~1; }
__host__ __device__ __forceinline__ int halo_count(int L0, int L1) { return halo_stride(L0) * (L1 + 2); }
// LDS bytes of a box with nreal real arrays and nbyte byte arrays (guards included)
__host__ __device__ __forceinline__ size_t box_bytes(int cnt, int nreal, int nbyte, size_t szT) {
  return (size_t)(cnt + 2 * kGuard) * (nreal * szT + nbyte);
}
// next array of n elements (plus guards) from the LDS cursor
template <typename U>
__device__ __forceinline__ U* carve(unsigned char*& cur, int n) {
  U* a = reinterpret_cast<U*>(cur) + kGuard;
  cur += (size_t)(n + 2 * kGuard) * sizeof(U);
  return a;
}

// ---------------------------------------------------------------------------
// lattices (Steps 1 and 4)
// ---------------------------------------------------------------------------

// lattice q: 0 -> offset (0,0); 1..M-1 -> (q,0); M..2M-2 -> (0, q-M+1)
__device__ __forceinline__ void lattice_offset(int q, int M, int& o0, int& o1) {
  if (q == 0) { o0 = 0; o1 = 0; }
  else if (q < M) { o0 = q; o1 = 0; }
  else { o0 = 0; o1 = q - M + 1; }
}

template <typename T>
__device__ __forceinline__ void lattice_init_body(const DD2<T>& A, int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  int o0, o1;
  lattice_offset(bx, A.M, o0, o1);
  const int L0 = (A.n0 - 1 - o0) / A.M + 1, L1 = (A.n1 - 1 - o1) / A.M + 1;
  const int SP = halo_stride(L0);
  const int cnt = halo_count(L0, L1);
  unsigned char* lc = smem;
  T* u = carve<T>(lc, cnt);
  T* rd = carve<T>(lc, cnt);
  uint8_t* w = carve<uint8_t>(lc, cnt);
  const T nan = T(__builtin_nan(""));
  for (int k = threadIdx.x; k < cnt; k += kBlock) { u[k] = pinf<T>(); rd[k] = nan; w[k] = 0; }
  __syncthreads();
  int nfree = 0;
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int xi = o0 + p0 * A.M, yi = o1 + p1 * A.M;
    const int X = xi + A.n0 * yi;
    const int x = (p1 + 1) * SP + (p0 + 1);
    const T g = gamma_at(A, X);
    if (!disnan(g)) {
      u[x] = g; w[x] = 0; rd[x] = nan;
    } else if (A.near_win[X] != 0x7fffffffffffffffll) {
      u[x] = (T)okey_dec(A.near_key[X]);
      const int64_t gg = A.gidx[A.near_win[X]];
      const int dx = xi - (int)(gg % A.n0), dy = yi - (int)(gg / A.n0);
      w[x] = wenc((dx > 0) - (dx < 0), (dy > 0) - (dy < 0));
      rd[x] = nan;
    } else {
      u[x] = pinf<T>(); w[x] = 0; rd[x] = A.r[X] * A.HT;
      ++nfree;
    }
  }
  __syncthreads();
  __shared__ int sh_ns, sh_free;
  __shared__ PipeSync ps;
  if (threadIdx.x == 0) {
    sh_free = 0;
    pipe_init(ps);
  }
  __syncthreads();
  if (fsm_wave()) {
    MinRule<T, true, false> R{u, w, rd, SP, A.coarse_homog != 0};
    const int ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
    if (threadIdx.x == 0) sh_ns = ns;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int X = (o0 + p0 * A.M) + A.n0 * (o1 + p1 * A.M);
    const int x = (p1 + 1) * SP + (p0 + 1);
    A.U[X] = u[x];
    A.W[X] = w[x];
  }
  for (int o = 32; o > 0; o >>= 1) nfree += __shfl_xor(nfree, o);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[1], (unsigned long long)sh_free * (unsigned long long)sh_ns);
  if (threadIdx.x == 0 && ps.err) atomicOr(&A.counters[3], 1ull);  // a two-wave wait gave up
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lattice_init(DD2<T> A) { lattice_init_body(A, (int)blockIdx.x); }
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lattice_init_b(const DD2<T>* descs, const int2* work) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  lattice_init_body(A, w.y);
}


// Step 4 on one lattice, fp32 with a constant weight (CorrRecF32 records);
// the same steps as lattice_correct_body
__device__ __forceinline__ void lattice_correct_f32(const DD2<float>& A, int bx) {
  extern __shared__ __align__(32) unsigned char smem[];
  int o0, o1;
  lattice_offset(bx, A.M, o0, o1);
  const int L0 = (A.n0 - 1 - o0) / A.M + 1, L1 = (A.n1 - 1 - o1) / A.M + 1;
  unsigned char* lc = smem;
  CorrRecF32* rec = carve<CorrRecF32>(lc, kCntf);
  const float inf = pinf<float>();
  const float nan = __builtin_nanf("");
  const bool nx = o0 == 0, ny = o1 == 0;  // normal axes shared by the whole lattice
  for (int k = threadIdx.x; k < kCntf; k += kBlock) rec[k] = CorrRecF32{inf, 0u, 0.f, 0.f, nan, nan, inf, inf};
  __syncthreads();
  // every global input of a node in one pass: U^k (into u, for C^k first),
  // u^k (g at Gamma nodes), r*H and 2 (r*H)^2, w^k | W^k << 4 in the mask
  // and the Gamma flag in C^k's slot until the C^k pass replaces them
  int nfree = 0;
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int X = (o0 + p0 * A.M) + A.n0 * (o1 + p1 * A.M);
    const int x = (p1 + 1) * kSPf + (p0 + 1);
    const float Uk = A.U[X];
    const float g = gamma_at(A, X);
    const float ukX = A.uk[X];
    const float r = A.r[X];
    const uint8_t wkX = A.wk[X], WkX = A.W[X];
    const bool gam = !disnan(g);
    const float rd = r * A.HT;
    float t2 = rd * rd;
    t2 = t2 + t2;
    rec[x] = CorrRecF32{Uk, (unsigned)((wkX & 15) | ((WkX & 15) << 4)), 0.f, 0.f, rd, t2, gam ? g : ukX,
                        gam ? 1.f : 0.f};
    if (!gam) ++nfree;
  }
  __syncthreads();
  // C^k = C_H(nbrs^H(U^k)) (or the homogenised solver) once per node
  // (Jacobi), and the condition masks; U^k stays in u until all are done
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int x = (p1 + 1) * kSPf + (p0 + 1);
    const float xm = rec[x - 1].u, xp = rec[x + 1].u, ym = rec[x - kSPf].u, yp = rec[x + kSPf].u;
    const float a = xm < xp ? xm : xp;
    const float b = ym < yp ? ym : yp;
    bool two;
    const float c = A.coarse_homog ? homog2(a, b, rec[x].rd) : godunov2(a, b, rec[x].rd, two);
    const unsigned st = rec[x].m;
    const bool gam = rec[x].ck != 0.f;
    rec[x].ck = c;
    rec[x].m = corr_mask((uint8_t)(st & 15), (uint8_t)(st >> 4), nx, ny, dfinite(c)) | (gam ? 128u : 0u);
  }
  __syncthreads();
  // start of Step 4: U = +inf, Gamma nodes at g (they keep it: r*H = NaN)
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int x = (p1 + 1) * kSPf + (p0 + 1);
    if (rec[x].m & 128u) {
      rec[x].u = rec[x].uk;  // g
      rec[x].rd = nan;
      rec[x].t2 = nan;
    } else {
      rec[x].u = inf;
    }
  }
  __syncthreads();
  __shared__ int sh_ns, sh_free;
  __shared__ PipeSync ps;
  if (threadIdx.x == 0) {
    sh_free = 0;
    pipe_init(ps);
  }
  __syncthreads();
  if (fsm_wave()) {
    CorrectRuleF32 R{rec, A.theta, A.coarse_homog != 0};
    const int ns = wave_fsm2(R, L0, L1, kSPf, A.max_coarse_sweeps, &ps);
    if (threadIdx.x == 0) sh_ns = ns;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int X = (o0 + p0 * A.M) + A.n0 * (o1 + p1 * A.M);
    const int x = (p1 + 1) * kSPf + (p0 + 1);
    A.Un[X] = rec[x].u;
    A.Wn[X] = (rec[x].m & 128u) ? (uint8_t)0 : A.wk[X];
  }
  for (int o = 32; o > 0; o >>= 1) nfree += __shfl_xor(nfree, o);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[1], (unsigned long long)sh_free * (unsigned long long)sh_ns);
  if (threadIdx.x == 0 && A.sweep_prof) {
    atomicAdd(&A.sweep_prof[2], (unsigned long long)ps.lsteps);
    atomicAdd(&A.sweep_prof[3], (unsigned long long)ps.lcyc);
  }
  if (threadIdx.x == 0 && ps.err) atomicOr(&A.counters[3], 1ull);  // a two-wave wait gave up
}

// TG: the weight terms (varying theta) in global memory, A.tglob, where
// they do not fit in LDS beside the lattice (fp64 lattices of 65 x 65)
template <typename T, bool TG>
__device__ __forceinline__ void lattice_correct_body_t(const DD2<T>& A, int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  if constexpr (sizeof(T) == 4 && !TG) {
    if (A.corr_packed) {
      lattice_correct_f32(A, bx);
      return;
    }
  }
  int o0, o1;
  lattice_offset(bx, A.M, o0, o1);
  const int L0 = (A.n0 - 1 - o0) / A.M + 1, L1 = (A.n1 - 1 - o1) / A.M + 1;
  const int SP = halo_stride(L0);
  const int cnt = halo_count(L0, L1);
  unsigned char* lc = smem;
  // the packed records, then the weight terms, come first (16- and 8-byte
  // alignment)
  CorrPack* pk = (sizeof(T) == 4 && A.corr_packed) ? carve<CorrPack>(lc, cnt) : nullptr;
  double* ta = nullptr;
  double* tb = nullptr;
  if constexpr (TG) {
    ta = A.tglob + (size_t)bx * 2 * A.tglob_stride;
    tb = ta + A.tglob_stride;
  } else if (A.theta_mode != 0) {
    ta = carve<double>(lc, cnt);
    tb = carve<double>(lc, cnt);
  }
  T* u = carve<T>(lc, cnt);
  T* uk = carve<T>(lc, cnt);
  T* ck = carve<T>(lc, cnt);
  T* rd = carve<T>(lc, cnt);
  uint8_t* mk = carve<uint8_t>(lc, cnt);
  const T inf = pinf<T>();
  const T nan = T(__builtin_nan(""));
  const bool nx = o0 == 0, ny = o1 == 0;  // normal axes shared by the whole lattice
  for (int k = threadIdx.x; k < cnt; k += kBlock) { u[k] = inf; rd[k] = nan; uk[k] = inf; ck[k] = inf; mk[k] = 0; }
  __syncthreads();
  // every global input of a node in one pass: U^k, u^k (g at Gamma nodes),
  // r*H, w^k | W^k << 4 in the mask byte and the Gamma flag in the C^k
  // array until the C^k pass replaces them (then the flag is bit 7 of the
  // mask, which the condition bits 0-6 leave free)
  int nfree = 0;
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int xi = o0 + p0 * A.M, yi = o1 + p1 * A.M;
    const int X = xi + A.n0 * yi;
    const int x = (p1 + 1) * SP + (p0 + 1);
    const T Uk = A.U[X];
    const T g = gamma_at(A, X);
    const T ukX = A.uk[X];
    const T r = A.r[X];
    const uint8_t wkX = A.wk[X], WkX = A.W[X];
    const bool gam = !disnan(g);
    u[x] = Uk;  // U^k, used for C^k first
    uk[x] = gam ? g : ukX;
    rd[x] = r * A.HT;
    mk[x] = (uint8_t)((wkX & 15) | ((WkX & 15) << 4));
    ck[x] = gam ? T(1) : T(0);
    if (!gam) ++nfree;
  }
  __syncthreads();
  // C^k = C_H(nbrs^H(U^k)) (or the homogenised solver) once per node
  // (Jacobi), and the condition masks
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int x = (p1 + 1) * SP + (p0 + 1);
    const int X = (o0 + p0 * A.M) + A.n0 * (o1 + p1 * A.M);
    const T xm = u[x - 1], xp = u[x + 1], ym = u[x - SP], yp = u[x + SP];
    const T a = xm < xp ? xm : xp;
    const T b = ym < yp ? ym : yp;
    bool two;
    const T c = A.coarse_homog ? homog2(a, b, rd[x]) : godunov2(a, b, rd[x], two);
    const unsigned st = mk[x];
    const bool gam = ck[x] != T(0);
    ck[x] = c;
    mk[x] = (uint8_t)(corr_mask((uint8_t)(st & 15), (uint8_t)(st >> 4), nx, ny, dfinite(c)) | (gam ? 128 : 0));
    if (A.theta_mode == 1) {
      // u^k - u^{k-1} (NaN when it cannot be used) and w1 d1 + w2 d2 with
      // d1 = C^k - C^{k-1}, d2 = C^{k-1} - C^{k-2}
      double num = __builtin_nan(""), hs = 0.0;
      if (A.ukm1 && A.ckm1 && A.ckm2) {
        num = (double)uk[x] - (double)A.ukm1[X];
        const double d1 = (double)c - (double)A.ckm1[X];
        const double d2 = (double)A.ckm1[X] - (double)A.ckm2[X];
        hs = A.tq.w1 * d1 + A.tq.w2 * d2;
        if (!finite_d(num) || !finite_d(hs)) num = __builtin_nan("");
      }
      ta[x] = num;
      tb[x] = hs;
      A.ck_out[X] = c;
    } else if (A.theta_mode == 2) {
      ta[x] = (double)A.tref[X] - (double)uk[x];
    } else if (A.theta_mode == 3) {
      ta[x] = (double)A.tref[X];
    }
  }
  __syncthreads();
  // start of Step 4: U = +inf, Gamma nodes at g (they keep it: r*H = NaN)
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int x = (p1 + 1) * SP + (p0 + 1);
    if (mk[x] & 128) {
      u[x] = uk[x];  // g
      rd[x] = nan;
    } else {
      u[x] = inf;
    }
  }
  __syncthreads();
  if (pk) {
    for (int k = threadIdx.x; k < cnt; k += kBlock)
      pk[k] = CorrPack{(float)rd[k], (float)uk[k], (float)ck[k], (unsigned)mk[k]};
    __syncthreads();
  }
  __shared__ int sh_ns, sh_free;
  __shared__ PipeSync ps;
  if (threadIdx.x == 0) {
    sh_free = 0;
    pipe_init(ps);
  }
  __syncthreads();
  if (fsm_wave()) {
    int ns;
    switch (TG ? (A.theta_mode == 0 ? 1 : A.theta_mode) : A.theta_mode) {  // TG: theta varies
      case 0: {
        if constexpr (sizeof(T) == 4) {
          if (pk) {
            CorrectRule<T, 0, true> R{u, uk, ck, rd, mk, A.theta, SP, ta, tb, A.tq, A.coarse_homog != 0, pk};
            ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
            break;
          }
        }
        CorrectRule<T, 0> R{u, uk, ck, rd, mk, A.theta, SP, ta, tb, A.tq, A.coarse_homog != 0, pk};
        ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
        break;
      }
      case 1: {
        CorrectRule<T, 1> R{u, uk, ck, rd, mk, A.theta, SP, ta, tb, A.tq, A.coarse_homog != 0, pk};
        ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
        break;
      }
      case 2: {
        CorrectRule<T, 2> R{u, uk, ck, rd, mk, A.theta, SP, ta, tb, A.tq, A.coarse_homog != 0, pk};
        ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
        break;
      }
      default: {
        CorrectRule<T, 3> R{u, uk, ck, rd, mk, A.theta, SP, ta, tb, A.tq, A.coarse_homog != 0, pk};
        ns = wave_fsm2(R, L0, L1, SP, A.max_coarse_sweeps, &ps);
        break;
      }
    }
    if (threadIdx.x == 0) sh_ns = ns;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int p0 = k % L0, p1 = k / L0;
    const int X = (o0 + p0 * A.M) + A.n0 * (o1 + p1 * A.M);
    const int x = (p1 + 1) * SP + (p0 + 1);
    A.Un[X] = u[x];
    A.Wn[X] = (mk[x] & 128) ? (uint8_t)0 : A.wk[X];
  }
  for (int o = 32; o > 0; o >>= 1) nfree += __shfl_xor(nfree, o);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[1], (unsigned long long)sh_free * (unsigned long long)sh_ns);
  if (threadIdx.x == 0 && A.sweep_prof) {
    atomicAdd(&A.sweep_prof[2], (unsigned long long)ps.lsteps);
    atomicAdd(&A.sweep_prof[3], (unsigned long long)ps.lcyc);
  }
  if (threadIdx.x == 0 && ps.err) atomicOr(&A.counters[3], 1ull);  // a two-wave wait gave up
}
template <typename T>
__device__ __forceinline__ void lattice_correct_body(const DD2<T>& A, int bx) {
  if (dd_stopped(A)) return;
  if (A.tglob)
    lattice_correct_body_t<T, true>(A, bx);
  else
    lattice_correct_body_t<T, false>(A, bx);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lattice_correct(DD2<T> A) { lattice_correct_body(A, (int)blockIdx.x); }
// Batched launches over a work table of (problem, box) items: next == NULL,
// one block per item; else a resident grid whose blocks take the items in
// table order from the counter *next (zero at launch) until nwork.  Each
// item is computed the same either way.
template <typename T, typename Body>
__device__ __forceinline__ void batch_items(const DD2<T>* descs, const int2* work, int nwork, int* next, Body body) {
  if (!next) {
    const int2 w = work[blockIdx.x];
    body(descs[w.x], w.y);
    return;
  }
  __shared__ int sh_item;
  for (;;) {
    if (threadIdx.x == 0) sh_item = atomicAdd(next, 1);
    __syncthreads();
    const int i = sh_item;
    __syncthreads();
    if (i >= nwork) return;
    const int2 w = work[i];
    body(descs[w.x], w.y);
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lattice_correct_b(const DD2<T>* descs, const int2* work, int nwork,
                                                              int* next) {
  batch_items(descs, work, nwork, next, [](const DD2<T>& A, int bx) { lattice_correct_body(A, bx); });
}


// ---------------------------------------------------------------------------
// Steps 2 and 3: one wave per subdomain
// ---------------------------------------------------------------------------

// LDS bytes of the subdomain kernel for boxes of L nodes a side
__host__ __device__ __forceinline__ size_t tile_lds_bytes(int L, size_t szT) {
  return szT == 4 ? 2 * (size_t)(kCntf + 2 * kGuard) * 8 : box_bytes(halo_count(L, L), 2, 1, szT);
}

// Steps 2 and 3 on one subdomain, fp32: the packed records (MinRuleF32)
__device__ __forceinline__ void tile_body_f32(const DD2<float>& A, int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int I = bx % A.P0, J = bx / A.P0;
  const int L = A.S + 1;
  unsigned char* lc = smem;
  UWf* uw = carve<UWf>(lc, kCntf);
  RTf* rt = carve<RTf>(lc, kCntf);
  const float nan = __builtin_nanf("");
  const float inf = pinf<float>();
  for (int k = threadIdx.x; k < kCntf; k += kBlock) {
    uw[k] = UWf{inf, 0u};
    rt[k] = RTf{nan, nan};
  }
  __syncthreads();
  const int bi = I * A.S, bj = J * A.S;
  int nfree = 0;
  for (int k = threadIdx.x; k < L * L; k += kBlock) {
    const int li = k % L, lj = k / L;
    const int xi = bi + li, yi = bj + lj;
    const int X = xi + A.n0 * yi;
    const int x = (lj + 1) * kSPf + (li + 1);
    const bool bxi = (li == 0 || li == A.S) && is_iface(xi, A.S, A.n0);
    const bool byi = (lj == 0 || lj == A.S) && is_iface(yi, A.S, A.n1);
    const float g = gamma_at(A, X);
    const float r = A.r[X];
    uint8_t Wc = 0;
    float Uc = inf;
    if (bxi || byi) {
      Wc = A.W[X];
      Uc = A.U[X];
    }
    if (!disnan(g)) {
      uw[x] = UWf{g, 0u};
      continue;
    }
    ++nfree;
    const float rd = r * A.hT;
    float t2 = rd * rd;
    t2 = t2 + t2;
    rt[x] = RTf{rd, t2};
    // Step 2 (see tile_body)
    bool inflow = false;
    if (bxi && ((li == 0 && wx_of(Wc) > 0) || (li == A.S && wx_of(Wc) < 0))) inflow = true;
    if (byi && ((lj == 0 && wy_of(Wc) > 0) || (lj == A.S && wy_of(Wc) < 0))) inflow = true;
    uw[x] = inflow ? UWf{Uc, (unsigned)Wc} : UWf{inf, 0u};
  }
  __syncthreads();
  __shared__ int sh_ns, sh_free;
  __shared__ PipeSync ps;
  if (threadIdx.x == 0) {
    sh_free = 0;
    pipe_init(ps);
  }
  __syncthreads();
  if (fsm_wave()) {
    MinRuleF32 R{uw, rt};
    const int ns = wave_fsm2(R, L, L, kSPf, A.max_fine_sweeps, &ps);
    if (threadIdx.x == 0) sh_ns = ns;
  }
  __syncthreads();
  const int tile = bx;
  for (int k = threadIdx.x; k < L * L; k += kBlock) {
    const int li = k % L, lj = k / L;
    const int xi = bi + li, yi = bj + lj;
    const int X = xi + A.n0 * yi;
    const int x = (lj + 1) * kSPf + (li + 1);
    const UWf q = uw[x];
    const float v = q.u;
    const uint8_t c = (uint8_t)q.w;
    const bool ifx = (li == 0 || li == A.S) && is_iface(xi, A.S, A.n0);
    const bool ify = (lj == 0 || lj == A.S) && is_iface(yi, A.S, A.n1);
    if (!ifx && !ify) {
      A.u_out[X] = v;
      if (xi % A.M == 0 || yi % A.M == 0) {
        A.uk[X] = v;
        A.wk[X] = c;
      }
    }
    if (li == 0) { A.edge_u[(tile * 4 + 0) * L + lj] = v; A.edge_w[(tile * 4 + 0) * L + lj] = c; }
    if (li == A.S) { A.edge_u[(tile * 4 + 1) * L + lj] = v; A.edge_w[(tile * 4 + 1) * L + lj] = c; }
    if (lj == 0) { A.edge_u[(tile * 4 + 2) * L + li] = v; A.edge_w[(tile * 4 + 2) * L + li] = c; }
    if (lj == A.S) { A.edge_u[(tile * 4 + 3) * L + li] = v; A.edge_w[(tile * 4 + 3) * L + li] = c; }
  }
  for (int o = 32; o > 0; o >>= 1) nfree += __shfl_xor(nfree, o);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[0], (unsigned long long)sh_free * (unsigned long long)sh_ns);
  if (threadIdx.x == 0 && A.sweep_prof) {
    atomicAdd(&A.sweep_prof[0], (unsigned long long)ps.lsteps);
    atomicAdd(&A.sweep_prof[1], (unsigned long long)ps.lcyc);
  }
  if (threadIdx.x == 0 && ps.err) atomicOr(&A.counters[3], 1ull);  // a two-wave wait gave up
}

template <typename T>
__device__ __forceinline__ void tile_body(const DD2<T>& A, int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  // this iteration's residual (taken by the causal sweep) starts at 0, also
  // when the iteration does not run
  if (bx == 0 && threadIdx.x == 0) *A.res_out = 0ull;
  if (dd_stopped(A)) return;
  if constexpr (sizeof(T) == 4) {
    tile_body_f32(A, bx);
    return;
  }
  const int I = bx % A.P0, J = bx / A.P0;
  const int L = A.S + 1;
  const int SP = halo_stride(L);
  const int cnt = halo_count(L, L);
  unsigned char* lc = smem;
  T* u = carve<T>(lc, cnt);
  T* rd = carve<T>(lc, cnt);
  uint8_t* w = carve<uint8_t>(lc, cnt);
  const T nan = T(__builtin_nan(""));
  for (int k = threadIdx.x; k < cnt; k += kBlock) { u[k] = pinf<T>(); rd[k] = nan; w[k] = 0; }
  __syncthreads();
  const int bi = I * A.S, bj = J * A.S;
  int nfree = 0;
  for (int k = threadIdx.x; k < L * L; k += kBlock) {
    const int li = k % L, lj = k / L;
    const int xi = bi + li, yi = bj + lj;
    const int X = xi + A.n0 * yi;
    const int x = (lj + 1) * SP + (li + 1);
    // all loads of the node first (independent), then the decisions
    const bool bx = (li == 0 || li == A.S) && is_iface(xi, A.S, A.n0);
    const bool by = (lj == 0 || lj == A.S) && is_iface(yi, A.S, A.n1);
    const T g = gamma_at(A, X);
    const T r = A.r[X];
    uint8_t Wc = 0;
    T Uc = pinf<T>();
    if (bx || by) {
      Wc = A.W[X];
      Uc = A.U[X];
    }
    if (!disnan(g)) {
      u[x] = g; w[x] = 0; rd[x] = nan;
      continue;
    }
    ++nfree;
    rd[x] = r * A.hT;
    // Step 2: a subdomain-boundary node on an interface is inflow if the
    // coarse wind points into the subdomain; it starts at U with wind W and,
    // like every non-Gamma node, still takes the FSM minimum.
    bool inflow = false;
    if (bx && ((li == 0 && wx_of(Wc) > 0) || (li == A.S && wx_of(Wc) < 0))) inflow = true;
    if (by && ((lj == 0 && wy_of(Wc) > 0) || (lj == A.S && wy_of(Wc) < 0))) inflow = true;
    if (inflow) {
      u[x] = Uc;
      w[x] = Wc;
    } else {
      u[x] = pinf<T>();
      w[x] = 0;
    }
  }
  __syncthreads();
  __shared__ int sh_ns, sh_free;
  __shared__ PipeSync ps;
  if (threadIdx.x == 0) {
    sh_free = 0;
    pipe_init(ps);
  }
  __syncthreads();
  if (fsm_wave()) {
    MinRule<T, false, false> R{u, w, rd, SP, false};
    const int ns = wave_fsm2(R, L, L, SP, A.max_fine_sweeps, &ps);
    if (threadIdx.x == 0) sh_ns = ns;
  }
  __syncthreads();
  const int tile = bx;
  for (int k = threadIdx.x; k < L * L; k += kBlock) {
    const int li = k % L, lj = k / L;
    const int xi = bi + li, yi = bj + lj;
    const int X = xi + A.n0 * yi;
    const int x = (lj + 1) * SP + (li + 1);
    const T v = u[x];
    const uint8_t c = w[x];
    const bool ifx = (li == 0 || li == A.S) && is_iface(xi, A.S, A.n0);
    const bool ify = (lj == 0 || lj == A.S) && is_iface(yi, A.S, A.n1);
    if (!ifx && !ify) {
      A.u_out[X] = v;
      if (xi % A.M == 0 || yi % A.M == 0) {
        A.uk[X] = v;
        A.wk[X] = c;
      }
    }
    if (li == 0) { A.edge_u[(tile * 4 + 0) * L + lj] = v; A.edge_w[(tile * 4 + 0) * L + lj] = c; }
    if (li == A.S) { A.edge_u[(tile * 4 + 1) * L + lj] = v; A.edge_w[(tile * 4 + 1) * L + lj] = c; }
    if (lj == 0) { A.edge_u[(tile * 4 + 2) * L + li] = v; A.edge_w[(tile * 4 + 2) * L + li] = c; }
    if (lj == A.S) { A.edge_u[(tile * 4 + 3) * L + li] = v; A.edge_w[(tile * 4 + 3) * L + li] = c; }
  }
  for (int o = 32; o > 0; o >>= 1) nfree += __shfl_xor(nfree, o);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&sh_free, nfree);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&A.counters[0], (unsigned long long)sh_free * (unsigned long long)sh_ns);
  if (threadIdx.x == 0 && A.sweep_prof) {
    atomicAdd(&A.sweep_prof[0], (unsigned long long)ps.lsteps);
    atomicAdd(&A.sweep_prof[1], (unsigned long long)ps.lcyc);
  }
  if (threadIdx.x == 0 && ps.err) atomicOr(&A.counters[3], 1ull);  // a two-wave wait gave up
}
// Workgroups go to the 8 compute dies round robin (block b to die b % 8),
// each die with its own L2: block b takes tile (b % 8) * n/8 + b / 8, so that
// every die holds a contiguous run of tiles (whole rows of tiles), whose
// shared boundary rows then come from one L2.  The tiles are independent:
// any order gives the same results.
__device__ __forceinline__ int die_local_tile(int b, int n) {
  if (n % 8 != 0) return b;
  return (b % 8) * (n / 8) + b / 8;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile(DD2<T> A) {
  tile_body(A, die_local_tile((int)blockIdx.x, (int)gridDim.x));
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_b(const DD2<T>* descs, const int2* work, int nwork, int* next) {
  batch_items(descs, work, nwork, next, [](const DD2<T>& A, int bx) { tile_body(A, bx); });
}


// ---------------------------------------------------------------------------
// eik_solve: one directional sweep of the whole grid, boxes in wavefront order
// ---------------------------------------------------------------------------

template <typename T>
struct GS2 {
  int n0, n1;
  int B;            // box side (nodes)
  int BX, BY;       // boxes per axis
  T hT;
  const T* r;
  const T* gfull;   // [member][N]
  T* u;             // [member][N]
  uint8_t* w;       // [member][N]
  unsigned int* changed;  // [member]
  const int* members;     // batch: blockIdx.y -> member (NULL: member = blockIdx.y)
  int* eval_at;           // [member][box] launch at which the box was last swept (-1: never)
  int* chg_at;            // [member][box] launch at which it last changed (-1: never)
};

// A box must be swept unless it changed nothing when it was last swept and
// none of its face neighbours has changed since: then every node's
// neighbours kept their values since the node was last computed, so the
// sweep would reproduce every value (the box is stationary).  t: this
// launch's number (sweep * diagonals + diagonal); boxes on one diagonal
// share no face.
__device__ __forceinline__ bool box_needed(const int* eval_at, const int* chg_at, int I, int J, int BX, int BY) {
  const int b = I + BX * J;
  const int ev = eval_at[b];
  if (chg_at[b] == ev) return true;  // changed at its last sweep, or never swept
  if (I > 0 && chg_at[b - 1] > ev) return true;
  if (I < BX - 1 && chg_at[b + 1] > ev) return true;
  if (J > 0 && chg_at[b - BX] > ev) return true;
  if (J < BY - 1 && chg_at[b + BX] > ev) return true;
  return false;
}

// Boxes with (I' + J') == diag in sweep order.  Box (I, J) reads its halo
// from global memory: the upwind neighbours were finished by the previous
// diagonals, the downwind ones are untouched, so the sweep of the whole grid
// is the paper's serial Gauss-Seidel sweep exactly.
// The sweeps, box diagonals and block ranges of one launch of k_grid_sweep:
// sweep 2m (dir[0]) and, BY + 1 box diagonals behind it, sweep 2m+1 (dir[1],
// y reversed).  A box on diagonal d of the first lies on d - 2J' + BY - 1 of
// the second (J' its y index in the first's order), so no box the second
// takes, nor a face neighbour of it, is still open in the first, and the
// second writes no box the first will still read: the two give the values
// of the sweeps one after the other.  Each sweep has its own change flags
// (chg_off: offset into A.changed) and launch numbers t.
struct GridLaunch2 {
  int n;
  int dir[2], diag[2], t[2], start[3], chg_off[2];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_grid_sweep(GS2<T> A, GridLaunch2 L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int g = (L.n > 1 && (int)blockIdx.x >= L.start[1]) ? 1 : 0;
  const int dir = L.dir[g], diag = L.diag[g], t = L.t[g];
  const int bxl = (int)blockIdx.x - L.start[g];
  A.changed += L.chg_off[g];
  const int sx = (dir & 2) ? 1 : -1, sy = (dir & 1) ? 1 : -1;
  // problem of the batch (same grid and slowness, its own Gamma)
  const int mem = A.members ? A.members[blockIdx.y] : (int)blockIdx.y;
  const int64_t mo = (int64_t)mem * A.n0 * A.n1;
  A.gfull += mo;
  A.u += mo;
  A.w += mo;
  A.changed += mem;
  A.eval_at += mem * A.BX * A.BY;
  A.chg_at += mem * A.BX * A.BY;
  const int q0 = max(0, diag - (A.BY - 1));
  const int Iq = q0 + bxl;
  const int Jq = diag - Iq;
  if (Iq >= A.BX || Jq < 0) return;
  const int I = sx > 0 ? Iq : A.BX - 1 - Iq;
  const int J = sy > 0 ? Jq : A.BY - 1 - Jq;
  if (!box_needed(A.eval_at, A.chg_at, I, J, A.BX, A.BY)) return;
  const int bi = I * A.B, bj = J * A.B;
  const int L0 = min(A.B, A.n0 - bi), L1 = min(A.B, A.n1 - bj);
  const int SP = halo_stride(L0);
  const int cnt = halo_count(L0, L1);
  unsigned char* lc = smem;
  T* u = carve<T>(lc, cnt);
  T* rd = carve<T>(lc, cnt);
  uint8_t* w = carve<uint8_t>(lc, cnt);
  const T inf = pinf<T>();
  const T nan = T(__builtin_nan(""));
  for (int k = threadIdx.x; k < cnt; k += kBlock) {
    const int hi = k % SP - 1, hj = k / SP - 1;
    const int xi = bi + hi, yi = bj + hj;
    const bool inside = hi >= 0 && hi < L0 && hj >= 0 && hj < L1;
    T v = inf, rv = nan;
    uint8_t c = 0;
    if (inside) {
      const int X = xi + A.n0 * yi;
      v = A.u[X];
      c = A.w[X];
      if (disnan(A.gfull[X])) rv = A.r[X] * A.hT;
    } else if (hi >= -1 && hi <= L0 && hj >= -1 && hj <= L1 && xi >= 0 && xi < A.n0 && yi >= 0 &&
               yi < A.n1) {
      v = A.u[xi + A.n0 * yi];
    }
    u[k] = v;
    w[k] = c;
    rd[k] = rv;
  }
  __syncthreads();
  __shared__ int sh_ch;
  if (threadIdx.x == 0) sh_ch = 0;
  __syncthreads();
  if (threadIdx.x < kWave) {
    MinRule<T, false, true> R{u, w, rd, SP, false};
    const bool ch = sweep_any(R, L0, L1, SP, dir);
    if (__any(ch) && threadIdx.x == 0) sh_ch = 1;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L0 * L1; k += kBlock) {
    const int li = k % L0, lj = k / L0;
    const int X = (bi + li) + A.n0 * (bj + lj);
    const int x = (lj + 1) * SP + (li + 1);
    A.u[X] = u[x];
    A.w[X] = w[x];
  }
  if (threadIdx.x == 0) {
    A.eval_at[I + A.BX * J] = t;
    if (sh_ch) {
      A.chg_at[I + A.BX * J] = t;
      atomicOr(A.changed, 1u);
    }
  }
}

template <typename T>
__global__ void k_grid_init(GS2<T> A) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = (int64_t)blockIdx.y * N + t;
  const T g = A.gfull[x];
  A.u[x] = disnan(g) ? pinf<T>() : g;
  A.w[x] = 0;
}

// Reconciliation (Alg. fineupdate, per interface axis) at every interface
// node.  Threads: (P0-1) vertical interface lines x n1 nodes, then (P1-1)
// horizontal lines x n0 nodes (crossings are done by the vertical pass).
template <typename T>
__device__ __forceinline__ void reconcile_body(const DD2<T>& A, int bx) {
  if (dd_stopped(A)) return;
  const int64_t nv = (int64_t)(A.P0 - 1) * A.n1;
  const int64_t nh = (int64_t)(A.P1 - 1) * A.n0;
  const int64_t t = bx * (int64_t)blockDim.x + threadIdx.x;
  int xi, yi;
  if (t < nv) {
    xi = (int)(t / A.n1 + 1) * A.S;
    yi = (int)(t % A.n1);
  } else if (t < nv + nh) {
    const int64_t s = t - nv;
    yi = (int)(s / A.n0 + 1) * A.S;
    xi = (int)(s % A.n0);
    if (is_iface(xi, A.S, A.n0)) return;  // done by the vertical pass
  } else {
    return;
  }
  const int L = A.S + 1;
  const bool ifx = is_iface(xi, A.S, A.n0), ify = is_iface(yi, A.S, A.n1);
  int tx[2], ty[2], nx, ny;
  if (ifx) { tx[0] = xi / A.S - 1; tx[1] = xi / A.S; nx = 2; }
  else { tx[0] = min(xi / A.S, A.P0 - 1); nx = 1; }
  if (ify) { ty[0] = yi / A.S - 1; ty[1] = yi / A.S; ny = 2; }
  else { ty[0] = min(yi / A.S, A.P1 - 1); ny = 1; }
  T cu[4];
  uint8_t cw[4];
  int sdx[4], sdy[4];
  int nc = 0;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b) {
      const int tile = tx[a] + A.P0 * ty[b];
      const int li = xi - tx[a] * A.S, lj = yi - ty[b] * A.S;
      int e;
      if (li == 0) e = (tile * 4 + 0) * L + lj;
      else if (li == A.S) e = (tile * 4 + 1) * L + lj;
      else if (lj == 0) e = (tile * 4 + 2) * L + li;
      else e = (tile * 4 + 3) * L + li;
      cu[nc] = A.edge_u[e];
      cw[nc] = A.edge_w[e];
      sdx[nc] = a;
      sdy[nc] = b;
      ++nc;
    }
  const int X = xi + A.n0 * yi;
  const uint8_t Wk = A.W[X];
  const T inf = pinf<T>();
  bool keep[4];
  int nf = 0;
  for (int c = 0; c < nc; ++c) { keep[c] = cu[c] < inf; nf += keep[c]; }
  if (nf == 0)
    for (int c = 0; c < nc; ++c) keep[c] = true;
  // allowed sides per interface axis: bit0 = minus, bit1 = plus
  int alx = 3, aly = 3;
  if (ifx) {
    bool le = wx_of(Wk) <= 0, ge = wx_of(Wk) >= 0;
    for (int c = 0; c < nc; ++c)
      if (keep[c]) { le = le && wx_of(cw[c]) <= 0; ge = ge && wx_of(cw[c]) >= 0; }
    if (le) alx = 2; else if (ge) alx = 1;
  }
  if (ify) {
    bool le = wy_of(Wk) <= 0, ge = wy_of(Wk) >= 0;
    for (int c = 0; c < nc; ++c)
      if (keep[c]) { le = le && wy_of(cw[c]) <= 0; ge = ge && wy_of(cw[c]) >= 0; }
    if (le) aly = 2; else if (ge) aly = 1;
  }
  int best = -1;
  for (int c = 0; c < nc; ++c) {
    if (!keep[c]) continue;
    if (ifx && !((alx >> sdx[c]) & 1)) continue;
    if (ify && !((aly >> sdy[c]) & 1)) continue;
    if (best < 0 || cu[c] < cu[best]) best = c;
  }
  if (best < 0)
    for (int c = 0; c < nc; ++c)
      if (keep[c] && (best < 0 || cu[c] < cu[best])) best = c;
  A.uk[X] = cu[best];
  A.wk[X] = cw[best];
  A.u_out[X] = cu[best];
}
template <typename T>
__global__ void k_reconcile(DD2<T> A) { reconcile_body(A, (int)blockIdx.x); }
template <typename T>
__global__ void k_reconcile_b(const DD2<T>* descs, const int2* work) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  reconcile_body(A, w.y);
}


constexpr int kCornerBlockMax = 1024;  // largest block that calls res_reduce
// |a - b| in double for the residual max |U^{k+1} - U^k| over the skeleton:
// equal values (also inf and inf) give 0, NaN counts as +inf
template <typename T>
__device__ __forceinline__ double res_term(T a, T b) {
  double dv = 0.0;
  if (!(a == b)) dv = dabs((double)a - (double)b);
  return disnan(dv) ? __builtin_huge_val() : dv;
}
// block maximum of dv (every thread of the block calls this), then one
// atomic maximum per block on the bits (the order of non-negative doubles is
// that of their bit patterns)
__device__ __forceinline__ void res_reduce(double dv, unsigned long long* out) {
  __shared__ double wmax[kCornerBlockMax / kWave];
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(dv, o);
    dv = dv < v ? v : dv;
  }
  const int nw = (int)blockDim.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = dv;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < nw; ++i) dv = dv < wmax[i] ? wmax[i] : dv;
    if (dv > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(dv));
  }
}

// ---------------------------------------------------------------------------
// causal sweep (Alg. causalsweep2D)
//
// In sweep direction (sx, sy) a coarse node X with wind component W_e = s_e
// (flow along the sweep) is raised to the NEW value of its upwind fine
// neighbour X - s_e e, and with W_e = -s_e to the OLD value of X + s_e e.
// Both are maxima, so the result is: V(X) = max(U(X), old successors), then
// U_new(X) = max(V(X), U_new of every linked predecessor).  Between corners
// the links form chains (segments of M-1 nodes); corners join the
// horizontal and vertical chains.  Per direction: phase A, V and the chain
// prefix maxima of every segment; phase B, the corner recurrence on the
// coarse grid in anti-diagonal order; phase C, fill the segments from their
// start corner.
//
// Two launches per direction: k_causal_seg, one thread per segment node,
// runs phase C of the previous direction, then phase A of this one (phase A
// of a segment reads only the segment and its end corner, both final after
// the previous phase B), and stores the value of the segment's node next to the
// corner it leaves in sweep order, which that corner's V needs (ncx / ncy);
// k_causal_corner, one block, evaluates V and the links of every corner from
// independent loads and runs phase B.  A last k_causal_c fills the segments
// of the fourth direction.  When the sweep finishes U^{k+1} (Step 4) the
// last corner kernel and k_causal_c also take the residual against U^k, as
// they write the skeleton's final values (corners, segment nodes).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T vmax(T a, T b) { return a < b ? b : a; }

// segment s of the skeleton: horizontal segments first (I < NI, J <= NJ),
// then vertical ones (I <= NI, J < NJ); corner (I, J) at its minus end
struct Seg {
  bool horiz;
  int I, J;
};
template <typename T>
__device__ __forceinline__ Seg seg_of(const DD2<T>& A, int s) {
  const int nH = A.NI * (A.NJ + 1);
  if (s < nH) return Seg{true, s % A.NI, s / A.NI};
  s -= nH;
  return Seg{false, s % (A.NI + 1), s / (A.NI + 1)};
}

// The corner recurrence U(C) = max(B(C), [ax] U(C - sx e_x), [ay] U(C - sy e_y))
// on the coarse grid of corners, by one wave, without the sweep engine's
// bookkeeping (nothing here can stop a sweep early): lane j holds row j in
// sweep order and at step t takes column t - j, its x predecessor being its
// own previous value and its y predecessor lane j-1's (DPP); a 65th row runs
// on lane 0 one step late (steps 65 .. 65 + CI - 1), taking lane 63's value
// of two steps back.  Each node's record {V, link addends} is read four
// steps ahead.  A link is the addend -0 (linked) or -inf (not): value + -0
// is the value itself (bit for bit, -0 included), value + -inf is -inf (or
// NaN, from +inf - inf), which never wins the strict comparison of the
// maximum, so the maximum is the same as with a link test.  Links exist only where the predecessor
// does, so the values a lane holds outside its row are never used.
template <typename T>
struct alignas(16) CornerOp {
  T b;
  float lx, ly;
};
// LDS bytes of the corner kernel: the records and the values
__host__ __device__ __forceinline__ size_t corner_lds_bytes(int CI, int CJ, size_t szT) {
  return (size_t)(halo_count(CI, CJ) + 2 * kGuard) * (sizeof(CornerOp<double>) + szT);
}
template <int SX, int SY, typename T>
__device__ __forceinline__ void corner_wave(T* cu, const CornerOp<T>* op, int CI, int CJ, int SP) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool extra = CJ > kWave;
  const bool rowA = lane < CJ;
  // record index at step t: x0 + SX t (row 64 on lane 0: x0B + SX t)
  const int JA = min(SY > 0 ? lane : CJ - 1 - lane, CJ - 1);
  const int JB = SY > 0 ? kWave : CJ - 1 - kWave;
  const int x0A = (JA + 1) * SP + 1 + (SX > 0 ? -lane : CI - 1 + lane);
  const int x0B = (JB + 1) * SP + 1 + (SX > 0 ? -(kWave + 1) : CI - 1 + kWave + 1);
  const int last = extra ? kWave + CI : min(CJ, kWave) - 1 + CI - 1;
  T cur = T(0), prev = T(0);
  auto run = [&](auto phase, int t0, int t1) {
    constexpr bool P2 = decltype(phase)::value;
    // B: lane 0 on row 64 (the steps after kWave)
    const bool B = P2 && extra && lane == 0;
    const int x0 = B ? x0B : x0A;
    const int off = B ? kWave + 1 : lane;
    const bool rowok = B || rowA;
    const int dmy = dummy_slot();
    auto index = [=](int t) {
      const bool act = rowok && (unsigned)(t - off) < (unsigned)CI;
      return act ? x0 + SX * t : dmy;
    };
    // four slots of {record index, record}: step t uses slot t % 4 and then
    // refills it with step t + 4's
    int x0s = index(t0), x1s = index(t0 + 1), x2s = index(t0 + 2), x3s = index(t0 + 3);
    CornerOp<T> o0 = op[x0s], o1 = op[x1s], o2 = op[x2s], o3 = op[x3s];
    auto step = [&](int t, int& xs, CornerOp<T>& o) {
      const int x = xs;
      T py = dpp_ror1(cur);
      if (P2) {
        const T py2 = dpp_ror1(prev);
        py = B ? py2 : py;
      }
      const T cx = cur + (T)o.lx, cy = py + (T)o.ly;
      T v = o.b;
      v = v < cx ? cx : v;
      v = v < cy ? cy : v;
      prev = cur;
      const bool act = x != dmy;
      cur = act ? v : cur;
      cu[x] = v;
      xs = index(t + 4);
      o = op[xs];
    };
    int t = t0;
    for (; t + 3 <= t1; t += 4) {
      step(t, x0s, o0);
      step(t + 1, x1s, o1);
      step(t + 2, x2s, o2);
      step(t + 3, x3s, o3);
    }
    if (t <= t1) step(t, x0s, o0);
    if (t + 1 <= t1) step(t + 1, x1s, o1);
    if (t + 2 <= t1) step(t + 2, x2s, o2);
  };
  // steps 0 .. kWave: rows 0 .. 63; then lane 0 switches to row 64
  run(std::integral_constant<bool, false>{}, 0, min(last, kWave));
  if (last > kWave) run(std::integral_constant<bool, true>{}, kWave + 1, last);
}

// phase B for one direction, by one block: the corners' V and links (from
// U, W, the segments' phase-A results and ncx / ncy) into LDS, the
// recurrence by one wave (meanwhile the other waves read the old corner
// values the residual needs), the corner values back to U
template <typename T>
__device__ __forceinline__ void causal_corner_body(const DD2<T>& A, T* U, const uint8_t* W, int dir, bool res) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (dd_stopped(A)) return;
  const int sx = (dir & 2) ? 1 : -1, sy = (dir & 1) ? 1 : -1;
  const int CI = A.NI + 1, CJ = A.NJ + 1;
  const int SP = halo_stride(CI);
  const int cnt = halo_count(CI, CJ);
  const int M = A.M;
  const int nH = A.NI * CJ, nV = CI * A.NJ;
  unsigned char* lc = smem;
  CornerOp<T>* op = carve<CornerOp<T>>(lc, cnt);
  T* cu = carve<T>(lc, cnt);
  const float ninf = -__builtin_huge_valf();
  // corner t = I + CI J: J from a float reciprocal (exact: t < 2^20, and
  // (t + 1/2) / CI stays more than 1/(2 CI) away from an integer)
  const float rCI = 1.0f / (float)CI;
  auto corner_ij = [&](int t, int& I, int& J) {
    J = (int)(((float)t + 0.5f) * rCI);
    I = t - J * CI;
  };
  // a thread's corners are blockDim.x apart; all loads of up to kPer corners
  // are issued before any is used (the loads are independent; in a loop
  // they would wait one corner at a time)
  constexpr int kPer = 5;
  const int nc = CI * CJ;
  for (int base = threadIdx.x; base < nc; base += kPer * (int)blockDim.x) {
    T u[kPer], nx[kPer], ny[kPer], hp[kPer], vp[kPer];
    uint8_t gm[kPer], cw[kPer], hl[kPer], vl[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int t = base + k * (int)blockDim.x;
      if (t < nc) {
        int I, J;
        corner_ij(t, I, J);
        // incoming segments in sweep order (clamped; used only when linked)
        const int hs = min(max((sx > 0 ? I - 1 : I) + A.NI * J, 0), nH - 1);
        const int vs = min(max(I + CI * (sy > 0 ? J - 1 : J), 0), nV - 1);
        u[k] = A.cU[t];
        gm[k] = A.cG[t];
        cw[k] = A.cW[t];
        nx[k] = A.ncx[t];
        ny[k] = A.ncy[t];
        hp[k] = A.hseg_p[hs];
        vp[k] = A.vseg_p[vs];
        hl[k] = A.hseg_l[hs];
        vl[k] = A.vseg_l[vs];
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int t = base + k * (int)blockDim.x;
      if (t >= nc) break;
      int I, J;
      corner_ij(t, I, J);
      const int xi = I * M, yi = J * M;
      T b = u[k];
      float lx = ninf, ly = ninf;
      if (gm[k] == 0) {
        const int ex = wx_of(cw[k]), ey = wy_of(cw[k]);
        const int nxi = xi + sx, nyi = yi + sy;
        if (ex == -sx && nxi >= 0 && nxi < A.n0) b = vmax(b, nx[k]);
        if (ey == -sy && nyi >= 0 && nyi < A.n1) b = vmax(b, ny[k]);
        const int pxi = xi - sx, pyi = yi - sy;
        if (ex == sx && pxi >= 0 && pxi < A.n0) {
          b = vmax(b, hp[k]);
          if (hl[k]) lx = -0.f;
        }
        if (ey == sy && pyi >= 0 && pyi < A.n1) {
          b = vmax(b, vp[k]);
          if (vl[k]) ly = -0.f;
        }
      }
      const int x = (J + 1) * SP + (I + 1);
      op[x] = CornerOp<T>{b, lx, ly};
    }
  }
  __syncthreads();
  // the residual's old corner values, read by waves 1.. while wave 0 runs
  // the recurrence (up to kPer per thread; the rest after it)
  const int nt = (int)blockDim.x - kWave;
  const int tid = (int)threadIdx.x - kWave;
  T old[kPer];
  if (threadIdx.x < kWave) {
    switch (dir) {
      case 0: corner_wave<-1, -1>(cu, op, CI, CJ, SP); break;
      case 1: corner_wave<-1, 1>(cu, op, CI, CJ, SP); break;
      case 2: corner_wave<1, -1>(cu, op, CI, CJ, SP); break;
      default: corner_wave<1, 1>(cu, op, CI, CJ, SP); break;
    }
  } else if (res) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int t = tid + k * nt;
      if (t < nc) {
        int I, J;
        corner_ij(t, I, J);
        old[k] = A.U[I * M + A.n0 * (J * M)];
      }
    }
  }
  __syncthreads();
  double dv = 0.0;
  if (tid >= 0) {
    for (int base = tid; base < nc; base += kPer * nt) {
      if (res && base != tid) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          const int t = base + k * nt;
          if (t < nc) {
            int I, J;
            corner_ij(t, I, J);
            old[k] = A.U[I * M + A.n0 * (J * M)];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int t = base + k * nt;
        if (t >= nc) break;
        int I, J;
        corner_ij(t, I, J);
        const T v = cu[(J + 1) * SP + (I + 1)];
        U[I * M + A.n0 * (J * M)] = v;
        if (res) {
          const double d = res_term(v, old[k]);
          dv = dv < d ? d : dv;
        }
      }
    }
  }
  if (res) res_reduce(dv, A.res_out);
}
constexpr int kCornerBlock = kCornerBlockMax;
template <typename T>
__global__ __launch_bounds__(kCornerBlock) void k_causal_corner(DD2<T> A, T* U, const uint8_t* W, int dir, int res) {
  causal_corner_body(A, U, W, dir, res != 0);
}
// batched: one block per problem (work = (problem, 0)); which = 0 sweeps
// U/W of each problem, 1 sweeps Un/Wn (and takes the residual in the last
// direction)
template <typename T>
__global__ __launch_bounds__(kCornerBlock) void k_causal_corner_b(const DD2<T>* descs, const int2* work, int which,
                                                                 int dir) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  causal_corner_body(A, which ? A.Un : A.U, which ? A.Wn : A.W, dir, which != 0 && dir == 3);
}

// The segment kernels run one thread per segment node: a block holds
// kBlock / (M-1) whole segments, node q = 1 .. M-1 of a segment (counted
// from its minus-end corner) at thread (segment slot) * (M-1) + q - 1.
template <typename T>
__host__ __device__ __forceinline__ int causal_seg_blocks(const DD2<T>& A) {
  const int nseg = A.NI * (A.NJ + 1) + (A.NI + 1) * A.NJ;
  const int per = kBlock / (A.M - 1);
  return (nseg + per - 1) / per;
}
// launch size of k_causal_seg and k_causal_c: the segment blocks, then the
// blocks that gather the corners (idle in k_causal_c)
template <typename T>
__host__ __device__ __forceinline__ int causal_blocks(const DD2<T>& A) {
  const int nc = (A.NI + 1) * (A.NJ + 1);
  return causal_seg_blocks(A) + (nc + kBlock - 1) / kBlock;
}
struct SegNode {
  bool on;    // a node of an existing segment
  Seg g;
  int s, q;   // segment, node position from the minus-end corner
  int slot;   // the segment's slot in the block
  int stride, base, X;
};
template <typename T>
__device__ __forceinline__ SegNode seg_node(const DD2<T>& A, int bx) {
  SegNode n;
  const int m1 = A.M - 1;
  const int per = kBlock / m1;
  const int nseg = A.NI * (A.NJ + 1) + (A.NI + 1) * A.NJ;
  n.slot = (int)threadIdx.x / m1;
  n.q = (int)threadIdx.x % m1 + 1;
  n.s = bx * per + n.slot;
  n.on = n.slot < per && n.s < nseg;
  n.g = seg_of(A, n.on ? n.s : 0);
  n.stride = n.g.horiz ? 1 : A.n0;
  n.base = (n.g.I * A.M) + A.n0 * (n.g.J * A.M);
  n.X = n.base + n.q * n.stride;
  return n;
}
// phase C of direction (sx, sy) at one node; returns the node's value
template <typename T>
__device__ __forceinline__ T seg_fill(const DD2<T>& A, const SegNode& n, T* U, int sx, int sy) {
  const int sg = n.g.horiz ? sx : sy;
  const T cs = U[sg > 0 ? n.base : n.base + A.M * n.stride];
  const T P = A.cwork[n.X];
  const uint8_t F = A.cflag[n.X];
  const T v = F ? vmax(P, cs) : P;
  U[n.X] = v;
  return v;
}

// phase C of direction prev (prev < 0: none) and phase A of direction dir
// on every segment node, then the value the corner each segment leaves needs
template <typename T>
__device__ __forceinline__ void causal_seg_body(const DD2<T>& A, int bx, T* U, const uint8_t* W, int dir, int prev) {
  __shared__ T sv[kBlock];
  __shared__ uint8_t sl[kBlock];
  if (dd_stopped(A)) return;
  const int nsb = causal_seg_blocks(A);
  if (bx >= nsb) {
    // the corners' U (final since the last corner kernel), W and Gamma flag
    const int CI = A.NI + 1;
    const int t = (bx - nsb) * kBlock + (int)threadIdx.x;
    if (t < CI * (A.NJ + 1)) {
      const int X = (t % CI) * A.M + A.n0 * ((t / CI) * A.M);
      A.cU[t] = U[X];
      A.cW[t] = W[X];
      A.cG[t] = disnan(A.gfull[X]) ? 0 : 1;
    }
    return;
  }
  const SegNode n = seg_node(A, bx);
  const int t = threadIdx.x;
  const int M = A.M, m1 = M - 1;
  const int sx = (dir & 2) ? 1 : -1, sy = (dir & 1) ? 1 : -1;
  const int sg = n.g.horiz ? sx : sy;
  T u = T(0), vv = T(0);
  bool link = false;
  // the node's successor in sweep order: a node of the same segment (its
  // value after phase C is in LDS) or the end corner (final; corners are not
  // written here).  Every global load of the node is issued in this first
  // phase, so the kernel waits for global memory once.
  const int qn = n.q + sg;
  const bool inner = qn >= 1 && qn <= m1;
  T g = T(0), endc = T(0);
  uint8_t wc = 0;
  if (n.on) {
    g = A.gfull[n.X];
    wc = W[n.X];
    if (!inner) endc = U[n.base + qn * n.stride];
    u = prev >= 0 ? seg_fill(A, n, U, (prev & 2) ? 1 : -1, (prev & 1) ? 1 : -1) : U[n.X];
    sv[t] = u;
  }
  __syncthreads();
  if (n.on) {
    const T nx = inner ? sv[t + sg] : endc;
    vv = u;
    if (disnan(g)) {
      const int e = n.g.horiz ? wx_of(wc) : wy_of(wc);
      if (e == -sg) vv = vmax(vv, nx);
      link = (e == sg);
    }
  }
  __syncthreads();
  if (n.on) {
    sv[t] = vv;
    sl[t] = link ? 1 : 0;
  }
  __syncthreads();
  // the chain prefix maximum and the link to the start corner, in sweep
  // order, by one thread per segment
  if (n.on && n.q == 1) {
    const int b0 = n.slot * m1;
    T P = T(0);
    bool L = true;
    for (int k = 1; k <= m1; ++k) {
      const int i = b0 + (sg > 0 ? k : M - k) - 1;
      const T v = sv[i];
      const bool lk = sl[i] != 0;
      P = (lk && k > 1) ? vmax(v, P) : v;
      L = L && lk;
      sv[i] = P;
      sl[i] = L ? 1 : 0;
    }
    const int nH = A.NI * (A.NJ + 1);
    if (n.g.horiz) { A.hseg_p[n.s] = P; A.hseg_l[n.s] = L ? 1 : 0; }
    else { A.vseg_p[n.s - nH] = P; A.vseg_l[n.s - nH] = L ? 1 : 0; }
  }
  __syncthreads();
  if (n.on) {
    A.cwork[n.X] = sv[t];
    A.cflag[n.X] = sl[t];
    // the corner the segment leaves in sweep order takes this node's value
    // as its successor value
    const int CI = A.NI + 1;
    if (n.q == (sg > 0 ? 1 : m1)) {
      if (n.g.horiz) A.ncx[(sg > 0 ? n.g.I : n.g.I + 1) + CI * n.g.J] = u;
      else A.ncy[n.g.I + CI * (sg > 0 ? n.g.J : n.g.J + 1)] = u;
    }
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_causal_seg(DD2<T> A, T* U, const uint8_t* W, int dir, int prev) {
  causal_seg_body(A, (int)blockIdx.x, U, W, dir, prev);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_causal_seg_b(const DD2<T>* descs, const int2* work, int which, int dir,
                                                        int prev) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  causal_seg_body(A, w.y, which ? A.Un : A.U, which ? A.Wn : A.W, dir, prev);
}

// phase C of the last direction (and the residual of the segment nodes)
template <typename T>
__device__ __forceinline__ void causal_c_body(const DD2<T>& A, int bx, T* U, int sx, int sy, bool res) {
  if (dd_stopped(A)) return;
  const SegNode n = seg_node(A, bx);
  double dv = 0.0;
  if (n.on) {
    // with res, U is the other array (U^{k+1}), so A.U can be read first
    const T old = res ? A.U[n.X] : T(0);
    const T v = seg_fill(A, n, U, sx, sy);
    if (res) dv = res_term(v, old);
  }
  if (res) res_reduce(dv, A.res_out);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_causal_c(DD2<T> A, T* U, int sx, int sy, int res) {
  causal_c_body(A, (int)blockIdx.x, U, sx, sy, res != 0);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_causal_c_b(const DD2<T>* descs, const int2* work, int which, int sx,
                                                      int sy) {
  const int2 w = work[blockIdx.x];
  const DD2<T> A = descs[w.x];
  causal_c_body(A, w.y, which ? A.Un : A.U, sx, sy, which != 0);
}


// U_out: U on the skeleton, NaN elsewhere
template <typename T>
__device__ __forceinline__ void export_U_body(const DD2<T>& A, int bx, const T* U, T* out) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t t = bx * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int xi = (int)(t % A.n0), yi = (int)(t / A.n0);
  out[t] = (xi % A.M == 0 || yi % A.M == 0) ? U[t] : T(__builtin_nan(""));
}
template <typename T>
__global__ void k_export_U(DD2<T> A, const T* U, T* out) { export_U_body(A, (int)blockIdx.x, U, out); }


template <typename T>
__global__ void k_import_U(DD2<T> A, const T* Uin, T* U) {
  const int64_t N = (int64_t)A.n0 * A.n1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int xi = (int)(t % A.n0), yi = (int)(t / A.n0);
  U[t] = (xi % A.M == 0 || yi % A.M == 0) ? Uin[t] : T(__builtin_nan(""));
}

}  // namespace eik
