// Host runtime and C ABI of the MI355X two-scale DD Eikonal solver
// (Martin & Tsai, arXiv 1805.04198).  See include/eik.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/eik.h"
#include "kernels2d.hpp"
#include "kernels3d.hpp"
#include "kernels_adj.hpp"

namespace {

thread_local std::string g_err;

eik_status fail(eik_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
eik_status fail(eik_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(EIK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxDevices = 64;
constexpr size_t kLdsBytes = 160 * 1024;

// LDS bytes of the lattice kernels (Steps 1 and 4) for NI x NJ coarse cells;
// packed: whether Step 4 runs on its fp32 records (CorrRecF32: fp32 with a
// constant weight, 150 KB at the fixed 65-node geometry)
// LDS bytes of the lattice kernels.  Step 4 holds two doubles more per node
// when the weight varies; where that does not fit (fp64, 65 x 65) they go to
// global memory instead (tglob: halo_count doubles twice per lattice).
inline size_t lattice_lds(int NI, int NJ, int tmode, size_t szT, bool& packed, bool& tglob) {
  const int cnt = eik::halo_count(NI + 1, NJ + 1);
  const size_t base4 = eik::box_bytes(cnt, 4, 1, szT);
  size_t step4 = base4 + (tmode ? eik::box_bytes(cnt, 2, 0, 8) : 0);
  tglob = tmode != 0 && step4 > kLdsBytes && base4 <= kLdsBytes;
  if (tglob) step4 = base4;
  const size_t step1 = eik::box_bytes(cnt, 2, 1, szT);
  packed = szT == 4 && tmode == 0 && eik::corr_f32_lds_bytes() <= kLdsBytes;
  return std::max(packed ? eik::corr_f32_lds_bytes() : step4, step1);
}

// Per-device workspace: one device buffer grown on demand, plus pinned host
// words for the per-iteration readback.  Calls on one device are serialised.
struct Workspace {
  std::mutex mu;
  void* dev = nullptr;
  size_t bytes = 0;
  unsigned long long* host = nullptr;  // pinned: 8 words
};
Workspace g_ws[kMaxDevices];

eik_status ws_get(int dev, size_t need, void** out, unsigned long long** host) {
  Workspace& w = g_ws[dev];
  if (w.bytes < need) {
    if (w.dev) HIPCHK(hipFree(w.dev));
    w.dev = nullptr;
    w.bytes = 0;
    HIPCHK(hipMalloc(&w.dev, need));
    w.bytes = need;
  }
  if (!w.host) HIPCHK(hipHostMalloc((void**)&w.host, 8 * sizeof(unsigned long long), hipHostMallocDefault));
  *out = w.dev;
  *host = w.host;
  return EIK_OK;
}

// Scratch of the allocation-free entry point (eik_dd_solve_noalloc): a
// fixed array in device memory, one copy per device, held until the
// process ends.  Host code uses the address hipGetSymbolAddress returns on
// each device, never the array's name.
constexpr size_t kScratchBytes = EIK_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_dev[kMaxDevices];
unsigned long long g_scratch_host[kMaxDevices][8];  // readback words (pageable)

// The scratch array of device `dev` (current) as a workspace: its device
// address, looked up on the first call on the device (under the device's
// lock), and plain host words.  Allocates nothing.
eik_status scratch_get(int dev, size_t need, void** out, unsigned long long** host) {
  if (need > kScratchBytes)
    return fail(EIK_ERR_UNSUPPORTED, "the allocation-free solve needs %zu bytes of scratch, more than its %zu",
                need, kScratchBytes);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  *host = g_scratch_host[dev];
  return EIK_OK;
}

// K device-time events of a call, or none (the allocation-free entry point:
// its timing fields stay 0).
template <int K>
struct Events {
  hipEvent_t e[K];
  bool on = false;
  int made = 0;
  eik_status init(bool want) {
    if (!want) return EIK_OK;
    for (; made < K; ++made) HIPCHK(hipEventCreate(&e[made]));
    on = true;
    return EIK_OK;
  }
  eik_status rec(int i, hipStream_t s) {
    if (on) HIPCHK(hipEventRecord(e[i], s));
    return EIK_OK;
  }
  eik_status ms(int a, int b, float* out) {
    *out = 0.f;
    if (on) HIPCHK(hipEventElapsedTime(out, e[a], e[b]));
    return EIK_OK;
  }
  ~Events() {
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(e[i]);
  }
};
#define EVCHK(expr)                  \
  do {                               \
    const eik_status es_ = (expr);   \
    if (es_ != EIK_OK) return es_;   \
  } while (0)

// Instantiated graphs of the 2D DD iteration block (EIK_LAUNCH_GRAPH), per
// device and block parity (the residual slots alternate between blocks),
// with the bytes of everything the captured launches depend on; guarded by
// the device's workspace lock.  Captured on a stream of their own (default
// priority) and kept until the process ends.
struct DDGraph {
  std::vector<unsigned char> key;
  hipGraphExec_t exec = nullptr;
};
DDGraph g_ddgraph[kMaxDevices][2];
hipStream_t g_capture_stream[kMaxDevices];

// carve aligned sub-buffers out of the workspace
struct Carver {
  char* base;
  size_t off = 0;
  template <typename U>
  U* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    U* p = reinterpret_cast<U*>(base + off);
    off += n * sizeof(U);
    return p;
  }
};

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename K>
eik_status allow_lds(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return EIK_OK;
}

// fp32 only: the smallest r * h accepted.  The correctly rounded fp32
// square root of the local solve (eik::dsqrt) needs its argument t >= 2^-96.
// A two-sided solve has t > (r Delta)^2: in 2D t = 2 (r Delta)^2 - (a - b)^2
// with |a - b| < r Delta; in 3D the three-term root runs only when the
// two-term one lies above the third neighbour, and then t/3 exceeds
// (r Delta)^2 - (2/3) (p^2 + q^2) with p^2 + q^2 < (r Delta)^2 (p, q: the
// gaps of the two smaller neighbours below the third).  Delta >= h, so
// r h >= 2^-40 keeps t above 2^-80, a margin of 2^16.
constexpr double kMinRhF32 = 0x1p-40;

template <typename T>
eik_status validate(const T* r, int64_t N, const eik_gamma* gam, unsigned int* dflag,
                    unsigned long long* host, hipStream_t s, double h) {
  HIPCHK(hipMemsetAsync(dflag, 0, sizeof(unsigned int), s));
  const int64_t n = std::max<int64_t>(N, gam->count);
  const double rh_min = sizeof(T) == 4 ? kMinRhF32 / h : 0.0;
  hipLaunchKernelGGL(eik::k_validate<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, r, N, gam->idx,
                     (const T*)gam->g, gam->count, rh_min, dflag);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(host, dflag, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  unsigned int bad = *(unsigned int*)host;
  if (bad & 1) return fail(EIK_ERR_ARG, "r must be > 0 and finite at every node");
  if (bad & 2) return fail(EIK_ERR_ARG, "Gamma indices must be strictly increasing and in [0, N)");
  if (bad & 4) return fail(EIK_ERR_ARG, "Gamma values must be finite");
  if (bad & 8)
    return fail(EIK_ERR_UNSUPPORTED, "fp32: r * h below 2^-40 somewhere; the correctly rounded square root of "
                "the local solve is not exact that far down (use fp64 or rescale r)");
  return EIK_OK;
}

template <typename T>
T* as(const void* p) { return (T*)p; }

// ---------------------------------------------------------------------------
// eik_dd_solve, d = 2
// ---------------------------------------------------------------------------

// Alg. causalsweep2D: per direction the segment kernel (phase C of the
// previous direction, phase A of this one) and the corner kernel (phase B),
// then phase C of the last direction.
// res: also take the residual max |U - A.U| into A.counters[2] (U = A.Un)
template <typename T>
void causal_sweep(eik::DD2<T>& A, T* U, const uint8_t* W, hipStream_t s, size_t ldsB, int res) {
  const int nb = eik::causal_blocks(A);
  for (int dir = 0; dir < 4; ++dir) {
    hipLaunchKernelGGL(eik::k_causal_seg<T>, dim3(nb), dim3(eik::kBlock), 0, s, A, U, W, dir, dir - 1);
    hipLaunchKernelGGL(eik::k_causal_corner<T>, dim3(1), dim3(eik::kCornerBlock), ldsB, s, A, U, W, dir,
                       res && dir == 3 ? 1 : 0);
  }
  hipLaunchKernelGGL(eik::k_causal_c<T>, dim3(nb), dim3(eik::kBlock), 0, s, A, U, 1, 1, res);
}

// the Step 4 weight options and the coarse solver choice
eik_status check_weight_solver(const eik_dd_opts* o) {
  if (o->coarse_solver != EIK_COARSE_GODUNOV && o->coarse_solver != EIK_COARSE_L1)
    return fail(EIK_ERR_ARG, "coarse_solver must be one of EIK_COARSE_*");
  if (o->theta_mode < EIK_THETA_CONSTANT || o->theta_mode > EIK_THETA_FIELD)
    return fail(EIK_ERR_ARG, "theta_mode must be one of EIK_THETA_*");
  if ((o->theta_mode == EIK_THETA_REFERENCE || o->theta_mode == EIK_THETA_FIELD) && !o->theta_ref)
    return fail(EIK_ERR_ARG, "theta_mode needs theta_ref");
  if (o->theta_mode == EIK_THETA_ESTIMATE) {
    const double* q = o->theta_params;
    if (!(q[0] > 0) || !std::isfinite(q[0]) || !std::isfinite(q[1]) || !std::isfinite(q[2]) ||
        !(q[3] >= 0 && q[4] >= 0 && q[5] >= 0) || !((q[3] + q[4]) + q[5] > 0))
      return fail(EIK_ERR_ARG, "theta_params: need gamma > 0, finite delta and x0, omegas >= 0 with a positive sum");
  }
  if (o->theta_mode == EIK_THETA_REFERENCE && !std::isfinite(o->theta_params[6]))
    return fail(EIK_ERR_ARG, "theta_params: margin must be finite");
  if (o->launch_mode < EIK_LAUNCH_STREAM || o->launch_mode > EIK_LAUNCH_PERSISTENT)
    return fail(EIK_ERR_ARG, "launch_mode must be one of EIK_LAUNCH_*");
  if (o->persistent_blocks < 0) return fail(EIK_ERR_ARG, "persistent_blocks must be >= 0");
  return EIK_OK;
}

template <typename T>
void set_theta(eik::ThetaPar& q, const eik_dd_opts* o) {
  q.gamma = o->theta_params[0];
  q.delta = o->theta_params[1];
  q.x0 = o->theta_params[2];
  q.w0 = o->theta_params[3];
  q.w1 = o->theta_params[4];
  q.w2 = o->theta_params[5];
  q.margin = o->theta_params[6];
}

// noalloc: take the workspace from the fixed scratch array and time nothing
// (eik_dd_solve_noalloc); the iteration and its kernels are the same.
template <typename T>
eik_status dd_solve_t(const eik_grid* G, const void* rv, const eik_gamma* gam, const eik_dd_opts* o,
                      void* u_outv, void* U_outv, int8_t* W_out, eik_stats* st, hipStream_t s,
                      bool noalloc = false) {
  const int n0 = (int)G->n[0], n1 = (int)G->n[1];
  const int S = o->S, M = o->M;
  if (M < 2 || S < M || S % M != 0) return fail(EIK_ERR_SHAPE, "need M >= 2 and S a multiple of M (S=%d M=%d)", S, M);
  if ((n0 - 1) % S != 0 || (n1 - 1) % S != 0)
    return fail(EIK_ERR_SHAPE, "(n-1) must be a multiple of S on every axis");
  if (S + 1 > eik::kMaxL) return fail(EIK_ERR_UNSUPPORTED, "subdomain side S+1 = %d > %d nodes", S + 1, eik::kMaxL);
  const int NI = (n0 - 1) / M, NJ = (n1 - 1) / M;
  if (NI + 1 > eik::kMaxL || NJ + 1 > eik::kMaxL)
    return fail(EIK_ERR_UNSUPPORTED, "coarse lattice extent > %d nodes", eik::kMaxL);
  if (!(o->theta >= 0.0 && o->theta <= 1.0)) return fail(EIK_ERR_ARG, "theta must lie in [0,1]");
  if (o->max_iter < 0 || o->max_fine_sweeps < 1 || o->max_coarse_sweeps < 1)
    return fail(EIK_ERR_ARG, "max_iter >= 0, max_fine_sweeps >= 1, max_coarse_sweeps >= 1");
  if ((o->U_init == nullptr) != (o->W_init == nullptr)) return fail(EIK_ERR_ARG, "U_init and W_init go together");
  const size_t szT = sizeof(T);
  const int L = S + 1;
  const size_t lds_tile = eik::tile_lds_bytes(L, szT);
  eik_status e = check_weight_solver(o);
  if (e != EIK_OK) return e;
  const int tmode = o->theta_mode;
  bool corr_packed = false, tglob = false;
  const size_t lds_lat = lattice_lds(NI, NJ, tmode, szT, corr_packed, tglob);
  const int nC = (NI + 1) * (NJ + 1);
  const size_t lds_cb = eik::corner_lds_bytes(NI + 1, NJ + 1, szT);
  if (lds_tile > kLdsBytes || lds_cb > kLdsBytes)
    return fail(EIK_ERR_UNSUPPORTED, "LDS footprint too large for this library");
  if (lds_lat > kLdsBytes)
    return fail(EIK_ERR_UNSUPPORTED, "coarse lattice of %d x %d nodes does not fit in LDS%s", NI + 1, NJ + 1,
                tmode ? " with a varying theta in this precision" : "");

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);

  const int64_t N = (int64_t)n0 * n1;
  const int P0 = (n0 - 1) / S, P1 = (n1 - 1) / S;
  const int ntile = P0 * P1;
  const int nH = NI * (NJ + 1), nV = (NI + 1) * NJ;
  size_t need = 0;
  need += 7 * (N * szT + 256);           // gfull U Un uk cwork + spare
  need += (N + 31) / 32 * 4 + 256;       // Gamma bit mask
  need += 6 * (N + 256);                 // W Wn wk cflag
  need += 2 * (N * 8 + 256);             // near keys
  need += ntile * 4 * L * (szT + 1) + 512;
  need += 3 * nC * szT + 2 * nC + (nH + nV) * (szT + 1) + 4096;
  need += 4096;
  if (tmode == EIK_THETA_ESTIMATE) need += 4 * (N * szT + 256);  // u^{k-1}, C^k, C^{k-1}, C^{k-2}
  const int tg_stride = eik::halo_count(NI + 1, NJ + 1);
  if (tglob) need += (size_t)(2 * M - 1) * 2 * tg_stride * sizeof(double) + 256;  // Step 4 weight terms
  void* wsv;
  unsigned long long* host;
  e = noalloc ? scratch_get(dev, need, &wsv, &host) : ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::DD2<T> A;
  std::memset(&A, 0, sizeof A);  // defined padding: the graph cache compares its bytes
  A.n0 = n0; A.n1 = n1; A.S = S; A.M = M; A.P0 = P0; A.P1 = P1; A.NI = NI; A.NJ = NJ;
  A.hT = (T)G->h;
  A.HT = (T)((double)M * G->h);
  A.theta = (T)o->theta;
  A.max_fine_sweeps = o->max_fine_sweeps;
  A.max_coarse_sweeps = o->max_coarse_sweeps;
  A.r = as<T>(rv);
  A.gidx = gam->idx;
  A.gval = as<T>(gam->g);
  A.ng = gam->count;
  T* gfull = cv.take<T>(N);
  A.gfull = gfull;
  uint32_t* gbits = cv.take<uint32_t>((N + 31) / 32);
  A.gbits = gbits;
  A.U = cv.take<T>(N);
  A.Un = cv.take<T>(N);
  A.uk = cv.take<T>(N);
  A.cwork = cv.take<T>(N);
  A.W = cv.take<uint8_t>(N);
  A.Wn = cv.take<uint8_t>(N);
  A.wk = cv.take<uint8_t>(N);
  A.cflag = cv.take<uint8_t>(N);
  A.near_key = cv.take<unsigned long long>(N);
  A.near_win = cv.take<long long>(N);
  A.edge_u = cv.take<T>((size_t)ntile * 4 * L);
  A.edge_w = cv.take<uint8_t>((size_t)ntile * 4 * L);
  A.ncx = cv.take<T>(nC);
  A.ncy = cv.take<T>(nC);
  A.cU = cv.take<T>(nC);
  A.cW = cv.take<uint8_t>(nC);
  A.cG = cv.take<uint8_t>(nC);
  A.hseg_p = cv.take<T>(std::max(nH, 1));
  A.hseg_l = cv.take<uint8_t>(std::max(nH, 1));
  A.vseg_p = cv.take<T>(std::max(nV, 1));
  A.vseg_l = cv.take<uint8_t>(std::max(nV, 1));
  A.counters = cv.take<unsigned long long>(8);
  A.sweep_prof = A.counters + 4;
  unsigned int* dflag = cv.take<unsigned int>(4);
  A.u_out = as<T>(u_outv);
  A.theta_mode = tmode;
  A.coarse_homog = o->coarse_solver;
  A.corr_packed = corr_packed ? 1 : 0;
  A.tglob = tglob ? cv.take<double>((size_t)(2 * M - 1) * 2 * tg_stride) : nullptr;
  A.tglob_stride = tglob ? tg_stride : 0;
  A.res_out = nullptr;   // set per DD iteration
  A.res_prev = nullptr;  // Step 1 always runs
  A.tol = o->tol;
  set_theta<T>(A.tq, o);
  A.tref = as<T>(o->theta_ref);
  A.ukm1 = A.ckm1 = A.ckm2 = nullptr;
  A.ck_out = nullptr;
  T* hist_u = nullptr;
  T* hist_c[3] = {nullptr, nullptr, nullptr};
  if (tmode == EIK_THETA_ESTIMATE) {
    hist_u = cv.take<T>(N);
    for (auto& c : hist_c) c = cv.take<T>(N);
  }

  if ((e = validate<T>(A.r, N, gam, dflag, host, s, G->h)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_tile<T>, lds_tile)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_lattice_init<T>, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_lattice_correct<T>, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_causal_corner<T>, lds_cb)) != EIK_OK) return e;

  Events<2> ev;
  EVCHK(ev.init(!noalloc));
  EVCHK(ev.rec(0, s));

  const T nanT = (T)NAN;
  const int bs = 256;
  HIPCHK(hipMemsetAsync(A.counters, 0, 8 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, gfull, nanT, N);
  HIPCHK(hipMemsetAsync(gbits, 0, (N + 31) / 32 * 4, s));
  if (gam->count > 0) {
    hipLaunchKernelGGL(eik::k_scatter_gamma<T>, dim3(nblocks(gam->count, bs)), dim3(bs), 0, s, gfull,
                       gam->idx, as<T>(gam->g), gam->count);
    hipLaunchKernelGGL(eik::k_gamma_bits, dim3(nblocks(gam->count, bs)), dim3(bs), 0, s, gbits, gam->idx,
                       gam->count);
  }
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.u_out, nanT, N);
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.uk, nanT, N);
  HIPCHK(hipMemsetAsync(A.wk, 0, N, s));
  HIPCHK(hipGetLastError());

  const int nlat = 2 * M - 1;
  float ms_fine = 0.f, ms_correct = 0.f, ms_causal = 0.f;
  if (o->U_init) {
    hipLaunchKernelGGL(eik::k_import_U<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A, as<T>(o->U_init), A.U);
    HIPCHK(hipMemcpyAsync(A.W, o->W_init, N, hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.U, nanT, N);
    HIPCHK(hipMemsetAsync(A.W, 0, N, s));
    HIPCHK(hipMemsetAsync(A.near_key, 0xff, N * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(eik::k_fill<long long>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.near_win,
                       (long long)0x7fffffffffffffffll, N);
    const int64_t W2 = 2 * M - 1;
    const int64_t npair = gam->count * W2 * W2;
    if (npair > 0) {
      hipLaunchKernelGGL(eik::k_near_a<T>, dim3(nblocks(npair, bs)), dim3(bs), 0, s, A);
      hipLaunchKernelGGL(eik::k_near_b<T>, dim3(nblocks(npair, bs)), dim3(bs), 0, s, A);
    }
    hipLaunchKernelGGL(eik::k_lattice_init<T>, dim3(nlat), dim3(eik::kBlock), lds_lat, s, A);
    causal_sweep(A, A.U, A.W, s, lds_cb, 0);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.Un, nanT, N);
  HIPCHK(hipMemsetAsync(A.Wn, 0, N, s));

  const eik_dd_debug* dbg = o->debug;
  int it = 0, conv = 0;
  double last = 0.0;
  // Iterations are launched up to `lag` ahead of the host's check of the
  // stopping rule; iteration k's residual goes to slot k % kSlots, and every
  // kernel of iteration k returns at once when iteration k-1 stopped (the
  // same rule, dd_stopped), so the launched-ahead iterations change nothing.
  // The debug snapshots are taken by plain copies: one iteration at a time.
  constexpr int kLag = 4, kSlots = 2 * kLag;
  static_assert(kSlots <= 8, "the pinned host buffer holds 8 words");
  const int lag = dbg ? 1 : kLag;
  unsigned long long* resid = cv.take<unsigned long long>(kSlots);
  HIPCHK(hipMemsetAsync(resid, 0, kSlots * sizeof(unsigned long long), s));
  A.tol = o->tol;
  Events<kLag * 4> evi;  // [iteration of the block][4]
  EVCHK(evi.init(!noalloc));
  // one DD iteration's launches on stream ls (timed: with the phase events)
  const int64_t nrec = (int64_t)(P0 - 1) * n1 + (int64_t)(P1 - 1) * n0;
  auto iteration = [&](int k, int E, bool timed, hipStream_t ls) -> eik_status {
    A.res_out = resid + k % kSlots;
    A.res_prev = k > 0 ? resid + (k - 1) % kSlots : nullptr;
    if (timed) EVCHK(evi.rec(E + 0, ls));
    hipLaunchKernelGGL(eik::k_tile<T>, dim3(ntile), dim3(eik::kBlock), lds_tile, ls, A);
    if (timed) EVCHK(evi.rec(E + 1, ls));
    if (nrec > 0) hipLaunchKernelGGL(eik::k_reconcile<T>, dim3(nblocks(nrec, bs)), dim3(bs), 0, ls, A);
    if (tmode == EIK_THETA_ESTIMATE) {
      // C^k goes to hist_c[k % 3]; the other two hold C^{k-1}, C^{k-2}
      A.ck_out = hist_c[k % 3];
      A.ckm1 = k >= 1 ? hist_c[(k + 2) % 3] : nullptr;
      A.ckm2 = k >= 2 ? hist_c[(k + 1) % 3] : nullptr;
      A.ukm1 = k >= 1 ? hist_u : nullptr;
    }
    hipLaunchKernelGGL(eik::k_lattice_correct<T>, dim3(nlat), dim3(eik::kBlock), lds_lat, ls, A);
    if (tmode == EIK_THETA_ESTIMATE) HIPCHK(hipMemcpyAsync(hist_u, A.uk, N * szT, hipMemcpyDeviceToDevice, ls));
    if (timed) EVCHK(evi.rec(E + 2, ls));
    if (dbg && dbg->U_pre_causal)
      HIPCHK(hipMemcpyAsync(dbg->U_pre_causal, A.Un, N * szT, hipMemcpyDeviceToDevice, ls));
    causal_sweep(A, A.Un, A.Wn, ls, lds_cb, 1);  // also the residual (resid slot, zeroed by k_tile)
    HIPCHK(hipGetLastError());
    if (timed) EVCHK(evi.rec(E + 3, ls));
    std::swap(A.U, A.Un);
    std::swap(A.W, A.Wn);
    return EIK_OK;
  };
  // EIK_LAUNCH_GRAPH: whole blocks after the first one replay a graph of the
  // block's launches (A is the same at the start of every block: an even
  // number of swaps; the residual slots depend on the block's parity)
  const bool use_graph = o->launch_mode == EIK_LAUNCH_GRAPH && !noalloc && !dbg && tmode != EIK_THETA_ESTIMATE;
  auto graph_block = [&](int k0) -> eik_status {
    DDGraph& g = g_ddgraph[dev][(k0 / kLag) & 1];
    const int shape[6] = {ntile, nlat, (int)lds_tile, (int)lds_lat, (int)lds_cb, (k0 / kLag) & 1};
    std::vector<unsigned char> key(sizeof A + sizeof shape + sizeof resid);
    std::memcpy(key.data(), &A, sizeof A);
    std::memcpy(key.data() + sizeof A, shape, sizeof shape);
    std::memcpy(key.data() + sizeof A + sizeof shape, &resid, sizeof resid);
    if (g.exec == nullptr || g.key != key) {
      if (g.exec) {
        HIPCHK(hipGraphExecDestroy(g.exec));
        g.exec = nullptr;
      }
      if (!g_capture_stream[dev]) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
      hipStream_t cs = g_capture_stream[dev];
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      eik_status ce = EIK_OK;
      for (int k = k0; k < k0 + kLag && ce == EIK_OK; ++k) ce = iteration(k, 0, false, cs);
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(cs, &graph);
      if (ce != EIK_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return ce;
      }
      HIPCHK(ee);
      const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(ie);
      g.key = key;
    } else {
      // the host-side effect of the block's iterations: none (even swaps)
    }
    HIPCHK(hipGraphLaunch(g.exec, s));
    return EIK_OK;
  };
  int launched = 0;
  bool done = false;
  while (!done && launched < o->max_iter) {
    const int k0 = launched, k1 = std::min(o->max_iter, k0 + lag);
    const bool timed = !(use_graph && k0 > 0 && k1 - k0 == kLag);
    if (timed) {
      for (int k = k0; k < k1; ++k) EVCHK(iteration(k, (k - k0) * 4, true, s));
    } else {
      EVCHK(graph_block(k0));
    }
    launched = k1;
    HIPCHK(hipMemcpyAsync(host, resid, kSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // the host's stopping rule on the iterations of this block, in order
    for (int k = k0; k < k1; ++k) {
      float a = 0.f, b = 0.f, c = 0.f;
      const int E = (k - k0) * 4;
      if (timed) {
        EVCHK(evi.ms(E + 0, E + 1, &a));
        EVCHK(evi.ms(E + 1, E + 2, &b));
        EVCHK(evi.ms(E + 2, E + 3, &c));
      }
      ms_fine += a;
      ms_correct += b;
      ms_causal += c;
      double delta;
      std::memcpy(&delta, &host[k % kSlots], sizeof delta);
      it = k + 1;
      last = delta;
      if (st && st->residual_history && k < st->history_cap) st->residual_history[k] = delta;
      if (std::isnan(delta)) return fail(EIK_ERR_NONFINITE, "residual is NaN");
      if (delta < o->tol || delta == 0.0) {
        conv = 1;
        done = true;
        break;
      }
    }
  }
  // U^it and W^it are where the it-th iteration put them: undo the swap of
  // an odd number of launched-ahead iterations
  if ((launched - it) % 2) {
    std::swap(A.U, A.Un);
    std::swap(A.W, A.Wn);
  }
  if (U_outv) hipLaunchKernelGGL(eik::k_export_U<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A, A.U, as<T>(U_outv));
  if (W_out) HIPCHK(hipMemcpyAsync(W_out, A.W, N, hipMemcpyDeviceToDevice, s));
  if (dbg && dbg->uk) HIPCHK(hipMemcpyAsync(dbg->uk, A.uk, N * szT, hipMemcpyDeviceToDevice, s));
  if (dbg && dbg->wk) HIPCHK(hipMemcpyAsync(dbg->wk, A.wk, N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(host, A.counters, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  EVCHK(ev.rec(1, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  if (st) {
    float tot = 0.f;
    EVCHK(ev.ms(0, 1, &tot));
    st->iterations = it;
    st->converged = conv;
    st->fine_updates = (int64_t)host[0];
    st->coarse_updates = (int64_t)host[1];
    st->sweeps = 0;
    st->final_residual = last;
    st->ms_total = tot;
    st->ms_fine = ms_fine;
    st->ms_coarse = tot - ms_fine;
    st->ms_correct = ms_correct;
    st->ms_causal = ms_causal;
    for (int q = 0; q < 2; ++q) {
      st->lead_steps[q] = (int64_t)host[4 + 2 * q];
      st->lead_ticks[q] = (int64_t)host[5 + 2 * q];
    }
  }
  if (host[3]) return fail(EIK_ERR_INTERNAL, "a wait between the two waves of a box sweep gave up");
  if (o->max_iter > 0 && !conv) return fail(EIK_ERR_NOCONV, "no convergence in %d iterations (residual %g)", it, last);
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// eik_dd_solve_batch, d = 2: many independent problems, every DD step one
// launch over the subdomains / lattices / segments of all active problems
// ---------------------------------------------------------------------------

template <typename T>
struct BatchProb {
  eik::DD2<T> A;
  int ntile = 0, nlat = 0, nC = 0, nH = 0, nV = 0;
  int64_t N = 0, nrec = 0, npair = 0;
  size_t lds_tile = 0, lds_lat = 0, lds_cb = 0;
  int tmode = 0;
  bool corr_packed = false;  // Step 4's CorrPack records (lattice_lds)
  bool tglob = false;        // Step 4's weight terms in global memory (lattice_lds)
  T* hist_u = nullptr;
  T* hist_c[3] = {nullptr, nullptr, nullptr};
  T* gfull = nullptr;
  uint32_t* gbits = nullptr;
  bool active = true, conv = false, resumed = false;
  int it = 0;
  double last = 0.0;
  unsigned long long* counters = nullptr;
};

// work table: (problem, block) for every block of every selected problem
template <typename F>
static void build_work(std::vector<int2>& out, int P, F blocks_of) {
  out.clear();
  for (int p = 0; p < P; ++p) {
    const int64_t nb = blocks_of(p);
    for (int64_t b = 0; b < nb; ++b) out.push_back(make_int2(p, (int)b));
  }
}

template <typename T>
eik_status dd_solve_batch_t(int P, const eik_grid* G, const void* const* rv, const eik_gamma* gam,
                            const eik_dd_opts* o, void* const* u_out, void* const* U_out, int8_t* const* W_out,
                            eik_stats* st, hipStream_t s) {
  const size_t szT = sizeof(T);
  const int bs = 256;
  std::vector<BatchProb<T>> pr(P);
  size_t need = 4096 + (size_t)P * (sizeof(eik::DD2<T>) + 4 * 8) + 512;
  int64_t tot_tile = 0, tot_lat = 0, tot_rec = 0, tot_cc = 0;
  size_t lds_tile = 0, lds_lat = 0, lds_cb = 0;
  for (int p = 0; p < P; ++p) {
    const eik_dd_opts* op = &o[p];
    BatchProb<T>& q = pr[p];
    const int n0 = (int)G[p].n[0], n1 = (int)G[p].n[1];
    const int S = op->S, M = op->M;
    if (G[p].dim != 2) return fail(EIK_ERR_UNSUPPORTED, "batch: problem %d is not 2D", p);
    if (G[p].dtype != G[0].dtype) return fail(EIK_ERR_ARG, "batch: all problems need the same dtype");
    if (M < 2 || S < M || S % M != 0) return fail(EIK_ERR_SHAPE, "problem %d: need M >= 2 and S a multiple of M", p);
    if ((n0 - 1) % S != 0 || (n1 - 1) % S != 0) return fail(EIK_ERR_SHAPE, "problem %d: (n-1) %% S != 0", p);
    if (S + 1 > eik::kMaxL) return fail(EIK_ERR_UNSUPPORTED, "problem %d: S+1 > %d", p, eik::kMaxL);
    const int NI = (n0 - 1) / M, NJ = (n1 - 1) / M;
    if (NI + 1 > eik::kMaxL || NJ + 1 > eik::kMaxL)
      return fail(EIK_ERR_UNSUPPORTED, "problem %d: coarse lattice extent > %d nodes", p, eik::kMaxL);
    if (!(op->theta >= 0.0 && op->theta <= 1.0)) return fail(EIK_ERR_ARG, "problem %d: theta outside [0,1]", p);
    if (op->max_iter < 0 || op->max_fine_sweeps < 1 || op->max_coarse_sweeps < 1)
      return fail(EIK_ERR_ARG, "problem %d: bad iteration or sweep caps", p);
    if ((op->U_init == nullptr) != (op->W_init == nullptr))
      return fail(EIK_ERR_ARG, "problem %d: U_init and W_init go together", p);
    if (op->debug) return fail(EIK_ERR_ARG, "problem %d: debug snapshots are not available in a batch", p);
    eik_status e = check_weight_solver(op);
    if (e != EIK_OK) return e;
    if (!rv[p] || !u_out[p] || rv[p] == u_out[p]) return fail(EIK_ERR_ARG, "problem %d: bad r / u_out", p);
    q.tmode = op->theta_mode;
    const int L = S + 1;
    q.lds_tile = eik::tile_lds_bytes(L, szT);
    q.lds_lat = lattice_lds(NI, NJ, q.tmode, szT, q.corr_packed, q.tglob);
    q.lds_cb = eik::corner_lds_bytes(NI + 1, NJ + 1, szT);
    if (q.lds_tile > kLdsBytes || q.lds_lat > kLdsBytes || q.lds_cb > kLdsBytes)
      return fail(EIK_ERR_UNSUPPORTED, "problem %d: LDS footprint too large", p);
    lds_tile = std::max(lds_tile, q.lds_tile);
    lds_lat = std::max(lds_lat, q.lds_lat);
    lds_cb = std::max(lds_cb, q.lds_cb);
    q.N = (int64_t)n0 * n1;
    const int P0 = (n0 - 1) / S, P1 = (n1 - 1) / S;
    q.ntile = P0 * P1;
    q.nlat = 2 * M - 1;
    q.nC = (NI + 1) * (NJ + 1);
    q.nH = NI * (NJ + 1);
    q.nV = (NI + 1) * NJ;
    q.nrec = (int64_t)(P0 - 1) * n1 + (int64_t)(P1 - 1) * n0;
    q.npair = gam[p].count * (int64_t)(2 * M - 1) * (2 * M - 1);
    q.resumed = op->U_init != nullptr;
    size_t nd = 0;
    nd += 7 * (q.N * szT + 256);
    nd += (q.N + 31) / 32 * 4 + 256;  // Gamma bit mask
    nd += 6 * (q.N + 256);
    nd += 2 * (q.N * 8 + 256);
    nd += (size_t)q.ntile * 4 * L * (szT + 1) + 512;
    nd += 3 * q.nC * szT + 2 * q.nC + (q.nH + q.nV) * (szT + 1) + 4096;
    if (q.tmode == EIK_THETA_ESTIMATE) nd += 4 * (q.N * szT + 256);
    if (q.tglob) nd += (size_t)q.nlat * 2 * eik::halo_count(NI + 1, NJ + 1) * sizeof(double) + 256;
    need += nd;
    tot_tile += q.ntile;
    tot_lat += q.nlat;
    tot_rec += nblocks(q.nrec, bs);
    tot_cc += nblocks(q.nH + q.nV, bs / (M - 1)) + nblocks(q.nC, bs);  // = causal_blocks(q.A)
  }
  int64_t tot_near = 0;
  for (int p = 0; p < P; ++p) tot_near += nblocks(pr[p].npair, bs);
  const int64_t tot_work = tot_tile + tot_lat + tot_rec + tot_cc + P + tot_near;
  need += (size_t)tot_work * sizeof(int2) + 8 * 256;

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::DD2<T>* d_desc = cv.take<eik::DD2<T>>(P);
  unsigned long long* d_cnt = cv.take<unsigned long long>(4 * (size_t)P);
  unsigned int* dflag = cv.take<unsigned int>(4);
  // one device table per kind of launch, sized for all problems
  // capacities: the tables of all problems (later tables hold a subset)
  const int64_t cap_tile = std::max<int64_t>(tot_tile, 1), cap_lat = std::max<int64_t>(tot_lat, 1),
                cap_rec = std::max<int64_t>(tot_rec, 1),
                cap_cc = std::max<int64_t>(tot_cc, 1), cap_near = std::max<int64_t>(tot_near, 1);
  int2* w_tile = cv.take<int2>(cap_tile);
  int2* w_lat = cv.take<int2>(cap_lat);
  int2* w_rec = cv.take<int2>(cap_rec);
  int2* w_cc = cv.take<int2>(cap_cc);
  int2* w_cb = cv.take<int2>(P);
  int2* w_near = cv.take<int2>(cap_near);
  int* d_next = cv.take<int>(2);  // EIK_LAUNCH_PERSISTENT: item counters of Steps 3 and 4
  for (int p = 0; p < P; ++p) {
    BatchProb<T>& q = pr[p];
    const eik_dd_opts* op = &o[p];
    eik::DD2<T>& A = q.A;
    const int n0 = (int)G[p].n[0], n1 = (int)G[p].n[1];
    const int S = op->S, M = op->M, L = S + 1;
    const int64_t N = q.N;
    A.n0 = n0; A.n1 = n1; A.S = S; A.M = M; A.P0 = (n0 - 1) / S; A.P1 = (n1 - 1) / S;
    A.NI = (n0 - 1) / M; A.NJ = (n1 - 1) / M;
    A.hT = (T)G[p].h;
    A.HT = (T)((double)M * G[p].h);
    A.theta = (T)op->theta;
    A.max_fine_sweeps = op->max_fine_sweeps;
    A.max_coarse_sweeps = op->max_coarse_sweeps;
    A.r = as<T>(rv[p]);
    A.gidx = gam[p].idx;
    A.gval = as<T>(gam[p].g);
    A.ng = gam[p].count;
    q.gfull = cv.take<T>(N);
    A.gfull = q.gfull;
    q.gbits = cv.take<uint32_t>((N + 31) / 32);
    A.gbits = q.gbits;
    A.U = cv.take<T>(N);
    A.Un = cv.take<T>(N);
    A.uk = cv.take<T>(N);
    A.cwork = cv.take<T>(N);
    A.W = cv.take<uint8_t>(N);
    A.Wn = cv.take<uint8_t>(N);
    A.wk = cv.take<uint8_t>(N);
    A.cflag = cv.take<uint8_t>(N);
    A.near_key = cv.take<unsigned long long>(N);
    A.near_win = cv.take<long long>(N);
    A.edge_u = cv.take<T>((size_t)q.ntile * 4 * L);
    A.edge_w = cv.take<uint8_t>((size_t)q.ntile * 4 * L);
    A.ncx = cv.take<T>(q.nC);
    A.ncy = cv.take<T>(q.nC);
    A.cU = cv.take<T>(q.nC);
    A.cW = cv.take<uint8_t>(q.nC);
    A.cG = cv.take<uint8_t>(q.nC);
    A.hseg_p = cv.take<T>(std::max(q.nH, 1));
    A.hseg_l = cv.take<uint8_t>(std::max(q.nH, 1));
    A.vseg_p = cv.take<T>(std::max(q.nV, 1));
    A.vseg_l = cv.take<uint8_t>(std::max(q.nV, 1));
    A.counters = d_cnt + 4 * (size_t)p;
    A.sweep_prof = nullptr;
    A.u_out = as<T>(u_out[p]);
    A.theta_mode = q.tmode;
    A.coarse_homog = op->coarse_solver;
    A.corr_packed = q.corr_packed ? 1 : 0;
    const int tg_stride = eik::halo_count(A.NI + 1, A.NJ + 1);
    A.tglob = q.tglob ? cv.take<double>((size_t)q.nlat * 2 * tg_stride) : nullptr;
    A.tglob_stride = q.tglob ? tg_stride : 0;
    A.res_out = A.counters + 2;  // read back after every iteration
    A.res_prev = nullptr;        // the batch checks on the host
    A.tol = op->tol;
    set_theta<T>(A.tq, op);
    A.tref = as<T>(op->theta_ref);
    A.ukm1 = A.ckm1 = A.ckm2 = nullptr;
    A.ck_out = nullptr;
    if (q.tmode == EIK_THETA_ESTIMATE) {
      q.hist_u = cv.take<T>(N);
      for (auto& c : q.hist_c) c = cv.take<T>(N);
    }
    if ((e = validate<T>(A.r, N, &gam[p], dflag, host, s, G[p].h)) != EIK_OK) return e;
  }
  if ((e = allow_lds(eik::k_tile_b<T>, lds_tile)) != EIK_OK) return e;
  // EIK_LAUNCH_PERSISTENT (o[0]): Steps 3 and 4 on as many blocks as are
  // resident at once, each taking items from a counter
  const bool persistent = o[0].launch_mode == EIK_LAUNCH_PERSISTENT;
  int64_t grid_tile = 0, grid_lat = 0;
  if (persistent) {
    int ncu = 0, bt = 0, bl = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bt, eik::k_tile_b<T>, eik::kBlock, lds_tile));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bl, eik::k_lattice_correct_b<T>, eik::kBlock, lds_lat));
    if (o[0].persistent_blocks > 0) {
      bt = std::min(bt, o[0].persistent_blocks);
      bl = std::min(bl, o[0].persistent_blocks);
    }
    grid_tile = (int64_t)std::max(1, bt) * ncu;
    grid_lat = (int64_t)std::max(1, bl) * ncu;
  }
  if ((e = allow_lds(eik::k_lattice_init_b<T>, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_lattice_correct_b<T>, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_causal_corner_b<T>, lds_cb)) != EIK_OK) return e;

  hipEvent_t ev[5];
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]); }
  } evg{ev};
  HIPCHK(hipEventRecord(ev[0], s));
  const T nanT = (T)NAN;
  HIPCHK(hipMemsetAsync(d_cnt, 0, 4 * (size_t)P * sizeof(unsigned long long), s));
  std::vector<eik::DD2<T>> hdesc(P);
  auto upload_desc = [&]() -> eik_status {
    for (int p = 0; p < P; ++p) hdesc[p] = pr[p].A;
    HIPCHK(hipMemcpyAsync(d_desc, hdesc.data(), (size_t)P * sizeof(eik::DD2<T>), hipMemcpyHostToDevice, s));
    return EIK_OK;
  };
  std::vector<int2> tab;
  auto upload = [&](int2* dst, int64_t cap, std::vector<int2>& v) -> eik_status {
    if ((int64_t)v.size() > cap) return fail(EIK_ERR_HIP, "batch: work table larger than its buffer (internal)");
    if (!v.empty()) HIPCHK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // the host vector is reused
    return EIK_OK;
  };
  // per-problem set-up (as in the single solve)
  for (int p = 0; p < P; ++p) {
    eik::DD2<T>& A = pr[p].A;
    const int64_t N = pr[p].N;
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, pr[p].gfull, nanT, N);
    HIPCHK(hipMemsetAsync(pr[p].gbits, 0, (N + 31) / 32 * 4, s));
    if (gam[p].count > 0) {
      hipLaunchKernelGGL(eik::k_scatter_gamma<T>, dim3(nblocks(gam[p].count, bs)), dim3(bs), 0, s, pr[p].gfull,
                         gam[p].idx, as<T>(gam[p].g), gam[p].count);
      hipLaunchKernelGGL(eik::k_gamma_bits, dim3(nblocks(gam[p].count, bs)), dim3(bs), 0, s, pr[p].gbits,
                         gam[p].idx, gam[p].count);
    }
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.u_out, nanT, N);
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.uk, nanT, N);
    HIPCHK(hipMemsetAsync(A.wk, 0, N, s));
    if (pr[p].resumed) {
      hipLaunchKernelGGL(eik::k_import_U<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A, as<T>(o[p].U_init), A.U);
      HIPCHK(hipMemcpyAsync(A.W, o[p].W_init, N, hipMemcpyDeviceToDevice, s));
    } else {
      hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.U, nanT, N);
      HIPCHK(hipMemsetAsync(A.W, 0, N, s));
      HIPCHK(hipMemsetAsync(A.near_key, 0xff, N * sizeof(unsigned long long), s));
      hipLaunchKernelGGL(eik::k_fill<long long>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.near_win,
                         (long long)0x7fffffffffffffffll, N);
    }
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.Un, nanT, N);
    HIPCHK(hipMemsetAsync(A.Wn, 0, N, s));
  }
  HIPCHK(hipGetLastError());
  if ((e = upload_desc()) != EIK_OK) return e;
  // Step 1 for the problems that do not resume
  auto fresh = [&](int p) { return !pr[p].resumed; };
  build_work(tab, P, [&](int p) { return fresh(p) ? (int64_t)nblocks(pr[p].npair, bs) : 0; });
  if (!tab.empty()) {
    if ((e = upload(w_near, cap_near, tab)) != EIK_OK) return e;
    hipLaunchKernelGGL(eik::k_near_a_b<T>, dim3(tab.size()), dim3(bs), 0, s, d_desc, w_near);
    hipLaunchKernelGGL(eik::k_near_b_b<T>, dim3(tab.size()), dim3(bs), 0, s, d_desc, w_near);
  }
  int64_t tot_cb = 0;
  auto causal_batch = [&](int which) -> eik_status {
    // tables of the selected problems: w_cc, causal_blocks() segment blocks
    // per problem (kBlock == bs); w_cb, one corner block per problem
    for (int dir = 0; dir < 4; ++dir) {
      hipLaunchKernelGGL(eik::k_causal_seg_b<T>, dim3((unsigned)tot_cc), dim3(eik::kBlock), 0, s, d_desc, w_cc,
                         which, dir, dir - 1);
      hipLaunchKernelGGL(eik::k_causal_corner_b<T>, dim3((unsigned)tot_cb), dim3(eik::kCornerBlock), lds_cb, s,
                         d_desc, w_cb, which, dir);
    }
    hipLaunchKernelGGL(eik::k_causal_c_b<T>, dim3((unsigned)tot_cc), dim3(eik::kBlock), 0, s, d_desc, w_cc, which, 1, 1);
    HIPCHK(hipGetLastError());
    return EIK_OK;
  };
  auto set_tables = [&](auto sel) -> eik_status {
    eik_status ee;
    build_work(tab, P, [&](int p) { return sel(p) ? (int64_t)pr[p].ntile : 0; });
    tot_tile = (int64_t)tab.size();
    if ((ee = upload(w_tile, cap_tile, tab)) != EIK_OK) return ee;
    build_work(tab, P, [&](int p) { return sel(p) ? (int64_t)pr[p].nlat : 0; });
    tot_lat = (int64_t)tab.size();
    if ((ee = upload(w_lat, cap_lat, tab)) != EIK_OK) return ee;
    build_work(tab, P, [&](int p) { return sel(p) ? (int64_t)nblocks(pr[p].nrec, bs) : 0; });
    tot_rec = (int64_t)tab.size();
    if ((ee = upload(w_rec, cap_rec, tab)) != EIK_OK) return ee;
    build_work(tab, P, [&](int p) { return sel(p) ? (int64_t)eik::causal_blocks(pr[p].A) : 0; });
    tot_cc = (int64_t)tab.size();
    if ((ee = upload(w_cc, cap_cc, tab)) != EIK_OK) return ee;
    build_work(tab, P, [&](int p) { return sel(p) ? (int64_t)1 : 0; });
    tot_cb = (int64_t)tab.size();
    if ((ee = upload(w_cb, (int64_t)P, tab)) != EIK_OK) return ee;
    return EIK_OK;
  };
  if ((e = set_tables(fresh)) != EIK_OK) return e;
  if (tot_lat > 0) {
    hipLaunchKernelGGL(eik::k_lattice_init_b<T>, dim3((unsigned)tot_lat), dim3(eik::kBlock), lds_lat, s, d_desc, w_lat);
    if ((e = causal_batch(0)) != EIK_OK) return e;
  }
  // the DD iteration
  int max_iter = 0;
  for (int p = 0; p < P; ++p) {
    max_iter = std::max(max_iter, o[p].max_iter);
    pr[p].active = o[p].max_iter > 0;
  }
  auto is_active = [&](int p) { return pr[p].active; };
  if ((e = set_tables(is_active)) != EIK_OK) return e;
  std::vector<unsigned long long> hc(4 * (size_t)P);
  float ms_fine = 0.f, ms_correct = 0.f, ms_causal = 0.f;
  eik_status bad = EIK_OK;
  for (int k = 0; k < max_iter && tot_tile > 0; ++k) {
    for (int p = 0; p < P; ++p) {
      BatchProb<T>& q = pr[p];
      if (!q.active || q.tmode != EIK_THETA_ESTIMATE) continue;
      q.A.ck_out = q.hist_c[k % 3];
      q.A.ckm1 = k >= 1 ? q.hist_c[(k + 2) % 3] : nullptr;
      q.A.ckm2 = k >= 2 ? q.hist_c[(k + 1) % 3] : nullptr;
      q.A.ukm1 = k >= 1 ? q.hist_u : nullptr;
    }
    if ((e = upload_desc()) != EIK_OK) return e;
    HIPCHK(hipEventRecord(ev[1], s));
    if (persistent) {
      HIPCHK(hipMemsetAsync(d_next, 0, 2 * sizeof(int), s));
      hipLaunchKernelGGL(eik::k_tile_b<T>, dim3((unsigned)std::min<int64_t>(tot_tile, grid_tile)), dim3(eik::kBlock),
                         lds_tile, s, d_desc, w_tile, (int)tot_tile, d_next);
    } else {
      hipLaunchKernelGGL(eik::k_tile_b<T>, dim3((unsigned)tot_tile), dim3(eik::kBlock), lds_tile, s, d_desc, w_tile,
                         (int)tot_tile, (int*)nullptr);
    }
    HIPCHK(hipEventRecord(ev[2], s));
    if (tot_rec > 0)
      hipLaunchKernelGGL(eik::k_reconcile_b<T>, dim3((unsigned)tot_rec), dim3(bs), 0, s, d_desc, w_rec);
    if (persistent) {
      hipLaunchKernelGGL(eik::k_lattice_correct_b<T>, dim3((unsigned)std::min<int64_t>(tot_lat, grid_lat)),
                         dim3(eik::kBlock), lds_lat, s, d_desc, w_lat, (int)tot_lat, d_next + 1);
    } else {
      hipLaunchKernelGGL(eik::k_lattice_correct_b<T>, dim3((unsigned)tot_lat), dim3(eik::kBlock), lds_lat, s, d_desc,
                         w_lat, (int)tot_lat, (int*)nullptr);
    }
    for (int p = 0; p < P; ++p)
      if (pr[p].active && pr[p].tmode == EIK_THETA_ESTIMATE)
        HIPCHK(hipMemcpyAsync(pr[p].hist_u, pr[p].A.uk, pr[p].N * szT, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipEventRecord(ev[3], s));
    // the sweep of U^{k+1} also takes each problem's residual (counters[2],
    // zeroed by the problem's k_tile)
    if ((e = causal_batch(1)) != EIK_OK) return e;
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[4], s));
    HIPCHK(hipMemcpyAsync(hc.data(), d_cnt, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float a = 0.f, b = 0.f, c = 0.f;
    HIPCHK(hipEventElapsedTime(&a, ev[1], ev[2]));
    HIPCHK(hipEventElapsedTime(&b, ev[2], ev[3]));
    HIPCHK(hipEventElapsedTime(&c, ev[3], ev[4]));
    ms_fine += a;
    ms_correct += b;
    ms_causal += c;
    bool changed_set = false;
    for (int p = 0; p < P; ++p) {
      BatchProb<T>& q = pr[p];
      if (!q.active) continue;
      double delta;
      std::memcpy(&delta, &hc[4 * (size_t)p + 2], sizeof delta);
      std::swap(q.A.U, q.A.Un);
      std::swap(q.A.W, q.A.Wn);
      q.it = k + 1;
      q.last = delta;
      if (st && st[p].residual_history && k < st[p].history_cap) st[p].residual_history[k] = delta;
      bool stop = false;
      if (std::isnan(delta)) {
        bad = fail(EIK_ERR_NONFINITE, "problem %d: residual is NaN", p);
        stop = true;
      } else if (delta < o[p].tol || delta == 0.0) {
        q.conv = true;
        stop = true;
      } else if (q.it >= o[p].max_iter) {
        stop = true;
      }
      if (stop) {
        q.active = false;
        changed_set = true;
      }
    }
    if (changed_set && (e = set_tables(is_active)) != EIK_OK) return e;
  }
  // outputs
  for (int p = 0; p < P; ++p) {
    eik::DD2<T>& A = pr[p].A;
    if (U_out && U_out[p])
      hipLaunchKernelGGL(eik::k_export_U<T>, dim3(nblocks(pr[p].N, bs)), dim3(bs), 0, s, A, A.U, as<T>(U_out[p]));
    if (W_out && W_out[p]) HIPCHK(hipMemcpyAsync(W_out[p], A.W, pr[p].N, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(hc.data(), d_cnt, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(ev[4], s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  float tot = 0.f;
  HIPCHK(hipEventElapsedTime(&tot, ev[0], ev[4]));
  bool all_conv = true;
  for (int p = 0; p < P; ++p) {
    const bool conv = pr[p].conv || o[p].max_iter == 0;
    all_conv = all_conv && conv;
    if (!st) continue;
    st[p].iterations = pr[p].it;
    st[p].converged = pr[p].conv ? 1 : 0;
    st[p].fine_updates = (int64_t)hc[4 * (size_t)p + 0];
    st[p].coarse_updates = (int64_t)hc[4 * (size_t)p + 1];
    st[p].sweeps = 0;
    st[p].final_residual = pr[p].last;
    st[p].ms_total = tot;
    st[p].ms_fine = ms_fine;
    st[p].ms_coarse = tot - ms_fine;
    st[p].ms_correct = ms_correct;
    st[p].ms_causal = ms_causal;
  }
  if (bad != EIK_OK) return bad;
  for (int p = 0; p < P; ++p)
    if (hc[4 * (size_t)p + 3]) return fail(EIK_ERR_INTERNAL, "a wait between the two waves of a box sweep gave up");
  if (!all_conv) return fail(EIK_ERR_NOCONV, "some problems did not converge within max_iter");
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// eik_dd_solve, d = 3
// ---------------------------------------------------------------------------

// number of coarse cells (in sweep coordinates) on anti-diagonal d
static int cells_on_diag(const int CN[3], int d) {
  int c = 0;
  for (int i = std::max(0, d - (CN[1] - 1) - (CN[2] - 1)); i <= std::min(d, CN[0] - 1); ++i) {
    const int r2 = d - i;
    const int jlo = std::max(0, r2 - (CN[2] - 1)), jhi = std::min(r2, CN[1] - 1);
    if (jhi >= jlo) c += jhi - jlo + 1;
  }
  return c;
}

// The 3D causal sweep (k_causal3p): the (direction, cell) items in the order
// of a coarse-cell wavefront schedule, listed once per solve; directions
// 4m .. 4m+3 interleaved, each behind the one before by the diagonals its
// reversed axes need (z: CN2 + 1; y and z: CN1 + CN2); the kernel waits per
// item for the cells it depends on.
struct Causal3Plan {
  int* items = nullptr;  // device: dir | C0 << 3 | C1 << 9 | C2 << 15, in schedule order
  int nitems = 0;
  int* done = nullptr;   // device: [8][cells] epoch of the sweep that finished the cell
  int* abort_flag = nullptr;
  int blocks = 0, threads = 0, per_cu = 0;
  size_t lds = 0;
  int epoch = 0;
};

template <typename T>
std::vector<int> causal3_items(const eik::DD3<T>& A) {
  const int CN[3] = {A.NC[0] + 1, A.NC[1] + 1, A.NC[2] + 1};
  const int ndiag = CN[0] + CN[1] + CN[2] - 2;
  const int off[4] = {0, CN[2] + 1, CN[2] + 1 + CN[1] + CN[2], 2 * (CN[2] + 1) + CN[1] + CN[2]};
  std::vector<int> items;
  for (int m = 0; m < 2; ++m)
    for (int tau = 0; tau < off[3] + ndiag; ++tau)
      for (int k = 0; k < 4; ++k) {
        const int d = tau - off[k];
        if (d < 0 || d >= ndiag) continue;
        const int dir = 4 * m + k;
        for (int i = std::max(0, d - (CN[1] - 1) - (CN[2] - 1)); i <= std::min(d, CN[0] - 1); ++i) {
          const int r2 = d - i;
          for (int j = std::max(0, r2 - (CN[2] - 1)); j <= std::min(r2, CN[1] - 1); ++j) {
            const int kk = r2 - j;
            const int C0 = (dir & 4) ? i : CN[0] - 1 - i, C1 = (dir & 2) ? j : CN[1] - 1 - j,
                      C2 = (dir & 1) ? kk : CN[2] - 1 - kk;
            items.push_back(dir | (C0 << 3) | (C1 << 9) | (C2 << 15));
          }
        }
      }
  return items;
}

template <typename T>
void causal_sweep3p(eik::DD3<T>& A, T* U, const uint8_t* W, Causal3Plan& P, hipStream_t s) {
  ++P.epoch;
  hipLaunchKernelGGL(eik::k_causal3p<T>, dim3(P.blocks), dim3(P.threads), P.lds, s, A, U, W, P.items, P.nitems,
                     P.done, P.epoch, P.abort_flag);
}

template <typename T>
eik_status dd_solve3_t(const eik_grid* G, const void* rv, const eik_gamma* gam, const eik_dd_opts* o,
                       void* u_outv, void* U_outv, int8_t* W_out, eik_stats* st, hipStream_t s) {
  int n[3];
  for (int a = 0; a < 3; ++a) n[a] = (int)G->n[a];
  const int S = o->S, M = o->M;
  if (M < 2 || S < M || S % M != 0) return fail(EIK_ERR_SHAPE, "need M >= 2 and S a multiple of M (S=%d M=%d)", S, M);
  for (int a = 0; a < 3; ++a)
    if ((n[a] - 1) % S != 0) return fail(EIK_ERR_SHAPE, "(n-1) must be a multiple of S on every axis");
  const size_t szT = sizeof(T);
  const int L = S + 1;
  int NC[3], P[3];
  for (int a = 0; a < 3; ++a) { NC[a] = (n[a] - 1) / M; P[a] = (n[a] - 1) / S; }
  const int Lmax = std::max(NC[0], std::max(NC[1], NC[2])) + 1;
  if (L > eik::kMaxL3 || Lmax > eik::kMaxL3)
    return fail(EIK_ERR_UNSUPPORTED, "3D boxes are limited to %d nodes per axis", eik::kMaxL3);
  const size_t lds_tile = (size_t)L * L * L * szT;
  const size_t lds_lat = (size_t)(NC[0] + 1) * (NC[1] + 1) * (NC[2] + 1) * szT;
  const size_t lds_cell = eik::causal3_lds<T>(M);
  if (lds_tile > kLdsBytes || lds_lat > kLdsBytes || lds_cell > kLdsBytes)
    return fail(EIK_ERR_UNSUPPORTED, "3D box does not fit in LDS in this precision");
  if (!(o->theta >= 0.0 && o->theta <= 1.0)) return fail(EIK_ERR_ARG, "theta must lie in [0,1]");
  if (o->max_iter < 0 || o->max_fine_sweeps < 1 || o->max_coarse_sweeps < 1)
    return fail(EIK_ERR_ARG, "max_iter >= 0, max_fine_sweeps >= 1, max_coarse_sweeps >= 1");
  if ((o->U_init == nullptr) != (o->W_init == nullptr)) return fail(EIK_ERR_ARG, "U_init and W_init go together");
  {
    const eik_status et = check_weight_solver(o);
    if (et != EIK_OK) return et;
  }
  const int tmode = o->theta_mode;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  const int ntile = P[0] * P[1] * P[2];
  const int nlat = 3 * M * M - 3 * M + 1;
  size_t need = 0;
  need += 8 * (N * szT + 256);
  need += 4 * (N + 256) + 2 * N + 256;
  need += 2 * (N * 8 + 256);
  need += (size_t)ntile * 6 * L * L * (szT + 1) + 512;
  need += (size_t)ntile * L * L * L + 256;
  need += 2 * ((size_t)ntile * sizeof(int) + 256);  // subdomain order and sweep counts
  need += 4096;
  if (tmode == EIK_THETA_ESTIMATE) need += 3 * (N * szT + 256);  // u^{k-1} and two more C arrays
  const int ncell = (NC[0] + 1) * (NC[1] + 1) * (NC[2] + 1);
  need += (size_t)8 * ncell * sizeof(int) * 2 + 1024;  // causal items (8 per cell) and flags
  const int rec_stride = ncell;  // lattice nodes <= (NC+1)^3
  if (tmode == EIK_THETA_CONSTANT) need += (size_t)nlat * rec_stride * sizeof(eik::Corr3Rec<T>) + 256;
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::DD3<T> A;
  for (int a = 0; a < 3; ++a) { A.n[a] = n[a]; A.P[a] = P[a]; A.NC[a] = NC[a]; }
  A.S = S; A.M = M; A.nlat = nlat;
  A.hT = (T)G->h;
  A.HT = (T)((double)M * G->h);
  A.theta = (T)o->theta;
  A.max_fine_sweeps = o->max_fine_sweeps;
  A.max_coarse_sweeps = o->max_coarse_sweeps;
  A.r = as<T>(rv);
  A.gidx = gam->idx;
  A.gval = as<T>(gam->g);
  A.ng = gam->count;
  T* gfull = cv.take<T>(N);
  A.gfull = gfull;
  A.rdh = cv.take<T>(N);
  A.rdH = cv.take<T>(N);
  A.U = cv.take<T>(N);
  A.Un = cv.take<T>(N);
  A.uk = cv.take<T>(N);
  A.ck = cv.take<T>(N);
  A.W = cv.take<uint8_t>(N);
  A.Wn = cv.take<uint8_t>(N);
  A.wk = cv.take<uint8_t>(N);
  A.mk = cv.take<uint16_t>(N);
  A.near_key = cv.take<unsigned long long>(N);
  A.near_win = cv.take<long long>(N);
  A.face_u = cv.take<T>((size_t)ntile * 6 * L * L);
  A.face_w = cv.take<uint8_t>((size_t)ntile * 6 * L * L);
  A.tile_w = cv.take<uint8_t>((size_t)ntile * L * L * L);
  // Step 3 runs one subdomain per compute unit at a time (a subdomain fills
  // its LDS), so with more subdomains than compute units the launch ends
  // with the last ones started.  Each iteration takes them longest first,
  // by the time each took in the previous one (the first iteration in index
  // order): that changes when a subdomain runs, not what it computes.
  int* tile_order = cv.take<int>(ntile);
  A.tile_time = cv.take<int>(ntile);
  A.tile_order = tile_order;
  std::vector<int> order_h(ntile), time_h(ntile);
  for (int i = 0; i < ntile; ++i) order_h[i] = i;
  A.cvals = nullptr;
  A.counters = cv.take<unsigned long long>(4);
  A.rec_stride = rec_stride;
  A.rec = tmode == EIK_THETA_CONSTANT ? (void*)cv.take<eik::Corr3Rec<T>>((size_t)nlat * rec_stride) : nullptr;
  unsigned int* dflag = cv.take<unsigned int>(4);
  Causal3Plan cp;
  {
    const std::vector<int> items = causal3_items(A);
    cp.nitems = (int)items.size();
    cp.items = cv.take<int>(items.size());
    cp.done = cv.take<int>((size_t)8 * ncell);
    cp.abort_flag = cv.take<int>(8);
    HIPCHK(hipMemcpyAsync(cp.items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(cp.done, 0, (size_t)8 * ncell * sizeof(int), s));
    HIPCHK(hipMemsetAsync(cp.abort_flag, 0, 8 * sizeof(int), s));
    // the copy reads `items` (pageable host memory) asynchronously: it must
    // be complete before the vector goes out of scope
    HIPCHK(hipStreamSynchronize(s));
    const int own = 3 * M * M - 3 * M + 1;
    cp.threads = std::min(256, (own + eik::kWave - 1) / eik::kWave * eik::kWave);
    cp.lds = eik::causal3_lds<T>(M);
    int per_cu = 0, ncu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, eik::k_causal3p<T>, cp.threads, cp.lds));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // every block resident at once (the waits rely on it): half of what the
    // occupancy calculation allows, so that the count does not depend on
    // that estimate being exact
    cp.per_cu = per_cu;
    cp.blocks = std::max(1, std::min(std::max(1, per_cu / 2) * ncu, cp.nitems));
  }
  A.u_out = as<T>(u_outv);
  A.coarse_homog = o->coarse_solver;
  set_theta<T>(A.tq, o);
  A.tref = as<T>(o->theta_ref);
  A.ukm1 = A.ckm1 = A.ckm2 = nullptr;
  T* hist_u = nullptr;
  T* hist_c[3] = {A.ck, nullptr, nullptr};
  if (tmode == EIK_THETA_ESTIMATE) {
    hist_u = cv.take<T>(N);
    hist_c[1] = cv.take<T>(N);
    hist_c[2] = cv.take<T>(N);
  }
  auto correct_kernel = [&]() -> void (*)(eik::DD3<T>) {
    switch (tmode) {
      case EIK_THETA_ESTIMATE: return eik::k_lattice_correct3<T, 1>;
      case EIK_THETA_REFERENCE: return eik::k_lattice_correct3<T, 2>;
      case EIK_THETA_FIELD: return eik::k_lattice_correct3<T, 3>;
      default: return eik::k_lattice_correct3<T, 0>;
    }
  }();
  if ((e = validate<T>(A.r, N, gam, dflag, host, s, G->h)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_tile3<T>, lds_tile)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_lattice_init3<T>, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(correct_kernel, lds_lat)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_causal3p<T>, lds_cell)) != EIK_OK) return e;

  hipEvent_t ev[6];
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]); }
  } evg{ev};
  HIPCHK(hipEventRecord(ev[0], s));
  const T nanT = (T)NAN;
  const int bs = 256;
  HIPCHK(hipMemsetAsync(A.counters, 0, 4 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, gfull, nanT, N);
  if (gam->count > 0)
    hipLaunchKernelGGL(eik::k_scatter_gamma<T>, dim3(nblocks(gam->count, bs)), dim3(bs), 0, s, gfull,
                       gam->idx, as<T>(gam->g), gam->count);
  hipLaunchKernelGGL(eik::k_rd3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.u_out, nanT, N);
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.uk, nanT, N);
  HIPCHK(hipMemsetAsync(A.wk, 0, N, s));
  HIPCHK(hipGetLastError());
  float ms_fine = 0.f, ms_correct = 0.f, ms_causal = 0.f;
  if (o->U_init) {
    hipLaunchKernelGGL(eik::k_skel3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A, as<T>(o->U_init), A.U);
    HIPCHK(hipMemcpyAsync(A.W, o->W_init, N, hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.U, nanT, N);
    HIPCHK(hipMemsetAsync(A.W, 0, N, s));
    HIPCHK(hipMemsetAsync(A.near_key, 0xff, N * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(eik::k_fill<long long>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.near_win,
                       (long long)0x7fffffffffffffffll, N);
    const int64_t W2 = 2 * M - 1;
    const int64_t npair = gam->count * W2 * W2 * W2;
    if (npair > 0) {
      hipLaunchKernelGGL(eik::k_near3_a<T>, dim3(nblocks(npair, bs)), dim3(bs), 0, s, A);
      hipLaunchKernelGGL(eik::k_near3_b<T>, dim3(nblocks(npair, bs)), dim3(bs), 0, s, A);
    }
    hipLaunchKernelGGL(eik::k_lattice_init3<T>, dim3(nlat), dim3(eik::kBlock3), lds_lat, s, A);
    causal_sweep3p(A, A.U, A.W, cp, s);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A.Un, nanT, N);
  HIPCHK(hipMemsetAsync(A.Wn, 0, N, s));
  const eik_dd_debug* dbg = o->debug;
  int it = 0, conv = 0;
  double last = 0.0;
  for (int k = 0; k < o->max_iter; ++k) {
    // the order (host memory read by the copy) changes only after the
    // stream has been synchronised again
    HIPCHK(hipMemcpyAsync(tile_order, order_h.data(), (size_t)ntile * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(ev[1], s));
    hipLaunchKernelGGL(eik::k_tile3<T>, dim3(ntile), dim3(eik::kBlock3), lds_tile, s, A);
    HIPCHK(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(eik::k_reconcile3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
    if (tmode == EIK_THETA_ESTIMATE) {
      // C^k goes to hist_c[k % 3]; the other two hold C^{k-1}, C^{k-2}
      A.ck = hist_c[k % 3];
      A.ckm1 = k >= 1 ? hist_c[(k + 2) % 3] : nullptr;
      A.ckm2 = k >= 2 ? hist_c[(k + 1) % 3] : nullptr;
      A.ukm1 = k >= 1 ? hist_u : nullptr;
    }
    hipLaunchKernelGGL(eik::k_ck3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
    hipLaunchKernelGGL(correct_kernel, dim3(nlat), dim3(eik::kBlock3), lds_lat, s, A);
    if (tmode == EIK_THETA_ESTIMATE) HIPCHK(hipMemcpyAsync(hist_u, A.uk, N * szT, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipEventRecord(ev[4], s));
    if (dbg && dbg->U_pre_causal)
      HIPCHK(hipMemcpyAsync(dbg->U_pre_causal, A.Un, N * szT, hipMemcpyDeviceToDevice, s));
    causal_sweep3p(A, A.Un, A.Wn, cp, s);
    HIPCHK(hipMemsetAsync(&A.counters[2], 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(eik::k_residual3<T>, dim3(std::min(nblocks(N, bs), 2048u)), dim3(bs), 0, s, A);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[3], s));
    HIPCHK(hipMemcpyAsync(host, &A.counters[2], sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(time_h.data(), A.tile_time, (size_t)ntile * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::iota(order_h.begin(), order_h.end(), 0);
    std::stable_sort(order_h.begin(), order_h.end(), [&](int x, int y) { return time_h[x] > time_h[y]; });
    float a = 0.f, b = 0.f, c = 0.f;
    HIPCHK(hipEventElapsedTime(&a, ev[1], ev[2]));
    HIPCHK(hipEventElapsedTime(&b, ev[2], ev[4]));
    HIPCHK(hipEventElapsedTime(&c, ev[4], ev[3]));
    ms_fine += a;
    ms_correct += b;
    ms_causal += c;
    unsigned long long bits = host[0];
    double delta;
    std::memcpy(&delta, &bits, sizeof delta);
    std::swap(A.U, A.Un);
    std::swap(A.W, A.Wn);
    it = k + 1;
    last = delta;
    if (st && st->residual_history && k < st->history_cap) st->residual_history[k] = delta;
    if (std::isnan(delta)) return fail(EIK_ERR_NONFINITE, "residual is NaN");
    if (delta < o->tol || delta == 0.0) {
      conv = 1;
      break;
    }
  }
  if (U_outv) hipLaunchKernelGGL(eik::k_skel3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A, A.U, as<T>(U_outv));
  if (W_out) HIPCHK(hipMemcpyAsync(W_out, A.W, N, hipMemcpyDeviceToDevice, s));
  if (dbg && dbg->uk) HIPCHK(hipMemcpyAsync(dbg->uk, A.uk, N * szT, hipMemcpyDeviceToDevice, s));
  if (dbg && dbg->wk) HIPCHK(hipMemcpyAsync(dbg->wk, A.wk, N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(host, A.counters, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(ev[3], s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  if (host[3]) {
    int ab[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    HIPCHK(hipMemcpy(ab, cp.abort_flag, sizeof ab, hipMemcpyDeviceToHost));
    return fail(EIK_ERR_INTERNAL,
                "a wait of the persistent causal sweep gave up (item %d of %d in block %d, flag %d read %d, "
                "epoch %d of %d; %d blocks of %d threads, %d per CU by occupancy)", ab[1], cp.nitems, ab[5], ab[2],
                ab[3], ab[4], cp.epoch, cp.blocks, cp.threads, cp.per_cu);
  }
  if (st) {
    float tot = 0.f;
    HIPCHK(hipEventElapsedTime(&tot, ev[0], ev[3]));
    st->iterations = it;
    st->converged = conv;
    st->fine_updates = (int64_t)host[0];
    st->coarse_updates = (int64_t)host[1];
    st->sweeps = 0;
    st->final_residual = last;
    st->ms_total = tot;
    st->ms_fine = ms_fine;
    st->ms_coarse = tot - ms_fine;
    st->ms_correct = ms_correct;
    st->ms_causal = ms_causal;
  }
  if (o->max_iter > 0 && !conv) return fail(EIK_ERR_NOCONV, "no convergence in %d iterations (residual %g)", it, last);
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// eik_solve, d = 3
// ---------------------------------------------------------------------------

template <typename T>
eik_status solve3_t(const eik_grid* G, const void* rv, const eik_gamma* gam, int32_t max_sweeps,
                    void* u_outv, int8_t* wind_out, eik_stats* st, hipStream_t s) {
  int n[3];
  for (int a = 0; a < 3; ++a) n[a] = (int)G->n[a];
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  if (max_sweeps < 1) return fail(EIK_ERR_ARG, "max_sweeps must be >= 1");
  const size_t szT = sizeof(T);
  // largest box side that fits in LDS, then even box sides per axis
  int Bmax = eik::kMaxL3;
  while ((size_t)Bmax * Bmax * Bmax * szT > kLdsBytes) --Bmax;
  int B = 1;
  for (int a = 0; a < 3; ++a) {
    const int nb = (n[a] + Bmax - 1) / Bmax;
    B = std::max(B, (n[a] + nb - 1) / nb);
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  size_t need = N * szT + 256 + (wind_out ? 0 : N + 256) + 4096;
  int nbx[3];
  for (int a = 0; a < 3; ++a) nbx[a] = (n[a] + B - 1) / B;
  const size_t nbox = (size_t)nbx[0] * nbx[1] * nbx[2];
  need += 2 * (nbox * sizeof(int) + 256);
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::GS3<T> A;
  for (int a = 0; a < 3; ++a) { A.n[a] = n[a]; A.nb[a] = (n[a] + B - 1) / B; }
  A.B = B;
  A.hT = (T)G->h;
  A.r = as<T>(rv);
  T* gfull = cv.take<T>(N);
  A.gfull = gfull;
  A.u = as<T>(u_outv);
  A.w = wind_out ? (uint8_t*)wind_out : cv.take<uint8_t>(N);
  unsigned int* dflag = cv.take<unsigned int>(8);
  A.changed = dflag + 1;
  A.eval_at = cv.take<int>(nbox);
  A.chg_at = cv.take<int>(nbox);
  if ((e = validate<T>(A.r, N, gam, dflag, host, s, G->h)) != EIK_OK) return e;
  const size_t lds = (size_t)B * B * B * szT;
  if ((e = allow_lds(eik::k_grid_sweep3<T>, lds)) != EIK_OK) return e;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  const int bs = 256;
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, gfull, (T)NAN, N);
  if (gam->count > 0)
    hipLaunchKernelGGL(eik::k_scatter_gamma<T>, dim3(nblocks(gam->count, bs)), dim3(bs), 0, s, gfull,
                       gam->idx, as<T>(gam->g), gam->count);
  hipLaunchKernelGGL(eik::k_grid_init3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
  HIPCHK(hipMemsetAsync(A.eval_at, 0xff, nbox * sizeof(int), s));
  HIPCHK(hipMemsetAsync(A.chg_at, 0xff, nbox * sizeof(int), s));
  HIPCHK(hipGetLastError());
  const int ndiag = A.nb[0] + A.nb[1] + A.nb[2] - 2;
  // sweeps 4m .. 4m+3 share launches, each behind the one before by the lag
  // its reversed axes need (as the causal sweep's directions); a sweep
  // without change leaves the grid stationary for every order, so the later
  // sweeps of its group then change nothing and the count stops there
  const int off[4] = {0, A.nb[2] + 1, A.nb[2] + 1 + A.nb[1] + A.nb[2], 2 * (A.nb[2] + 1) + A.nb[1] + A.nb[2]};
  int sw = 0, conv = 0;
  while (sw < max_sweeps) {
    const int nsw = std::min(4, max_sweeps - sw);
    HIPCHK(hipMemsetAsync(A.changed, 0, 4 * sizeof(unsigned int), s));
    for (int tau = 0; tau < off[nsw - 1] + ndiag; ++tau) {
      eik::GridLaunch3 L{};
      int nbk = 0;
      for (int k = 0; k < nsw; ++k) {
        const int d = tau - off[k];
        if (d < 0 || d >= ndiag) continue;
        L.dir[L.n] = (sw + k) & 7;
        L.diag[L.n] = d;
        L.t[L.n] = (sw + k) * ndiag + d;
        L.chg_off[L.n] = k;
        L.start[L.n] = nbk;
        nbk += cells_on_diag(A.nb, d);
        ++L.n;
      }
      L.start[L.n] = nbk;
      if (nbk == 0) continue;
      hipLaunchKernelGGL(eik::k_grid_sweep3<T>, dim3(nbk), dim3(eik::kBlock3), lds, s, A, L);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host, A.changed, 4 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const unsigned int* hc = (const unsigned int*)host;
    int k0 = -1;
    for (int k = 0; k < nsw && k0 < 0; ++k)
      if (hc[k] == 0) k0 = k;
    if (k0 >= 0) {
      sw += k0 + 1;
      conv = 1;
      break;
    }
    sw += nsw;
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    st->iterations = 0;
    st->converged = conv;
    st->sweeps = sw;
    st->fine_updates = (int64_t)sw * (N - gam->count);
    st->coarse_updates = 0;
    st->final_residual = 0.0;
    st->ms_total = ms;
    st->ms_fine = ms;
    st->ms_coarse = 0.f;
    st->ms_correct = 0.f;
    st->ms_causal = 0.f;
  }
  if (!conv) return fail(EIK_ERR_NOCONV, "no stationary sweep within %d sweeps", max_sweeps);
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// eik_solve, d = 2
// ---------------------------------------------------------------------------

// eik_solve on nb problems that share the grid and the slowness (one
// Gamma each, e.g. one source each): every launch of a sweep covers the
// boxes of one box diagonal of all problems that have not yet had a sweep
// without change; a problem that had one is stationary and is left alone.
template <typename T>
eik_status solve_t(const eik_grid* G, const void* rv, int nb, const eik_gamma* gam, int32_t max_sweeps,
                   void* u_outv, int8_t* wind_out, eik_stats* st, hipStream_t s) {
  const int n0 = (int)G->n[0], n1 = (int)G->n[1];
  const int64_t N = (int64_t)n0 * n1;
  const int64_t NB = (int64_t)nb * N;
  if (max_sweeps < 1) return fail(EIK_ERR_ARG, "max_sweeps must be >= 1");
  auto side = [](int n) { int k = (n + eik::kMaxL - 1) / eik::kMaxL; return (n + k - 1) / k; };
  const int B = std::max(side(n0), side(n1));
  const int BX = (n0 + B - 1) / B, BY = (n1 + B - 1) / B;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  const size_t szT = sizeof(T);
  size_t need = NB * szT + 256 + (wind_out ? 0 : NB + 256) + 4096 + 12 * (size_t)nb + 512;
  need += 2 * ((size_t)nb * BX * BY * sizeof(int) + 256);
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::GS2<T> A;
  A.n0 = n0; A.n1 = n1; A.B = B; A.BX = BX; A.BY = BY;
  A.hT = (T)G->h;
  A.r = as<T>(rv);
  T* gfull = cv.take<T>(NB);
  A.gfull = gfull;
  A.u = as<T>(u_outv);
  A.w = wind_out ? (uint8_t*)wind_out : cv.take<uint8_t>(NB);
  unsigned int* dflag = cv.take<unsigned int>(4);
  unsigned int* dchg = cv.take<unsigned int>(2 * (size_t)nb);  // per problem, for the two sweeps of a launch pair
  int* dmem = cv.take<int>(nb);
  A.changed = dchg;
  A.members = dmem;
  A.eval_at = cv.take<int>((size_t)nb * BX * BY);
  A.chg_at = cv.take<int>((size_t)nb * BX * BY);
  for (int b = 0; b < nb; ++b)
    if ((e = validate<T>(A.r, N, &gam[b], dflag, host, s, G->h)) != EIK_OK) return e;
  const size_t lds = eik::box_bytes(eik::halo_count(B, B), 2, 1, szT);
  if ((e = allow_lds(eik::k_grid_sweep<T>, lds)) != EIK_OK) return e;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } evg{e0, e1};
  HIPCHK(hipEventRecord(e0, s));
  const int bs = 256;
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(NB, bs)), dim3(bs), 0, s, gfull, (T)NAN, NB);
  for (int b = 0; b < nb; ++b)
    if (gam[b].count > 0)
      hipLaunchKernelGGL(eik::k_scatter_gamma<T>, dim3(nblocks(gam[b].count, bs)), dim3(bs), 0, s,
                         gfull + (int64_t)b * N, gam[b].idx, as<T>(gam[b].g), gam[b].count);
  hipLaunchKernelGGL(eik::k_grid_init<T>, dim3(nblocks(N, bs), nb), dim3(bs), 0, s, A);
  HIPCHK(hipMemsetAsync(A.eval_at, 0xff, (size_t)nb * BX * BY * sizeof(int), s));
  HIPCHK(hipMemsetAsync(A.chg_at, 0xff, (size_t)nb * BX * BY * sizeof(int), s));
  HIPCHK(hipGetLastError());
  std::vector<int> active(nb), sweeps(nb, 0);
  std::vector<unsigned int> hchg(2 * (size_t)nb);
  for (int b = 0; b < nb; ++b) active[b] = b;
  const int D = BX + BY - 1;  // box diagonals per sweep
  auto boxes_on = [&](int d) { return (d < 0 || d >= D) ? 0 : std::min(d, BX - 1) - std::max(0, d - (BY - 1)) + 1; };
  int sw = 0;
  while (sw < max_sweeps && !active.empty()) {
    // sweeps sw (even: x fixed, y - or +) and sw + 1 (y reversed) in shared
    // launches, the second BY + 1 diagonals behind; if sweep sw changes
    // nothing the grid is stationary for every order, so sweep sw + 1 then
    // changes nothing either and the problem stops after sweep sw
    const int nsw = (sw + 1 < max_sweeps) ? 2 : 1;
    const int lag = nsw == 2 ? BY + 1 : 0;
    const int na = (int)active.size();
    HIPCHK(hipMemcpyAsync(dmem, active.data(), na * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(dchg, 0, 2 * (size_t)nb * sizeof(unsigned int), s));
    for (int tau = 0; tau < D + lag; ++tau) {
      eik::GridLaunch2 L{};
      int nbk = 0;
      for (int k = 0; k < nsw; ++k) {
        const int d = tau - k * lag;
        const int cnt = boxes_on(d);
        if (cnt == 0) continue;
        L.dir[L.n] = (sw + k) & 3;
        L.diag[L.n] = d;
        L.t[L.n] = (sw + k) * D + d;
        L.chg_off[L.n] = k * nb;
        L.start[L.n] = nbk;
        nbk += cnt;
        ++L.n;
      }
      L.start[L.n] = nbk;
      if (nbk == 0) continue;
      hipLaunchKernelGGL(eik::k_grid_sweep<T>, dim3(nbk, na), dim3(eik::kBlock), lds, s, A, L);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hchg.data(), dchg, 2 * (size_t)nb * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int b : active) {
      if (!hchg[b]) {
        sweeps[b] = sw + 1;
      } else if (nsw == 2 && hchg[nb + b]) {
        sweeps[b] = sw + 2;
        next.push_back(b);
      } else {
        sweeps[b] = sw + nsw;
        if (nsw == 1) next.push_back(b);
      }
    }
    sw += nsw;
    active.swap(next);
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  if (st) {
    for (int b = 0; b < nb; ++b) {
      const bool done = std::find(active.begin(), active.end(), b) == active.end();
      st[b].iterations = 0;
      st[b].converged = done ? 1 : 0;
      st[b].sweeps = sweeps[b];
      st[b].fine_updates = (int64_t)sweeps[b] * (N - gam[b].count);
      st[b].coarse_updates = 0;
      st[b].final_residual = 0.0;
      st[b].ms_total = ms;
      st[b].ms_fine = ms;
      st[b].ms_coarse = st[b].ms_correct = st[b].ms_causal = 0.f;
    }
  }
  if (!active.empty()) return fail(EIK_ERR_NOCONV, "FSM not stationary after %d sweeps", sw);
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// travel-time gradient (adjoint), d = 2
// ---------------------------------------------------------------------------

template <typename T>
eik_status adjoint_t(const eik_grid* G, const void* rv, int32_t nb, const eik_gamma* gams, const void* uv,
                     const int8_t* wind, const void* seedv, void* gradv, void* lamv, int32_t max_sweeps,
                     eik_stats* st, hipStream_t s) {
  const int n0 = (int)G->n[0], n1 = (int)G->n[1];
  const int64_t N = (int64_t)n0 * n1;
  const size_t szT = sizeof(T);
  int Bmax = eik::kMaxL;
  while (Bmax > 8 && eik::adj_box_bytes(Bmax, szT) > kLdsBytes) --Bmax;
  auto side = [&](int n) { int k = (n + Bmax - 1) / Bmax; return (n + k - 1) / k; };
  const int B = std::max(side(n0), side(n1));
  const size_t lds = eik::adj_box_bytes(B, szT);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  const int64_t NB = (int64_t)nb * N;
  size_t need = (size_t)NB * (1 + 1) + 2 * 256;           // fixed, wd
  need += (size_t)NB * szT * (2 + 1 + 4) + 3 * 256;       // c, q, pc
  if (!lamv) need += (size_t)NB * szT + 256;
  const int BXa = (n0 + B - 1) / B, BYa = (n1 + B - 1) / B;
  need += 2 * ((size_t)nb * BXa * BYa * sizeof(int) + 256);  // box stamps
  need += 4096;
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::ADJ2<T> A;
  A.n0 = n0; A.n1 = n1; A.nb = nb;
  A.B = B; A.BX = (n0 + B - 1) / B; A.BY = (n1 + B - 1) / B;
  A.hT = (T)G->h;
  A.r = as<T>(rv);
  A.u = as<T>(uv);
  A.w = wind;
  A.seed = as<T>(seedv);
  A.fixed = cv.take<uint8_t>(NB);
  A.wd = cv.take<uint8_t>(NB);
  A.c = cv.take<T>(2 * NB);
  A.q = cv.take<T>(NB);
  A.pc = cv.take<T>(4 * NB);
  A.lam = lamv ? as<T>(lamv) : cv.take<T>(NB);
  A.grad = as<T>(gradv);
  unsigned int* dflag = cv.take<unsigned int>(4);
  A.changed = dflag + 1;
  A.eval_at = cv.take<int>((size_t)nb * BXa * BYa);
  A.chg_at = cv.take<int>((size_t)nb * BXa * BYa);
  // the slowness and every boundary set are checked like the forward solve's
  for (int b = 0; b < nb; ++b)
    if ((e = validate<T>(A.r, N, &gams[b], dflag, host, s, G->h)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_adj_sweep<T>, lds)) != EIK_OK) return e;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } evg{e0, e1};
  HIPCHK(hipEventRecord(e0, s));
  const int bs = 256;
  HIPCHK(hipMemsetAsync(A.fixed, 0, NB, s));
  for (int b = 0; b < nb; ++b)
    if (gams[b].count > 0)
      hipLaunchKernelGGL(eik::k_adj_mark<T>, dim3(nblocks(gams[b].count, bs)), dim3(bs), 0, s,
                         A.fixed + (int64_t)b * N, gams[b].idx, gams[b].count);
  const dim3 gridN(nblocks(N, bs), nb);
  hipLaunchKernelGGL(eik::k_adj_coef<T>, gridN, dim3(bs), 0, s, A);
  hipLaunchKernelGGL(eik::k_adj_pull<T>, gridN, dim3(bs), 0, s, A);
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(NB, bs)), dim3(bs), 0, s, A.lam, T(0), NB);
  HIPCHK(hipMemsetAsync(A.eval_at, 0xff, (size_t)nb * BXa * BYa * sizeof(int), s));
  HIPCHK(hipMemsetAsync(A.chg_at, 0xff, (size_t)nb * BXa * BYa * sizeof(int), s));
  HIPCHK(hipGetLastError());
  int sw = 0, conv = 0;
  const int D = A.BX + A.BY - 1;
  auto boxes_on = [&](int d) {
    return (d < 0 || d >= D) ? 0 : std::min(d, A.BX - 1) - std::max(0, d - (A.BY - 1)) + 1;
  };
  while (sw < max_sweeps) {
    // sweeps sw and sw + 1 (y reversed) in shared launches, as in eik_solve:
    // a sweep without change leaves every problem stationary, so the second
    // then changes nothing
    const int nsw = (sw + 1 < max_sweeps) ? 2 : 1;
    const int lag = nsw == 2 ? A.BY + 1 : 0;
    HIPCHK(hipMemsetAsync(A.changed, 0, 2 * sizeof(unsigned int), s));
    for (int tau = 0; tau < D + lag; ++tau) {
      eik::GridLaunch2 L{};
      int nbk = 0;
      for (int k = 0; k < nsw; ++k) {
        const int d = tau - k * lag;
        const int cnt = boxes_on(d);
        if (cnt == 0) continue;
        L.dir[L.n] = (sw + k) & 3;
        L.diag[L.n] = d;
        L.t[L.n] = (sw + k) * D + d;
        L.chg_off[L.n] = k;
        L.start[L.n] = nbk;
        nbk += cnt;
        ++L.n;
      }
      L.start[L.n] = nbk;
      if (nbk == 0) continue;
      hipLaunchKernelGGL(eik::k_adj_sweep<T>, dim3(nbk, nb), dim3(eik::kBlock), lds, s, A, L);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host, A.changed, 2 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const unsigned int* hc = (const unsigned int*)host;
    if (hc[0] == 0) {
      sw += 1;
      conv = 1;
      break;
    }
    sw += nsw;
    if (nsw == 2 && hc[1] == 0) {
      conv = 1;
      break;
    }
  }
  hipLaunchKernelGGL(eik::k_adj_grad<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  if (st) {
    st->iterations = 0;
    st->converged = conv;
    st->sweeps = sw;
    st->fine_updates = (int64_t)sw * NB;
    st->coarse_updates = 0;
    st->final_residual = 0.0;
    st->ms_total = ms;
    st->ms_fine = ms;
    st->ms_coarse = st->ms_correct = st->ms_causal = 0.f;
  }
  if (!conv) return fail(EIK_ERR_NOCONV, "adjoint sweeps not stationary after %d sweeps", max_sweeps);
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// travel-time gradient (adjoint), d = 3
// ---------------------------------------------------------------------------

template <typename T>
eik_status adjoint3_t(const eik_grid* G, const void* rv, int32_t nb, const eik_gamma* gams, const void* uv,
                      const int8_t* wind, const void* seedv, void* gradv, void* lamv, int32_t max_sweeps,
                      eik_stats* st, hipStream_t s) {
  int n[3];
  for (int a = 0; a < 3; ++a) n[a] = (int)G->n[a];
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  const size_t szT = sizeof(T);
  // largest box side whose lambda fits in LDS, then even box sides per axis
  int Bmax = eik::kMaxL3;
  while ((size_t)Bmax * Bmax * Bmax * szT > kLdsBytes) --Bmax;
  int B = 1;
  for (int a = 0; a < 3; ++a) {
    const int k = (n[a] + Bmax - 1) / Bmax;
    B = std::max(B, (n[a] + k - 1) / k);
  }
  const size_t lds = (size_t)B * B * B * szT;
  int nbx[3];
  for (int a = 0; a < 3; ++a) nbx[a] = (n[a] + B - 1) / B;
  const size_t nbox = (size_t)nbx[0] * nbx[1] * nbx[2];
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_ws[dev].mu);
  const int64_t NB = (int64_t)nb * N;
  size_t need = (size_t)NB * (1 + 1) + 2 * 256;           // fixed, wd
  need += (size_t)NB * szT * (3 + 1 + 6) + 3 * 256;       // c, q, pc
  if (!lamv) need += (size_t)NB * szT + 256;
  need += 2 * ((size_t)nb * nbox * sizeof(int) + 256);    // box stamps
  need += 4096;
  void* wsv;
  unsigned long long* host;
  eik_status e = ws_get(dev, need, &wsv, &host);
  if (e != EIK_OK) return e;
  Carver cv{(char*)wsv};
  eik::ADJ3<T> A;
  for (int a = 0; a < 3; ++a) { A.n[a] = n[a]; A.nbx[a] = nbx[a]; }
  A.nb = nb;
  A.B = B;
  A.hT = (T)G->h;
  A.r = as<T>(rv);
  A.u = as<T>(uv);
  A.w = wind;
  A.seed = as<T>(seedv);
  A.fixed = cv.take<uint8_t>(NB);
  A.wd = cv.take<uint8_t>(NB);
  A.c = cv.take<T>(3 * NB);
  A.q = cv.take<T>(NB);
  A.pc = cv.take<T>(6 * NB);
  A.lam = lamv ? as<T>(lamv) : cv.take<T>(NB);
  A.grad = as<T>(gradv);
  unsigned int* dflag = cv.take<unsigned int>(8);
  A.changed = dflag + 1;
  A.eval_at = cv.take<int>((size_t)nb * nbox);
  A.chg_at = cv.take<int>((size_t)nb * nbox);
  // the slowness and every boundary set are checked like the forward solve's
  for (int b = 0; b < nb; ++b)
    if ((e = validate<T>(A.r, N, &gams[b], dflag, host, s, G->h)) != EIK_OK) return e;
  if ((e = allow_lds(eik::k_adj_sweep3<T>, lds)) != EIK_OK) return e;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } evg{e0, e1};
  HIPCHK(hipEventRecord(e0, s));
  const int bs = 256;
  HIPCHK(hipMemsetAsync(A.fixed, 0, NB, s));
  for (int b = 0; b < nb; ++b)
    if (gams[b].count > 0)
      hipLaunchKernelGGL(eik::k_adj_mark<T>, dim3(nblocks(gams[b].count, bs)), dim3(bs), 0, s,
                         A.fixed + (int64_t)b * N, gams[b].idx, gams[b].count);
  const dim3 gridN(nblocks(N, bs), nb);
  hipLaunchKernelGGL(eik::k_adj_coef3<T>, gridN, dim3(bs), 0, s, A);
  hipLaunchKernelGGL(eik::k_adj_pull3<T>, gridN, dim3(bs), 0, s, A);
  hipLaunchKernelGGL(eik::k_fill<T>, dim3(nblocks(NB, bs)), dim3(bs), 0, s, A.lam, T(0), NB);
  HIPCHK(hipMemsetAsync(A.eval_at, 0xff, (size_t)nb * nbox * sizeof(int), s));
  HIPCHK(hipMemsetAsync(A.chg_at, 0xff, (size_t)nb * nbox * sizeof(int), s));
  HIPCHK(hipGetLastError());
  const int ndiag = nbx[0] + nbx[1] + nbx[2] - 2;
  // sweeps 4m .. 4m+3 share launches with the lags of eik_solve in 3D; a
  // sweep without change leaves every problem stationary, so the later
  // sweeps of its group change nothing and the count stops there
  const int off[4] = {0, nbx[2] + 1, nbx[2] + 1 + nbx[1] + nbx[2], 2 * (nbx[2] + 1) + nbx[1] + nbx[2]};
  int sw = 0, conv = 0;
  while (sw < max_sweeps) {
    const int nsw = std::min(4, max_sweeps - sw);
    HIPCHK(hipMemsetAsync(A.changed, 0, 4 * sizeof(unsigned int), s));
    for (int tau = 0; tau < off[nsw - 1] + ndiag; ++tau) {
      eik::GridLaunch3 L{};
      int nbk = 0;
      for (int k = 0; k < nsw; ++k) {
        const int d = tau - off[k];
        if (d < 0 || d >= ndiag) continue;
        L.dir[L.n] = (sw + k) & 7;
        L.diag[L.n] = d;
        L.t[L.n] = (sw + k) * ndiag + d;
        L.chg_off[L.n] = k;
        L.start[L.n] = nbk;
        nbk += cells_on_diag(nbx, d);
        ++L.n;
      }
      L.start[L.n] = nbk;
      if (nbk == 0) continue;
      hipLaunchKernelGGL(eik::k_adj_sweep3<T>, dim3(nbk, nb), dim3(eik::kBlock3), lds, s, A, L);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host, A.changed, 4 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const unsigned int* hc = (const unsigned int*)host;
    int k0 = -1;
    for (int k = 0; k < nsw && k0 < 0; ++k)
      if (hc[k] == 0) k0 = k;
    if (k0 >= 0) {
      sw += k0 + 1;
      conv = 1;
      break;
    }
    sw += nsw;
  }
  hipLaunchKernelGGL(eik::k_adj_grad3<T>, dim3(nblocks(N, bs)), dim3(bs), 0, s, A);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  if (st) {
    st->iterations = 0;
    st->converged = conv;
    st->sweeps = sw;
    st->fine_updates = (int64_t)sw * NB;
    st->coarse_updates = 0;
    st->final_residual = 0.0;
    st->ms_total = ms;
    st->ms_fine = ms;
    st->ms_coarse = st->ms_correct = st->ms_causal = 0.f;
  }
  if (!conv) return fail(EIK_ERR_NOCONV, "adjoint sweeps not stationary after %d sweeps", max_sweeps);
  return EIK_OK;
}

eik_status check_common(const eik_grid* G, const void* r, const eik_gamma* gam, const void* out) {
  if (!G || !r || !gam || !out) return fail(EIK_ERR_ARG, "NULL argument");
  if (G->dim != 2 && G->dim != 3) return fail(EIK_ERR_ARG, "dim must be 2 or 3");
  if (G->dtype != EIK_F32 && G->dtype != EIK_F64) return fail(EIK_ERR_ARG, "dtype must be EIK_F32 or EIK_F64");
  int64_t N = 1;
  for (int a = 0; a < G->dim; ++a) {
    if (G->n[a] < 2) return fail(EIK_ERR_SHAPE, "need at least 2 nodes per axis");
    N *= G->n[a];
  }
  if (N >= (int64_t)1 << 31) return fail(EIK_ERR_UNSUPPORTED, "grid too large for 32-bit indexing");
  if (!(G->h > 0) || !std::isfinite(G->h)) return fail(EIK_ERR_ARG, "h must be positive and finite");
  if (gam->count < 0 || (gam->count > 0 && (!gam->idx || !gam->g))) return fail(EIK_ERR_ARG, "bad Gamma");
  if (r == out) return fail(EIK_ERR_ARG, "u_out must not alias r");
  return EIK_OK;
}

}  // namespace

extern "C" {

eik_status eik_solve(const eik_grid* grid, const void* r, const eik_gamma* gamma, int32_t max_sweeps,
                     void* u_out, int8_t* wind_out, eik_stats* stats, void* hip_stream) {
  eik_status e = check_common(grid, r, gamma, u_out);
  if (e != EIK_OK) return e;
  hipStream_t s = (hipStream_t)hip_stream;
  if (grid->dim == 3) {
    if (grid->dtype == EIK_F32) return solve3_t<float>(grid, r, gamma, max_sweeps, u_out, wind_out, stats, s);
    return solve3_t<double>(grid, r, gamma, max_sweeps, u_out, wind_out, stats, s);
  }
  if (grid->dtype == EIK_F32) return solve_t<float>(grid, r, 1, gamma, max_sweeps, u_out, wind_out, stats, s);
  return solve_t<double>(grid, r, 1, gamma, max_sweeps, u_out, wind_out, stats, s);
}

eik_status eik_dd_solve(const eik_grid* grid, const void* r, const eik_gamma* gamma, const eik_dd_opts* opts,
                        void* u_out, void* U_out, int8_t* W_out, eik_stats* stats, void* hip_stream) {
  eik_status e = check_common(grid, r, gamma, u_out);
  if (e != EIK_OK) return e;
  if (!opts) return fail(EIK_ERR_ARG, "NULL opts");
  hipStream_t s = (hipStream_t)hip_stream;
  if (grid->dim == 3) {
    if (grid->dtype == EIK_F32) return dd_solve3_t<float>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s);
    return dd_solve3_t<double>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s);
  }
  if (grid->dtype == EIK_F32)
    return dd_solve_t<float>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s);
  return dd_solve_t<double>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s);
}

eik_status eik_dd_solve_noalloc(const eik_grid* grid, const void* r, const eik_gamma* gamma,
                                const eik_dd_opts* opts, void* u_out, void* U_out, int8_t* W_out,
                                eik_stats* stats, void* hip_stream) {
  eik_status e = check_common(grid, r, gamma, u_out);
  if (e != EIK_OK) return e;
  if (!opts) return fail(EIK_ERR_ARG, "NULL opts");
  if (grid->dim != 2) return fail(EIK_ERR_UNSUPPORTED, "the allocation-free solve is built for d = 2");
  hipStream_t s = (hipStream_t)hip_stream;
  if (grid->dtype == EIK_F32)
    return dd_solve_t<float>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s, true);
  return dd_solve_t<double>(grid, r, gamma, opts, u_out, U_out, W_out, stats, s, true);
}

eik_status eik_solve_batch(const eik_grid* grid, const void* r, int32_t nb, const eik_gamma* gammas,
                           int32_t max_sweeps, void* u_out, int8_t* wind_out, eik_stats* stats, void* hip_stream) {
  if (!gammas || nb < 1) return fail(EIK_ERR_ARG, "need nb >= 1 boundary sets");
  for (int b = 0; b < nb; ++b) {
    eik_status e = check_common(grid, r, &gammas[b], u_out);
    if (e != EIK_OK) return e;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (grid->dim == 3) {
    // the problems one after another on the stream, each a whole-grid 3D
    // solve; stats[b]: problem b's sweeps and updates, the whole call's time
    const int64_t N = grid->n[0] * grid->n[1] * grid->n[2];
    const size_t szT = grid->dtype == EIK_F32 ? 4 : 8;
    std::vector<eik_stats> one(nb);
    float ms = 0.f;
    int all_conv = 1;
    for (int b = 0; b < nb; ++b) {
      void* ub = (char*)u_out + (size_t)b * N * szT;
      int8_t* wb = wind_out ? wind_out + (size_t)b * N : nullptr;
      one[b] = eik_stats{};
      const eik_status e = grid->dtype == EIK_F32
                               ? solve3_t<float>(grid, r, &gammas[b], max_sweeps, ub, wb, &one[b], s)
                               : solve3_t<double>(grid, r, &gammas[b], max_sweeps, ub, wb, &one[b], s);
      if (e != EIK_OK && e != EIK_ERR_NOCONV) return e;
      all_conv = all_conv && one[b].converged;
      ms += one[b].ms_total;
    }
    if (stats)
      for (int b = 0; b < nb; ++b) {
        stats[b].iterations = 0;
        stats[b].converged = one[b].converged;
        stats[b].sweeps = one[b].sweeps;
        stats[b].fine_updates = one[b].fine_updates;
        stats[b].coarse_updates = 0;
        stats[b].final_residual = 0.0;
        stats[b].ms_total = stats[b].ms_fine = ms;
        stats[b].ms_coarse = stats[b].ms_correct = stats[b].ms_causal = 0.f;
      }
    if (!all_conv) return fail(EIK_ERR_NOCONV, "no stationary sweep within %d sweeps", max_sweeps);
    return EIK_OK;
  }
  if (grid->dtype == EIK_F32) return solve_t<float>(grid, r, nb, gammas, max_sweeps, u_out, wind_out, stats, s);
  return solve_t<double>(grid, r, nb, gammas, max_sweeps, u_out, wind_out, stats, s);
}

eik_status eik_dd_solve_batch(int32_t nprob, const eik_grid* grids, const void* const* r, const eik_gamma* gammas,
                              const eik_dd_opts* opts, void* const* u_out, void* const* U_out, int8_t* const* W_out,
                              eik_stats* stats, void* hip_stream) {
  if (nprob < 1 || !grids || !r || !gammas || !opts || !u_out) return fail(EIK_ERR_ARG, "NULL argument or nprob < 1");
  int n3 = 0;
  for (int p = 0; p < nprob; ++p) {
    eik_status e = check_common(&grids[p], r[p], &gammas[p], u_out[p]);
    if (e != EIK_OK) return e;
    n3 += grids[p].dim == 3;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (n3 > 0) {
    // 3D: the problems one after another on the stream, each exactly as its
    // own eik_dd_solve (a 3D problem's subdomains and lattices fill the
    // device by themselves); the device-time fields hold the batch's totals
    if (n3 != nprob) return fail(EIK_ERR_UNSUPPORTED, "batch: 2D and 3D problems cannot be mixed");
    for (int p = 0; p < nprob; ++p) {
      if (grids[p].dtype != grids[0].dtype) return fail(EIK_ERR_ARG, "batch: all problems need the same dtype");
      if (opts[p].debug) return fail(EIK_ERR_ARG, "problem %d: debug snapshots are not available in a batch", p);
    }
    eik_status agg = EIK_OK;
    float tot[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    std::vector<eik_stats> own(nprob);
    for (int p = 0; p < nprob; ++p) {
      eik_stats* sp = stats ? &stats[p] : &own[p];
      void* Up = U_out ? U_out[p] : nullptr;
      int8_t* Wp = W_out ? W_out[p] : nullptr;
      const eik_status e =
          grids[0].dtype == EIK_F32
              ? dd_solve3_t<float>(&grids[p], r[p], &gammas[p], &opts[p], u_out[p], Up, Wp, sp, s)
              : dd_solve3_t<double>(&grids[p], r[p], &gammas[p], &opts[p], u_out[p], Up, Wp, sp, s);
      if (e != EIK_OK && e != EIK_ERR_NOCONV) return e;
      if (e == EIK_ERR_NOCONV) agg = e;
      const float f[5] = {sp->ms_total, sp->ms_fine, sp->ms_coarse, sp->ms_correct, sp->ms_causal};
      for (int k = 0; k < 5; ++k) tot[k] += f[k];
    }
    if (stats)
      for (int p = 0; p < nprob; ++p) {
        stats[p].ms_total = tot[0];
        stats[p].ms_fine = tot[1];
        stats[p].ms_coarse = tot[2];
        stats[p].ms_correct = tot[3];
        stats[p].ms_causal = tot[4];
      }
    if (agg != EIK_OK) return fail(agg, "batch: a problem reached its max_iter");
    return EIK_OK;
  }
  if (grids[0].dtype == EIK_F32)
    return dd_solve_batch_t<float>(nprob, grids, r, gammas, opts, u_out, U_out, W_out, stats, s);
  return dd_solve_batch_t<double>(nprob, grids, r, gammas, opts, u_out, U_out, W_out, stats, s);
}

eik_status eik_adjoint_batch(const eik_grid* grid, const void* r, int32_t nb, const eik_gamma* gammas,
                             const void* u, const int8_t* wind, const void* dL_du, void* dL_dr_out,
                             void* lambda_out, int32_t max_sweeps, eik_stats* stats, void* hip_stream) {
  if (!gammas || nb < 1) return fail(EIK_ERR_ARG, "need nb >= 1 boundary sets");
  eik_status e = check_common(grid, r, &gammas[0], dL_dr_out);
  if (e != EIK_OK) return e;
  for (int b = 1; b < nb; ++b)
    if (gammas[b].count < 0 || (gammas[b].count > 0 && (!gammas[b].idx || !gammas[b].g)))
      return fail(EIK_ERR_ARG, "bad Gamma of problem %d", b);
  if (!u || !dL_du) return fail(EIK_ERR_ARG, "NULL u or dL_du");
  if (max_sweeps < 1) return fail(EIK_ERR_ARG, "max_sweeps must be >= 1");
  if (dL_dr_out == u || dL_dr_out == dL_du || (lambda_out && (lambda_out == u || lambda_out == dL_du)))
    return fail(EIK_ERR_ARG, "outputs must not alias inputs");
  hipStream_t s = (hipStream_t)hip_stream;
  if (grid->dim == 3) {
    if (grid->dtype == EIK_F32)
      return adjoint3_t<float>(grid, r, nb, gammas, u, wind, dL_du, dL_dr_out, lambda_out, max_sweeps, stats, s);
    return adjoint3_t<double>(grid, r, nb, gammas, u, wind, dL_du, dL_dr_out, lambda_out, max_sweeps, stats, s);
  }
  if (grid->dtype == EIK_F32)
    return adjoint_t<float>(grid, r, nb, gammas, u, wind, dL_du, dL_dr_out, lambda_out, max_sweeps, stats, s);
  return adjoint_t<double>(grid, r, nb, gammas, u, wind, dL_du, dL_dr_out, lambda_out, max_sweeps, stats, s);
}

eik_status eik_adjoint(const eik_grid* grid, const void* r, const eik_gamma* gamma, const void* u,
                       const int8_t* wind, const void* dL_du, void* dL_dr_out, void* hip_stream) {
  return eik_adjoint_batch(grid, r, 1, gamma, u, wind, dL_du, dL_dr_out, nullptr, 100000, nullptr, hip_stream);
}

const char* eik_last_error(void) { return g_err.c_str(); }

eik_status eik_release(void) {
  for (int d = 0; d < kMaxDevices; ++d) {
    std::lock_guard<std::mutex> lock(g_ws[d].mu);
    if (g_ws[d].dev) {
      int cur = 0;
      (void)hipGetDevice(&cur);
      (void)hipSetDevice(d);
      (void)hipFree(g_ws[d].dev);
      if (g_ws[d].host) (void)hipHostFree(g_ws[d].host);
      (void)hipSetDevice(cur);
      g_ws[d].dev = nullptr;
      g_ws[d].host = nullptr;
      g_ws[d].bytes = 0;
    }
  }
  return EIK_OK;
}

const char* eik_version(void) { return "eik-mi355x 0.1 (gfx950)"; }

}  // extern "C"
