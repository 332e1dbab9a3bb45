// Measured ceilings of the GPU the benchmark runs on, reported next to the
// published peaks: the non-FMA VALU issue rate (independent fp32 add chains
// in every lane of enough waves to fill every SIMD), the latency of one
// dependent fp32 add in a lone wave, and the LDS read bandwidth.  Not part of
// the solver: a separate library that bench.py loads.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

// kChains independent add chains per lane; every add is one VALU operation
__global__ __launch_bounds__(256) void k_valu(float* sink, int iters, float step) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = (float)(threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = v[c] + step;
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s = s + v[c];
  if (s == 1.2345f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the loop alive
}

// one wave, one dependent chain: cycles per dependent add from the clock
// (32 adds per loop trip, so the loop's own instructions hardly count)
__global__ __launch_bounds__(64) void k_latency(long long* out, int iters, float step) {
  float v = (float)threadIdx.x;
  const long long t0 = clock64();
  for (int i = 0; i < iters; i += 32) {
#pragma unroll
    for (int k = 0; k < 32; ++k) v = v + step;
  }
  const long long t1 = clock64();
  if (threadIdx.x == 0) {
    out[0] = t1 - t0;
    out[1] = (long long)v;  // keeps the chain alive
  }
}

// LDS reads of 16 bytes per lane per iteration over a 32 KiB buffer
__global__ __launch_bounds__(256) void k_lds(float* sink, int iters) {
  __shared__ float4 buf[2048];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) buf[i] = make_float4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  float4 acc = make_float4(0, 0, 0, 0);
  int idx = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
    const float4 a = buf[idx];
    acc.x += a.x; acc.y += a.y; acc.z += a.z; acc.w += a.w;
    idx = (idx + 256) & 2047;
    __asm__ __volatile__("" ::: "memory");  // every trip reads LDS again
  }
  const float s = (acc.x + acc.y) + (acc.z + acc.w);
  if (s == 1.2345f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

float timed(hipStream_t s, void (*launch)(hipStream_t, void*), void* arg) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
  launch(s, arg);  // warm-up
  (void)hipEventRecord(a, s);
  launch(s, arg);
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = -1.0f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

struct Args {
  int blocks, iters;
  float* sink;
  long long* lat;
};

}  // namespace

extern "C" {

// Fills out[0..3]: VALU adds/s, cycles per dependent add, LDS bytes/s,
// clock ticks per second of clock64 (measured against the event timer).
// sink: device scratch of blocks*256 floats; lat: device scratch of 2 int64.
// Returns 0, or -1 on a HIP error.
int ceil_measure(int blocks, int iters, float* sink, long long* lat, double* out, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  Args A{blocks, iters, sink, lat};
  const float ms_valu = timed(
      s, [](hipStream_t st, void* p) {
        const Args* a = (const Args*)p;
        hipLaunchKernelGGL(k_valu, dim3(a->blocks), dim3(256), 0, st, a->sink, a->iters, 1.0f);
      },
      &A);
  const float ms_lds = timed(
      s, [](hipStream_t st, void* p) {
        const Args* a = (const Args*)p;
        hipLaunchKernelGGL(k_lds, dim3(a->blocks), dim3(256), 0, st, a->sink, a->iters);
      },
      &A);
  const float ms_lat = timed(
      s, [](hipStream_t st, void* p) {
        const Args* a = (const Args*)p;
        hipLaunchKernelGGL(k_latency, dim3(1), dim3(64), 0, st, a->lat, a->iters * 64, 1.0f);
      },
      &A);
  if (hipGetLastError() != hipSuccess || ms_valu <= 0 || ms_lds <= 0 || ms_lat <= 0) return -1;
  long long h[2] = {0, 0};
  if (hipMemcpy(h, lat, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  const double adds = (double)blocks * 256.0 * iters * kChains;
  out[0] = adds / (ms_valu * 1e-3);
  out[1] = (double)h[0] / ((double)iters * 64.0);
  out[2] = (double)blocks * 256.0 * iters * 16.0 / (ms_lds * 1e-3);
  out[3] = (double)h[0] / (ms_lat * 1e-3);
  return 0;
}

}  // extern "C"
