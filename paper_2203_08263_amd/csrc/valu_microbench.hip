// Issue-rate microbenchmark of the gfx950 vector ALU operations the
// all-pairs kernels are made of: FP32/FP64 fused multiply-add, multiply and
// add, the hardware reciprocal square root (v_rsq_f32 / v_rsq_f64), FP64 ->
// FP32 conversion, and an FMA stream with one reciprocal square root per 12
// FMAs (the mixed forward pair's mix).
//
// Every thread runs kChains independent dependency chains for `iters`
// iterations and writes one value, so the loop cannot be removed; the grid
// covers every compute unit many times over.  Rates are reported per second
// of wall time measured with HIP events on one stream, in lane-operations
// (one lane executing one instruction).  It also measures the accuracy of
// the two hardware reciprocal square root estimates (largest relative error
// over 4M arguments spread over many binades), which sets how much
// refinement the FP64 kernels need.  Output: one JSON object per line.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_),   \
              __FILE__, __LINE__);                                        \
      exit(1);                                                            \
    }                                                                     \
  } while (0)

constexpr int kThreads = 256;
constexpr int kChains = 8;

template <int OP, typename T>
__global__ __launch_bounds__(kThreads) void chains(int iters, T seed,
                                                   T *__restrict__ out) {
  T a[kChains];
  const T b = seed * T(0.999), c = seed * T(1e-3);
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = seed + T(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      if constexpr (OP == 0) a[k] = fma(a[k], b, c);          // fma
      if constexpr (OP == 1) a[k] = a[k] * b;                  // mul
      if constexpr (OP == 2) a[k] = a[k] + c;                  // add
      if constexpr (OP == 3) {                                 // rsq
        if constexpr (sizeof(T) == 4) a[k] = __builtin_amdgcn_rsqf(a[k]);
        else a[k] = __builtin_amdgcn_rsq(a[k]);
      }
    }
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// 12 FMAs and one v_rsq_f32 per chain and iteration.
__global__ __launch_bounds__(kThreads) void fma12_rsq1(int iters, float seed,
                                                       float *__restrict__ out) {
  float a[kChains], r[kChains];
  const float b = seed * 0.999f, c = seed * 1e-3f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    a[k] = seed + float(threadIdx.x + k);
    r[k] = 1.0f + float(k);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
#pragma unroll
      for (int q = 0; q < 12; ++q) a[k] = fmaf(a[k], b, c);
      r[k] = __builtin_amdgcn_rsqf(r[k]);
    }
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k] + r[k];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// FP64 -> FP32 conversion chains (convert, widen back: 2 ops per link).
__global__ __launch_bounds__(kThreads) void cvt_chain(int iters, double seed,
                                                      double *__restrict__ out) {
  double a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = seed + double(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = double(float(a[k])) * 1.0000001;
  }
  double s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Relative error |1 - s y^2| / 2 of the hardware estimate y of s^(-1/2):
// FP64 arguments in [2^-60, 2^60), FP32 ones in [2^-20, 2^20), mantissas
// from a counter-based hash of the sample index.
__device__ double hash_u01(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return double(k >> 11) * (1.0 / 9007199254740992.0);
}

__global__ __launch_bounds__(kThreads) void rsq_accuracy(int n, double *err64,
                                                         double *err32) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double m = 1.0 + hash_u01(2 * uint64_t(i));
  const int ex = int(hash_u01(2 * uint64_t(i) + 1) * 120.0) - 60;
  const double s = ldexp(m, ex);
  const double y = __builtin_amdgcn_rsq(s);
  err64[i] = fabs(fma(-(s * y), y, 1.0)) * 0.5;
  const float sf = float(ldexp(m, ex / 3));
  const float yf = __builtin_amdgcn_rsqf(sf);
  err32[i] = fabs(1.0 - double(sf) * double(yf) * double(yf)) * 0.5;
}

template <typename K>
static double time_ms(K launch, hipStream_t st) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  launch();  // warm-up
  CHECK(hipStreamSynchronize(st));
  const int reps = 5;
  CHECK(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) launch();
  CHECK(hipEventRecord(e1, st));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  CHECK(hipGetLastError());
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return double(ms) / reps;
}

int main(int argc, char **argv) {
  int dev = 0;
  CHECK(hipSetDevice(dev));
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount;
  const int blocks = cus * 32;                 // 8 waves per SIMD
  const int iters = argc > 1 ? atoi(argv[1]) : 2048;
  const size_t nthreads = size_t(blocks) * kThreads;
  void *buf = nullptr;
  CHECK(hipMalloc(&buf, nthreads * sizeof(double)));
  hipStream_t st;
  CHECK(hipStreamCreate(&st));
  printf("{\"device\": \"%s\", \"cus\": %d, \"clock_khz\": %d, \"blocks\": %d, "
         "\"threads\": %d, \"iters\": %d, \"chains\": %d}\n",
         prop.name, cus, prop.clockRate, blocks, kThreads, iters, kChains);
  const double lane_ops = double(nthreads) * iters * kChains;
  auto report = [&](const char *name, double ms, double ops_per_link) {
    const double rate = lane_ops * ops_per_link / (ms * 1e-3);
    printf("{\"op\": \"%s\", \"ms\": %.4f, \"lane_ops_per_s\": %.4e, "
           "\"per_cu_per_clk_at_2.4GHz\": %.2f}\n",
           name, ms, rate, rate / (cus * 2.4e9));
    fflush(stdout);
  };
  float *f = static_cast<float *>(buf);
  double *d = static_cast<double *>(buf);
  report("v_fma_f32", time_ms([&] { chains<0, float><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 1);
  report("v_mul_f32", time_ms([&] { chains<1, float><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 1);
  report("v_add_f32", time_ms([&] { chains<2, float><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 1);
  report("v_rsq_f32", time_ms([&] { chains<3, float><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 1);
  report("v_fma_f64", time_ms([&] { chains<0, double><<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 1);
  report("v_mul_f64", time_ms([&] { chains<1, double><<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 1);
  report("v_add_f64", time_ms([&] { chains<2, double><<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 1);
  report("v_rsq_f64", time_ms([&] { chains<3, double><<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 1);
  report("fma_f32_x12_plus_rsq_f32 (per op)",
         time_ms([&] { fma12_rsq1<<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 13);
  report("cvt_f32_f64+cvt_f64_f32+mul_f64 (per op)",
         time_ms([&] { cvt_chain<<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 3);

  const int nacc = 1 << 22;
  double *err = nullptr;
  CHECK(hipMalloc(&err, size_t(2) * nacc * sizeof(double)));
  rsq_accuracy<<<nacc / kThreads, kThreads, 0, st>>>(nacc, err, err + nacc);
  CHECK(hipGetLastError());
  CHECK(hipStreamSynchronize(st));
  double *h = static_cast<double *>(malloc(size_t(2) * nacc * sizeof(double)));
  if (!h) return 1;
  CHECK(hipMemcpy(h, err, size_t(2) * nacc * sizeof(double), hipMemcpyDeviceToHost));
  for (int k = 0; k < 2; ++k) {
    double w = 0.0;
    for (int i = 0; i < nacc; ++i) w = fmax(w, h[size_t(k) * nacc + i]);
    printf("{\"op\": \"%s accuracy\", \"samples\": %d, \"max_rel_err\": %.4e, "
           "\"log2\": %.2f}\n", k ? "v_rsq_f32" : "v_rsq_f64", nacc, w, log2(w));
  }
  free(h);
  CHECK(hipFree(err));
  CHECK(hipStreamDestroy(st));
  CHECK(hipFree(buf));
  return 0;
}
