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
// (one lane executing one instruction).  Output: one JSON object per line.
#include <hip/hip_runtime.h>
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
  CHECK(hipStreamDestroy(st));
  CHECK(hipFree(buf));
  return 0;
}
