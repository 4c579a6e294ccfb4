// Issue-rate microbenchmark of the gfx950 vector ALU operations the
// all-pairs kernels are made of: FP32/FP64 fused multiply-add, multiply and
// add, the hardware reciprocal square root (v_rsq_f32 / v_rsq_f64), FP64 ->
// FP32 conversion, and an FMA stream with one reciprocal square root per 12
// FMAs (the mixed forward pair's mix).  It also times a grid-wide barrier
// (cooperative-groups grid sync in a kernel launched cooperatively) for
// several grid sizes: the cost a one-launch multi-step loop would pay per
// step.
//
// Every thread runs kChains independent dependency chains for `iters`
// iterations and writes one value, so the loop cannot be removed; the grid
// covers every compute unit many times over.  Rates are reported per second
// of wall time measured with HIP events on one stream, in lane-operations
// (one lane executing one instruction).  It also measures the accuracy of
// the two hardware reciprocal square root estimates (largest relative error
// over 4M arguments spread over many binades), which sets how much
// refinement the FP64 kernels need.  Output: one JSON object per line.
#include <hip/hip_cooperative_groups.h>
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

template <int OP, typename T, int NCH = kChains, bool VOPS = false>
__global__ __launch_bounds__(kThreads) void chains(int iters, T seed,
                                                   T *__restrict__ out) {
  T a[NCH];
  // VOPS: per-thread multiplier and addend (VGPR operands) instead of
  // wave-uniform ones (scalar registers)
  const T t = VOPS ? T(threadIdx.x) * T(1e-6) : T(0);
  const T b = seed * T(0.999) + t, c = seed * T(1e-3) + t;
#pragma unroll
  for (int k = 0; k < NCH; ++k) a[k] = seed + T(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
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
  for (int k = 0; k < NCH; ++k) s += a[k];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// The forward pair's operation mix, NCH independent pairs per thread and
// iteration: 3 sub, 3 FMA (r^2 + eps^2), v_rsq_f32, 3 mul, 3 FMA into
// per-chain accumulators -- exactly 13 operations per pair.  Each chain's
// next source is its own accumulator (no memory traffic, nothing the
// compiler can hoist out of the loop).  Thread 0 of every workgroup records
// the shader-clock counter (clock64) and the constant-rate counter
// (wall_clock64) at its start and end into stamp[4 * blockIdx.x ...], so the
// host can derive the clock the chip ran at under this load.
// The VJP pair of the library's FP32 kernels in split form (3 sub, 3 FMA,
// rsq, 2 mul, g_j.e and g_k.e, e.h, 2 mul, 8 FMA into the sums: 26
// operations + rsq), NCH independent chains per thread, the pair
// difference taken from the chain's own c sums so every iteration depends
// on the last.
template <int NCH>
__global__ __launch_bounds__(kThreads) void vjp_mix(int iters, float seed,
                                                    float *__restrict__ out,
                                                    unsigned long long *stamp) {
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) {
    c0 = clock64();
    w0 = wall_clock64();
  }
  const float xi = seed * float(threadIdx.x) * 1e-3f;
  const float yi = -xi, zi = 0.5f * xi, eps2 = 1e-6f;
  const float mk = 1e-4f, mj = 2e-4f, gkx = 0.3f, gky = -0.2f, gkz = 0.1f;
  float ax[NCH], ay[NCH], az[NCH], b[NCH], cx[NCH], cy[NCH], cz[NCH], dm[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    ax[k] = ay[k] = az[k] = b[k] = dm[k] = 0.0f;
    cx[k] = 0.25f + float(k);
    cy[k] = -0.5f;
    cz[k] = 0.75f - float(k);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const float gjx = 0.5f + 0.1f * float(k), gjy = -0.25f, gjz = seed;
      const float ex = cx[k] - xi, ey = cy[k] - yi, ez = cz[k] - zi;
      float s = fmaf(ex, ex, eps2);
      s = fmaf(ey, ey, s);
      s = fmaf(ez, ez, s);
      const float y = __builtin_amdgcn_rsqf(s);
      const float y2 = y * y;
      const float y3 = y2 * y;
      const float ge = fmaf(gjz, ez, fmaf(gjy, ey, gjx * ex));
      const float ek = fmaf(gkz, ez, fmaf(gky, ey, gkx * ex));
      const float eh = fmaf(mk, ge, -(mj * ek));
      const float w = y3 * (y2 * eh);
      dm[k] = fmaf(ge, y3, dm[k]);
      ax[k] = fmaf(y3, gjx, ax[k]);
      ay[k] = fmaf(y3, gjy, ay[k]);
      az[k] = fmaf(y3, gjz, az[k]);
      b[k] = fmaf(y3, mj, b[k]);
      cx[k] = fmaf(w, ex, cx[k]);
      cy[k] = fmaf(w, ey, cy[k]);
      cz[k] = fmaf(w, ez, cz[k]);
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int k = 0; k < NCH; ++k)
    r += ax[k] + ay[k] + az[k] + b[k] + cx[k] + cy[k] + cz[k] + dm[k];
  out[blockIdx.x * kThreads + threadIdx.x] = r;
  if (threadIdx.x == 0) {
    const unsigned long long c1 = clock64(), w1 = wall_clock64();
    unsigned long long *o = stamp + 4 * size_t(blockIdx.x);
    o[0] = c0;
    o[1] = c1;
    o[2] = w0;
    o[3] = w1;
  }
}

template <int NCH>
__global__ __launch_bounds__(kThreads) void pair_mix(int iters, float seed,
                                                     float *__restrict__ out,
                                                     unsigned long long *stamp) {
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) {
    c0 = clock64();
    w0 = wall_clock64();
  }
  const float xi = seed * float(threadIdx.x) * 1e-3f;
  const float yi = -xi, zi = 0.5f * xi, eps2 = 1e-6f;
  float ax[NCH], ay[NCH], az[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    ax[k] = 0.25f + float(k);
    ay[k] = -0.5f;
    az[k] = 0.75f - float(k);
  }
  const float m = 1e-4f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const float dx = ax[k] - xi, dy = ay[k] - yi, dz = az[k] - zi;
      float s = fmaf(dx, dx, eps2);
      s = fmaf(dy, dy, s);
      s = fmaf(dz, dz, s);
      const float y = __builtin_amdgcn_rsqf(s);
      const float w = (m * y) * (y * y);
      ax[k] = fmaf(w, dx, ax[k]);
      ay[k] = fmaf(w, dy, ay[k]);
      az[k] = fmaf(w, dz, az[k]);
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int k = 0; k < NCH; ++k) r += ax[k] + ay[k] + az[k];
  out[blockIdx.x * kThreads + threadIdx.x] = r;
  if (threadIdx.x == 0) {
    const unsigned long long c1 = clock64(), w1 = wall_clock64();
    unsigned long long *o = stamp + 4 * size_t(blockIdx.x);
    o[0] = c0;
    o[1] = c1;
    o[2] = w0;
    o[3] = w1;
  }
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

// `iters` grid-wide barriers (every workgroup runs the same count, so all
// of them reach every barrier); launched only through
// hipLaunchCooperativeKernel, which refuses a grid that cannot be resident.
__global__ __launch_bounds__(kThreads) void grid_syncs(int iters,
                                                       double *__restrict__ out) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  double acc = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    acc = acc * 1.0000001 + 1.0;
    grid.sync();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
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
  report("v_fma_f32, 16 chains",
         time_ms([&] { chains<0, float, 16><<<blocks, kThreads, 0, st>>>(iters / 2, 1.0f, f); }, st), 1);
  report("v_fma_f32, 8 chains, VGPR operands",
         time_ms([&] { chains<0, float, 8, true><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f); }, st), 1);
  report("v_add_f32, 16 chains",
         time_ms([&] { chains<2, float, 16><<<blocks, kThreads, 0, st>>>(iters / 2, 1.0f, f); }, st), 1);
  report("v_rsq_f32, 16 chains",
         time_ms([&] { chains<3, float, 16><<<blocks, kThreads, 0, st>>>(iters / 2, 1.0f, f); }, st), 1);

  // The forward pair mix (13 operations per pair) with 4, 8 and 16
  // independent pairs per thread, and the shader clock it ran at.
  int wall_khz = 0;
  CHECK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
  unsigned long long *stamp = nullptr;
  CHECK(hipMalloc(&stamp, size_t(4) * blocks * sizeof(unsigned long long)));
  unsigned long long *hs = static_cast<unsigned long long *>(
      malloc(size_t(4) * blocks * sizeof(unsigned long long)));
  if (!hs) return 1;
  auto mix = [&](const char *name, double ms, int nch) {
    CHECK(hipMemcpy(hs, stamp, size_t(4) * blocks * sizeof(unsigned long long),
                    hipMemcpyDeviceToHost));
    double cyc = 0.0, wall = 0.0, fmin = 1e30, fmax = 0.0;
    for (int b = 0; b < blocks; ++b) {
      const double dc = double(hs[4 * b + 1] - hs[4 * b]);
      const double dw = double(hs[4 * b + 3] - hs[4 * b + 2]);
      cyc += dc;
      wall += dw;
      if (dw > 0) {
        const double fb = dc / dw * wall_khz * 1e-6;
        fmin = fb < fmin ? fb : fmin;
        fmax = fb > fmax ? fb : fmax;
      }
    }
    const double ghz = wall > 0 ? cyc / wall * wall_khz * 1e-6 : 0.0;
    const double pairs = double(nthreads) * (iters / (nch / 4)) * nch;
    const double pps = pairs / (ms * 1e-3);
    printf("{\"op\": \"%s\", \"ms\": %.4f, \"pairs_per_s\": %.4e, "
           "\"pairs_per_cu_per_clk_at_2.4GHz\": %.3f, \"clock64_ghz_mean\": %.3f, "
           "\"clock64_ghz_min\": %.3f, \"clock64_ghz_max\": %.3f, "
           "\"wall_clock_khz\": %d}\n",
           name, ms, pps, pps / (cus * 2.4e9), ghz, fmin, fmax, wall_khz);
    fflush(stdout);
  };
  mix("pair_mix_f32, 4 pairs per thread",
      time_ms([&] { pair_mix<4><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f, stamp); }, st), 4);
  mix("pair_mix_f32, 8 pairs per thread",
      time_ms([&] { pair_mix<8><<<blocks, kThreads, 0, st>>>(iters / 2, 1.0f, f, stamp); }, st), 8);
  mix("pair_mix_f32, 16 pairs per thread",
      time_ms([&] { pair_mix<16><<<blocks, kThreads, 0, st>>>(iters / 4, 1.0f, f, stamp); }, st), 16);
  mix("vjp_mix_f32 (split form), 4 pairs per thread",
      time_ms([&] { vjp_mix<4><<<blocks, kThreads, 0, st>>>(iters, 1.0f, f, stamp); }, st), 4);
  mix("vjp_mix_f32 (split form), 8 pairs per thread",
      time_ms([&] { vjp_mix<8><<<blocks, kThreads, 0, st>>>(iters / 2, 1.0f, f, stamp); }, st), 8);
  free(hs);
  CHECK(hipFree(stamp));
  report("cvt_f32_f64+cvt_f64_f32+mul_f64 (per op)",
         time_ms([&] { cvt_chain<<<blocks, kThreads, 0, st>>>(iters, 1.0, d); }, st), 3);

  // Grid-wide barrier cost: 1000 barriers per launch, several grid sizes up
  // to what can be resident (the occupancy query bounds the grid).
  int coop = 0, per_cu = 0;
  CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, grid_syncs,
                                                     kThreads, 0));
  if (coop) {
    for (int gb : {8, 64, 256, 1024}) {
      if (gb > per_cu * cus || size_t(gb) > nthreads) continue;
      int nsync = 1000;
      void *args[] = {&nsync, &d};
      const double ms = time_ms([&] {
        CHECK(hipLaunchCooperativeKernel((void *)grid_syncs, dim3(gb),
                                         dim3(kThreads), args, 0, st));
      }, st);
      printf("{\"op\": \"cooperative grid sync\", \"workgroups\": %d, "
             "\"ms\": %.4f, \"us_per_sync\": %.3f}\n", gb, ms, ms * 1e3 / nsync);
      fflush(stdout);
    }
  }

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
