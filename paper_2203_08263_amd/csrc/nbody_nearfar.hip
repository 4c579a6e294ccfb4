// gfx950 kernels of the near / far precision modes (NBODY_MIXED_NF and
// NBODY_MIXED_NF64) and of the Morton (Z-order) sort that puts bodies in the
// spatial order those modes are fast in.
#include <type_traits>

#include "nbody_device.h"

namespace nbody {
namespace {

constexpr int kBodyThreadsSort = 256;

// ------------------------------------------------- near / far (mixed NF) --
//
// NBODY_MIXED_NF chooses the pair arithmetic per run of sources that one
// FP32 chunk sum covers (C consecutive entries per lane, C*L sources) and per
// wave:
//  - far runs: coordinates relative to the centre c of the workgroup's
//    target bounding box (half-diagonal b), x - c taken in FP64 and rounded
//    once to FP32, then the FP32 pair arithmetic of NBODY_MIXED.  A run is far
//    for a wave when the gap between the run's bounding box and the bounding
//    box of the wave's own targets exceeds kappa b, so every such pair has
//    |d| > kappa b, and the coordinate error is at most
//    u32 (|x_j - c| + |x_i - c| + |d|) <= u32 (2 |d| + 2 b) < (2 + 2/kappa) u32 |d|
//    (kappa = 1/2: below 6 u32 |d|, the order of one rounding of d itself);
//  - near runs: the NBODY_MIXED_D64 arithmetic (difference in FP64, rounded
//    once to FP32), which keeps the close pairs -- whose errors dominate --
//    as accurate as that mode; or, for NBODY_MIXED_NF64 (NEAR64), the FP64
//    pair added straight into the FP64 sums, so the close pairs carry FP64
//    rounding only.
// Both forms of every source are staged in LDS; the choice is uniform over
// each wave (no divergence) and depends only on positions, so results stay
// deterministic.  All boxes (source runs, the targets of each wave and of
// each workgroup) come from group_box_kernel, launched just before the
// all-pairs kernel, so the kernel itself only reads them.  With bodies in a
// spatial order
// (nbody_morton_sort) most runs are far and the kernel runs close to the
// NBODY_MIXED rate; in a random order every run is near and the results are
// bitwise those of NBODY_MIXED_D64.

constexpr double kNearFarKappa2 = 0.25;  // kappa = 1/2
// FP32 far-run sources whose weights are formed ahead of their sums
// (chunk_sum_f32): 4 keeps the forward kernels within 64 VGPRs (8 waves per
// SIMD), which 8 would not.
constexpr int kNfFarBatch = 4;

// FP32 sources per chunk sum, and so per near / far decision, of each kernel
// (per lane; a run of the tile is C*L consecutive sources).  The forward of
// NBODY_MIXED_NF64 takes chunks of 16: half the FP32 summation error in its
// far runs, which sets its worst relative error (bodies near the centre of a
// cluster, whose net acceleration almost cancels), and smaller run boxes, so
// fewer runs are near, for one more FP64 flush per 16 pairs (measured: the
// largest relative error over all 262144 bodies of a clustered Plummer
// system 1.1e-6 -> 7.2e-7; +4 % at N = 16384, -3 % at N = 262144).
constexpr int kNf64Chunk = 16;
// The NBODY_MIXED_NF64 VJP keeps runs of 16 sources (the other VJPs: 32):
// its near runs are FP64 pairs, and finer runs leave fewer of them near.
constexpr int kNf64VjpChunk = 16;

constexpr int nf_chunk(KernelKind kind, bool near64) {
  if (kind == kVjp) return near64 ? kNf64VjpChunk : kVjpChunk;
  return near64 ? kNf64Chunk : kChunk;
}

// Sources per near / far decision of each kernel at lanes-per-target L.
constexpr int nf_run(KernelKind kind, int L, bool near64) {
  return (kThreads / L < nf_chunk(kind, near64) ? kThreads / L
                                                : nf_chunk(kind, near64)) *
         L;
}

struct Box {
  double lo[3], hi[3];
};

// Near form of a source for NBODY_MIXED_NF: its FP64 coordinates only (the
// D64 arithmetic takes the mass and dL/da in FP32, from the far tile).
struct NearXYZ {
  double x, y, z;
};

// Minimum over the lanes of each aligned group of `width` lanes (a power of
// two up to 64) of the 6 values {x, y, z, -x, -y, -z}.
__device__ __forceinline__ void group_min6(double v[6], int width) {
  for (int m = 1; m < width; m <<= 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = fmin(v[c], __shfl_xor(v[c], m));
  }
}

__device__ __forceinline__ void box_init6(double v[6], bool ok, double x,
                                          double y, double z) {
  const double inf = __builtin_huge_val();
  v[0] = ok ? x : inf;
  v[1] = ok ? y : inf;
  v[2] = ok ? z : inf;
  v[3] = ok ? -x : inf;
  v[4] = ok ? -y : inf;
  v[5] = ok ? -z : inf;
}

// A value that is the same in every lane of the wave, moved to scalar
// registers (readfirstlane of both halves).
__device__ __forceinline__ double wave_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

// Boxes of the groups of w consecutive bodies base .. base + count - 1 of a
// [3][stride] position array, for up to three group widths wk (powers of two
// in [4, 256]; 0 = unused): bk[g*6 + {0,1,2}] = min of x, y, z over group g,
// bk[g*6 + {3,4,5}] = max, for every group that starts below count.
// NaN coordinates are ignored (minNum).
__global__ __launch_bounds__(kThreads) void group_box_kernel(
    int stride, int base, int count, const double *__restrict__ pos, int w0,
    double *__restrict__ b0, int w1, double *__restrict__ b1, int w2,
    double *__restrict__ b2) {
  __shared__ double red[4 * 6];
  const int j = blockIdx.x * kThreads + threadIdx.x;
  const bool ok = j < count;
  double v[6];
  box_init6(v, ok, ok ? pos[base + j] : 0.0, ok ? pos[stride + base + j] : 0.0,
            ok ? pos[2 * stride + base + j] : 0.0);
  auto emit = [&](int w, double *b) {
    if ((threadIdx.x & (w - 1)) == 0 && j < count) {
      double *o = b + size_t(j / w) * 6;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        o[c] = v[c];
        o[3 + c] = -v[3 + c];
      }
    }
  };
  for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = fmin(v[c], __shfl_xor(v[c], m));
    if (w0 == 2 * m) emit(w0, b0);
    if (w1 == 2 * m) emit(w1, b1);
    if (w2 == 2 * m) emit(w2, b2);
  }
  if (w0 > 64 || w1 > 64 || w2 > 64) {  // uniform: kernel arguments
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) red[wv * 6 + c] = v[c];
    }
    __syncthreads();
    for (int w = 128; w <= kThreads; w <<= 1) {
      if ((threadIdx.x & (w - 1)) == 0) {
        double u[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) u[c] = red[wv * 6 + c];
        for (int k = 1; k < w / 64; ++k) {
#pragma unroll
          for (int c = 0; c < 6; ++c) u[c] = fmin(u[c], red[(wv + k) * 6 + c]);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = u[c];
      }
      if (w0 == w) emit(w0, b0);
      if (w1 == w) emit(w1, b1);
      if (w2 == w) emit(w2, b2);
    }
  }
}

// Box g of a box array, in scalar registers (the index is uniform).
__device__ __forceinline__ Box read_box(const double *__restrict__ b, int g) {
  Box r;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r.lo[c] = wave_uniform(b[size_t(g) * 6 + c]);
    r.hi[c] = wave_uniform(b[size_t(g) * 6 + 3 + c]);
  }
  return r;
}

// Far / near decisions of the NR runs of one tile (first source jt) for the
// calling thread's wave: bit r of the result is set when run r is far.  Lane
// r of the wave evaluates run r (a box gap in FP64) and a ballot gathers the
// bits, so the per-chunk test is a scalar bit test.  Runs entirely past jend
// (tile padding) are near.
template <int RUN>
__device__ __forceinline__ uint64_t far_runs(const Box &wave, double thr2,
                                             const double *__restrict__ boxes,
                                             int jt, int jend) {
  constexpr int NR = kThreads / RUN;
  const int lane = threadIdx.x & 63;
  const int rs = jt + lane * RUN;
  bool far = false;
  if (lane < NR && rs < jend) {
    const double *sb = boxes + size_t(rs / RUN) * 6;
    double gap2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double g =
          fmax(0.0, fmax(sb[c] - wave.hi[c], wave.lo[c] - sb[3 + c]));
      gap2 += g * g;
    }
    far = gap2 > thr2;
  }
  return __ballot(far);
}

// far_runs' result when every run of a tile is far for the wave.
template <int RUN>
constexpr uint64_t all_runs_mask() {
  constexpr int NR = kThreads / RUN;
  return NR >= 64 ? ~uint64_t(0) : ((uint64_t(1) << NR) - 1);
}

// Whether any wave of the workgroup has a near run in the current tile (the
// flags each wave's first lane wrote before the barrier): only then is the
// near form of the tile staged.
__device__ __forceinline__ bool any_wave_near(const int *wave_near) {
  int any = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) any |= wave_near[w];
  return any != 0;
}

// Centre and far threshold (kappa b)^2 of the workgroup's target box.
__device__ __forceinline__ double far_frame(const Box &block, double c[3]) {
  double b2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.5 * (block.lo[k] + block.hi[k]);
    const double e = block.hi[k] - block.lo[k];
    b2 += e * e;
  }
  return kNearFarKappa2 * 0.25 * b2;
}

// Box arrays of the near / far kernels: run boxes over all n sources (RUN
// bodies each), wave boxes over the nt targets (64/L each) and workgroup
// boxes over the targets (256/L each).
struct NfBoxes {
  const double *run;
  const double *wave;
  const double *block;
};

// The wave's and the workgroup's target boxes; a wave with no valid target
// (tail of the last workgroup) gets an empty box, so every run is far for it.
template <int L>
__device__ __forceinline__ void target_boxes(const NfBoxes &bx, int nt, int ib,
                                             Box &wave, Box &block) {
  constexpr int GW = 64 / L;
  // wave index, uniform across the wave (scalar registers and branches)
  const int wg = __builtin_amdgcn_readfirstlane(
      ib * (kThreads / 64) + int(threadIdx.x) / 64);
  const bool has = wg * GW < nt;
  block = read_box(bx.block, ib);
  wave = read_box(bx.wave, has ? wg : 0);  // box 0 always exists
  const double inf = __builtin_huge_val();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    wave.lo[c] = has ? wave.lo[c] : inf;
    wave.hi[c] = has ? wave.hi[c] : -inf;
  }
}

// Dispatch order of the near / far launches.  A workgroup's task is one
// (target block ib, source split s) pair, numbered s * n_ib + ib, and its cost
// grows with the near runs it holds: in a spatially sorted clustered system
// the tasks of the dense core are all near and cost up to twice a far one, and
// when they are dispatched late in grid order they form the launch's tail.
// nf_load_kernel counts the near (wave, run) pairs of every task from the box
// arrays, nf_order_kernel sorts the task numbers into three load classes
// (near share >= 1/4, >= 1/128, the rest; stable, so each class keeps the
// split-major grid order and its L2 locality), and the kernels take task
// order[blockIdx.y * n_ib + blockIdx.x], so the costliest tasks start first.
// Each task writes only its own partial sums, so the order changes when work
// runs, never what it computes.
struct NfTask {
  int ib, s;
};

__device__ __forceinline__ NfTask nf_task(const int *__restrict__ order) {
  if (!order) return NfTask{int(blockIdx.x), int(blockIdx.y)};
  const int t = __builtin_amdgcn_readfirstlane(
      order[int(blockIdx.y) * int(gridDim.x) + int(blockIdx.x)]);
  return NfTask{t % int(gridDim.x), t / int(gridDim.x)};
}

constexpr int kOrderMaxSplits = 64;   // the plans' source split limit
// Load classes of the dispatch order: near share >= 2^-kOrderShift[k].
constexpr int kOrderShift[] = {2, 7};
constexpr int kOrderClasses = sizeof(kOrderShift) / sizeof(int) + 1;

// Load class of a task with `load` of at most `maxload` near (wave, run)
// pairs: the first k with load / maxload >= 2^-kOrderShift[k], else the last.
__device__ __forceinline__ int order_class(int load, int maxload) {
  const int64_t l = min(max(load, 0), maxload);
  int k = 0;
  while (k < kOrderClasses - 1 && (l << kOrderShift[k]) < int64_t(maxload)) ++k;
  return k;
}

// Near (wave, run) pairs of each task, as its load class (against the
// (wave, run) pairs of its split): one workgroup per target block ib
// (gridDim.x = n_ib), cls[s * n_ib + ib] for each source split s.  The test
// is the kernels' own (a run is near for a wave unless the gap between their
// boxes exceeds kappa b).
__global__ __launch_bounds__(kThreads) void nf_load_kernel(
    int n, int nt, NfBoxes bx, int run, int gw, SplitShape split, int nsplit,
    unsigned char *__restrict__ cls) {
  __shared__ int count[kOrderMaxSplits];
  const int ib = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < nsplit) count[tid] = 0;
  const Box block = read_box(bx.block, ib);
  double c[3];
  const double thr2 = far_frame(block, c);
  constexpr int W = kThreads / 64;
  Box wave[W];
  bool has[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int wg = ib * W + w;
    has[w] = wg * gw < nt;
    wave[w] = read_box(bx.wave, has[w] ? wg : 0);
  }
  __syncthreads();
  const int nr = (n + run - 1) / run;
  for (int r = tid; r < nr; r += kThreads) {
    const double *sb = bx.run + size_t(r) * 6;
    double lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = sb[k];
      hi[k] = sb[3 + k];
    }
    int near = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      double gap2 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double g =
            fmax(0.0, fmax(lo[k] - wave[w].hi[k], wave[w].lo[k] - hi[k]));
        gap2 += g * g;
      }
      near += (has[w] && !(gap2 > thr2)) ? 1 : 0;
    }
    if (near) atomicAdd(&count[split_of(split, r * run)], near);
  }
  __syncthreads();
  if (tid < nsplit) {
    int jb, je;
    split_range(split, tid, n, jb, je);
    const int maxload = max(1, W * ((je - jb + run - 1) / run));
    cls[size_t(tid) * gridDim.x + ib] =
        static_cast<unsigned char>(order_class(count[tid], maxload));
  }
}

// One workgroup: order <- the task numbers 0 .. ntask-1 by load class (class
// 0 first), and within a class in increasing task number (a stable counting
// sort).  Task numbers are split-major, so within a class the resident
// workgroups share few source splits and the L2 keeps their sources.  The
// classes are staged in LDS when they fit (kOrderLdsTasks), read from global
// memory otherwise; thread t sorts tasks [t * chunk, (t + 1) * chunk).
constexpr int kOrderLdsTasks = 16384;

__global__ __launch_bounds__(kThreads) void nf_order_kernel(
    int ntask, const unsigned char *__restrict__ cls, int *__restrict__ order) {
  constexpr int K = kOrderClasses;
  __shared__ int cnt[K * kThreads];  // [class][thread], then its exclusive scan
  __shared__ int part[kThreads];
  __shared__ unsigned char lcls[kOrderLdsTasks];
  const int tid = threadIdx.x;
  const bool staged = ntask <= kOrderLdsTasks;  // uniform
  if (staged)
    for (int t = tid; t < ntask; t += kThreads) lcls[t] = cls[t];
  auto cl = [&](int t) { return int(staged ? lcls[t] : cls[t]); };
  const int chunk = (ntask + kThreads - 1) / kThreads;
  const int t0 = min(ntask, tid * chunk), t1 = min(ntask, t0 + chunk);
#pragma unroll
  for (int k = 0; k < K; ++k) cnt[k * kThreads + tid] = 0;
  __syncthreads();
  for (int t = t0; t < t1; ++t) ++cnt[cl(t) * kThreads + tid];
  __syncthreads();
  // exclusive scan of cnt in [class][thread] order: thread t owns entries
  // [t * K, (t + 1) * K)
  int local = 0;
#pragma unroll
  for (int e = 0; e < K; ++e) local += cnt[tid * K + e];
  part[tid] = local;
  for (int off = 1; off < kThreads; off <<= 1) {
    __syncthreads();
    const int add = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += add;
  }
  __syncthreads();
  int run = part[tid] - local;
#pragma unroll
  for (int e = 0; e < K; ++e) {
    const int c = cnt[tid * K + e];
    cnt[tid * K + e] = run;
    run += c;
  }
  __syncthreads();
  for (int t = t0; t < t1; ++t) order[cnt[cl(t) * kThreads + tid]++] = t;
}

template <int L, bool NEAR64>
__global__ __launch_bounds__(kThreads) void accel_nf_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, NfBoxes bx, const int *__restrict__ order,
    double eps2d, double scale, SplitShape split, double *__restrict__ out,
    size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = nf_run(kAccel, L, NEAR64) / L;  // sources per lane and run
  constexpr int RUN = C * L;  // sources of one chunk run (box granularity)
  using NearSrc = std::conditional_t<NEAR64, Src<NBODY_FP64>, NearXYZ>;
  __shared__ NearSrc near_tile[kThreads];
  __shared__ Src<NBODY_MIXED> far_tile[kThreads];
  __shared__ int wave_near[kThreads / 64];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const NfTask task = nf_task(order);
  const int i = task.ib * G + g;
  int jbeg, jend;
  split_range(split, task.s, n, jbeg, jend);
  const bool ok = i < nt;
  const int gi = row0 + i;
  const double xi = ok ? pos[gi] : 0.0;
  const double yi = ok ? pos[n + gi] : 0.0;
  const double zi = ok ? pos[2 * n + gi] : 0.0;
  Box wave, block;
  target_boxes<L>(bx, nt, task.ib, wave, block);
  double c[3];
  const double thr2 = far_frame(block, c);
  const float xr = float(xi - c[0]);
  const float yr = float(yi - c[1]);
  const float zr = float(zi - c[2]);
  const float eps2 = float(eps2d);
  double ax = 0.0, ay = 0.0, az = 0.0;

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    const bool valid = j < jend;
    const double xj = valid ? pos[j] : 0.0;
    const double yj = valid ? pos[n + j] : 0.0;
    const double zj = valid ? pos[2 * n + j] : 0.0;
    const double mj64 = valid ? mass[j] : 0.0;
    const float mj = float(mj64);
    NearSrc bn{};
    bn.x = xj;
    bn.y = yj;
    bn.z = zj;
    if constexpr (NEAR64) bn.m = mj64;
    Src<NBODY_MIXED> bf{};
    if (valid) {
      bf.x = float(xj - c[0]);
      bf.y = float(yj - c[1]);
      bf.z = float(zj - c[2]);
      bf.m = mj;
    }
    const uint64_t far_mask = far_runs<RUN>(wave, thr2, bx.run, jt, jend);
    // the all-far path (measured: -2 % at N = 262144 for NBODY_MIXED_NF at
    // L = 1, -3 % for NBODY_MIXED_NF64) except NBODY_MIXED_NF at L > 1, where
    // its second copy of the pair loop would cost occupancy (66 VGPRs)
    constexpr bool kFast = NEAR64 || L == 1;
    const bool all_far = kFast && far_mask == all_runs_mask<RUN>();
    if (kFast && (tid & 63) == 0) wave_near[tid / 64] = !all_far;
    __syncthreads();  // previous tile fully consumed; the waves' flags visible
    if (!kFast || any_wave_near(wave_near)) near_tile[tid] = bn;
    far_tile[tid] = bf;
    __syncthreads();

    if constexpr (kFast) if (all_far) {
      // every run of this tile is far for the wave: no per-chunk decisions
#pragma unroll 2
      for (int u0 = 0; u0 < PER; u0 += C) {
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        chunk_sum_f32<C, kNfFarBatch>(
            [&](int u, float &dx, float &dy, float &dz, float &m) {
              const Src<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
              dx = s.x - xr;
              dy = s.y - yr;
              dz = s.z - zr;
              m = s.m;
            },
            eps2, fx, fy, fz);
        ax += double(fx);
        ay += double(fy);
        az += double(fz);
      }
      continue;
    }
    for (int u0 = 0; u0 < PER; u0 += C) {
      const bool far = (far_mask >> (u0 / C)) & 1u;  // run u0 / C of the tile
      if constexpr (NEAR64) {
        if (!far) {
#pragma unroll 4
          for (int u = 0; u < C; ++u) {
            const NearSrc s = near_tile[(u0 + u) * L + q];
            pair_f64(s.x - xi, s.y - yi, s.z - zi, double(s.m), eps2d, ax, ay,
                     az);
          }
          continue;
        }
      }
      float fx = 0.0f, fy = 0.0f, fz = 0.0f;
      if (far) {
        chunk_sum_f32<C, kNfFarBatch>(
            [&](int u, float &dx, float &dy, float &dz, float &m) {
              const Src<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
              dx = s.x - xr;
              dy = s.y - yr;
              dz = s.z - zr;
              m = s.m;
            },
            eps2, fx, fy, fz);
      } else if constexpr (!NEAR64) {
        chunk_sum_f32<C, 1>(
            [&](int u, float &dx, float &dy, float &dz, float &m) {
              const NearSrc s = near_tile[(u0 + u) * L + q];
              dx = float(s.x - xi);
              dy = float(s.y - yi);
              dz = float(s.z - zi);
              m = far_tile[(u0 + u) * L + q].m;
            },
            eps2, fx, fy, fz);
      }
      ax += double(fx);
      ay += double(fy);
      az += double(fz);
    }
  }

  double *o = out + size_t(task.s) * split_stride;
  const double sx = group_sum<L>(ax);
  const double sy = group_sum<L>(ay);
  const double sz = group_sum<L>(az);
  if (q == 0 && ok) {
    o[i] = scale * sx;
    o[nt + i] = scale * sy;
    o[2 * nt + i] = scale * sz;
  }
}

template <int L, bool NEAR64>
__global__ __launch_bounds__(kThreads) void vjp_nf_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, const double *__restrict__ gacc,
    NfBoxes bx, const int *__restrict__ order, double eps2d, double scale,
    SplitShape split, double *__restrict__ out_x, double *__restrict__ out_m,
    size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = nf_run(kVjp, L, NEAR64) / L;
  constexpr int RUN = C * L;
  using NearSrc = std::conditional_t<NEAR64, VSrc<NBODY_FP64>, NearXYZ>;
  __shared__ NearSrc near_tile[kThreads];
  __shared__ VSrc<NBODY_MIXED> far_tile[kThreads];
  __shared__ int wave_near[kThreads / 64];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const NfTask task = nf_task(order);
  const int k = task.ib * G + g;
  int jbeg, jend;
  split_range(split, task.s, n, jbeg, jend);
  const bool ok = k < nt;
  const int gk = row0 + k;
  const double xk = ok ? pos[gk] : 0.0;
  const double yk = ok ? pos[n + gk] : 0.0;
  const double zk = ok ? pos[2 * n + gk] : 0.0;
  const double mk64 = ok ? mass[gk] : 0.0;
  const double gkx64 = ok ? gacc[gk] : 0.0;
  const double gky64 = ok ? gacc[n + gk] : 0.0;
  const double gkz64 = ok ? gacc[2 * n + gk] : 0.0;
  const float mk = float(mk64);
  const float gkx = float(gkx64);
  const float gky = float(gky64);
  const float gkz = float(gkz64);
  Box wave, block;
  target_boxes<L>(bx, nt, task.ib, wave, block);
  double c[3];
  const double thr2 = far_frame(block, c);
  const float xr = float(xk - c[0]);
  const float yr = float(yk - c[1]);
  const float zr = float(zk - c[2]);
  const float eps2 = float(eps2d);
  double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    const bool valid = j < jend;
    const double xj = valid ? pos[j] : 0.0;
    const double yj = valid ? pos[n + j] : 0.0;
    const double zj = valid ? pos[2 * n + j] : 0.0;
    const double mj64 = valid ? mass[j] : 0.0;
    const double gjx64 = valid ? gacc[j] : 0.0;
    const double gjy64 = valid ? gacc[n + j] : 0.0;
    const double gjz64 = valid ? gacc[2 * n + j] : 0.0;
    const float mj = float(mj64);
    const float gjx = float(gjx64);
    const float gjy = float(gjy64);
    const float gjz = float(gjz64);
    NearSrc bn{};
    bn.x = xj;
    bn.y = yj;
    bn.z = zj;
    if constexpr (NEAR64) {
      bn.m = mj64;
      bn.gx = gjx64;
      bn.gy = gjy64;
      bn.gz = gjz64;
    }
    VSrc<NBODY_MIXED> bf{};
    if (valid) {
      bf.x = float(xj - c[0]);
      bf.y = float(yj - c[1]);
      bf.z = float(zj - c[2]);
    }
    bf.m = mj;
    bf.gx = gjx;
    bf.gy = gjy;
    bf.gz = gjz;
    const uint64_t far_mask = far_runs<RUN>(wave, thr2, bx.run, jt, jend);
    // NBODY_MIXED_NF64 only (measured: -3 % time there; for NBODY_MIXED_NF
    // the second copy of the pair loop costs occupancy, 64 -> 67 VGPRs, and
    // gains nothing)
    const bool all_far = NEAR64 && far_mask == all_runs_mask<RUN>();
    if (NEAR64 && (tid & 63) == 0) wave_near[tid / 64] = !all_far;
    __syncthreads();  // previous tile fully consumed; the waves' flags visible
    if (!NEAR64 || any_wave_near(wave_near)) near_tile[tid] = bn;
    far_tile[tid] = bf;
    __syncthreads();

    if constexpr (NEAR64) if (all_far) {
      // every run of this tile is far for the wave: no per-chunk decisions
      for (int u0 = 0; u0 < PER; u0 += C) {
        VjpSplit acc;
        vjp_split_zero(acc);
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const VSrc<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
          vjp_pair_split(s.x - xr, s.y - yr, s.z - zr, s.m, s.gx, s.gy, s.gz,
                         mk, gkx, gky, gkz, eps2, false, acc);
        }
        vjp_split_flush(acc, mk, gkx, gky, gkz, sx, sy, sz, sm);
      }
      continue;
    }
    // Tiles that hold some of this workgroup's own targets: the FP32 near
    // runs drop their self pairs (vjp_pair_split); far runs never hold one.
    const int kblk = row0 + task.ib * G;
    const bool diag = jt < kblk + G && jt + kThreads > kblk;
    auto tile_pass = [&](auto diag_tag) {
      constexpr bool D = decltype(diag_tag)::value;
      for (int u0 = 0; u0 < PER; u0 += C) {
        const bool far = (far_mask >> (u0 / C)) & 1u;
        if constexpr (NEAR64) {
          if (!far) {
#pragma unroll 2
            for (int u = 0; u < C; ++u) {
              const NearSrc s = near_tile[(u0 + u) * L + q];
              vjp_pair<double>(s.x - xk, s.y - yk, s.z - zk, double(s.m),
                               double(s.gx), double(s.gy), double(s.gz), mk64,
                               gkx64, gky64, gkz64, eps2d, sx, sy, sz, sm);
            }
            continue;
          }
        }
        VjpSplit acc;
        vjp_split_zero(acc);
        if (far) {
#pragma unroll
          for (int u = 0; u < C; ++u) {
            const VSrc<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
            vjp_pair_split(s.x - xr, s.y - yr, s.z - zr, s.m, s.gx, s.gy,
                           s.gz, mk, gkx, gky, gkz, eps2, false, acc);
          }
        } else if constexpr (!NEAR64) {
#pragma unroll
          for (int u = 0; u < C; ++u) {
            const NearSrc s = near_tile[(u0 + u) * L + q];
            const VSrc<NBODY_MIXED> f = far_tile[(u0 + u) * L + q];
            const int j = jt + (u0 + u) * L + q;
            vjp_pair_split(float(s.x - xk), float(s.y - yk), float(s.z - zk),
                           f.m, f.gx, f.gy, f.gz, mk, gkx, gky, gkz, eps2,
                           D && j == gk, acc);
          }
        }
        vjp_split_flush(acc, mk, gkx, gky, gkz, sx, sy, sz, sm);
      }
    };
    if (!NEAR64 && diag)
      tile_pass(std::true_type{});
    else
      tile_pass(std::false_type{});
  }

  double *ox = out_x + size_t(task.s) * split_stride;
  double *om = out_m + size_t(task.s) * split_stride;
  double tx = group_sum<L>(sx);
  double ty = group_sum<L>(sy);
  double tz = group_sum<L>(sz);
  const double tm = group_sum<L>(sm);
  if (q == 0 && ok) {
    // this split holds the self pair (e = 0), always in a near run (its run
    // box contains x_k, gap 0): FP64 there for NBODY_MIXED_NF64, dropped by
    // the FP32 near runs otherwise
    if (NEAR64 && gk >= jbeg && gk < jend) {
      tx -= self_pair_term<double>(mk64, gkx64, eps2d);
      ty -= self_pair_term<double>(mk64, gky64, eps2d);
      tz -= self_pair_term<double>(mk64, gkz64, eps2d);
    }
    ox[k] = scale * tx;
    ox[nt + k] = scale * ty;
    ox[2 * nt + k] = scale * tz;
    om[k] = -scale * tm;
  }
}


// ------------------------------------------------------ Morton (Z) order --
//
// Key of body i: its position quantised on a 1024^3 grid spanning the cube
// [lo, lo + ext]^3 (lo the componentwise minimum, ext the largest extent),
// q = min(1023, floor((x - lo) * (1024 / ext))) per axis (all FP64, no
// contraction), bits interleaved x, y, z from the most significant down
// (bit 3b+2 = bit b of qx, 3b+1 of qy, 3b of qz), then shifted above a 33-bit
// body index: key = (morton << 33) | i.  Keys are unique, so ascending order
// is the stable sort by Morton code.  Padding keys are all ones.

constexpr int kMortonBits = 10;
constexpr int kIndexBits = 33;
constexpr int kSortChunk = 2048;  // keys per workgroup in the LDS stages

// Reduce group boxes to the global box: gbox[0..2] = lo, gbox[3..5] = hi.
__global__ __launch_bounds__(kThreads) void box_merge_kernel(
    int ngroups, const double *__restrict__ boxes, double *__restrict__ gbox) {
  __shared__ double red[4 * 6];
  const double inf = __builtin_huge_val();
  double v[6] = {inf, inf, inf, inf, inf, inf};
  for (int t = threadIdx.x; t < ngroups; t += kThreads) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], boxes[size_t(t) * 6 + c]);
      v[3 + c] = fmin(v[3 + c], -boxes[size_t(t) * 6 + 3 + c]);
    }
  }
  group_min6(v, 64);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) red[w * 6 + c] = v[c];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 6) {
    double m = red[t];
    for (int k = 1; k < kThreads / 64; ++k) m = fmin(m, red[k * 6 + t]);
    gbox[t] = t < 3 ? m : -m;
  }
}

__device__ __forceinline__ uint64_t quantise(double x, double lo, double sc) {
#pragma clang fp contract(off)
  const double v = floor((x - lo) * sc);
  if (!(v > 0.0)) return 0;  // also NaN
  return v >= 1023.0 ? 1023u : uint64_t(v);
}

__global__ __launch_bounds__(kThreads) void morton_key_kernel(
    int n, int64_t npad, const double *__restrict__ pos,
    const double *__restrict__ gbox, uint64_t *__restrict__ keys) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= npad) return;
  if (i >= n) {
    keys[i] = ~uint64_t(0);
    return;
  }
  const double ext = fmax(gbox[3] - gbox[0], fmax(gbox[4] - gbox[1], gbox[5] - gbox[2]));
  const double sc = ext > 0.0 ? 1024.0 / ext : 0.0;
  const uint64_t qx = quantise(pos[i], gbox[0], sc);
  const uint64_t qy = quantise(pos[n + i], gbox[1], sc);
  const uint64_t qz = quantise(pos[2 * n + i], gbox[2], sc);
  uint64_t m = 0;
#pragma unroll
  for (int b = 0; b < kMortonBits; ++b) {
    m |= ((qx >> b) & 1u) << (3 * b + 2);
    m |= ((qy >> b) & 1u) << (3 * b + 1);
    m |= ((qz >> b) & 1u) << (3 * b);
  }
  keys[i] = (m << kIndexBits) | uint64_t(i);
}

// Bitonic network on npad (a power of two) keys.  Pair (i, i + j) with
// i & j == 0 is ordered ascending when i & k == 0, descending otherwise.
__device__ __forceinline__ void cmp_swap(uint64_t &a, uint64_t &b, bool asc) {
  if ((a > b) == asc) {
    const uint64_t t = a;
    a = b;
    b = t;
  }
}

// Stages k = 2 .. chunk (each chunk of `chunk` keys fully sorted, direction
// by the global index) when kmin == 2; otherwise the j < chunk steps of stage
// k = kmin.
__global__ __launch_bounds__(kThreads) void bitonic_lds_kernel(
    uint64_t *__restrict__ keys, int chunk, int64_t kmin) {
  __shared__ uint64_t s[kSortChunk];
  const int64_t base = int64_t(blockIdx.x) * chunk;
  for (int e = threadIdx.x; e < chunk; e += kThreads) s[e] = keys[base + e];
  __syncthreads();
  const int64_t kfirst = kmin, klast = kmin == 2 ? chunk : kmin;
  for (int64_t k = kfirst; k <= klast; k <<= 1) {
    for (int j = int((k < chunk ? k : int64_t(chunk)) >> 1); j > 0; j >>= 1) {
      for (int p = threadIdx.x; p < chunk / 2; p += kThreads) {
        const int i = 2 * j * (p / j) + (p % j);
        const bool asc = ((base + i) & k) == 0;
        uint64_t a = s[i], b = s[i + j];
        cmp_swap(a, b, asc);
        s[i] = a;
        s[i + j] = b;
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < chunk; e += kThreads) keys[base + e] = s[e];
}

// One global step (stride j >= chunk) of stage k.
__global__ __launch_bounds__(kThreads) void bitonic_step_kernel(
    uint64_t *__restrict__ keys, int64_t npad, int64_t j, int64_t k) {
  const int64_t p = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (p >= npad / 2) return;
  const int64_t i = 2 * j * (p / j) + (p % j);
  uint64_t a = keys[i], b = keys[i + j];
  cmp_swap(a, b, (i & k) == 0);
  keys[i] = a;
  keys[i + j] = b;
}

// perm[r] = index of the body at sorted position r; gather the state.
__global__ __launch_bounds__(kBodyThreadsSort) void morton_gather_kernel(
    int n, const uint64_t *__restrict__ keys, const double *__restrict__ pos,
    const double *__restrict__ vel, const double *__restrict__ mass,
    int64_t *__restrict__ perm, double *__restrict__ pos_out,
    double *__restrict__ vel_out, double *__restrict__ mass_out) {
  const int r = blockIdx.x * kBodyThreadsSort + threadIdx.x;
  if (r >= n) return;
  int64_t src = int64_t(keys[r] & ((uint64_t(1) << kIndexBits) - 1));
  if (src >= n) src = n - 1;  // unreachable for a correct sort; keeps reads in bounds
  perm[r] = src;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pos_out[size_t(c) * n + r] = pos[size_t(c) * n + src];
    if (vel) vel_out[size_t(c) * n + r] = vel[size_t(c) * n + src];
  }
  mass_out[r] = mass[src];
}

// Launches with fewer pairs keep the grid order: the two ordering launches
// cost a few microseconds, which only pays back on a launch of a millisecond
// or more (measured on MI355X, clustered system in Morton order: -4 % forward
// and -2.5 % VJP time at N = 262144).
constexpr int64_t kNfOrderMinPairs = int64_t(1) << 32;

bool nf_ordered(const Plan &pl, int64_t n, int64_t nt) {
  return nt * n >= kNfOrderMinPairs && pl.sj <= kOrderMaxSplits;
}

// Layout (in doubles) of the near / far scratch of one all-pairs launch: run
// boxes over the n sources, wave and workgroup boxes over the nt targets,
// then (ordered launches) the tasks' load classes (n_ib * sj bytes) and the
// dispatch order (n_ib * sj ints).
struct NfLayout {
  int run, gw, gb;
  bool ordered;
  int ntask;
  size_t off_wave, off_block, off_load, off_order, total;
};

NfLayout nf_layout(const Plan &pl, KernelKind kind, bool near64, int64_t n,
                   int64_t nt) {
  NfLayout l;
  l.run = nf_run(kind, pl.L, near64);
  l.gw = 64 / pl.L;
  l.gb = kThreads / pl.L;
  l.ordered = nf_ordered(pl, n, nt);
  l.ntask = int(pl.n_ib * pl.sj);
  const size_t nr = size_t((n + l.run - 1) / l.run);
  const size_t nw = size_t((nt + l.gw - 1) / l.gw);
  const size_t nb = size_t((nt + l.gb - 1) / l.gb);
  // in doubles
  const size_t bytes = l.ordered ? size_t(l.ntask + 7) / 8 : 0;
  const size_t ints = l.ordered ? size_t(l.ntask + 1) / 2 : 0;
  l.off_wave = nr * 6;
  l.off_block = l.off_wave + nw * 6;
  l.off_load = l.off_block + nb * 6;
  l.off_order = l.off_load + bytes;
  l.total = l.off_order + ints;
  return l;
}

// Fill the box area for a launch over targets row0 .. row0 + nt - 1 (one
// pass when the targets are all n bodies, otherwise one over the sources and
// one over the target rows), then, for an ordered launch, the task loads and
// the dispatch order; order is left NULL (grid order) otherwise.
hipError_t launch_nf_boxes(const Plan &pl, KernelKind kind, bool near64, int n,
                           int row0, int nt, const double *pos, double *area,
                           NfBoxes &bx, const int *&order, hipStream_t st) {
  const NfLayout l = nf_layout(pl, kind, near64, n, nt);
  double *rb = area, *wb = area + l.off_wave, *bb = area + l.off_block;
  bx.run = rb;
  bx.wave = wb;
  bx.block = bb;
  order = nullptr;
  const unsigned sblocks = unsigned((n + kThreads - 1) / kThreads);
  if (row0 == 0 && nt == n) {
    group_box_kernel<<<sblocks, kThreads, 0, st>>>(n, 0, n, pos, l.run, rb, l.gw,
                                                   wb, l.gb, bb);
  } else {
    group_box_kernel<<<sblocks, kThreads, 0, st>>>(n, 0, n, pos, l.run, rb, 0,
                                                   nullptr, 0, nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned tblocks = unsigned((nt + kThreads - 1) / kThreads);
    group_box_kernel<<<tblocks, kThreads, 0, st>>>(n, row0, nt, pos, l.gw, wb,
                                                   l.gb, bb, 0, nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !l.ordered) return e;
  auto *cls = reinterpret_cast<unsigned char *>(area + l.off_load);
  int *ord = reinterpret_cast<int *>(area + l.off_order);
  nf_load_kernel<<<unsigned(pl.n_ib), kThreads, 0, st>>>(n, nt, bx, l.run, l.gw,
                                                         pl.split, int(pl.sj), cls);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  nf_order_kernel<<<1, kThreads, 0, st>>>(l.ntask, cls, ord);
  e = hipGetLastError();
  if (e == hipSuccess) order = ord;
  return e;
}

}  // namespace

hipError_t launch_accel_nf(const Plan &pl, int n, int row0, int nt,
                           const double *pos, const double *mass,
                           double *boxes, double eps2, double scale,
                           double *out, size_t stride, bool near64,
                           hipStream_t st) {
  if (pl.R != 1) return hipErrorInvalidValue;
  NfBoxes bx;
  const int *order;
  const hipError_t e = launch_nf_boxes(pl, kAccel, near64, n, row0, nt, pos,
                                       boxes, bx, order, st);
  if (e != hipSuccess) return e;
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const SplitShape jc = pl.split;
#define NBODY_ACCEL_NF(L_, N64_)                                                 \
  accel_nf_kernel<L_, N64_><<<grid, kThreads, 0, st>>>(n, row0, nt, pos, mass,   \
                                                       bx, order, eps2, scale,   \
                                                       jc, out, stride)
  if (pl.L == 1) { if (near64) NBODY_ACCEL_NF(1, true); else NBODY_ACCEL_NF(1, false); }
  else if (pl.L == 4) { if (near64) NBODY_ACCEL_NF(4, true); else NBODY_ACCEL_NF(4, false); }
  else if (pl.L == 16) { if (near64) NBODY_ACCEL_NF(16, true); else NBODY_ACCEL_NF(16, false); }
  else return hipErrorInvalidValue;
#undef NBODY_ACCEL_NF
  return hipGetLastError();
}

hipError_t launch_vjp_nf(const Plan &pl, int n, int row0, int nt,
                         const double *pos, const double *mass,
                         const double *gacc, double *boxes, double eps2,
                         double scale, double *ox, double *om, size_t stride,
                         bool near64, hipStream_t st) {
  if (pl.R != 1) return hipErrorInvalidValue;
  NfBoxes bx;
  const int *order;
  const hipError_t e = launch_nf_boxes(pl, kVjp, near64, n, row0, nt, pos,
                                       boxes, bx, order, st);
  if (e != hipSuccess) return e;
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const SplitShape jc = pl.split;
#define NBODY_VJP_NF(L_, N64_)                                                   \
  vjp_nf_kernel<L_, N64_><<<grid, kThreads, 0, st>>>(n, row0, nt, pos, mass,     \
                                                     gacc, bx, order, eps2,      \
                                                     scale, jc, ox, om, stride)
  if (pl.L == 1) { if (near64) NBODY_VJP_NF(1, true); else NBODY_VJP_NF(1, false); }
  else if (pl.L == 4) { if (near64) NBODY_VJP_NF(4, true); else NBODY_VJP_NF(4, false); }
  else if (pl.L == 16) { if (near64) NBODY_VJP_NF(16, true); else NBODY_VJP_NF(16, false); }
  else return hipErrorInvalidValue;
#undef NBODY_VJP_NF
  return hipGetLastError();
}

size_t near_far_box_doubles(const Plan &pl, KernelKind kind, bool near64,
                            int64_t n, int64_t nt) {
  return nf_layout(pl, kind, near64, n, nt).total;
}

int64_t morton_padded(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

hipError_t launch_morton_sort(int n, const double *pos, const double *vel,
                              const double *mass, int64_t *perm,
                              double *pos_out, double *vel_out,
                              double *mass_out, double *boxes, double *gbox,
                              uint64_t *keys, hipStream_t st) {
  const int ntiles = (n + kThreads - 1) / kThreads;
  const int64_t npad = morton_padded(n);
  group_box_kernel<<<unsigned(ntiles), kThreads, 0, st>>>(
      n, 0, n, pos, kThreads, boxes, 0, nullptr, 0, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  box_merge_kernel<<<1, kThreads, 0, st>>>(ntiles, boxes, gbox);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  morton_key_kernel<<<unsigned((npad + kThreads - 1) / kThreads), kThreads, 0,
                      st>>>(n, npad, pos, gbox, keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (npad > 1) {
    const int chunk = int(npad < kSortChunk ? npad : kSortChunk);
    const unsigned nchunks = unsigned(npad / chunk);
    bitonic_lds_kernel<<<nchunks, kThreads, 0, st>>>(keys, chunk, 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned step_blocks = unsigned((npad / 2 + kThreads - 1) / kThreads);
    for (int64_t k = int64_t(chunk) * 2; k <= npad; k <<= 1) {
      for (int64_t j = k >> 1; j >= chunk; j >>= 1) {
        bitonic_step_kernel<<<step_blocks, kThreads, 0, st>>>(keys, npad, j, k);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      bitonic_lds_kernel<<<nchunks, kThreads, 0, st>>>(keys, chunk, k);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  morton_gather_kernel<<<unsigned((n + kBodyThreadsSort - 1) / kBodyThreadsSort),
                         kBodyThreadsSort, 0, st>>>(n, keys, pos, vel, mass, perm,
                                                    pos_out, vel_out, mass_out);
  return hipGetLastError();
}

}  // namespace nbody
