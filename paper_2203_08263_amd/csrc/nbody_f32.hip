// gfx950 kernels of the FP32-state variant (the paper's single-precision
// runs): FP32 arrays and FP32 arithmetic, including every sum.
#include "nbody_device.h"

namespace nbody {
namespace {

// --------------------------------------------------------- FP32 state --
//
// The paper's single-precision variant (its float32 runs): positions,
// velocities, masses and accelerations stored in FP32 and every operation in
// FP32, including the sum over sources -- each lane's share of a split, the
// L lane sums and the splits, in that fixed order.  No FP64 anywhere.

template <int L>
__device__ __forceinline__ float group_sum_f(float v) {
#pragma unroll
  for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

template <int L>
__global__ __launch_bounds__(kThreads) void accel_f32_kernel(
    int n, const float *__restrict__ pos, const float *__restrict__ mass,
    float eps2, float scale, SplitShape split, float *__restrict__ out,
    size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  __shared__ Src<NBODY_MIXED> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int i = blockIdx.x * G + g;
  int jbeg, jend;
  split_range(split, blockIdx.y, n, jbeg, jend);
  const bool ok = i < n;
  const float xi = ok ? pos[i] : 0.0f;
  const float yi = ok ? pos[n + i] : 0.0f;
  const float zi = ok ? pos[2 * n + i] : 0.0f;
  float ax = 0.0f, ay = 0.0f, az = 0.0f;

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    Src<NBODY_MIXED> b{};
    if (j < jend) {
      b.x = pos[j];
      b.y = pos[n + j];
      b.z = pos[2 * n + j];
      b.m = mass[j];
    }
    __syncthreads();
    tile[tid] = b;
    __syncthreads();
    constexpr int U = PER < 16 ? PER : 16;  // sources per unrolled step
    for (int u0 = 0; u0 < PER; u0 += U)
      chunk_sum_f32<U, kPairBatch>(
          [&](int u, float &dx, float &dy, float &dz, float &m) {
            const Src<NBODY_MIXED> s = tile[(u0 + u) * L + q];
            dx = s.x - xi;
            dy = s.y - yi;
            dz = s.z - zi;
            m = s.m;
          },
          eps2, ax, ay, az);
  }
  float *o = out + size_t(blockIdx.y) * split_stride;
  const float sx = group_sum_f<L>(ax);
  const float sy = group_sum_f<L>(ay);
  const float sz = group_sum_f<L>(az);
  if (q == 0 && ok) {
    o[i] = scale * sx;
    o[n + i] = scale * sy;
    o[2 * n + i] = scale * sz;
  }
}

__device__ __forceinline__ float split_sum_f(const float *__restrict__ part,
                                             size_t stride, int sj, size_t off) {
  float s = part[off];
  for (int p = 1; p < sj; ++p) s += part[size_t(p) * stride + off];
  return s;
}

__global__ __launch_bounds__(kBodyThreads) void reduce_f32_kernel(
    int n, int sj, const float *__restrict__ part, size_t stride, float G,
    float *__restrict__ out) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(3) * n) return;
  out[q] = G * split_sum_f(part, stride, sj, q);
}

// The FP32 counterpart of update_kernel (no checkpoint record).
__global__ __launch_bounds__(kBodyThreads) void update_f32_kernel(
    int n, int sj, const float *__restrict__ part, size_t stride, float G,
    const float *a_in, float *acc_out, float *x_io, float *v_io, float h,
    float dt, unsigned flags) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(3) * n) return;
  const float a = part ? G * split_sum_f(part, stride, sj, q) : a_in[q];
  float v = v_io[q];
  if (flags & kClose) v = v + h * a;
  if (flags & kOpen) {
    v = v + h * a;
    x_io[q] = x_io[q] + dt * v;
  }
  v_io[q] = v;
  if (acc_out) acc_out[q] = a;
}

}  // namespace

hipError_t launch_accel_f32(const Plan &pl, int n, const float *pos,
                            const float *mass, float eps2, float scale,
                            float *out, size_t stride, hipStream_t st) {
  if (pl.R != 1) return hipErrorInvalidValue;
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const SplitShape jc = pl.split;
  if (pl.L == 1)
    accel_f32_kernel<1><<<grid, kThreads, 0, st>>>(n, pos, mass, eps2, scale, jc,
                                                   out, stride);
  else if (pl.L == 4)
    accel_f32_kernel<4><<<grid, kThreads, 0, st>>>(n, pos, mass, eps2, scale, jc,
                                                   out, stride);
  else if (pl.L == 16)
    accel_f32_kernel<16><<<grid, kThreads, 0, st>>>(n, pos, mass, eps2, scale,
                                                    jc, out, stride);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_reduce_f32(int n, int sj, const float *part, size_t stride,
                             float G, float *out, hipStream_t st) {
  reduce_f32_kernel<<<grid_body(n, 3), kBodyThreads, 0, st>>>(n, sj, part,
                                                             stride, G, out);
  return hipGetLastError();
}

hipError_t launch_update_f32(int n, int sj, const float *part, size_t stride,
                             float G, const float *a_in, float *acc_out,
                             float *x, float *v, float h, float dt,
                             unsigned flags, hipStream_t st) {
  update_f32_kernel<<<grid_body(n, 3), kBodyThreads, 0, st>>>(
      n, sj, part, stride, G, a_in, acc_out, x, v, h, dt, flags);
  return hipGetLastError();
}

}  // namespace nbody
