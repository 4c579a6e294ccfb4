// gfx950 kernels of the all-pairs gravitational N-body hot path.
//
// The all-pairs kernels (acceleration and its VJP) share one shape:
//  - a workgroup of 256 threads (4 wave64s) owns kThreads*R target bodies,
//    R per thread, strided by kThreads so every load and store is coalesced;
//  - blockIdx.y selects a contiguous source range of jchunk bodies, staged
//    through LDS in tiles of 256 bodies, one body loaded per thread from the
//    structure-of-arrays FP64 state.  In the mixed modes the staging step is
//    where positions and masses are rounded to FP32 (the "pack" of the source
//    stream happens on the way into LDS, so no packed copy is ever written to
//    HBM);
//  - every thread walks the whole tile in ascending order reading each source
//    body as a wave-uniform LDS broadcast, so one LDS read feeds 64*R pairs;
//  - the tail of the last tile is padded with zero-mass bodies at the origin,
//    whose contribution w*d with w = 0 is exactly zero;
//  - each source split writes its own FP64 partial sum; the partials are
//    added in ascending split order by the reduce / update kernels.  No
//    atomics anywhere, so results are bitwise reproducible.
//
// The mixed modes sum FP32 pair terms over chunks of kChunk sources and add
// each chunk into FP64 per-body accumulators.  The pair arithmetic is the
// direct-summation force of arxiv 2203.08263 section 2.3 (force loop of the
// section 3.2 / 3.3 listings) with the acceleration taken directly as
// G sum_j m_j d s^-3/2 and the reciprocal square root from the hardware
// approximation (v_rsq_f32 / v_rsq_f64), refined by Newton's method in FP64.
#include <algorithm>

#include "nbody_internal.h"
#include "../../include/nbody.h"

namespace nbody {
namespace {

constexpr int kChunk = 32;     // FP32 sources per FP64 flush (forward)
constexpr int kBodyThreadsSort = 256;
constexpr int kVjpChunk = 16;  // FP32 sources per FP64 flush (VJP)

// -------------------------------------------------------------- arithmetic --

// 1/sqrt(s) in FP64: hardware estimate (about 23 correct bits) refined by two
// Newton steps y <- y (3 - s y^2) / 2, written as y + y (1/2 - (s/2) y y).
__device__ __forceinline__ double rsqrt_f64(double s) {
  double y = __builtin_amdgcn_rsq(s);
  const double hs = 0.5 * s;
  double e = fma(-(hs * y), y, 0.5);
  y = fma(y, e, y);
  e = fma(-(hs * y), y, 0.5);
  y = fma(y, e, y);
  return y;
}

__device__ __forceinline__ float rsqrt_f32(float s) {
  return __builtin_amdgcn_rsqf(s);
}

// One source j acting on one target: a += m_j d (|d|^2 + eps^2)^-3/2.
__device__ __forceinline__ void pair_f64(double dx, double dy, double dz,
                                         double m, double eps2, double &ax,
                                         double &ay, double &az) {
  double s = fma(dx, dx, eps2);
  s = fma(dy, dy, s);
  s = fma(dz, dz, s);
  const double y = rsqrt_f64(s);
  const double w = (m * y) * (y * y);
  ax = fma(w, dx, ax);
  ay = fma(w, dy, ay);
  az = fma(w, dz, az);
}

__device__ __forceinline__ void pair_f32(float dx, float dy, float dz, float m,
                                         float eps2, float &ax, float &ay,
                                         float &az) {
  float s = fmaf(dx, dx, eps2);
  s = fmaf(dy, dy, s);
  s = fmaf(dz, dz, s);
  const float y = rsqrt_f32(s);
  const float w = (m * y) * (y * y);
  ax = fmaf(w, dx, ax);
  ay = fmaf(w, dy, ay);
  az = fmaf(w, dz, az);
}

// One source j against target k for the VJP (row formulation):
//   g += s^-3/2 (h + t e),  t = -3 (e.h) / s,   dm += (gbar_j . e) s^-3/2
// with e = x_j - x_k and h = m_k gbar_j - m_j gbar_k, formed as
// fma(m_k, gbar_j, -(m_j gbar_k)).  For the self pair j == k that h is not
// zero but the exact rounding error delta of m_k gbar_k, and since e = 0 the
// pair adds exactly fma(y3_self, delta, g): see self_pair_term, which the
// kernel subtracts afterwards so the self pair contributes nothing.
template <typename T>
__device__ __forceinline__ void vjp_pair(T ex, T ey, T ez, T mj, T gjx, T gjy,
                                         T gjz, T mk, T gkx, T gky, T gkz,
                                         T eps2, T &gx, T &gy, T &gz, T &dm) {
  T s = fma(ex, ex, eps2);
  s = fma(ey, ey, s);
  s = fma(ez, ez, s);
  T y;
  if constexpr (sizeof(T) == 8) y = rsqrt_f64(s); else y = rsqrt_f32(s);
  const T y2 = y * y;
  const T y3 = y2 * y;
  const T hx = fma(mk, gjx, -(mj * gkx));
  const T hy = fma(mk, gjy, -(mj * gky));
  const T hz = fma(mk, gjz, -(mj * gkz));
  const T eh = fma(ez, hz, fma(ey, hy, ex * hx));
  const T ge = fma(gjz, ez, fma(gjy, ey, gjx * ex));
  dm = fma(ge, y3, dm);
  const T t = (y2 * T(-3)) * eh;
  gx = fma(y3, fma(t, ex, hx), gx);
  gy = fma(y3, fma(t, ey, hy), gy);
  gz = fma(y3, fma(t, ez, hz), gz);
}

// What vjp_pair adds to g for the self pair j == k (e = 0, s = eps^2): the
// same y3 and h operations, evaluated once per target.  The product is
// rounded like the pair's own fma(y3, delta, 0) (exact for FP32 operands);
// contraction is off so the caller's subtraction cannot absorb it into an
// FMA, which would leave the product's rounding error behind.
template <typename T>
__device__ __forceinline__ double self_pair_term(T mk, T gk, T eps2) {
#pragma clang fp contract(off)
  T y;
  if constexpr (sizeof(T) == 8) y = rsqrt_f64(eps2); else y = rsqrt_f32(eps2);
  const T y3 = (y * y) * y;
  const T delta = fma(mk, gk, -(mk * gk));
  return double(y3) * double(delta);
}

// ------------------------------------------------------ source tile layout --

template <int PREC> struct Src;
template <> struct Src<NBODY_FP64> { double x, y, z, m; };
template <> struct Src<NBODY_MIXED> { float x, y, z, m; };
template <> struct Src<NBODY_MIXED_D64> { double x, y, z; float m, pad; };

template <int PREC>
__device__ __forceinline__ Src<PREC> load_src(const double *__restrict__ pos,
                                              const double *__restrict__ mass,
                                              int n, int j, bool valid) {
  Src<PREC> b{};
  if (valid) {
    b.x = pos[j];
    b.y = pos[n + j];
    b.z = pos[2 * n + j];
    b.m = mass[j];   // rounds to FP32 in the mixed modes
  }
  return b;
}

template <int PREC> struct VSrc;
template <> struct VSrc<NBODY_FP64> { double x, y, z, m, gx, gy, gz, pad; };
template <> struct VSrc<NBODY_MIXED> { float x, y, z, m, gx, gy, gz, pad; };
template <> struct VSrc<NBODY_MIXED_D64> {
  double x, y, z;
  float m, gx, gy, gz, pad0, pad1;
};

// Coordinate type of a target body and of its pair difference.
template <int PREC> struct Coord { using T = double; using D = double; };
template <> struct Coord<NBODY_MIXED> { using T = float; using D = float; };
template <> struct Coord<NBODY_MIXED_D64> { using T = double; using D = float; };

// Sum over the L consecutive lanes that share a target (L a power of two
// dividing the wave size) by an xor butterfly: every stage adds the same two
// values in both partner lanes, so all L lanes end with the bitwise same
// total, in an order fixed by L alone.
template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// ------------------------------------------------------------ acceleration --
//
// Thread t of a workgroup serves target group g = t / L with lane q = t % L;
// the group owns R targets i = blockIdx.x * (256/L) * R + g + r * (256/L),
// and lane q visits the tile entries q, q + L, q + 2L, ...  With L > 1 a
// small system still yields enough waves without splitting the source range
// into many FP64 partials.
//
// Targets are the nt bodies row0 .. row0 + nt - 1 of the n-body system (all
// of it when row0 = 0, nt = n), sources are all n bodies; output row i (of
// stride nt) belongs to body row0 + i.

template <int PREC, int R, int L>
__global__ __launch_bounds__(kThreads) void accel_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, double eps2d, double scale, int jchunk,
    double *__restrict__ out, size_t split_stride) {
  using CT = typename Coord<PREC>::T;
  using DT = typename Coord<PREC>::D;
  constexpr int G = kThreads / L;             // target groups per workgroup
  constexpr int PER = kThreads / L;           // tile entries per lane
  constexpr int C = PER < kChunk ? PER : kChunk;
  __shared__ Src<PREC> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int ibase = blockIdx.x * (G * R) + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);

  CT xi[R], yi[R], zi[R];
  double ax[R], ay[R], az[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * G;
    const bool ok = i < nt;
    const int gi = row0 + i;
    xi[r] = ok ? CT(pos[gi]) : CT(0);
    yi[r] = ok ? CT(pos[n + gi]) : CT(0);
    zi[r] = ok ? CT(pos[2 * n + gi]) : CT(0);
    ax[r] = ay[r] = az[r] = 0.0;
  }

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    const Src<PREC> b = load_src<PREC>(pos, mass, n, j, j < jend);
    __syncthreads();  // previous tile fully consumed
    tile[tid] = b;
    __syncthreads();

    if constexpr (PREC == NBODY_FP64) {
#pragma unroll 4
      for (int u = 0; u < PER; ++u) {
        const Src<PREC> s = tile[u * L + q];
#pragma unroll
        for (int r = 0; r < R; ++r)
          pair_f64(s.x - xi[r], s.y - yi[r], s.z - zi[r], s.m, eps2d, ax[r],
                   ay[r], az[r]);
      }
    } else {
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
        float fx[R], fy[R], fz[R];
#pragma unroll
        for (int r = 0; r < R; ++r) fx[r] = fy[r] = fz[r] = 0.0f;
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const Src<PREC> s = tile[(u0 + u) * L + q];
#pragma unroll
          for (int r = 0; r < R; ++r)
            pair_f32(DT(s.x - xi[r]), DT(s.y - yi[r]), DT(s.z - zi[r]), s.m,
                     eps2, fx[r], fy[r], fz[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ax[r] += double(fx[r]);
          ay[r] += double(fy[r]);
          az[r] += double(fz[r]);
        }
      }
    }
  }

  double *o = out + size_t(blockIdx.y) * split_stride;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double sx = group_sum<L>(ax[r]);
    const double sy = group_sum<L>(ay[r]);
    const double sz = group_sum<L>(az[r]);
    const int i = ibase + r * G;
    if (q == 0 && i < nt) {
      o[i] = scale * sx;
      o[nt + i] = scale * sy;
      o[2 * nt + i] = scale * sz;
    }
  }
}

// ---------------------------------------------------------------------- VJP --

// Rows as in accel_kernel: targets k = row0 .. row0 + nt - 1, sources all n
// bodies (with their dL/da), output row k - row0 of stride nt.
template <int PREC, int R, int L>
__global__ __launch_bounds__(kThreads) void vjp_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, const double *__restrict__ gacc,
    double eps2d, double scale, int jchunk, double *__restrict__ out_x,
    double *__restrict__ out_m, size_t split_stride) {
  using CT = typename Coord<PREC>::T;
  using DT = typename Coord<PREC>::D;
  using AT = typename Coord<PREC>::D;  // arithmetic type of the pair terms
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = PER < kVjpChunk ? PER : kVjpChunk;
  __shared__ VSrc<PREC> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int kbase = blockIdx.x * (G * R) + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);

  CT xk[R], yk[R], zk[R];
  AT mk[R], gkx[R], gky[R], gkz[R];
  double sx[R], sy[R], sz[R], sm[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = kbase + r * G;
    const bool ok = k < nt;
    const int gk = row0 + k;
    xk[r] = ok ? CT(pos[gk]) : CT(0);
    yk[r] = ok ? CT(pos[n + gk]) : CT(0);
    zk[r] = ok ? CT(pos[2 * n + gk]) : CT(0);
    mk[r] = ok ? AT(mass[gk]) : AT(0);
    gkx[r] = ok ? AT(gacc[gk]) : AT(0);
    gky[r] = ok ? AT(gacc[n + gk]) : AT(0);
    gkz[r] = ok ? AT(gacc[2 * n + gk]) : AT(0);
    sx[r] = sy[r] = sz[r] = sm[r] = 0.0;
  }

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    VSrc<PREC> b{};
    if (j < jend) {
      b.x = pos[j];
      b.y = pos[n + j];
      b.z = pos[2 * n + j];
      b.m = mass[j];
      b.gx = gacc[j];
      b.gy = gacc[n + j];
      b.gz = gacc[2 * n + j];
    }
    __syncthreads();
    tile[tid] = b;
    __syncthreads();

    if constexpr (PREC == NBODY_FP64) {
#pragma unroll 2
      for (int u = 0; u < PER; ++u) {
        const VSrc<PREC> s = tile[u * L + q];
#pragma unroll
        for (int r = 0; r < R; ++r)
          vjp_pair<double>(s.x - xk[r], s.y - yk[r], s.z - zk[r], s.m, s.gx,
                           s.gy, s.gz, mk[r], gkx[r], gky[r], gkz[r], eps2d,
                           sx[r], sy[r], sz[r], sm[r]);
      }
    } else {
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
        float fx[R], fy[R], fz[R], fm[R];
#pragma unroll
        for (int r = 0; r < R; ++r) fx[r] = fy[r] = fz[r] = fm[r] = 0.0f;
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const VSrc<PREC> s = tile[(u0 + u) * L + q];
#pragma unroll
          for (int r = 0; r < R; ++r)
            vjp_pair<float>(DT(s.x - xk[r]), DT(s.y - yk[r]), DT(s.z - zk[r]),
                            s.m, s.gx, s.gy, s.gz, mk[r], gkx[r], gky[r],
                            gkz[r], eps2, fx[r], fy[r], fz[r], fm[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sx[r] += double(fx[r]);
          sy[r] += double(fy[r]);
          sz[r] += double(fz[r]);
          sm[r] += double(fm[r]);
        }
      }
    }
  }

  double *ox = out_x + size_t(blockIdx.y) * split_stride;
  double *om = out_m + size_t(blockIdx.y) * split_stride;
  const AT eps2a = AT(eps2d);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double tx = group_sum<L>(sx[r]);
    double ty = group_sum<L>(sy[r]);
    double tz = group_sum<L>(sz[r]);
    const double tm = group_sum<L>(sm[r]);
    const int k = kbase + r * G;
    const int gk = row0 + k;
    if (q == 0 && k < nt) {
      if (gk >= jbeg && gk < jend) {  // this split holds the self pair
        tx -= self_pair_term<AT>(mk[r], gkx[r], eps2a);
        ty -= self_pair_term<AT>(mk[r], gky[r], eps2a);
        tz -= self_pair_term<AT>(mk[r], gkz[r], eps2a);
      }
      ox[k] = scale * tx;
      ox[nt + k] = scale * ty;
      ox[2 * nt + k] = scale * tz;
      om[k] = -scale * tm;
    }
  }
}

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

struct Box {
  double lo[3], hi[3];
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
__device__ __forceinline__ void target_boxes(const NfBoxes &bx, int nt,
                                             Box &wave, Box &block) {
  constexpr int GW = 64 / L;
  // wave index, uniform across the wave (scalar registers and branches)
  const int wg = __builtin_amdgcn_readfirstlane(
      int(blockIdx.x) * (kThreads / 64) + int(threadIdx.x) / 64);
  const bool has = wg * GW < nt;
  block = read_box(bx.block, blockIdx.x);
  wave = read_box(bx.wave, has ? wg : 0);  // box 0 always exists
  const double inf = __builtin_huge_val();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    wave.lo[c] = has ? wave.lo[c] : inf;
    wave.hi[c] = has ? wave.hi[c] : -inf;
  }
}

template <int L, bool NEAR64>
__global__ __launch_bounds__(kThreads) void accel_nf_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, NfBoxes bx, double eps2d, double scale,
    int jchunk, double *__restrict__ out, size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = PER < kChunk ? PER : kChunk;
  constexpr int RUN = C * L;  // sources of one chunk run (box granularity)
  using NearSrc = Src<NEAR64 ? NBODY_FP64 : NBODY_MIXED_D64>;
  __shared__ NearSrc near_tile[kThreads];
  __shared__ Src<NBODY_MIXED> far_tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int i = blockIdx.x * G + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
  const bool ok = i < nt;
  const int gi = row0 + i;
  const double xi = ok ? pos[gi] : 0.0;
  const double yi = ok ? pos[n + gi] : 0.0;
  const double zi = ok ? pos[2 * n + gi] : 0.0;
  Box wave, block;
  target_boxes<L>(bx, nt, wave, block);
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
    if constexpr (NEAR64) bn.m = mj64; else bn.m = mj;
    Src<NBODY_MIXED> bf{};
    if (valid) {
      bf.x = float(xj - c[0]);
      bf.y = float(yj - c[1]);
      bf.z = float(zj - c[2]);
      bf.m = mj;
    }
    const uint64_t far_mask = far_runs<RUN>(wave, thr2, bx.run, jt, jend);
    __syncthreads();  // previous tile fully consumed
    near_tile[tid] = bn;
    far_tile[tid] = bf;
    __syncthreads();

    for (int u0 = 0; u0 < PER; u0 += C) {
      const bool far = (far_mask >> (u0 / C)) & 1u;  // run u0 / C of the tile
      if (NEAR64 && !far) {
#pragma unroll 4
        for (int u = 0; u < C; ++u) {
          const NearSrc s = near_tile[(u0 + u) * L + q];
          pair_f64(s.x - xi, s.y - yi, s.z - zi, double(s.m), eps2d, ax, ay, az);
        }
        continue;
      }
      float fx = 0.0f, fy = 0.0f, fz = 0.0f;
      if (far) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const Src<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
          pair_f32(s.x - xr, s.y - yr, s.z - zr, s.m, eps2, fx, fy, fz);
        }
      } else if constexpr (!NEAR64) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const NearSrc s = near_tile[(u0 + u) * L + q];
          pair_f32(float(s.x - xi), float(s.y - yi), float(s.z - zi), float(s.m),
                   eps2, fx, fy, fz);
        }
      }
      ax += double(fx);
      ay += double(fy);
      az += double(fz);
    }
  }

  double *o = out + size_t(blockIdx.y) * split_stride;
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
    NfBoxes bx, double eps2d, double scale, int jchunk,
    double *__restrict__ out_x, double *__restrict__ out_m,
    size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = PER < kVjpChunk ? PER : kVjpChunk;
  constexpr int RUN = C * L;
  using NearSrc = VSrc<NEAR64 ? NBODY_FP64 : NBODY_MIXED_D64>;
  __shared__ NearSrc near_tile[kThreads];
  __shared__ VSrc<NBODY_MIXED> far_tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int k = blockIdx.x * G + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
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
  target_boxes<L>(bx, nt, wave, block);
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
    } else {
      bn.m = mj;
      bn.gx = gjx;
      bn.gy = gjy;
      bn.gz = gjz;
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
    __syncthreads();
    near_tile[tid] = bn;
    far_tile[tid] = bf;
    __syncthreads();

    for (int u0 = 0; u0 < PER; u0 += C) {
      const bool far = (far_mask >> (u0 / C)) & 1u;
      if (NEAR64 && !far) {
#pragma unroll 2
        for (int u = 0; u < C; ++u) {
          const NearSrc s = near_tile[(u0 + u) * L + q];
          vjp_pair<double>(s.x - xk, s.y - yk, s.z - zk, double(s.m),
                           double(s.gx), double(s.gy), double(s.gz), mk64, gkx64,
                           gky64, gkz64, eps2d, sx, sy, sz, sm);
        }
        continue;
      }
      float fx = 0.0f, fy = 0.0f, fz = 0.0f, fm = 0.0f;
      if (far) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const VSrc<NBODY_MIXED> s = far_tile[(u0 + u) * L + q];
          vjp_pair<float>(s.x - xr, s.y - yr, s.z - zr, s.m, s.gx, s.gy, s.gz,
                          mk, gkx, gky, gkz, eps2, fx, fy, fz, fm);
        }
      } else if constexpr (!NEAR64) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const NearSrc s = near_tile[(u0 + u) * L + q];
          vjp_pair<float>(float(s.x - xk), float(s.y - yk), float(s.z - zk),
                          float(s.m), float(s.gx), float(s.gy), float(s.gz), mk,
                          gkx, gky, gkz, eps2, fx, fy, fz, fm);
        }
      }
      sx += double(fx);
      sy += double(fy);
      sz += double(fz);
      sm += double(fm);
    }
  }

  double *ox = out_x + size_t(blockIdx.y) * split_stride;
  double *om = out_m + size_t(blockIdx.y) * split_stride;
  double tx = group_sum<L>(sx);
  double ty = group_sum<L>(sy);
  double tz = group_sum<L>(sz);
  const double tm = group_sum<L>(sm);
  if (q == 0 && ok) {
    if (gk >= jbeg && gk < jend) {  // this split holds the self pair (e = 0),
      // always in a near run (its run box contains x_k, gap 0)
      if constexpr (NEAR64) {
        tx -= self_pair_term<double>(mk64, gkx64, eps2d);
        ty -= self_pair_term<double>(mk64, gky64, eps2d);
        tz -= self_pair_term<double>(mk64, gkz64, eps2d);
      } else {
        tx -= self_pair_term<float>(mk, gkx, eps2);
        ty -= self_pair_term<float>(mk, gky, eps2);
        tz -= self_pair_term<float>(mk, gkz, eps2);
      }
    }
    ox[k] = scale * tx;
    ox[nt + k] = scale * ty;
    ox[2 * nt + k] = scale * tz;
    om[k] = -scale * tm;
  }
}

// Sources per near / far decision of each kernel at lanes-per-target L.
constexpr int nf_run(KernelKind kind, int L) {
  return (kThreads / L < (kind == kVjp ? kVjpChunk : kChunk)
              ? kThreads / L
              : (kind == kVjp ? kVjpChunk : kChunk)) *
         L;
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

// --------------------------------------------------- potential (diagnostic) --
//
// phi_i = sum_j m_j (|x_j - x_i|^2 + eps^2)^(-1/2) over all j, written as
// split partials like the force; the self pair's term m_i rsqrt(eps^2) is
// removed afterwards by the per-body reduction (self_potential_term).

template <typename T>
__device__ __forceinline__ double self_potential_term(T m, T eps2) {
#pragma clang fp contract(off)
  T y;
  if constexpr (sizeof(T) == 8) y = rsqrt_f64(eps2); else y = rsqrt_f32(eps2);
  return double(m) * double(y);  // exact for FP32 operands
}

template <int PREC, int L>
__global__ __launch_bounds__(kThreads) void potential_kernel(
    int n, const double *__restrict__ pos, const double *__restrict__ mass,
    double eps2d, int jchunk, double *__restrict__ out) {
  using CT = typename Coord<PREC>::T;
  using DT = typename Coord<PREC>::D;
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = PER < kChunk ? PER : kChunk;
  __shared__ Src<PREC> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int i = blockIdx.x * G + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
  const bool ok = i < n;
  const CT xi = ok ? CT(pos[i]) : CT(0);
  const CT yi = ok ? CT(pos[n + i]) : CT(0);
  const CT zi = ok ? CT(pos[2 * n + i]) : CT(0);
  double phi = 0.0;

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    const Src<PREC> b = load_src<PREC>(pos, mass, n, j, j < jend);
    __syncthreads();
    tile[tid] = b;
    __syncthreads();
    if constexpr (PREC == NBODY_FP64) {
#pragma unroll 4
      for (int u = 0; u < PER; ++u) {
        const Src<PREC> s = tile[u * L + q];
        const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        double r2 = fma(dx, dx, eps2d);
        r2 = fma(dy, dy, r2);
        r2 = fma(dz, dz, r2);
        phi = fma(s.m, rsqrt_f64(r2), phi);
      }
    } else {
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
        float f = 0.0f;
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const Src<PREC> s = tile[(u0 + u) * L + q];
          const float dx = DT(s.x - xi), dy = DT(s.y - yi), dz = DT(s.z - zi);
          float r2 = fmaf(dx, dx, eps2);
          r2 = fmaf(dy, dy, r2);
          r2 = fmaf(dz, dz, r2);
          f = fmaf(s.m, rsqrt_f32(r2), f);
        }
        phi += double(f);
      }
    }
  }
  phi = group_sum<L>(phi);
  if (q == 0 && ok) out[size_t(blockIdx.y) * n + i] = phi;
}

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
    float eps2, float scale, int jchunk, float *__restrict__ out,
    size_t split_stride) {
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  __shared__ Src<NBODY_MIXED> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int i = blockIdx.x * G + g;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
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
#pragma unroll 16
    for (int u = 0; u < PER; ++u) {
      const Src<NBODY_MIXED> s = tile[u * L + q];
      pair_f32(s.x - xi, s.y - yi, s.z - zi, s.m, eps2, ax, ay, az);
    }
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

// --------------------------------------------------- per-body FP64 kernels --
//
// One thread per (component, body): q = c * n + i.  The split partials of
// one output are added in ascending split order; their loads are issued in
// batches of 8 ahead of the (sequential) additions.

constexpr int kBodyThreads = 64;

__device__ __forceinline__ double split_sum(const double *__restrict__ part,
                                            size_t stride, int sj, size_t off) {
  double s = part[off];
  int p = 1;
  for (; p + 8 <= sj; p += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = part[size_t(p + k) * stride + off];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; p < sj; ++p) s += part[size_t(p) * stride + off];
  return s;
}

__global__ __launch_bounds__(kBodyThreads) void reduce_kernel(
    int n, int ncomp, int sj, const double *__restrict__ part, size_t stride,
    double G, double *__restrict__ out_x, double *__restrict__ out_m) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(ncomp) * n) return;
  const double v = G * split_sum(part, stride, sj, q);
  if (q < size_t(3) * n) out_x[q] = v;
  else out_m[q - size_t(3) * n] = v;
}

__global__ __launch_bounds__(kBodyThreads) void update_kernel(
    int n, int sj, const double *__restrict__ part, size_t stride, double G,
    const double *a_in, double *acc_out, const double *x_in, double *x_out,
    const double *v_in, double *v_out, double h, double dt, double *rec,
    unsigned flags) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(3) * n) return;
  const double a = part ? G * split_sum(part, stride, sj, q) : a_in[q];
  const double x = x_in[q];
  double v = v_in[q];
  if (flags & kClose) v = v + h * a;
  if (rec) {
    rec[q] = x;
    rec[size_t(3) * n + q] = v;
    rec[size_t(6) * n + q] = a;
  }
  if (flags & kOpen) {
    v = v + h * a;
    x_out[q] = x + dt * v;
  }
  v_out[q] = v;
  if (acc_out) acc_out[q] = a;
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

__global__ __launch_bounds__(kBodyThreads) void adj_init_kernel(
    int n, const double *__restrict__ gvel, const double *__restrict__ gacc_T,
    double h, int add_hv, double *__restrict__ abar,
    double *__restrict__ gmass) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(4) * n) return;
  if (q >= size_t(3) * n) {
    gmass[q - size_t(3) * n] = 0.0;
    return;
  }
  double ab = gacc_T ? gacc_T[q] : 0.0;
  if (add_hv) ab = ab + h * gvel[q];
  abar[q] = ab;
}

__global__ __launch_bounds__(kBodyThreads) void adj_combine_kernel(
    int n, int sj, const double *__restrict__ part, size_t stride, double G,
    double dt, double h, double *__restrict__ gpos, double *__restrict__ gvel,
    double *__restrict__ gmass, double *__restrict__ abar, int mode) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(4) * n) return;
  const double d = G * split_sum(part, stride, sj, q);
  if (q >= size_t(3) * n) {
    const size_t i = q - size_t(3) * n;
    gmass[i] = gmass[i] + d;
    return;
  }
  const double gx = gpos[q] + d;
  gpos[q] = gx;
  if (mode != kAdjFinal) {
    const double gv = gvel[q] + dt * gx;
    gvel[q] = gv;
    double ab = h * gv;
    if (mode == kAdjMid) ab = ab + h * gv;
    abar[q] = ab;
  }
}

// Diagnostics, first level: per body the 9 quantities
//   m|v|^2/2, m (phi - self term), m v (3), m x (3), m
// summed over the block's bodies by a fixed-order LDS tree into
// blocksum[blockIdx.x][9].  Second level: one block adds the block sums in
// ascending order.
constexpr int kDiag = 9;

template <int PREC>
__global__ __launch_bounds__(kThreads) void diag_block_kernel(
    int n, int sj, const double *__restrict__ phi_part,
    const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ mass, double eps2d,
    double *__restrict__ blocksum) {
  using AT = typename Coord<PREC>::D;
  __shared__ double red[kDiag][kThreads];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double v[kDiag];
#pragma unroll
  for (int c = 0; c < kDiag; ++c) v[c] = 0.0;
  if (i < n) {
    const double m = mass[i];
    const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
    const double phi = split_sum(phi_part, size_t(n), sj, size_t(i)) -
                       self_potential_term<AT>(AT(m), AT(eps2d));
    v[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
    v[1] = m * phi;
    v[2] = m * vx;
    v[3] = m * vy;
    v[4] = m * vz;
    v[5] = m * pos[i];
    v[6] = m * pos[n + i];
    v[7] = m * pos[2 * n + i];
    v[8] = m;
  }
#pragma unroll
  for (int c = 0; c < kDiag; ++c) red[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < kDiag; ++c)
        red[c][threadIdx.x] = red[c][threadIdx.x] + red[c][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < kDiag)
    blocksum[size_t(blockIdx.x) * kDiag + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void diag_final_kernel(
    int nblocks, const double *__restrict__ blocksum, double G,
    double *__restrict__ out) {
  const int c = threadIdx.x;
  if (c >= kDiag) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += blocksum[size_t(b) * kDiag + c];
  // out: K, W = -(G/2) sum_i m_i phi_i, momentum (3), sum m x (3), mass
  out[c] = (c == 1) ? -0.5 * G * s : s;
}

inline dim3 grid_body(int n, int ncomp) {
  return dim3(unsigned((size_t(ncomp) * n + kBodyThreads - 1) / kBodyThreads));
}

// Layout (in doubles) of the near / far box area of one all-pairs launch:
// run boxes over the n sources, then wave and workgroup boxes over the nt
// targets.
struct NfLayout {
  int run, gw, gb;
  size_t off_wave, off_block, total;
};

NfLayout nf_layout(KernelKind kind, int L, int64_t n, int64_t nt) {
  NfLayout l;
  l.run = nf_run(kind, L);
  l.gw = 64 / L;
  l.gb = kThreads / L;
  const size_t nr = size_t((n + l.run - 1) / l.run);
  const size_t nw = size_t((nt + l.gw - 1) / l.gw);
  const size_t nb = size_t((nt + l.gb - 1) / l.gb);
  l.off_wave = nr * 6;
  l.off_block = l.off_wave + nw * 6;
  l.total = l.off_block + nb * 6;
  return l;
}

// Fill the box area for a launch over targets row0 .. row0 + nt - 1: one
// pass when the targets are all n bodies, otherwise one over the sources and
// one over the target rows.
hipError_t launch_nf_boxes(KernelKind kind, int L, int n, int row0, int nt,
                           const double *pos, double *area, NfBoxes &bx,
                           hipStream_t st) {
  const NfLayout l = nf_layout(kind, L, n, nt);
  double *rb = area, *wb = area + l.off_wave, *bb = area + l.off_block;
  bx.run = rb;
  bx.wave = wb;
  bx.block = bb;
  const unsigned sblocks = unsigned((n + kThreads - 1) / kThreads);
  if (row0 == 0 && nt == n) {
    group_box_kernel<<<sblocks, kThreads, 0, st>>>(n, 0, n, pos, l.run, rb, l.gw,
                                                   wb, l.gb, bb);
    return hipGetLastError();
  }
  group_box_kernel<<<sblocks, kThreads, 0, st>>>(n, 0, n, pos, l.run, rb, 0,
                                                 nullptr, 0, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned tblocks = unsigned((nt + kThreads - 1) / kThreads);
  group_box_kernel<<<tblocks, kThreads, 0, st>>>(n, row0, nt, pos, l.gw, wb,
                                                 l.gb, bb, 0, nullptr);
  return hipGetLastError();
}

#define NBODY_RL_SWITCH(R_, L_, CALL)                                        \
  do {                                                                      \
    if (R_ == 1 && L_ == 1) { CALL(1, 1); }                                 \
    else if (R_ == 1 && L_ == 4) { CALL(1, 4); }                            \
    else if (R_ == 1 && L_ == 16) { CALL(1, 16); }                          \
    else if (R_ == 2 && L_ == 1) { CALL(2, 1); }                            \
    else if (R_ == 2 && L_ == 4) { CALL(2, 4); }                            \
    else if (R_ == 2 && L_ == 16) { CALL(2, 16); }                          \
    else return hipErrorInvalidValue;                                       \
  } while (0)

template <int PREC>
hipError_t launch_accel_p(const Plan &pl, int n, int row0, int nt,
                          const double *pos, const double *mass, double eps2,
                          double scale, double *out, size_t stride,
                          hipStream_t st) {
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const int jc = int(pl.jchunk);
#define NBODY_ACCEL_CALL(R_, L_)                                             \
  accel_kernel<PREC, R_, L_><<<grid, kThreads, 0, st>>>(                    \
      n, row0, nt, pos, mass, eps2, scale, jc, out, stride)
  NBODY_RL_SWITCH(pl.R, pl.L, NBODY_ACCEL_CALL);
#undef NBODY_ACCEL_CALL
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_vjp_p(const Plan &pl, int n, int row0, int nt,
                        const double *pos, const double *mass,
                        const double *gacc, double eps2, double scale,
                        double *ox, double *om, size_t stride, hipStream_t st) {
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const int jc = int(pl.jchunk);
#define NBODY_VJP_CALL(R_, L_)                                               \
  vjp_kernel<PREC, R_, L_><<<grid, kThreads, 0, st>>>(                      \
      n, row0, nt, pos, mass, gacc, eps2, scale, jc, ox, om, stride)
  NBODY_RL_SWITCH(pl.R, pl.L, NBODY_VJP_CALL);
#undef NBODY_VJP_CALL
  return hipGetLastError();
}

#undef NBODY_RL_SWITCH

}  // namespace

// ------------------------------------------------------------ launch plans --

Plan make_plan(KernelKind kind, int precision, int64_t n) {
  return make_plan(kind, precision, n, n);
}

Plan make_plan(KernelKind kind, int precision, int64_t nt, int64_t n) {
  // Chosen from launch-shape sweeps on MI355X (all-pairs kernel plus split
  // reduction).  Targets per lane R: 2 for FP64, 1 for the FP32-pair modes
  // (their pair chain is latency-bound, so more resident waves beat more
  // independent chains per lane).  About 8192 workgroups (32 per CU: 8
  // resident waves per SIMD, several rounds of them), reached with the
  // smallest lanes-per-target L in {1, 4, 16} that needs at most 64 source
  // splits, each at least one 256-body tile long.  Target blocks count the
  // nt target rows, source splits the n source bodies.
  const int R = (precision == NBODY_FP64 && kind != kPotential) ? 2 : 1;
  const int64_t target = 8192, max_sj = 64;
  const int64_t ntiles = (n + kThreads - 1) / kThreads;
  Plan p{};
  for (int L : {1, 4, 16}) {
    const int64_t per_block = int64_t(kThreads / L) * R;
    p.R = R;
    p.L = L;
    p.n_ib = (nt + per_block - 1) / per_block;
    p.sj = (target + p.n_ib - 1) / p.n_ib;
    if (p.sj <= std::min(max_sj, ntiles)) break;
  }
  p.sj = std::max<int64_t>(1, std::min({p.sj, ntiles, max_sj}));
  const int64_t tiles_per_split = (ntiles + p.sj - 1) / p.sj;
  p.jchunk = tiles_per_split * kThreads;
  p.sj = (n + p.jchunk - 1) / p.jchunk;
  return p;
}

hipError_t launch_accel(const Plan &pl, int precision, int n, int row0, int nt,
                        const double *pos, const double *mass, double *boxes,
                        double eps2, double scale, double *out, size_t stride,
                        hipStream_t st) {
  switch (precision) {
    case NBODY_MIXED_NF:
    case NBODY_MIXED_NF64: {
      if (pl.R != 1) return hipErrorInvalidValue;
      NfBoxes bx;
      const hipError_t e = launch_nf_boxes(kAccel, pl.L, n, row0, nt, pos, boxes, bx, st);
      if (e != hipSuccess) return e;
      const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
      const int jc = int(pl.jchunk);
#define NBODY_ACCEL_NF(L_, N64_)                                                 \
  accel_nf_kernel<L_, N64_><<<grid, kThreads, 0, st>>>(n, row0, nt, pos, mass,   \
                                                       bx, eps2, scale, jc, out, \
                                                       stride)
      const bool n64 = precision == NBODY_MIXED_NF64;
      if (pl.L == 1) { if (n64) NBODY_ACCEL_NF(1, true); else NBODY_ACCEL_NF(1, false); }
      else if (pl.L == 4) { if (n64) NBODY_ACCEL_NF(4, true); else NBODY_ACCEL_NF(4, false); }
      else if (pl.L == 16) { if (n64) NBODY_ACCEL_NF(16, true); else NBODY_ACCEL_NF(16, false); }
      else return hipErrorInvalidValue;
#undef NBODY_ACCEL_NF
      return hipGetLastError();
    }
    case NBODY_FP64:
      return launch_accel_p<NBODY_FP64>(pl, n, row0, nt, pos, mass, eps2,
                                        scale, out, stride, st);
    case NBODY_MIXED:
      return launch_accel_p<NBODY_MIXED>(pl, n, row0, nt, pos, mass, eps2,
                                         scale, out, stride, st);
    case NBODY_MIXED_D64:
      return launch_accel_p<NBODY_MIXED_D64>(pl, n, row0, nt, pos, mass, eps2,
                                             scale, out, stride, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_vjp(const Plan &pl, int precision, int n, int row0, int nt,
                      const double *pos, const double *mass, const double *gacc,
                      double *boxes, double eps2, double scale, double *ox,
                      double *om, size_t stride, hipStream_t st) {
  switch (precision) {
    case NBODY_MIXED_NF:
    case NBODY_MIXED_NF64: {
      if (pl.R != 1) return hipErrorInvalidValue;
      NfBoxes bx;
      const hipError_t e = launch_nf_boxes(kVjp, pl.L, n, row0, nt, pos, boxes, bx, st);
      if (e != hipSuccess) return e;
      const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
      const int jc = int(pl.jchunk);
#define NBODY_VJP_NF(L_, N64_)                                                   \
  vjp_nf_kernel<L_, N64_><<<grid, kThreads, 0, st>>>(n, row0, nt, pos, mass,     \
                                                     gacc, bx, eps2, scale, jc,  \
                                                     ox, om, stride)
      const bool n64 = precision == NBODY_MIXED_NF64;
      if (pl.L == 1) { if (n64) NBODY_VJP_NF(1, true); else NBODY_VJP_NF(1, false); }
      else if (pl.L == 4) { if (n64) NBODY_VJP_NF(4, true); else NBODY_VJP_NF(4, false); }
      else if (pl.L == 16) { if (n64) NBODY_VJP_NF(16, true); else NBODY_VJP_NF(16, false); }
      else return hipErrorInvalidValue;
#undef NBODY_VJP_NF
      return hipGetLastError();
    }
    case NBODY_FP64:
      return launch_vjp_p<NBODY_FP64>(pl, n, row0, nt, pos, mass, gacc, eps2,
                                      scale, ox, om, stride, st);
    case NBODY_MIXED:
      return launch_vjp_p<NBODY_MIXED>(pl, n, row0, nt, pos, mass, gacc, eps2,
                                       scale, ox, om, stride, st);
    case NBODY_MIXED_D64:
      return launch_vjp_p<NBODY_MIXED_D64>(pl, n, row0, nt, pos, mass, gacc,
                                           eps2, scale, ox, om, stride, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_potential(const Plan &pl, int precision, int n,
                            const double *pos, const double *mass, double eps2,
                            double *out, hipStream_t st) {
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const int jc = int(pl.jchunk);
#define NBODY_POT(PREC_)                                                      \
  do {                                                                        \
    if (pl.L == 1)                                                            \
      potential_kernel<PREC_, 1><<<grid, kThreads, 0, st>>>(n, pos, mass,     \
                                                            eps2, jc, out);   \
    else if (pl.L == 4)                                                       \
      potential_kernel<PREC_, 4><<<grid, kThreads, 0, st>>>(n, pos, mass,     \
                                                            eps2, jc, out);   \
    else if (pl.L == 16)                                                      \
      potential_kernel<PREC_, 16><<<grid, kThreads, 0, st>>>(n, pos, mass,    \
                                                             eps2, jc, out);  \
    else                                                                      \
      return hipErrorInvalidValue;                                            \
  } while (0)
  switch (precision) {
    case NBODY_FP64:
    case NBODY_MIXED_NF64: NBODY_POT(NBODY_FP64); break;
    case NBODY_MIXED: NBODY_POT(NBODY_MIXED); break;
    case NBODY_MIXED_D64:
    case NBODY_MIXED_NF: NBODY_POT(NBODY_MIXED_D64); break;
    default: return hipErrorInvalidValue;
  }
#undef NBODY_POT
  return hipGetLastError();
}

hipError_t launch_diagnostics(int precision, int n, int sj,
                              const double *phi_part, const double *pos,
                              const double *vel, const double *mass,
                              double eps2, double G, double *blocksum,
                              double *out, hipStream_t st) {
  const int nblocks = (n + kThreads - 1) / kThreads;
  switch (precision) {
    case NBODY_FP64:
    case NBODY_MIXED_NF64:
      diag_block_kernel<NBODY_FP64><<<nblocks, kThreads, 0, st>>>(
          n, sj, phi_part, pos, vel, mass, eps2, blocksum);
      break;
    case NBODY_MIXED:
      diag_block_kernel<NBODY_MIXED><<<nblocks, kThreads, 0, st>>>(
          n, sj, phi_part, pos, vel, mass, eps2, blocksum);
      break;
    case NBODY_MIXED_D64:
    case NBODY_MIXED_NF:
      diag_block_kernel<NBODY_MIXED_D64><<<nblocks, kThreads, 0, st>>>(
          n, sj, phi_part, pos, vel, mass, eps2, blocksum);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  diag_final_kernel<<<1, 64, 0, st>>>(nblocks, blocksum, G, out);
  return hipGetLastError();
}

hipError_t launch_reduce(int n, int sj, const double *part, size_t stride,
                         double G, double *out_x, double *out_m,
                         hipStream_t st) {
  const int ncomp = out_m ? 4 : 3;
  reduce_kernel<<<grid_body(n, ncomp), kBodyThreads, 0, st>>>(
      n, ncomp, sj, part, stride, G, out_x, out_m);
  return hipGetLastError();
}

hipError_t launch_update(int n, int sj, const double *part, size_t stride,
                         double G, const double *a_in, double *acc_out,
                         const double *x_in, double *x_out, const double *v_in,
                         double *v_out, double h, double dt, double *rec,
                         unsigned flags, hipStream_t st) {
  update_kernel<<<grid_body(n, 3), kBodyThreads, 0, st>>>(
      n, sj, part, stride, G, a_in, acc_out, x_in, x_out, v_in, v_out, h, dt,
      rec, flags);
  return hipGetLastError();
}

hipError_t launch_adj_init(int n, const double *gvel, const double *gacc_T,
                           double h, int add_hv, double *abar, double *gmass,
                           hipStream_t st) {
  adj_init_kernel<<<grid_body(n, 4), kBodyThreads, 0, st>>>(
      n, gvel, gacc_T, h, add_hv, abar, gmass);
  return hipGetLastError();
}

hipError_t launch_adj_combine(int n, int sj, const double *part, size_t stride,
                              double G, double dt, double h, double *gpos,
                              double *gvel, double *gmass, double *abar,
                              int mode, hipStream_t st) {
  adj_combine_kernel<<<grid_body(n, 4), kBodyThreads, 0, st>>>(
      n, sj, part, stride, G, dt, h, gpos, gvel, gmass, abar, mode);
  return hipGetLastError();
}

size_t near_far_box_doubles(KernelKind kind, int L, int64_t n, int64_t nt) {
  return nf_layout(kind, L, n, nt).total;
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

hipError_t launch_accel_f32(const Plan &pl, int n, const float *pos,
                            const float *mass, float eps2, float scale,
                            float *out, size_t stride, hipStream_t st) {
  if (pl.R != 1) return hipErrorInvalidValue;
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const int jc = int(pl.jchunk);
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
