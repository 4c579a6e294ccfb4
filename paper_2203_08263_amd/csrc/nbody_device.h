// Device-side building blocks shared by the gfx950 kernel sources of the
// all-pairs N-body library: the pair arithmetic of the force and its VJP,
// the LDS source-tile layouts, the lane butterfly sum and launch helpers.
// Everything lives in an unnamed namespace, so each kernel source gets its
// own inlined copy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nbody_internal.h"
#include "../../include/nbody.h"

namespace nbody {
namespace {

constexpr int kChunk = 32;        // FP32 sources per FP64 flush (forward)
constexpr int kVjpChunk = 32;     // FP32 sources per FP64 flush (VJP)
constexpr int kPairBatch = 8;     // FP32 pair weights formed ahead of their sums
constexpr int kDsBatch = 4;       // the same for two-float differences
constexpr int kBodyThreads = 64;  // threads per workgroup, per-body kernels

// Source range [jbeg, jend) of split s.
__device__ __forceinline__ void split_range(const SplitShape &sp, int s, int n,
                                            int &jbeg, int &jend) {
  const bool lng = s < sp.nlong;
  const int64_t b = lng ? int64_t(s) * sp.llong
                        : int64_t(sp.nlong) * sp.llong +
                              int64_t(s - sp.nlong) * sp.lshort;
  jbeg = int(b < n ? b : n);
  const int64_t e = b + (lng ? sp.llong : sp.lshort);
  jend = int(e < n ? e : n);
}

// The split that holds source j.
__device__ __forceinline__ int split_of(const SplitShape &sp, int j) {
  const int64_t edge = int64_t(sp.nlong) * sp.llong;
  return j < edge ? j / sp.llong : sp.nlong + int((j - edge) / sp.lshort);
}

// -------------------------------------------------------------- arithmetic --

// 1/sqrt(s) in FP64: the hardware estimate y0 refined by one third-order
// step.  With e = 1 - s y0^2, s^(-1/2) = y0 (1 - e)^(-1/2) = y0 (1 + e/2 +
// 3e^2/8 + O(e^3)), so y0 + (y0 e)(1/2 + 3e/8) leaves a truncation error of
// about 2.5 d^3 for an estimate of relative error d.  The estimate is within
// 2^-24 of s^(-1/2) (measured over 4M arguments spanning 2^-60 .. 2^60), so
// that is far below one rounding; emulated with exact FMAs the step is within
// 1.23 units of 2^-53 for any |d| <= 2^-21, as two Newton steps are.  Five
// FP64 operations instead of the seven of two Newton steps.
__device__ __forceinline__ double rsqrt_f64(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  const double e = fma(-(s * y), y, 1.0);
  const double p = fma(e, 0.375, 0.5);
  return fma(y * e, p, y);
}

__device__ __forceinline__ float rsqrt_f32(float s) {
  return __builtin_amdgcn_rsqf(s);
}

// m s^(-3/2) in FP64 from the hardware estimate y0 of s^(-1/2): with
// e = 1 - s y0^2, s^(-3/2) = y0^3 (1 - e)^(-3/2) = y0^3 (1 + 3e/2 + 15e^2/8
// + O(e^3)), so m y0^3 + (m y0^3 e)(3/2 + 15e/8) leaves a truncation error
// of about 35/16 e^3 (below 2^-64 for the estimate's |e| <= 2^-23).  Seven
// FP64 operations where refining y first (rsqrt_f64) and cubing it takes
// eight; emulated with exact FMAs over s in 1e-30 .. 1e30 and the estimate
// anywhere within 2^-24.2, within 2.0 units of 2^-53 of m s^(-3/2), against
// 4.5 for the refined y cubed.
__device__ __forceinline__ double weight_f64(double m, double s) {
  const double y0 = __builtin_amdgcn_rsq(s);
  const double y02 = y0 * y0;
  const double e = fma(-s, y02, 1.0);
  const double my3 = (m * y0) * y02;
  const double p = fma(e, 1.875, 1.5);
  return fma(my3 * e, p, my3);
}

// One source j acting on one target: a += m_j d (|d|^2 + eps^2)^-3/2.
__device__ __forceinline__ void pair_f64(double dx, double dy, double dz,
                                         double m, double eps2, double &ax,
                                         double &ay, double &az) {
  double s = fma(dx, dx, eps2);
  s = fma(dy, dy, s);
  s = fma(dz, dz, s);
  const double w = weight_f64(m, s);
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

// The FP32 pair terms of the C sources u = 0 .. C-1 of one chunk, added in
// ascending u into (fx, fy, fz); src(u, dx, dy, dz, m) yields source u's
// difference x_j - x_i and mass in FP32.  The weights of B sources are formed
// before their terms are added: B independent pair chains for the scheduler
// (one source at a time, the compiler waits on each LDS read before its
// pair).  The additions keep the ascending order, so the sums are bitwise
// those of pair_f32 applied source by source.
template <int C, int B, typename SrcF>
__device__ __forceinline__ void chunk_sum_f32(SrcF src, float eps2, float &fx,
                                              float &fy, float &fz) {
  constexpr int BB = B < C ? B : C;
  static_assert(C % BB == 0, "chunk length must be a multiple of the batch");
#pragma unroll
  for (int u0 = 0; u0 < C; u0 += BB) {
    float dx[BB], dy[BB], dz[BB], w[BB];
#pragma unroll
    for (int q = 0; q < BB; ++q) {
      float m;
      src(u0 + q, dx[q], dy[q], dz[q], m);
      float s = fmaf(dx[q], dx[q], eps2);
      s = fmaf(dy[q], dy[q], s);
      s = fmaf(dz[q], dz[q], s);
      const float y = rsqrt_f32(s);
      w[q] = (m * y) * (y * y);
    }
#pragma unroll
    for (int q = 0; q < BB; ++q) {
      fx = fmaf(w[q], dx[q], fx);
      fy = fmaf(w[q], dy[q], fy);
      fz = fmaf(w[q], dz[q], fz);
    }
  }
}

// One source j against target k for the VJP (row formulation), with h formed
// per pair (the FP64 near runs of NBODY_MIXED_NF64; every other VJP pair
// takes the split form below):
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

// The FP32 VJP pair in split form.  The row term y3 (h - 3 y2 (e.h) e) is
// linear in h = m_k gbar_j - m_j gbar_k, so a chunk of sources accumulates
//   a = sum y3 gbar_j,   b = sum y3 m_j,   c = sum y3 (y2 (e.h)) e,
//   dm = sum y3 (gbar_j . e)                   (y = s^-1/2, y2 = y^2, y3 = y^3)
// and the target adds m_k a - gbar_k b - 3 c once per chunk (vjp_split_flush).
// e.h is formed as m_k (gbar_j . e) - m_j (gbar_k . e), reusing the mass
// term's dot product: 26 operations per pair (10 two-operand, 16 FMA) where
// forming h per pair takes 29 (12 and 17).  The error of each sum stays
// within u32 times the sum of its terms' magnitudes, which m_k, |gbar_k| and
// 3 scale to the same s^-3/2 (m_k |gbar_j| + m_j |gbar_k|) budget as before.
// y2 (e.h) <= |e| H / s <= H / (2 eps) with H = m_k |gbar_j| + m_j |gbar_k|,
// and y3 times it at most 0.29 eps^-4 H, so the FP32 form needs eps^-4 H
// below FLT_MAX.  `drop` zeroes the pair (y = 0): the self pair j == k,
// whose y3 m_k gbar_k in a and y3 m_k in b cancel in the flush only up to the
// rounding of those sums, so it is left out instead.
struct VjpSplit {
  float ax, ay, az, b, cx, cy, cz, dm;
};

__device__ __forceinline__ void vjp_split_zero(VjpSplit &a) {
  a.ax = a.ay = a.az = a.b = 0.0f;
  a.cx = a.cy = a.cz = a.dm = 0.0f;
}

__device__ __forceinline__ void vjp_pair_split(float ex, float ey, float ez,
                                               float mj, float gjx, float gjy,
                                               float gjz, float mk, float gkx,
                                               float gky, float gkz,
                                               float eps2, bool drop,
                                               VjpSplit &a) {
  float s = fmaf(ex, ex, eps2);
  s = fmaf(ey, ey, s);
  s = fmaf(ez, ez, s);
  const float y = drop ? 0.0f : rsqrt_f32(s);
  const float y2 = y * y;
  const float y3 = y2 * y;
  const float ge = fmaf(gjz, ez, fmaf(gjy, ey, gjx * ex));
  const float ek = fmaf(gkz, ez, fmaf(gky, ey, gkx * ex));
  const float eh = fmaf(mk, ge, -(mj * ek));
  const float w = y3 * (y2 * eh);
  a.dm = fmaf(ge, y3, a.dm);
  a.ax = fmaf(y3, gjx, a.ax);
  a.ay = fmaf(y3, gjy, a.ay);
  a.az = fmaf(y3, gjz, a.az);
  a.b = fmaf(y3, mj, a.b);
  a.cx = fmaf(w, ex, a.cx);
  a.cy = fmaf(w, ey, a.cy);
  a.cz = fmaf(w, ez, a.cz);
}

// The split-form pair in FP64 (the FP64 VJP): the same sums, in FP64
// straight over the whole source range; the target forms its row from them
// once, after the last source.  26 FP64 operations plus the reciprocal
// square root instead of 29.
struct VjpSplit64 {
  double ax, ay, az, b, cx, cy, cz, dm;
};

__device__ __forceinline__ void vjp_pair_split64(double ex, double ey,
                                                 double ez, double mj,
                                                 double gjx, double gjy,
                                                 double gjz, double mk,
                                                 double gkx, double gky,
                                                 double gkz, double eps2,
                                                 bool drop, VjpSplit64 &a) {
  double s = fma(ex, ex, eps2);
  s = fma(ey, ey, s);
  s = fma(ez, ez, s);
  const double y = drop ? 0.0 : rsqrt_f64(s);
  const double y2 = y * y;
  const double y3 = y2 * y;
  const double ge = fma(gjz, ez, fma(gjy, ey, gjx * ex));
  const double ek = fma(gkz, ez, fma(gky, ey, gkx * ex));
  const double eh = fma(mk, ge, -(mj * ek));
  const double w = y3 * (y2 * eh);
  a.dm = fma(ge, y3, a.dm);
  a.ax = fma(y3, gjx, a.ax);
  a.ay = fma(y3, gjy, a.ay);
  a.az = fma(y3, gjz, a.az);
  a.b = fma(y3, mj, a.b);
  a.cx = fma(w, ex, a.cx);
  a.cy = fma(w, ey, a.cy);
  a.cz = fma(w, ez, a.cz);
}

// The chunk's row terms m_k a - gbar_k b - 3 c (and dm), added to the FP64
// accumulators of the target.
__device__ __forceinline__ void vjp_split_flush(const VjpSplit &a, float mk,
                                                float gkx, float gky,
                                                float gkz, double &sx,
                                                double &sy, double &sz,
                                                double &sm) {
  sx += double(fmaf(-3.0f, a.cx, fmaf(mk, a.ax, -(gkx * a.b))));
  sy += double(fmaf(-3.0f, a.cy, fmaf(mk, a.ay, -(gky * a.b))));
  sz += double(fmaf(-3.0f, a.cz, fmaf(mk, a.az, -(gkz * a.b))));
  sm += double(a.dm);
}

// ------------------------------------------------------ source tile layout --

// NBODY_MIXED_DS splits a coordinate v into two FP32 numbers, hi = fl32(v)
// and lo = fl32(v - hi) (v - hi is exact in FP64), so hi + lo carries v to
// within u32^2 |v|.  The pair difference is then formed as
// (x_j^hi - x_i^hi) + (x_j^lo - x_i^lo) in FP32: the first difference is
// exact for close pairs (Sterbenz), the second is of order u32 |x| and
// rounds at the u32^2 level, so d carries about 2 u32 |d| + 4 u32^2
// (|x_i| + |x_j|) instead of the u32 (|x_i| + |x_j|) of rounding the
// positions themselves.
__device__ __forceinline__ void split_f32(double v, float &hi, float &lo) {
  hi = float(v);
  lo = float(v - double(hi));
}

__device__ __forceinline__ float ds_diff(float sh, float sl, float th,
                                         float tl) {
  return (sh - th) + (sl - tl);
}

template <int PREC> struct Src;
template <> struct Src<NBODY_FP64> { double x, y, z, m; };
template <> struct Src<NBODY_MIXED> { float x, y, z, m; };
template <> struct Src<NBODY_MIXED_D64> { double x, y, z; float m, pad; };
// x, y, z: the hi parts; xl, yl, zl: the lo parts
template <> struct Src<NBODY_MIXED_DS> { float x, y, z, m, xl, yl, zl, pad; };

template <int PREC>
__device__ __forceinline__ Src<PREC> load_src(const double *__restrict__ pos,
                                              const double *__restrict__ mass,
                                              int n, int j, bool valid) {
  Src<PREC> b{};
  if (valid) {
    if constexpr (PREC == NBODY_MIXED_DS) {
      split_f32(pos[j], b.x, b.xl);
      split_f32(pos[n + j], b.y, b.yl);
      split_f32(pos[2 * n + j], b.z, b.zl);
    } else {
      b.x = pos[j];
      b.y = pos[n + j];
      b.z = pos[2 * n + j];
    }
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
template <> struct VSrc<NBODY_MIXED_DS> {
  float x, y, z, m, gx, gy, gz, pad0, xl, yl, zl, pad1;
};

// Coordinate type of a target body and of its pair difference (for
// NBODY_MIXED_DS the type of each of the two parts).
template <int PREC> struct Coord { using T = double; using D = double; };
template <> struct Coord<NBODY_MIXED> { using T = float; using D = float; };
template <> struct Coord<NBODY_MIXED_D64> { using T = double; using D = float; };
template <> struct Coord<NBODY_MIXED_DS> { using T = float; using D = float; };

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

inline dim3 grid_body(int n, int ncomp) {
  return dim3(unsigned((size_t(ncomp) * n + kBodyThreads - 1) / kBodyThreads));
}

}  // namespace
}  // namespace nbody
