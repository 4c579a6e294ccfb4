// gfx950 kernels of the all-pairs gravitational N-body hot path.
//
// The all-pairs kernels (acceleration and its VJP) share one shape:
//  - a workgroup of 256 threads (4 wave64s) owns kThreads*R target bodies,
//    R per thread, strided by kThreads so every load and store is coalesced;
//  - blockIdx.y selects a contiguous source range (SplitShape), staged
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
// approximation (v_rsq_f32 / v_rsq_f64), refined in FP64 by one third-order step.
#include <algorithm>
#include <type_traits>

#include "nbody_device.h"

namespace nbody {
namespace {

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

// Largest system the one-launch step serves, per precision (small_system on
// the host): the step kernel stages all of its sources in LDS at once.
template <int PREC> constexpr int kSmallMax =
    PREC == NBODY_FP64 ? 2048 : (PREC == NBODY_MIXED ? 512 : 1024);

// The sums of one lane: its share (tile entries q, q + L, ...) of the sources
// jbeg .. jend - 1 acting on the R targets of its lane group, without G.
// With ALL (the one-launch step of a small system) every source is staged in
// `tile` (kSmallMax<PREC> entries) before the first pair, so the global loads
// of all tiles are in flight together; the pairs are then visited in the same
// order as tile by tile, so the sums are bitwise those of the tiled form.
template <int PREC, int R, int L, bool ALL = false>
__device__ __forceinline__ void accel_lane_sums(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, double eps2d, int jbeg, int jend,
    Src<PREC> *tile, double (&ax)[R], double (&ay)[R], double (&az)[R]) {
  using CT = typename Coord<PREC>::T;
  using DT = typename Coord<PREC>::D;
  constexpr int G = kThreads / L;             // target groups per workgroup
  constexpr int PER = kThreads / L;           // tile entries per lane
  constexpr int C = PER < kChunk ? PER : kChunk;

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int ibase = blockIdx.x * (G * R) + g;

  CT xi[R], yi[R], zi[R];
  float xl[R], yl[R], zl[R];  // lo parts (NBODY_MIXED_DS only)
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * G;
    const bool ok = i < nt;
    const int gi = row0 + i;
    if constexpr (PREC == NBODY_MIXED_DS) {
      split_f32(ok ? pos[gi] : 0.0, xi[r], xl[r]);
      split_f32(ok ? pos[n + gi] : 0.0, yi[r], yl[r]);
      split_f32(ok ? pos[2 * n + gi] : 0.0, zi[r], zl[r]);
    } else {
      xi[r] = ok ? CT(pos[gi]) : CT(0);
      yi[r] = ok ? CT(pos[n + gi]) : CT(0);
      zi[r] = ok ? CT(pos[2 * n + gi]) : CT(0);
    }
    ax[r] = ay[r] = az[r] = 0.0;
  }

  if constexpr (ALL) {
    constexpr int K = kSmallMax<PREC> / kThreads;
    Src<PREC> b[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {  // only the tiles the sources reach
      const int j = jbeg + k * kThreads + tid;
      if (jbeg + k * kThreads < jend) b[k] = load_src<PREC>(pos, mass, n, j, j < jend);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (jbeg + k * kThreads < jend) tile[k * kThreads + tid] = b[k];
    __syncthreads();
  }
  for (int jt = jbeg; jt < jend; jt += kThreads) {
    if constexpr (!ALL) {
      const int j = jt + tid;
      const Src<PREC> b = load_src<PREC>(pos, mass, n, j, j < jend);
      __syncthreads();  // previous tile fully consumed
      tile[tid] = b;
      __syncthreads();
    }
    const Src<PREC> *t = ALL ? tile + (jt - jbeg) : tile;

    if constexpr (PREC == NBODY_FP64) {
#pragma unroll 4
      for (int u = 0; u < PER; ++u) {
        const Src<PREC> s = t[u * L + q];
#pragma unroll
        for (int r = 0; r < R; ++r)
          pair_f64(s.x - xi[r], s.y - yi[r], s.z - zi[r], s.m, eps2d, ax[r],
                   ay[r], az[r]);
      }
    } else if constexpr (PREC == NBODY_MIXED && R == 1) {
      // FP32 sources: the weights of kPairBatch sources are formed ahead of
      // their sums (chunk_sum_f32; measured +2-3 % at N = 65536 - 262144)
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        chunk_sum_f32<C, kPairBatch>(
            [&](int u, float &dx, float &dy, float &dz, float &m) {
              const Src<PREC> s = t[(u0 + u) * L + q];
              dx = s.x - xi[0];
              dy = s.y - yi[0];
              dz = s.z - zi[0];
              m = s.m;
            },
            eps2, fx, fy, fz);
        ax[0] += double(fx);
        ay[0] += double(fy);
        az[0] += double(fz);
      }
    } else if constexpr (PREC == NBODY_MIXED_DS) {
      // two-float differences (ds_diff), then the FP32 pair of NBODY_MIXED
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float fx = 0.0f, fy = 0.0f, fz = 0.0f;
          chunk_sum_f32<C, kDsBatch>(
              [&](int u, float &dx, float &dy, float &dz, float &m) {
                const Src<PREC> s = t[(u0 + u) * L + q];
                dx = ds_diff(s.x, s.xl, xi[r], xl[r]);
                dy = ds_diff(s.y, s.yl, yi[r], yl[r]);
                dz = ds_diff(s.z, s.zl, zi[r], zl[r]);
                m = s.m;
              },
              eps2, fx, fy, fz);
          ax[r] += double(fx);
          ay[r] += double(fy);
          az[r] += double(fz);
        }
      }
    } else {
      // FP64 sources (difference rounded once): batching would hold the FP64
      // coordinates of several sources at once and cost occupancy
      const float eps2 = float(eps2d);
      for (int u0 = 0; u0 < PER; u0 += C) {
        float fx[R], fy[R], fz[R];
#pragma unroll
        for (int r = 0; r < R; ++r) fx[r] = fy[r] = fz[r] = 0.0f;
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const Src<PREC> s = t[(u0 + u) * L + q];
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
}

template <int PREC, int R, int L>
__global__ __launch_bounds__(kThreads) void accel_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, double eps2d, double scale, SplitShape split,
    double *__restrict__ out, size_t split_stride) {
  constexpr int G = kThreads / L;
  __shared__ Src<PREC> tile[kThreads];
  const int g = threadIdx.x / L, q = threadIdx.x % L;
  const int ibase = blockIdx.x * (G * R) + g;
  int jbeg, jend;
  split_range(split, blockIdx.y, n, jbeg, jend);
  double ax[R], ay[R], az[R];
  accel_lane_sums<PREC, R, L>(n, row0, nt, pos, mass, eps2d, jbeg, jend, tile,
                              ax, ay, az);

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

// Resident waves per SIMD the VJP kernels are compiled for.  Left free, the
// compiler hoists a whole chunk's LDS reads in the FP32-pair kernels and needs
// over 100 VGPRs (4 waves); held to 8 waves (64 VGPRs) they lose nothing
// and do not spill, except the D64 kernel at L = 16 (77 VGPRs, 6 waves, no
// spill) and the mixed kernel at L = 1, which with chunks of 32 sources
// spills at 8 waves and is held to 7 (72 VGPRs; seven spilled, and still
// 1.3-1.9 % faster than chunks of 16 at 8 waves; at 6 waves it spills more).
// FP64 (78 VGPRs and 6 waves at one target per lane, about 90 and 5 at two)
// is left to the compiler: the split form spills at 7 or 8.
constexpr int vjp_waves(int prec, int L) {
  if (prec == NBODY_FP64) return 1;
  if (prec == NBODY_MIXED_D64 && L == 16) return 6;
  return prec == NBODY_MIXED && L == 1 ? 7 : 8;
}

// Rows as in accel_kernel: targets k = row0 .. row0 + nt - 1, sources all n
// bodies (with their dL/da), output row k - row0 of stride nt.
template <int PREC, int R, int L>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(vjp_waves(PREC, L)))) void vjp_kernel(
    int n, int row0, int nt, const double *__restrict__ pos,
    const double *__restrict__ mass, const double *__restrict__ gacc,
    double eps2d, double scale, SplitShape split, double *__restrict__ out_x,
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
  int jbeg, jend;
  split_range(split, blockIdx.y, n, jbeg, jend);

  CT xk[R], yk[R], zk[R];
  float xl[R], yl[R], zl[R];  // lo parts (NBODY_MIXED_DS only)
  AT mk[R], gkx[R], gky[R], gkz[R];
  double sx[R], sy[R], sz[R], sm[R];
  VjpSplit64 acc64[R];  // NBODY_FP64 only
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = kbase + r * G;
    const bool ok = k < nt;
    const int gk = row0 + k;
    if constexpr (PREC == NBODY_MIXED_DS) {
      split_f32(ok ? pos[gk] : 0.0, xk[r], xl[r]);
      split_f32(ok ? pos[n + gk] : 0.0, yk[r], yl[r]);
      split_f32(ok ? pos[2 * n + gk] : 0.0, zk[r], zl[r]);
    } else {
      xk[r] = ok ? CT(pos[gk]) : CT(0);
      yk[r] = ok ? CT(pos[n + gk]) : CT(0);
      zk[r] = ok ? CT(pos[2 * n + gk]) : CT(0);
    }
    mk[r] = ok ? AT(mass[gk]) : AT(0);
    gkx[r] = ok ? AT(gacc[gk]) : AT(0);
    gky[r] = ok ? AT(gacc[n + gk]) : AT(0);
    gkz[r] = ok ? AT(gacc[2 * n + gk]) : AT(0);
    sx[r] = sy[r] = sz[r] = sm[r] = 0.0;
    acc64[r] = VjpSplit64{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  }

  for (int jt = jbeg; jt < jend; jt += kThreads) {
    const int j = jt + tid;
    VSrc<PREC> b{};
    if (j < jend) {
      if constexpr (PREC == NBODY_MIXED_DS) {
        split_f32(pos[j], b.x, b.xl);
        split_f32(pos[n + j], b.y, b.yl);
        split_f32(pos[2 * n + j], b.z, b.zl);
      } else {
        b.x = pos[j];
        b.y = pos[n + j];
        b.z = pos[2 * n + j];
      }
      b.m = mass[j];
      b.gx = gacc[j];
      b.gy = gacc[n + j];
      b.gz = gacc[2 * n + j];
    }
    __syncthreads();
    tile[tid] = b;
    __syncthreads();

    if constexpr (PREC == NBODY_FP64 && R == 2) {
      // two targets per lane (small systems): h formed per pair
#pragma unroll 2
      for (int u = 0; u < PER; ++u) {
        const VSrc<PREC> s = tile[u * L + q];
#pragma unroll
        for (int r = 0; r < R; ++r)
          vjp_pair<double>(s.x - xk[r], s.y - yk[r], s.z - zk[r], s.m, s.gx,
                           s.gy, s.gz, mk[r], gkx[r], gky[r], gkz[r], eps2d,
                           sx[r], sy[r], sz[r], sm[r]);
      }
    } else if constexpr (PREC == NBODY_FP64) {
      // split form in FP64, self pairs dropped in the diagonal tiles as below
      const int kblk = row0 + blockIdx.x * (G * R);
      const bool diag = jt < kblk + G * R && jt + kThreads > kblk;
      auto tile_pass64 = [&](auto diag_tag) {
        constexpr bool D = decltype(diag_tag)::value;
#pragma unroll 2
        for (int u = 0; u < PER; ++u) {
          const VSrc<PREC> s = tile[u * L + q];
          const int j = jt + u * L + q;
#pragma unroll
          for (int r = 0; r < R; ++r)
            vjp_pair_split64(s.x - xk[r], s.y - yk[r], s.z - zk[r], s.m, s.gx,
                             s.gy, s.gz, mk[r], gkx[r], gky[r], gkz[r], eps2d,
                             D && j == row0 + kbase + r * G, acc64[r]);
        }
      };
      if (diag)
        tile_pass64(std::true_type{});
      else
        tile_pass64(std::false_type{});
    } else {
      const float eps2 = float(eps2d);
      // Tiles that hold some of this workgroup's own targets drop their self
      // pairs (vjp_pair_split); every other tile runs without the test.
      const int kblk = row0 + blockIdx.x * (G * R);
      const bool diag = jt < kblk + G * R && jt + kThreads > kblk;
      auto tile_pass = [&](auto diag_tag) {
        constexpr bool D = decltype(diag_tag)::value;
        for (int u0 = 0; u0 < PER; u0 += C) {
          VjpSplit acc[R];
#pragma unroll
          for (int r = 0; r < R; ++r) vjp_split_zero(acc[r]);
#pragma unroll
          for (int u = 0; u < C; ++u) {
            const VSrc<PREC> s = tile[(u0 + u) * L + q];
            const int j = jt + (u0 + u) * L + q;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              float ex, ey, ez;
              if constexpr (PREC == NBODY_MIXED_DS) {
                ex = ds_diff(s.x, s.xl, xk[r], xl[r]);
                ey = ds_diff(s.y, s.yl, yk[r], yl[r]);
                ez = ds_diff(s.z, s.zl, zk[r], zl[r]);
              } else {
                ex = DT(s.x - xk[r]);
                ey = DT(s.y - yk[r]);
                ez = DT(s.z - zk[r]);
              }
              vjp_pair_split(ex, ey, ez, s.m, s.gx, s.gy, s.gz, mk[r],
                             gkx[r], gky[r], gkz[r], eps2,
                             D && j == row0 + kbase + r * G, acc[r]);
            }
          }
#pragma unroll
          for (int r = 0; r < R; ++r)
            vjp_split_flush(acc[r], mk[r], gkx[r], gky[r], gkz[r], sx[r],
                            sy[r], sz[r], sm[r]);
        }
      };
      if (diag)
        tile_pass(std::true_type{});
      else
        tile_pass(std::false_type{});
    }
  }

  double *ox = out_x + size_t(blockIdx.y) * split_stride;
  double *om = out_m + size_t(blockIdx.y) * split_stride;
  const double eps2a = eps2d;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (PREC == NBODY_FP64 && R == 1) {
      const VjpSplit64 &a = acc64[r];
      sx[r] = fma(-3.0, a.cx, fma(mk[r], a.ax, -(gkx[r] * a.b)));
      sy[r] = fma(-3.0, a.cy, fma(mk[r], a.ay, -(gky[r] * a.b)));
      sz[r] = fma(-3.0, a.cz, fma(mk[r], a.az, -(gkz[r] * a.b)));
      sm[r] = a.dm;
    }
    double tx = group_sum<L>(sx[r]);
    double ty = group_sum<L>(sy[r]);
    double tz = group_sum<L>(sz[r]);
    const double tm = group_sum<L>(sm[r]);
    const int k = kbase + r * G;
    const int gk = row0 + k;
    if (q == 0 && k < nt) {
      // the self pair: removed here after h formed per pair (FP64 with two
      // targets per lane), dropped by the split-form pairs
      if constexpr (PREC == NBODY_FP64 && R == 2) {
        if (gk >= jbeg && gk < jend) {
          tx -= self_pair_term<double>(mk[r], gkx[r], eps2a);
          ty -= self_pair_term<double>(mk[r], gky[r], eps2a);
          tz -= self_pair_term<double>(mk[r], gkz[r], eps2a);
        }
      }
      ox[k] = scale * tx;
      ox[nt + k] = scale * ty;
      ox[2 * nt + k] = scale * tz;
      om[k] = -scale * tm;
    }
  }
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
    double eps2d, SplitShape split, double *__restrict__ out) {
  using CT = typename Coord<PREC>::T;
  using DT = typename Coord<PREC>::D;
  constexpr int G = kThreads / L;
  constexpr int PER = kThreads / L;
  constexpr int C = PER < kChunk ? PER : kChunk;
  __shared__ Src<PREC> tile[kThreads];

  const int tid = threadIdx.x;
  const int g = tid / L, q = tid % L;
  const int i = blockIdx.x * G + g;
  int jbeg, jend;
  split_range(split, blockIdx.y, n, jbeg, jend);
  const bool ok = i < n;
  CT xi, yi, zi;
  float xl = 0.0f, yl = 0.0f, zl = 0.0f;  // lo parts (NBODY_MIXED_DS only)
  if constexpr (PREC == NBODY_MIXED_DS) {
    split_f32(ok ? pos[i] : 0.0, xi, xl);
    split_f32(ok ? pos[n + i] : 0.0, yi, yl);
    split_f32(ok ? pos[2 * n + i] : 0.0, zi, zl);
  } else {
    xi = ok ? CT(pos[i]) : CT(0);
    yi = ok ? CT(pos[n + i]) : CT(0);
    zi = ok ? CT(pos[2 * n + i]) : CT(0);
  }
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
          float dx, dy, dz;
          if constexpr (PREC == NBODY_MIXED_DS) {
            dx = ds_diff(s.x, s.xl, xi, xl);
            dy = ds_diff(s.y, s.yl, yi, yl);
            dz = ds_diff(s.z, s.zl, zi, zl);
          } else {
            dx = DT(s.x - xi);
            dy = DT(s.y - yi);
            dz = DT(s.z - zi);
          }
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

// --------------------------------------------------- per-body FP64 kernels --
//
// One thread per (component, body): q = c * n + i.  The split partials of
// one output are added in ascending split order; their loads are issued in
// batches of 8 ahead of the (sequential) additions.

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

// The state update of one (component, body) entry q of [3][n] with its new
// acceleration a: closing half-kick, checkpoint record, opening half-kick and
// drift (flags kClose / kOpen).
// update_entry on the entry's position x and velocity v, already loaded.
__device__ __forceinline__ void update_entry_xv(
    int n, size_t q, double a, double x, double v, double *x_out,
    double *v_out, double *acc_out, double h, double dt, double *rec,
    unsigned flags) {
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

__device__ __forceinline__ void update_entry(
    int n, size_t q, double a, const double *x_in, double *x_out,
    const double *v_in, double *v_out, double *acc_out, double h, double dt,
    double *rec, unsigned flags) {
  update_entry_xv(n, q, a, x_in[q], v_in[q], x_out, v_out, acc_out, h, dt, rec,
                  flags);
}

__global__ __launch_bounds__(kBodyThreads) void update_kernel(
    int n, int sj, const double *__restrict__ part, size_t stride, double G,
    const double *a_in, double *acc_out, const double *x_in, double *x_out,
    const double *v_in, double *v_out, double h, double dt, double *rec,
    unsigned flags) {
  const size_t q = size_t(blockIdx.x) * kBodyThreads + threadIdx.x;
  if (q >= size_t(3) * n) return;
  const double a = part ? G * split_sum(part, stride, sj, q) : a_in[q];
  update_entry(n, q, a, x_in, x_out, v_in, v_out, acc_out, h, dt, rec, flags);
}

// One whole time step of a small system in one launch: a wave per target
// body (L = 64 lanes share it, kThreads / 64 targets per workgroup) sums the
// force of all n sources, then its first lane applies update_entry to the
// three components.  x_in must not alias x_out: every workgroup still reads
// all of x_in while others write their drifted positions.
template <int PREC>
__global__ __launch_bounds__(kThreads) void step_small_kernel(
    int n, const double *__restrict__ x_in, const double *__restrict__ mass,
    double eps2d, double G, const double *v_in, double *v_out,
    double *__restrict__ x_out, double *acc_out, double *rec, double h,
    double dt, unsigned flags) {
  constexpr int L = 64;
  __shared__ Src<PREC> tile[kSmallMax<PREC>];
  const int i = blockIdx.x * (kThreads / L) + int(threadIdx.x) / L;
  const bool upd = threadIdx.x % L == 0 && i < n;
  // the target's position and velocity, loaded before the force sum so their
  // latency hides under it (after it, v_in may alias v_out, so the three
  // components' loads and stores would follow one another)
  double xs[3] = {0.0, 0.0, 0.0}, vs[3] = {0.0, 0.0, 0.0};
  if (upd) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xs[c] = x_in[size_t(c) * n + i];
      vs[c] = v_in[size_t(c) * n + i];
    }
  }
  double ax[1], ay[1], az[1];
  accel_lane_sums<PREC, 1, L, true>(n, 0, n, x_in, mass, eps2d, 0, n, tile, ax,
                                    ay, az);
  const double s[3] = {group_sum<L>(ax[0]), group_sum<L>(ay[0]),
                       group_sum<L>(az[0])};
  if (upd) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      update_entry_xv(n, size_t(c) * n + i, G * s[c], xs[c], vs[c], x_out,
                      v_out, acc_out, h, dt, rec, flags);
  }
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
    if (int(threadIdx.x) < w) {
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

#define NBODY_RL_SWITCH(R_, L_, CALL)                                        \
  do {                                                                      \
    if (R_ == 1 && L_ == 1) { CALL(1, 1); }                                 \
    else if (R_ == 1 && L_ == 4) { CALL(1, 4); }                            \
    else if (R_ == 1 && L_ == 16) { CALL(1, 16); }                          \
    else if (R_ == 1 && L_ == 64) { CALL(1, 64); }                          \
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
  const SplitShape jc = pl.split;
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
  const SplitShape jc = pl.split;
#define NBODY_VJP_CALL(R_, L_)                                               \
  vjp_kernel<PREC, R_, L_><<<grid, kThreads, 0, st>>>(                      \
      n, row0, nt, pos, mass, gacc, eps2, scale, jc, ox, om, stride)
  // the shapes the VJP plans use: one target per lane with 1, 4 or 16 lanes
  // per target, and for small FP64 systems two targets per lane with 16
  if (pl.R == 1 && pl.L == 1) NBODY_VJP_CALL(1, 1);
  else if (pl.R == 1 && pl.L == 4) NBODY_VJP_CALL(1, 4);
  else if (pl.R == 1 && pl.L == 16) NBODY_VJP_CALL(1, 16);
  else if (pl.R == 2 && pl.L == 16) {
    if constexpr (PREC == NBODY_FP64) NBODY_VJP_CALL(2, 16);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef NBODY_VJP_CALL
  return hipGetLastError();
}

#undef NBODY_RL_SWITCH

}  // namespace


hipError_t launch_accel(const Plan &pl, int precision, int n, int row0, int nt,
                        const double *pos, const double *mass, double *boxes,
                        double eps2, double scale, double *out, size_t stride,
                        hipStream_t st) {
  switch (precision) {
    case NBODY_MIXED_NF:
    case NBODY_MIXED_NF64:
      return launch_accel_nf(pl, n, row0, nt, pos, mass, boxes, eps2, scale,
                             out, stride, precision == NBODY_MIXED_NF64, st);
    case NBODY_FP64:
      return launch_accel_p<NBODY_FP64>(pl, n, row0, nt, pos, mass, eps2,
                                        scale, out, stride, st);
    case NBODY_MIXED:
      return launch_accel_p<NBODY_MIXED>(pl, n, row0, nt, pos, mass, eps2,
                                         scale, out, stride, st);
    case NBODY_MIXED_D64:
      return launch_accel_p<NBODY_MIXED_D64>(pl, n, row0, nt, pos, mass, eps2,
                                             scale, out, stride, st);
    case NBODY_MIXED_DS:
      return launch_accel_p<NBODY_MIXED_DS>(pl, n, row0, nt, pos, mass, eps2,
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
    case NBODY_MIXED_NF64:
      return launch_vjp_nf(pl, n, row0, nt, pos, mass, gacc, boxes, eps2, scale,
                           ox, om, stride, precision == NBODY_MIXED_NF64, st);
    case NBODY_FP64:
      return launch_vjp_p<NBODY_FP64>(pl, n, row0, nt, pos, mass, gacc, eps2,
                                      scale, ox, om, stride, st);
    case NBODY_MIXED:
      return launch_vjp_p<NBODY_MIXED>(pl, n, row0, nt, pos, mass, gacc, eps2,
                                       scale, ox, om, stride, st);
    case NBODY_MIXED_D64:
      return launch_vjp_p<NBODY_MIXED_D64>(pl, n, row0, nt, pos, mass, gacc,
                                           eps2, scale, ox, om, stride, st);
    case NBODY_MIXED_DS:
      return launch_vjp_p<NBODY_MIXED_DS>(pl, n, row0, nt, pos, mass, gacc,
                                          eps2, scale, ox, om, stride, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_potential(const Plan &pl, int precision, int n,
                            const double *pos, const double *mass, double eps2,
                            double *out, hipStream_t st) {
  const dim3 grid(unsigned(pl.n_ib), unsigned(pl.sj));
  const SplitShape jc = pl.split;
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
    case NBODY_MIXED_DS: NBODY_POT(NBODY_MIXED_DS); break;
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
    case NBODY_MIXED_DS:
      diag_block_kernel<NBODY_MIXED_DS><<<nblocks, kThreads, 0, st>>>(
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

hipError_t launch_step_small(int precision, int n, const double *x_in,
                             const double *mass, double eps2, double G,
                             const double *v_in, double *v_out, double *x_out,
                             double *acc_out, double *rec, double h, double dt,
                             unsigned flags, hipStream_t st) {
  const dim3 grid(unsigned((n + kThreads / 64 - 1) / (kThreads / 64)));
  // the kernel stages all n sources in LDS: n must fit its array
#define NBODY_STEP_SMALL(PREC_)                                              \
  if (n > kSmallMax<PREC_>) return hipErrorInvalidValue;                     \
  step_small_kernel<PREC_><<<grid, kThreads, 0, st>>>(                      \
      n, x_in, mass, eps2, G, v_in, v_out, x_out, acc_out, rec, h, dt, flags)
  switch (precision) {
    case NBODY_FP64: NBODY_STEP_SMALL(NBODY_FP64); break;
    case NBODY_MIXED: NBODY_STEP_SMALL(NBODY_MIXED); break;
    case NBODY_MIXED_D64: NBODY_STEP_SMALL(NBODY_MIXED_D64); break;
    case NBODY_MIXED_DS: NBODY_STEP_SMALL(NBODY_MIXED_DS); break;
    default: return hipErrorInvalidValue;
  }
#undef NBODY_STEP_SMALL
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

}  // namespace nbody
