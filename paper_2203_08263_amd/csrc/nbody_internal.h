// Internal interface between the C-ABI host layer (nbody_api.hip) and the
// gfx950 kernels (nbody_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nbody {

// Threads per workgroup of every kernel (4 wave64s) and bodies per LDS tile.
constexpr int kThreads = 256;

// Source ranges of the sj splits of an all-pairs launch: nlong splits of
// llong bodies, then splits of lshort bodies (both multiples of kThreads),
// the last one ending at n.  Uniform splits have nlong = sj.
struct SplitShape {
  int nlong, llong, lshort;
};

// Launch plan of one all-pairs kernel: L lanes share each target body and
// each lane group serves R targets, so a workgroup owns (kThreads/L)*R
// targets; n_ib target blocks; sj source splits shaped by split.  Depends
// only on (kind, precision, nt, n), so a recomputation reproduces every
// partial sum bitwise.
struct Plan {
  int R;
  int L;
  int64_t n_ib;
  int64_t sj;
  SplitShape split;
};

enum KernelKind { kAccel = 0, kVjp = 1, kPotential = 2 };

// Plan for nt target rows against n source bodies; the one-argument form is
// the whole system (nt = n).  Force evaluations of a small system
// (small_system) get one shape, R = 1, L = 64, one source split, so every
// call that evaluates its forces sums in the same order as its one-launch
// step; make_plan_general is the shape search without that rule.
bool small_system(int precision, int64_t n);
// NBODY_MIXED_NF / NBODY_MIXED_NF64 of a small system are evaluated as
// NBODY_MIXED_D64 / NBODY_FP64 (every run near); other precisions unchanged.
int effective_precision(int precision, int64_t n);
Plan make_plan(KernelKind kind, int precision, int64_t n);
Plan make_plan(KernelKind kind, int precision, int64_t nt, int64_t n);
Plan make_plan_general(KernelKind kind, int precision, int64_t nt, int64_t n);

// Targets are bodies row0 .. row0 + nt - 1 of the n-body system (pos is
// [3][n]), sources all n bodies; plan from make_plan(kind, precision, nt, n).
// out + s*split_stride + c*nt + i  <-  scale * sum over source split s of the
// acceleration sum of body row0 + i (without G when scale == 1), c = 0..2.
// boxes: scratch of near_far_box_doubles(pl, kAccel, near64, n, nt) doubles that
// NBODY_MIXED_NF fills with bounding boxes before its kernel (NULL otherwise).
hipError_t launch_accel(const Plan &pl, int precision, int n, int row0, int nt,
                        const double *pos, const double *mass, double *boxes,
                        double eps2, double scale, double *out,
                        size_t split_stride, hipStream_t st);

// Rows as launch_accel, gacc [3][n]:
// out_x + s*stride + c*nt + i <- scale * sum_j [s^-3/2 h - 3 s^-5/2 (e.h) e],
// out_m + s*stride + i        <- -scale * sum_j (gbar_j . e) s^-3/2.
hipError_t launch_vjp(const Plan &pl, int precision, int n, int row0, int nt,
                      const double *pos, const double *mass, const double *gacc,
                      double *boxes, double eps2, double scale, double *out_x,
                      double *out_m, size_t split_stride, hipStream_t st);

// The NBODY_MIXED_NF / NBODY_MIXED_NF64 (near64) forms of launch_accel and
// launch_vjp: fill the box scratch, then run the near / far kernel.
hipError_t launch_accel_nf(const Plan &pl, int n, int row0, int nt,
                           const double *pos, const double *mass,
                           double *boxes, double eps2, double scale,
                           double *out, size_t stride, bool near64,
                           hipStream_t st);
hipError_t launch_vjp_nf(const Plan &pl, int n, int row0, int nt,
                         const double *pos, const double *mass,
                         const double *gacc, double *boxes, double eps2,
                         double scale, double *ox, double *om, size_t stride,
                         bool near64, hipStream_t st);

// Doubles of near / far scratch (bounding boxes, and the dispatch order of
// launches large enough to take one) that an NBODY_MIXED_NF / NF64 launch of
// `kind` with plan pl needs for nt targets against n sources.
size_t near_far_box_doubles(const Plan &pl, KernelKind kind, bool near64,
                            int64_t n, int64_t nt);

// Morton (Z-order) sort: keys holds morton_padded(n) entries, boxes
// ceil(n/256) * 6 doubles, gbox 6; vel / vel_out may both be NULL.
int64_t morton_padded(int64_t n);
hipError_t launch_morton_sort(int n, const double *pos, const double *vel,
                              const double *mass, int64_t *perm,
                              double *pos_out, double *vel_out,
                              double *mass_out, double *boxes, double *gbox,
                              uint64_t *keys, hipStream_t st);

// out_x[c*n+i] = G * sum_s part[s*stride + c*n + i], c < 3; if out_m:
// out_m[i] = G * sum_s part[s*stride + 3*n + i].  Fixed ascending s order.
hipError_t launch_reduce(int n, int sj, const double *part, size_t stride,
                         double G, double *out_x, double *out_m,
                         hipStream_t st);

// Per-body state update of the kick-drift-kick loop (all FP64):
//   a = part ? G * sum_s part[s] : a_in
//   v = v_in;  if (close) v += h a            (closing half-kick)
//   if (rec) rec <- (x_in, v, a)              (checkpoint record, 9n doubles)
//   if (open) { v += h a; x_out = x_in + dt v }  (opening half-kick + drift)
//   v_out = v;  if (acc_out) acc_out = a
enum UpdateFlags { kClose = 1, kOpen = 2 };
hipError_t launch_update(int n, int sj, const double *part, size_t stride,
                         double G, const double *a_in, double *acc_out,
                         const double *x_in, double *x_out, const double *v_in,
                         double *v_out, double h, double dt, double *rec,
                         unsigned flags, hipStream_t st);

// One time step of a small system in a single launch (NBODY_FP64,
// NBODY_MIXED, NBODY_MIXED_D64): a = G * A(x_in) with one wave per target
// and the whole source range in one sum, then update_kernel's per-entry
// update with that a (x_in, x_out distinct buffers).
hipError_t launch_step_small(int precision, int n, const double *x_in,
                             const double *mass, double eps2, double G,
                             const double *v_in, double *v_out, double *x_out,
                             double *acc_out, double *rec, double h, double dt,
                             unsigned flags, hipStream_t st);

// Reverse sweep helpers (all FP64).
//   abar = (gacc_T ? gacc_T : 0) + (add_hv ? h * gvel : 0);  gmass = 0
hipError_t launch_adj_init(int n, const double *gvel, const double *gacc_T,
                           double h, int add_hv, double *abar, double *gmass,
                           hipStream_t st);
//   gpos += G sum_s part_x;  gmass += G sum_s part_m
//   mode kAdjMid:   gvel += dt gpos; abar = h gvel; abar += h gvel
//   mode kAdjLast:  gvel += dt gpos; abar = h gvel
//   mode kAdjFinal: nothing more
enum AdjMode { kAdjMid = 0, kAdjLast = 1, kAdjFinal = 2 };
hipError_t launch_adj_combine(int n, int sj, const double *part, size_t stride,
                              double G, double dt, double h, double *gpos,
                              double *gvel, double *gmass, double *abar,
                              int mode, hipStream_t st);

// Diagnostics.  launch_potential writes split partials of
// phi_i = sum_j m_j (|x_j - x_i|^2 + eps^2)^(-1/2) to out[s*n + i];
// launch_diagnostics reduces them with the O(N) sums into out[9]:
// K, W, momentum (3), sum m x (3), total mass (blocksum: ceil(n/256)*9
// doubles of scratch).
hipError_t launch_potential(const Plan &pl, int precision, int n,
                            const double *pos, const double *mass, double eps2,
                            double *out, hipStream_t st);
hipError_t launch_diagnostics(int precision, int n, int sj,
                              const double *phi_part, const double *pos,
                              const double *vel, const double *mass,
                              double eps2, double G, double *blocksum,
                              double *out, hipStream_t st);

// FP32 state (the paper's single-precision variant): plan from
// make_plan(kAccel, NBODY_MIXED, n).  out + s*stride + c*n + i <- scale *
// FP32 sum over split s; reduce: out = G * sum_s part (ascending s);
// update: the KDK / half-kick + drift state update of update_kernel in FP32,
// in place on x and v (flags kClose / kOpen), no checkpoint record.
hipError_t launch_accel_f32(const Plan &pl, int n, const float *pos,
                            const float *mass, float eps2, float scale,
                            float *out, size_t stride, hipStream_t st);
hipError_t launch_reduce_f32(int n, int sj, const float *part, size_t stride,
                             float G, float *out, hipStream_t st);
hipError_t launch_update_f32(int n, int sj, const float *part, size_t stride,
                             float G, const float *a_in, float *acc_out,
                             float *x, float *v, float h, float dt,
                             unsigned flags, hipStream_t st);

}  // namespace nbody
