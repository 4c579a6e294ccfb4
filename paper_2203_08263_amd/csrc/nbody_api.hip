// C ABI of libnbody_hip.so: argument validation, the launch plans,
// workspace carving, the kick-drift-kick step loop and the checkpointed
// reverse sweep.  All device
// work is enqueued on the caller's stream; nothing here allocates device
// memory or synchronises.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>

#include "../../include/nbody.h"
#include "nbody_internal.h"

using nbody::Plan;

namespace nbody {

// ------------------------------------------------------------ launch plans --

// Small systems are launch-bound: their step loop runs one launch per step
// (the force with one wave per target over all sources, then the update of
// that target), alternating positions between pos and a workspace copy.
// With one wave per target such a launch holds n / 4 workgroups, too few
// waves to hide latency as n grows; measured crossovers against the two-launch
// loop (100 steps, HIP graph): FP64 wins up to n = 2048 (-40 % per step at
// n <= 256, -15 % at 1024, -4 % at 2048); the FP32-pair modes, whose pairs
// are cheaper, up to about n = 512 (-22 % at 256, +2 % at 1024).  Every
// force evaluation of such a system -- nbody_accel, the row-range form, the
// step's first one -- uses the same shape (one wave per target, no source
// split), so all of them sum in one order: A(x) is one function, and a
// rollout run backwards retraces its steps.
bool small_system(int precision, int64_t n) {
  switch (precision) {
    case NBODY_FP64: return n <= 2048;
    case NBODY_MIXED_D64:
    case NBODY_MIXED_DS: return n <= 1024;
    case NBODY_MIXED: return n <= 512;
    default: return false;
  }
}

// The arithmetic a near / far precision stands for in a system of n bodies:
// a small system counts every run as near -- in a launch-bound system the
// split saves nothing and its box pass would add a launch -- which is
// exactly NBODY_MIXED_D64 for NBODY_MIXED_NF and NBODY_FP64 for
// NBODY_MIXED_NF64 (with their small-system shapes and one-launch steps).
int effective_precision(int precision, int64_t n) {
  if (precision == NBODY_MIXED_NF && small_system(NBODY_MIXED_D64, n))
    return NBODY_MIXED_D64;
  if (precision == NBODY_MIXED_NF64 && small_system(NBODY_FP64, n))
    return NBODY_FP64;
  return precision;
}

Plan make_plan(KernelKind kind, int precision, int64_t n) {
  return make_plan(kind, precision, n, n);
}

Plan make_plan(KernelKind kind, int precision, int64_t nt, int64_t n) {
  if (kind == kAccel && small_system(precision, n)) {
    // one wave per target, every source in one sum (the small-system step)
    const int len = int((n + kThreads - 1) / kThreads * kThreads);
    return Plan{1, 64, (nt + kThreads / 64 - 1) / (kThreads / 64), 1,
                SplitShape{1, len, len}};
  }
  return make_plan_general(kind, precision, nt, n);
}

Plan make_plan_general(KernelKind kind, int precision, int64_t nt, int64_t n) {
  // Chosen from launch-shape sweeps on MI355X (all-pairs kernel plus split
  // reduction).  About 8192 workgroups (32 per CU: 8 resident waves per SIMD,
  // several rounds of them), reached with the smallest lanes-per-target L in
  // {1, 4, 16} that needs at most 64 source splits, each at least one
  // 256-body tile long.  Target blocks count the nt target rows, source
  // splits the n source bodies.  Targets per lane R: 2 for the FP64 force, 1
  // for the FP32-pair modes (their pair chain is latency-bound, so more
  // resident waves beat more independent chains per lane).  The FP64 VJP
  // takes R = 1 (its split-form sums, 8 FP64 values per target, would need
  // 162 VGPRs for two targets) unless that needs L = 16 (small systems):
  // there a lane's 16 sources per tile leave too little work between the
  // tile barriers (measured: -12 % at N = 2048, -37 % at 8192), and R = 2
  // with h formed per pair is faster.  NBODY_MIXED_NF64 starts at L = 4: its
  // near runs are FP64 pairs, and the finer target waves and source runs of
  // L = 4 leave fewer pairs near (measured: +21 % forward at N = 65536, +8 %
  // at 262144, equal at 16384; L = 16 is slower for both near / far modes).
  // A VJP source split spans at most 64 tiles (sj raised, to at most 64):
  // shorter workgroups leave a shorter tail when the last round drains
  // (measured at N = 262144, 16 splits of 64 tiles against 8 of 128: -1.3 to
  // -1.6 % for the mixed and near / far VJP, -2.1 % for the forward; 32 of 32:
  // about the same, at twice the partial sums; no change at N = 65536 and
  // below).  The force keeps its 8192-workgroup shape: more splits would
  // more than double the partial sums of large systems, which the
  // allocation-free force call must hold in its fixed static scratch.
  const int64_t target = 8192, max_sj = 64;
  const int64_t ntiles = (n + kThreads - 1) / kThreads;
  const int64_t max_split_tiles = kind == kVjp ? 64 : ntiles;
  auto shape = [&](int R) {
    Plan p{};
    for (int L : {1, 4, 16}) {
      if (precision == NBODY_MIXED_NF64 && L < 4) continue;
      const int64_t per_block = int64_t(kThreads / L) * R;
      p.R = R;
      p.L = L;
      p.n_ib = (nt + per_block - 1) / per_block;
      p.sj = (target + p.n_ib - 1) / p.n_ib;
      if (p.sj <= std::min(max_sj, ntiles)) break;
    }
    return p;
  };
  Plan p;
  if (precision == NBODY_FP64 && kind == kAccel) {
    p = shape(2);
  } else {
    p = shape(1);
    if (precision == NBODY_FP64 && kind == kVjp && p.L == 16) p = shape(2);
  }
  p.sj = std::max<int64_t>(1, std::min({p.sj, ntiles, max_sj}));
  p.sj = std::min(max_sj, std::max(p.sj, (ntiles + max_split_tiles - 1) / max_split_tiles));
  const int64_t tiles_per_split = (ntiles + p.sj - 1) / p.sj;
  p.sj = (ntiles + tiles_per_split - 1) / tiles_per_split;  // none left empty
  const int len = int(tiles_per_split * kThreads);
  p.split = SplitShape{int(p.sj), len, len};
  // Splits of 8 tiles or more: the last quarter of them (at least one) a
  // quarter as long as the others, so the launch's last round holds short
  // workgroups and drains quickly (measured at N = 262144, the mixed force in
  // 8 splits: -4.1 %, where 16 uniform splits gain -2.5 % at twice the
  // partial sums; at N = 65536, 32 splits of 8 tiles: -2.4 %).
  const int64_t two_level_tiles = 8;
  if (tiles_per_split >= two_level_tiles && p.sj >= 2) {
    const int64_t nshort = std::max<int64_t>(1, p.sj / 4), nlong = p.sj - nshort;
    for (int64_t tl = (4 * ntiles + 4 * nlong + nshort - 1) / (4 * nlong + nshort);;
         ++tl) {
      const int64_t ts = std::max<int64_t>(1, tl / 4);
      if (nlong * tl + nshort * ts < ntiles) continue;
      if (nlong * tl + (nshort - 1) * ts < ntiles)  // the last split is not empty
        p.split = SplitShape{int(nlong), int(tl * kThreads), int(ts * kThreads)};
      break;
    }
  }
  return p;
}

}  // namespace nbody

namespace {

thread_local char g_last_error[512] = "";

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char *where) {
  return fail(NBODY_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr size_t kInvalid = (size_t)-1;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// a * b * elem bytes, or kInvalid when that exceeds 2^62 (no size_t wrap).
size_t checked_bytes(int64_t a, int64_t b, int64_t elem) {
  const unsigned __int128 v = (unsigned __int128)a * (unsigned __int128)b *
                              (unsigned __int128)elem;
  return v > ((unsigned __int128)1 << 62) ? kInvalid : size_t(v);
}

bool valid_steps(int64_t steps) { return steps >= 0 && steps <= NBODY_MAX_STEPS; }
size_t dbytes(int64_t count) { return round_up(size_t(count) * sizeof(double)); }

bool valid_precision(int p) {
  return p == NBODY_FP64 || p == NBODY_MIXED || p == NBODY_MIXED_D64 ||
         p == NBODY_MIXED_NF || p == NBODY_MIXED_NF64 || p == NBODY_MIXED_DS;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

int check_common(int64_t n, const nbody_params *p, int precision,
                 bool need_dt, bool vjp = false) {
  if (n < 1 || n > NBODY_MAX_N)
    return fail(NBODY_ERR_INVALID_ARGUMENT, "n = %lld outside [1, %lld]",
                (long long)n, (long long)NBODY_MAX_N);
  if (!p) return fail(NBODY_ERR_INVALID_ARGUMENT, "params pointer is NULL");
  if (!isfinite(p->G))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "G is not finite");
  if (!isfinite(p->eps) || !(p->eps > 0.0))
    return fail(NBODY_ERR_INVALID_ARGUMENT,
                "eps must be finite and > 0 (the j == i term needs it)");
  if (!(p->eps * p->eps > 0.0) || !isfinite(p->eps * p->eps))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "eps^2 underflows or overflows");
  if (need_dt && !isfinite(p->dt))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "dt is not finite");
  if (!valid_precision(precision))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "unknown precision %d", precision);
  // Every precision but NBODY_FP64 evaluates pairs in FP32, the self pair
  // (d = 0) included: its weight m eps^-3 multiplies d = 0, which gives 0 only
  // while eps^2 is a normal FP32 number (not flushed to 0) and eps^-3 is
  // finite in FP32; otherwise every output would be NaN.  The FP32 VJP pair
  // also forms s^-5/2 (e.h) before multiplying by e, which reaches
  // 0.29 eps^-4 (m_k |gbar_j| + m_j |gbar_k|): a larger smallest eps there.
  if (precision != NBODY_FP64) {
    const float e2 = float(p->eps * p->eps);
    const double min_eps = vjp ? NBODY_MIN_EPS_FP32_VJP : NBODY_MIN_EPS_FP32;
    if (!(p->eps >= min_eps) || !isfinite(e2))
      return fail(NBODY_ERR_INVALID_ARGUMENT,
                  "eps = %g outside the FP32 pair range [%g, 1.8e19] of "
                  "precision %d%s",
                  p->eps, min_eps, precision, vjp ? " (VJP)" : "");
  }
  return NBODY_OK;
}

int check_ptr(const void *ptr, const char *name) {
  if (!ptr) return fail(NBODY_ERR_INVALID_ARGUMENT, "%s is NULL", name);
  if (!aligned8(ptr))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "%s is not 8-byte aligned", name);
  return NBODY_OK;
}

int check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (need == 0) return NBODY_OK;
  if (ws_bytes < need)
    return fail(NBODY_ERR_WORKSPACE_TOO_SMALL,
                "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (!ws) return fail(NBODY_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (!aligned8(ws))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "workspace is not 8-byte aligned");
  return NBODY_OK;
}

int64_t num_tiles(int64_t n) { return (n + nbody::kThreads - 1) / nbody::kThreads; }

// Bounding-box scratch of an NBODY_MIXED_NF launch (nt targets, n sources);
// it sits at the start of the workspace of every all-pairs operation, the
// partial sums after it.
size_t nf_bytes(nbody::KernelKind kind, int prec, int64_t n, int64_t nt) {
  if (prec != NBODY_MIXED_NF && prec != NBODY_MIXED_NF64) return 0;
  const Plan pl = nbody::make_plan(kind, prec, nt, n);
  return round_up(nbody::near_far_box_doubles(pl, kind, prec == NBODY_MIXED_NF64,
                                              n, nt) *
                  sizeof(double));
}
size_t box_bytes_fwd(int64_t n, int prec) { return nf_bytes(nbody::kAccel, prec, n, n); }
size_t box_bytes_vjp(int64_t n, int prec) { return nf_bytes(nbody::kVjp, prec, n, n); }

// Workspace sizes of each operation (see the layouts in the entry points).
size_t ws_accel(int64_t n, int prec) {
  const Plan pl = nbody::make_plan(nbody::kAccel, prec, n);
  return box_bytes_fwd(n, prec) + (pl.sj > 1 ? dbytes(pl.sj * 3 * n) : 0);
}
size_t ws_step(int64_t n, int prec) {
  const Plan pl = nbody::make_plan(nbody::kAccel, prec, n);
  return box_bytes_fwd(n, prec) + dbytes(pl.sj * 3 * n) +
         (nbody::small_system(prec, n) ? dbytes(3 * n) : 0);
}
size_t ws_vjp(int64_t n, int prec) {
  const Plan pl = nbody::make_plan(nbody::kVjp, prec, n);
  return box_bytes_vjp(n, prec) + (pl.sj > 1 ? dbytes(pl.sj * 4 * n) : 0);
}
size_t ws_morton(int64_t n) {
  return dbytes(6 * num_tiles(n)) + dbytes(6) +
         round_up(size_t(nbody::morton_padded(n)) * sizeof(uint64_t));
}
size_t ws_diag(int64_t n, int prec) {
  const Plan pl = nbody::make_plan(nbody::kPotential, prec, n);
  return dbytes(pl.sj * n) + dbytes(((n + nbody::kThreads - 1) / nbody::kThreads) * 9);
}
size_t ws_accel_rows(int64_t n, int64_t nt, int prec) {
  if (nt == 0) return 0;
  const Plan pl = nbody::make_plan(nbody::kAccel, prec, nt, n);
  return nf_bytes(nbody::kAccel, prec, n, nt) +
         (pl.sj > 1 ? dbytes(pl.sj * 3 * nt) : 0);
}
size_t ws_vjp_rows(int64_t n, int64_t nt, int prec) {
  if (nt == 0) return 0;
  const Plan pl = nbody::make_plan(nbody::kVjp, prec, nt, n);
  return nf_bytes(nbody::kVjp, prec, n, nt) +
         (pl.sj > 1 ? dbytes(pl.sj * 4 * nt) : 0);
}
size_t box_bytes_adj(int64_t n, int prec) {
  return std::max(box_bytes_fwd(n, prec), box_bytes_vjp(n, prec));
}
size_t ws_part_adjoint(int64_t n, int prec) {
  const Plan pf = nbody::make_plan(nbody::kAccel, prec, n);
  const Plan pv = nbody::make_plan(nbody::kVjp, prec, n);
  return std::max(dbytes(pf.sj * 3 * n), dbytes(pv.sj * 4 * n));
}
size_t ws_adjoint(int64_t n, int64_t steps, int64_t K, int prec) {
  const int64_t seg = std::min<int64_t>(K, std::max<int64_t>(steps, 1));
  const size_t seg_bytes = checked_bytes(seg, 3 * n, sizeof(double));
  if (seg_bytes == kInvalid) return kInvalid;
  // v, a, abar, segment positions, box scratch, partial sums
  return 3 * dbytes(3 * n) + round_up(seg_bytes) + box_bytes_adj(n, prec) +
         ws_part_adjoint(n, prec);
}

int check_rows(int64_t n, int64_t row_begin, int64_t row_count) {
  if (row_begin < 0 || row_count < 0 || row_begin > n ||
      row_count > n - row_begin)
    return fail(NBODY_ERR_INVALID_ARGUMENT,
                "rows [%lld, %lld + %lld) outside [0, n = %lld)",
                (long long)row_begin, (long long)row_begin,
                (long long)row_count, (long long)n);
  return NBODY_OK;
}

// ---- FP32 state
size_t fbytes(int64_t count) { return round_up(size_t(count) * sizeof(float)); }

// The FP32-state kernels take the mixed mode's general plan shapes (they have
// no small-system step).
Plan plan_f32(int64_t n) {
  return nbody::make_plan_general(nbody::kAccel, NBODY_MIXED, n, n);
}

size_t ws_accel_f32(int64_t n) {
  const Plan pl = plan_f32(n);
  return pl.sj > 1 ? fbytes(pl.sj * 3 * n) : 0;
}
size_t ws_step_f32(int64_t n) { return fbytes(plan_f32(n).sj * 3 * n); }

bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int check_fptr(const void *ptr, const char *name) {
  if (!ptr) return fail(NBODY_ERR_INVALID_ARGUMENT, "%s is NULL", name);
  if (!aligned4(ptr))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "%s is not 4-byte aligned", name);
  return NBODY_OK;
}

// The FP64-state checks, plus what FP32 arithmetic needs: G, eps^2 (and dt)
// finite in FP32 and eps^2 not flushed to zero.
int check_f32(int64_t n, const nbody_params *p, bool need_dt) {
  int rc;
  if ((rc = check_common(n, p, NBODY_MIXED, need_dt))) return rc;
  const float G = float(p->G), e2 = float(p->eps * p->eps);
  if (!isfinite(G)) return fail(NBODY_ERR_INVALID_ARGUMENT, "G overflows FP32");
  if (!(e2 > 0.0f) || !isfinite(e2))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "eps^2 is not a positive FP32 value");
  if (need_dt && !isfinite(float(p->dt)))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "dt overflows FP32");
  return NBODY_OK;
}

int64_t num_records(int64_t steps, int64_t K) {
  return std::max<int64_t>(1, (steps + K - 1) / K);
}

// The all-pairs launches (NBODY_MIXED_NF fills its box scratch first).
hipError_t run_accel(const Plan &pl, int prec, int n, int r0, int nt,
                     const double *pos, const double *mass, double *boxes,
                     double eps2, double scale, double *out, size_t stride,
                     hipStream_t st) {
  return nbody::launch_accel(pl, prec, n, r0, nt, pos, mass, boxes, eps2,
                             scale, out, stride, st);
}

hipError_t run_vjp(const Plan &pl, int prec, int n, int r0, int nt,
                   const double *pos, const double *mass, const double *gacc,
                   double *boxes, double eps2, double scale, double *ox,
                   double *om, size_t stride, hipStream_t st) {
  return nbody::launch_vjp(pl, prec, n, r0, nt, pos, mass, gacc, boxes, eps2,
                           scale, ox, om, stride, st);
}

// Workspace carving: box scratch (NBODY_MIXED_NF only, box_bytes long) then
// partial sums.
double *ws_boxes(void *ws) { return static_cast<double *>(ws); }
double *ws_parts(void *ws, size_t box_bytes) {
  return reinterpret_cast<double *>(static_cast<char *>(ws) + box_bytes);
}

// One force evaluation into partial sums (unscaled; G is applied by the
// consumer) -- the form the step loop and the recomputation share.
int accel_to_parts(const Plan &pl, int prec, int n, const double *pos,
                   const double *mass, double *boxes, double eps2,
                   double *part, hipStream_t st) {
  hipError_t e = run_accel(pl, prec, n, 0, n, pos, mass, boxes, eps2, 1.0,
                           part, size_t(3) * n, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "accel kernel launch");
}

// Argument checks of nbody_accel (everything but the workspace).
int check_accel_args(int64_t n, const double *pos, const double *mass,
                     const double *acc, const nbody_params *p, int precision) {
  int rc;
  if ((rc = check_common(n, p, precision, false))) return rc;
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(acc, "acc")))
    return rc;
  return NBODY_OK;
}

// The force evaluation of nbody_accel once its arguments are checked:
// precision is already the effective one and ws holds ws_accel(n, precision)
// bytes.  Box scratch | split partials, then the split reduction (scaled by
// G); a single split writes acc directly.
int accel_enqueue(int64_t n, const double *pos, const double *mass,
                  double *acc, const nbody_params *p, int precision, void *ws,
                  hipStream_t st) {
  const int nn = int(n);
  const double eps2 = p->eps * p->eps;
  const Plan pl = nbody::make_plan(nbody::kAccel, precision, n);
  double *boxes = ws_boxes(ws);
  hipError_t e;
  if (pl.sj == 1) {
    e = run_accel(pl, precision, nn, 0, nn, pos, mass, boxes, eps2, p->G, acc,
                  0, st);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "accel kernel launch");
  }
  double *part = ws_parts(ws, box_bytes_fwd(n, precision));
  int rc;
  if ((rc = accel_to_parts(pl, precision, nn, pos, mass, boxes, eps2, part,
                           st)))
    return rc;
  e = nbody::launch_reduce(nn, int(pl.sj), part, size_t(3) * n, p->G, acc,
                           nullptr, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "reduce kernel launch");
}

// ---- Static scratch of nbody_accel_noalloc (for callers that cannot
// allocate device memory).  The array is zero-initialised device memory of
// the code object: every GPU the library runs this entry point on holds its
// own copy, at its own address, until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address is taken once per device with hipGetSymbolAddress (that device
// current) and only that address is passed to kernels.  Calls on one device
// share the array, so calls that overlap in time on one device (two streams,
// two threads) race; nothing in it has to start at zero (the box scratch and
// the split partials are written in full before they are read).
constexpr size_t kStaticScratchBytes = NBODY_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The device address of the stream's device's copy of `scratch`.
int static_scratch(hipStream_t st, void **out) {
  int cur = -1, dev = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  dev = cur;
  if (st) {
    e = hipStreamGetDevice(st, &dev);
    if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
  }
  if (dev < 0 || dev >= kMaxDevices)
    return fail(NBODY_ERR_UNSUPPORTED, "device %d beyond the %d the static "
                "scratch table covers", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess)
      return hip_fail(e, "hipSetDevice");
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    const hipError_t e2 = dev != cur ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
    if (!ptr) return fail(NBODY_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NBODY_OK;
}

}  // namespace

extern "C" {

const char *nbody_error_string(int code) {
  switch (code) {
    case NBODY_OK: return "success";
    case NBODY_ERR_INVALID_ARGUMENT: return "invalid argument";
    case NBODY_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NBODY_ERR_HIP: return "HIP runtime error";
    case NBODY_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status code";
}

const char *nbody_last_error(void) { return g_last_error; }

size_t nbody_workspace_bytes(int op, int64_t n, int64_t steps,
                             int64_t ckpt_every, int precision) {
  if (n < 1 || n > NBODY_MAX_N || !valid_precision(precision)) return kInvalid;
  precision = nbody::effective_precision(precision, n);
  switch (op) {
    case NBODY_OP_ACCEL: return ws_accel(n, precision);
    case NBODY_OP_STEP: return ws_step(n, precision);
    case NBODY_OP_VJP: return ws_vjp(n, precision);
    case NBODY_OP_STEP_ADJOINT:
      if (!valid_steps(steps) || ckpt_every < 1) return kInvalid;
      return ws_adjoint(n, steps, ckpt_every, precision);
    case NBODY_OP_DIAGNOSTICS: return ws_diag(n, precision);
    case NBODY_OP_MORTON_SORT: return ws_morton(n);
  }
  return kInvalid;
}

size_t nbody_rows_workspace_bytes(int op, int64_t n, int64_t row_count,
                                  int precision) {
  if (n < 1 || n > NBODY_MAX_N || !valid_precision(precision) ||
      row_count < 0 || row_count > n)
    return kInvalid;
  precision = nbody::effective_precision(precision, n);
  switch (op) {
    case NBODY_OP_ACCEL: return ws_accel_rows(n, row_count, precision);
    case NBODY_OP_VJP: return ws_vjp_rows(n, row_count, precision);
  }
  return kInvalid;
}

size_t nbody_checkpoint_bytes(int64_t n, int64_t steps, int64_t ckpt_every) {
  if (n < 1 || n > NBODY_MAX_N || !valid_steps(steps) || ckpt_every < 1)
    return kInvalid;
  return checked_bytes(num_records(steps, ckpt_every), 9 * n, sizeof(double));
}

int nbody_accel(int64_t n, const double *pos, const double *mass, double *acc,
                const nbody_params *p, int precision, void *ws,
                size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_accel_args(n, pos, mass, acc, p, precision))) return rc;
  precision = nbody::effective_precision(precision, n);
  if ((rc = check_ws(ws, ws_bytes, ws_accel(n, precision)))) return rc;
  return accel_enqueue(n, pos, mass, acc, p, precision, ws,
                       static_cast<hipStream_t>(stream));
}

int nbody_accel_noalloc(int64_t n, const double *pos, const double *mass,
                        double *acc, const nbody_params *p, int precision,
                        void *stream) {
  int rc;
  if ((rc = check_accel_args(n, pos, mass, acc, p, precision))) return rc;
  precision = nbody::effective_precision(precision, n);
  const size_t need = ws_accel(n, precision);
  if (need > kStaticScratchBytes)
    return fail(NBODY_ERR_WORKSPACE_TOO_SMALL,
                "n = %lld, precision %d needs %zu bytes of scratch; the "
                "library's static scratch holds %zu (use nbody_accel with a "
                "workspace)",
                (long long)n, precision, need, kStaticScratchBytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  void *ws = nullptr;
  if (need > 0 && (rc = static_scratch(st, &ws))) return rc;
  return accel_enqueue(n, pos, mass, acc, p, precision, ws, st);
}

int nbody_accel_rows(int64_t n, int64_t row_begin, int64_t row_count,
                     const double *pos, const double *mass, double *acc,
                     const nbody_params *p, int precision, void *ws,
                     size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, false))) return rc;
  precision = nbody::effective_precision(precision, n);
  if ((rc = check_rows(n, row_begin, row_count))) return rc;
  if (row_count == 0) return NBODY_OK;
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(acc, "acc")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_accel_rows(n, row_count, precision))))
    return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n), r0 = int(row_begin), nt = int(row_count);
  const double eps2 = p->eps * p->eps;
  const Plan pl = nbody::make_plan(nbody::kAccel, precision, row_count, n);
  double *boxes = ws_boxes(ws);
  hipError_t e;
  if (pl.sj == 1) {
    e = run_accel(pl, precision, nn, r0, nt, pos, mass, boxes, eps2, p->G, acc,
                  0, st);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "accel kernel launch");
  }
  double *part = ws_parts(ws, nf_bytes(nbody::kAccel, precision, n, row_count));
  e = run_accel(pl, precision, nn, r0, nt, pos, mass, boxes, eps2, 1.0, part,
                size_t(3) * nt, st);
  if (e != hipSuccess) return hip_fail(e, "accel kernel launch");
  e = nbody::launch_reduce(nt, int(pl.sj), part, size_t(3) * nt, p->G, acc,
                           nullptr, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "reduce kernel launch");
}

int nbody_accel_vjp_rows(int64_t n, int64_t row_begin, int64_t row_count,
                         const double *pos, const double *mass,
                         const double *gacc, double *gpos, double *gmass,
                         const nbody_params *p, int precision, void *ws,
                         size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, false, true))) return rc;
  precision = nbody::effective_precision(precision, n);
  if ((rc = check_rows(n, row_begin, row_count))) return rc;
  if (row_count == 0) return NBODY_OK;
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(gacc, "gacc")) || (rc = check_ptr(gpos, "gpos")) ||
      (rc = check_ptr(gmass, "gmass")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_vjp_rows(n, row_count, precision))))
    return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n), r0 = int(row_begin), nt = int(row_count);
  const double eps2 = p->eps * p->eps;
  const Plan pl = nbody::make_plan(nbody::kVjp, precision, row_count, n);
  double *boxes = ws_boxes(ws);
  hipError_t e;
  if (pl.sj == 1) {
    e = run_vjp(pl, precision, nn, r0, nt, pos, mass, gacc, boxes, eps2, p->G,
                gpos, gmass, 0, st);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "vjp kernel launch");
  }
  double *part = ws_parts(ws, nf_bytes(nbody::kVjp, precision, n, row_count));
  const size_t stride = size_t(4) * nt;
  e = run_vjp(pl, precision, nn, r0, nt, pos, mass, gacc, boxes, eps2, 1.0,
              part, part + size_t(3) * nt, stride, st);
  if (e != hipSuccess) return hip_fail(e, "vjp kernel launch");
  e = nbody::launch_reduce(nt, int(pl.sj), part, stride, p->G, gpos, gmass,
                           st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "reduce kernel launch");
}

int nbody_step(int64_t n, int64_t steps, double *pos, double *vel,
               double *acc, const double *mass, const nbody_params *p,
               int precision, unsigned flags, double *ckpt,
               int64_t ckpt_every, void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, true))) return rc;
  precision = nbody::effective_precision(precision, n);
  if (!valid_steps(steps))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "steps = %lld outside [0, %lld]",
                (long long)steps, (long long)NBODY_MAX_STEPS);
  if (flags & ~(NBODY_ACC_VALID | NBODY_HALF_KICK_DRIFT))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "unknown flag bits 0x%x",
                flags & ~(NBODY_ACC_VALID | NBODY_HALF_KICK_DRIFT));
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(vel, "vel")) ||
      (rc = check_ptr(acc, "acc")) || (rc = check_ptr(mass, "mass")))
    return rc;
  if (ckpt) {
    if (ckpt_every < 1)
      return fail(NBODY_ERR_INVALID_ARGUMENT,
                  "ckpt_every = %lld < 1 with a checkpoint buffer",
                  (long long)ckpt_every);
    if ((rc = check_ptr(ckpt, "ckpt"))) return rc;
    if (nbody_checkpoint_bytes(n, steps, ckpt_every) == kInvalid)
      return fail(NBODY_ERR_INVALID_ARGUMENT,
                  "checkpoint buffer size overflows (n = %lld, steps = %lld)",
                  (long long)n, (long long)steps);
  }
  if ((rc = check_ws(ws, ws_bytes, ws_step(n, precision)))) return rc;

  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const double eps2 = p->eps * p->eps, G = p->G, dt = p->dt, h = 0.5 * dt;
  const Plan pl = nbody::make_plan(nbody::kAccel, precision, n);
  const size_t stride = size_t(3) * n;
  const size_t rec_len = size_t(9) * n;
  // Workspace layout: boxes | split partials | (small systems) positions.
  double *boxes = ws_boxes(ws);
  double *part = ws_parts(ws, box_bytes_fwd(n, precision));
  const bool small = nbody::small_system(precision, n);
  double *xbuf = small ? reinterpret_cast<double *>(
                             reinterpret_cast<char *>(part) +
                             dbytes(pl.sj * 3 * n))
                       : nullptr;
  hipError_t e;

  // Step 0: a_0 (computed or given), checkpoint record 0, opening half-kick
  // and drift.  The paper's update has no closing half-kick.  On the
  // one-launch path every step reads the positions from one buffer and
  // drifts them into the other; x_1 goes to the buffer that makes x_steps
  // land in pos.
  const bool have_acc = flags & NBODY_ACC_VALID;
  const unsigned close_flag =
      (flags & NBODY_HALF_KICK_DRIFT) ? 0u : unsigned(nbody::kClose);
  double *x_cur = (small && steps % 2 == 0) ? xbuf : pos;
  double *x_next = x_cur == pos ? xbuf : pos;
  if (!have_acc) {
    if ((rc = accel_to_parts(pl, precision, nn, pos, mass, boxes, eps2, part,
                             st)))
      return rc;
  }
  if (!have_acc || ckpt || steps > 0) {
    e = nbody::launch_update(nn, int(pl.sj), have_acc ? nullptr : part, stride,
                             G, acc, have_acc ? nullptr : acc, pos,
                             steps > 0 ? x_cur : pos, vel, vel, h, dt, ckpt,
                             steps > 0 ? unsigned(nbody::kOpen) : 0u, st);
    if (e != hipSuccess) return hip_fail(e, "update kernel launch");
  }
  for (int64_t t = 0; t < steps; ++t) {
    const bool more = t + 1 < steps;
    double *rec = nullptr;
    if (ckpt && more && (t + 1) % ckpt_every == 0)
      rec = ckpt + size_t((t + 1) / ckpt_every) * rec_len;
    const unsigned fl = close_flag | (more ? unsigned(nbody::kOpen) : 0u);
    if (small) {
      e = nbody::launch_step_small(precision, nn, x_cur, mass, eps2, G, vel,
                                   vel, x_next, acc, rec, h, dt, fl, st);
      if (e != hipSuccess) return hip_fail(e, "step kernel launch");
      std::swap(x_cur, x_next);
      continue;
    }
    if ((rc = accel_to_parts(pl, precision, nn, pos, mass, boxes, eps2, part,
                             st)))
      return rc;
    e = nbody::launch_update(nn, int(pl.sj), part, stride, G, nullptr, acc,
                             pos, pos, vel, vel, h, dt, rec, fl, st);
    if (e != hipSuccess) return hip_fail(e, "update kernel launch");
  }
  return NBODY_OK;
}

int nbody_accel_vjp(int64_t n, const double *pos, const double *mass,
                    const double *gacc, double *gpos, double *gmass,
                    const nbody_params *p, int precision, void *ws,
                    size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, false, true))) return rc;
  precision = nbody::effective_precision(precision, n);
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(gacc, "gacc")) || (rc = check_ptr(gpos, "gpos")) ||
      (rc = check_ptr(gmass, "gmass")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_vjp(n, precision)))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const double eps2 = p->eps * p->eps;
  const Plan pl = nbody::make_plan(nbody::kVjp, precision, n);
  double *boxes = ws_boxes(ws);
  hipError_t e;
  if (pl.sj == 1) {
    e = run_vjp(pl, precision, nn, 0, nn, pos, mass, gacc, boxes, eps2, p->G,
                gpos, gmass, 0, st);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "vjp kernel launch");
  }
  double *part = ws_parts(ws, box_bytes_vjp(n, precision));
  const size_t stride = size_t(4) * n;
  e = run_vjp(pl, precision, nn, 0, nn, pos, mass, gacc, boxes, eps2, 1.0, part,
              part + size_t(3) * n, stride, st);
  if (e != hipSuccess) return hip_fail(e, "vjp kernel launch");
  e = nbody::launch_reduce(nn, int(pl.sj), part, stride, p->G, gpos, gmass, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "reduce kernel launch");
}

int nbody_step_adjoint(int64_t n, int64_t steps, int64_t ckpt_every,
                       const double *ckpt, const double *mass,
                       const nbody_params *p, int precision, unsigned flags,
                       double *gpos, double *gvel, const double *gacc_T,
                       double *gmass, void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, true, true))) return rc;
  precision = nbody::effective_precision(precision, n);
  if (flags & ~NBODY_HALF_KICK_DRIFT)
    return fail(NBODY_ERR_INVALID_ARGUMENT, "unknown flag bits 0x%x",
                flags & ~NBODY_HALF_KICK_DRIFT);
  const bool kdk = !(flags & NBODY_HALF_KICK_DRIFT);
  if (!valid_steps(steps))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "steps = %lld outside [0, %lld]",
                (long long)steps, (long long)NBODY_MAX_STEPS);
  if (ckpt_every < 1)
    return fail(NBODY_ERR_INVALID_ARGUMENT, "ckpt_every = %lld < 1",
                (long long)ckpt_every);
  if ((rc = check_ptr(ckpt, "ckpt")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(gpos, "gpos")) || (rc = check_ptr(gvel, "gvel")) ||
      (rc = check_ptr(gmass, "gmass")))
    return rc;
  if (gacc_T && (rc = check_ptr(gacc_T, "gacc_T"))) return rc;
  const size_t ws_need = ws_adjoint(n, steps, ckpt_every, precision);
  if (ws_need == kInvalid || nbody_checkpoint_bytes(n, steps, ckpt_every) == kInvalid)
    return fail(NBODY_ERR_INVALID_ARGUMENT,
                "workspace or checkpoint size overflows (n = %lld, steps = %lld)",
                (long long)n, (long long)steps);
  if ((rc = check_ws(ws, ws_bytes, ws_need))) return rc;

  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const double eps2 = p->eps * p->eps, G = p->G, dt = p->dt, h = 0.5 * dt;
  const Plan pf = nbody::make_plan(nbody::kAccel, precision, n);
  const Plan pv = nbody::make_plan(nbody::kVjp, precision, n);
  const size_t q3 = size_t(3) * n, rec_len = size_t(9) * n;
  const int64_t seg_max = std::min<int64_t>(ckpt_every,
                                            std::max<int64_t>(steps, 1));
  // Workspace layout: v | a | abar | seg[seg_max] positions | tile boxes |
  // partial sums.
  char *w = static_cast<char *>(ws);
  double *v_ws = reinterpret_cast<double *>(w);
  w += dbytes(3 * n);
  double *a_ws = reinterpret_cast<double *>(w);
  w += dbytes(3 * n);
  double *abar = reinterpret_cast<double *>(w);
  w += dbytes(3 * n);
  double *seg = reinterpret_cast<double *>(w);
  w += dbytes(seg_max * 3 * n);
  double *boxes = reinterpret_cast<double *>(w);
  w += box_bytes_adj(n, precision);
  double *part = reinterpret_cast<double *>(w);
  hipError_t e;

  // abar_S = dL/da_S, plus (dt/2) dL/dv_S through the closing half-kick of
  // the last step (kick-drift-kick only).
  e = nbody::launch_adj_init(nn, gvel, gacc_T, h, kdk && steps > 0, abar,
                             gmass, st);
  if (e != hipSuccess) return hip_fail(e, "adjoint init launch");

  const int64_t nrec = num_records(steps, ckpt_every);
  for (int64_t c = (steps > 0 ? nrec - 1 : -1); c >= 0; --c) {
    const int64_t s0 = c * ckpt_every;
    const int64_t k = std::min<int64_t>(ckpt_every, steps - s0);
    const double *rec = ckpt + size_t(c) * rec_len;
    // Recompute x_{s0+1} .. x_{s0+k} from the checkpoint with the forward's
    // own update and force kernels (bitwise the forward trajectory).
    e = nbody::launch_update(nn, int(pf.sj), nullptr, q3, G, rec + 6 * n,
                             nullptr, rec, seg, rec + 3 * n, v_ws, h, dt,
                             nullptr, nbody::kOpen, st);
    if (e != hipSuccess) return hip_fail(e, "update kernel launch");
    const unsigned fl =
        (kdk ? unsigned(nbody::kClose) : 0u) | unsigned(nbody::kOpen);
    for (int64_t t = 1; t < k; ++t) {
      const double *xp = seg + size_t(t - 1) * q3;
      if (nbody::small_system(precision, n)) {
        e = nbody::launch_step_small(precision, nn, xp, mass, eps2, G, v_ws,
                                     v_ws, seg + size_t(t) * q3, a_ws, nullptr,
                                     h, dt, fl, st);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        continue;
      }
      if ((rc = accel_to_parts(pf, precision, nn, xp, mass, boxes, eps2, part,
                               st)))
        return rc;
      e = nbody::launch_update(nn, int(pf.sj), part, q3, G, nullptr, a_ws, xp,
                               seg + size_t(t) * q3, v_ws, v_ws, h, dt,
                               nullptr, fl, st);
      if (e != hipSuccess) return hip_fail(e, "update kernel launch");
    }
    // Reverse sweep over steps s0+k-1 .. s0: VJP at x_{t+1} = seg[t - s0].
    for (int64_t t = s0 + k - 1; t >= s0; --t) {
      const double *xt1 = seg + size_t(t - s0) * q3;
      e = run_vjp(pv, precision, nn, 0, nn, xt1, mass, abar, boxes, eps2, 1.0,
                  part, part + q3, size_t(4) * n, st);
      if (e != hipSuccess) return hip_fail(e, "vjp kernel launch");
      // abar_t = (dt/2) vbar from the opening half-kick of step t, plus the
      // closing half-kick of step t-1 under kick-drift-kick.
      e = nbody::launch_adj_combine(nn, int(pv.sj), part, size_t(4) * n, G, dt,
                                    h, gpos, gvel, gmass, abar,
                                    (kdk && t > 0) ? nbody::kAdjMid
                                                   : nbody::kAdjLast,
                                    st);
      if (e != hipSuccess) return hip_fail(e, "adjoint combine launch");
    }
  }
  // a_0 = A(x_0): final VJP at the initial positions (checkpoint record 0).
  e = run_vjp(pv, precision, nn, 0, nn, ckpt, mass, abar, boxes, eps2, 1.0,
              part, part + q3, size_t(4) * n, st);
  if (e != hipSuccess) return hip_fail(e, "vjp kernel launch");
  e = nbody::launch_adj_combine(nn, int(pv.sj), part, size_t(4) * n, G, dt, h,
                                gpos, gvel, gmass, abar, nbody::kAdjFinal, st);
  if (e != hipSuccess) return hip_fail(e, "adjoint combine launch");
  return NBODY_OK;
}

int nbody_diagnostics(int64_t n, const double *pos, const double *vel,
                      const double *mass, const nbody_params *p, int precision,
                      double *out, void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_common(n, p, precision, false))) return rc;
  precision = nbody::effective_precision(precision, n);
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(vel, "vel")) ||
      (rc = check_ptr(mass, "mass")) || (rc = check_ptr(out, "out")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_diag(n, precision)))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const double eps2 = p->eps * p->eps;
  const Plan pl = nbody::make_plan(nbody::kPotential, precision, n);
  double *phi = static_cast<double *>(ws);
  double *blocksum = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                                dbytes(pl.sj * n));
  hipError_t e = nbody::launch_potential(pl, precision, nn, pos, mass, eps2,
                                         phi, st);
  if (e != hipSuccess) return hip_fail(e, "potential kernel launch");
  e = nbody::launch_diagnostics(precision, nn, int(pl.sj), phi, pos, vel, mass,
                                eps2, p->G, blocksum, out, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "diagnostics launch");
}

int nbody_morton_sort(int64_t n, const double *pos, const double *vel,
                      const double *mass, int64_t *perm, double *pos_out,
                      double *vel_out, double *mass_out, void *ws,
                      size_t ws_bytes, void *stream) {
  int rc;
  if (n < 1 || n > NBODY_MAX_N)
    return fail(NBODY_ERR_INVALID_ARGUMENT, "n = %lld outside [1, %lld]",
                (long long)n, (long long)NBODY_MAX_N);
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) ||
      (rc = check_ptr(perm, "perm")) || (rc = check_ptr(pos_out, "pos_out")) ||
      (rc = check_ptr(mass_out, "mass_out")))
    return rc;
  if ((vel == nullptr) != (vel_out == nullptr))
    return fail(NBODY_ERR_INVALID_ARGUMENT,
                "vel and vel_out must be both NULL or both set");
  if (vel && ((rc = check_ptr(vel, "vel")) || (rc = check_ptr(vel_out, "vel_out"))))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_morton(n)))) return rc;
  // Workspace layout: tile boxes | bounding box | keys.
  char *w = static_cast<char *>(ws);
  double *boxes = reinterpret_cast<double *>(w);
  w += dbytes(6 * num_tiles(n));
  double *gbox = reinterpret_cast<double *>(w);
  w += dbytes(6);
  uint64_t *keys = reinterpret_cast<uint64_t *>(w);
  const hipError_t e = nbody::launch_morton_sort(
      int(n), pos, vel, mass, perm, pos_out, vel_out, mass_out, boxes, gbox,
      keys, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "morton sort launch");
}

size_t nbody_f32_workspace_bytes(int op, int64_t n) {
  if (n < 1 || n > NBODY_MAX_N) return kInvalid;
  switch (op) {
    case NBODY_OP_ACCEL: return ws_accel_f32(n);
    case NBODY_OP_STEP: return ws_step_f32(n);
  }
  return kInvalid;
}

int nbody_accel_f32(int64_t n, const float *pos, const float *mass, float *acc,
                    const nbody_params *p, void *ws, size_t ws_bytes,
                    void *stream) {
  int rc;
  if ((rc = check_f32(n, p, false))) return rc;
  if ((rc = check_fptr(pos, "pos")) || (rc = check_fptr(mass, "mass")) ||
      (rc = check_fptr(acc, "acc")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_accel_f32(n)))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const float eps2 = float(p->eps * p->eps), G = float(p->G);
  const Plan pl = plan_f32(n);
  hipError_t e;
  if (pl.sj == 1) {
    e = nbody::launch_accel_f32(pl, nn, pos, mass, eps2, G, acc, 0, st);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "accel kernel launch");
  }
  float *part = static_cast<float *>(ws);
  e = nbody::launch_accel_f32(pl, nn, pos, mass, eps2, 1.0f, part,
                              size_t(3) * n, st);
  if (e != hipSuccess) return hip_fail(e, "accel kernel launch");
  e = nbody::launch_reduce_f32(nn, int(pl.sj), part, size_t(3) * n, G, acc, st);
  return e == hipSuccess ? NBODY_OK : hip_fail(e, "reduce kernel launch");
}

int nbody_step_f32(int64_t n, int64_t steps, float *pos, float *vel,
                   float *acc, const float *mass, const nbody_params *p,
                   unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_f32(n, p, true))) return rc;
  if (!valid_steps(steps))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "steps = %lld outside [0, %lld]",
                (long long)steps, (long long)NBODY_MAX_STEPS);
  if (flags & ~(NBODY_ACC_VALID | NBODY_HALF_KICK_DRIFT))
    return fail(NBODY_ERR_INVALID_ARGUMENT, "unknown flag bits 0x%x",
                flags & ~(NBODY_ACC_VALID | NBODY_HALF_KICK_DRIFT));
  if ((rc = check_fptr(pos, "pos")) || (rc = check_fptr(vel, "vel")) ||
      (rc = check_fptr(acc, "acc")) || (rc = check_fptr(mass, "mass")))
    return rc;
  if ((rc = check_ws(ws, ws_bytes, ws_step_f32(n)))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nn = int(n);
  const float eps2 = float(p->eps * p->eps), G = float(p->G);
  const float dt = float(p->dt), h = 0.5f * dt;
  const Plan pl = plan_f32(n);
  float *part = static_cast<float *>(ws);
  const size_t stride = size_t(3) * n;
  const bool have_acc = flags & NBODY_ACC_VALID;
  const unsigned close_flag =
      (flags & NBODY_HALF_KICK_DRIFT) ? 0u : unsigned(nbody::kClose);
  hipError_t e;
  if (!have_acc) {
    e = nbody::launch_accel_f32(pl, nn, pos, mass, eps2, 1.0f, part, stride, st);
    if (e != hipSuccess) return hip_fail(e, "accel kernel launch");
  }
  if (!have_acc || steps > 0) {
    e = nbody::launch_update_f32(nn, int(pl.sj), have_acc ? nullptr : part,
                                 stride, G, acc, have_acc ? nullptr : acc, pos,
                                 vel, h, dt,
                                 steps > 0 ? unsigned(nbody::kOpen) : 0u, st);
    if (e != hipSuccess) return hip_fail(e, "update kernel launch");
  }
  for (int64_t t = 0; t < steps; ++t) {
    e = nbody::launch_accel_f32(pl, nn, pos, mass, eps2, 1.0f, part, stride, st);
    if (e != hipSuccess) return hip_fail(e, "accel kernel launch");
    const bool more = t + 1 < steps;
    e = nbody::launch_update_f32(nn, int(pl.sj), part, stride, G, nullptr, acc,
                                 pos, vel, h, dt,
                                 close_flag | (more ? unsigned(nbody::kOpen) : 0u),
                                 st);
    if (e != hipSuccess) return hip_fail(e, "update kernel launch");
  }
  return NBODY_OK;
}

}  // extern "C"
