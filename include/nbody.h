/*
 * nbody.h -- C ABI of the MI355X (gfx950) all-pairs gravitational N-body
 * library libnbody_hip.so.
 *
 * The operation is the direct-summation N-body problem of arxiv 2203.08263,
 * section 2.3 (every body feels the Newtonian pull of every other body; no
 * body moves until all forces of the step are summed, and no body starts the
 * next step before the current one ends), with the force loop of the
 * section 3.2 / 3.3 listings and the 20-flop-per-pair convention of
 * section 4.1.  The paper gives no values for G, the softening or the time
 * step; they are call parameters here.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Layout: structure of arrays, component-major.  A "vector" argument is
 *    one pointer to 3*n doubles {x_0..x_{n-1}, y_0..y_{n-1}, z_0..z_{n-1}}
 *    (the paper keeps one contiguous 1-D array per coordinate, section 3.2
 *    "arrays with simple data types" and the typed signature of section 3.3);
 *    a "scalar" argument is n doubles.  n is the row stride.
 *  - Memory: every array pointer is a DEVICE pointer (hipMalloc'd or from a
 *    torch tensor on the same device), 8-byte aligned, unless the comment
 *    says "host".  The caller owns all buffers, including the workspace and
 *    checkpoint buffers; the library never allocates or frees device memory
 *    and keeps no device state between calls (one exception:
 *    nbody_accel_noalloc's static scratch array).  Input and output arrays of one
 *    call must not overlap unless the comment says "in/out".
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  All work
 *    is enqueued on it and the call returns without synchronising; a fault
 *    inside a kernel surfaces at the caller's next synchronisation.
 *  - Errors: every int-returning call returns an nbody_status.  Argument
 *    errors are detected on the host before anything is enqueued; on any
 *    error nothing has been written.  nbody_last_error() gives a message for
 *    the calling thread's most recent failure.  No call prints, throws or
 *    exits.
 *  - Determinism: no atomics are used; every sum is taken in a fixed order
 *    that depends only on (n, precision) (and the row count, for the
 *    row-range calls).  Repeated calls with the same inputs give bitwise
 *    identical results.
 *  - Interactions: one force evaluation visits all n*n ordered pairs,
 *    including j == i, whose contribution is exactly zero since eps > 0.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Physical constants of a call.  eps is the Plummer softening length: eps^2
 * is added to |x_j - x_i|^2 (the paper's softening constant, added to the
 * squared distance in the section 3.1-3.3 force loops).  dt is the time step
 * (ignored by nbody_accel / nbody_accel_vjp).  Passed by host pointer. */
typedef struct nbody_params {
  double G;
  double eps;
  double dt;
} nbody_params;

/* Arithmetic of the pair force.  State, accumulation across source tiles,
 * the integrator and every output are FP64 in every precision.
 *  NBODY_FP64       every operation in FP64.
 *  NBODY_MIXED      positions and masses rounded to FP32; pair difference,
 *                   r^2 + eps^2, reciprocal square root, cube and the
 *                   multiply-adds in FP32; FP32 partial sums over chunks of
 *                   32 sources are added into FP64 per-body accumulators.
 *  NBODY_MIXED_D64  as NBODY_MIXED, but the coordinate difference x_j - x_i
 *                   is taken in FP64 and rounded once to FP32, removing the
 *                   error of rounding each position to FP32 first.
 *  NBODY_MIXED_NF   near / far: for each run of sources one FP32 chunk sum
 *                   covers and each wave of targets, a run whose bounding
 *                   box is farther from the wave's targets' box than half the
 *                   half-diagonal b of the workgroup's target box uses
 *                   coordinates relative to that box's centre c (x - c in
 *                   FP64, rounded once to FP32) with the NBODY_MIXED
 *                   arithmetic; every other run uses the NBODY_MIXED_D64
 *                   arithmetic.  Coordinate error per pair below
 *                   6 u32 |x_j - x_i| (u32 = 2^-24).  Close to NBODY_MIXED
 *                   speed when the bodies are in a spatial order
 *                   (nbody_morton_sort); in a random order every run is near
 *                   and results are bitwise those of NBODY_MIXED_D64.
 *                   A system of at most 1024 bodies counts every run as
 *                   near: it is evaluated exactly as NBODY_MIXED_D64.
 *                   nbody_diagnostics evaluates W as NBODY_MIXED_D64.
 *  NBODY_MIXED_NF64 as NBODY_MIXED_NF, but near runs use the FP64 pair and add
 *                   it straight into the FP64 sums, so close pairs -- whose
 *                   FP32 rounding dominates the mixed modes' error when
 *                   forces nearly cancel -- carry FP64 error only; the
 *                   forward's runs and FP32 chunk sums span 16 sources per
 *                   lane instead of 32.  In a
 *                   random order every run is near and the arithmetic is
 *                   FP64 throughout; a system of at most 2048 bodies is
 *                   evaluated exactly as NBODY_FP64.  nbody_diagnostics
 *                   evaluates W in FP64.
 *  NBODY_MIXED_DS   as NBODY_MIXED, but every coordinate v is carried as two
 *                   FP32 numbers, hi = fl32(v) and lo = fl32(v - hi), and
 *                   the pair difference is (x_j^hi - x_i^hi) +
 *                   (x_j^lo - x_i^lo) in FP32 (the first difference is exact
 *                   for close pairs): coordinate error per pair at most
 *                   about 2 u32 |x_j - x_i| + 4 u32^2 (|x_i| + |x_j|), with
 *                   no FP64 operation in the pair (the two-float reading of
 *                   the paper's float32 / float64 comparison, section 4).
 * Every force evaluation of a small system (NBODY_FP64 up to 2048 bodies,
 * NBODY_MIXED_D64 and NBODY_MIXED_DS up to 1024, NBODY_MIXED up to 512) sums
 * in one order, whether it comes from nbody_accel, the row-range form or
 * nbody_step, whose loop then takes one launch per step. */
enum nbody_precision {
  NBODY_FP64 = 0,
  NBODY_MIXED = 1,
  NBODY_MIXED_D64 = 2,
  NBODY_MIXED_NF = 3,
  NBODY_MIXED_NF64 = 4,
  NBODY_MIXED_DS = 5
};

enum nbody_status {
  NBODY_OK = 0,
  NBODY_ERR_INVALID_ARGUMENT = 1,
  NBODY_ERR_WORKSPACE_TOO_SMALL = 2,
  NBODY_ERR_HIP = 3,
  NBODY_ERR_UNSUPPORTED = 4
};

/* nbody_step flag: `acc` already holds A(pos), skip the initial evaluation.
 * Chaining nbody_step(a steps) then nbody_step(b steps, NBODY_ACC_VALID) is
 * bitwise identical to nbody_step(a + b steps). */
#define NBODY_ACC_VALID 1u

/* nbody_step / nbody_step_adjoint flag: integrate with the update the
 * paper's listings print (sections 3.1-3.3) instead of kick-drift-kick: one
 * half-kick and one drift per step with the force of the step's start,
 *     v += (dt/2) a;  x += dt v;  a = A(x)
 * (no closing half-kick; it is symplectic Euler for half the force). */
#define NBODY_HALF_KICK_DRIFT 2u

/* Operation selector for nbody_workspace_bytes. */
enum nbody_op {
  NBODY_OP_ACCEL = 0,
  NBODY_OP_STEP = 1,
  NBODY_OP_VJP = 2,
  NBODY_OP_STEP_ADJOINT = 3,
  NBODY_OP_DIAGNOSTICS = 4,
  NBODY_OP_MORTON_SORT = 5
};

/* Smallest softening length accepted by every precision other than
 * NBODY_FP64 (2^-42): their FP32 pair arithmetic evaluates the self pair with
 * weight m eps^-3, so eps^2 must be a normal FP32 number and eps^-3 finite in
 * FP32.  The masses must also keep m_j * eps^-3 below FLT_MAX (3.4e38), which
 * the library cannot check on the host (masses live in device memory). */
#define NBODY_MIN_EPS_FP32 (0x1p-42)

/* Smallest softening length the VJP calls (nbody_accel_vjp,
 * nbody_accel_vjp_rows, nbody_step_adjoint) accept in every precision other
 * than NBODY_FP64 (2^-32).  Their FP32 pair keeps the weight
 * s^(-5/2) (e.h) of the e term apart from e, and over all pair distances
 * that weight reaches 0.29 eps^-4 H with H = m_k |gbar_j| + m_j |gbar_k|:
 * 2^-32 keeps it finite for H up to about 3.5 (the data-dependent part, H,
 * is again the caller's to keep in range). */
#define NBODY_MIN_EPS_FP32_VJP (0x1p-32)

/* Largest supported body count. */
#define NBODY_MAX_N ((int64_t)1 << 28)

/* Largest supported step count of one nbody_step / nbody_step_adjoint call
 * (larger counts, and checkpoint or workspace sizes beyond 2^62 bytes, are
 * rejected as INVALID_ARGUMENT rather than overflowing a size). */
#define NBODY_MAX_STEPS ((int64_t)1 << 40)

/* Workspace (device scratch) bytes that `op` needs for these arguments; 0 if
 * none is needed, and (size_t)-1 if the arguments are invalid.  steps and
 * ckpt_every only matter for NBODY_OP_STEP_ADJOINT. */
size_t nbody_workspace_bytes(int op, int64_t n, int64_t steps,
                             int64_t ckpt_every, int precision);

/* Bytes of the checkpoint buffer nbody_step fills and nbody_step_adjoint
 * reads: max(1, ceil(steps / ckpt_every)) records of 9*n doubles, record c
 * holding x, v, a (three vectors) at step c*ckpt_every.  (size_t)-1 if the
 * arguments are invalid. */
size_t nbody_checkpoint_bytes(int64_t n, int64_t steps, int64_t ckpt_every);

/* All-pairs softened acceleration (section 2.3; force loop of sections
 * 3.1-3.3):
 *     a_i = G * sum_{j=0}^{n-1} m_j (x_j - x_i) (|x_j - x_i|^2 + eps^2)^(-3/2)
 *  pos  [vector] in    body positions
 *  mass [scalar] in    body masses
 *  acc  [vector] out   accelerations
 *  p    host     in    G (finite), eps (finite, > 0); dt unused
 *  ws   device   scratch of ws_bytes >= nbody_workspace_bytes(NBODY_OP_ACCEL)
 *                (may be NULL when that is 0)
 * Errors: INVALID_ARGUMENT (n outside [1, NBODY_MAX_N], NULL pointer,
 * non-finite G/eps, eps <= 0, eps < NBODY_MIN_EPS_FP32 or FP32 eps^2 infinite
 * for a precision other than NBODY_FP64, unknown precision, misaligned
 * pointer), WORKSPACE_TOO_SMALL, HIP (launch failure; see nbody_last_error). */
int nbody_accel(int64_t n, const double *pos, const double *mass, double *acc,
                const nbody_params *p, int precision, void *ws,
                size_t ws_bytes, void *stream);

/* nbody_accel without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels, launch plan and
 * result -- bitwise -- as nbody_accel, with the split partial sums and the
 * near / far box scratch in a static array of NBODY_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that the library holds on every device it runs this call on until
 * the process ends (its device address is looked up once per device, on the
 * first call there).  The call allocates and frees nothing.  All calls on one
 * device share that array: calls that overlap in time on one device (two
 * streams, two host threads) race and must be serialised by the caller.
 * Arguments as nbody_accel, minus the workspace; `stream`'s device (the
 * current device for NULL) selects the array.
 * Errors: as nbody_accel; WORKSPACE_TOO_SMALL, before anything is enqueued,
 * when nbody_workspace_bytes(NBODY_OP_ACCEL, n, 0, 1, precision) exceeds
 * NBODY_NOALLOC_SCRATCH_BYTES.  Every n below 932068 fits for NBODY_MIXED,
 * NBODY_MIXED_D64 and NBODY_MIXED_DS, below 681198 for NBODY_MIXED_NF, below
 * 14658561 for NBODY_MIXED_NF64 and below 65025 for NBODY_FP64 (larger n
 * only where that workspace happens to fit).  UNSUPPORTED for a device index
 * of 64 or more. */
#define NBODY_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int nbody_accel_noalloc(int64_t n, const double *pos, const double *mass,
                        double *acc, const nbody_params *p, int precision,
                        void *stream);

/* `steps` kick-drift-kick leapfrog steps, in place (the paper's step loop of
 * section 2.3 with its two dependencies; the integrator is KDK):
 *     v += (dt/2) a;  x += dt v;  a = A(x);  v += (dt/2) a
 * one force evaluation per step.
 *  pos  [vector] in/out  positions x_0 -> x_steps
 *  vel  [vector] in/out  velocities v_0 -> v_steps
 *  acc  [vector] in/out  in: A(x_0) if flags has NBODY_ACC_VALID (otherwise
 *                        ignored and computed first); out: A(x_steps)
 *  mass [scalar] in
 *  p    host     in      G, eps as nbody_accel; dt finite
 *  flags                 0, NBODY_ACC_VALID, NBODY_HALF_KICK_DRIFT or both
 *  ckpt device   out     nullable.  If given, ckpt_every >= 1 and it must
 *                        hold nbody_checkpoint_bytes(n, steps, ckpt_every)
 *                        bytes; record c receives (x, v, a) at step
 *                        c*ckpt_every, as nbody_step_adjoint needs them.
 *  ws   device           >= nbody_workspace_bytes(NBODY_OP_STEP)
 * steps == 0 is a no-op that still fills acc when NBODY_ACC_VALID is absent.
 * Errors: as nbody_accel, plus steps < 0, ckpt_every < 1 with ckpt, unknown
 * flag bits, non-finite dt. */
int nbody_step(int64_t n, int64_t steps, double *pos, double *vel,
               double *acc, const double *mass, const nbody_params *p,
               int precision, unsigned flags, double *ckpt,
               int64_t ckpt_every, void *ws, size_t ws_bytes, void *stream);

/* Vector-Jacobian product of nbody_accel (the exact derivative of the
 * section 2.3 force sum; the paper itself has no derivative).  Given
 * gbar = dL/da, with e_kj = x_j - x_k, s = |e_kj|^2 + eps^2 and
 * h_kj = m_k gbar_j - m_j gbar_k:
 *     dL/dm_k = -G sum_j (gbar_j . e_kj) s^(-3/2)
 *     dL/dx_k =  G sum_j [ s^(-3/2) h_kj - 3 s^(-5/2) (e_kj . h_kj) e_kj ]
 * Each output row k is owned by one thread (no scatter).
 *  pos, mass     in    as nbody_accel
 *  gacc [vector] in    dL/da
 *  gpos [vector] out   dL/dx (overwritten, not accumulated)
 *  gmass[scalar] out   dL/dm (overwritten)
 *  ws            >= nbody_workspace_bytes(NBODY_OP_VJP)
 * Errors: as nbody_accel, with NBODY_MIN_EPS_FP32_VJP in place of
 * NBODY_MIN_EPS_FP32. */
int nbody_accel_vjp(int64_t n, const double *pos, const double *mass,
                    const double *gacc, double *gpos, double *gmass,
                    const nbody_params *p, int precision, void *ws,
                    size_t ws_bytes, void *stream);

/* Reverse sweep of nbody_step (called without NBODY_ACC_VALID, or with a
 * valid acc = A(x_0)): gradients of L(x_S, v_S, a_S) with respect to x_0,
 * v_0 and the masses.  Uses the checkpoints nbody_step wrote with the same
 * n, steps, ckpt_every, p, precision and integrator flag; each segment of
 * ckpt_every steps is recomputed from its checkpoint with the forward's own
 * kernels (bitwise the same trajectory), then walked backwards:
 *     abar += (dt/2) vbar;  (xbar, mbar) += VJP(x_{t+1}; abar);
 *     vbar += dt xbar;      abar = (dt/2) vbar
 * ending with (xbar, mbar) += VJP(x_0; abar).  With NBODY_HALF_KICK_DRIFT
 * the first update is absent (no closing half-kick).
 *  ckpt  device in     checkpoint buffer from nbody_step
 *  mass  [scalar] in
 *  gpos  [vector] in/out  in: dL/dx_S   out: dL/dx_0
 *  gvel  [vector] in/out  in: dL/dv_S   out: dL/dv_0
 *  gacc_T[vector] in      nullable: dL/da_S (taken as 0 when NULL)
 *  gmass [scalar] out     dL/dm (overwritten)
 *  ws             >= nbody_workspace_bytes(NBODY_OP_STEP_ADJOINT, n, steps,
 *                    ckpt_every, precision)
 *  flags          0 or NBODY_HALF_KICK_DRIFT (as given to nbody_step)
 * steps == 0 gives gpos += VJP_x(x_0; gacc_T), gmass = VJP_m(x_0; gacc_T)
 * (gvel unchanged), reading x_0 from checkpoint record 0.
 * Errors: as nbody_step, with NBODY_MIN_EPS_FP32_VJP in place of
 * NBODY_MIN_EPS_FP32; ckpt_every must be >= 1. */
int nbody_step_adjoint(int64_t n, int64_t steps, int64_t ckpt_every,
                       const double *ckpt, const double *mass,
                       const nbody_params *p, int precision, unsigned flags,
                       double *gpos, double *gvel, const double *gacc_T,
                       double *gmass, void *ws, size_t ws_bytes, void *stream);

/* Conserved quantities of the softened system, a diagnostic for energy
 * drift and momentum conservation along a rollout (the energy whose negative
 * gradient is the section 2.3 force):
 *  out [device, 9 doubles, written]:
 *    out[0] K = sum_i m_i |v_i|^2 / 2
 *    out[1] W = -G sum_{i<j} m_i m_j (|x_i - x_j|^2 + eps^2)^(-1/2)
 *    out[2..4] sum_i m_i v_i      out[5..7] sum_i m_i x_i     out[8] sum_i m_i
 *  pos, vel [vector] in; mass [scalar] in; p: G, eps as nbody_accel
 *  precision  pair arithmetic of W as in nbody_accel (FP32 partial sums over
 *             chunks of 32 sources in the mixed modes); every other sum is
 *             FP64.  All sums are taken in a fixed order (no atomics).
 *  ws >= nbody_workspace_bytes(NBODY_OP_DIAGNOSTICS)
 * Errors: as nbody_accel. */
int nbody_diagnostics(int64_t n, const double *pos, const double *vel,
                      const double *mass, const nbody_params *p, int precision,
                      double *out, void *ws, size_t ws_bytes, void *stream);

/* Row ranges.  The force sum and its VJP for the target bodies
 * row_begin .. row_begin + row_count - 1 of an n-body system, against all n
 * sources: the share of one device when the target rows of the section 2.3
 * sum are divided among devices that each hold every body's position and
 * mass (and dL/da).  Outputs have row_count rows: a "row vector" is 3 *
 * row_count doubles, component-major with stride row_count, and a "row
 * scalar" row_count doubles; output row r belongs to body row_begin + r.
 * With row_begin = 0 and row_count = n the results are bitwise those of
 * nbody_accel / nbody_accel_vjp.  row_count == 0 is a valid no-op: nothing
 * is enqueued and the array pointers are not examined.
 *
 * Workspace bytes for op NBODY_OP_ACCEL or NBODY_OP_VJP on row_count target
 * rows; (size_t)-1 for any other op or invalid arguments. */
size_t nbody_rows_workspace_bytes(int op, int64_t n, int64_t row_count,
                                  int precision);

/* a_i (as nbody_accel) for i = row_begin .. row_begin + row_count - 1.
 *  pos  [vector] in   all n positions;  mass [scalar] in  all n masses
 *  acc  [row vector] out
 *  ws   >= nbody_rows_workspace_bytes(NBODY_OP_ACCEL, n, row_count, precision)
 * Errors: as nbody_accel, plus row_begin < 0, row_count < 0 or
 * row_begin + row_count > n. */
int nbody_accel_rows(int64_t n, int64_t row_begin, int64_t row_count,
                     const double *pos, const double *mass, double *acc,
                     const nbody_params *p, int precision, void *ws,
                     size_t ws_bytes, void *stream);

/* dL/dx_k and dL/dm_k (as nbody_accel_vjp) for k = row_begin .. row_begin +
 * row_count - 1; every source j contributes through gbar_j and gbar_k.
 *  pos, mass [all n] in;  gacc [vector] in  dL/da of all n bodies
 *  gpos [row vector] out;  gmass [row scalar] out
 *  ws   >= nbody_rows_workspace_bytes(NBODY_OP_VJP, n, row_count, precision)
 * Errors: as nbody_accel_rows, with NBODY_MIN_EPS_FP32_VJP in place of
 * NBODY_MIN_EPS_FP32. */
int nbody_accel_vjp_rows(int64_t n, int64_t row_begin, int64_t row_count,
                         const double *pos, const double *mass,
                         const double *gacc, double *gpos, double *gmass,
                         const nbody_params *p, int precision, void *ws,
                         size_t ws_bytes, void *stream);

/* Spatial order for NBODY_MIXED_NF (the GPU counterpart of the paper's data
 * locality concern, section 3.3: bodies that interact strongly sit in the
 * same tiles).  Sorts the bodies by the Morton (Z-order) code of their
 * positions on a 1024^3 grid spanning the cube [lo, lo + ext]^3 (lo the
 * componentwise minimum, ext the largest extent of the bounding box):
 *     q_c = min(1023, floor((x_c - lo_c) * (1024 / ext)))   (FP64)
 * with the bits of q_x, q_y, q_z interleaved from the most significant
 * down (x first); equal codes keep their original order (stable sort).
 *  pos, mass [vector / scalar] in;  vel [vector] in, nullable
 *  perm     [n int64] out  perm[r] = original index of sorted body r
 *  pos_out, mass_out out   pos_out[:, r] = pos[:, perm[r]], likewise mass
 *  vel_out  [vector] out   NULL exactly when vel is NULL
 *  ws       >= nbody_workspace_bytes(NBODY_OP_MORTON_SORT, n, 0, 1, any
 *              precision): tile boxes, the bounding box and 2^ceil(log2 n)
 *              64-bit keys
 * Outputs must not overlap the inputs.  Not on the per-step path: a rollout
 * re-sorts as often as its bodies mix (every call permutes the state, so the
 * caller keeps perm to map results back).
 * Errors: INVALID_ARGUMENT (n, NULL or misaligned pointers, vel / vel_out
 * not both NULL or both set), WORKSPACE_TOO_SMALL, HIP. */
int nbody_morton_sort(int64_t n, const double *pos, const double *vel,
                      const double *mass, int64_t *perm, double *pos_out,
                      double *vel_out, double *mass_out, void *ws,
                      size_t ws_bytes, void *stream);

/* Single-precision state: the paper's float32 variant (its FP32 runs of the
 * section 3 listings; section 4 reports them next to FP64).  Positions,
 * velocities, masses and accelerations are FP32 arrays ("f32 vector" = 3*n
 * floats, component-major; "f32 scalar" = n floats, 4-byte aligned) and
 * every operation is FP32, including the sum over sources (no FP64
 * accumulation: results carry FP32 summation error over n terms).  Same
 * launch plan, determinism and error rules as the FP64-state calls; there is
 * no VJP / adjoint for this state type.
 *
 * Workspace bytes for op NBODY_OP_ACCEL or NBODY_OP_STEP; (size_t)-1 for any
 * other op or invalid n. */
size_t nbody_f32_workspace_bytes(int op, int64_t n);

/* a_i = G sum_j m_j (x_j - x_i) (|x_j - x_i|^2 + eps^2)^(-3/2), all in FP32.
 *  pos  [f32 vector] in;  mass [f32 scalar] in;  acc [f32 vector] out
 *  p    host: G, eps as nbody_accel; G and eps^2 must also be finite and
 *       eps^2 nonzero in FP32
 * Errors: as nbody_accel. */
int nbody_accel_f32(int64_t n, const float *pos, const float *mass, float *acc,
                    const nbody_params *p, void *ws, size_t ws_bytes,
                    void *stream);

/* `steps` steps in place, all in FP32: kick-drift-kick, or the paper's
 * half-kick + drift with NBODY_HALF_KICK_DRIFT (as nbody_step).
 *  pos, vel [f32 vector] in/out;  acc [f32 vector] in (NBODY_ACC_VALID) /
 *  out A(x_steps);  mass [f32 scalar] in
 *  flags 0, NBODY_ACC_VALID, NBODY_HALF_KICK_DRIFT or both; no checkpoints
 *  ws >= nbody_f32_workspace_bytes(NBODY_OP_STEP, n)
 * Chaining is bitwise as for nbody_step.  Errors: as nbody_step. */
int nbody_step_f32(int64_t n, int64_t steps, float *pos, float *vel,
                   float *acc, const float *mass, const nbody_params *p,
                   unsigned flags, void *ws, size_t ws_bytes, void *stream);

/* Static description of a status code (never NULL). */
const char *nbody_error_string(int code);

/* Message for the calling thread's most recent failing call ("" if none). */
const char *nbody_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
