/*
 * FP64 CPU oracle for the all-pairs gravitational N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Every routine is the plain definition (or the plain sequence of steps) of
 * what it computes, in IEEE double precision, compiled with
 * -O2 -fno-fast-math -ffp-contract=off so that no FMA contraction or
 * reassociation changes the arithmetic.  OpenMP splits only the outer loop
 * over target bodies; every target body is computed by one thread with its
 * source loop in ascending order, so results do not depend on the thread
 * count.
 *
 * Layout: component-major structure of arrays, x[3*n] = {x0..x_{n-1},
 * y0..y_{n-1}, z0..z_{n-1}}, mass m[n]; the paper keeps one contiguous 1-D
 * array per coordinate (Numba "arrays with simple data types", section 3.2,
 * and the typed Cython signature, section 3.3).
 *
 * Readings of the paper taken here (the paper gives no values for them):
 *  - the softening constant added to r^2 has units of length^2; it is eps^2
 *    (Plummer softening);
 *  - the source loop includes j == i; with eps > 0 that term is exactly 0
 *    (section 2.3 pseudo-code loops j over all N bodies, and the 20 N^2
 *    flop count of section 4.1 counts it);
 *  - the paper forms the force G m_i m_j d s^-3/2 and divides by m_i; the
 *    acceleration is computed here directly as G sum_j m_j d s^-3/2, which is
 *    the same quantity in exact arithmetic;
 *  - the integrator is kick-drift-kick leapfrog (scheme 0); the update the
 *    paper's listings print -- one half-kick and one drift per step -- is
 *    scheme 1.
 *
 * Parity pins: tests/test_oracle_pins.py checks every function here against
 * closed forms, a 40-digit decimal brute force, an independent whole-matrix
 * NumPy form, invariants and central finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Acceleration of target body i by all n sources (paper section 2.3, the
 * force loop of the section 3.2 / 3.3 listings):
 *   a_i = G sum_j m_j (x_j - x_i) (|x_j - x_i|^2 + eps^2)^(-3/2). */
static void accel_one(int64_t n, const double *x, const double *m, double G,
                      double eps2, const double xi[3], double out[3]) {
  const double *px = x, *py = x + n, *pz = x + 2 * n;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double dx = px[j] - xi[0];
    double dy = py[j] - xi[1];
    double dz = pz[j] - xi[2];
    double s = dx * dx + dy * dy + dz * dz + eps2;
    double inv_s32 = 1.0 / (s * sqrt(s)); /* s^(-3/2) */
    double w = m[j] * inv_s32;
    ax += w * dx;
    ay += w * dy;
    az += w * dz;
  }
  out[0] = G * ax;
  out[1] = G * ay;
  out[2] = G * az;
}

/* All n accelerations: acc[3*n]. */
void oracle_accel(int64_t n, const double *x, const double *m, double G,
                  double eps, double *acc) {
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double xi[3] = {x[i], x[n + i], x[2 * n + i]};
    double a[3];
    accel_one(n, x, m, G, eps2, xi, a);
    acc[i] = a[0];
    acc[n + i] = a[1];
    acc[2 * n + i] = a[2];
  }
}

/* Accelerations of a subset of target rows only: out[3*k], component-major
 * over the k selected rows.  Same arithmetic as oracle_accel. */
void oracle_accel_rows(int64_t n, const double *x, const double *m, double G,
                       double eps, int64_t k, const int64_t *rows,
                       double *out) {
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < k; ++r) {
    int64_t i = rows[r];
    double xi[3] = {x[i], x[n + i], x[2 * n + i]};
    double a[3];
    accel_one(n, x, m, G, eps2, xi, a);
    out[r] = a[0];
    out[k + r] = a[1];
    out[2 * k + r] = a[2];
  }
}

/* Time integration, `steps` steps, state updated in place.
 *  scheme 0, kick-drift-kick leapfrog:
 *    v <- v + (dt/2) a ;  x <- x + dt v ;  a <- A(x) ;  v <- v + (dt/2) a
 *  scheme 1, the update printed in the paper's listings (sections 3.1-3.3):
 *    one half-kick and one drift per step with the force of the step's start,
 *    v <- v + (dt/2) a ;  x <- x + dt v ;  a <- A(x)
 * If acc_valid is 0, acc is first set to A(x).  On return acc = A(x_final).
 * The per-step data dependencies (no body moves before every force is
 * summed; no body starts step t+1 before step t ends) are those stated with
 * the pseudo-code of section 2.3. */
void oracle_step(int64_t n, int64_t steps, double *x, double *v, double *acc,
                 const double *m, double G, double eps, double dt,
                 int acc_valid, int scheme) {
  const double half = 0.5 * dt;
  if (!acc_valid) oracle_accel(n, x, m, G, eps, acc);
  for (int64_t t = 0; t < steps; ++t) {
    for (int64_t q = 0; q < 3 * n; ++q) {
      v[q] = v[q] + half * acc[q];
      x[q] = x[q] + dt * v[q];
    }
    oracle_accel(n, x, m, G, eps, acc);
    if (scheme == 0)
      for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q] + half * acc[q];
  }
}

/* Same integrator, also recording the positions x_0..x_steps into
 * traj[(steps+1)*3*n] (used by the reverse sweep). */
static void step_record(int64_t n, int64_t steps, double *x, double *v,
                        double *acc, const double *m, double G, double eps,
                        double dt, int scheme, double *traj) {
  memcpy(traj, x, (size_t)(3 * n) * sizeof(double));
  oracle_accel(n, x, m, G, eps, acc);
  for (int64_t t = 0; t < steps; ++t) {
    oracle_step(n, 1, x, v, acc, m, G, eps, dt, 1, scheme);
    memcpy(traj + (size_t)(t + 1) * 3 * n, x, (size_t)(3 * n) * sizeof(double));
  }
}

/* Total energy of the softened system:
 *   E = sum_i m_i |v_i|^2 / 2 - G sum_{i<j} m_i m_j (|x_i-x_j|^2+eps^2)^(-1/2),
 * the Plummer-softened potential whose negative gradient is the acceleration
 * above.  out[0] = kinetic, out[1] = potential. */
void oracle_energy(int64_t n, const double *x, const double *v,
                   const double *m, double G, double eps, double *out) {
  const double eps2 = eps * eps;
  const double *px = x, *py = x + n, *pz = x + 2 * n;
  double kin = 0.0, pot = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double vx = v[i], vy = v[n + i], vz = v[2 * n + i];
    kin += 0.5 * m[i] * (vx * vx + vy * vy + vz * vz);
  }
#pragma omp parallel for schedule(static) reduction(+ : pot)
  for (int64_t i = 0; i < n; ++i) {
    double row = 0.0;
    for (int64_t j = i + 1; j < n; ++j) {
      double dx = px[j] - px[i], dy = py[j] - py[i], dz = pz[j] - pz[i];
      double s = dx * dx + dy * dy + dz * dz + eps2;
      row += m[j] / sqrt(s);
    }
    pot += m[i] * row;
  }
  out[0] = kin;
  out[1] = -G * pot;
}

/* Linear momentum sum_i m_i v_i -> out[3]. */
void oracle_momentum(int64_t n, const double *v, const double *m, double *out) {
  double p[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 3; ++c)
    for (int64_t i = 0; i < n; ++i) p[c] += m[i] * v[c * n + i];
  memcpy(out, p, sizeof p);
}

/* Vector-Jacobian product of the acceleration for one output row k.
 * With gbar_i = dL/da_i, e_kj = x_j - x_k, s = |e_kj|^2 + eps^2 and
 * h_kj = m_k gbar_j - m_j gbar_k, differentiating a_i above gives
 *   dL/dm_k = -G sum_j (gbar_j . e_kj) s^(-3/2)
 *   dL/dx_k =  G sum_j [ s^(-3/2) h_kj - 3 s^(-5/2) (e_kj . h_kj) e_kj ].
 * The j == k term is exactly zero (e = 0, h = 0). */
static void vjp_one(int64_t n, const double *x, const double *m,
                    const double *g, double G, double eps2, int64_t k,
                    double gx_out[3], double *gm_out) {
  const double *px = x, *py = x + n, *pz = x + 2 * n;
  const double *gx = g, *gy = g + n, *gz = g + 2 * n;
  const double xk = px[k], yk = py[k], zk = pz[k], mk = m[k];
  const double gxk = gx[k], gyk = gy[k], gzk = gz[k];
  double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double ex = px[j] - xk, ey = py[j] - yk, ez = pz[j] - zk;
    double s = ex * ex + ey * ey + ez * ez + eps2;
    double s32 = 1.0 / (s * sqrt(s)); /* s^(-3/2) */
    double s52 = s32 / s;              /* s^(-5/2) */
    double hx = mk * gx[j] - m[j] * gxk;
    double hy = mk * gy[j] - m[j] * gyk;
    double hz = mk * gz[j] - m[j] * gzk;
    double eh = ex * hx + ey * hy + ez * hz;
    double ge = gx[j] * ex + gy[j] * ey + gz[j] * ez;
    sm += ge * s32;
    sx += s32 * hx - 3.0 * s52 * eh * ex;
    sy += s32 * hy - 3.0 * s52 * eh * ey;
    sz += s32 * hz - 3.0 * s52 * eh * ez;
  }
  gx_out[0] = G * sx;
  gx_out[1] = G * sy;
  gx_out[2] = G * sz;
  *gm_out = -G * sm;
}

/* Full VJP: gpos[3*n] = dL/dx, gmass[n] = dL/dm, given gacc[3*n] = dL/da. */
void oracle_accel_vjp(int64_t n, const double *x, const double *m,
                      const double *gacc, double G, double eps, double *gpos,
                      double *gmass) {
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    double gxk[3], gmk;
    vjp_one(n, x, m, gacc, G, eps2, k, gxk, &gmk);
    gpos[k] = gxk[0];
    gpos[n + k] = gxk[1];
    gpos[2 * n + k] = gxk[2];
    gmass[k] = gmk;
  }
}

/* VJP for a subset of output rows: gpos_rows[3*k] component-major,
 * gmass_rows[k]. */
void oracle_accel_vjp_rows(int64_t n, const double *x, const double *m,
                           const double *gacc, double G, double eps,
                           int64_t k, const int64_t *rows, double *gpos_rows,
                           double *gmass_rows) {
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < k; ++r) {
    double gxk[3], gmk;
    vjp_one(n, x, m, gacc, G, eps2, rows[r], gxk, &gmk);
    gpos_rows[r] = gxk[0];
    gpos_rows[k + r] = gxk[1];
    gpos_rows[2 * k + r] = gxk[2];
    gmass_rows[r] = gmk;
  }
}

/* Reverse sweep of the integrator (the exact adjoint of oracle_step with
 * acc_valid = 0).  It stores every position x_0..x_S (no checkpointing) and
 * walks the steps backwards.  For kick-drift-kick (scheme 0):
 *   abar += (dt/2) vbar                  v_{t+1} = v_{t+1/2} + dt/2 a_{t+1}
 *   (xbar, mbar) += VJP(x_{t+1}; abar)   a_{t+1} = A(x_{t+1}); abar = 0
 *   vbar += dt xbar                      x_{t+1} = x_t + dt v_{t+1/2}
 *   abar  = (dt/2) vbar                  v_{t+1/2} = v_t + dt/2 a_t
 * and for the paper's half-kick + drift (scheme 1) the same without the
 * first line (there is no closing half-kick).  It finishes with
 * (xbar, mbar) += VJP(x_0; abar) for a_0 = A(x_0).
 *
 * Inputs: initial state x0, v0; gx, gv hold dL/dx_S, dL/dv_S on entry and
 * dL/dx_0, dL/dv_0 on return; ga_T (nullable) is dL/da_S; gm receives dL/dm.
 * Returns 0, or -1 if memory could not be allocated. */
int oracle_step_adjoint(int64_t n, int64_t steps, const double *x0,
                        const double *v0, const double *m, double G,
                        double eps, double dt, int scheme, double *gx,
                        double *gv, const double *ga_T, double *gm) {
  const size_t q3 = (size_t)(3 * n);
  double *traj = (double *)malloc((size_t)(steps + 1) * q3 * sizeof(double));
  double *x = (double *)malloc(q3 * sizeof(double));
  double *v = (double *)malloc(q3 * sizeof(double));
  double *a = (double *)malloc(q3 * sizeof(double));
  double *ab = (double *)malloc(q3 * sizeof(double));
  double *dx = (double *)malloc(q3 * sizeof(double));
  double *dm = (double *)malloc((size_t)n * sizeof(double));
  if (!traj || !x || !v || !a || !ab || !dx || !dm) {
    free(traj); free(x); free(v); free(a); free(ab); free(dx); free(dm);
    return -1;
  }
  memcpy(x, x0, q3 * sizeof(double));
  memcpy(v, v0, q3 * sizeof(double));
  step_record(n, steps, x, v, a, m, G, eps, dt, scheme, traj);

  const double half = 0.5 * dt;
  for (size_t q = 0; q < q3; ++q) ab[q] = ga_T ? ga_T[q] : 0.0;
  for (int64_t i = 0; i < n; ++i) gm[i] = 0.0;

  for (int64_t t = steps - 1; t >= 0; --t) {
    if (scheme == 0)
      for (size_t q = 0; q < q3; ++q) ab[q] = ab[q] + half * gv[q];
    oracle_accel_vjp(n, traj + (size_t)(t + 1) * q3, m, ab, G, eps, dx, dm);
    for (size_t q = 0; q < q3; ++q) gx[q] = gx[q] + dx[q];
    for (int64_t i = 0; i < n; ++i) gm[i] = gm[i] + dm[i];
    for (size_t q = 0; q < q3; ++q) gv[q] = gv[q] + dt * gx[q];
    for (size_t q = 0; q < q3; ++q) ab[q] = half * gv[q];
  }
  oracle_accel_vjp(n, traj, m, ab, G, eps, dx, dm);
  for (size_t q = 0; q < q3; ++q) gx[q] = gx[q] + dx[q];
  for (int64_t i = 0; i < n; ++i) gm[i] = gm[i] + dm[i];

  free(traj); free(x); free(v); free(a); free(ab); free(dx); free(dm);
  return 0;
}

/* Number of OpenMP threads the oracle uses (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
