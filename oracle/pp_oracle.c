/*
 * pp_oracle.c -- plain FP64 CPU oracle for the electrostatic particle-particle
 * (PP) model of arXiv 2502.10640 ("Comparison between electrostatic PP and PIC
 * simulations on electron bunch expansion").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the package smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or constant with the HIP library.
 *
 * What it computes, each function citing the passage it follows:
 *   oracle_field  -- the direct field sum of Eq. (B) (Coulomb's law Eq. (A)
 *                    summed over all j != i), with Plummer softening eps
 *                    (eps = 0 gives Eq. (B) exactly), the matching potential
 *                    and, for error metrics, the sums of the magnitudes of the
 *                    field's and of the potential's terms.
 *   oracle_vv     -- the Velocity Verlet integrator of Eqs. (G) and (H), with
 *                    the acceleration a = (q/m) E of Eqs. (D)/(F).
 *   oracle_diag   -- energies, momentum, centre of mass and the beam moments
 *                    of Sec. 2.2 / 3.2: emittance Eq. (I), <x^2>^(1/2), x_max,
 *                    <v_x^2>^(1/2), v_x,max.
 *
 * Precision and build: IEEE FP64, round to nearest, no fast-math, no FMA
 * contraction (-ffp-contract=off).  Every per-particle sum over j uses
 * Neumaier's compensated summation so that the oracle is the more accurate
 * side of any comparison.  OpenMP parallelises over the receiving particle i
 * only; each i's sum runs over j in index order, so results do not depend on
 * the thread count.
 *
 * Units are SI.  Per particle: position r, velocity v, real-particle charge q
 * and mass m.  One bunch shares one macro-particle weight w (Sec. 2.1): the
 * macro charge is Q = q w and the macro mass is M = m w.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Coulomb constant 1/(4 pi eps0), CODATA 2018 vacuum permittivity. */
#define ORACLE_EPS0 8.8541878128e-12
#define ORACLE_PI 3.14159265358979323846

static double coulomb_k(void) { return 1.0 / (4.0 * ORACLE_PI * ORACLE_EPS0); }

/* Neumaier compensated accumulation: *s holds the running sum, *c the
 * accumulated rounding error; the value of the sum is *s + *c. */
static void neumaier_add(double *s, double *c, double v) {
  double t = *s + v;
  if (fabs(*s) >= fabs(v))
    *c += (*s - t) + v;
  else
    *c += (v - t) + *s;
  *s = t;
}

/*
 * Field of one bunch at a set of receiving particles (Sec. 2.1, Eq. (B) with
 * Plummer softening):
 *   E_i   = k sum_{j != i} (w q_j) (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^(3/2)
 *   phi_i = k sum_{j != i} (w q_j) / (|r_i - r_j|^2 + eps^2)^(1/2)
 *   A_i   = k sum_{j != i} |w q_j| |r_i - r_j| / (|r_i - r_j|^2 + eps^2)^(3/2)
 *   P_i   = k sum_{j != i} |w q_j| / (|r_i - r_j|^2 + eps^2)^(1/2)
 * A_i is the sum of the magnitudes of the terms of E_i and P_i that of the
 * terms of phi_i: what the sums had to cancel, the scale of a per-particle
 * error.  The separation vector is r_ij = r_i - r_j as Eq. (A) defines it, so like
 * charges repel.  The self term j = i is excluded by index, as the sum in
 * Eq. (B) states, whatever eps is.
 *
 * n           particles in the bunch (all of them act as sources j)
 * x,y,z,q     source positions [m] and real-particle charges [C], length n
 * w, eps      macro weight and softening length [m]
 * n_recv      number of receivers; recv = NULL means receivers 0..n-1
 *             (then n_recv must equal n), else recv[k] is the index of the
 *             k-th receiver
 * ex,ey,ez    out, length n_recv [V/m]
 * phi, amag, pmag   out, length n_recv, may be NULL
 */
void oracle_field(int64_t n, const double *x, const double *y, const double *z,
                  const double *q, double w, double eps, int64_t n_recv,
                  const int64_t *recv, double *ex, double *ey, double *ez,
                  double *phi, double *amag, double *pmag) {
  const double k = coulomb_k();
  const double eps2 = eps * eps;
  int64_t r;
#pragma omp parallel for schedule(dynamic, 8)
  for (r = 0; r < n_recv; ++r) {
    const int64_t i = recv ? recv[r] : r;
    double sx = 0, cx = 0, sy = 0, cy = 0, sz = 0, cz = 0;
    double sp = 0, cp = 0, sa = 0, ca = 0, sb = 0, cb = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = x[i] - x[j];
      const double dy = y[i] - y[j];
      const double dz = z[i] - z[j];
      const double d2 = dx * dx + dy * dy + dz * dz;
      const double s2 = d2 + eps2;
      const double inv = 1.0 / sqrt(s2);     /* (|r_ij|^2 + eps^2)^(-1/2) */
      const double inv3 = inv * inv * inv;   /* (|r_ij|^2 + eps^2)^(-3/2) */
      const double qj = w * q[j];
      neumaier_add(&sx, &cx, qj * dx * inv3);
      neumaier_add(&sy, &cy, qj * dy * inv3);
      neumaier_add(&sz, &cz, qj * dz * inv3);
      if (phi) neumaier_add(&sp, &cp, qj * inv);
      if (amag) neumaier_add(&sa, &ca, fabs(qj) * sqrt(d2) * inv3);
      if (pmag) neumaier_add(&sb, &cb, fabs(qj) * inv);
    }
    ex[r] = k * (sx + cx);
    ey[r] = k * (sy + cy);
    ez[r] = k * (sz + cz);
    if (phi) phi[r] = k * (sp + cp);
    if (amag) amag[r] = k * (sa + ca);
    if (pmag) pmag[r] = k * (sb + cb);
  }
}

/* a_i = (q_i / m_i) E_i : Eqs. (D) and (F); the weight w cancels. */
static void accel(int64_t n, const double *x, const double *y, const double *z,
                  const double *q, const double *m, double w, double eps,
                  double *ax, double *ay, double *az) {
  oracle_field(n, x, y, z, q, w, eps, n, NULL, ax, ay, az, NULL, NULL, NULL);
  for (int64_t i = 0; i < n; ++i) {
    const double qm = q[i] / m[i];
    ax[i] *= qm;
    ay[i] *= qm;
    az[i] *= qm;
  }
}

/*
 * Velocity Verlet, Sec. 2.1 Eqs. (G) and (H).  State (r, v) is advanced in
 * place by n_steps steps of length dt:
 *   r(t+dt) = r(t) + v(t) dt + a(t) dt^2 / 2                        (G)
 *   a(t+dt) = (q/m) E(r(t+dt))
 *   v(t+dt) = v(t) + [a(t) + a(t+dt)] dt / 2                        (H)
 * ax,ay,az hold a(t) on entry when a_valid != 0; otherwise a(t) is first
 * computed from r(t).  On return they hold a at the final time, so a run may
 * be split into pieces without changing a single bit.
 */
void oracle_vv(int64_t n, double *x, double *y, double *z, double *vx,
               double *vy, double *vz, const double *q, const double *m,
               double w, double eps, double dt, int64_t n_steps, double *ax,
               double *ay, double *az, int a_valid) {
  double *bx = (double *)malloc((size_t)n * sizeof(double));
  double *by = (double *)malloc((size_t)n * sizeof(double));
  double *bz = (double *)malloc((size_t)n * sizeof(double));
  if (!a_valid) accel(n, x, y, z, q, m, w, eps, ax, ay, az);
  for (int64_t s = 0; s < n_steps; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      x[i] = x[i] + vx[i] * dt + ax[i] * dt * dt / 2.0;
      y[i] = y[i] + vy[i] * dt + ay[i] * dt * dt / 2.0;
      z[i] = z[i] + vz[i] * dt + az[i] * dt * dt / 2.0;
    }
    accel(n, x, y, z, q, m, w, eps, bx, by, bz);
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] + (ax[i] + bx[i]) * dt / 2.0;
      vy[i] = vy[i] + (ay[i] + by[i]) * dt / 2.0;
      vz[i] = vz[i] + (az[i] + bz[i]) * dt / 2.0;
      ax[i] = bx[i];
      ay[i] = by[i];
      az[i] = bz[i];
    }
  }
  free(bx);
  free(by);
  free(bz);
}

/* Diagnostics record; the Python side mirrors this layout. */
typedef struct {
  double kinetic;            /* sum_i (1/2) w m_i |v_i|^2                    */
  double potential;          /* (1/2) sum_i w q_i phi_i                      */
  double total;              /* kinetic + potential                          */
  double momentum[3];        /* sum_i w m_i v_i                              */
  double com[3];             /* sum_i m_i r_i / sum_i m_i                    */
  double com_velocity[3];    /* sum_i m_i v_i / sum_i m_i                    */
  double emittance[3];       /* Eq. (I) with raw moments, per axis           */
  double emittance_centered[3]; /* Eq. (I) with moments about the means      */
  double x_rms[3];           /* <x^2>^(1/2) per axis (raw)                   */
  double x_max[3];           /* max_i x_i per axis                           */
  double v_rms[3];           /* <v_x^2>^(1/2) per axis (raw)                 */
  double v_max[3];           /* max_i v_x,i per axis                         */
  int64_t nonfinite;         /* particles with a non-finite r or v           */
} oracle_diag_t;

/* Compensated sum of an array, in index order. */
static double csum(int64_t n, const double *a) {
  double s = 0, c = 0;
  for (int64_t i = 0; i < n; ++i) neumaier_add(&s, &c, a[i]);
  return s + c;
}

/*
 * Diagnostics of one bunch (Sec. 2.2 Eq. (I); Sec. 3.2 observables) plus the
 * conserved quantities.  Averages <.> are plain means over all n particles,
 * since all macro-particles share one weight.  Needs one O(n^2) potential
 * evaluation.
 */
void oracle_diag(int64_t n, const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz,
                 const double *q, const double *m, double w, double eps,
                 oracle_diag_t *out) {
  const double *r[3] = {x, y, z};
  const double *v[3] = {vx, vy, vz};
  memset(out, 0, sizeof(*out));
  if (n <= 0) return;
  double *t = (double *)calloc((size_t)n, sizeof(double));
  double *ex = (double *)malloc((size_t)n * sizeof(double));
  double *ey = (double *)malloc((size_t)n * sizeof(double));
  double *ez = (double *)malloc((size_t)n * sizeof(double));
  double *phi = (double *)malloc((size_t)n * sizeof(double));

  for (int64_t i = 0; i < n; ++i)
    t[i] = 0.5 * w * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
  out->kinetic = csum(n, t);

  oracle_field(n, x, y, z, q, w, eps, n, NULL, ex, ey, ez, phi, NULL, NULL);
  for (int64_t i = 0; i < n; ++i) t[i] = 0.5 * w * q[i] * phi[i];
  out->potential = csum(n, t);
  out->total = out->kinetic + out->potential;

  for (int64_t i = 0; i < n; ++i) t[i] = m[i];
  const double msum = csum(n, t);
  for (int a = 0; a < 3; ++a) {
    for (int64_t i = 0; i < n; ++i) t[i] = w * m[i] * v[a][i];
    out->momentum[a] = csum(n, t);
    for (int64_t i = 0; i < n; ++i) t[i] = m[i] * r[a][i];
    out->com[a] = csum(n, t) / msum;
    for (int64_t i = 0; i < n; ++i) t[i] = m[i] * v[a][i];
    out->com_velocity[a] = csum(n, t) / msum;

    /* raw moments, as Eq. (I) prints them */
    for (int64_t i = 0; i < n; ++i) t[i] = r[a][i] * r[a][i];
    const double xx = csum(n, t) / (double)n;
    for (int64_t i = 0; i < n; ++i) t[i] = v[a][i] * v[a][i];
    const double vv = csum(n, t) / (double)n;
    for (int64_t i = 0; i < n; ++i) t[i] = r[a][i] * v[a][i];
    const double xv = csum(n, t) / (double)n;
    const double e2 = xx * vv - xv * xv;
    out->emittance[a] = sqrt(e2 > 0 ? e2 : 0.0);
    out->x_rms[a] = sqrt(xx);
    out->v_rms[a] = sqrt(vv);

    /* moments about the means */
    const double xm = csum(n, r[a]) / (double)n;
    const double vm = csum(n, v[a]) / (double)n;
    for (int64_t i = 0; i < n; ++i) t[i] = (r[a][i] - xm) * (r[a][i] - xm);
    const double cxx = csum(n, t) / (double)n;
    for (int64_t i = 0; i < n; ++i) t[i] = (v[a][i] - vm) * (v[a][i] - vm);
    const double cvv = csum(n, t) / (double)n;
    for (int64_t i = 0; i < n; ++i) t[i] = (r[a][i] - xm) * (v[a][i] - vm);
    const double cxv = csum(n, t) / (double)n;
    const double c2 = cxx * cvv - cxv * cxv;
    out->emittance_centered[a] = sqrt(c2 > 0 ? c2 : 0.0);

    double xmax = -INFINITY, vmax = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
      if (r[a][i] > xmax) xmax = r[a][i];
      if (v[a][i] > vmax) vmax = v[a][i];
    }
    out->x_max[a] = xmax;
    out->v_max[a] = vmax;
  }
  for (int64_t i = 0; i < n; ++i) {
    int bad = 0;
    for (int a = 0; a < 3; ++a)
      if (!isfinite(r[a][i]) || !isfinite(v[a][i])) bad = 1;
    out->nonfinite += bad;
  }
  free(t);
  free(ex);
  free(ey);
  free(ez);
  free(phi);
}

/* Coulomb constant as compiled into this oracle, for the tests. */
double oracle_coulomb_k(void) { return coulomb_k(); }

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_num_threads(void) {
  int nt = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    nt = omp_get_num_threads();
  }
#endif
  return nt;
}

/* Sets the thread count of later parallel regions (n >= 1); the results do
 * not depend on it.  Without OpenMP the oracle is serial and this does
 * nothing. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
