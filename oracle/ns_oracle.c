/*
 * ns_oracle.c -- plain FP64 CPU oracle for the staggered-grid incompressible
 * Navier-Stokes step.  TEST INFRASTRUCTURE ONLY: the product path never
 * links, loads or calls this file.  It shares nothing with the HIP library.
 *
 * Everything here is written as plain loops over the grid, in the order the
 * method states, with no blocking, fusion or reordering.  Build with
 * -ffp-contract=off so that no fused multiply-add changes the rounding.
 * OpenMP splits the outer k loop only where iterations are independent;
 * reductions are summed per k plane and then serially, so results do not
 * depend on the thread count.
 *
 * Governing equations: the paper's eq. (1) ("Background and Governing
 * Equations"): du/dt + (u.grad)u = -grad phi + nu lap u + f, div u = 0,
 * phi = p / rho.  With rho = 1, phi == p; nu = 1 / Re.
 */
#include "ns_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* padded index, x fastest */
#define SX ((long)c->nx + 2)
#define SY ((long)c->ny + 2)
#define IX(i, j, k) (((long)(k) * SY + (long)(j)) * SX + (long)(i))

int nso_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int nn(const nso_cfg *c, int a) { return a == 0 ? c->nx : (a == 1 ? c->ny : c->nz); }
static double hh(const nso_cfg *c, int a) { return a == 0 ? c->dx : (a == 1 ? c->dy : c->dz); }

/* Index of the last normal-velocity unknown along its own axis: walls keep
 * faces 1..n-1 (faces 0 and n are the walls), periodic axes faces 1..n. */
static int last_face(const nso_cfg *c, int a) { return c->per[a] ? nn(c, a) : nn(c, a) - 1; }

/* ------------------------------------------------------------------------ */
/* Boundary / ghost fill (the driver-managed ghost regions of "MPI-Based Data
 * Parallelism in Cactus": physical boundaries are set from the boundary
 * conditions).  No-slip walls: the wall-normal face velocity is zero; a
 * tangential ghost is the reflection 2*U_wall - (adjacent interior value), so
 * the average across the wall equals the wall speed.  Periodic axes copy.
 * Order: wall-normal faces, tangential reflections, then periodic copies
 * x, y, z over the full extent of the other two indices, so that edge
 * ghosts that a periodic stencil reads hold the right periodic image.  */
static void fill_axis_periodic(const nso_cfg *c, double *q, int a) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  if (a == 0) {
    for (int k = 0; k <= nz + 1; k++)
      for (int j = 0; j <= ny + 1; j++) {
        q[IX(0, j, k)] = q[IX(nx, j, k)];
        q[IX(nx + 1, j, k)] = q[IX(1, j, k)];
      }
  } else if (a == 1) {
    for (int k = 0; k <= nz + 1; k++)
      for (int i = 0; i <= nx + 1; i++) {
        q[IX(i, 0, k)] = q[IX(i, ny, k)];
        q[IX(i, ny + 1, k)] = q[IX(i, 1, k)];
      }
  } else {
    for (int j = 0; j <= ny + 1; j++)
      for (int i = 0; i <= nx + 1; i++) {
        q[IX(i, j, 0)] = q[IX(i, j, nz)];
        q[IX(i, j, nz + 1)] = q[IX(i, j, 1)];
      }
  }
}

void nso_bc_vel(const nso_cfg *c, double *u, double *v, double *w) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double *q[3] = {u, v, w};
  /* 1. wall-normal faces */
  if (!c->per[0])
    for (int k = 0; k <= nz + 1; k++)
      for (int j = 0; j <= ny + 1; j++) { u[IX(0, j, k)] = 0.0; u[IX(nx, j, k)] = 0.0; }
  if (!c->per[1])
    for (int k = 0; k <= nz + 1; k++)
      for (int i = 0; i <= nx + 1; i++) { v[IX(i, 0, k)] = 0.0; v[IX(i, ny, k)] = 0.0; }
  if (!c->per[2])
    for (int j = 0; j <= ny + 1; j++)
      for (int i = 0; i <= nx + 1; i++) { w[IX(i, j, 0)] = 0.0; w[IX(i, j, nz)] = 0.0; }
  /* 2. tangential reflections; wall[f][comp], f = 2*axis + side */
  if (!c->per[0])
    for (int k = 1; k <= nz; k++)
      for (int j = 1; j <= ny; j++)
        for (int comp = 1; comp <= 2; comp++) {
          double *f = q[comp];
          f[IX(0, j, k)] = 2.0 * c->wall[0][comp] - f[IX(1, j, k)];
          f[IX(nx + 1, j, k)] = 2.0 * c->wall[1][comp] - f[IX(nx, j, k)];
        }
  if (!c->per[1])
    for (int k = 1; k <= nz; k++)
      for (int i = 1; i <= nx; i++)
        for (int comp = 0; comp <= 2; comp += 2) {
          double *f = q[comp];
          f[IX(i, 0, k)] = 2.0 * c->wall[2][comp] - f[IX(i, 1, k)];
          f[IX(i, ny + 1, k)] = 2.0 * c->wall[3][comp] - f[IX(i, ny, k)];
        }
  if (!c->per[2])
    for (int j = 1; j <= ny; j++)
      for (int i = 1; i <= nx; i++)
        for (int comp = 0; comp <= 1; comp++) {
          double *f = q[comp];
          f[IX(i, j, 0)] = 2.0 * c->wall[4][comp] - f[IX(i, j, 1)];
          f[IX(i, j, nz + 1)] = 2.0 * c->wall[5][comp] - f[IX(i, j, nz)];
        }
  /* 3. periodic copies */
  for (int a = 0; a < 3; a++)
    if (c->per[a])
      for (int comp = 0; comp < 3; comp++) fill_axis_periodic(c, q[comp], a);
}

void nso_p_ghosts(const nso_cfg *c, double *p) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  if (!c->per[0])
    for (int k = 1; k <= nz; k++)
      for (int j = 1; j <= ny; j++) { p[IX(0, j, k)] = p[IX(1, j, k)]; p[IX(nx + 1, j, k)] = p[IX(nx, j, k)]; }
  if (!c->per[1])
    for (int k = 1; k <= nz; k++)
      for (int i = 1; i <= nx; i++) { p[IX(i, 0, k)] = p[IX(i, 1, k)]; p[IX(i, ny + 1, k)] = p[IX(i, ny, k)]; }
  if (!c->per[2])
    for (int j = 1; j <= ny; j++)
      for (int i = 1; i <= nx; i++) { p[IX(i, j, 0)] = p[IX(i, j, 1)]; p[IX(i, j, nz + 1)] = p[IX(i, j, nz)]; }
  for (int a = 0; a < 3; a++)
    if (c->per[a]) fill_axis_periodic(c, p, a);
}

/* ------------------------------------------------------------------------ */
/* Momentum predictor.  The convective term of eq. (1) in conservation form,
 * (u.grad)u_c = sum_d d(u_d u_c)/dx_d (valid because div u = 0), is
 * differenced on the staggered grid: for the unknown q of component c and
 * each direction d, the flux through the half-way point between q and its
 * +d neighbour is psi(t, q, q[+d]) with t the d-velocity there (mean of the
 * two d-faces flanking that point: at pos and pos + e_c).  The flux blends
 * central and donor-cell (upwind) differencing with weight gamma:
 *     psi(t, a, b) = t (a + b)/2 + gamma |t| (a - b)/2
 * (gamma = 0: central; gamma = 1: the upwind value times t).  For d == c the
 * transport velocity is the mean of q and q[+d], giving the (u^2)_x term.
 * Viscous term: 7-point Laplacian.  Explicit Euler:
 *     F_c = q + dt (nu lap q - sum_d (psi_hi - psi_lo)/h_d + f_c).
 * Wall faces keep F = u (the wall value).                                  */
static double psi(double t, double a, double b, double gamma) {
  return t * (a + b) / 2.0 + gamma * fabs(t) * (a - b) / 2.0;
}

/* The other form of the lineage the paper follows (Hirt's SOLA family and
 * NASA-VOF2D): the convective term in advective form, (u.grad)u_c =
 * sum_d a_d dq/dx_d, with a_d the d-velocity at the unknown's own position
 * (the unknown itself for d == c, else the mean of the four d-faces around
 * it: at pos and pos + e_c, on both sides in d) and the derivative an
 * alpha-weighted blend of the backward and forward differences:
 *     a (dq/dx)_h = a [ (1 + alpha s)(q - q[-d]) + (1 - alpha s)(q[+d] - q) ] / (2 h)
 * with s = sign(a), sign(0) = 0 (alpha = 0: central; alpha = 1: upwind).
 * Selected by cfg->advective with alpha = cfg->gamma.                     */
static double adv_term(double a, double qm, double qc, double qp, double alpha, double h) {
  double s = (a > 0.0) - (a < 0.0);
  return a * ((1.0 + alpha * s) * (qc - qm) + (1.0 - alpha * s) * (qp - qc)) / (2.0 * h);
}

static long stride(const nso_cfg *c, int a) { return a == 0 ? 1 : (a == 1 ? SX : SX * SY); }

void nso_fgh(const nso_cfg *c, double dt, const double *u, const double *v,
             const double *w, const double *fx, const double *fy,
             const double *fz, double *F, double *G, double *H) {
  const double *vel[3] = {u, v, w};
  const double *frc[3] = {fx, fy, fz};
  double *out[3] = {F, G, H};
  double nu = 1.0 / c->re;
  long ntot = SX * SY * ((long)c->nz + 2);
  for (int comp = 0; comp < 3; comp++) {
    const double *q = vel[comp];
    double *o = out[comp];
    /* F = u everywhere first: covers the wall faces (F := wall value). */
    memcpy(o, q, sizeof(double) * (size_t)ntot);
    int hi[3] = {c->nx, c->ny, c->nz};
    hi[comp] = last_face(c, comp);
    long sc = stride(c, comp);
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= hi[2]; k++)
      for (int j = 1; j <= hi[1]; j++)
        for (int i = 1; i <= hi[0]; i++) {
          long id = IX(i, j, k);
          double qc = q[id];
          double lap = 0.0, conv = 0.0;
          for (int d = 0; d < 3; d++) {
            long sd = stride(c, d);
            double h = hh(c, d);
            double qp = q[id + sd], qm = q[id - sd];
            lap += (qp - 2.0 * qc + qm) / (h * h);
            const double *T = vel[d];
            if (c->advective) {
              double a = d == comp ? qc : (T[id] + T[id + sc] + T[id - sd] + T[id - sd + sc]) / 4.0;
              conv += adv_term(a, qm, qc, qp, c->gamma, h);
              continue;
            }
            double thi = (T[id] + T[id + sc]) / 2.0;
            double tlo = (T[id - sd] + T[id - sd + sc]) / 2.0;
            conv += (psi(thi, qc, qp, c->gamma) - psi(tlo, qm, qc, c->gamma)) / h;
          }
          double f = c->g[comp] + (frc[comp] ? frc[comp][id] : 0.0);
          o[id] = qc + dt * (nu * lap - conv + f);
        }
    /* periodic images of the new face values (rhs reads face 0 == face n) */
    for (int a = 0; a < 3; a++)
      if (c->per[a]) fill_axis_periodic(c, o, a);
  }
}

/* Discrete divergence on cell centres: D q = sum_d (q_d[pos] - q_d[pos - e_d]) / h_d. */
void nso_divergence(const nso_cfg *c, const double *u, const double *v,
                    const double *w, double *div) {
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= c->nz; k++)
    for (int j = 1; j <= c->ny; j++)
      for (int i = 1; i <= c->nx; i++) {
        long id = IX(i, j, k);
        div[id] = (u[id] - u[id - 1]) / c->dx + (v[id] - v[id - SX]) / c->dy +
                  (w[id] - w[id - SX * SY]) / c->dz;
      }
}

/* Pressure-Poisson right-hand side: div u^{n+1} = 0 with
 * u^{n+1} = F - dt grad p gives lap p = (D F) / dt on every cell.         */
void nso_rhs(const nso_cfg *c, double dt, const double *F, const double *G,
             const double *H, double *rhs) {
  nso_divergence(c, F, G, H, rhs);
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= c->nz; k++)
    for (int j = 1; j <= c->ny; j++)
      for (int i = 1; i <= c->nx; i++) rhs[IX(i, j, k)] /= dt;
}

/* ------------------------------------------------------------------------ */
/* Poisson operator: boundary-eliminated homogeneous-Neumann 7-point
 * Laplacian.  a_nb = 1/h^2 for each neighbour that is an interior cell (or
 * its periodic image) and 0 across a wall; A p = sum_nb a_nb (p_nb - p).  */
static void nb_coef(const nso_cfg *c, int i, int j, int k, long nb[6], double a[6]) {
  int idx[3] = {i, j, k};
  for (int d = 0; d < 3; d++) {
    int n = nn(c, d);
    double h2 = 1.0 / (hh(c, d) * hh(c, d));
    for (int s = 0; s < 2; s++) {
      int t[3] = {idx[0], idx[1], idx[2]};
      t[d] += s ? 1 : -1;
      double coef = h2;
      if (t[d] < 1) { if (c->per[d]) t[d] = n; else { coef = 0.0; t[d] = 1; } }
      if (t[d] > n) { if (c->per[d]) t[d] = 1; else { coef = 0.0; t[d] = n; } }
      nb[2 * d + s] = IX(t[0], t[1], t[2]);
      a[2 * d + s] = coef;
    }
  }
}

double nso_rms(const nso_cfg *c, const double *q) {
  double *plane = (double *)calloc((size_t)c->nz + 2, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= c->nz; k++) {
    double s = 0.0;
    for (int j = 1; j <= c->ny; j++)
      for (int i = 1; i <= c->nx; i++) s += q[IX(i, j, k)] * q[IX(i, j, k)];
    plane[k] = s;
  }
  double s = 0.0;
  for (int k = 1; k <= c->nz; k++) s += plane[k];
  free(plane);
  return sqrt(s / ((double)c->nx * c->ny * c->nz));
}

double nso_residual(const nso_cfg *c, const double *p, const double *rhs, double *r) {
  double *plane = (double *)calloc((size_t)c->nz + 2, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= c->nz; k++) {
    double s = 0.0;
    for (int j = 1; j <= c->ny; j++)
      for (int i = 1; i <= c->nx; i++) {
        long nb[6];
        double a[6];
        nb_coef(c, i, j, k, nb, a);
        long id = IX(i, j, k);
        double ap = 0.0;
        for (int m = 0; m < 6; m++) ap += a[m] * (p[nb[m]] - p[id]);
        double res = ap - rhs[id];
        if (r) r[id] = res;
        s += res * res;
      }
    plane[k] = s;
  }
  double s = 0.0;
  for (int k = 1; k <= c->nz; k++) s += plane[k];
  free(plane);
  return sqrt(s / ((double)c->nx * c->ny * c->nz));
}

/* One SOR half-sweep over the cells of one colour, (i+j+k) % 2 == colour,
 * in place: p <- (1-w) p + w (sum_nb a_nb p_nb - rhs) / sum_nb a_nb.       */
static void sor_colour(const nso_cfg *c, double *p, const double *rhs, double omega, int colour) {
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= c->nz; k++)
    for (int j = 1; j <= c->ny; j++)
      for (int i = 1; i <= c->nx; i++) {
        if (((i + j + k) & 1) != colour) continue;
        long nb[6];
        double a[6];
        nb_coef(c, i, j, k, nb, a);
        double sum = 0.0, ac = 0.0;
        for (int m = 0; m < 6; m++) { sum += a[m] * p[nb[m]]; ac += a[m]; }
        long id = IX(i, j, k);
        p[id] = (1.0 - omega) * p[id] + omega * (sum - rhs[id]) / ac;
      }
}

void nso_sor_sweep(const nso_cfg *c, double *p, const double *rhs, double omega) {
  sor_colour(c, p, rhs, omega, 0); /* red: (i+j+k) even */
  sor_colour(c, p, rhs, omega, 1); /* black */
}

/* Stop rule: after every full sweep, stop once the RMS residual is at most
 * tol * RMS(rhs); at most itermax sweeps; rhs == 0 needs no sweep.         */
int nso_sor_solve(const nso_cfg *c, double *p, const double *rhs, double *res) {
  double rr = nso_rms(c, rhs);
  double thr = c->tol * (rr > 1e-300 ? rr : 1e-300);
  *res = 0.0;
  if (rr == 0.0) return 0;
  int it = 0;
  while (it < c->itermax) {
    nso_sor_sweep(c, p, rhs, c->omega);
    it++;
    *res = nso_residual(c, p, rhs, NULL);
    if (!(*res > thr)) break; /* also stops on NaN */
  }
  return it;
}

/* Defect-correction form (the Poisson solve in an outer/inner split):
 *   outer: r = rhs - A p, stop when RMS(r) <= tol * RMS(rhs);
 *   inner: SOR sweeps on A e = r from e = 0 until RMS(r - A e) <= eta *
 *          RMS(r) or the shared sweep budget is spent; then p += e.
 * All arithmetic here is FP64; the GPU runs the inner sweeps in FP32.       */
int nso_sor_defect(const nso_cfg *c, double *p, const double *rhs, double *res, int *outer) {
  long ntot = SX * SY * ((long)c->nz + 2);
  double *r = (double *)calloc((size_t)ntot, sizeof(double));
  double *e = (double *)calloc((size_t)ntot, sizeof(double));
  double rr = nso_rms(c, rhs);
  double thr = c->tol * (rr > 1e-300 ? rr : 1e-300);
  int sweeps = 0;
  *outer = 0;
  *res = 0.0;
  if (rr == 0.0) { free(r); free(e); return 0; }
  for (;;) {
    /* residual of the Poisson equation, with the sign of the correction:
     * r = rhs - A p (nso_residual returns A p - rhs). */
    double ro = nso_residual(c, p, rhs, r);
    for (long m = 0; m < ntot; m++) r[m] = -r[m];
    *res = ro;
    if (!(ro > thr) || sweeps >= c->itermax) break;
    (*outer)++;
    memset(e, 0, sizeof(double) * (size_t)ntot);
    double thr_in = c->eta * ro;
    while (sweeps < c->itermax) {
      nso_sor_sweep(c, e, r, c->omega);
      sweeps++;
      double re = nso_residual(c, e, r, NULL);
      if (!(re > thr_in)) break;
    }
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= c->nz; k++)
      for (int j = 1; j <= c->ny; j++)
        for (int i = 1; i <= c->nx; i++) p[IX(i, j, k)] += e[IX(i, j, k)];
  }
  free(r);
  free(e);
  return sweeps;
}

/* Projection (the paper's UPDATE_VELOCITY: velocity from the predictor and
 * the pressure gradient, density 1): u = F - dt (p[+x] - p) / dx on the
 * normal-velocity unknowns of each component.  Pressure ghosts must hold
 * their periodic images (nso_p_ghosts) before this call.                   */
void nso_project(const nso_cfg *c, double dt, const double *F, const double *G,
                 const double *H, const double *p, double *u, double *v, double *w) {
  const double *in[3] = {F, G, H};
  double *out[3] = {u, v, w};
  for (int comp = 0; comp < 3; comp++) {
    int hi[3] = {c->nx, c->ny, c->nz};
    hi[comp] = last_face(c, comp);
    long sc = stride(c, comp);
    double h = hh(c, comp);
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= hi[2]; k++)
      for (int j = 1; j <= hi[1]; j++)
        for (int i = 1; i <= hi[0]; i++) {
          long id = IX(i, j, k);
          out[comp][id] = in[comp][id] - dt * (p[id + sc] - p[id]) / h;
        }
  }
}

/* Adaptive step: tau * min(diffusive limit Re/2 / sum 1/h^2, h_d / max|u_d|),
 * where max|u_d| includes the wall speeds; a zero maximum sets no limit.   */
double nso_dt(const nso_cfg *c, const double *u, const double *v, const double *w) {
  const double *vel[3] = {u, v, w};
  double lim = (c->re / 2.0) /
               (1.0 / (c->dx * c->dx) + 1.0 / (c->dy * c->dy) + 1.0 / (c->dz * c->dz));
  for (int comp = 0; comp < 3; comp++) {
    double m = 0.0;
    for (int f = 0; f < 6; f++) m = fmax(m, fabs(c->wall[f][comp]));
    int hi[3] = {c->nx, c->ny, c->nz};
    hi[comp] = last_face(c, comp);
    for (int k = 1; k <= hi[2]; k++)
      for (int j = 1; j <= hi[1]; j++)
        for (int i = 1; i <= hi[0]; i++) m = fmax(m, fabs(vel[comp][IX(i, j, k)]));
    if (m > 0.0) lim = fmin(lim, hh(c, comp) / m);
  }
  return c->tau * lim;
}

/* ------------------------------------------------------------------------ */
/* One projected Euler stage from the current velocity with step dt:
 * velocity BC, predictor, rhs, Poisson solve, pressure ghosts, projection,
 * velocity BC.  Returns the sweeps; *res, *outer, *thr of the solve.      */
static int euler_stage(const nso_cfg *c, double dt, double *u, double *v, double *w, double *p,
                       const double *fx, const double *fy, const double *fz, double *work, int mode,
                       double *res, int *outer, double *thr) {
  long ntot = SX * SY * ((long)c->nz + 2);
  double *F = work, *G = work + ntot, *H = work + 2 * ntot, *rhs = work + 3 * ntot;
  nso_bc_vel(c, u, v, w);
  nso_fgh(c, dt, u, v, w, fx, fy, fz, F, G, H);
  nso_rhs(c, dt, F, G, H, rhs);
  *res = 0.0;
  *outer = 0;
  int sweeps;
  if (mode == 0) sweeps = nso_sor_solve(c, p, rhs, res);
  else sweeps = nso_sor_defect(c, p, rhs, res, outer);
  nso_p_ghosts(c, p);
  nso_project(c, dt, F, G, H, p, u, v, w);
  nso_bc_vel(c, u, v, w);
  double rr = nso_rms(c, rhs);
  *thr = c->tol * (rr > 1e-300 ? rr : 1e-300);
  return sweeps;
}

/* One step n -> n+1.  dt from u^n (adaptive) or fixed.  Euler: one stage.
 * Two stages (the second-order strong-stability-preserving Runge-Kutta
 * method of Heun, the method-of-lines form: y1 = y + dt f(y),
 * y+ = (y + y1 + dt f(y1)) / 2): u1 = P(u^n + dt N(u^n)),
 * u2 = P(u1 + dt N(u1)), u^{n+1} = (u^n + u2) / 2 on every entry, then the
 * velocity BC.  P is linear and u^n divergence-free, so the average is too;
 * the pressure left is the second stage's.                                  */
int nso_run(const nso_cfg *c, double *u, double *v, double *w, double *p,
            const double *fx, const double *fy, const double *fz,
            double *work, int nsteps, int mode, nso_stats *st) {
  long ntot = SX * SY * ((long)c->nz + 2);
  double *save = NULL;
  if (c->stages == 2) {
    save = (double *)malloc(3 * ntot * sizeof(double));
    if (!save) return -5;
  }
  int rc = 0;
  for (int s = 0; s < nsteps; s++) {
    double dt = c->dt > 0.0 ? c->dt : nso_dt(c, u, v, w);
    if (save) {
      memcpy(save, u, ntot * sizeof(double));
      memcpy(save + ntot, v, ntot * sizeof(double));
      memcpy(save + 2 * ntot, w, ntot * sizeof(double));
    }
    double res, thr;
    int outer;
    int sweeps = euler_stage(c, dt, u, v, w, p, fx, fy, fz, work, mode, &res, &outer, &thr);
    int unconv = res > thr;
    if (save && isfinite(res)) {
      double res2, thr2;
      int outer2;
      sweeps += euler_stage(c, dt, u, v, w, p, fx, fy, fz, work, mode, &res2, &outer2, &thr2);
      unconv |= res2 > thr2;
      if (outer2 > outer) outer = outer2;
      res = res2;
      double *q[3] = {u, v, w};
      for (int f = 0; f < 3; f++)
        for (long e = 0; e < ntot; e++) q[f][e] = 0.5 * (save[f * ntot + e] + q[f][e]);
      nso_bc_vel(c, u, v, w);
    }
    if (!isfinite(res)) {
      rc = -4;
      break;
    }
    st->t += dt;
    st->dt_last = dt;
    st->res_last = res;
    st->sweeps_total += sweeps;
    if (sweeps > st->sweeps_max) st->sweeps_max = sweeps;
    if (outer > st->outer_max) st->outer_max = outer;
    if (unconv) st->steps_unconverged++;
    st->steps++;
  }
  free(save);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint (reverse mode) of one step u^n -> u^{n+1} = P Phi(B(u^n)), where B
 * is the boundary fill, Phi the predictor and P = I - G A^+ D the exact
 * projection.  With G = -D^T (true for the MAC operators on any spacing), P
 * is symmetric, so its transpose is itself: rhs = D lambda, A q = rhs,
 * mu = lambda - G q (the forward solve with dt = 1).                        */
static void zero_non_unknowns(const nso_cfg *c, double *q, int comp) {
  int hi[3] = {c->nx, c->ny, c->nz};
  hi[comp] = last_face(c, comp);
  for (int k = 0; k <= c->nz + 1; k++)
    for (int j = 0; j <= c->ny + 1; j++)
      for (int i = 0; i <= c->nx + 1; i++)
        if (i < 1 || i > hi[0] || j < 1 || j > hi[1] || k < 1 || k > hi[2]) q[IX(i, j, k)] = 0.0;
}

int nso_adj_project(const nso_cfg *c, double *lu, double *lv, double *lw, double *p, double *rhs) {
  double *l[3] = {lu, lv, lw};
  for (int comp = 0; comp < 3; comp++) {
    zero_non_unknowns(c, l[comp], comp);
    /* the divergence reads face 0 == face n on periodic axes */
    for (int a = 0; a < 3; a++)
      if (c->per[a]) fill_axis_periodic(c, l[comp], a);
  }
  nso_divergence(c, lu, lv, lw, rhs);
  double res;
  int sw = nso_sor_solve(c, p, rhs, &res);
  nso_p_ghosts(c, p);
  /* mu = lambda - G q on the unknowns: same arithmetic as the projection
   * with F = lambda, dt = 1. */
  nso_project(c, 1.0, lu, lv, lw, p, lu, lv, lw);
  for (int comp = 0; comp < 3; comp++) zero_non_unknowns(c, l[comp], comp);
  return sw;
}

/* Partial derivatives of psi(t, a, b) = t (a+b)/2 + gamma |t| (a-b)/2, with
 * sign(0) := 0. */
static void dpsi(double t, double a, double b, double gamma, double *dt_, double *da, double *db) {
  double sg = t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0);
  *dt_ = (a + b) / 2.0 + gamma * sg * (a - b) / 2.0;
  *da = t / 2.0 + gamma * fabs(t) / 2.0;
  *db = t / 2.0 - gamma * fabs(t) / 2.0;
}

/* Reverse of the boundary fill: the fill is a sequence of assignments
 * ghost := s * source + const; its transpose runs them backwards as
 * z[source] += s * z[ghost]; z[ghost] = 0.                                  */
static void fold_periodic(const nso_cfg *c, double *z, int a) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  if (a == 0) {
    for (int k = nz + 1; k >= 0; k--)
      for (int j = ny + 1; j >= 0; j--) {
        z[IX(1, j, k)] += z[IX(nx + 1, j, k)]; z[IX(nx + 1, j, k)] = 0.0;
        z[IX(nx, j, k)] += z[IX(0, j, k)]; z[IX(0, j, k)] = 0.0;
      }
  } else if (a == 1) {
    for (int k = nz + 1; k >= 0; k--)
      for (int i = nx + 1; i >= 0; i--) {
        z[IX(i, 1, k)] += z[IX(i, ny + 1, k)]; z[IX(i, ny + 1, k)] = 0.0;
        z[IX(i, ny, k)] += z[IX(i, 0, k)]; z[IX(i, 0, k)] = 0.0;
      }
  } else {
    for (int j = ny + 1; j >= 0; j--)
      for (int i = nx + 1; i >= 0; i--) {
        z[IX(i, j, 1)] += z[IX(i, j, nz + 1)]; z[IX(i, j, nz + 1)] = 0.0;
        z[IX(i, j, nz)] += z[IX(i, j, 0)]; z[IX(i, j, 0)] = 0.0;
      }
  }
}

static void fold_bc(const nso_cfg *c, double *zu, double *zv, double *zw) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double *z[3] = {zu, zv, zw};
  for (int a = 2; a >= 0; a--)
    if (c->per[a])
      for (int comp = 2; comp >= 0; comp--) fold_periodic(c, z[comp], a);
  if (!c->per[2])
    for (int j = ny; j >= 1; j--)
      for (int i = nx; i >= 1; i--)
        for (int comp = 1; comp >= 0; comp--) {
          double *f = z[comp];
          f[IX(i, j, nz)] -= f[IX(i, j, nz + 1)]; f[IX(i, j, nz + 1)] = 0.0;
          f[IX(i, j, 1)] -= f[IX(i, j, 0)]; f[IX(i, j, 0)] = 0.0;
        }
  if (!c->per[1])
    for (int k = nz; k >= 1; k--)
      for (int i = nx; i >= 1; i--)
        for (int comp = 2; comp >= 0; comp -= 2) {
          double *f = z[comp];
          f[IX(i, ny, k)] -= f[IX(i, ny + 1, k)]; f[IX(i, ny + 1, k)] = 0.0;
          f[IX(i, 1, k)] -= f[IX(i, 0, k)]; f[IX(i, 0, k)] = 0.0;
        }
  if (!c->per[0])
    for (int k = nz; k >= 1; k--)
      for (int j = ny; j >= 1; j--)
        for (int comp = 2; comp >= 1; comp--) {
          double *f = z[comp];
          f[IX(nx, j, k)] -= f[IX(nx + 1, j, k)]; f[IX(nx + 1, j, k)] = 0.0;
          f[IX(1, j, k)] -= f[IX(0, j, k)]; f[IX(0, j, k)] = 0.0;
        }
  /* wall-normal faces are constants: no sensitivity flows through them */
  for (int comp = 0; comp < 3; comp++) zero_non_unknowns(c, z[comp], comp);
}

/* (ou,ov,ow) = B^T J_Phi(B u)^T (mu,mv,mw), scatter form: every unknown q
 * of the predictor sends mu_q * dPhi_q/d(input) to each input it reads.   */
void nso_adj_fgh(const nso_cfg *c, double dt, const double *u, const double *v,
                 const double *w, const double *mu, const double *mv,
                 const double *mw, double *ou, double *ov, double *ow) {
  const double *vel[3] = {u, v, w};
  const double *m[3] = {mu, mv, mw};
  double *z[3] = {ou, ov, ow};
  double nu = 1.0 / c->re;
  long ntot = SX * SY * ((long)c->nz + 2);
  for (int comp = 0; comp < 3; comp++) memset(z[comp], 0, sizeof(double) * (size_t)ntot);
  for (int comp = 0; comp < 3; comp++) {
    const double *q = vel[comp];
    int hi[3] = {c->nx, c->ny, c->nz};
    hi[comp] = last_face(c, comp);
    long sc = stride(c, comp);
    for (int k = 1; k <= hi[2]; k++)
      for (int j = 1; j <= hi[1]; j++)
        for (int i = 1; i <= hi[0]; i++) {
          long id = IX(i, j, k);
          double mq = m[comp][id];
          if (mq == 0.0) continue;
          double *zq = z[comp];
          zq[id] += mq; /* identity */
          for (int d = 0; d < 3; d++) {
            long sd = stride(c, d);
            double h = hh(c, d);
            /* viscous */
            double wv = dt * nu * mq / (h * h);
            zq[id + sd] += wv;
            zq[id - sd] += wv;
            zq[id] -= 2.0 * wv;
            /* convective: Phi_q contains -dt * (psi_hi - psi_lo) / h */
            const double *T = vel[d];
            double *zT = z[d];
            double wc = -dt * mq / h;
            double qc = q[id], qp = q[id + sd], qm = q[id - sd];
            double thi = (T[id] + T[id + sc]) / 2.0;
            double tlo = (T[id - sd] + T[id - sd + sc]) / 2.0;
            double gt, ga, gb;
            dpsi(thi, qc, qp, c->gamma, &gt, &ga, &gb);
            zq[id] += wc * ga;
            zq[id + sd] += wc * gb;
            zT[id] += wc * gt / 2.0;
            zT[id + sc] += wc * gt / 2.0;
            dpsi(tlo, qm, qc, c->gamma, &gt, &ga, &gb);
            zq[id - sd] -= wc * ga;
            zq[id] -= wc * gb;
            zT[id - sd] -= wc * gt / 2.0;
            zT[id - sd + sc] -= wc * gt / 2.0;
          }
        }
  }
  fold_bc(c, ou, ov, ow);
}
