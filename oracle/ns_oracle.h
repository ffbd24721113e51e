/*
 * ns_oracle.h -- plain FP64 CPU oracle for the incompressible Navier-Stokes
 * stencil step (test infrastructure only).
 *
 * This library exists to check the HIP product path.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * The method is the one the paper's CFD section describes: the incompressible
 * Navier-Stokes equations (momentum + incompressibility, phi = p / rho,
 * kinematic viscosity nu, body force f; "Background and Governing Equations",
 * eq. (1)) discretised by finite differences on a regular rectangular
 * staggered grid in the Hirt / NASA-VOF2D lineage, evaluated as stencils
 * ("Background and Governing Equations", the paragraph after eq. (1)).  The
 * paper prints no stencil, integrator or solver, so every discrete choice
 * below is a reading of the paper, stated where it is implemented: the MAC arrangement,
 * the donor-cell-blended conservative momentum predictor (F, G, H), the
 * pressure-Poisson right-hand side, red-black SOR on the boundary-eliminated
 * Neumann Laplacian with an RMS residual stop rule, and the velocity
 * projection (the paper's UPDATE_VELOCITY kernel descriptor in the
 * "CaCUDA Kernel Abstraction" section).
 *
 * Layout: every field is a C-contiguous [nz+2][ny+2][nx+2] array of doubles,
 * x fastest, one ghost layer on every side.
 *   u[k][j][i] sits at (i*dx, (j-1/2)*dy, (k-1/2)*dz)  (x faces)
 *   v[k][j][i] sits at ((i-1/2)*dx, j*dy, (k-1/2)*dz)  (y faces)
 *   w[k][j][i] sits at ((i-1/2)*dx, (j-1/2)*dy, k*dz)  (z faces)
 *   p, rhs     sit at cell centres ((i-1/2)*dx, ...), i = 1..nx.
 * Wall axis: the normal-velocity unknowns are faces 1..n-1 (faces 0 and n
 * are the walls).  Periodic axis: unknowns 1..n, face 0 == face n.
 */
#ifndef NS_ORACLE_H
#define NS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny, nz;       /* interior cells per axis */
  int per[3];           /* 1 = periodic axis, 0 = no-slip walls */
  double dx, dy, dz;    /* cell widths */
  double re;            /* Reynolds number; nu = 1/re */
  double dt;            /* > 0: fixed step; <= 0: adaptive with tau */
  double tau;           /* adaptive safety factor */
  double gamma;         /* donor-cell blend in [0,1] */
  double omega;         /* SOR relaxation */
  double tol;           /* relative RMS residual tolerance */
  int itermax;          /* SOR sweep budget per step */
  double wall[6][3];    /* wall velocity on faces -x,+x,-y,+y,-z,+z */
  double g[3];          /* constant body force */
  double eta;           /* defect-correction inner tolerance factor */
  int advective;        /* 0: conservative fluxes blended by gamma; 1: advective form
                           weighted by alpha = gamma (see nso_fgh) */
  int stages;           /* time integrator: 0 or 1 = explicit Euler with projection;
                           2 = two-stage SSP Runge-Kutta (Heun) whose stages are
                           projected Euler steps with the same dt (see nso_run) */
} nso_cfg;

typedef struct {
  double t, dt_last, res_last;
  long long sweeps_total;
  int steps, sweeps_max, steps_unconverged, outer_max;
} nso_stats;

/* Ghost / boundary fill for the three velocity fields. */
void nso_bc_vel(const nso_cfg *c, double *u, double *v, double *w);
/* Pressure ghosts (Neumann copy on walls, periodic copy); output only. */
void nso_p_ghosts(const nso_cfg *c, double *p);
/* Momentum predictor F, G, H; fx, fy, fz may be NULL (then only g is used). */
void nso_fgh(const nso_cfg *c, double dt, const double *u, const double *v,
             const double *w, const double *fx, const double *fy,
             const double *fz, double *F, double *G, double *H);
/* Pressure-Poisson right-hand side on cell centres. */
void nso_rhs(const nso_cfg *c, double dt, const double *F, const double *G,
             const double *H, double *rhs);
/* Residual field r = A p - rhs (A: boundary-eliminated Laplacian); r may be
 * NULL.  Returns the RMS of r over the interior cells. */
double nso_residual(const nso_cfg *c, const double *p, const double *rhs,
                    double *r);
/* RMS of a cell-centred field over the interior. */
double nso_rms(const nso_cfg *c, const double *q);
/* One red-black SOR sweep in place (red = (i+j+k) even first). */
void nso_sor_sweep(const nso_cfg *c, double *p, const double *rhs, double omega);
/* Red-black SOR to the stop rule; returns sweeps done, *res = final RMS. */
int nso_sor_solve(const nso_cfg *c, double *p, const double *rhs, double *res);
/* Defect-correction form of the Poisson solve, all in FP64 arithmetic;
 * returns total inner sweeps, *res the last outer RMS, *outer the outer
 * iterations. */
int nso_sor_defect(const nso_cfg *c, double *p, const double *rhs, double *res,
                   int *outer);
/* Velocity projection u = F - dt * grad p on the unknowns (no BC fill). */
void nso_project(const nso_cfg *c, double dt, const double *F, const double *G,
                 const double *H, const double *p, double *u, double *v,
                 double *w);
/* Discrete divergence D u on cell centres. */
void nso_divergence(const nso_cfg *c, const double *u, const double *v,
                    const double *w, double *div);
/* Adaptive step from the current velocity. */
double nso_dt(const nso_cfg *c, const double *u, const double *v,
              const double *w);
/* nsteps full steps; work holds 4 padded fields (F, G, H, rhs).  mode 0 =
 * plain SOR, 1 = defect-correction form.  Returns 0, or -4 when a
 * non-finite residual appears (st->steps counts completed steps), -5 when
 * the two-stage integrator cannot get its scratch memory.  With two stages
 * a step's sweeps are those of both solves, its residual the second's, and
 * it counts as unconverged when either solve stopped above its threshold. */
int nso_run(const nso_cfg *c, double *u, double *v, double *w, double *p,
            const double *fx, const double *fy, const double *fz,
            double *work, int nsteps, int mode, nso_stats *st);

/* ---- adjoint (reverse mode) of one step with an exact Poisson solve ---- */
/* Transpose of the projection map P = I - G A^+ D applied to (lu,lv,lw) in
 * place; p is scratch (its content on entry is the SOR warm start). */
int nso_adj_project(const nso_cfg *c, double *lu, double *lv, double *lw,
                    double *p, double *rhs);
/* Transpose of the predictor Jacobian at state (u,v,w) (ghosts filled by
 * the boundary map): (ou,ov,ow) = J_F^T (mu,mv,mw) on the unknowns. */
void nso_adj_fgh(const nso_cfg *c, double dt, const double *u, const double *v,
                 const double *w, const double *mu, const double *mv,
                 const double *mw, double *ou, double *ov, double *ow);

int nso_threads(void);

#ifdef __cplusplus
}
#endif
#endif
