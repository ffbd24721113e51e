/*
 * ns.h -- C ABI of the MI355X (gfx950) incompressible Navier-Stokes stencil
 * step: libns.so.
 *
 * What it computes.  The time step of the 3D CFD code the paper uses to
 * demonstrate its framework ("CFD Implementation"): the incompressible
 * Navier-Stokes equations of eq. (1) (du/dt + (u.grad)u = -grad phi +
 * nu lap u + f, div u = 0, phi = p / rho) discretised by finite differences
 * on a regular rectangular staggered grid and evaluated as stencils over a
 * cell's close neighbourhood (the paragraph after eq. (1)).  One step is
 *   1. dt (fixed, or adaptive from the velocity),
 *   2. ghost / boundary fill of the velocity (the ghost regions of
 *      "MPI-Based Data Parallelism in Cactus": physical boundaries set from
 *      the boundary conditions),
 *   3. momentum predictor F, G, H with a donor-cell blend gamma,
 *   4. pressure-Poisson right-hand side (div F) / dt,
 *   5. red-black SOR on the Neumann Laplacian with an RMS residual stop rule
 *      (FP64, or FP32 sweeps inside an FP64 defect-correction loop),
 *   6. velocity projection u = F - dt grad p (the paper's UPDATE_VELOCITY
 *      kernel: velocity in/out, pressure in, density parameter = 1),
 *   7. ghost / boundary fill again.
 * The paper prints no stencil, so the discrete operators are the documented
 * reading: MAC staggering, conservative central / donor-cell convection,
 * 7-point Laplacians, explicit Euler, Chorin projection.
 *
 * Conventions (all entry points):
 *  - Return codes only; no abort, exit or exception crosses the ABI.
 *    ns_last_error() gives a message for the last failing call.
 *  - Fields at the boundary are FP64, C-contiguous [nz+2][ny+2][nx+2]
 *    (x fastest) with one ghost layer:
 *      u[k][j][i] at (i dx, (j-1/2) dy, (k-1/2) dz)   (x faces)
 *      v[k][j][i] at ((i-1/2) dx, j dy, (k-1/2) dz)   (y faces)
 *      w[k][j][i] at ((i-1/2) dx, (j-1/2) dy, k dz)   (z faces)
 *      p          at cell centres ((i-1/2) dx, (j-1/2) dy, (k-1/2) dz).
 *    On a wall axis the normal-velocity unknowns are faces 1..n-1 (faces 0
 *    and n are the walls); on a periodic axis faces 1..n (face 0 == n).
 *    Entries that are neither unknowns nor read ghosts hold unspecified
 *    values on return.  The internal layout and storage precision are
 *    private; set/get convert.
 *  - Ownership: the caller owns every pointer it passes; the library copies
 *    (on the handle's stream) and keeps no caller pointer.  on_device = 1
 *    means the pointer is HIP device memory, 0 host memory; host-pointer
 *    calls return after the copy completed.  The library owns all device
 *    memory it allocates (in ns_create, freed in ns_destroy).
 *  - ns_step is synchronous: it returns when the steps are done.
 *  - One host thread per handle at a time.  Handles may be driven from
 *    different threads at once (on different streams); the persistent
 *    launches of batched handles on one device then take turns, since each
 *    needs the whole device.
 */
#ifndef NSMI_NS_H_
#define NSMI_NS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_solver ns_solver; /* opaque; created, owned, freed by the library */

typedef enum {
  NS_OK = 0,
  NS_E_INVALID = -1,   /* bad argument or parameter */
  NS_E_OOM = -2,       /* device allocation failed */
  NS_E_DEVICE = -3,    /* a HIP call failed */
  NS_E_NONFINITE = -4, /* NaN / Inf reached the residual norm; state undefined */
  NS_E_UNSTABLE = -5,  /* fixed dt beyond the explicit stability bounds */
  NS_E_STATE = -6      /* call not valid in the handle's current state */
} ns_status;

/* field ids for ns_set_state / ns_get_state */
enum {
  NS_U = 0, NS_V = 1, NS_W = 2, NS_P = 3,  /* state (set / get) */
  NS_FX = 4, NS_FY = 5, NS_FZ = 6,         /* face-centred body force (set / get) */
  NS_F = 7, NS_G = 8, NS_H = 9, NS_RHS = 10 /* last predictor and rhs (get; set for stage tests) */
};
enum { NS_BC_WALL = 0, NS_BC_PERIODIC = 1 };
enum { NS_FP64 = 0, NS_MIXED = 1 };
enum {
  NS_ALLOW_UNSTABLE = 1, /* accept a fixed dt beyond the stability bounds */
  NS_TIMING = 2,         /* record per-stage GPU times (ns_get_timing) */
  NS_BATCH_LAUNCHES = 4, /* several instances (flag of instance 0): one launch per stage and per
                            pass of sweeps, polled by the host, instead of the persistent launch */
  NS_GENERATED = 8,      /* one instance: the projection too is the kernel the build generates
                            from its kernel descriptor (UPDATE_VELOCITY) instead of the
                            hand-written one (same results); the predictor of the conservative
                            form is always the generated PREDICT_VELOCITY kernel */
  NS_ADVECTIVE = 16,     /* one instance: the convective term in advective form weighted by
                            alpha = gamma (SOLA / NASA-VOF2D) instead of conservative fluxes
                            blended by gamma; not with checkpoint_every */
  NS_RK2 = 32            /* one instance: two-stage SSP Runge-Kutta (Heun) time integration,
                            the method-of-lines integrator of the Cactus framework the paper
                            builds on ("Cactus Computational Framework"): two projected Euler
                            stages with the same dt (the adaptive dt from u^n), then
                            u^{n+1} = (u^n + u^(2)) / 2 and the boundary fill; the pressure is
                            the second stage's.  A step's sweeps count both solves.  Not with
                            checkpoint_every or ns_step_noalloc */
};

typedef struct {
  uint32_t struct_size;   /* = sizeof(ns_params); ABI version check */
  int32_t nx, ny, nz;     /* interior cells per axis, >= 2; even on periodic axes */
  double lx, ly, lz;      /* domain extent */
  double re;              /* Reynolds number; nu = 1 / re (rho = 1, phi = p) */
  double dt;              /* > 0: fixed step; <= 0: adaptive with tau */
  double tau;             /* adaptive safety factor in (0, 1] */
  double gamma;           /* donor-cell blend in [0, 1] (NS_ADVECTIVE: the upwind weight alpha) */
  double omega;           /* SOR relaxation in (0, 2) */
  double tol;             /* stop when RMS residual <= tol * RMS(rhs) */
  int32_t itermax;        /* SOR sweeps per step (mixed: inner sweeps in total) */
  int32_t bc[3];          /* NS_BC_WALL / NS_BC_PERIODIC per axis x, y, z */
  double wall_vel[6][3];  /* wall velocity on faces -x,+x,-y,+y,-z,+z (tangential parts used) */
  double g[3];            /* constant body force */
  double eta;             /* mixed: inner stop at eta * outer residual (0 < eta < 1) */
  int32_t precision;      /* NS_FP64 or NS_MIXED */
  int32_t checkpoint_every; /* > 0: record checkpoints every k steps for ns_backward */
  int32_t flags;          /* NS_ALLOW_UNSTABLE | NS_TIMING */
  int32_t tile[2];        /* SOR sweep shape: {rows, z chunk}.  z chunk k > 0: chunks of k
                             planes; k < 0: each domain split into the fewest equal chunks of
                             at most -k planes; 0: the whole column (two-sweep shapes on a
                             single-domain handle: an equal share of the plane-columns per
                             resident workgroup).
                             rows 4, 8 or 12: one sweep per launch, that many interior rows
                             per workgroup; rows 16, 24 or 32 (NS_FP64: 16 only): two
                             sweeps per launch (temporal blocking), that many rows per
                             workgroup including a 4-row halo on each side (periodic axes
                             need >= 4 cells);
                             {0, 0} = chosen by the autotuner; rows = -1 selects the unfused
                             one-pass-per-colour sweeps (reference path). The fused shapes
                             address a plane with 31-bit byte offsets: larger planes need
                             rows = -1. Sweep counts and iterates do not depend on it beyond
                             rounding. */
} ns_params;

typedef struct {
  double t;               /* simulated time since creation */
  double dt_last;         /* last step size */
  double res_last;        /* last RMS residual of the pressure equation */
  int64_t sweeps_total;   /* SOR sweeps whose result was used */
  int32_t steps;          /* completed steps */
  int32_t sweeps_max;     /* most sweeps in one step */
  int32_t steps_unconverged; /* steps that stopped at itermax above the tolerance */
  int32_t outer_max;      /* mixed: most defect-correction iterations in one step */
} ns_stats;

/* Stage timers (NS_TIMING): GPU milliseconds and launch counts summed over
 * all ns_step calls, measured with HIP events on the handle's stream around
 * each stage's launches. */
enum { NS_T_BC = 0, NS_T_FGH = 1, NS_T_RHS = 2, NS_T_SOR = 3, NS_T_DEFECT = 4,
       NS_T_PROJECT = 5, NS_T_OTHER = 6, NS_T_COUNT = 8 };
typedef struct {
  double ms[NS_T_COUNT];
  int64_t launches[NS_T_COUNT];
  int64_t sor_bytes;     /* algorithmic HBM bytes of the SOR launches timed */
  int32_t sor_tile[2];   /* sweep shape in use on instance 0 (see ns_params.tile); a batched
                            handle may report sor_tile[1] = -k: each domain split into the
                            fewest equal z chunks of at most k planes */
} ns_timing;

/* Source: the lid-driven cavity at Re 100 of the paper's "Code Validation
 * and Verification" section (grid, dt and solver settings are an extension:
 * the paper prints none).
 * Fill *p with the defaults of the 16^3 lid-driven cavity (Re 100, dt 0.01,
 * gamma 0.5, omega 1.7, tol 1e-6, 200 sweeps, lid (1,0,0) on +z, FP64).
 * Host only; never fails for a non-NULL pointer. */
ns_status ns_params_default(ns_params *p);

/* Source: the problem eq. (1) states ("Background and Governing Equations":
 * nu, body force f, phi = p / rho with rho = 1) on the regular staggered grid
 * with one ghost layer ("MPI-Based Data Parallelism in Cactus"); several
 * instances per handle are an extension (many independent cavities).
 * Create a solver for n_instances independent domains (params[n_instances]).
 * hip_stream: a hipStream_t (NULL = the default stream) that every call of
 * this handle uses.  Validates every parameter (NS_E_INVALID), checks the
 * explicit stability bounds of a fixed dt -- diffusion number
 * nu dt sum 1/h^2 <= 1/2 (NS_E_UNSTABLE unless NS_ALLOW_UNSTABLE) -- and
 * allocates all device memory (NS_E_OOM).  The state starts at zero with the
 * boundary fill applied. */
ns_status ns_create(const ns_params *params, int32_t n_instances, void *hip_stream,
                    ns_solver **out);

/* Source: the staggered (MAC) placement of velocity and pressure the
 * paragraph after eq. (1) names; the ghost layer as above.
 * Copy one field of instance inst in (layout above).  Setting u, v or w
 * starts a new recording epoch for ns_backward. */
ns_status ns_set_state(ns_solver *s, int32_t inst, int32_t field, const double *src,
                       int32_t on_device);

/* Source: one time step of the CFD code ("CFD Implementation"; eq. (1));
 * its last stage is the UPDATE_VELOCITY kernel of the descriptor listing in
 * "CaCUDA Kernel Abstraction".
 * Advance every instance nsteps steps.  stats: NULL or an array of
 * n_instances entries that receives the cumulative statistics.  Returns
 * NS_E_NONFINITE if a NaN/Inf appears (stats.steps counts completed steps). */
ns_status ns_step(ns_solver *s, int32_t nsteps, ns_stats *stats);

/* Source: as ns_set_state.
 * Copy one field of instance inst out (layout above). */
ns_status ns_get_state(const ns_solver *s, int32_t inst, int32_t field, double *dst,
                       int32_t on_device);

/* Source: an extension beyond the paper (the paper has no adjoint): the
 * transpose of the step ns_step computes.
 * Reverse-mode gradient of a loss of the final velocity with respect to the
 * velocity set at the start of the current recording epoch:
 * g_final[3] = dL/d(u,v,w)(T) (padded layout; only unknowns are read),
 * g_init[3]  = out: dL/d(u,v,w)(0) (zero off the unknowns).
 * The adjoint of one step is P^T J^T with P the exact projection (symmetric:
 * the same divergence, SOR and projection with dt = 1) and J the predictor
 * Jacobian transposed in gather form; forward states are recomputed from
 * checkpoints taken every checkpoint_every steps.  Requires
 * checkpoint_every > 0, a fixed dt and NS_FP64 (else NS_E_INVALID), and at
 * least one recorded step since the velocity was last set (else
 * NS_E_STATE).  Does not change the forward state. */
ns_status ns_backward(ns_solver *s, int32_t inst, const double *const g_final[3],
                      double *const g_init[3], int32_t on_device);

/* Source: an extension for measurement (the paper reports whole-code
 * GFlop/s in "Performance and Scalability", no per-stage times).
 * Stage timers accumulated while NS_TIMING is set on instance 0.  Returns
 * NS_E_INVALID for a NULL handle or out pointer. */
ns_status ns_get_timing(const ns_solver *s, ns_timing *out);

/* A debugging aid (no passage of the paper: a check of the library itself).
 * While the environment variable NS_GUARD is set (to anything but "" or
 * "0"), every device buffer the library allocates lies between two 4 KiB
 * guard bands of a fixed byte pattern; a buffer's bands are compared with
 * the pattern when it is freed (ns_destroy).  Returns the number of bands
 * found changed since the process started -- bands of freed buffers, plus
 * those of live buffers checked now, after a device synchronisation -- so
 * 0 means no device write went past either end of a buffer.  self_test != 0
 * (with NS_GUARD set) first allocates a guarded buffer, sets the byte just
 * past its end with a host-side fill and frees it, which adds one to the
 * count.  Not for use while another thread runs a handle on the device.
 * Buffers allocated while NS_GUARD was unset have no bands. */
int64_t ns_guard_check(int32_t self_test);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the step of ns_step for one FP64 domain
 * without a handle and without any allocation.
 * params: one instance, precision NS_FP64, checkpoint_every 0, no NS_TIMING
 * (else NS_E_INVALID); validated and stability-checked as in ns_create.
 * u, v, w, p: device memory of the current device, FP64, the padded layout
 * above, read and overwritten in place with the state after nsteps steps
 * (the result equals ns_create + ns_set_state of u, v, w, p + ns_step +
 * ns_get_state).  hip_stream: the stream every launch goes to (NULL = the
 * default stream); the call returns after the steps are done.  stats: NULL
 * or one ns_stats that receives this call's statistics.
 * Scratch: F, G, H, rhs, a second pressure buffer, partial sums and the
 * control block live in one static device array of 21.5 MB per device (held
 * until the process ends), so (nx+2)(ny+2)(nz+2) must not exceed 524288
 * (e.g. 78^3 interior cells); larger grids return NS_E_INVALID.  The array
 * keeps the last call's contents and is cleared at the start of each call.
 * Calls on one device share it: the library serialises its own calls per
 * device with a lock, and any other use of the array that overlapped a call
 * would race.  Errors: NS_E_INVALID (arguments, sizes, pointers that are not
 * memory of the current device), NS_E_NONFINITE, NS_E_DEVICE; the message is
 * ns_last_error(NULL).  No hipMalloc, hipFree, pinned-host or other device
 * allocation happens in the call (the first call on a device looks up the
 * array's address and builds the host-side solver shell once). */
ns_status ns_step_noalloc(const ns_params *params, double *u, double *v, double *w, double *p,
                          int32_t nsteps, void *hip_stream, ns_stats *stats);

/* Frees every device buffer and host resource of the handle; NULL is a
 * no-op.  The handle's stream is the caller's and is not destroyed. */
void ns_destroy(ns_solver *s);

/* Message of the last failure of this handle (or of the last ns_create
 * when s is NULL); never NULL. */
const char *ns_last_error(const ns_solver *s);

#ifdef __cplusplus
}
#endif
#endif
