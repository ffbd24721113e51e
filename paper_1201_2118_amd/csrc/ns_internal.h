// ns_internal.h -- shared declarations of the gfx950 HIP implementation of
// the staggered-grid Navier-Stokes step (kernels + host runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ns.h"

namespace ns {

// Grid geometry passed by value to every kernel.  Fields use the padded
// layout [nz+2][ny+2][nx+2], x fastest: index = k*sxy + j*sx + i.
struct Geo {
  int nx, ny, nz;
  long sx, sxy, ntot;
  double dx, dy, dz;
  double idx, idy, idz;     // 1/h
  double idx2, idy2, idz2;  // 1/h^2
  int per[3];               // 1 = periodic axis
  int hi[3];                // last normal-velocity unknown of u, v, w along its own axis
};

// Per-instance device control block.  Written by the last workgroup of the
// reduction kernels; read by later kernels of the same step and polled by
// the host (one small async copy per chunk of sweeps).
struct Ctl {
  double dt;       // current step size
  double thr;      // absolute stop threshold of the Poisson solve: tol * RMS(rhs)
  double thr_in;   // mixed: inner threshold eta * outer residual
  double res;      // RMS residual of the accepted pressure (or of the last outer check)
  double rhs_rms;  // RMS of the right-hand side
  double res_in;   // mixed: last inner residual checked
  double umax[3];  // adaptive dt: max |u|, |v|, |w|
  int32_t done;    // solve (FP64) or inner loop (mixed) finished
  int32_t final_;  // sweep index whose iterate is the answer
  int32_t nonfinite;
  int32_t outer_done;  // mixed: outer residual met the tolerance
  uint32_t ticket;     // last-workgroup counter of reductions (reset by the last group)
  int32_t pad_[3];
};

// Tunables of the red-black sweep (chosen per grid by the autotuner).
// ty > 0: fused single-pass kernel with ty interior rows per workgroup (the
// x width is fixed at 60 = 64 - 4 halo) and zc planes per z chunk (0 =
// whole column); ty < 0: unfused reference kernels (one pass per colour).
struct SorShape {
  int ty;
  int zc;
};

// ---- kernel launchers (kernels.hip / sor.hip / adjoint.hip) ----
// All launchers enqueue on `st` and return the hipGetLastError() status.
template <class T> hipError_t launch_bc_vel(hipStream_t st, const Geo& g, T* u, T* v, T* w,
                                           const double wall[6][3]);
template <class T> hipError_t launch_p_ghosts(hipStream_t st, const Geo& g, T* p);
template <class T> hipError_t launch_fgh(hipStream_t st, const Geo& g, const T* u, const T* v,
                                        const T* w, const T* fx, const T* fy, const T* fz,
                                        T* F, T* G, T* H, const Ctl* ctl, double re, double gamma,
                                        const double gforce[3]);
template <class T> hipError_t launch_rhs(hipStream_t st, const Geo& g, const T* F, const T* G,
                                        const T* H, T* rhs, Ctl* ctl, double* part, double tol,
                                        double dt_scale_one);
template <class T> hipError_t launch_project(hipStream_t st, const Geo& g, const T* F, const T* G,
                                            const T* H, const double* p, T* u, T* v, T* w,
                                            const Ctl* ctl, double dt_scale_one);
template <class T> hipError_t launch_umax(hipStream_t st, const Geo& g, const T* u, const T* v,
                                         const T* w, Ctl* ctl, double* part, double re,
                                         double tau, const double wall[6][3]);

// One red-black SOR sweep p_in -> p_out (out of place) on A p = rhs, fused
// with the RMS residual of p_in.  sweep_idx = index m of this sweep (1-based):
// the residual computed is that of iterate m-1; the last workgroup decides
// convergence (iterate m-1 accepted when m-1 >= 1 and res <= thr) and sets
// ctl->done / ctl->final_.  write = 0 computes only the residual (used after
// the last allowed sweep).  zero_in = 1 treats p_in as identically zero (it
// is not read).  thr_is_inner selects ctl->thr_in.
template <class T> hipError_t launch_sor_sweep(hipStream_t st, const Geo& g, const T* p_in, T* p_out,
                                              const T* rhs, Ctl* ctl, double* part, double omega,
                                              int sweep_idx, int itermax, int write, int zero_in,
                                              int thr_is_inner, const SorShape& shape);
// Mixed-precision outer step: p_out = p_in + e (e == null: p_out unused and
// not written), r = rhs - A p_out in FP64 stored as float, RMS(r) -> ctl.
hipError_t launch_defect(hipStream_t st, const Geo& g, const double* p_in, const float* e,
                         double* p_out, const float* rhs, float* r, Ctl* ctl, double* part,
                         double eta);

size_t reduce_blocks(const Geo& g);  // partial-sum slots any reduction may need
int sor_num_blocks(const Geo& g, const SorShape& s);
// Fused sweep (one pass): shape.ty rows per workgroup in {4, 8, 12},
// shape.zc planes per z chunk (0 = whole column).
template <class T> hipError_t launch_sor_fused(hipStream_t st, const Geo& g, const T* p_in, T* p_out,
                                              const T* rhs, Ctl* ctl, double* part, double omega,
                                              int sweep_idx, int itermax, int write, int zero_in,
                                              int thr_is_inner, const SorShape& shape);
int fused_num_blocks(const Geo& g, const SorShape& s);
bool fused_shape_ok(const SorShape& s);
int fused_resident(int ty, bool f32);       // workgroups resident on the device at once
int fused_columns(const Geo& g, int ty);    // x-y tiles of one z chunk

// One domain of a batched sweep (device-resident table, sorted by `first`).
struct BatchItem {
  Geo g;
  void* p[2];      // iterate buffers; sweep m reads p[(cur + m - 1) & 1], writes p[(cur + m) & 1]
  const void* rhs;
  Ctl* ctl;
  double* part;
  double omega;
  int cur;
  int first;       // first workgroup of this domain
  int ntiles, ntx, nty, zc;
  int budget;      // the solve stops at iterate `budget` at the latest
  int inner;       // 1: correction solve (stop at ctl->thr_in)
};
// Fill ntx, nty, zc and ntiles of an item for a sweep shape.
void batch_item_shape(BatchItem& it, int ty, int zc);
// One sweep of every domain of a batch in one launch (nblocks = sum of ntiles).
template <class T> hipError_t launch_sor_batched(hipStream_t st, const BatchItem* d_items, int nitems,
                                                int nblocks, int ty, int m, int write, int zero_in);

// Adjoint of the predictor in gather form (FP64 only): z = B^T J_Phi(u)^T mu.
hipError_t launch_adj_fgh(hipStream_t st, const Geo& g, const double* u, const double* v,
                          const double* w, const double* mu, const double* mv, const double* mw,
                          double* zu, double* zv, double* zw, double dt, double re, double gamma);
hipError_t launch_adj_fold(hipStream_t st, const Geo& g, double* zu, double* zv, double* zw);
// Zero every entry that is not an unknown of component comp (3 = cells).
hipError_t launch_mask_unknowns(hipStream_t st, const Geo& g, double* q, int comp);
// Periodic images of face / cell fields (full extent), axis by axis.
template <class T> hipError_t launch_periodic(hipStream_t st, const Geo& g, T* q, int axis);
template <class T> hipError_t launch_divergence(hipStream_t st, const Geo& g, const T* u, const T* v,
                                               const T* w, T* out);

}  // namespace ns
