// cells.h -- per-cell work of the stages other than the sweeps (predictor,
// Poisson right-hand side, projection, adaptive dt, mixed-precision defect),
// shared by the single-domain kernels, the batched stage kernels and the
// persistent batched kernel.  Each reducing stage is split into the cells
// of one block (returning the thread's partial) and the finish that turns
// the domain's total into control-block fields, so a caller can reduce in
// its own way.  Blocks are 64 lanes in x times blockDim.y rows in y.
#pragma once

#include <hip/hip_runtime.h>

#include "ns_internal.h"
#include "reduce.h"

namespace ns {

namespace {

// ---------------------------------------------------------------------------
// Momentum predictor.  For the unknown q of component c and direction d the
// convective flux through the half-way point between q and q[+d] blends
// central and donor-cell differencing:
//     flux(t, a, b) = t (a + b)/2 + gamma |t| (a - b)/2,
// t = the d-velocity interpolated to that point (mean of the two d-faces at
// pos and pos + e_c; for d == c the mean of q and q[+d]).
// F_c = q + dt (nu lap q - sum_d (flux_hi - flux_lo)/h_d + g_c + f_c).
// The predictor's expressions fuse multiply-adds only within one source
// expression (contract(on)), so every kernel that inlines them (the
// hand-written ones, the generated ones) rounds each value alike whatever
// code surrounds it.
__device__ __forceinline__ double flux(double t, double a, double b, double gamma) {
#pragma clang fp contract(on)
  return 0.5 * (t * (a + b) + gamma * fabs(t) * (a - b));
}

// The predictor's value of each component at cell c (u, v, w with a
// one-cell neighbourhood of c inside the padded arrays), in FP64.  HAS_F:
// body-force fields fx, fy, fz are present (all three or none), a
// compile-time choice so the loop body carries no per-cell branch.
template <class T, bool HAS_F>
__device__ __forceinline__ double F_at(const Geo& g, long c, const T* __restrict__ u, const T* __restrict__ v,
                                       const T* __restrict__ w, const T* __restrict__ fx, double dt, double nu,
                                       double gamma, double gx) {
#pragma clang fp contract(on)
  const long sx = g.sx, sxy = g.sxy;
  const double q = u[c], qe = u[c + 1], qw = u[c - 1], qn = u[c + sx], qs = u[c - sx], qt = u[c + sxy],
               qb = u[c - sxy];
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double cx = (flux(0.5 * (q + qe), q, qe, gamma) - flux(0.5 * (qw + q), qw, q, gamma)) * g.idx;
  const double vn = 0.5 * ((double)v[c] + (double)v[c + 1]);
  const double vs = 0.5 * ((double)v[c - sx] + (double)v[c - sx + 1]);
  const double cy = (flux(vn, q, qn, gamma) - flux(vs, qs, q, gamma)) * g.idy;
  const double wt = 0.5 * ((double)w[c] + (double)w[c + 1]);
  const double wb = 0.5 * ((double)w[c - sxy] + (double)w[c - sxy + 1]);
  const double cz = (flux(wt, q, qt, gamma) - flux(wb, qb, q, gamma)) * g.idz;
  const double f = gx + (HAS_F ? (double)fx[c] : 0.0);
  return q + dt * (nu * lap - cx - cy - cz + f);
}
template <class T, bool HAS_F>
__device__ __forceinline__ double G_at(const Geo& g, long c, const T* __restrict__ u, const T* __restrict__ v,
                                       const T* __restrict__ w, const T* __restrict__ fy, double dt, double nu,
                                       double gamma, double gy) {
#pragma clang fp contract(on)
  const long sx = g.sx, sxy = g.sxy;
  const double q = v[c], qe = v[c + 1], qw = v[c - 1], qn = v[c + sx], qs = v[c - sx], qt = v[c + sxy],
               qb = v[c - sxy];
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double ue = 0.5 * ((double)u[c] + (double)u[c + sx]);
  const double uw = 0.5 * ((double)u[c - 1] + (double)u[c - 1 + sx]);
  const double cx = (flux(ue, q, qe, gamma) - flux(uw, qw, q, gamma)) * g.idx;
  const double cy = (flux(0.5 * (q + qn), q, qn, gamma) - flux(0.5 * (qs + q), qs, q, gamma)) * g.idy;
  const double wt = 0.5 * ((double)w[c] + (double)w[c + sx]);
  const double wb = 0.5 * ((double)w[c - sxy] + (double)w[c - sxy + sx]);
  const double cz = (flux(wt, q, qt, gamma) - flux(wb, qb, q, gamma)) * g.idz;
  const double f = gy + (HAS_F ? (double)fy[c] : 0.0);
  return q + dt * (nu * lap - cx - cy - cz + f);
}
template <class T, bool HAS_F>
__device__ __forceinline__ double H_at(const Geo& g, long c, const T* __restrict__ u, const T* __restrict__ v,
                                       const T* __restrict__ w, const T* __restrict__ fz, double dt, double nu,
                                       double gamma, double gz) {
#pragma clang fp contract(on)
  const long sx = g.sx, sxy = g.sxy;
  const double q = w[c], qe = w[c + 1], qw = w[c - 1], qn = w[c + sx], qs = w[c - sx], qt = w[c + sxy],
               qb = w[c - sxy];
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double ue = 0.5 * ((double)u[c] + (double)u[c + sxy]);
  const double uw = 0.5 * ((double)u[c - 1] + (double)u[c - 1 + sxy]);
  const double cx = (flux(ue, q, qe, gamma) - flux(uw, qw, q, gamma)) * g.idx;
  const double vn = 0.5 * ((double)v[c] + (double)v[c + sxy]);
  const double vs = 0.5 * ((double)v[c - sx] + (double)v[c - sx + sxy]);
  const double cy = (flux(vn, q, qn, gamma) - flux(vs, qs, q, gamma)) * g.idy;
  const double cz = (flux(0.5 * (q + qt), q, qt, gamma) - flux(0.5 * (qb + q), qb, q, gamma)) * g.idz;
  const double f = gz + (HAS_F ? (double)fz[c] : 0.0);
  return q + dt * (nu * lap - cx - cy - cz + f);
}

template <class T, bool HAS_F>
__device__ __forceinline__ void fgh_cells(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ u,
                                          const T* __restrict__ v, const T* __restrict__ w,
                                          const T* __restrict__ fx, const T* __restrict__ fy,
                                          const T* __restrict__ fz, T* __restrict__ F, T* __restrict__ G,
                                          T* __restrict__ H, const Ctl* __restrict__ ctl, double nu, double gamma,
                                          double gx, double gy, double gz) {
  const double dt = ctl->dt;
  // All three components are formed at every cell (their stencils stay
  // inside the padded arrays) and stored where they are unknowns: the body
  // is one straight block, so the loads of all three are in flight together.
  for_cells<2>(g, zr, blk, [&](int ci, int cj, int ck, long c) {
    const double Fv = F_at<T, HAS_F>(g, c, u, v, w, fx, dt, nu, gamma, gx);
    const double Gv = G_at<T, HAS_F>(g, c, u, v, w, fy, dt, nu, gamma, gy);
    const double Hv = H_at<T, HAS_F>(g, c, u, v, w, fz, dt, nu, gamma, gz);
    if (ci <= g.hi[0]) F[c] = T(Fv);
    if (cj <= g.hi[1]) G[c] = T(Gv);
    if (ck <= g.hi[2]) H[c] = T(Hv);
  });
}

// The advective form of the convective term (the SOLA / NASA-VOF2D form):
// sum_d a_d dq/dx_d, with a_d the d-velocity at the unknown's position (the
// unknown itself along its own axis, else the mean of the four d-faces
// around it) and the derivative an alpha-weighted blend of the backward and
// forward differences: a [(1 + alpha s)(q - q[-d]) + (1 - alpha s)(q[+d] - q)] / (2 h),
// s = sign(a) with sign(0) = 0 (alpha 0: central, 1: upwind).
__device__ __forceinline__ double adv_d(double a, double qm, double qc, double qp, double alpha, double ih) {
  const double s = (double)((a > 0.0) - (a < 0.0));
  return a * ((1.0 + alpha * s) * (qc - qm) + (1.0 - alpha * s) * (qp - qc)) * (0.5 * ih);
}

// Predictor with the advective form (alpha in place of gamma); otherwise as
// fgh_cells.
template <class T, bool HAS_F>
__device__ __forceinline__ void fgh_adv_cells(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ u,
                                              const T* __restrict__ v, const T* __restrict__ w,
                                              const T* __restrict__ fx, const T* __restrict__ fy,
                                              const T* __restrict__ fz, T* __restrict__ F, T* __restrict__ G,
                                              T* __restrict__ H, const Ctl* __restrict__ ctl, double nu,
                                              double alpha, double gx, double gy, double gz) {
  const double dt = ctl->dt;
  const long sx = g.sx, sxy = g.sxy;
  for_cells<2>(g, zr, blk, [&](int ci, int cj, int ck, long c) {
    double Fv, Gv, Hv;
    {  // F on the x face i
      const double q = u[c], qe = u[c + 1], qw = u[c - 1], qn = u[c + sx], qs = u[c - sx],
                   qt = u[c + sxy], qb = u[c - sxy];
      const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 +
                         (qt - 2.0 * q + qb) * g.idz2;
      const double ay = 0.25 * ((double)v[c] + (double)v[c + 1] + (double)v[c - sx] + (double)v[c - sx + 1]);
      const double az = 0.25 * ((double)w[c] + (double)w[c + 1] + (double)w[c - sxy] + (double)w[c - sxy + 1]);
      const double conv = adv_d(q, qw, q, qe, alpha, g.idx) + adv_d(ay, qs, q, qn, alpha, g.idy) +
                          adv_d(az, qb, q, qt, alpha, g.idz);
      const double f = gx + (HAS_F ? (double)fx[c] : 0.0);
      Fv = q + dt * (nu * lap - conv + f);
    }
    {  // G on the y face j
      const double q = v[c], qe = v[c + 1], qw = v[c - 1], qn = v[c + sx], qs = v[c - sx],
                   qt = v[c + sxy], qb = v[c - sxy];
      const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 +
                         (qt - 2.0 * q + qb) * g.idz2;
      const double ax = 0.25 * ((double)u[c] + (double)u[c + sx] + (double)u[c - 1] + (double)u[c - 1 + sx]);
      const double az = 0.25 * ((double)w[c] + (double)w[c + sx] + (double)w[c - sxy] + (double)w[c - sxy + sx]);
      const double conv = adv_d(ax, qw, q, qe, alpha, g.idx) + adv_d(q, qs, q, qn, alpha, g.idy) +
                          adv_d(az, qb, q, qt, alpha, g.idz);
      const double f = gy + (HAS_F ? (double)fy[c] : 0.0);
      Gv = q + dt * (nu * lap - conv + f);
    }
    {  // H on the z face k
      const double q = w[c], qe = w[c + 1], qw = w[c - 1], qn = w[c + sx], qs = w[c - sx],
                   qt = w[c + sxy], qb = w[c - sxy];
      const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 +
                         (qt - 2.0 * q + qb) * g.idz2;
      const double ax = 0.25 * ((double)u[c] + (double)u[c + sxy] + (double)u[c - 1] + (double)u[c - 1 + sxy]);
      const double ay = 0.25 * ((double)v[c] + (double)v[c + sxy] + (double)v[c - sx] + (double)v[c - sx + sxy]);
      const double conv = adv_d(ax, qw, q, qe, alpha, g.idx) + adv_d(ay, qs, q, qn, alpha, g.idy) +
                          adv_d(q, qb, q, qt, alpha, g.idz);
      const double f = gz + (HAS_F ? (double)fz[c] : 0.0);
      Hv = q + dt * (nu * lap - conv + f);
    }
    if (ci <= g.hi[0]) F[c] = T(Fv);
    if (cj <= g.hi[1]) G[c] = T(Gv);
    if (ck <= g.hi[2]) H[c] = T(Hv);
  });
}

// ---------------------------------------------------------------------------
// Poisson right-hand side rhs = (div F) / dt on every cell (the face below
// cell 1 of a periodic axis is face n), with the RMS of rhs reduced into the
// control block: thr = tol * max(RMS, 1e-300); an identically zero rhs
// finishes the solve before any sweep.  unit_dt != 0 uses dt = 1 (the
// adjoint projection).
// rhs_acc: the cells of one block; returns this thread's sum of rhs^2.
template <class T>
__device__ __forceinline__ double rhs_acc(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ F,
                                          const T* __restrict__ G, const T* __restrict__ H, T* __restrict__ rhs,
                                          const Ctl* ctl, int unit_dt) {
  const double idt = unit_dt ? 1.0 : 1.0 / ctl->dt;
  double acc = 0.0;
  for_cells(g, zr, blk, [&](int ci, int cj, int ck, long c) {
    const long cw = (ci > 1 || !g.per[0]) ? c - 1 : c + (g.nx - 1);
    const long cs = (cj > 1 || !g.per[1]) ? c - g.sx : c + (long)(g.ny - 1) * g.sx;
    const long cb = (ck > 1 || !g.per[2]) ? c - g.sxy : c + (long)(g.nz - 1) * g.sxy;
    const double d = ((double)F[c] - (double)F[cw]) * g.idx + ((double)G[c] - (double)G[cs]) * g.idy +
                     ((double)H[c] - (double)H[cb]) * g.idz;
    const T r = T(d * idt);
    rhs[c] = r;
    acc += (double)r * (double)r;
  });
  return acc;
}
// The control block's fields set from the domain's sum of rhs^2 (every
// field the solve starts from except the ticket).
__device__ __forceinline__ void rhs_finish(Ctl* ctl, double tot, long n, double tol) {
  const double rms = sqrt(tot / (double)n);
  ctl->rhs_rms = rms;
  ctl->thr = tol * (rms > 1e-300 ? rms : 1e-300);
  ctl->res = 0.0;
  ctl->final_ = 0;
  ctl->nonfinite = !isfinite(rms);
  ctl->done = (rms == 0.0) || !isfinite(rms);
  ctl->outer_done = ctl->done;
}
template <class T>
__device__ __forceinline__ void rhs_cells(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ F,
                                          const T* __restrict__ G, const T* __restrict__ H, T* __restrict__ rhs,
                                          Ctl* ctl, double* part, double tol, int unit_dt, double* sh,
                                          int* sh_last) {
  const long n = (long)g.nx * g.ny * g.nz;
  const double acc = rhs_acc<T>(g, zr, blk, F, G, H, rhs, ctl, unit_dt);
  double s = block_sum(acc, sh);
  if (publish_partial(part, blk.id, s, ctl, blk.count, sh_last)) {
    double tot = sum_partials(part, blk.count, sh);
    if (flat_tid() == 0) {
      rhs_finish(ctl, tot, n, tol);
      ctl->ticket = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Projection (UPDATE_VELOCITY): u = F - dt (p[+x] - p) / dx on the unknowns
// of each component; p ghosts hold periodic images where needed.
template <class T>
__device__ __forceinline__ void project_cells(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ F,
                                              const T* __restrict__ G, const T* __restrict__ H,
                                              const double* __restrict__ p, T* __restrict__ u, T* __restrict__ v,
                                              T* __restrict__ w, const Ctl* __restrict__ ctl, int unit_dt) {
  const double dt = unit_dt ? 1.0 : ctl->dt;
  for_cells(g, zr, blk, [&](int ci, int cj, int ck, long c) {
    const double pc = p[c];
    if (ci <= g.hi[0]) u[c] = T((double)F[c] - dt * (p[c + 1] - pc) * g.idx);
    if (cj <= g.hi[1]) v[c] = T((double)G[c] - dt * (p[c + g.sx] - pc) * g.idy);
    if (ck <= g.hi[2]) w[c] = T((double)H[c] - dt * (p[c + g.sxy] - pc) * g.idz);
  });
}

// Adaptive step: tau * min(diffusive limit, h_d / max|u_d|) with the maxima
// over the unknowns and the wall speeds.
// umax_acc: this thread's maxima of |u|, |v|, |w| over the unknowns of one
// block, folded into m.
template <class T>
__device__ __forceinline__ void umax_acc(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ u,
                                         const T* __restrict__ v, const T* __restrict__ w, double m[3]) {
  for_cells(g, zr, blk, [&](int ci, int cj, int ck, long c) {
    if (ci <= g.hi[0]) m[0] = fmax(m[0], fabs((double)u[c]));
    if (cj <= g.hi[1]) m[1] = fmax(m[1], fabs((double)v[c]));
    if (ck <= g.hi[2]) m[2] = fmax(m[2], fabs((double)w[c]));
  });
}
// dt from the domain's maxima mm (control block fields dt and umax).
__device__ __forceinline__ void umax_finish(Ctl* ctl, const double mm[3], const Geo& g, double re, double tau,
                                            double wu, double wv, double ww) {
  const double wall[3] = {wu, wv, ww};
  const double h[3] = {g.dx, g.dy, g.dz};
  double lim = (re / 2.0) / (g.idx2 + g.idy2 + g.idz2);
  for (int d = 0; d < 3; d++) {
    const double md = fmax(mm[d], wall[d]);
    ctl->umax[d] = md;
    if (md > 0.0) lim = fmin(lim, h[d] / md);
  }
  ctl->dt = tau * lim;
}
template <class T>
__device__ __forceinline__ void umax_cells(const Geo& g, int zr, const CellBlk& blk, const T* __restrict__ u,
                                           const T* __restrict__ v, const T* __restrict__ w, Ctl* ctl,
                                           double* part, double re, double tau, double wu, double wv, double ww,
                                           double* sh, int* sh_last) {
  double m[3] = {0.0, 0.0, 0.0};
  umax_acc<T>(g, zr, blk, u, v, w, m);
  double r[3];
  for (int d = 0; d < 3; d++) r[d] = block_max(m[d], sh);
  const unsigned bid = blk.id;
  const unsigned nb = blk.count;
  if (flat_tid() == 0) {
    part[bid] = r[0];
    part[nb + bid] = r[1];
    part[2 * nb + bid] = r[2];
  }
  if (publish_partial(part + 3 * nb, bid, 0.0, ctl, nb, sh_last)) {
    double mm[3];
    for (int d = 0; d < 3; d++) mm[d] = max_partials(part + d * nb, nb, sh);
    if (flat_tid() == 0) {
      umax_finish(ctl, mm, g, re, tau, wu, wv, ww);
      ctl->ticket = 0;
    }
  }
}

// Neighbour offsets and coefficients of cell (i, j, k): a missing neighbour
// (wall) gets coefficient 0 and points at the cell itself so that the load
// stays in bounds and finite.
struct Nb {
  long o[6];
  double a[6];
  double ac;
};

__device__ __forceinline__ Nb neighbours(const Geo& g, int i, int j, int k) {
  Nb n;
  const int sz[3] = {g.nx, g.ny, g.nz};
  const int id[3] = {i, j, k};
  const long st[3] = {1, g.sx, g.sxy};
  const double h2[3] = {g.idx2, g.idy2, g.idz2};
  n.ac = 0.0;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    // minus side
    if (id[d] > 1) { n.o[2 * d] = -st[d]; n.a[2 * d] = h2[d]; }
    else if (g.per[d]) { n.o[2 * d] = (long)(sz[d] - 1) * st[d]; n.a[2 * d] = h2[d]; }
    else { n.o[2 * d] = 0; n.a[2 * d] = 0.0; }
    // plus side
    if (id[d] < sz[d]) { n.o[2 * d + 1] = st[d]; n.a[2 * d + 1] = h2[d]; }
    else if (g.per[d]) { n.o[2 * d + 1] = -(long)(sz[d] - 1) * st[d]; n.a[2 * d + 1] = h2[d]; }
    else { n.o[2 * d + 1] = 0; n.a[2 * d + 1] = 0.0; }
    n.ac += n.a[2 * d] + n.a[2 * d + 1];
  }
  return n;
}

// Mixed-precision outer step: p_out = p_in + e, r = rhs - A p_out (FP64
// arithmetic, stored as FP32), RMS of the FP64 r into ctl->res; decides
// outer convergence and sets the inner threshold eta * RMS(r).
// HAS_E: p_out = p_in + e is formed and stored (e non-null); else p = p_in.
// A compile-time choice, so the loop body carries no per-load branch and
// its loads can be in flight together.
// defect_acc: the cells of one block; returns this thread's sum of r^2.
template <bool HAS_E>
__device__ __forceinline__ double defect_acc(const Geo& g, int zr, const CellBlk& blk,
                                             const double* __restrict__ p_in, const float* __restrict__ e,
                                             double* __restrict__ p_out, const float* __restrict__ rhs,
                                             float* __restrict__ r) {
  double acc = 0.0;
  // A thread marches its (i, j) column through a run of zr planes and keeps
  // p + e of the planes below, at and above the cell in registers.
  const int i = blk.x * kCellX + threadIdx.x + 1;
  const int j = blk.y * (int)blockDim.y + threadIdx.y + 1;
  if (i <= g.nx && j <= g.ny) {
    const Nb nb = neighbours(g, i, j, 1);  // x and y entries; z per plane below
    const int k0 = blk.z * zr + 1;
    const int k1 = min(g.nz, k0 + zr - 1);
    auto q = [&](long c) {
      if constexpr (HAS_E)
        return p_in[c] + (double)e[c];
      else
        return p_in[c] + 0.0;
    };
    const int per2 = g.per[2];
    auto zdn = [&](int k) -> long { return k > 1 ? -g.sxy : (per2 ? (long)(g.nz - 1) * g.sxy : 0L); };
    auto zup = [&](int k) -> long { return k < g.nz ? g.sxy : (per2 ? -(long)(g.nz - 1) * g.sxy : 0L); };
    long c = (long)k0 * g.sxy + (long)j * g.sx + i;
    double qc = q(c), qd = q(c + zdn(k0));
    // two planes per trip: the loads of the second are issued with those of
    // the first (measured 5 % faster than one, and faster than four)
#pragma unroll 2
    for (int k = k0; k <= k1; k++, c += g.sxy) {
      const double qu = q(c + zup(k));
      const double azm = (k > 1 || per2) ? g.idz2 : 0.0;
      const double azp = (k < g.nz || per2) ? g.idz2 : 0.0;
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 4; t++) s += nb.a[t] * (q(c + nb.o[t]) - qc);
      s += azm * (qd - qc);
      s += azp * (qu - qc);
      const double rr = (double)rhs[c] - s;
      r[c] = (float)rr;
      acc += rr * rr;
      if constexpr (HAS_E) p_out[c] = qc;
      qd = qc;
      qc = qu;
    }
  }
  return acc;
}
// The control block's fields set from the domain's sum of r^2 (all but the
// ticket).
__device__ __forceinline__ void defect_finish(Ctl* ctl, double tot, long n, double eta) {
  // an identically zero rhs needs no correction at all
  const double res = ctl->rhs_rms == 0.0 ? 0.0 : sqrt(tot / (double)n);
  const bool fin = isfinite(res);
  ctl->res = res;
  ctl->outer_done = !(res > ctl->thr) || !fin;
  if (!fin) ctl->nonfinite = 1;
  ctl->thr_in = eta * res;
  ctl->done = ctl->outer_done;
  ctl->final_ = 0;
}
template <bool HAS_E>
__device__ __forceinline__ void defect_cells(const Geo& g, int zr, const CellBlk& blk,
                                             const double* __restrict__ p_in, const float* __restrict__ e,
                                             double* __restrict__ p_out, const float* __restrict__ rhs,
                                             float* __restrict__ r, Ctl* ctl, double* part, double eta, double* sh,
                                             int* sh_last) {
  const long n = (long)g.nx * g.ny * g.nz;
  const double acc = defect_acc<HAS_E>(g, zr, blk, p_in, e, p_out, rhs, r);
  double s = block_sum(acc, sh);
  if (publish_partial(part, blk.id, s, ctl, blk.count, sh_last)) {
    double tot = sum_partials(part, blk.count, sh);
    if (flat_tid() == 0) {
      defect_finish(ctl, tot, n, eta);
      ctl->ticket = 0;
    }
  }
}

}  // namespace

}  // namespace ns
