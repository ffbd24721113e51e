// predict_velocity.h -- per-cell body of the generated PREDICT_VELOCITY
// kernel: the momentum predictor F, G, H (explicit Euler step of viscous,
// convective and body-force terms; conservative fluxes with the donor-cell
// blend gamma), u, v, w cached with a one-cell halo.  The same expressions,
// in the same order, as the predictor cells of cells.h: all three components
// are formed at every cell and stored where they are unknowns.
#pragma once

namespace ns {
namespace gen {

template <class K>
__device__ __forceinline__ double body_force(const K& x, double gc, int c) {
#pragma clang fp contract(on)
  if constexpr (K::has_BODY_FORCE)
    return gc + (double)(c == 0 ? x.fx() : (c == 1 ? x.fy() : x.fz()));
  else
    return gc + 0.0;
}

// The three components, one function each (the body below, and a caller
// that needs one component at a face outside its cells, run the same
// expressions).
template <class K>
__device__ __forceinline__ double PREDICT_VELOCITY_F(const K& x) {
#pragma clang fp contract(on)  // as in the predictor cells of cells.h
  const Geo& g = x.g;
  const double dt = x.dt, nu = x.nu, gamma = x.gamma;
  const double q = x.u(), qe = x.u(1, 0, 0), qw = x.u(-1, 0, 0), qn = x.u(0, 1, 0), qs = x.u(0, -1, 0),
               qt = x.u(0, 0, 1), qb = x.u(0, 0, -1);
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double cx = (flux(0.5 * (q + qe), q, qe, gamma) - flux(0.5 * (qw + q), qw, q, gamma)) * g.idx;
  const double vn = 0.5 * ((double)x.v() + (double)x.v(1, 0, 0));
  const double vs = 0.5 * ((double)x.v(0, -1, 0) + (double)x.v(1, -1, 0));
  const double cy = (flux(vn, q, qn, gamma) - flux(vs, qs, q, gamma)) * g.idy;
  const double wt = 0.5 * ((double)x.w() + (double)x.w(1, 0, 0));
  const double wb = 0.5 * ((double)x.w(0, 0, -1) + (double)x.w(1, 0, -1));
  const double cz = (flux(wt, q, qt, gamma) - flux(wb, qb, q, gamma)) * g.idz;
  const double f = body_force(x, x.gx, 0);
  return q + dt * (nu * lap - cx - cy - cz + f);
}

template <class K>
__device__ __forceinline__ double PREDICT_VELOCITY_G(const K& x) {
#pragma clang fp contract(on)
  const Geo& g = x.g;
  const double dt = x.dt, nu = x.nu, gamma = x.gamma;
  const double q = x.v(), qe = x.v(1, 0, 0), qw = x.v(-1, 0, 0), qn = x.v(0, 1, 0), qs = x.v(0, -1, 0),
               qt = x.v(0, 0, 1), qb = x.v(0, 0, -1);
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double ue = 0.5 * ((double)x.u() + (double)x.u(0, 1, 0));
  const double uw = 0.5 * ((double)x.u(-1, 0, 0) + (double)x.u(-1, 1, 0));
  const double cx = (flux(ue, q, qe, gamma) - flux(uw, qw, q, gamma)) * g.idx;
  const double cy = (flux(0.5 * (q + qn), q, qn, gamma) - flux(0.5 * (qs + q), qs, q, gamma)) * g.idy;
  const double wt = 0.5 * ((double)x.w() + (double)x.w(0, 1, 0));
  const double wb = 0.5 * ((double)x.w(0, 0, -1) + (double)x.w(0, 1, -1));
  const double cz = (flux(wt, q, qt, gamma) - flux(wb, qb, q, gamma)) * g.idz;
  const double f = body_force(x, x.gy, 1);
  return q + dt * (nu * lap - cx - cy - cz + f);
}

template <class K>
__device__ __forceinline__ double PREDICT_VELOCITY_H(const K& x) {
#pragma clang fp contract(on)
  const Geo& g = x.g;
  const double dt = x.dt, nu = x.nu, gamma = x.gamma;
  const double q = x.w(), qe = x.w(1, 0, 0), qw = x.w(-1, 0, 0), qn = x.w(0, 1, 0), qs = x.w(0, -1, 0),
               qt = x.w(0, 0, 1), qb = x.w(0, 0, -1);
  const double lap = (qe - 2.0 * q + qw) * g.idx2 + (qn - 2.0 * q + qs) * g.idy2 + (qt - 2.0 * q + qb) * g.idz2;
  const double ue = 0.5 * ((double)x.u() + (double)x.u(0, 0, 1));
  const double uw = 0.5 * ((double)x.u(-1, 0, 0) + (double)x.u(-1, 0, 1));
  const double cx = (flux(ue, q, qe, gamma) - flux(uw, qw, q, gamma)) * g.idx;
  const double vn = 0.5 * ((double)x.v() + (double)x.v(0, 0, 1));
  const double vs = 0.5 * ((double)x.v(0, -1, 0) + (double)x.v(0, -1, 1));
  const double cy = (flux(vn, q, qn, gamma) - flux(vs, qs, q, gamma)) * g.idy;
  const double cz = (flux(0.5 * (q + qt), q, qt, gamma) - flux(0.5 * (qb + q), qb, q, gamma)) * g.idz;
  const double f = body_force(x, x.gz, 2);
  return q + dt * (nu * lap - cx - cy - cz + f);
}

template <class K>
__device__ __forceinline__ void PREDICT_VELOCITY_body(const K& x) {
  const Geo& g = x.g;
  const double Fv = PREDICT_VELOCITY_F(x);
  const double Gv = PREDICT_VELOCITY_G(x);
  const double Hv = PREDICT_VELOCITY_H(x);
  if (x.i <= g.hi[0]) x.store_F(Fv);
  if (x.j <= g.hi[1]) x.store_G(Gv);
  if (x.k <= g.hi[2]) x.store_H(Hv);
}

}  // namespace gen
}  // namespace ns
