// convection.h -- the predictor with the advective convective form (the
// SOLA / NASA-VOF2D form, weighted by alpha; kernels.hip), run in place of
// the conservative one by handles created with NS_ADVECTIVE.  u, v, w: the
// velocity with filled ghosts; fx, fy, fz: body-force fields or null; F, G,
// H: the predicted velocities (written at the unknowns); ctl->dt the step;
// re the Reynolds number; alpha the donor-cell weight of the advective
// differences; gforce the constant body force.
#pragma once

#include "ns_internal.h"

namespace ns {

template <class T>
hipError_t launch_fgh_advective(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, const T* fx,
                                const T* fy, const T* fz, T* F, T* G, T* H, const Ctl* ctl, double re, double alpha,
                                const double gforce[3]);

}  // namespace ns
