// convection.h -- the predictor with the advective convective form (the
// SOLA / NASA-VOF2D form, weighted by alpha; kernels.hip), run in place of
// the conservative one by handles created with NS_ADVECTIVE.  Arguments as
// launch_fgh with alpha in place of gamma.
#pragma once

#include "ns_internal.h"

namespace ns {

template <class T>
hipError_t launch_fgh_advective(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, const T* fx,
                                const T* fy, const T* fz, T* F, T* G, T* H, const Ctl* ctl, double re, double alpha,
                                const double gforce[3]);

}  // namespace ns
