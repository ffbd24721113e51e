// generated.hip -- launchers of the kernels generated at build time from the
// kernel descriptors (descriptors/kernels.ccl -> gen_<name>.h, with the
// hand-written bodies in bodies/): the predictor (PREDICT_VELOCITY, the
// predictor of every single-domain step in the conservative form) and the
// projection (UPDATE_VELOCITY, run in place of the hand-written one by a
// handle created with NS_GENERATED).
#include <hip/hip_runtime.h>

#include "cells.h"
#include "gen_predict_velocity.h"
#include "gen_update_velocity.h"
#include "generated.h"
#include "ns_internal.h"

namespace ns {

template <class T>
hipError_t launch_gen_project(hipStream_t st, const Geo& g, const T* F, const T* G, const T* H, const double* p, T* u,
                              T* v, T* w, const Ctl* ctl) {
  return gen::launch_UPDATE_VELOCITY<T>(st, g, ctl, F, u, G, v, H, w, p);
}

template <class T>
hipError_t launch_gen_fgh(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, const T* fx, const T* fy,
                          const T* fz, T* F, T* G, T* H, const Ctl* ctl, double re, double gamma,
                          const double gf[3]) {
  return gen::launch_PREDICT_VELOCITY<T>(st, g, ctl, u, v, w, F, G, H, fx, fy, fz, 1.0 / re, gamma, gf[0], gf[1],
                                         gf[2]);
}

template hipError_t launch_gen_project<double>(hipStream_t, const Geo&, const double*, const double*, const double*,
                                               const double*, double*, double*, double*, const Ctl*);
template hipError_t launch_gen_project<float>(hipStream_t, const Geo&, const float*, const float*, const float*,
                                              const double*, float*, float*, float*, const Ctl*);
template hipError_t launch_gen_fgh<double>(hipStream_t, const Geo&, const double*, const double*, const double*,
                                           const double*, const double*, const double*, double*, double*, double*,
                                           const Ctl*, double, double, const double[3]);
template hipError_t launch_gen_fgh<float>(hipStream_t, const Geo&, const float*, const float*, const float*,
                                          const float*, const float*, const float*, float*, float*, float*,
                                          const Ctl*, double, double, const double[3]);

}  // namespace ns
