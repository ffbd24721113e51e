// generated.h -- launchers of the predictor and projection generated from
// the kernel descriptors (generated.hip); a handle created with
// NS_GENERATED runs them in place of the hand-written kernels.  Same
// arguments and results as launch_fgh / launch_project.
#pragma once

#include "ns_internal.h"

namespace ns {

template <class T>
hipError_t launch_gen_project(hipStream_t st, const Geo& g, const T* F, const T* G, const T* H, const double* p, T* u,
                              T* v, T* w, const Ctl* ctl);
template <class T>
hipError_t launch_gen_fgh(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, const T* fx, const T* fy,
                          const T* fz, T* F, T* G, T* H, const Ctl* ctl, double re, double gamma, const double gf[3]);

}  // namespace ns
