// generated.h -- launchers of the predictor and projection generated from
// the kernel descriptors (generated.hip).  launch_gen_fgh is the predictor
// of every single-domain step in the conservative form (its values equal
// the hand-written predictor cells of cells.h bit for bit);
// launch_gen_project replaces launch_project (same arguments and results)
// on a handle created with NS_GENERATED.
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
