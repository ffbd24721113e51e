// reduce.h -- deterministic workgroup and grid reductions for wave64.
#pragma once

#include <hip/hip_runtime.h>

#include "ns_internal.h"

namespace ns {

// Sum over a 1D workgroup (blockDim.x a multiple of 64, at most 1024) in a
// fixed order: wave64 shuffles, then the per-wave sums by wave 0.  The
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh /* >= 16 */) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  v = 0.0;
  if (wid == 0) {
    v = lane < nw ? sh[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  }
  return v;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  v = 0.0;
  if (wid == 0) {
    v = lane < nw ? sh[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  }
  return v;
}

// Publish one partial per workgroup; returns true in every thread of the
// workgroup that finished last.  That group may then read all partials
// (fence-acquire done here) and must reset ctl->ticket.
__device__ __forceinline__ bool publish_partial(double* part, int slot, double v, Ctl* ctl,
                                                unsigned nblocks, int* sh_last) {
  if (threadIdx.x == 0) {
    part[slot] = v;
    __threadfence();
    unsigned t = atomicAdd(&ctl->ticket, 1u);
    *sh_last = (t == nblocks - 1);
  }
  __syncthreads();
  const bool last = *sh_last != 0;
  if (last) __threadfence();
  return last;
}

// Deterministic sum of n partials by one workgroup (fixed strided order,
// then block_sum); valid in thread 0.
__device__ __forceinline__ double sum_partials(const double* part, unsigned n, double* sh) {
  double s = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  return block_sum(s, sh);
}

__device__ __forceinline__ double max_partials(const double* part, unsigned n, double* sh) {
  double s = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += blockDim.x) s = fmax(s, part[i]);
  return block_max(s, sh);
}

}  // namespace ns
