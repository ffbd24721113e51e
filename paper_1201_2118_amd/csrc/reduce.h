// reduce.h -- deterministic workgroup and grid reductions for wave64.
#pragma once

#include <hip/hip_runtime.h>

#include "ns_internal.h"

namespace ns {

// Flattened thread index and workgroup size (1D, 2D or 3D workgroups).
__device__ __forceinline__ int flat_tid() {
  return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}
__device__ __forceinline__ int flat_size() { return blockDim.x * blockDim.y * blockDim.z; }

// Sum over a workgroup (size a multiple of 64, at most 1024) in a fixed
// order: wave64 shuffles, then the per-wave sums by wave 0.  The result is
// valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh /* >= 16 */) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int t = flat_tid();
  const int lane = t & 63, wid = t >> 6, nw = flat_size() >> 6;
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
  const int t = flat_tid();
  const int lane = t & 63, wid = t >> 6, nw = flat_size() >> 6;
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
  if (flat_tid() == 0) {
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
  // four independent loads in flight per thread, then a fixed combination
  const unsigned t = flat_tid(), w = flat_size();
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  unsigned i = t;
  for (; i + 3 * w < n; i += 4 * w) {
    s0 += part[i];
    s1 += part[i + w];
    s2 += part[i + 2 * w];
    s3 += part[i + 3 * w];
  }
  for (; i < n; i += w) s0 += part[i];
  return block_sum((s0 + s1) + (s2 + s3), sh);
}

__device__ __forceinline__ double max_partials(const double* part, unsigned n, double* sh) {
  double s = 0.0;
  for (unsigned i = flat_tid(); i < n; i += flat_size()) s = fmax(s, part[i]);
  return block_max(s, sh);
}

}  // namespace ns
