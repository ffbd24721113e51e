// sor.hip -- red-black SOR sweeps and the mixed-precision defect step.
//
// Operator: boundary-eliminated homogeneous-Neumann 7-point Laplacian,
// A p = sum_nb a_nb (p_nb - p), a_nb = 1/h^2 for a neighbour inside the
// domain (or its periodic image) and 0 across a wall.  Colour of a cell is
// (i + j + k) mod 2 on 1-based interior indices; red (even) goes first.
// A sweep maps p_in -> p_out out of place (so that a sweep never reads a
// value another workgroup of the same sweep has already replaced):
//   red:   p_out = p_in + omega r / a_c,   r = A p_in - rhs at the cell
//   black: p_out = p_in + omega r' / a_c,  r' from the new red neighbours
// which is (1 - omega) p + omega (sum a_nb p_nb - rhs) / a_c written as an
// increment.  The residual r of p_in at every cell is summed in FP64 in the
// same pass, so sweep m reports the RMS residual of iterate m - 1; the last
// workgroup of the red pass applies the stop rule and raises ctl->done.
#include <hip/hip_runtime.h>

#include "cells.h"
#include "ns_internal.h"
#include "reduce.h"

namespace ns {

namespace {

constexpr int kBlock = 256;

inline int grid_for(long n, int cap = 8192) {
  long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

struct Cell {
  int i, j, k;
  long c;
};
__device__ __forceinline__ Cell cell_of(const Geo& g, long t) {
  Cell r;
  long row = t / g.nx;
  r.i = (int)(t - row * g.nx) + 1;
  r.k = (int)(row / g.ny) + 1;
  r.j = (int)(row - (long)(r.k - 1) * g.ny) + 1;
  r.c = (long)r.k * g.sxy + (long)r.j * g.sx + r.i;
  return r;
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_sor_red(const T* __restrict__ p_in, T* __restrict__ p_out, const T* __restrict__ rhs, Geo g,
          Ctl* ctl, double* part, double omega, int m, int itermax, int write, int zero_in,
          int inner) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  if (ctl->done) return;
  const long n = (long)g.nx * g.ny * g.nz;
  double acc = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const Cell cl = cell_of(g, t);
    const Nb nb = neighbours(g, cl.i, cl.j, cl.k);
    double r;
    double pc = 0.0;
    if (zero_in) {
      r = -(double)rhs[cl.c];
    } else {
      pc = p_in[cl.c];
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 6; q++) s += nb.a[q] * ((double)p_in[cl.c + nb.o[q]] - pc);
      r = s - (double)rhs[cl.c];
    }
    acc += r * r;
    if (write && !((cl.i + cl.j + cl.k) & 1)) p_out[cl.c] = T(pc + omega * r / nb.ac);
  }
  double s = block_sum(acc, sh);
  if (publish_partial(part, blockIdx.x, s, ctl, gridDim.x, &sh_last)) {
    double tot = sum_partials(part, gridDim.x, sh);
    if (threadIdx.x == 0) {
      const double res = sqrt(tot / (double)n);
      const int mm = m - 1;  // iterate whose residual this is
      const double thr = inner ? ctl->thr_in : ctl->thr;
      if (mm >= 1 || itermax == 0) {
        if (inner) ctl->res_in = res; else ctl->res = res;
        const bool fin = isfinite(res);
        if (!(res > thr) || mm >= itermax || !fin) {
          ctl->done = 1;
          ctl->final_ = mm;
          if (!fin) ctl->nonfinite = 1;
        }
      }
      ctl->ticket = 0;
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_sor_black(const T* __restrict__ p_in, T* __restrict__ p_out, const T* __restrict__ rhs, Geo g,
            const Ctl* ctl, double omega, int zero_in) {
  if (ctl->done) return;
  const long n = (long)g.nx * g.ny * g.nz;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const Cell cl = cell_of(g, t);
    if (!((cl.i + cl.j + cl.k) & 1)) continue;
    const Nb nb = neighbours(g, cl.i, cl.j, cl.k);
    const double pc = zero_in ? 0.0 : (double)p_in[cl.c];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) s += nb.a[q] * ((double)p_out[cl.c + nb.o[q]] - pc);
    const double r = s - (double)rhs[cl.c];
    p_out[cl.c] = T(pc + omega * r / nb.ac);
  }
}

__global__ void __launch_bounds__(kBlock)
k_defect(int zr, const double* __restrict__ p_in, const float* __restrict__ e, double* __restrict__ p_out,
         const float* __restrict__ rhs, float* __restrict__ r, Geo g, Ctl* ctl, double* part,
         double eta) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  if (e)
    defect_cells<true>(g, zr, own_blk(), p_in, e, p_out, rhs, r, ctl, part, eta, sh, &sh_last);
  else
    defect_cells<false>(g, zr, own_blk(), p_in, e, p_out, rhs, r, ctl, part, eta, sh, &sh_last);
}

// Every domain of a batch in one launch (workgroup -> domain as for the
// other batched stages).
__global__ void __launch_bounds__(kBlock) k_defect_batched(const StageItem* __restrict__ items, int nitems) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  const int b = blockIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  const StageItem& it = items[lo];
  const int l = b - it.first;
  CellBlk blk;
  blk.x = l % it.gx;
  blk.y = (l / it.gx) % it.gy;
  blk.z = l / (it.gx * it.gy);
  blk.id = (unsigned)l;
  blk.count = (unsigned)(it.gx * it.gy * it.gz);
  const double* p_in = (const double*)it.in[0];
  const float* e = (const float*)it.in[1];
  const float* rhs = (const float*)it.in[2];
  if (e)
    defect_cells<true>(it.g, it.zr, blk, p_in, e, (double*)it.out[0], rhs, (float*)it.out[1], it.ctl, it.part,
                       it.s[0], sh, &sh_last);
  else
    defect_cells<false>(it.g, it.zr, blk, p_in, e, (double*)it.out[0], rhs, (float*)it.out[1], it.ctl, it.part,
                        it.s[0], sh, &sh_last);
}

}  // namespace

int sor_num_blocks(const Geo& g, const SorShape& s) {
  const int a = grid_for((long)g.nx * g.ny * g.nz);
  const int b = s.ty > 0 ? fused_num_blocks(g, s) : 0;
  return a > b ? a : b;
}

template <class T>
hipError_t launch_sor_sweep(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs,
                            Ctl* ctl, double* part, double omega, int sweep_idx, int itermax,
                            int write, int zero_in, int thr_is_inner, const SorShape& shape) {
  if (shape.ty > 0)
    return launch_sor_fused<T>(st, g, p_in, p_out, rhs, ctl, part, omega, sweep_idx, itermax, write, zero_in,
                               thr_is_inner, shape);
  const long n = (long)g.nx * g.ny * g.nz;
  const int nb = grid_for(n);
  k_sor_red<T><<<nb, kBlock, 0, st>>>(p_in, p_out, rhs, g, ctl, part, omega, sweep_idx, itermax, write,
                                      zero_in, thr_is_inner);
  if (write) k_sor_black<T><<<nb, kBlock, 0, st>>>(p_in, p_out, rhs, g, ctl, omega, zero_in);
  return hipGetLastError();
}

hipError_t launch_defect(hipStream_t st, const Geo& g, const double* p_in, const float* e,
                         double* p_out, const float* rhs, float* r, Ctl* ctl, double* part,
                         double eta) {
  const long n = (long)g.nx * g.ny * g.nz;
  k_defect<<<cell_grid(g, kRedDefect), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, kRedDefect), p_in, e, p_out, rhs, r, g, ctl, part, eta);
  return hipGetLastError();
}

hipError_t launch_defect_batched(hipStream_t st, const StageItem* d_items, int nitems, int nblocks) {
  k_defect_batched<<<nblocks, dim3(kCellX, kCellY), 0, st>>>(d_items, nitems);
  return hipGetLastError();
}

template hipError_t launch_sor_sweep<double>(hipStream_t, const Geo&, const double*, double*,
                                             const double*, Ctl*, double*, double, int, int, int,
                                             int, int, const SorShape&);
template hipError_t launch_sor_sweep<float>(hipStream_t, const Geo&, const float*, float*,
                                            const float*, Ctl*, double*, double, int, int, int, int,
                                            int, const SorShape&);

}  // namespace ns
