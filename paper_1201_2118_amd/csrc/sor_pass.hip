// sor_pass.hip -- NS (1 or 2) red-black SOR sweeps in one pass over HBM.
//
// The tile itself (pass_tile) is in pass_tile.h; this file holds the
// single-domain and batched kernels and their launchers.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "ns_internal.h"
#include "pass_tile.h"
#include "reduce.h"

namespace ns {

namespace {

// One pass of NS sweeps with first sweep index m (input iterate m - 1).
// With part == nullptr the pass is forced: it runs whatever the done flag
// says and applies no stop rule (the host uses it to materialise an
// iterate a two-sweep pass held only in registers).
// Stop rule after a pass with first sweep index m: sweep m reports the RMS
// residual of iterate m - 1 (sum t1), sweep m + 1 that of iterate m (t2).
__device__ __forceinline__ void stop_rule(Ctl* ctl, int inner, int itermax, long n, int m, int ns, double t1,
                                          double t2) {
  const double thr = inner ? ctl->thr_in : ctl->thr;
  auto check = [&](int mm, double tot) -> bool {
    const double res = sqrt(tot / (double)n);
    if (!(mm >= 1 || itermax == 0)) return false;
    if (inner) ctl->res_in = res; else ctl->res = res;
    const bool fin = isfinite(res);
    if (!(res > thr) || mm >= itermax || !fin) {
      ctl->done = 1;
      ctl->final_ = mm;
      if (!fin) ctl->nonfinite = 1;
      return true;
    }
    return false;
  };
  if (!check(m - 1, t1) && ns == 2) check(m, t2);
  ctl->ticket = 0;
}

#ifndef NS_PASS_MINW
#define NS_PASS_MINW 1
#endif
template <class T, int NS, int R, int W, bool ZIN>
__global__ void __launch_bounds__(kLanes * W, NS_PASS_MINW)
k_sor_pass(const T* __restrict__ p_in, T* __restrict__ p_out, const T* __restrict__ rhs, Geo g, Ctl* ctl,
           double* part, double omega, int m, int itermax, int write, int inner, int zc, int ntx, int nty,
           int ntiles) {
  __shared__ T E[2 * NS * 2 * kEdge<W>];
  __shared__ double shred[16];
  __shared__ int sh_last;
  if (part != nullptr && ctl->done) return;
  double acc1 = 0.0, acc2 = 0.0;
  // edge rows a step reads before this tile wrote them hold finite values
  for (int q = flat_tid(); q < 2 * NS * 2 * kEdge<W>; q += kLanes * W) E[q] = T(0);
  __syncthreads();

  // Persistent workgroups.  Workgroup b runs on XCD b % 8; its position in
  // XCD-major order, li, makes the work of neighbouring workgroups on one
  // XCD neighbouring columns (same L2).
  const int G = gridDim.x;
  const bool by_xcd = G >= 8;
  const int xcd = by_xcd ? (blockIdx.x & 7) : 0;
  const int slot = by_xcd ? (blockIdx.x >> 3) : blockIdx.x;
  const int li = by_xcd ? xcd * (G >> 3) + min(xcd, G & 7) + slot : blockIdx.x;
  const int ncols = ntx * nty;
  if (zc > 0) {
    // tiles of zc planes: column-major tile list, dealt round-robin in li order
    for (int tile = li; tile < ntiles; tile += G) {
      const int col = tile % ncols, bz = tile / ncols;
      const int z0 = 1 + bz * zc;
      pass_tile<T, NS, R, W, ZIN, false>(p_in, p_out, rhs, g, omega, write, col, z0, min(g.nz, z0 + zc - 1), ntx, E,
                                  acc1, acc2);
      __syncthreads();
    }
  } else {
    // balanced: workgroup li takes an equal share of the (column, plane)
    // space in column order, cut at column ends into z ranges
    const long ptot = (long)ncols * g.nz;
    long q0 = ptot * li / G;
    const long q1 = ptot * (li + 1) / G;
    while (q0 < q1) {
      const int col = (int)(q0 / g.nz);
      const int z0 = (int)(q0 - (long)col * g.nz) + 1;
      const int z1 = (int)min((long)g.nz, (long)z0 + (q1 - q0) - 1);
      pass_tile<T, NS, R, W, ZIN, false>(p_in, p_out, rhs, g, omega, write, col, z0, z1, ntx, E, acc1,
                                  acc2);
      __syncthreads();
      q0 += z1 - z0 + 1;
    }
  }
  if (part == nullptr) return;

  const long n = (long)g.nx * g.ny * g.nz;
  const double s1 = block_sum(acc1, shred);
  const double s2 = NS == 2 ? block_sum(acc2, shred) : 0.0;
  if (NS == 2 && flat_tid() == 0) part[G + blockIdx.x] = s2;
  if (publish_partial(part, blockIdx.x, s1, ctl, G, &sh_last)) {
    const double t1 = sum_partials(part, G, shred);
    const double t2 = NS == 2 ? sum_partials(part + G, G, shred) : 0.0;
    if (flat_tid() == 0) stop_rule(ctl, inner, itermax, n, m, NS, t1, t2);
  }
}

// Batched pass: one launch covers a pass of every domain of a batch.
// Workgroup b belongs to the domain whose [first, first + ntiles) range
// holds b and sweeps one tile of it (chunks of zc planes, zc = nz for whole
// columns); each domain has its own partial sums, ticket, stop rule, budget
// and done flag.  Pass q of a domain reads p[(cur + q) & 1] and writes the
// other buffer.  force: sweep regardless of the done flag, no residuals.
template <class T, int NS, int R, int W, bool ZIN>
__global__ void __launch_bounds__(kLanes * W)
k_pass_batched(const BatchItem* __restrict__ items, int nitems, int m, int q, int force) {
  __shared__ T E[2 * NS * 2 * kEdge<W>];
  __shared__ double shred[16];
  __shared__ int sh_last;
  const int b = blockIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  const BatchItem& it = items[lo];
  Ctl* ctl = it.ctl;
  if (!force && ctl->done) return;
  for (int k = flat_tid(); k < 2 * NS * 2 * kEdge<W>; k += kLanes * W) E[k] = T(0);
  __syncthreads();
  const Geo g = it.g;
  const int tile = b - it.first;
  const int ncols = it.ntx * it.nty;
  const int col = tile % ncols, bz = tile / ncols;
  const int z0 = 1 + bz * it.zc;
  const int in = (it.cur + q) & 1;
  double acc1 = 0.0, acc2 = 0.0;
  pass_tile<T, NS, R, W, ZIN, true>((const T*)it.p[in], (T*)it.p[in ^ 1], (const T*)it.rhs, g, it.omega, 1, col, z0,
                              min(g.nz, z0 + it.zc - 1), it.ntx, E, acc1, acc2);
  __syncthreads();
  if (force) return;
  const double s1 = block_sum(acc1, shred);
  const double s2 = NS == 2 ? block_sum(acc2, shred) : 0.0;
  if (NS == 2 && flat_tid() == 0) it.part[it.ntiles + tile] = s2;
  if (publish_partial(it.part, tile, s1, ctl, it.ntiles, &sh_last)) {
    const double t1 = sum_partials(it.part, it.ntiles, shred);
    const double t2 = NS == 2 ? sum_partials(it.part + it.ntiles, it.ntiles, shred) : 0.0;
    if (flat_tid() == 0) stop_rule(ctl, it.inner, it.budget, (long)g.nx * g.ny * g.nz, m, NS, t1, t2);
  }
}

template <class T, int NS, int R, int W>
int pass_resident() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sor_pass<T, NS, R, W, false>, kLanes * W, 0) !=
      hipSuccess)
    return 0;
  cached = cus * (per_cu > 0 ? per_cu : 1);
  return cached;
}

template <class T, int NS, int R, int W>
hipError_t launch_w(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs, Ctl* ctl, double* part,
                    double omega, int m, int itermax, int write, int zero_in, int inner, int zc) {
  constexpr int H = 2 * NS;
  constexpr int ROWS = R * W;
  const int ntx = (g.nx + (kLanes - 2 * H) - 1) / (kLanes - 2 * H);
  const int nty = (g.ny + (ROWS - 2 * H) - 1) / (ROWS - 2 * H);
  // zc = 0: as many workgroups as are resident (each with a balanced share),
  // but no more than there are plane-columns
  const long ntiles_l = zc > 0 ? (long)ntx * nty * ((g.nz + zc - 1) / zc) : (long)ntx * nty * g.nz;
  const int ntiles = (int)(ntiles_l < (1L << 30) ? ntiles_l : (1L << 30));
  int nb = pass_resident<T, NS, R, W>();
  if (nb <= 0 || nb > ntiles) nb = ntiles;
  const dim3 blk(kLanes, W);
  if (zero_in)
    k_sor_pass<T, NS, R, W, true><<<nb, blk, 0, st>>>(p_in, p_out, rhs, g, ctl, part, omega, m, itermax, write,
                                                          inner, zc, ntx, nty, ntiles);
  else
    k_sor_pass<T, NS, R, W, false><<<nb, blk, 0, st>>>(p_in, p_out, rhs, g, ctl, part, omega, m, itermax, write,
                                                           inner, zc, ntx, nty, ntiles);
  return hipGetLastError();
}

// FP64 tiles have 16 rows: with 12 or 16 waves the FP64 state of two rows per
// lane does not fit the registers of the occupancy those workgroups need.
template <class T>
constexpr bool rows_ok(int rows) {
  return rows == 16 || (sizeof(T) == 4 && (rows == 24 || rows == 32));
}

template <class T, int NS>
hipError_t launch_ns(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs, Ctl* ctl, double* part,
                     double omega, int m, int itermax, int write, int zero_in, int inner, int zc, int rows) {
  if (rows == 16)
    return launch_w<T, NS, 2, 8>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc);
  if constexpr (sizeof(T) == 4) {
    constexpr int R24 = kR24, R32 = kR32;
    if (rows == 24)
      return launch_w<T, NS, R24, 24 / R24>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in,
                                            inner, zc);
    if (rows == 32)
      return launch_w<T, NS, R32, 32 / R32>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in,
                                            inner, zc);
  }
  return hipErrorInvalidValue;
}

template <class T, int NS, int R, int W>
hipError_t launch_batched_w(hipStream_t st, const BatchItem* items, int nitems, int nblocks, int m, int q,
                            int zero_in, int force) {
  const dim3 blk(kLanes, W);
  if (zero_in)
    k_pass_batched<T, NS, R, W, true><<<nblocks, blk, 0, st>>>(items, nitems, m, q, force);
  else
    k_pass_batched<T, NS, R, W, false><<<nblocks, blk, 0, st>>>(items, nitems, m, q, force);
  return hipGetLastError();
}

template <class T, int NS>
hipError_t launch_batched_ns(hipStream_t st, const BatchItem* items, int nitems, int nblocks, int rows, int m,
                             int q, int zero_in, int force) {
  if (rows == 16) return launch_batched_w<T, NS, 2, 8>(st, items, nitems, nblocks, m, q, zero_in, force);
  if constexpr (sizeof(T) == 4) {
    constexpr int R24 = kR24, R32 = kR32;
    if (rows == 24)
      return launch_batched_w<T, NS, R24, 24 / R24>(st, items, nitems, nblocks, m, q, zero_in, force);
    if (rows == 32)
      return launch_batched_w<T, NS, R32, 32 / R32>(st, items, nitems, nblocks, m, q, zero_in, force);
  }
  return hipErrorInvalidValue;
}

}  // namespace

void pass_item_shape(BatchItem& it, int rows, int zc, int ns) {
  const int h = 2 * ns;
  it.ntx = (it.g.nx + (kLanes - 2 * h) - 1) / (kLanes - 2 * h);
  it.nty = (it.g.ny + (rows - 2 * h) - 1) / (rows - 2 * h);
  it.zc = item_chunk(it.g.nz, zc);
  it.ntiles = it.ntx * it.nty * ((it.g.nz + it.zc - 1) / it.zc);
}

template <class T>
hipError_t launch_pass_batched(hipStream_t st, const BatchItem* d_items, int nitems, int nblocks, int rows, int m,
                               int q, int ns, int zero_in, int force) {
  if (ns == 1) return launch_batched_ns<T, 1>(st, d_items, nitems, nblocks, rows, m, q, zero_in, force);
  if (ns == 2) return launch_batched_ns<T, 2>(st, d_items, nitems, nblocks, rows, m, q, zero_in, force);
  return hipErrorInvalidValue;
}

template hipError_t launch_pass_batched<double>(hipStream_t, const BatchItem*, int, int, int, int, int, int, int,
                                                int);
template hipError_t launch_pass_batched<float>(hipStream_t, const BatchItem*, int, int, int, int, int, int, int,
                                               int);

bool pass_shape_ok(const SorShape& s) { return s.ty == 16 || s.ty == 24 || s.ty == 32; }

bool pass_grid_ok(const Geo& g, size_t esz) {
  // one wrap of the 4-cell halo on periodic axes; plane offsets in 31 bits
  for (int a = 0; a < 3; a++) {
    const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
    if (g.per[a] && n < 4) return false;
  }
  return (double)g.sxy * (double)esz < 2147483648.0;
}

int pass_max_partials(const Geo& g) {
  // resident workgroups never exceed the tile count of the smallest tiles
  const int ntx = (g.nx + 55) / 56, nty = (g.ny + 7) / 8;
  return 2 * ntx * nty * g.nz;
}

int pass_resident_groups(int ty, bool f32, int ns) {
  if (ty == 16)
    return ns == 1 ? (f32 ? pass_resident<float, 1, 2, 8>() : pass_resident<double, 1, 2, 8>())
                   : (f32 ? pass_resident<float, 2, 2, 8>() : pass_resident<double, 2, 2, 8>());
  if (!f32) return 0;  // FP64 tiles have 16 rows
  constexpr int R24 = kR24, R32 = kR32;
  if (ty == 24)
    return ns == 1 ? pass_resident<float, 1, R24, 24 / R24>() : pass_resident<float, 2, R24, 24 / R24>();
  if (ty == 32)
    return ns == 1 ? pass_resident<float, 1, R32, 32 / R32>() : pass_resident<float, 2, R32, 32 / R32>();
  return 0;
}

bool pass_rows_ok(int rows, bool f32) { return f32 ? rows_ok<float>(rows) : rows_ok<double>(rows); }

int pass_columns(const Geo& g, int ty, int ns) {
  const int h = 2 * ns;
  return ((g.nx + (kLanes - 2 * h) - 1) / (kLanes - 2 * h)) * ((g.ny + (ty - 2 * h) - 1) / (ty - 2 * h));
}

template <class T>
hipError_t launch_sor_pass(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs, Ctl* ctl,
                           double* part, double omega, int m, int itermax, int write, int zero_in, int inner,
                           int ns, const SorShape& s) {
  // zc = 0: balanced z ranges over the resident workgroups
  const int zc = s.zc != 0 ? item_chunk(g.nz, s.zc) : 0;
  if (ns == 1) return launch_ns<T, 1>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc, s.ty);
  if (ns == 2) return launch_ns<T, 2>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc, s.ty);
  return hipErrorInvalidValue;
}

template hipError_t launch_sor_pass<double>(hipStream_t, const Geo&, const double*, double*, const double*, Ctl*,
                                            double*, double, int, int, int, int, int, int, const SorShape&);
template hipError_t launch_sor_pass<float>(hipStream_t, const Geo&, const float*, float*, const float*, Ctl*,
                                           double*, double, int, int, int, int, int, int, const SorShape&);

}  // namespace ns
