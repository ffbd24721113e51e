// kernels.hip -- gfx950 stencil kernels of the staggered-grid Navier-Stokes
// step other than the Poisson sweeps: boundary / ghost fill, momentum
// predictor, Poisson right-hand side, projection, adaptive dt.
//
// Every kernel streams the padded [nz+2][ny+2][nx+2] fields with
// consecutive lanes on consecutive x, so each wave64 reads 64 contiguous
// values per row (512 B in FP64).  Stencil neighbours are re-read through
// the L1/L2 caches.  FP32-stored fields (mixed precision) are widened to
// FP64 for the arithmetic.
#include <hip/hip_runtime.h>

#include "cells.h"
#include "convection.h"
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

// ---------------------------------------------------------------------------
// Ghost / boundary fill.  Walls: wall-normal faces := 0 (full extent), then
// tangential ghosts := 2 U_wall - adjacent interior (interior extent of the
// other two indices), then periodic images axis by axis (full extent).  The
// three phases are separate launches so that every read sees the previous
// phase's writes.

// Face loop helper: thread (a, b) of a face of axis `ax`, a on the faster
// of the two other axes.
template <class T>
__global__ void k_bc_normal(T* __restrict__ u, T* __restrict__ v, T* __restrict__ w, Geo g) {
  const int ax = blockIdx.z;
  if (g.per[ax]) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y * blockDim.y + threadIdx.y;
  if (ax == 0) {  // u faces 0 and nx; (a, b) = (j, k)
    if (a > g.ny + 1 || b > g.nz + 1) return;
    long base = (long)b * g.sxy + (long)a * g.sx;
    u[base] = T(0);
    u[base + g.nx] = T(0);
  } else if (ax == 1) {  // v faces 0 and ny; (a, b) = (i, k)
    if (a > g.nx + 1 || b > g.nz + 1) return;
    long base = (long)b * g.sxy + a;
    v[base] = T(0);
    v[base + (long)g.ny * g.sx] = T(0);
  } else {  // w faces 0 and nz; (a, b) = (i, j)
    if (a > g.nx + 1 || b > g.ny + 1) return;
    long base = (long)b * g.sx + a;
    w[base] = T(0);
    w[base + (long)g.nz * g.sxy] = T(0);
  }
}

struct Wall {
  double v[6][3];
};

template <class T>
__global__ void k_bc_reflect(T* __restrict__ u, T* __restrict__ v, T* __restrict__ w, Geo g,
                             Wall wl) {
  const int ax = blockIdx.z;
  if (g.per[ax]) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int b = blockIdx.y * blockDim.y + threadIdx.y + 1;
  if (ax == 0) {  // x walls: v and w ghosts at i = 0, nx+1; (a, b) = (j, k)
    if (a > g.ny || b > g.nz) return;
    long base = (long)b * g.sxy + (long)a * g.sx;
    v[base] = T(2.0 * wl.v[0][1] - (double)v[base + 1]);
    w[base] = T(2.0 * wl.v[0][2] - (double)w[base + 1]);
    v[base + g.nx + 1] = T(2.0 * wl.v[1][1] - (double)v[base + g.nx]);
    w[base + g.nx + 1] = T(2.0 * wl.v[1][2] - (double)w[base + g.nx]);
  } else if (ax == 1) {  // y walls: u and w ghosts at j = 0, ny+1; (a, b) = (i, k)
    if (a > g.nx || b > g.nz) return;
    long base = (long)b * g.sxy + a;
    long top = base + (long)(g.ny + 1) * g.sx;
    u[base] = T(2.0 * wl.v[2][0] - (double)u[base + g.sx]);
    w[base] = T(2.0 * wl.v[2][2] - (double)w[base + g.sx]);
    u[top] = T(2.0 * wl.v[3][0] - (double)u[top - g.sx]);
    w[top] = T(2.0 * wl.v[3][2] - (double)w[top - g.sx]);
  } else {  // z walls: u and v ghosts at k = 0, nz+1; (a, b) = (i, j)
    if (a > g.nx || b > g.ny) return;
    long base = (long)b * g.sx + a;
    long top = base + (long)(g.nz + 1) * g.sxy;
    u[base] = T(2.0 * wl.v[4][0] - (double)u[base + g.sxy]);
    v[base] = T(2.0 * wl.v[4][1] - (double)v[base + g.sxy]);
    u[top] = T(2.0 * wl.v[5][0] - (double)u[top - g.sxy]);
    v[top] = T(2.0 * wl.v[5][1] - (double)v[top - g.sxy]);
  }
}

// Periodic images along one axis over the full extent of the other two;
// up to three fields per launch (null pointers skipped).
template <class T>
__global__ void k_periodic(T* __restrict__ q0, T* __restrict__ q1, T* __restrict__ q2, Geo g,
                           int ax) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y * blockDim.y + threadIdx.y;
  long lo, hi, src_lo, src_hi;
  if (ax == 0) {
    if (a > g.ny + 1 || b > g.nz + 1) return;
    long base = (long)b * g.sxy + (long)a * g.sx;
    lo = base; hi = base + g.nx + 1; src_lo = base + g.nx; src_hi = base + 1;
  } else if (ax == 1) {
    if (a > g.nx + 1 || b > g.nz + 1) return;
    long base = (long)b * g.sxy + a;
    lo = base; hi = base + (long)(g.ny + 1) * g.sx;
    src_lo = base + (long)g.ny * g.sx; src_hi = base + g.sx;
  } else {
    if (a > g.nx + 1 || b > g.ny + 1) return;
    long base = (long)b * g.sx + a;
    lo = base; hi = base + (long)(g.nz + 1) * g.sxy;
    src_lo = base + (long)g.nz * g.sxy; src_hi = base + g.sxy;
  }
  T* q[3] = {q0, q1, q2};
#pragma unroll
  for (int f = 0; f < 3; f++)
    if (q[f]) {
      T a0 = q[f][src_lo], a1 = q[f][src_hi];
      q[f][lo] = a0;
      q[f][hi] = a1;
    }
}

// Pressure ghosts on wall axes: Neumann copy of the adjacent cell.
template <class T>
__global__ void k_p_neumann(T* __restrict__ p, Geo g) {
  const int ax = blockIdx.z;
  if (g.per[ax]) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int b = blockIdx.y * blockDim.y + threadIdx.y + 1;
  if (ax == 0) {
    if (a > g.ny || b > g.nz) return;
    long base = (long)b * g.sxy + (long)a * g.sx;
    p[base] = p[base + 1];
    p[base + g.nx + 1] = p[base + g.nx];
  } else if (ax == 1) {
    if (a > g.nx || b > g.nz) return;
    long base = (long)b * g.sxy + a;
    p[base] = p[base + g.sx];
    p[base + (long)(g.ny + 1) * g.sx] = p[base + (long)g.ny * g.sx];
  } else {
    if (a > g.nx || b > g.ny) return;
    long base = (long)b * g.sx + a;
    p[base] = p[base + g.sxy];
    p[base + (long)(g.nz + 1) * g.sxy] = p[base + (long)g.nz * g.sxy];
  }
}

dim3 face_grid(const Geo& g, dim3 blk, int zdim) {
  int m = g.nx > g.ny ? g.nx : g.ny;
  m = m > g.nz ? m : g.nz;
  m += 2;
  return dim3((m + blk.x - 1) / blk.x, (m + blk.y - 1) / blk.y, zdim);
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_rhs(int zr, const T* __restrict__ F, const T* __restrict__ G, const T* __restrict__ H,
      T* __restrict__ rhs, Geo g, Ctl* ctl, double* part, double tol, int unit_dt) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  rhs_cells<T>(g, zr, own_blk(), F, G, H, rhs, ctl, part, tol, unit_dt, sh, &sh_last);
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_project(int zr, const T* __restrict__ F, const T* __restrict__ G, const T* __restrict__ H,
          const double* __restrict__ p, T* __restrict__ u, T* __restrict__ v, T* __restrict__ w,
          Geo g, const Ctl* __restrict__ ctl, int unit_dt) {
  project_cells<T>(g, zr, own_blk(), F, G, H, p, u, v, w, ctl, unit_dt);
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_umax(int zr, const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w, Geo g, Ctl* ctl,
       double* part, double re, double tau, double wu, double wv, double ww) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  umax_cells<T>(g, zr, own_blk(), u, v, w, ctl, part, re, tau, wu, wv, ww, sh, &sh_last);
}

// ---------------------------------------------------------------------------
// Batched stages: workgroup b of the launch belongs to the domain whose
// [first, first + gx gy gz) holds it (binary search of the item table) and
// takes that domain's block b - first, x fastest.
__device__ __forceinline__ const StageItem& stage_item(const StageItem* __restrict__ items, int nitems,
                                                       CellBlk& blk) {
  const int b = blockIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  const StageItem& it = items[lo];
  const int l = b - it.first;
  blk.x = l % it.gx;
  blk.y = (l / it.gx) % it.gy;
  blk.z = l / (it.gx * it.gy);
  blk.id = (unsigned)l;
  blk.count = (unsigned)(it.gx * it.gy * it.gz);
  return it;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fgh_batched(const StageItem* __restrict__ items, int nitems) {
  CellBlk blk;
  const StageItem& it = stage_item(items, nitems, blk);
  const T* u = (const T*)it.in[0];
  const T* v = (const T*)it.in[1];
  const T* w = (const T*)it.in[2];
  const T* fx = (const T*)it.in[3];
  const T* fy = (const T*)it.in[4];
  const T* fz = (const T*)it.in[5];
  if (fx)
    fgh_cells<T, true>(it.g, it.zr, blk, u, v, w, fx, fy, fz, (T*)it.out[0], (T*)it.out[1], (T*)it.out[2], it.ctl,
                       it.s[0], it.s[1], it.s[2], it.s[3], it.s[4]);
  else
    fgh_cells<T, false>(it.g, it.zr, blk, u, v, w, fx, fy, fz, (T*)it.out[0], (T*)it.out[1], (T*)it.out[2], it.ctl,
                        it.s[0], it.s[1], it.s[2], it.s[3], it.s[4]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_rhs_batched(const StageItem* __restrict__ items, int nitems) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  CellBlk blk;
  const StageItem& it = stage_item(items, nitems, blk);
  rhs_cells<T>(it.g, it.zr, blk, (const T*)it.in[0], (const T*)it.in[1], (const T*)it.in[2], (T*)it.out[0], it.ctl,
               it.part, it.s[0], 0, sh, &sh_last);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_project_batched(const StageItem* __restrict__ items, int nitems) {
  CellBlk blk;
  const StageItem& it = stage_item(items, nitems, blk);
  project_cells<T>(it.g, it.zr, blk, (const T*)it.in[0], (const T*)it.in[1], (const T*)it.in[2],
                   (const double*)it.in[3], (T*)it.out[0], (T*)it.out[1], (T*)it.out[2], it.ctl, 0);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_umax_batched(const StageItem* __restrict__ items, int nitems) {
  __shared__ double sh[16];
  __shared__ int sh_last;
  CellBlk blk;
  const StageItem& it = stage_item(items, nitems, blk);
  umax_cells<T>(it.g, it.zr, blk, (const T*)it.in[0], (const T*)it.in[1], (const T*)it.in[2], it.ctl, it.part,
                it.s[0], it.s[1], it.s[2], it.s[3], it.s[4], sh, &sh_last);
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_divergence(int zr, const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
             T* __restrict__ out, Geo g) {
  for_cells(g, zr, [&](int, int, int, long c) {
    out[c] = T(((double)u[c] - (double)u[c - 1]) * g.idx + ((double)v[c] - (double)v[c - g.sx]) * g.idy +
               ((double)w[c] - (double)w[c - g.sxy]) * g.idz);
  });
}

__global__ void k_mask(double* __restrict__ q, Geo g, int comp) {
  const long n = g.ntot;
  int hi[3] = {g.nx, g.ny, g.nz};
  if (comp < 3) hi[comp] = g.hi[comp];
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const long k = t / g.sxy;
    const long rem = t - k * g.sxy;
    const long j = rem / g.sx;
    const long i = rem - j * g.sx;
    if (i < 1 || i > hi[0] || j < 1 || j > hi[1] || k < 1 || k > hi[2]) q[t] = 0.0;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_fgh_adv(int zr, const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
          const T* __restrict__ fx, const T* __restrict__ fy, const T* __restrict__ fz,
          T* __restrict__ F, T* __restrict__ G, T* __restrict__ H, Geo g, const Ctl* __restrict__ ctl,
          double nu, double alpha, double gx, double gy, double gz) {
  if (fx)
    fgh_adv_cells<T, true>(g, zr, own_blk(), u, v, w, fx, fy, fz, F, G, H, ctl, nu, alpha, gx, gy, gz);
  else
    fgh_adv_cells<T, false>(g, zr, own_blk(), u, v, w, fx, fy, fz, F, G, H, ctl, nu, alpha, gx, gy, gz);
}


// u = (a + u) / 2 (and v, w) on every entry of the padded fields: the
// combination of the two-stage Runge-Kutta step.
template <class T>
__global__ void __launch_bounds__(256)
k_average(long n, const T* __restrict__ a0, const T* __restrict__ a1, const T* __restrict__ a2,
          T* __restrict__ q0, T* __restrict__ q1, T* __restrict__ q2) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    q0[e] = T(0.5 * ((double)a0[e] + (double)q0[e]));
    q1[e] = T(0.5 * ((double)a1[e] + (double)q1[e]));
    q2[e] = T(0.5 * ((double)a2[e] + (double)q2[e]));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

template <class T>
hipError_t launch_bc_vel(hipStream_t st, const Geo& g, T* u, T* v, T* w, const double wall[6][3]) {
  dim3 blk(64, 4);
  dim3 grd = face_grid(g, blk, 3);
  if (!(g.per[0] && g.per[1] && g.per[2])) {
    Wall wl;
    for (int f = 0; f < 6; f++)
      for (int c = 0; c < 3; c++) wl.v[f][c] = wall[f][c];
    k_bc_normal<T><<<grd, blk, 0, st>>>(u, v, w, g);
    k_bc_reflect<T><<<grd, blk, 0, st>>>(u, v, w, g, wl);
  }
  for (int ax = 0; ax < 3; ax++)
    if (g.per[ax]) k_periodic<T><<<face_grid(g, blk, 1), blk, 0, st>>>(u, v, w, g, ax);
  return hipGetLastError();
}

template <class T>
hipError_t launch_p_ghosts(hipStream_t st, const Geo& g, T* p) {
  dim3 blk(64, 4);
  if (!(g.per[0] && g.per[1] && g.per[2])) k_p_neumann<T><<<face_grid(g, blk, 3), blk, 0, st>>>(p, g);
  for (int ax = 0; ax < 3; ax++)
    if (g.per[ax]) k_periodic<T><<<face_grid(g, blk, 1), blk, 0, st>>>(p, nullptr, nullptr, g, ax);
  return hipGetLastError();
}

template <class T>
hipError_t launch_periodic(hipStream_t st, const Geo& g, T* q, int axis) {
  dim3 blk(64, 4);
  k_periodic<T><<<face_grid(g, blk, 1), blk, 0, st>>>(q, nullptr, nullptr, g, axis);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fgh_advective(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, const T* fx,
                                const T* fy, const T* fz, T* F, T* G, T* H, const Ctl* ctl, double re, double alpha,
                                const double gf[3]) {
  k_fgh_adv<T><<<cell_grid(g, 0), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, 0), u, v, w, fx, fy, fz, F, G, H, g,
                                                                  ctl, 1.0 / re, alpha, gf[0], gf[1], gf[2]);
  return hipGetLastError();
}
template hipError_t launch_fgh_advective<double>(hipStream_t, const Geo&, const double*, const double*, const double*,
                                                 const double*, const double*, const double*, double*, double*,
                                                 double*, const Ctl*, double, double, const double[3]);
template hipError_t launch_fgh_advective<float>(hipStream_t, const Geo&, const float*, const float*, const float*,
                                                const float*, const float*, const float*, float*, float*, float*,
                                                const Ctl*, double, double, const double[3]);

size_t reduce_blocks(const Geo& g) {
  long n = (long)g.nx * g.ny * g.nz;
  size_t m = (size_t)grid_for(n);
  if ((size_t)cell_blocks(g, kRedRhs) > m) m = cell_blocks(g, kRedRhs);
  if ((size_t)cell_blocks(g, kRedDefect) > m) m = cell_blocks(g, kRedDefect);
  // the fused sweep has the most workgroups with 4 rows and 1-plane chunks
  const size_t f = (size_t)fused_num_blocks(g, SorShape{4, 1});
  if (f > m) m = f;
  if ((size_t)pass_max_partials(g) > m) m = pass_max_partials(g);
  return 4 * m + 64;
}

template <class T>
hipError_t launch_rhs(hipStream_t st, const Geo& g, const T* F, const T* G, const T* H, T* rhs,
                      Ctl* ctl, double* part, double tol, double unit_dt) {
  k_rhs<T><<<cell_grid(g, kRedRhs), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, kRedRhs), F, G, H, rhs, g, ctl, part, tol, unit_dt != 0.0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_average(hipStream_t st, const Geo& g, const T* a0, const T* a1, const T* a2, T* q0, T* q1, T* q2) {
  const long n = g.ntot;
  long nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  k_average<T><<<(unsigned)nb, 256, 0, st>>>(n, a0, a1, a2, q0, q1, q2);
  return hipGetLastError();
}

template <class T>
hipError_t launch_project(hipStream_t st, const Geo& g, const T* F, const T* G, const T* H,
                          const double* p, T* u, T* v, T* w, const Ctl* ctl, double unit_dt) {
  k_project<T><<<cell_grid(g, 0), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, 0), F, G, H, p, u, v, w, g, ctl, unit_dt != 0.0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_umax(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, Ctl* ctl,
                       double* part, double re, double tau, const double wall[6][3]) {
  double wm[3] = {0, 0, 0};
  for (int f = 0; f < 6; f++)
    for (int c = 0; c < 3; c++) wm[c] = fmax(wm[c], fabs(wall[f][c]));
  k_umax<T><<<cell_grid(g, kRedRhs), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, kRedRhs), u, v, w, g, ctl, part, re, tau, wm[0], wm[1], wm[2]);
  return hipGetLastError();
}

template <class T>
hipError_t launch_divergence(hipStream_t st, const Geo& g, const T* u, const T* v, const T* w, T* out) {
  k_divergence<T><<<cell_grid(g, 0), dim3(kCellX, kCellY), 0, st>>>(cell_zrun(g, 0), u, v, w, out, g);
  return hipGetLastError();
}

template <class T>
hipError_t launch_stage_batched(hipStream_t st, int kind, const StageItem* d_items, int nitems, int nblocks) {
  if (nitems <= 0 || nblocks <= 0) return hipSuccess;
  const dim3 blk(kCellX, kCellY);
  switch (kind) {
    case kStageFgh: k_fgh_batched<T><<<nblocks, blk, 0, st>>>(d_items, nitems); break;
    case kStageRhs: k_rhs_batched<T><<<nblocks, blk, 0, st>>>(d_items, nitems); break;
    case kStageProject: k_project_batched<T><<<nblocks, blk, 0, st>>>(d_items, nitems); break;
    case kStageUmax: k_umax_batched<T><<<nblocks, blk, 0, st>>>(d_items, nitems); break;
    case kStageDefect: return launch_defect_batched(st, d_items, nitems, nblocks);
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mask_unknowns(hipStream_t st, const Geo& g, double* q, int comp) {
  k_mask<<<grid_for(g.ntot, 1 << 16), kBlock, 0, st>>>(q, g, comp);
  return hipGetLastError();
}

#define NS_INST(T)                                                                                  \
  template hipError_t launch_bc_vel<T>(hipStream_t, const Geo&, T*, T*, T*, const double[6][3]);    \
  template hipError_t launch_p_ghosts<T>(hipStream_t, const Geo&, T*);                              \
  template hipError_t launch_periodic<T>(hipStream_t, const Geo&, T*, int);                         \
  template hipError_t launch_rhs<T>(hipStream_t, const Geo&, const T*, const T*, const T*, T*,      \
                                    Ctl*, double*, double, double);                                 \
  template hipError_t launch_average<T>(hipStream_t, const Geo&, const T*, const T*, const T*, T*, T*, T*); \
  template hipError_t launch_project<T>(hipStream_t, const Geo&, const T*, const T*, const T*,      \
                                        const double*, T*, T*, T*, const Ctl*, double);             \
  template hipError_t launch_umax<T>(hipStream_t, const Geo&, const T*, const T*, const T*, Ctl*,   \
                                     double*, double, double, const double[6][3]);                  \
  template hipError_t launch_divergence<T>(hipStream_t, const Geo&, const T*, const T*, const T*, T*);       \
  template hipError_t launch_stage_batched<T>(hipStream_t, int, const StageItem*, int, int);

NS_INST(double)
NS_INST(float)

}  // namespace ns
