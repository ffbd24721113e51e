// ns_internal.h -- shared declarations of the gfx950 HIP implementation of
// the staggered-grid Navier-Stokes step (kernels + host runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ns.h"

namespace ns {

// Grid geometry passed by value to every kernel.  Fields use the padded
// layout [nz+2][ny+2][nx+2], x fastest: index = k*sxy + j*sx + i.
struct Geo {
  int nx, ny, nz;
  long sx, sxy, ntot;
  double dx, dy, dz;
  double idx, idy, idz;     // 1/h
  double idx2, idy2, idz2;  // 1/h^2
  int per[3];               // 1 = periodic axis
  int hi[3];                // last normal-velocity unknown of u, v, w along its own axis
};

// Per-instance device control block.  Written by the last workgroup of the
// reduction kernels; read by later kernels of the same step and polled by
// the host (one small async copy per chunk of sweeps).
struct Ctl {
  double dt;       // current step size
  double thr;      // absolute stop threshold of the Poisson solve: tol * RMS(rhs)
  double thr_in;   // mixed: inner threshold eta * outer residual
  double res;      // RMS residual of the accepted pressure (or of the last outer check)
  double rhs_rms;  // RMS of the right-hand side
  double res_in;   // mixed: last inner residual checked
  double umax[3];  // adaptive dt: max |u|, |v|, |w|
  int32_t done;    // solve (FP64) or inner loop (mixed) finished
  int32_t final_;  // sweep index whose iterate is the answer
  int32_t nonfinite;
  int32_t outer_done;  // mixed: outer residual met the tolerance
  uint32_t ticket;     // last-workgroup counter of reductions (reset by the last group)
  int32_t pad_[9];     // one 128-byte cache line per control block: kernels of different
                       // instances run concurrently on different XCDs, whose L2s are not
                       // coherent with each other, and must not share a line
};
static_assert(sizeof(Ctl) == 128, "control block is one 128-byte line");

// Tunables of the red-black sweep (chosen per grid by the autotuner).
// ty = 4 / 8 / 12: fused one-sweep kernel with ty interior rows per
// workgroup (the x width is fixed at 60 = 64 - 4 halo); ty = 16 / 24 / 32:
// pass kernel, two sweeps per launch, ty rows per workgroup including the
// 4-cell halo on each side; zc planes per z chunk (0 = whole column).
// ty < 0: unfused reference kernels (one pass per colour).
struct SorShape {
  int ty;
  int zc;
};
inline bool shape_is_pass(const SorShape& s) { return s.ty >= 16; }

// ---- kernel launchers (kernels.hip / sor.hip / adjoint.hip) ----
// All launchers enqueue on `st` and return the hipGetLastError() status.
template <class T> hipError_t launch_bc_vel(hipStream_t st, const Geo& g, T* u, T* v, T* w,
                                           const double wall[6][3]);
template <class T> hipError_t launch_p_ghosts(hipStream_t st, const Geo& g, T* p);
// q = (a + q) / 2 on every entry of three padded fields (the two-stage
// Runge-Kutta combination).
template <class T> hipError_t launch_average(hipStream_t st, const Geo& g, const T* a0, const T* a1, const T* a2,
                                            T* q0, T* q1, T* q2);
template <class T> hipError_t launch_rhs(hipStream_t st, const Geo& g, const T* F, const T* G,
                                        const T* H, T* rhs, Ctl* ctl, double* part, double tol,
                                        double dt_scale_one);
template <class T> hipError_t launch_project(hipStream_t st, const Geo& g, const T* F, const T* G,
                                            const T* H, const double* p, T* u, T* v, T* w,
                                            const Ctl* ctl, double dt_scale_one);
template <class T> hipError_t launch_umax(hipStream_t st, const Geo& g, const T* u, const T* v,
                                         const T* w, Ctl* ctl, double* part, double re,
                                         double tau, const double wall[6][3]);

// One red-black SOR sweep p_in -> p_out (out of place) on A p = rhs, fused
// with the RMS residual of p_in.  sweep_idx = index m of this sweep (1-based):
// the residual computed is that of iterate m-1; the last workgroup decides
// convergence (iterate m-1 accepted when m-1 >= 1 and res <= thr) and sets
// ctl->done / ctl->final_.  write = 0 computes only the residual (used after
// the last allowed sweep).  zero_in = 1 treats p_in as identically zero (it
// is not read).  thr_is_inner selects ctl->thr_in.
template <class T> hipError_t launch_sor_sweep(hipStream_t st, const Geo& g, const T* p_in, T* p_out,
                                              const T* rhs, Ctl* ctl, double* part, double omega,
                                              int sweep_idx, int itermax, int write, int zero_in,
                                              int thr_is_inner, const SorShape& shape);
// Mixed-precision outer step: p_out = p_in + e (e == null: p_out unused and
// not written), r = rhs - A p_out in FP64 stored as float, RMS(r) -> ctl.
hipError_t launch_defect(hipStream_t st, const Geo& g, const double* p_in, const float* e,
                         double* p_out, const float* rhs, float* r, Ctl* ctl, double* part,
                         double eta);

size_t reduce_blocks(const Geo& g);  // partial-sum slots any reduction may need

// Cell kernels run 64 x 4 threads per workgroup over (x, y); the
// workgroups of one (x, y) tile split z into runs of consecutive planes.
// Consecutive lanes take consecutive x, so a wave reads 64 contiguous values
// per row.  Kernels without a reduction take short runs (many workgroups);
// kernels with one take runs long enough that about `target` workgroups
// remain, whose partial sums the last workgroup adds up (measured at 512^3:
// 1024, i.e. whole z columns there).
#ifndef NS_CELL_Z
#define NS_CELL_Z 4  // planes per workgroup, kernels without a reduction
#endif
constexpr int kCellX = 64, kCellY = 4;
constexpr long kRedRhs = 1024, kRedDefect = 1024;
inline int cell_zrun(const Geo& g, long target) {
  const long cols = (long)((g.nx + kCellX - 1) / kCellX) * ((g.ny + kCellY - 1) / kCellY);
  long z = NS_CELL_Z;
  if (target > 0) {
    const long want = (cols * g.nz + target - 1) / target;
    if (want > z) z = want;
  }
  const long minz = (g.nz + 65534) / 65535;  // grid z limit
  if (z < minz) z = minz;
  return (int)(z < g.nz ? z : g.nz);
}
inline dim3 cell_grid(const Geo& g, long target) {
  const int bx = (g.nx + kCellX - 1) / kCellX, by = (g.ny + kCellY - 1) / kCellY;
  const int zr = cell_zrun(g, target);
  return dim3(bx, by, (g.nz + zr - 1) / zr);
}
// Position of a cell-kernel workgroup in the workgroup grid of its domain:
// block (x, y, z), its linear index and the domain's workgroup count (the
// slot and count of a reduction's partial sums).
struct CellBlk {
  int x, y, z;
  unsigned id, count;
};
__device__ __forceinline__ CellBlk own_blk() {
  return CellBlk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z,
                 blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                 gridDim.x * gridDim.y * gridDim.z};
}
// f(i, j, k, c) for every interior cell of workgroup b's (x, y) tile and
// run of zr planes; UNROLL planes per loop trip (their loads in flight
// together).
template <int UNROLL = 1, class F>
__device__ __forceinline__ void for_cells(const Geo& g, int zr, const CellBlk& b, F&& f) {
  const int i = b.x * kCellX + threadIdx.x + 1;
  const int j = b.y * (int)blockDim.y + threadIdx.y + 1;
  if (i > g.nx || j > g.ny) return;
  const int k0 = b.z * zr + 1;
  const int k1 = min(g.nz, k0 + zr - 1);
  long c = (long)k0 * g.sxy + (long)j * g.sx + i;
#pragma unroll(UNROLL)
  for (int k = k0; k <= k1; k++, c += g.sxy) f(i, j, k, c);
}
template <class F>
__device__ __forceinline__ void for_cells(const Geo& g, int zr, F&& f) {
  for_cells(g, zr, own_blk(), f);
}
inline unsigned cell_blocks(const Geo& g, long target) {
  const dim3 d = cell_grid(g, target);
  return d.x * d.y * d.z;
}
int sor_num_blocks(const Geo& g, const SorShape& s);
// Fused sweep (one pass): shape.ty rows per workgroup in {4, 8, 12},
// shape.zc planes per z chunk (0 = whole column).
template <class T> hipError_t launch_sor_fused(hipStream_t st, const Geo& g, const T* p_in, T* p_out,
                                              const T* rhs, Ctl* ctl, double* part, double omega,
                                              int sweep_idx, int itermax, int write, int zero_in,
                                              int thr_is_inner, const SorShape& shape);
int fused_num_blocks(const Geo& g, const SorShape& s);
// Pass kernel (sor_pass.hip): ns = 1 or 2 sweeps per launch, first sweep
// index m (input iterate m - 1).  part == nullptr forces the sweep whatever
// the done flag says and skips the residual and stop rule.
template <class T> hipError_t launch_sor_pass(hipStream_t st, const Geo& g, const T* p_in, T* p_out,
                                             const T* rhs, Ctl* ctl, double* part, double omega, int m,
                                             int itermax, int write, int zero_in, int inner, int ns,
                                             const SorShape& shape);
bool pass_shape_ok(const SorShape& s);
bool pass_rows_ok(int rows, bool f32);  // FP64: 16 rows only; FP32: 16, 24 or 32
bool pass_grid_ok(const Geo& g, size_t esz);  // periodic axes >= 4 cells, plane offsets in 31 bits
int pass_max_partials(const Geo& g);
int pass_resident_groups(int ty, bool f32, int ns);
int pass_columns(const Geo& g, int ty, int ns);
bool fused_shape_ok(const SorShape& s);
int fused_resident(int ty, bool f32);       // workgroups resident on the device at once
int fused_columns(const Geo& g, int ty);    // x-y tiles of one z chunk

// One domain of a batched sweep (device-resident table, sorted by `first`).
struct BatchItem {
  Geo g;
  void* p[2];      // iterate buffers; sweep m reads p[(cur + m - 1) & 1], writes p[(cur + m) & 1]
  const void* rhs;
  Ctl* ctl;
  double* part;
  double omega;
  int cur;
  int first;       // first workgroup of this domain
  int ntiles, ntx, nty, zc;
  int budget;      // the solve stops at iterate `budget` at the latest
  int inner;       // 1: correction solve (stop at ctl->thr_in)
};
// Planes per z chunk of a domain with nz planes: zc > 0 fixed chunks of zc
// planes, zc = 0 the whole column, zc < 0 the fewest chunks of at most -zc
// planes, equally long (so the tiles of domains of different heights come
// out of similar length).
inline int item_chunk(int nz, int zc) {
  if (zc > 0) return zc < nz ? zc : nz;
  if (zc < 0) {
    const int parts = (nz - zc - 1) / (-zc);
    return (nz + parts - 1) / parts;
  }
  return nz;
}
// Fill ntx, nty, zc and ntiles of an item for a sweep shape.
void batch_item_shape(BatchItem& it, int ty, int zc);
// One sweep of every domain of a batch in one launch (nblocks = sum of ntiles).
template <class T> hipError_t launch_sor_batched(hipStream_t st, const BatchItem* d_items, int nitems,
                                                int nblocks, int ty, int m, int write, int zero_in);
// Pass-kernel geometry of an item (rows 16 / 24 / 32, ns sweeps per pass)
// and one batched pass: first sweep index m, pass q of every domain reads
// p[(cur + q) & 1]; force sweeps regardless of done flags without residuals.
void pass_item_shape(BatchItem& it, int rows, int zc, int ns);
template <class T> hipError_t launch_pass_batched(hipStream_t st, const BatchItem* d_items, int nitems,
                                                 int nblocks, int rows, int m, int q, int ns, int zero_in,
                                                 int force);

// One domain of a batched cell-kernel launch (one launch of a stage covers
// every domain of a batch): the domain's geometry, its workgroups
// [first, first + gx gy gz) of the launch, planes per workgroup, and the
// stage's arguments (meaning per stage, see launch_stage_batched).
struct StageItem {
  Geo g;
  int first;
  int gx, gy, gz, zr;
  const void* in[6];
  void* out[3];
  Ctl* ctl;
  double* part;
  double s[6];
};
// Host: workgroup grid of a domain for a batched stage: whole z columns for
// a reducing stage, the single-domain grid otherwise.
inline void stage_item_grid(StageItem& it, bool whole_columns) {
  const dim3 d = cell_grid(it.g, 0);
  it.gx = (int)d.x;
  it.gy = (int)d.y;
  it.gz = whole_columns ? 1 : (int)d.z;
  it.zr = whole_columns ? it.g.nz : cell_zrun(it.g, 0);
}
enum StageKind { kStageFgh = 0, kStageRhs, kStageProject, kStageUmax, kStageDefect, kStageKinds };
// Stages that end in a reduction over the domain.  Every workgroup of such
// a stage publishes its partial behind a device-scope fence, whose cost does
// not shrink with the workgroup's share of the work; a batched launch
// therefore gives each workgroup of these stages a whole z column (the
// other stages keep the single-domain grid).
inline bool stage_reduces(int kind) { return kind == kStageRhs || kind == kStageUmax || kind == kStageDefect; }
// One launch of a stage over nitems domains (nblocks = sum of their
// workgroups), the same per-cell arithmetic as the single-domain kernels.
//   kStageFgh:     in = u, v, w, fx, fy, fz; out = F, G, H; s = nu, gamma, gx, gy, gz (dt from ctl)
//   kStageRhs:     in = F, G, H; out = rhs; s = tol (dt from ctl)
//   kStageProject: in = F, G, H, p (FP64); out = u, v, w (dt from ctl)
//   kStageUmax:    in = u, v, w; s = re, tau, wall speed x, y, z
//   kStageDefect:  in = p_in (FP64), e (FP32 or null), rhs (FP32); out = p_out (FP64), r (FP32); s = eta
template <class T> hipError_t launch_stage_batched(hipStream_t st, int kind, const StageItem* d_items, int nitems,
                                                  int nblocks);
hipError_t launch_defect_batched(hipStream_t st, const StageItem* d_items, int nitems, int nblocks);

// ---- persistent batched launch (persist.hip) ----
// Workgroups of 64 x W threads (W waves: 16 for FP32 storage, 8 for FP64,
// one workgroup per compute unit); cell-stage blocks of 64 x W cells and
// kPersistZr planes; two-sweep pass tiles of R rows per lane, R x W rows.
constexpr int kPersistWaves32 = 16, kPersistWaves64 = 8;
constexpr int kPersistRpl32 = 2, kPersistRpl64 = 2;
inline int persist_waves(bool f32) { return f32 ? kPersistWaves32 : kPersistWaves64; }
inline int persist_rows(bool f32) {
  return f32 ? kPersistRpl32 * kPersistWaves32 : kPersistRpl64 * kPersistWaves64;
}
constexpr int kPersistZr = 4;
// Statistics of one domain, kept on the device across the launch (the
// host's ns_stats plus the pressure buffer in use and the sweep time).
struct PStats {
  double t, dt_last, res_last;
  long long sweeps_total;
  int steps, sweeps_max, steps_unconverged, outer_max;
  int pcur;          // pressure buffer holding the state
  int nonfinite;     // a NaN / Inf reached a residual norm
  double sweep_ticks;  // wall-clock ticks the team's lead spent in Poisson solves
};
// One domain of a persistent launch.  Buffers hold the storage type T of
// the launch (float: mixed precision, double: FP64) except p (FP64).
struct PItem {
  Geo g;
  void* u;
  void* v;
  void* w;
  void* F;
  void* G;
  void* H;
  void* rhs;
  const void* frc[3];  // body-force fields or null
  double* p[2];        // pressure buffers
  void* e[2];          // mixed: correction iterates (FP32)
  void* r;             // mixed: defect (FP32)
  double* part;        // partial sums, at least 6 * team + 8 slots
  Ctl* ctl;            // control block (initial dt in, final state out)
  PStats* st;
  unsigned* bar;       // team barrier counter, zero at launch
  double wall[6][3];
  double wmax[3];      // largest wall speed per component
  double gforce[3];
  double re, tau, gamma, omega, tol, eta;
  int adaptive;        // dt from the velocity every step
  int itermax;
  int ns_max;          // sweeps per pass (1 or 2)
  int team;            // workgroups of the domain's team
  int cgx, cgy, cgz;   // cell-stage blocks per axis
};
// Workgroup b of the launch: its domain (-1: idle) and rank in the team.
struct PSlot {
  int item, rank;
};
int persistent_resident(bool f32);  // co-resident workgroups of the launch
// Cooperative launch of nblocks workgroups running nsteps steps of every
// domain; err: device flag raised when a barrier wait exceeds `limit`
// wall-clock ticks (the grid then drains).
hipError_t launch_persistent(hipStream_t st, bool f32, const PItem* items, const PSlot* slots, int nblocks,
                             int nsteps, int* err, long long limit);

// Adjoint of the predictor in gather form (FP64 only): z = B^T J_Phi(u)^T mu.
hipError_t launch_adj_fgh(hipStream_t st, const Geo& g, const double* u, const double* v,
                          const double* w, const double* mu, const double* mv, const double* mw,
                          double* zu, double* zv, double* zw, double dt, double re, double gamma);
hipError_t launch_adj_fold(hipStream_t st, const Geo& g, double* zu, double* zv, double* zw);
// Zero every entry that is not an unknown of component comp (3 = cells).
hipError_t launch_mask_unknowns(hipStream_t st, const Geo& g, double* q, int comp);
// Periodic images of face / cell fields (full extent), axis by axis.
template <class T> hipError_t launch_periodic(hipStream_t st, const Geo& g, T* q, int axis);
template <class T> hipError_t launch_divergence(hipStream_t st, const Geo& g, const T* u, const T* v,
                                               const T* w, T* out);

}  // namespace ns
