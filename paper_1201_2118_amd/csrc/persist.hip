// persist.hip -- every step of every domain of a batch in one persistent
// cooperative launch.
//
// The workgroups of the launch (as many as are co-resident) are split into
// teams, one per domain, sized by the length of the domain's pass and placed on
// one XCD each (workgroup b runs on XCD b mod 8).  A team runs its domain's
// steps on its own: every stage (time step, boundary fill, predictor, rhs,
// the Poisson solve, pressure ghosts, projection) is spread over the team's
// workgroups, and a team barrier (a counter in device memory, device-scope
// release / acquire) separates a stage from the next one that reads what it
// wrote.  Reductions write one partial per workgroup; after the barrier
// every workgroup of the team sums the partials in the same order, so all
// of them take the same decision (stop rule, time step) without a second
// barrier and without the host: the stop rules, the sweep budget, the
// mixed-precision defect correction and the choice of the buffer that
// holds the accepted iterate all run on the device.  Per-cell arithmetic is
// that of the other paths (cells.h, pass_tile.h): two red-black sweeps per
// pass with temporal blocking, the forced single sweep that materialises an
// iterate a pass held only in registers, the residual-only pass after the
// last allowed sweep.
//
// Every barrier wait is bounded: a workgroup that waits longer than the
// launch's limit (wall-clock ticks) raises the error flag and returns; a
// waiting workgroup that sees the flag returns too, so the grid always
// drains and the host reports the failure.
#include <hip/hip_runtime.h>

#include "cells.h"
#include "ns_internal.h"
#include "pass_tile.h"
#include "reduce.h"

namespace ns {

namespace {

template <class T>
constexpr int waves_of() {
  return sizeof(T) == 4 ? kPersistWaves32 : kPersistWaves64;
}
template <class T>
constexpr int rpl_of() {  // rows per lane of the pass tile
  return sizeof(T) == 4 ? kPersistRpl32 : kPersistRpl64;
}

// A value every lane of the wave holds alike (read from LDS after a
// barrier), made visibly uniform so that what depends on it (buffer
// choices, loop exits) stays in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class P>
__device__ __forceinline__ P* uni_ptr(P* p) {
  const unsigned long long b = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long uni_long(long v) {
  const unsigned long long b = (unsigned long long)v;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return (long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uni_dbl(double v) {
  return __builtin_bit_cast(double, uni_long(__builtin_bit_cast(long, v)));
}
// The domain's geometry in scalar registers (read from the item table once).
__device__ __forceinline__ Geo uni_geo(const Geo& s) {
  Geo g;
  g.nx = uni(s.nx); g.ny = uni(s.ny); g.nz = uni(s.nz);
  g.sx = uni_long(s.sx); g.sxy = uni_long(s.sxy); g.ntot = uni_long(s.ntot);
  g.dx = uni_dbl(s.dx); g.dy = uni_dbl(s.dy); g.dz = uni_dbl(s.dz);
  g.idx = uni_dbl(s.idx); g.idy = uni_dbl(s.idy); g.idz = uni_dbl(s.idz);
  g.idx2 = uni_dbl(s.idx2); g.idy2 = uni_dbl(s.idy2); g.idz2 = uni_dbl(s.idz2);
  for (int a = 0; a < 3; a++) {
    g.per[a] = uni(s.per[a]);
    g.hi[a] = uni(s.hi[a]);
  }
  return g;
}

struct Team {
  int rank, size;
  unsigned gen;  // barriers passed
  unsigned* bar;
  int* err;
  long long limit;
};

// Team barrier; false (in every thread) when the wait gave up or another
// workgroup raised the error flag.
__device__ __forceinline__ bool team_sync(Team& t, int* sh_flag) {
  __syncthreads();
  t.gen += 1;
  if (flat_tid() == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this workgroup's writes before its arrival
    atomicAdd(t.bar, 1u);
    const unsigned target = t.gen * (unsigned)t.size;
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(t.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(t.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      if (wall_clock64() - t0 > t.limit) {
        atomicExch(t.err, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the team's writes after the wait
    *sh_flag = ok;
  }
  __syncthreads();
  return uni(*sh_flag) != 0;
}

// Cell-stage block vb of a domain (64 lanes x one row per wave, kPersistZr
// planes).
__device__ __forceinline__ CellBlk vblock(const PItem& it, int vb) {
  CellBlk b;
  b.x = vb % it.cgx;
  b.y = (vb / it.cgx) % it.cgy;
  b.z = vb / (it.cgx * it.cgy);
  b.id = (unsigned)vb;
  b.count = (unsigned)(it.cgx * it.cgy * it.cgz);
  return b;
}

// f(e) for the entries e = 0 .. n - 1 of a face phase, spread over the
// team's threads.
template <class F>
__device__ __forceinline__ void team_loop(const Team& t, long n, F&& f) {
  const int nt = (int)(blockDim.x * blockDim.y);
  for (long e = (long)t.rank * nt + flat_tid(); e < n; e += (long)t.size * nt) f(e);
}

// Periodic images of entry (a, b) of the face of axis ax (full extent of
// the other two axes) for up to three fields (null skipped); the body of the
// single-domain periodic kernel.
template <class T>
__device__ __forceinline__ void periodic_entry(const Geo& g, int ax, int a, int b, T* q0, T* q1, T* q2) {
  long lo, hi, src_lo, src_hi;
  if (ax == 0) {
    if (a > g.ny + 1 || b > g.nz + 1) return;
    const long base = (long)b * g.sxy + (long)a * g.sx;
    lo = base; hi = base + g.nx + 1; src_lo = base + g.nx; src_hi = base + 1;
  } else if (ax == 1) {
    if (a > g.nx + 1 || b > g.nz + 1) return;
    const long base = (long)b * g.sxy + a;
    lo = base; hi = base + (long)(g.ny + 1) * g.sx;
    src_lo = base + (long)g.ny * g.sx; src_hi = base + g.sx;
  } else {
    if (a > g.nx + 1 || b > g.ny + 1) return;
    const long base = (long)b * g.sx + a;
    lo = base; hi = base + (long)(g.nz + 1) * g.sxy;
    src_lo = base + (long)g.nz * g.sxy; src_hi = base + g.sxy;
  }
  T* q[3] = {q0, q1, q2};
#pragma unroll
  for (int f = 0; f < 3; f++)
    if (q[f]) {
      const T a0 = q[f][src_lo], a1 = q[f][src_hi];
      q[f][lo] = a0;
      q[f][hi] = a1;
    }
}

// Boundary fill of the velocity: wall-normal faces, then tangential
// reflections, then periodic images axis by axis (the order of the
// single-domain launches), one team barrier after each phase.
template <class T>
__device__ __forceinline__ bool bc_vel_team(const PItem& it, const Geo& g, Team& t, T* u, T* v, T* w, int* fl) {
  int M = g.nx > g.ny ? g.nx : g.ny;
  M = (M > g.nz ? M : g.nz) + 2;
  const long MM = (long)M * M;
  if (!(g.per[0] && g.per[1] && g.per[2])) {
    team_loop(t, 3 * MM, [&](long e) {
      const int ax = (int)(e / MM);
      const long rem = e - ax * MM;
      const int a = (int)(rem % M), b = (int)(rem / M);
      if (g.per[ax]) return;
      if (ax == 0) {
        if (a > g.ny + 1 || b > g.nz + 1) return;
        const long base = (long)b * g.sxy + (long)a * g.sx;
        u[base] = T(0);
        u[base + g.nx] = T(0);
      } else if (ax == 1) {
        if (a > g.nx + 1 || b > g.nz + 1) return;
        const long base = (long)b * g.sxy + a;
        v[base] = T(0);
        v[base + (long)g.ny * g.sx] = T(0);
      } else {
        if (a > g.nx + 1 || b > g.ny + 1) return;
        const long base = (long)b * g.sx + a;
        w[base] = T(0);
        w[base + (long)g.nz * g.sxy] = T(0);
      }
    });
    if (!team_sync(t, fl)) return false;
    team_loop(t, 3 * MM, [&](long e) {
      const int ax = (int)(e / MM);
      const long rem = e - ax * MM;
      const int a = (int)(rem % M) + 1, b = (int)(rem / M) + 1;
      if (g.per[ax]) return;
      const double(*wl)[3] = it.wall;
      if (ax == 0) {
        if (a > g.ny || b > g.nz) return;
        const long base = (long)b * g.sxy + (long)a * g.sx;
        v[base] = T(2.0 * wl[0][1] - (double)v[base + 1]);
        w[base] = T(2.0 * wl[0][2] - (double)w[base + 1]);
        v[base + g.nx + 1] = T(2.0 * wl[1][1] - (double)v[base + g.nx]);
        w[base + g.nx + 1] = T(2.0 * wl[1][2] - (double)w[base + g.nx]);
      } else if (ax == 1) {
        if (a > g.nx || b > g.nz) return;
        const long base = (long)b * g.sxy + a;
        const long top = base + (long)(g.ny + 1) * g.sx;
        u[base] = T(2.0 * wl[2][0] - (double)u[base + g.sx]);
        w[base] = T(2.0 * wl[2][2] - (double)w[base + g.sx]);
        u[top] = T(2.0 * wl[3][0] - (double)u[top - g.sx]);
        w[top] = T(2.0 * wl[3][2] - (double)w[top - g.sx]);
      } else {
        if (a > g.nx || b > g.ny) return;
        const long base = (long)b * g.sx + a;
        const long top = base + (long)(g.nz + 1) * g.sxy;
        u[base] = T(2.0 * wl[4][0] - (double)u[base + g.sxy]);
        v[base] = T(2.0 * wl[4][1] - (double)v[base + g.sxy]);
        u[top] = T(2.0 * wl[5][0] - (double)u[top - g.sxy]);
        v[top] = T(2.0 * wl[5][1] - (double)v[top - g.sxy]);
      }
    });
    if (!team_sync(t, fl)) return false;
  }
  for (int ax = 0; ax < 3; ax++) {
    if (!g.per[ax]) continue;
    team_loop(t, MM, [&](long e) { periodic_entry(g, ax, (int)(e % M), (int)(e / M), u, v, w); });
    if (!team_sync(t, fl)) return false;
  }
  return true;
}

// Pressure ghosts: Neumann copies on wall axes, periodic images otherwise.
__device__ __forceinline__ bool p_ghosts_team(const PItem& it, const Geo& g, Team& t, double* p, int* fl) {
  int M = g.nx > g.ny ? g.nx : g.ny;
  M = (M > g.nz ? M : g.nz) + 2;
  const long MM = (long)M * M;
  if (!(g.per[0] && g.per[1] && g.per[2])) {
    team_loop(t, 3 * MM, [&](long e) {
      const int ax = (int)(e / MM);
      const long rem = e - ax * MM;
      const int a = (int)(rem % M) + 1, b = (int)(rem / M) + 1;
      if (g.per[ax]) return;
      if (ax == 0) {
        if (a > g.ny || b > g.nz) return;
        const long base = (long)b * g.sxy + (long)a * g.sx;
        p[base] = p[base + 1];
        p[base + g.nx + 1] = p[base + g.nx];
      } else if (ax == 1) {
        if (a > g.nx || b > g.nz) return;
        const long base = (long)b * g.sxy + a;
        p[base] = p[base + g.sx];
        p[base + (long)(g.ny + 1) * g.sx] = p[base + (long)g.ny * g.sx];
      } else {
        if (a > g.nx || b > g.ny) return;
        const long base = (long)b * g.sx + a;
        p[base] = p[base + g.sxy];
        p[base + (long)(g.nz + 1) * g.sxy] = p[base + (long)g.nz * g.sxy];
      }
    });
    if (!team_sync(t, fl)) return false;
  }
  for (int ax = 0; ax < 3; ax++) {
    if (!g.per[ax]) continue;
    team_loop(t, MM, [&](long e) { periodic_entry<double>(g, ax, (int)(e % M), (int)(e / M), p, nullptr, nullptr); });
    if (!team_sync(t, fl)) return false;
  }
  return true;
}

// One pass of NS sweeps of the team over its domain: rank r takes an equal
// share of the (plane-column, plane) space in column order, cut at column
// ends into z ranges.  acc1 / acc2: this workgroup's sums of the squared
// residuals of the input iterate and (NS = 2) of the first sweep's iterate.
template <class T, int NS, bool ZIN>
__device__ __forceinline__ void team_pass(const PItem& it, const Geo& g, const Team& t, const T* pin, T* pout, const T* rhs, int write,
                          T* E, double& acc1, double& acc2) {
  constexpr int H = 2 * NS;
  constexpr int W = waves_of<T>(), R = rpl_of<T>();
  const int ntx = (g.nx + (64 - 2 * H) - 1) / (64 - 2 * H);
  const int nty = (g.ny + (R * W - 2 * H) - 1) / (R * W - 2 * H);
  const long ptot = (long)ntx * nty * g.nz;
  long q0 = ptot * t.rank / t.size;
  const long q1 = ptot * (t.rank + 1) / t.size;
  while (q0 < q1) {
    const int col = (int)(q0 / g.nz);
    const int z0 = (int)(q0 - (long)col * g.nz) + 1;
    const int z1 = (int)min((long)g.nz, (long)z0 + (q1 - q0) - 1);
    pass_tile<T, NS, R, W, ZIN, true>(uni_ptr(pin), uni_ptr(pout), uni_ptr(rhs), g, it.omega, write, col, z0, z1,
                                          ntx, E, acc1, acc2);
    __syncthreads();
    q0 += z1 - z0 + 1;
  }
}

template <class T>
__device__ __forceinline__ void team_pass_any(const PItem& it, const Geo& g, const Team& t, int ns, bool zin, const T* pin, T* pout,
                              const T* rhs, int write, T* E, double& a1, double& a2) {
  if (ns == 2) {
    if (zin) team_pass<T, 2, true>(it, g, t, pin, pout, rhs, write, E, a1, a2);
    else team_pass<T, 2, false>(it, g, t, pin, pout, rhs, write, E, a1, a2);
  } else {
    if (zin) team_pass<T, 1, true>(it, g, t, pin, pout, rhs, write, E, a1, a2);
    else team_pass<T, 1, false>(it, g, t, pin, pout, rhs, write, E, a1, a2);
  }
}

// Sum of the team's partials part[0 .. size) (every workgroup, same order),
// broadcast to all threads.
__device__ __forceinline__ double team_total(const double* part, int size, double* sh, double* bc) {
  const double s = sum_partials(part, (unsigned)size, sh);
  if (flat_tid() == 0) *bc = s;
  __syncthreads();
  const double r = *bc;
  __syncthreads();
  return r;
}

// Sums of a and b over the workgroup, each in the order block_sum takes (the
// same results bit for bit) but with one pair of barriers for both; valid in
// thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh /* >= 32 */) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int t = flat_tid();
  const int lane = t & 63, wid = t >> 6, nw = flat_size() >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[wid] = a;
    sh[16 + wid] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  if (wid == 0) {
    a = lane < nw ? sh[lane] : 0.0;
    b = lane < nw ? sh[16 + lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_down(a, o, 64);
      b += __shfl_down(b, o, 64);
    }
  }
}

// The team's totals of two partial arrays (pa, pb: one entry per team
// workgroup), broadcast to every thread.  A team of at most 64 workgroups
// is summed by wave 0 alone with the shuffle tree team_total's reduction
// applies to the same values (the other waves only add zeros there), so the
// totals equal team_total's bit for bit with one barrier; larger teams take
// team_total.
__device__ __forceinline__ void team_total2(const double* pa, const double* pb, int size, double* sh, double* bc,
                                            double& ta, double& tb) {
  if (size > 64) {
    ta = team_total(pa, size, sh, bc);
    tb = team_total(pb, size, sh, bc);
    return;
  }
  const int t = flat_tid();
  if (t < 64) {
    double a = t < size ? 0.0 + pa[t] : 0.0;
    double b = t < size ? 0.0 + pb[t] : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_down(a, o, 64);
      b += __shfl_down(b, o, 64);
    }
    if (t == 0) {
      bc[0] = a;
      bc[1] = b;
    }
  }
  __syncthreads();
  ta = bc[0];
  tb = bc[1];
}

struct Shared {
  Ctl lc;          // this workgroup's copy of the domain's control block
  double sh[32];
  double bc[2];
  int flag;
};

// T = float: FP32 fields and sweeps inside the FP64 defect correction;
// T = double: the FP64 solve.
template <class T>
__device__ __forceinline__ void persist_body(const PItem* __restrict__ items, const PSlot* __restrict__ slots,
                                             int nsteps, int* err, long long limit, T* E, Shared& S) {
  const PSlot slot{uni(slots[blockIdx.x].item), uni(slots[blockIdx.x].rank)};
  if (slot.item < 0) return;
  const PItem& it = items[slot.item];
  const Geo g = uni_geo(it.g);
  Team t{slot.rank, uni(it.team), 0u, it.bar, err, limit};
  const bool lead = slot.rank == 0 && flat_tid() == 0;
  const long n = (long)g.nx * g.ny * g.nz;
  const int nvb = uni(it.cgx * it.cgy * it.cgz);
  const int itermax = uni(it.itermax);
  const int ns_max = uni(it.ns_max);
  const int adaptive = uni(it.adaptive);
  const bool has_f = uni(it.frc[0] != nullptr);
  for (int q = flat_tid(); q < 2 * 2 * 2 * kEdge<waves_of<T>()>; q += 64 * waves_of<T>()) E[q] = T(0);
  if (flat_tid() == 0) S.lc = *it.ctl;
  int pc = uni(it.st->pcur);
  __syncthreads();
  T* u = (T*)it.u;
  T* v = (T*)it.v;
  T* w = (T*)it.w;
  T* F = (T*)it.F;
  T* G = (T*)it.G;
  T* H = (T*)it.H;
  T* rhs = (T*)it.rhs;
  int* fl = &S.flag;
  const int ts = t.size;
  // Reductions alternate between two halves of the partial-sum array (3
  // slots per team workgroup each), so a workgroup can publish the next
  // reduction's partials while a slower one still reads the previous
  // ones: a reduction needs one barrier, not two.
  int red = 0;
  auto next_part = [&]() -> double* { return it.part + (red++ & 1) * 3 * ts; };
  double sweep_ticks = 0.0;

  for (int step = 0; step < nsteps; step++) {
    // time step (adaptive): maxima over the unknowns, wall speeds included
    if (adaptive) {
      double m3[3] = {0.0, 0.0, 0.0};
      for (int vb = t.rank; vb < nvb; vb += ts) umax_acc<T>(g, kPersistZr, vblock(it, vb), u, v, w, m3);
      double r3[3];
      for (int d = 0; d < 3; d++) r3[d] = block_max(m3[d], S.sh);
      double* part = next_part();
      if (flat_tid() == 0)
        for (int d = 0; d < 3; d++) part[d * ts + t.rank] = r3[d];
      if (!team_sync(t, fl)) return;
      double mm[3];
      for (int d = 0; d < 3; d++) mm[d] = max_partials(part + d * ts, (unsigned)ts, S.sh);
      if (flat_tid() == 0) umax_finish(&S.lc, mm, g, it.re, it.tau, it.wmax[0], it.wmax[1], it.wmax[2]);
      __syncthreads();
    }
    if (!bc_vel_team<T>(it, g, t, u, v, w, fl)) return;
    // predictor
    for (int vb = t.rank; vb < nvb; vb += ts) {
      if (has_f)
        fgh_cells<T, true>(g, kPersistZr, vblock(it, vb), u, v, w, (const T*)it.frc[0], (const T*)it.frc[1],
                           (const T*)it.frc[2], F, G, H, &S.lc, 1.0 / it.re, it.gamma, it.gforce[0], it.gforce[1],
                           it.gforce[2]);
      else
        fgh_cells<T, false>(g, kPersistZr, vblock(it, vb), u, v, w, nullptr, nullptr, nullptr, F, G, H, &S.lc,
                            1.0 / it.re, it.gamma, it.gforce[0], it.gforce[1], it.gforce[2]);
    }
    if (!team_sync(t, fl)) return;
    // right-hand side and its RMS
    {
      double acc = 0.0;
      for (int vb = t.rank; vb < nvb; vb += ts) acc += rhs_acc<T>(g, kPersistZr, vblock(it, vb), F, G, H, rhs, &S.lc, 0);
      const double s = block_sum(acc, S.sh);
      double* part = next_part();
      if (flat_tid() == 0) part[t.rank] = s;
      if (!team_sync(t, fl)) return;
      const double tot = team_total(part, ts, S.sh, S.bc);
      if (flat_tid() == 0) rhs_finish(&S.lc, tot, n, it.tol);
      __syncthreads();
    }
    const long long tsw0 = wall_clock64();
    int sweeps = 0, outer = 0;
    if constexpr (sizeof(T) == 4) {
      // ---- FP32 sweeps on A e = r inside the FP64 defect correction
      float* const e[2] = {(float*)it.e[0], (float*)it.e[1]};
      float* r = (float*)it.r;
      const float* rf = (const float*)it.rhs;
      {
        double acc = 0.0;
        for (int vb = t.rank; vb < nvb; vb += ts)
          acc += defect_acc<false>(g, kPersistZr, vblock(it, vb), it.p[pc], nullptr, nullptr, rf, r);
        const double s = block_sum(acc, S.sh);
        double* part = next_part();
        if (flat_tid() == 0) part[t.rank] = s;
        if (!team_sync(t, fl)) return;
        const double tot = team_total(part, ts, S.sh, S.bc);
        if (flat_tid() == 0) defect_finish(&S.lc, tot, n, it.eta);
        __syncthreads();
      }
      int used = 0;
      while (!uni(S.lc.outer_done) && !uni(S.lc.nonfinite) && used < itermax) {
        outer++;
        const int budget = itermax - used;
        int m = 0, cur = 0, f = 0, fb = 0;
        for (;;) {
          const int ns = ns_max == 2 && m + 2 <= budget ? 2 : 1;
          double a1 = 0.0, a2 = 0.0;
          team_pass_any<float>(it, g, t, ns, m == 0, e[cur], e[cur ^ 1], r, 1, (float*)E, a1, a2);
          block_sum2(a1, a2, S.sh);
          double* part = next_part();
          if (flat_tid() == 0) {
            part[t.rank] = a1;
            part[ts + t.rank] = a2;
          }
          if (!team_sync(t, fl)) return;
          double t1, t2;
          team_total2(part, part + ts, ts, S.sh, S.bc, t1, t2);
          // every thread takes the decision from the same totals; thread 0
          // keeps the control-block copy
          int stop = 0, fin = 0;
          {
            const double thr = S.lc.thr_in;
            auto check = [&](int mm, double tot) {
              const double res = sqrt(tot / (double)n);
              const bool ok = isfinite(res);
              if (flat_tid() == 0) {
                S.lc.res_in = res;
                if (!ok) S.lc.nonfinite = 1;
              }
              if (!(res > thr) || mm >= budget || !ok) {
                stop = 1;
                fin = mm;
              }
            };
            if (m >= 1) check(m, t1);
            if (!stop && ns == 2) check(m + 1, t2);
            if (!stop && m + ns >= budget) {
              stop = 1;
              fin = budget;
            }
          }
          stop = uni(stop);
          fin = uni(fin);
          if (!stop) {
            m += ns;
            cur ^= 1;
            continue;
          }
          f = fin;
          if (fin == m) {
            fb = cur;
          } else if (fin == m + 1 && ns == 2) {
            // the iterate the pass held only in registers: sweep it again
            // from the pass's input into the pass's output buffer
            team_pass_any<float>(it, g, t, 1, m == 0, e[cur], e[cur ^ 1], r, 1, (float*)E, a1, a2);
            if (!team_sync(t, fl)) return;
            fb = cur ^ 1;
          } else {
            fb = cur ^ 1;
          }
          break;
        }
        used += f;
        // p' = p + e, r = rhs - A p', RMS(r)
        double acc = 0.0;
        for (int vb = t.rank; vb < nvb; vb += ts)
          acc += defect_acc<true>(g, kPersistZr, vblock(it, vb), it.p[pc], e[fb], it.p[pc ^ 1], rf, r);
        const double s = block_sum(acc, S.sh);
        double* part = next_part();
        if (flat_tid() == 0) part[t.rank] = s;
        if (!team_sync(t, fl)) return;
        const double tot = team_total(part, ts, S.sh, S.bc);
        if (flat_tid() == 0) defect_finish(&S.lc, tot, n, it.eta);
        __syncthreads();
        pc ^= 1;
      }
      sweeps = used;
    } else {
      // ---- FP64 red-black SOR on A p = rhs
      double* const P[2] = {it.p[0], it.p[1]};
      const double* rd = (const double*)it.rhs;
      int m = 0, cur = pc, f = 0, fb = pc;
      if (!uni(S.lc.done)) {
        for (;;) {
          const int ns = m < itermax ? (ns_max == 2 && m + 2 <= itermax ? 2 : 1) : 0;
          double a1 = 0.0, a2 = 0.0;
          if (ns > 0) team_pass_any<double>(it, g, t, ns, false, P[cur], P[cur ^ 1], rd, 1, (double*)E, a1, a2);
          else team_pass_any<double>(it, g, t, 1, false, P[cur], P[cur ^ 1], rd, 0, (double*)E, a1, a2);
          block_sum2(a1, a2, S.sh);
          double* part = next_part();
          if (flat_tid() == 0) {
            part[t.rank] = a1;
            part[ts + t.rank] = a2;
          }
          if (!team_sync(t, fl)) return;
          double t1, t2;
          team_total2(part, part + ts, ts, S.sh, S.bc, t1, t2);
          int stop = 0, fin = 0;
          {
            const double thr = S.lc.thr;
            auto check = [&](int mm, double tot) {
              const double res = sqrt(tot / (double)n);
              const bool ok = isfinite(res);
              if (flat_tid() == 0) {
                S.lc.res = res;
                if (!ok) S.lc.nonfinite = 1;
              }
              if (!(res > thr) || mm >= itermax || !ok) {
                stop = 1;
                fin = mm;
              }
            };
            if (m >= 1 || itermax == 0) check(m, t1);
            if (!stop && ns == 2) check(m + 1, t2);
          }
          stop = uni(stop);
          fin = uni(fin);
          if (!stop) {
            m += ns;
            cur ^= 1;
            continue;
          }
          f = fin;
          if (fin == m) {
            fb = cur;
          } else {  // fin == m + 1 of a two-sweep pass: held only in registers
            team_pass_any<double>(it, g, t, 1, false, P[cur], P[cur ^ 1], rd, 1, (double*)E, a1, a2);
            if (!team_sync(t, fl)) return;
            fb = cur ^ 1;
          }
          break;
        }
      }
      __syncthreads();  // thread 0's control-block writes of the stop decision
      sweeps = f;
      pc = fb;
    }
    sweep_ticks += (double)(wall_clock64() - tsw0);
    if (uni(S.lc.nonfinite)) {
      if (lead) it.st->nonfinite = 1;
      break;
    }
    // pressure ghosts, projection, boundary fill
    if (!p_ghosts_team(it, g, t, it.p[pc], fl)) return;
    for (int vb = t.rank; vb < nvb; vb += ts) project_cells<T>(g, kPersistZr, vblock(it, vb), F, G, H, it.p[pc], u, v, w, &S.lc, 0);
    if (!team_sync(t, fl)) return;
    if (!bc_vel_team<T>(it, g, t, u, v, w, fl)) return;
    if (lead) {
      PStats& st = *it.st;
      st.t += S.lc.dt;
      st.dt_last = S.lc.dt;
      st.res_last = S.lc.res;
      st.sweeps_total += sweeps;
      st.sweeps_max = max(st.sweeps_max, sweeps);
      st.outer_max = max(st.outer_max, outer);
      if (S.lc.res > S.lc.thr) st.steps_unconverged++;
      st.steps++;
      st.pcur = pc;
    }
  }
  if (lead) {
    *it.ctl = S.lc;
    it.st->pcur = pc;
    it.st->sweep_ticks += sweep_ticks;
  }
}

// One workgroup per compute unit: FP32 16 waves (four per SIMD, 128
// registers), FP64 8 waves (two per SIMD).
__global__ void __launch_bounds__(64 * kPersistWaves32, kPersistWaves32 / 4)
k_persist_f32(const PItem* __restrict__ items, const PSlot* __restrict__ slots, int nsteps, int* err,
              long long limit) {
  __shared__ float E[2 * 2 * 2 * kEdge<kPersistWaves32>];
  __shared__ Shared S;
  persist_body<float>(items, slots, nsteps, err, limit, E, S);
}
__global__ void __launch_bounds__(64 * kPersistWaves64, kPersistWaves64 / 4)
k_persist_f64(const PItem* __restrict__ items, const PSlot* __restrict__ slots, int nsteps, int* err,
              long long limit) {
  __shared__ double E[2 * 2 * 2 * kEdge<kPersistWaves64>];
  __shared__ Shared S;
  persist_body<double>(items, slots, nsteps, err, limit, E, S);
}

template <class T>
int resident_of() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sizeof(T) == 4 ? (const void*)k_persist_f32 : (const void*)k_persist_f64, 64 * waves_of<T>(), 0) != hipSuccess)
    return 0;
  cached = cus * per_cu;
  return cached;
}

}  // namespace

int persistent_resident(bool f32) { return f32 ? resident_of<float>() : resident_of<double>(); }

hipError_t launch_persistent(hipStream_t st, bool f32, const PItem* items, const PSlot* slots, int nblocks,
                             int nsteps, int* err, long long limit) {
  void* args[] = {(void*)&items, (void*)&slots, (void*)&nsteps, (void*)&err, (void*)&limit};
  const dim3 grid(nblocks), blk(64, persist_waves(f32));  // 64 lanes in x, one wave per row group in y
  if (f32) return hipLaunchCooperativeKernel((const void*)k_persist_f32, grid, blk, args, 0, st);
  return hipLaunchCooperativeKernel((const void*)k_persist_f64, grid, blk, args, 0, st);
}

}  // namespace ns
