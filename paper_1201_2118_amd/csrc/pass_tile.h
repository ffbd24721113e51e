// pass_tile.h -- the tile of the NS-sweep red-black SOR pass (temporal
// blocking), shared by the pass kernels and the persistent batched kernel.
//
// Temporal blocking of the red-black iteration: a workgroup reads its tile of
// the input iterate and of the rhs once and carries it through NS complete
// sweeps (red then black, repeated) before writing the last iterate, so a
// pass of two sweeps costs the HBM traffic of one.  Each sweep is exactly
// the sweep of the unfused kernels (the same per-cell update in the same
// colour order); the residual of every input iterate is accumulated on the
// way, so the stop rule is applied after every sweep as before.
//
// Workgroup: 8 waves stacked in y; wave w owns R consecutive rows of the
// tile (rows w R .. w R + R - 1) and each lane one x position, so a lane
// keeps R cells of a plane in registers.  x neighbours come from the
// adjacent lanes through DPP wave shifts, y neighbours inside a wave's rows
// from its own registers, and across waves from one LDS row per wave edge.
// The tile is marched through z; with plane L the newest loaded, one step
// computes
//   A: residual of the input and red update at plane L - 1,
//   B: black update at plane L - 2 (first sweep's iterate),
// and for NS = 2 additionally
//   C: residual of that iterate and its red update at plane L - 3,
//   D: black update at plane L - 4 (second sweep's iterate),
// then writes the last stage's plane.  Each stage consumes its own plane
// and the planes on either side from registers; a value that crosses a
// wave edge goes through LDS with one barrier per step.  The halo is
// 2 NS cells in x, y and z and is recomputed redundantly, so no workgroup
// reads what another writes; input and output are different buffers.
//
// The residual r = sum_nb a_nb p_nb - a_c p_c - rhs is evaluated with an
// explicit fused multiply-add chain (one rounding sequence for every
// instantiation), and a cell's update is p + (omega / a_c) r.  Across a
// wall the coefficient is zero and positions outside the domain load a
// clamped cell (finite); periodic axes load the periodic image.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "ns_internal.h"

namespace ns {

namespace {

constexpr int kLanes = 64;  // x positions per row (one wave)
// Rows per lane of the 24- and 32-row tiles (the 16-row tile has 2 rows on
// 8 waves); waves = rows / rows per lane.
constexpr int kR24 = 2, kR32 = 2;  // 3 rows on 8 waves and 4 rows on 8 waves ran slower at 512^3
// Planes per register ring (input and rhs) = steps per unrolled trip: a
// plane is loaded ring - 2 steps before the step that first reads it.  Six
// planes (loads four steps ahead) for the single-domain kernel's FP64 tiles
// and 12- and 16-wave FP32 tiles and for the batched kernel's 12-wave FP32
// tiles; four for the rest (8-wave FP32 tiles would drop from two
// workgroups per CU to one, the other batched tiles would spill).  FP32 tiles of 16
// waves need 5 more registers than the 128 of their occupancy: the compiler
// keeps 5 values in scratch, and the tile still runs 5 % faster than with
// loads two steps ahead (the loads' latency is the larger cost).  Eight
// planes measured: FP64 2 % faster but spilling, FP32 16-wave tiles much
// slower (24 values in scratch).
template <class T, int R, int W, bool BATCH>
constexpr int ring_of() {
  if constexpr (R != 2) return 4;
  if constexpr (BATCH) return sizeof(T) == 4 && W == 12 ? 6 : 4;
  return sizeof(T) == 8 || W >= 12 ? 6 : 4;
}

__device__ __forceinline__ int dpp_left(int v) {  // lane l receives lane l - 1 (0 at lane 0)
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_right(int v) {  // lane l receives lane l + 1 (0 at lane 63)
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, dpp_left(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, dpp_right(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)dpp_left((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_left((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, (long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double from_right(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)dpp_right((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_right((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, (long long)(((unsigned long long)hi << 32) | lo));
}

// Index of the cell a virtual position loads: the periodic image (one wrap;
// the axis is at least as long as the halo), clamped to the domain.
__device__ __forceinline__ int wrap_clamp(int i, int n, int per) {
  if (per) i += (i < 1 ? n : 0) - (i > n ? n : 0);
  return i < 1 ? 1 : (i > n ? n : i);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// sum_nb a_nb p_nb - diag p_c, one rounding sequence; the x neighbours
// are lane l - 1's and lane l + 1's pc.
template <class T>
__device__ __forceinline__ T stencil_chain(T t, T ps, T pn, T pd, T pu, T pc, T aym, T ayp, T azm, T azp,
                                           T diag) {
  t = fmaT(aym, ps, t);
  t = fmaT(ayp, pn, t);
  t = fmaT(azm, pd, t);
  t = fmaT(azp, pu, t);
  return fmaT(-diag, pc, t);
}
__device__ __forceinline__ double stencil(double pc, double ps, double pn, double pd, double pu, double axm,
                                          double axp, double aym, double ayp, double azm, double azp,
                                          double diag) {
  double t = from_left(pc) * axm;
  t = fmaT(from_right(pc), axp, t);
  return stencil_chain(t, ps, pn, pd, pu, pc, aym, ayp, azm, azp, diag);
}
// FP32: t + (lane l + 1's v) c in one DPP-sourced v_fmac (the compiler
// folds a shifted operand into a multiply but not into an fmac).  The
// s_nop covers the two wait states a DPP read needs after a VALU write of
// its source.
__device__ __forceinline__ float fma_from_right(float v, float c, float t) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(t)
      : "v"(v), "v"(c));
  return t;
}
__device__ __forceinline__ float stencil(float pc, float ps, float pn, float pd, float pu, float axm, float axp,
                                         float aym, float ayp, float azm, float azp, float diag) {
  float t = from_left(pc) * axm;
  t = fma_from_right(pc, axp, t);
  return stencil_chain(t, ps, pn, pd, pu, pc, aym, ayp, azm, azp, diag);
}

// acc + r^2 in FP64 (r^2 is exact).  A cell that does not count passes
// r = 0 (r times a 0 / 1 ownership factor), which leaves acc unchanged.
__device__ __forceinline__ double add_sq(float r, double acc) {
  const double d = r;
  return __builtin_fma(d, d, acc);
}
__device__ __forceinline__ double add_sq(double r, double acc) { return __builtin_fma(r, r, acc); }

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One z plane of a field: a global pointer made opaque to the optimiser,
// which keeps it from folding the per-lane offset into a hoisted 64-bit
// per-lane address (loads then take the scalar base + 32-bit offset form).
#define NS_GLOBAL __attribute__((address_space(1)))
struct Plane {
  NS_GLOBAL char* b;
};
template <class T>
__device__ __forceinline__ Plane plane_at(const T* p, long elems, long) {
  NS_GLOBAL char* q = (NS_GLOBAL char*)(p + elems);
  asm volatile("" : "+s"(q));
  return Plane{q};
}
// The offset is made opaque in place at each use as well, so its widening
// to 64 bits stays next to the access (a 64-bit offset hoisted out of the
// loop would cost one 64-bit address add per access; an opaque copy would
// cost a move).
template <class T>
__device__ __forceinline__ T ld_plane(const Plane& b, unsigned& off, T*) {
  asm volatile("" : "+v"(off));
  return *(const NS_GLOBAL T*)(b.b + off);
}
template <class T>
__device__ __forceinline__ void st_plane(const Plane& b, unsigned& off, T v) {
  asm volatile("" : "+v"(off));
  *(NS_GLOBAL T*)(b.b + off) = v;
}

// LDS edge rows: per quantity and step parity, two rows (top, bottom) per
// wave, between a padding row before the first wave's and one after the
// last wave's (zero, never written: the rows beyond the workgroup's ends,
// whose values only reach halo rows), so every wave finds the rows above
// and below its own at fixed offsets from one address.
template <int W>
constexpr int kEdge = (W * 2 + 2) * kLanes;

template <class T, int NS, int R, int W, bool ZIN, bool BATCH>
__device__ __forceinline__ void pass_tile(const T* __restrict__ p_in, T* __restrict__ p_out,
                                          const T* __restrict__ rhs, const Geo& g, double omega, int write,
                                          int col, int z0, int z1, int ntx, T* __restrict__ E, double& acc1,
                                          double& acc2) {
  constexpr int H = 2 * NS;
  constexpr int TX = kLanes - 2 * H;
  constexpr int ROWS = R * W;
  constexpr int kRing = ring_of<T, R, W, BATCH>();
  constexpr int TY = ROWS - 2 * H;
  const int tx = threadIdx.x;
  const int wy = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  const int bx = col % ntx;
  const int by = col / ntx;
  const int i = bx * TX + tx - (H - 1);
  const int j0 = by * TY + wy * R - (H - 1);  // row 0 of this wave (uniform)
  const int per0 = g.per[0], per1 = g.per[1], per2 = g.per[2];

  const bool ownx = tx >= H && tx < kLanes - H && i <= g.nx;
  const bool xlo = i > 1 || per0, xhi = i < g.nx || per0;
  const T axm = xlo ? T(g.idx2) : T(0);
  const T axp = xhi ? T(g.idx2) : T(0);
  const int iw = wrap_clamp(i, g.nx, per0);
  const T idy2 = T(g.idy2), idz2 = T(g.idz2);
  auto aym = [&](int j) -> T { return (j > 1 || per1) ? idy2 : T(0); };
  auto ayp = [&](int j) -> T { return (j < g.ny || per1) ? idy2 : T(0); };
  auto owny = [&](int r) -> bool { return wy * R + r >= H && wy * R + r < ROWS - H && j0 + r <= g.ny; };
  // 1 where row r's cell of this lane is one the tile owns (its residual
  // counts), 0 on the halo
  T ownf[R];
#pragma unroll
  for (int r = 0; r < R; r++) ownf[r] = owny(r) && ownx ? T(1) : T(0);
  // FP32 applies the same ownership as a lane mask per row held in scalar
  // registers, with one v_cndmask (no vector register for the factor; the
  // compiler would split the compound condition into several selects)
  unsigned long long ownm[R];
#pragma unroll
  for (int r = 0; r < R; r++) ownm[r] = owny(r) ? __builtin_amdgcn_ballot_w64(ownx) : 0ull;
  // the residual of row r's cell where it counts (and the plane lies in the
  // chunk), 0 elsewhere
  auto counted = [&](T res, int r, bool chunk) -> T {
    if constexpr (sizeof(T) == 4) {
      float out;
      asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(out) : "v"(res), "s"(chunk ? ownm[r] : 0ull));
      return out;
    } else {
      return res * (chunk ? ownf[r] : T(0));
    }
  };
  // diagonal a_c and relaxation factor omega / a_c of row r's cell with both
  // z neighbours (d2, w2) or one (d1, w1, planes next to a z wall)
  auto dxy_of = [&](int j) -> double {
    return ((xlo ? g.idx2 : 0.0) + (xhi ? g.idx2 : 0.0)) +
           (((j > 1 || per1) ? g.idy2 : 0.0) + ((j < g.ny || per1) ? g.idy2 : 0.0));
  };
  const int Lbeg = z0 + 2 - 2 * NS;  // first step: the ring holds planes Lbeg - 2 .. Lbeg + 1
  const int Lend = z1 + 2 * NS;      // last step: the last stage reaches z1
  T d1[R], d2[R], w1[R], wA[R], wB[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const double dd = dxy_of(j0 + r) + (g.idz2 + g.idz2);
    d2[r] = T(dd);
    const double d1d = dxy_of(j0 + r) + g.idz2;
    d1[r] = T(d1d);
    w1[r] = T(omega / d1d);
    // The colour is folded into the relaxation factor: wA is omega / a_c
    // where the cell is red on planes of Lbeg's parity (0 elsewhere), wB
    // where it is red on the other planes.  A red stage on a plane of
    // Lbeg's parity and a black stage on the other parity use wA; a cell
    // with weight 0 keeps its value exactly.
    const bool redA = ((i + j0 + r + Lbeg) & 1) == 0;
    const T w2 = T(omega / dd);
    wA[r] = redA ? w2 : T(0);
    wB[r] = redA ? T(0) : w2;
  }
  // FAST: every plane of the step has both z neighbours.  wsel is the
  // step's weight (wA or wB); planes next to a z wall swap in omega / a_c
  // of the cell with one z neighbour.
  auto coef = [&](auto FASTc, int r, int k, T wsel, T& d, T& w) {
    if constexpr (decltype(FASTc)::value) {
      d = d2[r];
      w = wsel;
    } else {
      const bool both = (k > 1 || per2) && (k < g.nz || per2);
      d = both ? d2[r] : d1[r];
      w = both ? wsel : (wsel != T(0) ? w1[r] : T(0));
    }
  };

  unsigned off[R];  // byte offset of the loaded cell in its plane
#pragma unroll
  for (int r = 0; r < R; r++)
    off[r] = (unsigned)((long)wrap_clamp(j0 + r, g.ny, per1) * g.sx + iw) * (unsigned)sizeof(T);

  // LDS: this wave's top / bottom rows, and the rows above / below it (the
  // padding rows at the workgroup's ends)
  const int e_top = (wy * 2 + 1) * kLanes + tx;
  const int e_bot = e_top + kLanes;
  const int e_above = e_top - kLanes;
  const int e_below = e_bot + kLanes;
  auto ebuf = [&](int q, int par) -> T* { return E + (q * 2 + par) * kEdge<W>; };

  auto plane_of = [&](int k) -> long {
    int kw = k;
    if (per2) kw += (kw < 1 ? g.nz : 0) - (kw > g.nz ? g.nz : 0);
    kw = kw < 1 ? 1 : (kw > g.nz ? g.nz : kw);
    return (long)kw * g.sxy;
  };


  // rings: slot (S + q) % kRing holds plane L - 2 + q at a step with
  // (L - Lbeg) % kRing == S; planes L .. L + kRing - 3 may still be in flight
  T P[kRing][R], Q[kRing][R];
  T hC[R], hD[R];                       // rhs at L - 3, L - 4
  T X1a[R], X1b[R], Ma[R], Mb[R];       // first sweep: red at L-3, L-2; iterate at L-4, L-3
  T X2a[R], X2b[R];                     // second sweep: red at L-5, L-4
#pragma unroll
  for (int q = 0; q < kRing; q++) {
    const long pl = plane_of(Lbeg - 2 + q);
    const Plane bp = plane_at(p_in, pl, g.sxy);
    const Plane br = plane_at(rhs, pl, g.sxy);
#pragma unroll
    for (int r = 0; r < R; r++) {
      P[q][r] = ZIN ? T(0) : ld_plane(bp, off[r], (T*)nullptr);
      Q[q][r] = ld_plane(br, off[r], (T*)nullptr);
    }
  }
#pragma unroll
  for (int r = 0; r < R; r++) {
    hC[r] = hD[r] = X1a[r] = X1b[r] = Ma[r] = Mb[r] = X2a[r] = X2b[r] = T(0);
  }

  auto zcoef = [&](auto FASTc, int k, T& azm, T& azp) {
    if constexpr (decltype(FASTc)::value) {
      azm = azp = idz2;
    } else {
      azm = (k > 1 || per2) ? idz2 : T(0);
      azp = (k < g.nz || per2) ? idz2 : T(0);
    }
  };

  auto step = [&](auto Sc, auto Fc, auto Ic, int L) {
    constexpr int S = decltype(Sc)::value;
    constexpr bool IN = decltype(Ic)::value;  // every stage plane of the step lies in the chunk
    constexpr int SP = S & 1;
    T(&pm2)[R] = P[S];
    T(&pm1)[R] = P[(S + 1) % kRing];
    T(&p0)[R] = P[(S + 2) % kRing];
    T(&qm2)[R] = Q[S];
    T(&qm1)[R] = Q[(S + 1) % kRing];

    // the input plane's edge rows
    ebuf(0, SP)[e_top] = pm1[0];
    ebuf(0, SP)[e_bot] = pm1[R - 1];
    lds_barrier();
    // FP32 tiles issue the plane's arithmetic at raised wave priority and drop
    // it before the next plane's loads (measured 1 % faster single-domain and
    // 2 % batched; FP64 tiles, two waves per SIMD, measured 1.5 % slower)
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(1);
    const T inA = ebuf(0, SP)[e_above], inB = ebuf(0, SP)[e_below];
    const T x1A = ebuf(1, SP ^ 1)[e_above], x1B = ebuf(1, SP ^ 1)[e_below];

    // A: residual of the input and red update at plane a = L - 1
    T X1n[R];
    {
      const int a = L - 1;
      T azm, azp;
      zcoef(Fc, a, azm, azp);
      const bool in_chunk = a >= z0 && a <= z1;
#pragma unroll
      for (int r = 0; r < R; r++) {
        const T pc = pm1[r];
        const T ps = r > 0 ? pm1[r - 1] : inA;
        const T pn = r < R - 1 ? pm1[r + 1] : inB;
        T dg, wg;
        coef(Fc, r, a, (S & 1) ? wA[r] : wB[r], dg, wg);
        const T res = stencil(pc, ps, pn, pm2[r], p0[r], axm, axp, aym(j0 + r),
                              ayp(j0 + r), azm, azp, dg) -
                      qm1[r];
        acc1 = add_sq(counted(res, r, IN || in_chunk), acc1);
        X1n[r] = fmaT(wg, res, pc);
      }
    }
    // B: black update at plane b = L - 2 (the first sweep's iterate)
    T Mn[R];
    {
      const int b = L - 2;
      T azm, azp;
      zcoef(Fc, b, azm, azp);
#pragma unroll
      for (int r = 0; r < R; r++) {
        const T pc = X1b[r];
        const T ps = r > 0 ? X1b[r - 1] : x1A;
        const T pn = r < R - 1 ? X1b[r + 1] : x1B;
        T dg, wg;
        coef(Fc, r, b, (S & 1) ? wA[r] : wB[r], dg, wg);
        const T res = stencil(pc, ps, pn, X1a[r], X1n[r], axm, axp, aym(j0 + r),
                              ayp(j0 + r), azm, azp, dg) -
                      qm2[r];
        Mn[r] = fmaT(wg, res, pc);
      }
      if constexpr (NS == 1) {
        if (write && b >= z0 && b <= z1) {
          const Plane bo = plane_at(p_out, (long)b * g.sxy, g.sxy);
#pragma unroll
          for (int r = 0; r < R; r++)
            if (owny(r) && ownx) st_plane(bo, off[r], Mn[r]);
        }
      }
    }
    if constexpr (NS == 2) {
      const T mA = ebuf(2, SP ^ 1)[e_above], mB = ebuf(2, SP ^ 1)[e_below];
      const T x2A = ebuf(3, SP ^ 1)[e_above], x2B = ebuf(3, SP ^ 1)[e_below];
        // C: residual of the first sweep's iterate and red update at c = L - 3
      T X2n[R];
      {
        const int c = L - 3;
        T azm, azp;
        zcoef(Fc, c, azm, azp);
        const bool in_chunk = c >= z0 && c <= z1;
#pragma unroll
        for (int r = 0; r < R; r++) {
          const T pc = Mb[r];
          const T ps = r > 0 ? Mb[r - 1] : mA;
          const T pn = r < R - 1 ? Mb[r + 1] : mB;
          T dg, wg;
          coef(Fc, r, c, (S & 1) ? wA[r] : wB[r], dg, wg);
          const T res = stencil(pc, ps, pn, Ma[r], Mn[r], axm, axp, aym(j0 + r),
                                ayp(j0 + r), azm, azp, dg) -
                        hC[r];
          acc2 = add_sq(counted(res, r, IN || in_chunk), acc2);
          X2n[r] = fmaT(wg, res, pc);
        }
      }
        // D: black update at d = L - 4, written out
      {
        const int d = L - 4;
        T azm, azp;
        zcoef(Fc, d, azm, azp);
        T out[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
          const T pc = X2b[r];
          const T ps = r > 0 ? X2b[r - 1] : x2A;
          const T pn = r < R - 1 ? X2b[r + 1] : x2B;
          T dg, wg;
          coef(Fc, r, d, (S & 1) ? wA[r] : wB[r], dg, wg);
          const T res = stencil(pc, ps, pn, X2a[r], X2n[r], axm, axp, aym(j0 + r),
                                ayp(j0 + r), azm, azp, dg) -
                        hD[r];
          out[r] = fmaT(wg, res, pc);
        }
        if (write && d >= z0 && d <= z1) {
          const Plane bo = plane_at(p_out, (long)d * g.sxy, g.sxy);
#pragma unroll
          for (int r = 0; r < R; r++)
            if (owny(r) && ownx) st_plane(bo, off[r], out[r]);
        }
      }
      ebuf(2, SP)[e_top] = Mn[0];
      ebuf(2, SP)[e_bot] = Mn[R - 1];
      ebuf(3, SP)[e_top] = X2n[0];
      ebuf(3, SP)[e_bot] = X2n[R - 1];
#pragma unroll
      for (int r = 0; r < R; r++) {
        Ma[r] = Mb[r];
        Mb[r] = Mn[r];
        X2a[r] = X2b[r];
        X2b[r] = X2n[r];
        hD[r] = hC[r];
        hC[r] = qm2[r];
      }
    }
    ebuf(1, SP)[e_top] = X1n[0];
    ebuf(1, SP)[e_bot] = X1n[R - 1];
#pragma unroll
    for (int r = 0; r < R; r++) {
      X1a[r] = X1b[r];
      X1b[r] = X1n[r];
    }
    // refill the dead ring slots with plane L + kRing - 2
    const long pl = plane_of(L + kRing - 2);
    const Plane bp = plane_at(p_in, pl, g.sxy);
    const Plane br = plane_at(rhs, pl, g.sxy);
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int r = 0; r < R; r++) {
      pm2[r] = ZIN ? T(0) : ld_plane(bp, off[r], (T*)nullptr);
      qm2[r] = ld_plane(br, off[r], (T*)nullptr);
    }
  };

  // Trips of kRing steps.  A trip whose stage planes all lie strictly
  // inside the domain in z (every trip on a periodic axis) and that ends by
  // Lend takes the constant z coefficients; the last trip stops after Lend.
  const int fast_lo = per2 ? INT_MIN : 2 * NS + 2;  // first step with all stage planes >= 2
  const int fast_hi = min(per2 ? INT_MAX : g.nz, Lend);  // last such step <= nz - 1, within the chunk
  using F0 = std::integral_constant<int, 0>;
  using F1 = std::integral_constant<int, 1>;
  using F2 = std::integral_constant<int, 2>;
  using F3 = std::integral_constant<int, 3>;
  using F4 = std::integral_constant<int, 4>;
  using F5 = std::integral_constant<int, 5>;
  using FAST = std::true_type;
  using GEN = std::false_type;
  // steps whose residual planes (L - 1, and L - 3 for two sweeps) all lie
  // in [z0, z1] need no chunk test
  const int in_lo = z0 + 2 * NS - 1, in_hi = z1 + 1;
  using IN = std::true_type;
  using MASK = std::false_type;
  auto trip = [&](auto Fc, auto Ic, int L) {
    step(F0{}, Fc, Ic, L);
    step(F1{}, Fc, Ic, L + 1);
    step(F2{}, Fc, Ic, L + 2);
    step(F3{}, Fc, Ic, L + 3);
    if constexpr (kRing > 4) {
      step(F4{}, Fc, Ic, L + 4);
      step(F5{}, Fc, Ic, L + 5);
    }
  };
  for (int L = Lbeg; L <= Lend; L += kRing) {
    if (L >= fast_lo && L + kRing - 1 <= fast_hi) {
      if (L >= in_lo && L + kRing - 1 <= in_hi)
        trip(FAST{}, IN{}, L);
      else
        trip(FAST{}, MASK{}, L);
    } else {
      step(F0{}, GEN{}, MASK{}, L);
      if (L + 1 > Lend) break;
      step(F1{}, GEN{}, MASK{}, L + 1);
      if (L + 2 > Lend) break;
      step(F2{}, GEN{}, MASK{}, L + 2);
      if (L + 3 > Lend) break;
      step(F3{}, GEN{}, MASK{}, L + 3);
      if constexpr (kRing > 4) {
        if (L + 4 > Lend) break;
        step(F4{}, GEN{}, MASK{}, L + 4);
        if (L + 5 > Lend) break;
        step(F5{}, GEN{}, MASK{}, L + 5);
      }
    }
  }
}


}  // namespace

}  // namespace ns
