// sor_fused.hip -- one red-black SOR sweep in one pass over HBM.
//
// A workgroup owns a column of TX x TY interior cells (TX = 60) and marches
// it through a chunk of z planes.  Its 64 x (TY + 4) threads cover the
// column plus a 2-cell halo in x and y (one x row per wave64, so every load
// is a contiguous 512-byte row in FP64).  Each thread keeps the planes of
// its own (x, y) position in registers and exchanges x / y neighbours
// through two double-buffered LDS planes, with one workgroup barrier per z
// plane.  With plane L the newest loaded:
//   - residual of the input iterate at plane L-1 (tile cells),
//   - red update at plane L-1 (tile + 1-cell halo; needs input at L-2..L),
//   - black update at plane L-2 (tile; needs the new red values at L-3..L-1),
//   - the tile row of plane L-2 is written out.
// The halo is recomputed redundantly, so no workgroup reads a value another
// workgroup writes in the same sweep; input and output are different
// buffers.  The arithmetic per cell is that of the unfused sweep: the
// residual r = sum_nb a_nb (p_nb - p) - rhs and p + (omega / a_c) r.
// Positions outside the domain load a clamped (wall) or wrapped (periodic)
// cell, so every load is in bounds and finite; across a wall the
// coefficient is zero.
#include <hip/hip_runtime.h>

#include "ns_internal.h"
#include "reduce.h"

namespace ns {

namespace {

constexpr int kW = 64;   // threads per row (x), one wave
constexpr int kTX = 60;  // interior cells per row

// Cell index that a virtual position loads: one periodic image on each
// side, clamped beyond (positions that far out are never used).
__device__ __forceinline__ int wrapc(int i, int n, int per) {
  if (i < 1) return (per && i + n >= 1) ? i + n : 1;
  if (i > n) return (per && i - n <= n) ? i - n : n;
  return i;
}

// Load / store at a uniform base plus a 32-bit per-lane byte offset (the
// scalar-base addressing form: no 64-bit address per lane).
template <class T>
__device__ __forceinline__ T ld_off(const T* base, unsigned off) {
  return *(const T*)((const char*)base + off);
}
template <class T>
__device__ __forceinline__ void st_off(T* base, unsigned off, T v) {
  *(T*)((char*)base + off) = v;
}

// Barrier that orders LDS only: global loads issued before it stay in
// flight (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Compute type: FP64 for FP64 storage; FP32 storage sweeps in FP32 (the
// correction equation of the mixed form), with FP64 residual sums either way.
template <class T> struct Acc { using type = double; };
template <> struct Acc<float> { using type = float; };

// One tile of one sweep: the 60 x TY column (bx, by) through the z chunk bz,
// red and black updates written to p_out, the residual of p_in accumulated
// into acc (own cells only).  Used by the single-domain and the batched
// kernels.
template <class T, int TYH, bool ZIN>
__device__ __forceinline__ void sweep_tile(const T* __restrict__ p_in, T* __restrict__ p_out,
                                           const T* __restrict__ rhs, const Geo& g, double omega, int write,
                                           int tile, int zc, int ntx, int nty, T (&sp)[2][TYH * kW],
                                           T (&sr)[2][TYH * kW], double& acc) {
  using A = typename Acc<T>::type;
  constexpr int TY = TYH - 4;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int lid = ty * kW + tx;
  const int per0 = g.per[0], per1 = g.per[1], per2 = g.per[2];
  const bool halo1 = tx >= 1 && tx <= kTX + 2 && ty >= 1 && ty <= TY + 2;
  const A idz2 = (A)g.idz2;
  const int bx = tile % ntx;
  const int rest = tile / ntx;
  const int by = rest % nty;
  const int bz = rest / nty;
  const int i = bx * kTX + tx - 1;  // virtual global x index (1-based interior)
  const int j = by * TY + ty - 1;
  const int z0 = 1 + bz * zc;
  const int z1 = min(g.nz, z0 + zc - 1);
  const long col = (long)wrapc(j, g.ny, per1) * g.sx + wrapc(i, g.nx, per0);
  const unsigned colb = (unsigned)col * (unsigned)sizeof(T);  // < one plane in bytes
  const bool own = tx >= 2 && tx <= kTX + 1 && ty >= 2 && ty <= TY + 1 && i <= g.nx && j <= g.ny;

  // boundary-eliminated coefficients in x and y (fixed per thread)
  const A axm = (i > 1 || per0) ? (A)g.idx2 : A(0);
  const A axp = (i < g.nx || per0) ? (A)g.idx2 : A(0);
  const A aym = (j > 1 || per1) ? (A)g.idy2 : A(0);
  const A ayp = (j < g.ny || per1) ? (A)g.idy2 : A(0);
  const double axy = ((double)axm + (double)axp) + ((double)aym + (double)ayp);
  // omega / a_c for the first, interior and last plane
  const double az_lo = per2 ? 2.0 * g.idz2 : g.idz2;
  const A w_lo = (A)(omega / (axy + az_lo));
  const A w_mid = (A)(omega / (axy + 2.0 * g.idz2));
  const int cpar = (i + j) & 1;
  bool red_first = false;  // steady state: this thread's cell at plane L-1 is red

  // Loads are unconditional and their plane index is computed without
  // branches, so no control flow separates a load from its use (the
  // wait-count insertion would otherwise drain every load at the joins).
  auto plane = [&](int k) -> long {
    int kw = k + (per2 ? g.nz * ((k < 1) - (k > g.nz)) : 0);
    kw = kw < 1 ? 1 : (kw > g.nz ? g.nz : kw);
    return (long)kw * g.sxy + col;
  };
  auto ldp = [&](int k) -> A { return ZIN ? A(0) : (A)p_in[plane(k)]; };
  auto ldr = [&](int k) -> A { return (A)rhs[plane(k)]; };

  // Register rings of 4 planes for the input and the rhs: at plane L the
  // slots hold L-2, L-1, L, L+1 (the last two possibly still in flight);
  // after the plane, the dead L-2 slot receives plane L+2.  Bodies are
  // called with the slots rotated, four per loop trip, so a loaded register
  // is never moved (a move would wait for its load).
  A P0 = ldp(z0 - 2), P1 = ldp(z0 - 1), P2 = ldp(z0), P3 = ldp(z0 + 1);
  A R0 = A(0), R1 = ldr(z0 - 1), R2 = ldr(z0), R3 = ldr(z0 + 1);
  A rnA = A(0), rnB = A(0);  // new red values at L-3, L-2

  // Generic plane: boundary coefficients, chunk limits and wrapped loads
  // evaluated per plane.
  auto body = [&](int L, A& pm2, A& pm1, A& p0, A& rh2, A& rh1) {
    sp[(L - 1) & 1][lid] = (T)pm1;
    lds_barrier();

    // residual of the input and red update at plane k1 = L - 1.  A plane with
    // both z neighbours takes the z term in the steady-state planes' form, so
    // a cell's value does not depend on which of the two paths (and thus on
    // which z chunking) computed it; at a z wall the missing term is dropped.
    const int k1 = L - 1;
    const bool zin1 = (k1 > 1 && k1 < g.nz) || per2;  // uniform over the workgroup
    const A azm1 = k1 > 1 ? idz2 : A(0);
    const A azp1 = k1 < g.nz ? idz2 : A(0);
    const A two = A(2);
    A rnew = pm1;
    if (halo1) {
      const T* P = sp[(L - 1) & 1];
      const A pc = pm1;
      A s;
      if (zin1)
        s = axm * ((A)P[lid - 1] - pc) + axp * ((A)P[lid + 1] - pc) +
            aym * ((A)P[lid - kW] - pc) + ayp * ((A)P[lid + kW] - pc) +
            idz2 * (pm2 + p0 - two * pc);
      else
        s = axm * ((A)P[lid - 1] - pc) + axp * ((A)P[lid + 1] - pc) +
            aym * ((A)P[lid - kW] - pc) + ayp * ((A)P[lid + kW] - pc) +
            azm1 * (pm2 - pc) + azp1 * (p0 - pc);
      const A r = s - rh1;
      if (own && k1 >= z0 && k1 <= z1) acc += (double)r * (double)r;
      if (!((cpar + k1) & 1)) {
        const A wk = (k1 > 1 && k1 < g.nz) ? w_mid : w_lo;
        rnew = (A)(T)(pc + wk * r);  // stored precision, as the LDS copy
      }
    }
    sr[(L - 1) & 1][lid] = (T)rnew;

    // black update and output at plane k2 = L - 2
    const int k2 = L - 2;
    if (own && k2 >= z0 && k2 <= z1) {
      A out;
      if ((cpar + k2) & 1) {
        const T* R = sr[(L - 2) & 1];
        const A pc = pm2;
        const bool zin2 = (k2 > 1 && k2 < g.nz) || per2;
        const A azm2 = k2 > 1 ? idz2 : A(0);
        const A azp2 = k2 < g.nz ? idz2 : A(0);
        A s;
        if (zin2)
          s = axm * ((A)R[lid - 1] - pc) + axp * ((A)R[lid + 1] - pc) +
              aym * ((A)R[lid - kW] - pc) + ayp * ((A)R[lid + kW] - pc) +
              idz2 * (rnA + rnew - two * pc);
        else
          s = axm * ((A)R[lid - 1] - pc) + axp * ((A)R[lid + 1] - pc) +
              aym * ((A)R[lid - kW] - pc) + ayp * ((A)R[lid + kW] - pc) +
              azm2 * (rnA - pc) + azp2 * (rnew - pc);
        const A r = s - rh2;
        const A wk = (k2 > 1 && k2 < g.nz) ? w_mid : w_lo;
        out = pc + wk * r;
      } else {
        out = rnB;
      }
      if (write) p_out[(long)k2 * g.sxy + col] = (T)out;
    }
    rnA = rnB;
    rnB = rnew;
    // refill the dead slots with plane L + 2
    pm2 = ldp(L + 2);
    rh2 = ldr(L + 2);
  };
  // Up to four generic planes from L (a multiple of 4 past z0), stopping
  // after plane `last`; returns the next plane.
  auto gen_block = [&](int L, int last) -> int {
    body(L, P0, P1, P2, R0, R1);
    if (L + 1 > last) return L + 1;
    body(L + 1, P1, P2, P3, R1, R2);
    if (L + 2 > last) return L + 2;
    body(L + 2, P2, P3, P0, R2, R3);
    if (L + 3 > last) return L + 3;
    body(L + 3, P3, P0, P1, R3, R0);
    return L + 4;
  };

  // Steady-state plane: both planes it touches are interior planes of the
  // chunk and of the domain and its loads need no wrap, so the z
  // coefficients are idz2, the relaxation factor is w_mid, and the load
  // and store addresses advance by one plane per call from scalar bases.
  // The LDS buffer of each call position is fixed for the loop.
  const int parity = (z0 - 1) & 1;
  T* const spA = sp[parity];
  T* const spB = sp[parity ^ 1];
  T* const srA = sr[parity];
  T* const srB = sr[parity ^ 1];
  const T* qp = nullptr;   // p_in at plane L + 2
  const T* qr = nullptr;   // rhs at plane L + 2
  T* qo = nullptr;         // p_out at plane L - 2
  const A two = A(2);
  auto fast = [&](T* spw, T* srw, T* srr, A& pm2, A& pm1, A& p0, A& rh2, A& rh1) {
    spw[lid] = (T)pm1;
    lds_barrier();
    A rnew = pm1;
    if (halo1) {
      const A pc = pm1;
      const A s = axm * ((A)spw[lid - 1] - pc) + axp * ((A)spw[lid + 1] - pc) +
                  aym * ((A)spw[lid - kW] - pc) + ayp * ((A)spw[lid + kW] - pc) +
                  idz2 * (pm2 + p0 - two * pc);
      const A r = s - rh1;
      if (own) acc += (double)r * (double)r;
      if (red_first) rnew = (A)(T)(pc + w_mid * r);
    }
    srw[lid] = (T)rnew;
    // the cell below a red cell is black: when this thread's cell at L-1
    // is red, its cell at L-2 takes the black update; otherwise the cell
    // at L-2 is red and was updated one plane ago
    if (own) {
      A out = rnB;
      if (red_first) {
        const A pc = pm2;
        const A s = axm * ((A)srr[lid - 1] - pc) + axp * ((A)srr[lid + 1] - pc) +
                    aym * ((A)srr[lid - kW] - pc) + ayp * ((A)srr[lid + kW] - pc) +
                    idz2 * (rnA + rnew - two * pc);
        out = pc + w_mid * (s - rh2);
      }
      if (write) st_off(qo, colb, (T)out);
    }
    rnA = rnB;
    rnB = rnew;
    // after a plane the colour of this thread's cell flips
    red_first = !red_first;
    pm2 = ZIN ? A(0) : (A)ld_off(qp, colb);
    rh2 = (A)ld_off(qr, colb);
    qp += g.sxy;
    qr += g.sxy;
    qo += g.sxy;
  };

  const int Lf0 = max(z0 + 2, per2 ? z0 + 2 : 4);
  const int Lf1 = min(z1 + 1, g.nz - 2);
  const int Lend = z1 + 2;
  int L = z0;
  while (L <= Lend && L < Lf0) L = gen_block(L, Lend);
  if (L <= Lend && L + 3 <= Lf1) {
    qp = p_in + (long)(L + 2) * g.sxy;
    qr = rhs + (long)(L + 2) * g.sxy;
    qo = p_out + (long)(L - 2) * g.sxy;
    // colour of this thread's cell at plane L - 1 (red = even)
    red_first = !((cpar + L - 1) & 1);
    // Drain once here so that the loop header inherits no unknown pending
    // loads from the generic planes (the wait-count pass would otherwise
    // drain at every trip).
    __builtin_amdgcn_s_waitcnt(0);
    for (; L + 3 <= Lf1; L += 4) {
      fast(spA, srA, srB, P0, P1, P2, R0, R1);
      fast(spB, srB, srA, P1, P2, P3, R1, R2);
      fast(spA, srA, srB, P2, P3, P0, R2, R3);
      fast(spB, srB, srA, P3, P0, P1, R3, R0);
    }
  }
  // the epilogue resumes at a multiple of 4 past z0 (the ring phase)
  while (L <= Lend) L = gen_block(L, Lend);
}

// ZIN: the input iterate is identically zero (first sweep of a correction
// solve); it is then never read.
template <class T, int TYH, bool ZIN>
__global__ void __launch_bounds__(kW * TYH)
k_sor_fused(const T* __restrict__ p_in, T* __restrict__ p_out, const T* __restrict__ rhs, Geo g,
            Ctl* ctl, double* part, double omega, int m, int itermax, int write, int inner,
            int zc, int ntx, int nty, int ntiles) {
  __shared__ T sp[2][TYH * kW];
  __shared__ T sr[2][TYH * kW];
  __shared__ double shred[16];
  __shared__ int sh_last;
  if (ctl->done) return;
  double acc = 0.0;

  // Persistent loop over tiles.  Workgroup b runs on XCD b % 8; the tiles
  // are split into 8 contiguous ranges, one per XCD, dealt round-robin to
  // that XCD's workgroups, so the tiles in flight on one XCD are neighbours.
  // (Fewer than 8 workgroups: plain strided order.)
  const int G = gridDim.x;
  const bool by_xcd = G >= 8;
  const int xcd = by_xcd ? (blockIdx.x & 7) : 0;
  const int slot = by_xcd ? (blockIdx.x >> 3) : blockIdx.x;
  const int nwg_x = by_xcd ? (G >> 3) + (xcd < (G & 7) ? 1 : 0) : G;  // workgroups on this XCD
  const int lo = by_xcd ? (int)((long)ntiles * xcd / 8) : 0;
  const int hi = by_xcd ? (int)((long)ntiles * (xcd + 1) / 8) : ntiles;
  for (int tile = lo + slot; tile < hi; tile += nwg_x) {
    sweep_tile<T, TYH, ZIN>(p_in, p_out, rhs, g, omega, write, tile, zc, ntx, nty, sp, sr, acc);
    // the next tile reuses the LDS planes
    __syncthreads();
  }

  // FP64 residual partial of this workgroup; the last one applies the stop rule
  const long n = (long)g.nx * g.ny * g.nz;
  double s = block_sum(acc, shred);
  if (publish_partial(part, blockIdx.x, s, ctl, gridDim.x, &sh_last)) {
    double tot = sum_partials(part, gridDim.x, shred);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      const double res = sqrt(tot / (double)n);
      const int mm = m - 1;
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

// Resident workgroups of one kernel on this device (occupancy x CUs),
// cached per kernel.
template <class T, int TYH>
int resident_groups() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sor_fused<T, TYH, false>, kW * TYH, 0) !=
      hipSuccess)
    return 0;
  cached = cus * (per_cu > 0 ? per_cu : 1);
  return cached;
}

template <class T, int TYH>
hipError_t launch_ty(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs, Ctl* ctl,
                     double* part, double omega, int m, int itermax, int write, int zero_in, int inner,
                     int zc) {
  constexpr int TY = TYH - 4;
  const int ntx = (g.nx + kTX - 1) / kTX;
  const int nty = (g.ny + TY - 1) / TY;
  const int ntz = (g.nz + zc - 1) / zc;
  const int ntiles = ntx * nty * ntz;
  int nb = resident_groups<T, TYH>();
  if (nb <= 0 || nb > ntiles) nb = ntiles;
  if (zero_in)
    k_sor_fused<T, TYH, true><<<nb, dim3(kW, TYH), 0, st>>>(p_in, p_out, rhs, g, ctl, part, omega, m, itermax,
                                                            write, inner, zc, ntx, nty, ntiles);
  else
    k_sor_fused<T, TYH, false><<<nb, dim3(kW, TYH), 0, st>>>(p_in, p_out, rhs, g, ctl, part, omega, m, itermax,
                                                             write, inner, zc, ntx, nty, ntiles);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched sweep: one launch sweeps every domain of a batch.  Workgroup b
// belongs to the domain whose [first, first + ntiles) range holds b (found by
// binary search in the item table) and sweeps one tile of it; each domain has
// its own partial sums, ticket, stop rule and sweep budget, and its
// workgroups return at once when its done flag is set.
template <class T, int TYH, bool ZIN>
__global__ void __launch_bounds__(kW * TYH)
k_sor_batched(const BatchItem* __restrict__ items, int nitems, int m, int write) {
  __shared__ T sp[2][TYH * kW];
  __shared__ T sr[2][TYH * kW];
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
  if (ctl->done) return;
  const int tile = b - it.first;
  const T* p_in = (const T*)it.p[(it.cur + m - 1) & 1];
  T* p_out = (T*)it.p[(it.cur + m) & 1];
  const Geo g = it.g;
  double acc = 0.0;
  sweep_tile<T, TYH, ZIN>(p_in, p_out, (const T*)it.rhs, g, it.omega, write, tile, it.zc, it.ntx, it.nty, sp, sr,
                          acc);
  __syncthreads();
  const double s = block_sum(acc, shred);
  if (publish_partial(it.part, tile, s, ctl, it.ntiles, &sh_last)) {
    const double tot = sum_partials(it.part, it.ntiles, shred);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      const long n = (long)g.nx * g.ny * g.nz;
      const double res = sqrt(tot / (double)n);
      const int mm = m - 1;
      const double thr = it.inner ? ctl->thr_in : ctl->thr;
      if (mm >= 1 || it.budget == 0) {
        if (it.inner) ctl->res_in = res; else ctl->res = res;
        const bool fin = isfinite(res);
        if (!(res > thr) || mm >= it.budget || !fin) {
          ctl->done = 1;
          ctl->final_ = mm;
          if (!fin) ctl->nonfinite = 1;
        }
      }
      ctl->ticket = 0;
    }
  }
}

template <class T, int TYH>
hipError_t launch_batched_ty(hipStream_t st, const BatchItem* items, int nitems, int nblocks, int m, int write,
                             int zero_in) {
  if (zero_in)
    k_sor_batched<T, TYH, true><<<nblocks, dim3(kW, TYH), 0, st>>>(items, nitems, m, write);
  else
    k_sor_batched<T, TYH, false><<<nblocks, dim3(kW, TYH), 0, st>>>(items, nitems, m, write);
  return hipGetLastError();
}

}  // namespace

int fused_num_blocks(const Geo& g, const SorShape& s) {
  const int ty = s.ty;
  const int zc = item_chunk(g.nz, s.zc);
  return ((g.nx + kTX - 1) / kTX) * ((g.ny + ty - 1) / ty) * ((g.nz + zc - 1) / zc);
}

bool fused_shape_ok(const SorShape& s) { return s.ty == 4 || s.ty == 8 || s.ty == 12; }

int fused_resident(int ty, bool f32) {
  switch (ty) {
    case 4: return f32 ? resident_groups<float, 8>() : resident_groups<double, 8>();
    case 8: return f32 ? resident_groups<float, 12>() : resident_groups<double, 12>();
    case 12: return f32 ? resident_groups<float, 16>() : resident_groups<double, 16>();
    default: return 0;
  }
}

int fused_columns(const Geo& g, int ty) { return ((g.nx + kTX - 1) / kTX) * ((g.ny + ty - 1) / ty); }

template <class T>
hipError_t launch_sor_fused(hipStream_t st, const Geo& g, const T* p_in, T* p_out, const T* rhs, Ctl* ctl,
                            double* part, double omega, int m, int itermax, int write, int zero_in, int inner,
                            const SorShape& s) {
  const int zc = item_chunk(g.nz, s.zc);
  switch (s.ty) {
    case 4: return launch_ty<T, 8>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc);
    case 8: return launch_ty<T, 12>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc);
    case 12: return launch_ty<T, 16>(st, g, p_in, p_out, rhs, ctl, part, omega, m, itermax, write, zero_in, inner, zc);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_sor_fused<double>(hipStream_t, const Geo&, const double*, double*, const double*, Ctl*,
                                             double*, double, int, int, int, int, int, const SorShape&);
template hipError_t launch_sor_fused<float>(hipStream_t, const Geo&, const float*, float*, const float*, Ctl*,
                                            double*, double, int, int, int, int, int, const SorShape&);

}  // namespace ns

namespace ns {

void batch_item_shape(BatchItem& it, int ty, int zc) {
  it.ntx = (it.g.nx + kTX - 1) / kTX;
  it.nty = (it.g.ny + ty - 1) / ty;
  it.zc = item_chunk(it.g.nz, zc);
  it.ntiles = it.ntx * it.nty * ((it.g.nz + it.zc - 1) / it.zc);
}

template <class T>
hipError_t launch_sor_batched(hipStream_t st, const BatchItem* d_items, int nitems, int nblocks, int ty, int m,
                              int write, int zero_in) {
  switch (ty) {
    case 4: return launch_batched_ty<T, 8>(st, d_items, nitems, nblocks, m, write, zero_in);
    case 8: return launch_batched_ty<T, 12>(st, d_items, nitems, nblocks, m, write, zero_in);
    case 12: return launch_batched_ty<T, 16>(st, d_items, nitems, nblocks, m, write, zero_in);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_sor_batched<double>(hipStream_t, const BatchItem*, int, int, int, int, int, int);
template hipError_t launch_sor_batched<float>(hipStream_t, const BatchItem*, int, int, int, int, int, int);

}  // namespace ns
