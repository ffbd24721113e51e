// adjoint.hip -- transpose of the momentum predictor (gather form) and of
// the boundary fill, FP64.
//
// The predictor writes, for the unknown q of component c,
//   Phi_c = q + dt (nu lap q - sum_d (flux_cd(y=x) - flux_cd(y=x-e_d))/h_d + f_c)
// where flux_cd(y) = psi(t, a, b), t = (V_d[y] + V_d[y+e_c])/2,
// a = q_c[y], b = q_c[y+e_d] and psi(t,a,b) = t(a+b)/2 + gamma |t|(a-b)/2.
// Each flux is shared by the unknown below (+) and above (-) it, so its
// total weight in J^T mu is W_cd(y) = -dt/h_d (mu_c[y] - mu_c[y+e_d]) with mu
// zero off the unknowns.  The transpose at an entry e of component c'
// gathers every flux that reads e:
//   as a:          W_{c'd}(e)      dpsi/da
//   as b:          W_{c'd}(e-e_d)  dpsi/db
//   as transport:  W_{c,c'}(e) and W_{c,c'}(e-e_c), each dpsi/dt / 2
// plus the identity and the (symmetric) viscous term.  No atomics: every
// output entry is written by one thread.  z is computed on the whole padded
// range (ghosts included) and then folded back onto the unknowns by the
// transpose of the boundary fill (k_fold_*), with sign(0) := 0.
#include <hip/hip_runtime.h>

#include "ns_internal.h"

namespace ns {

namespace {

constexpr int kBlock = 256;

struct Fields {
  const double* q[3];   // velocity components (boundary-filled)
  const double* mu[3];  // adjoint weights, zero off the unknowns
};

__device__ __forceinline__ long stride_of(const Geo& g, int a) { return a == 0 ? 1 : (a == 1 ? g.sx : g.sxy); }
__device__ __forceinline__ int extent_of(const Geo& g, int a) { return a == 0 ? g.nx : (a == 1 ? g.ny : g.nz); }
__device__ __forceinline__ double h_of(const Geo& g, int a) { return a == 0 ? g.dx : (a == 1 ? g.dy : g.dz); }

// Contribution of flux (c, d) at edge position y (index triple yi) to the
// entry of role `role` (0 = a, 1 = b, 2 = transport).  Returns 0 when the
// flux has no weight (both flanking entries are not unknowns) or lies
// outside the padded box.
__device__ __forceinline__ double flux_term(const Geo& g, const Fields& f, int c, int d, const int yi[3],
                                            int role, double dt, double gamma) {
  // y and y + e_d must be inside the padded box
  if (yi[0] < 0 || yi[1] < 0 || yi[2] < 0) return 0.0;
  if (yi[0] > g.nx + 1 || yi[1] > g.ny + 1 || yi[2] > g.nz + 1) return 0.0;
  if (yi[d] + 1 > extent_of(g, d) + 1 || yi[c] + 1 > extent_of(g, c) + 1) return 0.0;
  const long y = (long)yi[2] * g.sxy + (long)yi[1] * g.sx + yi[0];
  const long sd = stride_of(g, d), sc = stride_of(g, c);
  const double W = -dt / h_of(g, d) * (f.mu[c][y] - f.mu[c][y + sd]);
  if (W == 0.0) return 0.0;
  // W != 0 implies y or y + e_d is an unknown of c, so y + e_c is in bounds.
  const double t = 0.5 * (f.q[d][y] + f.q[d][y + sc]);
  const double a = f.q[c][y], b = f.q[c][y + sd];
  if (role == 0) return W * 0.5 * (t + gamma * fabs(t));
  if (role == 1) return W * 0.5 * (t - gamma * fabs(t));
  const double sg = t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0);
  return W * 0.5 * 0.5 * ((a + b) + gamma * sg * (a - b));
}

__global__ void __launch_bounds__(kBlock)
k_adj_fgh(Fields f, double* __restrict__ zu, double* __restrict__ zv, double* __restrict__ zw, Geo g,
          double dt, double nu, double gamma) {
  double* z[3] = {zu, zv, zw};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g.ntot; e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e / g.sxy);
    const long rem = e - (long)k * g.sxy;
    const int j = (int)(rem / g.sx);
    const int i = (int)(rem - (long)j * g.sx);
    const int ei[3] = {i, j, k};
#pragma unroll
    for (int cp = 0; cp < 3; cp++) {
      const double* mu = f.mu[cp];
      double acc = mu[e];  // identity
      // viscous: dt nu sum_d (mu[e+e_d] + mu[e-e_d] - 2 mu[e]) / h_d^2
      const double ih2[3] = {g.idx2, g.idy2, g.idz2};
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const long sd = stride_of(g, d);
        const double up = ei[d] + 1 <= extent_of(g, d) + 1 ? mu[e + sd] : 0.0;
        const double dn = ei[d] - 1 >= 0 ? mu[e - sd] : 0.0;
        acc += dt * nu * (up + dn - 2.0 * mu[e]) * ih2[d];
      }
      // convective fluxes of component cp reading e as a or b
#pragma unroll
      for (int d = 0; d < 3; d++) {
        acc += flux_term(g, f, cp, d, ei, 0, dt, gamma);
        int yi[3] = {ei[0], ei[1], ei[2]};
        yi[d] -= 1;
        acc += flux_term(g, f, cp, d, yi, 1, dt, gamma);
      }
      // fluxes of every component c transported by velocity component cp
#pragma unroll
      for (int c = 0; c < 3; c++) {
        acc += flux_term(g, f, c, cp, ei, 2, dt, gamma);
        int yi[3] = {ei[0], ei[1], ei[2]};
        yi[c] -= 1;
        acc += flux_term(g, f, c, cp, yi, 2, dt, gamma);
      }
      z[cp][e] = acc;
    }
  }
}

// Transpose of the periodic copy along one axis (full extent):
// z[1] += z[n+1]; z[n] += z[0]; ghosts := 0.
__global__ void k_fold_periodic(double* __restrict__ z0, double* __restrict__ z1, double* __restrict__ z2,
                                Geo g, int ax) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y * blockDim.y + threadIdx.y;
  long base, st;
  int n;
  if (ax == 0) {
    if (a > g.ny + 1 || b > g.nz + 1) return;
    base = (long)b * g.sxy + (long)a * g.sx; st = 1; n = g.nx;
  } else if (ax == 1) {
    if (a > g.nx + 1 || b > g.nz + 1) return;
    base = (long)b * g.sxy + a; st = g.sx; n = g.ny;
  } else {
    if (a > g.nx + 1 || b > g.ny + 1) return;
    base = (long)b * g.sx + a; st = g.sxy; n = g.nz;
  }
  double* z[3] = {z0, z1, z2};
#pragma unroll
  for (int c = 0; c < 3; c++) {
    double* q = z[c];
    q[base + st] += q[base + (long)(n + 1) * st];
    q[base + (long)(n + 1) * st] = 0.0;
    q[base + (long)n * st] += q[base];
    q[base] = 0.0;
  }
}

// Transpose of the tangential reflections of one wall axis:
// z[interior] -= z[ghost]; z[ghost] := 0 (the wall value is a constant).
__global__ void k_fold_reflect(double* __restrict__ zu, double* __restrict__ zv, double* __restrict__ zw,
                               Geo g, int ax) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int b = blockIdx.y * blockDim.y + threadIdx.y + 1;
  long base, st;
  int n;
  double *f0, *f1;
  if (ax == 0) {
    if (a > g.ny || b > g.nz) return;
    base = (long)b * g.sxy + (long)a * g.sx; st = 1; n = g.nx; f0 = zv; f1 = zw;
  } else if (ax == 1) {
    if (a > g.nx || b > g.nz) return;
    base = (long)b * g.sxy + a; st = g.sx; n = g.ny; f0 = zu; f1 = zw;
  } else {
    if (a > g.nx || b > g.ny) return;
    base = (long)b * g.sx + a; st = g.sxy; n = g.nz; f0 = zu; f1 = zv;
  }
  double* f[2] = {f0, f1};
#pragma unroll
  for (int q = 0; q < 2; q++) {
    double* z = f[q];
    z[base + (long)n * st] -= z[base + (long)(n + 1) * st];
    z[base + (long)(n + 1) * st] = 0.0;
    z[base + st] -= z[base];
    z[base] = 0.0;
  }
}

dim3 face_grid(const Geo& g, dim3 blk) {
  int m = g.nx > g.ny ? g.nx : g.ny;
  m = m > g.nz ? m : g.nz;
  m += 2;
  return dim3((m + blk.x - 1) / blk.x, (m + blk.y - 1) / blk.y, 1);
}

}  // namespace

hipError_t launch_adj_fgh(hipStream_t st, const Geo& g, const double* u, const double* v,
                          const double* w, const double* mu, const double* mv, const double* mw,
                          double* zu, double* zv, double* zw, double dt, double re, double gamma) {
  Fields f;
  f.q[0] = u; f.q[1] = v; f.q[2] = w;
  f.mu[0] = mu; f.mu[1] = mv; f.mu[2] = mw;
  long nb = (g.ntot + kBlock - 1) / kBlock;
  if (nb > 65536) nb = 65536;
  k_adj_fgh<<<(int)nb, kBlock, 0, st>>>(f, zu, zv, zw, g, dt, 1.0 / re, gamma);
  return hipGetLastError();
}

hipError_t launch_adj_fold(hipStream_t st, const Geo& g, double* zu, double* zv, double* zw) {
  dim3 blk(64, 4);
  dim3 grd = face_grid(g, blk);
  for (int ax = 2; ax >= 0; ax--)
    if (g.per[ax]) k_fold_periodic<<<grd, blk, 0, st>>>(zu, zv, zw, g, ax);
  for (int ax = 2; ax >= 0; ax--)
    if (!g.per[ax]) k_fold_reflect<<<grd, blk, 0, st>>>(zu, zv, zw, g, ax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_mask_unknowns(st, g, zu, 0);
  if (e == hipSuccess) e = launch_mask_unknowns(st, g, zv, 1);
  if (e == hipSuccess) e = launch_mask_unknowns(st, g, zw, 2);
  return e;
}

}  // namespace ns
