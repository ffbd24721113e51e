// runtime.hip -- host runtime and C ABI of libns.so (see include/ns.h).
//
// One handle owns one HIP stream (the caller's) and, per instance, every
// device buffer of the step.  A step enqueues its stage kernels on that
// stream; the Poisson solve enqueues red-black sweeps in chunks and, after
// each chunk, reads the instance's 128-byte control block back (the only
// device-to-host traffic inside a step).  Sweeps launched after the stop
// rule fired return at once on the device flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include <sys/stat.h>

#include "convection.h"
#include "generated.h"
#include "ns.h"
#include "ns_internal.h"

using namespace ns;

namespace {

thread_local std::string g_create_err = "no error";

struct State {
  void* u = nullptr;
  void* v = nullptr;
  void* w = nullptr;
  double* p[2] = {nullptr, nullptr};
  int pcur = 0;
};

struct Inst {
  ns_params prm{};
  Geo g{};
  bool mixed = false;
  size_t esz = 8;      // bytes per element of u, v, w, F, G, H, rhs, forces
  size_t bytes = 0;    // ntot * esz
  size_t pbytes = 0;   // ntot * 8
  State s;
  void* F = nullptr;
  void* G = nullptr;
  void* H = nullptr;
  void* rhs = nullptr;
  void* frc[3] = {nullptr, nullptr, nullptr};
  float* e[2] = {nullptr, nullptr};
  float* r = nullptr;
  void* save[3] = {nullptr, nullptr, nullptr};  // NS_RK2: u^n, v^n, w^n
  double* part = nullptr;
  Ctl* ctl = nullptr;
  ns_stats st{};
  int pred = 0;
  SorShape shape{8, 0};
  // adjoint recording (FP64)
  std::vector<State> ck;
  int rec_steps = 0;
  bool rec_valid = false;
  // adjoint work (lazily allocated)
  State R;
  double* lam[3] = {nullptr, nullptr, nullptr};
  double* z[3] = {nullptr, nullptr, nullptr};
  double* q[2] = {nullptr, nullptr};
  int qcur = 0;
  std::vector<double*> hist;
};

// Launches of one solve, to find the buffer of the accepted iterate.
struct SweepLaunch {
  int m1, ns, in, out;  // first sweep index, sweeps, input / output buffer
};

struct EvRec {
  hipEvent_t a, b;
  int stage;
  int m;            // sweep index (SOR) or 0
  long long bytes;  // algorithmic bytes of the launch
};

}  // namespace

struct ns_solver {
  std::vector<Inst> in;
  hipStream_t stream = nullptr;
  Ctl* hctl = nullptr;  // pinned host mirror, one per instance
  std::string err = "no error";
  int device = 0;
  bool timing = false;
  ns_timing tm{};
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  std::vector<EvRec> recs;
  double* stage = nullptr;  // FP64 staging buffer for conversions
  size_t stage_n = 0;
  Ctl* ctl_all = nullptr;   // control blocks of all instances, contiguous
  // batched sweeps (several instances of one precision)
  bool batched = false;
  int batch_ty = 8, batch_zc = 0;
  BatchItem* items_h = nullptr;  // pinned
  BatchItem* items_d = nullptr;
  // batched cell stages: one table slice per stage kind (a slice is
  // rewritten only after a stream synchronisation has passed its last copy)
  StageItem* stage_h = nullptr;  // pinned
  StageItem* stage_d = nullptr;
  // batched: the per-domain stages (boundary fill, predictor, rhs, defect,
  // projection) are spread over a few library streams so that the small
  // kernels of different domains overlap
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kAux] = {};
  // launches of the current FP64 solve (kept across solves so that its
  // capacity is reused)
  std::vector<SweepLaunch> launch_log;
  // batched: every step of every domain in one persistent launch (teams of
  // workgroups per domain, device-side barriers and stop rules)
  bool persist = false;
  int persist_blocks = 0;
  long long persist_limit = 0;  // wall-clock ticks a barrier wait may take
  double clock_khz = 0.0;       // device wall-clock rate
  PItem* pitems_h = nullptr;    // pinned
  PItem* pitems_d = nullptr;
  PSlot* pslots_d = nullptr;
  PStats* pstats_h = nullptr;   // pinned
  PStats* pstats_d = nullptr;
  unsigned* pbar_d = nullptr;
  int* perr_d = nullptr;
  int* perr_h = nullptr;        // pinned
};

namespace {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

ns_status fail(ns_solver* s, ns_status code, const std::string& msg) {
  if (s) s->err = msg;
  else g_create_err = msg;
  return code;
}

ns_status fail_hip(ns_solver* s, const char* what, hipError_t e) {
  // the failure is reported here: clear it from the thread's last-error
  // state, or the launch check of a later call would report it again
  (void)hipGetLastError();
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(s, e == hipErrorOutOfMemory ? NS_E_OOM : NS_E_DEVICE, m);
}

#define HCK(s, x)                                      \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return fail_hip((s), #x, e_); \
  } while (0)

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}
__global__ void k_to_f64(const float* __restrict__ a, double* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}
int conv_grid(long n) {
  long b = (n + 255) / 256;
  return (int)std::min<long>(std::max<long>(b, 1), 16384);
}

Geo make_geo(const ns_params& p) {
  Geo g{};
  g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
  g.sx = p.nx + 2;
  g.sxy = g.sx * (long)(p.ny + 2);
  g.ntot = g.sxy * (long)(p.nz + 2);
  g.dx = p.lx / p.nx; g.dy = p.ly / p.ny; g.dz = p.lz / p.nz;
  g.idx = 1.0 / g.dx; g.idy = 1.0 / g.dy; g.idz = 1.0 / g.dz;
  g.idx2 = g.idx * g.idx; g.idy2 = g.idy * g.idy; g.idz2 = g.idz * g.idz;
  for (int a = 0; a < 3; a++) g.per[a] = p.bc[a] == NS_BC_PERIODIC;
  const int n[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; a++) g.hi[a] = g.per[a] ? n[a] : n[a] - 1;
  return g;
}

ns_status validate(const ns_params& p, int idx) {
  char b[256];
  auto bad = [&](const char* what) {
    snprintf(b, sizeof b, "instance %d: %s", idx, what);
    return fail(nullptr, NS_E_INVALID, b);
  };
  if (p.struct_size != sizeof(ns_params)) return bad("struct_size != sizeof(ns_params)");
  const int n[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; a++) {
    if (n[a] < 2) return bad("every axis needs at least 2 cells");
    if (n[a] > 32768) return bad("axis longer than 32768 cells");
    if (p.bc[a] != NS_BC_WALL && p.bc[a] != NS_BC_PERIODIC) return bad("bc must be wall or periodic");
    if (p.bc[a] == NS_BC_PERIODIC && (n[a] & 1)) return bad("periodic axes need an even cell count");
  }
  if ((double)(p.nx + 2) * (p.ny + 2) * (p.nz + 2) > 4.0e9) return bad("grid too large");
  if (!(p.lx > 0 && p.ly > 0 && p.lz > 0)) return bad("domain extents must be positive");
  if (!(p.re > 0) || !std::isfinite(p.re)) return bad("re must be positive");
  if (!std::isfinite(p.dt)) return bad("dt must be finite");
  if (p.dt <= 0 && !(p.tau > 0 && p.tau <= 1)) return bad("adaptive dt needs tau in (0, 1]");
  if (!(p.gamma >= 0 && p.gamma <= 1)) return bad("gamma must lie in [0, 1]");
  if (!(p.omega > 0 && p.omega < 2)) return bad("omega must lie in (0, 2)");
  if (!(p.tol >= 0) || !std::isfinite(p.tol)) return bad("tol must be >= 0");
  if (p.itermax < 0) return bad("itermax must be >= 0");
  if (p.precision != NS_FP64 && p.precision != NS_MIXED) return bad("precision must be NS_FP64 or NS_MIXED");
  if (p.precision == NS_MIXED && !(p.eta > 0 && p.eta < 1)) return bad("mixed precision needs eta in (0, 1)");
  if (p.checkpoint_every < 0) return bad("checkpoint_every must be >= 0");
  if (p.checkpoint_every > 0 && (p.precision != NS_FP64 || p.dt <= 0))
    return bad("recording for ns_backward needs NS_FP64 and a fixed dt");
  for (int f = 0; f < 6; f++)
    for (int c = 0; c < 3; c++)
      if (!std::isfinite(p.wall_vel[f][c])) return bad("wall velocities must be finite");
  for (int c = 0; c < 3; c++)
    if (!std::isfinite(p.g[c])) return bad("body force must be finite");
  if (p.flags & ~(NS_ALLOW_UNSTABLE | NS_TIMING | NS_BATCH_LAUNCHES | NS_GENERATED | NS_ADVECTIVE | NS_RK2))
    return bad("unknown flag bits");
  if ((p.flags & NS_ADVECTIVE) && p.checkpoint_every > 0)
    return bad("the adjoint covers the conservative form only (NS_ADVECTIVE with checkpoint_every)");
  if ((p.flags & NS_RK2) && p.checkpoint_every > 0)
    return bad("the adjoint covers the Euler step only (NS_RK2 with checkpoint_every)");
  if (!(p.tile[0] == -1 || p.tile[0] == 0 || p.tile[0] == 4 || p.tile[0] == 8 || p.tile[0] == 12 ||
        p.tile[0] == 16 || p.tile[0] == 24 || p.tile[0] == 32))
    return bad("tile[0] must be -1, 0, 4, 8, 12, 16, 24 or 32");
  if (p.tile[0] > 0 && (double)(p.nx + 2) * (p.ny + 2) * (p.precision == NS_MIXED ? 4 : 8) >= 2147483648.0)
    return bad("planes this large need the unfused sweeps (tile = {-1, 0})");
  if (p.tile[0] > 16 && p.precision == NS_FP64)
    return bad("FP64 two-sweep tiles have 16 rows (tile[0] = 16)");
  if (p.tile[0] >= 16)
    for (int a = 0; a < 3; a++)
      if (p.bc[a] == NS_BC_PERIODIC && n[a] < 4) return bad("the two-sweep pass needs periodic axes of at least 4 cells");
  if (p.dt > 0 && !(p.flags & NS_ALLOW_UNSTABLE)) {
    const double dx = p.lx / p.nx, dy = p.ly / p.ny, dz = p.lz / p.nz;
    const double diff = p.dt / p.re * (1 / (dx * dx) + 1 / (dy * dy) + 1 / (dz * dz));
    double wmax = 0;
    for (int f = 0; f < 6; f++)
      for (int c = 0; c < 3; c++) wmax = std::max(wmax, std::fabs(p.wall_vel[f][c]));
    const double cfl = wmax * p.dt / std::min(dx, std::min(dy, dz));
    if (diff > 0.5 || cfl > 1.0) {
      snprintf(b, sizeof b,
               "instance %d: dt = %g exceeds the explicit bounds (diffusion number %.3g > 0.5 or "
               "wall CFL %.3g > 1); set NS_ALLOW_UNSTABLE to run anyway",
               idx, p.dt, diff, cfl);
      return fail(nullptr, NS_E_UNSTABLE, b);
    }
  }
  return NS_OK;
}

// The fused one-sweep kernels address a plane with 32-bit byte offsets:
// planes must stay under 2^31 bytes (the two-sweep pass has the same limit,
// pass_grid_ok).  Larger planes take the unfused sweeps.
bool fused_grid_ok(const Geo& g, size_t esz) { return (double)g.sxy * (double)esz < 2147483648.0; }

// Whether a sweep shape may run on a grid: fused shapes need fused_grid_ok,
// pass shapes pass_grid_ok and their row count; the unfused sweeps run on
// every grid.
bool shape_fits_grid(const SorShape& sh, const Geo& g, size_t esz) {
  if (sh.ty < 0) return true;
  if (sh.ty == 4 || sh.ty == 8 || sh.ty == 12) return fused_grid_ok(g, esz);
  return pass_grid_ok(g, esz) && pass_rows_ok(sh.ty, esz == 4);
}

// Sweep shape: the caller's tile descriptor, or a size-based default that
// the autotuner may replace (see autotune()).
SorShape pick_shape(const ns_params& p, const Geo& g, size_t esz) {
  if (p.tile[0] < 0) return SorShape{-1, 0};
  if (p.tile[0] > 0) return SorShape{p.tile[0], p.tile[1]};
  if (!fused_grid_ok(g, esz)) return SorShape{-1, 0};
  const long n = (long)g.nx * g.ny * g.nz;
  if (n >= (1L << 24)) return SorShape{8, 128};
  return SorShape{8, 0};
}

hipError_t dmalloc(void** p, size_t bytes);
void dfree(void* p);

// ---- autotuner ---------------------------------------------------------------
// For grids of at least 2^21 cells with tile = {0, 0}: time candidate shapes
// on the instance's own (still zero) pressure buffers with HIP events, 1
// warm-up and 3 timed sweeps each, and keep the fastest.  Candidates: rows
// 4 / 8 / 12, each with the whole column, z chunks 32 / 64 / 128, and the z
// chunks that make the tile count just fit k times the resident workgroups
// (k = 1..8), which avoids a nearly empty last round of tiles.  Results are
// cached per grid shape, storage precision and boundary kind: in the process,
// and in a text file shared by processes (one line per result, keyed also by
// the device's architecture name, its compute-unit count and the library
// build, so a rebuilt library or another GPU tunes afresh).  The file is
// $NS_TUNE_CACHE, else $XDG_CACHE_HOME/nsmi/tune.txt, else
// $HOME/.cache/nsmi/tune.txt; NS_TUNE_CACHE=off (or empty) keeps results in
// the process only.  A line that does not parse or names a shape the
// library would not run is ignored.
struct TuneKey {
  int nx, ny, nz, esz, per;
  bool operator==(const TuneKey& o) const {
    return nx == o.nx && ny == o.ny && nz == o.nz && esz == o.esz && per == o.per;
  }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, SorShape>> g_tune_cache;
bool g_tune_loaded = false;
constexpr const char* kTuneBuild = "v1-" __DATE__ "-" __TIME__;

std::string tune_file() {
  const char* e = getenv("NS_TUNE_CACHE");
  if (e) return (e[0] == 0 || strcmp(e, "off") == 0) ? std::string() : std::string(e);
  if (const char* x = getenv("XDG_CACHE_HOME"); x && x[0]) return std::string(x) + "/nsmi/tune.txt";
  if (const char* h = getenv("HOME"); h && h[0]) return std::string(h) + "/.cache/nsmi/tune.txt";
  return std::string();
}

// "<arch> <compute units> <build>" of the current device, spaces in the
// build stamp replaced.
std::string tune_device_tag(int device) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, device) != hipSuccess) return std::string();
  std::string b = kTuneBuild;
  for (char& c : b)
    if (c == ' ') c = '_';
  char buf[512];
  snprintf(buf, sizeof buf, "%s %d %s", pr.gcnArchName, pr.multiProcessorCount, b.c_str());
  for (char* q = buf; *q; q++)
    if (*q == '\n') *q = ' ';
  return std::string(buf);
}

bool tune_shape_valid(const SorShape& sh, int esz) {
  if (sh.ty == 4 || sh.ty == 8 || sh.ty == 12) return sh.zc >= 0;
  if (sh.ty == 16 || sh.ty == 24 || sh.ty == 32) return sh.zc >= 0 && pass_rows_ok(sh.ty, esz == 4);
  return false;
}

// Reads the file's lines for this device into the process cache (caller
// holds g_tune_mu).
void tune_load(const std::string& tag) {
  const std::string path = tune_file();
  if (path.empty() || tag.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char arch[256], build[256];
    int cus, nx, ny, nz, esz, per, ty, zc;
    if (sscanf(line, "%255s %d %255s %d %d %d %d %d %d %d", arch, &cus, build, &nx, &ny, &nz, &esz, &per, &ty,
               &zc) != 10)
      continue;
    char mine[512];
    snprintf(mine, sizeof mine, "%s %d %s", arch, cus, build);
    if (tag != mine) continue;
    const TuneKey k{nx, ny, nz, esz, per};
    const SorShape sh{ty, zc};
    if (!tune_shape_valid(sh, esz)) continue;
    bool have = false;
    for (auto& kv : g_tune_cache) have |= kv.first == k;
    if (!have) g_tune_cache.push_back({k, sh});
  }
  fclose(f);
}

// Appends one result to the file (creating its directory); failures leave
// the process cache as the only record.
void tune_store(const std::string& tag, const TuneKey& k, const SorShape& sh) {
  const std::string path = tune_file();
  if (path.empty() || tag.empty()) return;
  for (size_t q = 1; q < path.size(); q++)
    if (path[q] == '/') (void)mkdir(path.substr(0, q).c_str(), 0755);
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %d %d %d %d\n", tag.c_str(), k.nx, k.ny, k.nz, k.esz, k.per, sh.ty, sh.zc);
  fclose(f);
}

template <class T>
ns_status tune_run(ns_solver* s, Inst& I, Ctl* tctl, const SorShape& sh, float* ms) {
  hipEvent_t a, b;
  HCK(s, hipEventCreate(&a));
  HCK(s, hipEventCreate(&b));
  const T* in = (const T*)(I.mixed ? (void*)I.e[0] : (void*)I.s.p[0]);
  T* out = (T*)(I.mixed ? (void*)I.e[1] : (void*)I.s.p[1]);
  const T* rhs = (const T*)(I.mixed ? (void*)I.r : I.rhs);
  hipError_t e = hipSuccess;
  // one warm-up launch, then eight timed (the shapes of a batch lie within a
  // few per cent of each other, so fewer launches let noise pick)
  for (int it = 0; it < 9 && e == hipSuccess; it++) {
    if (it == 1) e = hipEventRecord(a, s->stream);
    // sweep index 1 (pass: 0): no residual of these launches is a stop decision
    if (e == hipSuccess)
      e = shape_is_pass(sh) ? launch_sor_pass<T>(s->stream, I.g, in, out, rhs, tctl, I.part, I.prm.omega, 0,
                                                 1 << 30, 1, 0, 0, 2, sh)
                            : launch_sor_sweep<T>(s->stream, I.g, in, out, rhs, tctl, I.part, I.prm.omega, 1,
                                                  1 << 30, 1, 0, 0, sh);
  }
  if (e == hipSuccess) e = hipEventRecord(b, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail_hip(s, "autotune", e);
  if (shape_is_pass(sh)) *ms *= 0.5f;  // per sweep
  return NS_OK;
}

ns_status autotune(ns_solver* s, Inst& I) {
  const long n = (long)I.g.nx * I.g.ny * I.g.nz;
  // planes too large for the fused kernels are too large for the pass too:
  // the unfused sweeps are the only shape
  if (I.prm.tile[0] != 0 || n < (1L << 21) || !fused_grid_ok(I.g, I.esz)) return NS_OK;
  const TuneKey key{I.g.nx, I.g.ny, I.g.nz, (int)I.esz, I.g.per[0] | (I.g.per[1] << 1) | (I.g.per[2] << 2)};
  const std::string tag = tune_device_tag(s->device);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
      tune_load(tag);
      g_tune_loaded = true;
    }
    for (auto& kv : g_tune_cache)
      if (kv.first == key && shape_fits_grid(kv.second, I.g, I.esz)) { I.shape = kv.second; return NS_OK; }
  }
  Ctl* tctl = nullptr;
  HCK(s, dmalloc((void**)&tctl, sizeof(Ctl)));
  const bool pass_ok = pass_grid_ok(I.g, I.esz);
  const int rows[6] = {4, 8, 12, 16, 24, 32};
  float best = 1e30f;
  SorShape pick = I.shape;
  ns_status st = NS_OK;
  for (int r = 0; r < 6 && st == NS_OK; r++) {
    const bool pass = rows[r] >= 16;
    if (pass && (!pass_ok || !pass_rows_ok(rows[r], I.mixed))) continue;
    std::vector<int> zcs = {0, 32, 64, 128};
    const int res = pass ? pass_resident_groups(rows[r], I.mixed, 2) : fused_resident(rows[r], I.mixed);
    const int cols = pass ? pass_columns(I.g, rows[r], 2) : fused_columns(I.g, rows[r]);
    for (int k = 1; k <= 8 && res > 0; k++) {
      const int ntz = (int)((long)k * res / cols);
      if (ntz < 1) continue;
      const int zc = (I.g.nz + ntz - 1) / ntz;
      if (zc >= 8 && zc < I.g.nz) zcs.push_back(zc);
    }
    std::sort(zcs.begin(), zcs.end());
    zcs.erase(std::unique(zcs.begin(), zcs.end()), zcs.end());
    for (int zc : zcs) {
      if (st != NS_OK) break;
      const SorShape sh{rows[r], zc};
      float ms = 0.f;
      st = I.mixed ? tune_run<float>(s, I, tctl, sh, &ms) : tune_run<double>(s, I, tctl, sh, &ms);
      if (st == NS_OK && ms < best) { best = ms; pick = sh; }
    }
  }
  dfree(tctl);
  if (st != NS_OK) return st;
  I.shape = pick;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.push_back({key, pick});
  tune_store(tag, key, pick);
  return NS_OK;
}

// Puts the items of a batch table in order of decreasing chunk length
// (stable) and numbers their workgroups.  Workgroups start in index order as
// compute units free up, so a launch whose longest tiles start first does
// not end waiting on one long tile that started last (longest-first list
// scheduling).  Returns the permutation: table entry k is the caller's item
// ord[k].
std::vector<int> order_longest_first(BatchItem* items, int n) {
  std::vector<int> ord(n);
  for (int k = 0; k < n; k++) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return items[a].zc > items[b].zc; });
  std::vector<BatchItem> tmp(items, items + n);
  int nb = 0;
  for (int k = 0; k < n; k++) {
    items[k] = tmp[ord[k]];
    items[k].first = nb;
    nb += items[k].ntiles;
  }
  return ord;
}

// Batch shape: time the one-sweep rows 4 / 8 / 12 and the two-sweep pass
// rows 16 / 24 / 32 (per sweep) x z chunks (whole column, 32, 16, and
// chunks of at most 48 planes balanced per domain) with one batched launch
// each over all instances (zero buffers, a scratch control array that
// never converges), keep the fastest.
template <class T>
ns_status tune_batch_run(ns_solver* s, Ctl* tctl, int ty, int zc, float* ms) {
  const int n = (int)s->in.size();
  int nblocks = 0;
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    BatchItem& it = s->items_h[i];
    it.g = I.g;
    it.p[0] = I.mixed ? (void*)I.e[0] : (void*)I.s.p[0];
    it.p[1] = I.mixed ? (void*)I.e[1] : (void*)I.s.p[1];
    it.rhs = I.mixed ? (const void*)I.r : (const void*)I.rhs;
    it.ctl = tctl + i;
    it.part = I.part;
    it.omega = I.prm.omega;
    it.cur = 0;
    it.budget = 1 << 30;
    it.inner = 0;
    if (ty >= 16) pass_item_shape(it, ty, zc, 2);
    else batch_item_shape(it, ty, zc);
    nblocks += it.ntiles;
  }
  (void)order_longest_first(s->items_h, n);
  HCK(s, hipMemcpyAsync(s->items_d, s->items_h, sizeof(BatchItem) * n, hipMemcpyHostToDevice, s->stream));
  hipEvent_t a, b;
  HCK(s, hipEventCreate(&a));
  HCK(s, hipEventCreate(&b));
  hipError_t e = hipSuccess;
  // one warm-up launch, then eight timed (the shapes of a batch lie within a
  // few per cent of each other, so fewer launches let noise pick)
  for (int it = 0; it < 9 && e == hipSuccess; it++) {
    if (it == 1) e = hipEventRecord(a, s->stream);
    // sweep index 1 (pass: 0): no residual of these launches is a stop decision
    if (e == hipSuccess)
      e = ty >= 16 ? launch_pass_batched<T>(s->stream, s->items_d, n, nblocks, ty, 0, 0, 2, 0, 0)
                   : launch_sor_batched<T>(s->stream, s->items_d, n, nblocks, ty, 1, 1, 0);
  }
  if (e == hipSuccess) e = hipEventRecord(b, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail_hip(s, "batch autotune", e);
  if (ty >= 16) *ms *= 0.5f;  // per sweep
  return NS_OK;
}

ns_status autotune_batch(ns_solver* s) {
  const int n = (int)s->in.size();
  Ctl* tctl = nullptr;
  HCK(s, dmalloc((void**)&tctl, sizeof(Ctl) * n));
  bool pass_ok = true;
  for (auto& I : s->in) pass_ok &= pass_grid_ok(I.g, I.esz);
  const int rows[6] = {4, 8, 12, 16, 24, 32};
  const int zcs[4] = {0, 32, 16, -48};
  // Two rounds over the shapes, each shape keeping its faster time: in one
  // round the shapes timed first ran while the device was still warming up
  // and lost to later ones that are slower in the solve.
  float ms_of[6][4];
  for (int r = 0; r < 6; r++)
    for (int z = 0; z < 4; z++) ms_of[r][z] = 1e30f;
  ns_status st = NS_OK;
  for (int round = 0; round < 2 && st == NS_OK; round++)
    for (int r = 0; r < 6 && st == NS_OK; r++)
      for (int z = 0; z < 4 && st == NS_OK; z++) {
        if (rows[r] >= 16 && (!pass_ok || !pass_rows_ok(rows[r], s->in[0].mixed))) continue;
        float ms = 0.f;
        st = s->in[0].mixed ? tune_batch_run<float>(s, tctl, rows[r], zcs[z], &ms)
                            : tune_batch_run<double>(s, tctl, rows[r], zcs[z], &ms);
        if (st == NS_OK && ms < ms_of[r][z]) ms_of[r][z] = ms;
      }
  float best = 1e30f;
  for (int r = 0; r < 6; r++)
    for (int z = 0; z < 4; z++)
      if (ms_of[r][z] < best) {
        best = ms_of[r][z];
        s->batch_ty = rows[r];
        s->batch_zc = zcs[z];
      }
  dfree(tctl);
  return st;
}

// ---- guard bands (debugging) ------------------------------------------------
// While NS_GUARD is set in the environment (to anything but "" or "0"), every
// buffer dmalloc returns sits between two bands of kGuard bytes that hold
// kGuardByte.  dfree, and ns_guard_check, compare both bands with the
// pattern and count each band that differs: a kernel that writes past either
// end of a buffer -- into memory that may belong to a neighbouring
// allocation, so that nothing faults -- shows up as a count.  Buffers
// allocated without the bands are freed as usual.
constexpr size_t kGuard = 4096;
constexpr int kGuardByte = 0xA5;
struct GuardRec {
  char* base;    // start of the lower band
  size_t bytes;  // the buffer's own size
};
std::mutex g_guard_mu;
std::unordered_map<void*, GuardRec> g_guard;  // live guarded buffers, by the pointer handed out
long long g_guard_bad = 0;                    // bands found overwritten when their buffer was freed

bool guard_on() {
  const char* e = getenv("NS_GUARD");
  return e && e[0] && strcmp(e, "0") != 0;
}

// Number of bands of one buffer (0, 1 or 2) that no longer hold the pattern;
// the device is idle and the caller holds g_guard_mu.
int guard_scan(const GuardRec& r) {
  std::vector<unsigned char> h(kGuard);
  int bad = 0;
  const char* band[2] = {r.base, r.base + kGuard + r.bytes};
  for (int b = 0; b < 2; b++) {
    if (hipMemcpy(h.data(), band[b], kGuard, hipMemcpyDeviceToHost) != hipSuccess) {
      bad++;
      continue;
    }
    for (size_t i = 0; i < kGuard; i++)
      if (h[i] != kGuardByte) {
        fprintf(stderr, "libns: guard band %s a %zu-byte buffer overwritten (%zu bytes %s it)\n",
                b ? "after" : "before", r.bytes, b ? i : kGuard - i, b ? "past the end of" : "before");
        bad++;
        break;
      }
  }
  return bad;
}

// Zero-filled device buffer (with guard bands under NS_GUARD).
hipError_t dmalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (guard_on()) {
    const size_t body = (bytes + 255) & ~size_t(255);  // the upper band's page stays 256-byte aligned
    char* base = nullptr;
    hipError_t e = hipMalloc((void**)&base, body + 2 * kGuard);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // reported by the caller; not a later launch's error
      return e;
    }
    if ((e = hipMemset(base, kGuardByte, body + 2 * kGuard)) != hipSuccess ||
        (e = hipMemset(base + kGuard, 0, bytes)) != hipSuccess) {
      (void)hipFree(base);
      return e;
    }
    std::lock_guard<std::mutex> lk(g_guard_mu);
    g_guard[base + kGuard] = GuardRec{base, bytes};
    *p = base + kGuard;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // reported by the caller; not a later launch's error
    *p = nullptr;
    return e;
  }
  return hipMemset(*p, 0, bytes);
}

// Frees a dmalloc buffer (checking its bands if it has them); null is a no-op.
void dfree(void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_guard_mu);
    auto it = g_guard.find(p);
    if (it != g_guard.end()) {
      (void)hipDeviceSynchronize();
      g_guard_bad += guard_scan(it->second);
      (void)hipFree(it->second.base);
      g_guard.erase(it);
      return;
    }
  }
  (void)hipFree(p);
}

void free_state(State& s) {
  dfree(s.u); dfree(s.v); dfree(s.w);
  dfree(s.p[0]); dfree(s.p[1]);
  s = State{};
}

void free_inst(Inst& I) {
  free_state(I.s);
  dfree(I.F); dfree(I.G); dfree(I.H); dfree(I.rhs);
  for (int c = 0; c < 3; c++) dfree(I.frc[c]);
  dfree(I.e[0]); dfree(I.e[1]); dfree(I.r);
  for (int c = 0; c < 3; c++) dfree(I.save[c]);
  dfree(I.part);  // I.ctl lives in the handle's ctl_all
  for (auto& c : I.ck) free_state(c);
  I.ck.clear();
  free_state(I.R);
  for (int c = 0; c < 3; c++) { dfree(I.lam[c]); dfree(I.z[c]); }
  dfree(I.q[0]); dfree(I.q[1]);
  for (auto* h : I.hist) dfree(h);
  I.hist.clear();
}

hipError_t alloc_state(State& S, const Inst& I) {
  hipError_t e;
  if ((e = dmalloc(&S.u, I.bytes)) != hipSuccess) return e;
  if ((e = dmalloc(&S.v, I.bytes)) != hipSuccess) return e;
  if ((e = dmalloc(&S.w, I.bytes)) != hipSuccess) return e;
  if ((e = dmalloc((void**)&S.p[0], I.pbytes)) != hipSuccess) return e;
  if ((e = dmalloc((void**)&S.p[1], I.pbytes)) != hipSuccess) return e;
  S.pcur = 0;
  return hipSuccess;
}

// ---- timing ----------------------------------------------------------------
struct Timed {
  ns_solver* s;
  bool on;
  size_t idx;
  Timed(ns_solver* s_, int stage, int m = 0, long long bytes = 0) : s(s_), on(s_->timing), idx(0) {
    if (!on) return;
    if (s->pool_used + 2 > s->pool.size()) {
      for (int i = 0; i < 64; i++) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
        s->pool.push_back(e);
      }
    }
    EvRec r{s->pool[s->pool_used], s->pool[s->pool_used + 1], stage, m, bytes};
    s->pool_used += 2;
    (void)hipEventRecord(r.a, s->stream);
    idx = s->recs.size();
    s->recs.push_back(r);
  }
  ~Timed() {
    if (on) (void)hipEventRecord(s->recs[idx].b, s->stream);
  }
};

// After a synchronised step: fold recorded launches into the totals.  SOR
// launches with sweep index above `last_real` returned on the done flag and
// are not counted.
void harvest(ns_solver* s, int last_real) {
  if (!s->timing) return;
  for (auto& r : s->recs) {
    if (r.stage == NS_T_COUNT - 1) continue;  // returned on the done flag
    if (r.stage == NS_T_SOR && r.m < 1000000 && r.m > last_real) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    s->tm.ms[r.stage] += ms;
    s->tm.launches[r.stage] += 1;
    if (r.stage == NS_T_SOR) s->tm.sor_bytes += r.bytes;
  }
  s->recs.clear();
  s->pool_used = 0;
}

ns_status poll(ns_solver* s, int idx) {
  Inst& I = s->in[idx];
  HCK(s, hipMemcpyAsync(&s->hctl[idx], I.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  HCK(s, hipStreamSynchronize(s->stream));
  return NS_OK;
}

// ---- Poisson solves ----------------------------------------------------------
// FP64 red-black SOR on A p = rhs from P[*cur]; on return *cur indexes the
// accepted iterate, *sweeps its sweep count.
// One launch of a solve: ns sweeps (2 only with a pass shape) from the
// iterate in p_in into p_out, first sweep index m; ns = 0 computes only the
// residual of p_in.  force: sweep whatever the done flag says, no residual.
template <class T>
hipError_t sweep_launch(ns_solver* s, Inst& I, const T* p_in, T* p_out, const T* rhs, int m, int itermax,
                        int zero_in, int inner, int ns, bool force = false) {
  const int write = ns > 0;
  if (shape_is_pass(I.shape))
    return launch_sor_pass<T>(s->stream, I.g, p_in, p_out, rhs, I.ctl, force ? nullptr : I.part, I.prm.omega, m,
                              itermax, write, zero_in, inner, ns > 0 ? ns : 1, I.shape);
  if (force || ns > 1) return hipErrorInvalidValue;
  return launch_sor_sweep<T>(s->stream, I.g, p_in, p_out, rhs, I.ctl, I.part, I.prm.omega, m, itermax, write,
                             zero_in, inner, I.shape);
}


// Buffer holding iterate f, or -1.  An iterate that a two-sweep pass held
// only in registers is swept again (forced, bitwise the same arithmetic)
// from the pass's input into its output buffer.
template <class T>
int locate_iterate(ns_solver* s, Inst& I, const std::vector<SweepLaunch>& L, T* const buf[2], const T* rhs, int f,
                   int inner, int tag, long long bytes, ns_status* st) {
  *st = NS_OK;
  for (const SweepLaunch& l : L) {
    if (l.m1 - 1 == f) return l.in;
    if (l.ns == 2 && l.m1 == f) {
      Timed t(s, NS_T_SOR, tag, bytes);
      const hipError_t e =
          sweep_launch<T>(s, I, buf[l.in], buf[l.out], rhs, f, 1 << 30, l.m1 == 1 && inner, inner, 1, true);
      if (e != hipSuccess) {
        *st = fail_hip(s, "sweep", e);
        return -1;
      }
      return l.out;
    }
  }
  return -1;
}

// FP64 red-black SOR on A p = rhs from P[*cur]; on return *cur indexes the
// accepted iterate, *sweeps its sweep count.
ns_status solve_fp64(ns_solver* s, int idx, double* P[2], int* cur, int* sweeps) {
  Inst& I = s->in[idx];
  const int itermax = I.prm.itermax;
  const long N = (long)I.g.nx * I.g.ny * I.g.nz;
  const bool pairs = shape_is_pass(I.shape);
  int m = 0;     // newest iterate launched
  int b = *cur;  // its buffer
  std::vector<SweepLaunch>& L = s->launch_log;
  L.clear();
  int pred = std::min(std::max(I.pred + 2, 4), itermax + 1);
  bool first = true;
  for (;;) {
    int chunk = first ? pred : std::max(4, pred / 4);
    first = false;
    bool last_pass = false;
    for (int c = 0; c < chunk;) {
      if (m < itermax) {
        const int ns = pairs && m + 2 <= itermax ? 2 : 1;
        Timed t(s, NS_T_SOR, m + 1, 24LL * N);
        HCK(s, sweep_launch<double>(s, I, P[b], P[b ^ 1], (const double*)I.rhs, m + 1, itermax, 0, 0, ns));
        L.push_back({m + 1, ns, b, b ^ 1});
        b ^= 1;
        m += ns;
        c += ns;
      } else {
        Timed t(s, NS_T_SOR, m + 1, 16LL * N);
        HCK(s, sweep_launch<double>(s, I, P[b], (double*)nullptr, (const double*)I.rhs, m + 1, itermax, 0, 0, 0));
        L.push_back({m + 1, 0, b, -1});
        last_pass = true;
        break;
      }
    }
    ns_status e = poll(s, idx);
    if (e != NS_OK) return e;
    if (s->hctl[idx].done || last_pass) break;
  }
  const Ctl& h = s->hctl[idx];
  if (!h.done) return fail(s, NS_E_DEVICE, "Poisson solve ended without a decision");
  ns_status st = NS_OK;
  const int fb = locate_iterate<double>(s, I, L, P, (const double*)I.rhs, h.final_, 0, h.final_, 24LL * N, &st);
  if (st != NS_OK) return st;
  if (fb < 0) return fail(s, NS_E_DEVICE, "accepted iterate not found");
  *sweeps = h.final_;
  *cur = fb;
  I.pred = h.final_;
  return NS_OK;
}

// Mixed precision: FP64 outer defect correction around FP32 red-black
// sweeps on A e = r.  P (FP64) ping-pongs once per outer iteration.
ns_status solve_mixed(ns_solver* s, int idx, int* sweeps, int* outer) {
  Inst& I = s->in[idx];
  State& S = I.s;
  const int itermax = I.prm.itermax;
  const long N = (long)I.g.nx * I.g.ny * I.g.nz;
  const bool pairs = shape_is_pass(I.shape);
  int used = 0;
  *outer = 0;
  {
    Timed t(s, NS_T_DEFECT, 0, 20LL * N);
    HCK(s, launch_defect(s->stream, I.g, S.p[S.pcur], nullptr, nullptr, (const float*)I.rhs, I.r, I.ctl,
                         I.part, I.prm.eta));
  }
  for (;;) {
    ns_status e = poll(s, idx);
    if (e != NS_OK) return e;
    const Ctl& h = s->hctl[idx];
    if (h.outer_done || h.nonfinite || used >= itermax) break;
    (*outer)++;
    const int budget = itermax - used;
    int m = 0;
    int b = 0;  // buffer of iterate m (iterate 0 is zero and never read)
    std::vector<SweepLaunch> L;
    int pred = std::min(std::max(I.pred + 2, 4), budget);
    bool first = true;
    int f = -1, fb = -1;
    const size_t rec0 = s->recs.size();
    for (;;) {
      int chunk = first ? pred : std::max(4, pred / 4);
      first = false;
      for (int c = 0; c < chunk && m < budget;) {
        const int ns = pairs && m + 2 <= budget ? 2 : 1;
        Timed t(s, NS_T_SOR, 1000000 + m + 1, (m == 0 ? 8LL : 12LL) * N);
        HCK(s, sweep_launch<float>(s, I, I.e[b], I.e[b ^ 1], I.r, m + 1, itermax + 1, m == 0, 1, ns));
        L.push_back({m + 1, ns, b, b ^ 1});
        b ^= 1;
        m += ns;
        c += ns;
      }
      e = poll(s, idx);
      if (e != NS_OK) return e;
      if (s->hctl[idx].done) {
        f = s->hctl[idx].final_;
        ns_status st = NS_OK;
        fb = locate_iterate<float>(s, I, L, I.e, I.r, f, 1, 1000000 + f, 12LL * N, &st);
        if (st != NS_OK) return st;
        if (fb < 0) return fail(s, NS_E_DEVICE, "accepted correction not found");
        break;
      }
      if (m >= budget) { f = budget; fb = b; break; }
    }
    used += f;
    I.pred = f;
    // launches past the one that found convergence returned on the flag
    for (size_t q = rec0; q < s->recs.size(); q++)
      if (s->recs[q].stage == NS_T_SOR && s->recs[q].m - 1000000 > f + 1) s->recs[q].stage = NS_T_COUNT - 1;
    Timed t(s, NS_T_DEFECT, 0, 40LL * N);
    HCK(s, launch_defect(s->stream, I.g, S.p[S.pcur], I.e[fb], S.p[S.pcur ^ 1], (const float*)I.rhs, I.r,
                         I.ctl, I.part, I.prm.eta));
    S.pcur ^= 1;
  }
  *sweeps = used;
  return NS_OK;
}

// ---- one step ------------------------------------------------------------------
// Stages before the Poisson solve: dt, boundary fill, predictor, rhs.
template <class T>
ns_status step_pre(ns_solver* s, int idx, State& S, bool new_dt = true) {
  Inst& I = s->in[idx];
  const Geo& g = I.g;
  const ns_params& p = I.prm;
  T* u = (T*)S.u;
  T* v = (T*)S.v;
  T* w = (T*)S.w;
  if (p.dt <= 0 && new_dt) {
    Timed t(s, NS_T_OTHER);
    HCK(s, launch_umax<T>(s->stream, g, u, v, w, I.ctl, I.part, p.re, p.tau, p.wall_vel));
  }
  {
    Timed t(s, NS_T_BC);
    HCK(s, launch_bc_vel<T>(s->stream, g, u, v, w, p.wall_vel));
  }
  {
    Timed t(s, NS_T_FGH);
    // the conservative predictor is the kernel generated from its descriptor
    // (streamed through z with the velocity in an LDS plane ring)
    if (p.flags & NS_ADVECTIVE)
      HCK(s, launch_fgh_advective<T>(s->stream, g, u, v, w, (const T*)I.frc[0], (const T*)I.frc[1],
                                     (const T*)I.frc[2], (T*)I.F, (T*)I.G, (T*)I.H, I.ctl, p.re, p.gamma, p.g));
    else
      HCK(s, launch_gen_fgh<T>(s->stream, g, u, v, w, (const T*)I.frc[0], (const T*)I.frc[1], (const T*)I.frc[2],
                               (T*)I.F, (T*)I.G, (T*)I.H, I.ctl, p.re, p.gamma, p.g));
  }
  {
    Timed t(s, NS_T_RHS);
    HCK(s, launch_rhs<T>(s->stream, g, (const T*)I.F, (const T*)I.G, (const T*)I.H, (T*)I.rhs, I.ctl, I.part,
                         p.tol, 0.0));
  }
  return NS_OK;
}

// The step's statistics from the last polled control block (and the
// non-finite check of the solve).
ns_status step_account(ns_solver* s, int idx, int sweeps, int outer, bool account) {
  Inst& I = s->in[idx];
  const Ctl h = s->hctl[idx];
  if (h.nonfinite) return fail(s, NS_E_NONFINITE, "non-finite residual in the pressure solve");
  if (account) {
    ns_stats& st = I.st;
    st.t += h.dt;
    st.dt_last = h.dt;
    st.res_last = h.res;
    st.sweeps_total += sweeps;
    st.sweeps_max = std::max(st.sweeps_max, sweeps);
    st.outer_max = std::max(st.outer_max, outer);
    if (h.res > h.thr) st.steps_unconverged++;
    st.steps++;
  }
  return NS_OK;
}

// Stages after the solve: pressure ghosts, projection, boundary fill; then
// the statistics from the last polled control block.
template <class T>
ns_status step_post(ns_solver* s, int idx, State& S, int sweeps, int outer, bool account) {
  Inst& I = s->in[idx];
  const Geo& g = I.g;
  const ns_params& p = I.prm;
  T* u = (T*)S.u;
  T* v = (T*)S.v;
  T* w = (T*)S.w;
  {
    Timed t(s, NS_T_PROJECT);
    HCK(s, launch_p_ghosts<double>(s->stream, g, S.p[S.pcur]));
    if (p.flags & NS_GENERATED)
      HCK(s, launch_gen_project<T>(s->stream, g, (const T*)I.F, (const T*)I.G, (const T*)I.H, S.p[S.pcur], u, v,
                                   w, I.ctl));
    else
      HCK(s, launch_project<T>(s->stream, g, (const T*)I.F, (const T*)I.G, (const T*)I.H, S.p[S.pcur], u, v, w,
                               I.ctl, 0.0));
  }
  {
    Timed t(s, NS_T_BC);
    HCK(s, launch_bc_vel<T>(s->stream, g, u, v, w, p.wall_vel));
  }
  return step_account(s, idx, sweeps, outer, account);
}

// Two-stage SSP Runge-Kutta (Heun) step of a single-domain handle: u^n
// saved, two projected Euler stages with the step size of the first (the
// second skips the adaptive rule), u^{n+1} = (u^n + u^(2)) / 2 on every
// entry, boundary fill.  A step's sweeps are both solves'; it counts as
// unconverged when either solve stopped above its threshold; the residual
// and pressure are the second stage's.
template <class T>
ns_status step_rk2(ns_solver* s, int idx, State& S, bool account) {
  Inst& I = s->in[idx];
  {
    Timed t(s, NS_T_OTHER);
    HCK(s, hipMemcpyAsync(I.save[0], S.u, I.bytes, hipMemcpyDeviceToDevice, s->stream));
    HCK(s, hipMemcpyAsync(I.save[1], S.v, I.bytes, hipMemcpyDeviceToDevice, s->stream));
    HCK(s, hipMemcpyAsync(I.save[2], S.w, I.bytes, hipMemcpyDeviceToDevice, s->stream));
  }
  int sweeps = 0, outer = 0;
  bool unconv = false;
  for (int stage = 0; stage < 2; stage++) {
    ns_status e = step_pre<T>(s, idx, S, stage == 0);
    if (e != NS_OK) return e;
    int sw = 0, ou = 0;
    e = I.mixed ? solve_mixed(s, idx, &sw, &ou) : solve_fp64(s, idx, S.p, &S.pcur, &sw);
    if (e != NS_OK) return e;
    e = step_post<T>(s, idx, S, sw, ou, false);
    if (e != NS_OK) return e;
    sweeps += sw;
    outer = std::max(outer, ou);
    unconv |= s->hctl[idx].res > s->hctl[idx].thr;
    if (s->timing) {
      HCK(s, hipStreamSynchronize(s->stream));
      harvest(s, I.mixed ? 1 << 30 : sw + 1);
    }
  }
  {
    Timed t(s, NS_T_OTHER);
    HCK(s, launch_average<T>(s->stream, I.g, (const T*)I.save[0], (const T*)I.save[1], (const T*)I.save[2],
                             (T*)S.u, (T*)S.v, (T*)S.w));
  }
  {
    Timed t(s, NS_T_BC);
    HCK(s, launch_bc_vel<T>(s->stream, I.g, (T*)S.u, (T*)S.v, (T*)S.w, I.prm.wall_vel));
  }
  if (s->timing) {
    HCK(s, hipStreamSynchronize(s->stream));
    harvest(s, 1 << 30);
  }
  if (account) {
    const Ctl h = s->hctl[idx];
    ns_stats& st = I.st;
    st.t += h.dt;
    st.dt_last = h.dt;
    st.res_last = h.res;
    st.sweeps_total += sweeps;
    st.sweeps_max = std::max(st.sweeps_max, sweeps);
    st.outer_max = std::max(st.outer_max, outer);
    if (unconv) st.steps_unconverged++;
    st.steps++;
  }
  return NS_OK;
}

template <class T>
ns_status step_inst(ns_solver* s, int idx, State& S, bool account) {
  Inst& I = s->in[idx];
  if (I.prm.flags & NS_RK2) return step_rk2<T>(s, idx, S, account);
  ns_status e = step_pre<T>(s, idx, S);
  if (e != NS_OK) return e;
  int sweeps = 0, outer = 0;
  e = I.mixed ? solve_mixed(s, idx, &sweeps, &outer) : solve_fp64(s, idx, S.p, &S.pcur, &sweeps);
  if (e != NS_OK) return e;
  e = step_post<T>(s, idx, S, sweeps, outer, account);
  if (s->timing) {
    HCK(s, hipStreamSynchronize(s->stream));
    harvest(s, I.mixed ? 1 << 30 : sweeps + 1);
  }
  return e;
}

// Runs f(i) for the domains i of `ids` with the work of the q-th on library
// stream q % kAux, ordered after everything queued so far on the handle's
// stream, which then waits for all of it.  keep_going: run every domain and
// return the first error, else stop at the first error.
template <class F>
ns_status fan_out(ns_solver* s, const std::vector<int>& ids, bool keep_going, F&& f) {
  ns_status ret = NS_OK;
  if (!s->aux[0]) {
    for (int i : ids) {
      const ns_status e = f(i);
      if (e != NS_OK && ret == NS_OK) ret = e;
      if (ret != NS_OK && !keep_going) return ret;
    }
    return ret;
  }
  hipStream_t main = s->stream;
  HCK(s, hipEventRecord(s->ev_fork, main));
  for (int k = 0; k < ns_solver::kAux; k++) HCK(s, hipStreamWaitEvent(s->aux[k], s->ev_fork, 0));
  for (size_t q = 0; q < ids.size(); q++) {
    s->stream = s->aux[q % ns_solver::kAux];
    const ns_status e = f(ids[q]);
    if (e != NS_OK && ret == NS_OK) ret = e;
    if (ret != NS_OK && !keep_going) break;
  }
  s->stream = main;
  for (int k = 0; k < ns_solver::kAux; k++) {
    HCK(s, hipEventRecord(s->ev_join[k], s->aux[k]));
    HCK(s, hipStreamWaitEvent(main, s->ev_join[k], 0));
  }
  return ret;
}

std::vector<int> all_ids(int n) {
  std::vector<int> v(n);
  for (int i = 0; i < n; i++) v[i] = i;
  return v;
}

// One launch of cell stage `kind` over the domains `ids` (the same
// workgroup grid per domain as its single-domain launch); fill(i, item)
// sets domain i's stage arguments.
template <class T, class Fill>
ns_status stage_batched(ns_solver* s, int kind, const std::vector<int>& ids, Fill&& fill) {
  const int n = (int)ids.size();
  if (n == 0) return NS_OK;
  StageItem* h = s->stage_h + (size_t)kind * s->in.size();
  StageItem* d = s->stage_d + (size_t)kind * s->in.size();
  int nb = 0;
  for (int q = 0; q < n; q++) {
    StageItem& it = h[q];
    it = StageItem{};
    it.g = s->in[ids[q]].g;
    stage_item_grid(it, stage_reduces(kind));
    it.first = nb;
    nb += it.gx * it.gy * it.gz;
    fill(ids[q], it);
  }
  HCK(s, hipMemcpyAsync(d, h, sizeof(StageItem) * n, hipMemcpyHostToDevice, s->stream));
  HCK(s, launch_stage_batched<T>(s->stream, kind, d, n, nb));
  return NS_OK;
}

// Largest wall speed per velocity component (the adaptive step's bound).
void wall_speed_max(const ns_params& p, double wm[3]) {
  for (int c = 0; c < 3; c++) wm[c] = 0.0;
  for (int f = 0; f < 6; f++)
    for (int c = 0; c < 3; c++) wm[c] = std::max(wm[c], std::fabs(p.wall_vel[f][c]));
}

// ---- batched solves ------------------------------------------------------------
// Every domain of the handle is swept by one launch per sweep
// (launch_sor_batched); each domain keeps its own stop rule, budget and done
// flag, and the host reads all control blocks with one copy per chunk.
ns_status poll_all(ns_solver* s) {
  HCK(s, hipMemcpyAsync(s->hctl, s->ctl_all, sizeof(Ctl) * s->in.size(), hipMemcpyDeviceToHost, s->stream));
  HCK(s, hipStreamSynchronize(s->stream));
  return NS_OK;
}

// Batched solve with the two-sweep pass kernel: pass q (sweeps 2q + 1 and
// 2q + 2) of every domain in one launch until every domain is done.  A
// domain that stops on the iterate a pass held only in registers (odd
// final) is swept again from that pass's input (forced one-sweep launch,
// the same arithmetic); the accepted iterate f of a domain then sits in
// buffer (cur + ceil(f / 2)) & 1.
template <class T>
ns_status run_batched_pass(ns_solver* s, int n, int max_budget, int pred, int zero_first, long long bpc,
                           const std::vector<int>& idx_of_item, std::vector<int>& fbuf) {
  const int rows = s->batch_ty;
  int nblocks = 0;
  long long cells = 0;
  for (int q = 0; q < n; q++) {
    const BatchItem& it = s->items_h[q];
    nblocks += it.ntiles;
    cells += (long long)it.g.nx * it.g.ny * it.g.nz;
  }
  HCK(s, hipMemcpyAsync(s->items_d, s->items_h, sizeof(BatchItem) * n, hipMemcpyHostToDevice, s->stream));
  const size_t rec0 = s->recs.size();
  int m = 0;  // sweeps launched
  bool first = true;
  for (;;) {
    const int chunk = first ? std::min(std::max(pred + 2, 4), max_budget + 2) : std::max(4, pred / 4);
    first = false;
    for (int c = 0; c < chunk && m < max_budget + 1; c += 2) {
      Timed t(s, NS_T_SOR, 2000000 + m + 1, bpc * cells);
      HCK(s, launch_pass_batched<T>(s->stream, s->items_d, n, nblocks, rows, m + 1, m / 2, 2, zero_first && m == 0,
                                    0));
      m += 2;
    }
    ns_status e = poll_all(s);
    if (e != NS_OK) return e;
    bool all = true;
    for (int q = 0; q < n; q++) all &= s->hctl[idx_of_item[q]].done != 0;
    if (all) break;
    if (m >= max_budget + 1) return fail(s, NS_E_DEVICE, "batched solve ended without a decision");
  }
  for (size_t q = rec0; q < s->recs.size(); q++) {
    EvRec& rc = s->recs[q];
    if (rc.stage != NS_T_SOR || rc.m < 2000000) continue;
    const int mm = rc.m - 2000000;
    long long by = 0;
    for (int it = 0; it < n; it++) {
      const BatchItem& bi = s->items_h[it];
      if (s->hctl[idx_of_item[it]].final_ + 1 >= mm) by += bpc * (long long)bi.g.nx * bi.g.ny * bi.g.nz;
    }
    if (by == 0) rc.stage = NS_T_COUNT - 1;
    else rc.bytes = by;
  }
  // re-sweep the iterates held only in registers: one forced launch per
  // kind of input (zero or stored)
  fbuf.resize(n);
  for (int zin = 0; zin < 2; zin++) {
    std::vector<BatchItem> fix;
    long long fcells = 0;
    int fblocks = 0;
    for (int q = 0; q < n; q++) {
      const int f = s->hctl[idx_of_item[q]].final_;
      const BatchItem& bi = s->items_h[q];
      fbuf[q] = (bi.cur + (f + 1) / 2) & 1;
      if (!(f & 1)) continue;
      const int pq = (f - 1) / 2;  // the pass that held iterate f
      if ((zero_first && pq == 0) != (zin == 1)) continue;
      BatchItem it = bi;
      it.cur = (bi.cur + pq) & 1;
      pass_item_shape(it, rows, s->batch_zc, 1);
      it.first = fblocks;
      fblocks += it.ntiles;
      fcells += (long long)it.g.nx * it.g.ny * it.g.nz;
      fix.push_back(it);
    }
    if (fix.empty()) continue;
    if ((int)fix.size() > n) return fail(s, NS_E_DEVICE, "batch table overflow");
    // the launch reads its table before the copy below can overwrite it
    // (same stream), and the next use of items_d uploads a full table
    BatchItem* hbuf = s->items_h + n;
    std::copy(fix.begin(), fix.end(), hbuf);
    HCK(s, hipMemcpyAsync(s->items_d + n, hbuf, sizeof(BatchItem) * fix.size(), hipMemcpyHostToDevice, s->stream));
    Timed t(s, NS_T_SOR, 2000000, bpc * fcells);
    HCK(s, launch_pass_batched<T>(s->stream, s->items_d + n, (int)fix.size(), fblocks, rows, 1, 0, 1, zin, 1));
    HCK(s, hipStreamSynchronize(s->stream));
  }
  return NS_OK;
}

// Runs launches m = 1, 2, ... over the items in s->items_h[0..n) until every
// item is done; bpc = algorithmic bytes per cell of one sweep; fbuf[q]
// receives the buffer of item q's accepted iterate.
template <class T>
ns_status run_batched_sweeps(ns_solver* s, int n, int max_budget, int pred, int zero_first, long long bpc,
                             const std::vector<int>& idx_of_item, std::vector<int>& fbuf) {
  int nblocks = 0;
  long long cells = 0;
  for (int q = 0; q < n; q++) {
    const BatchItem& it = s->items_h[q];
    nblocks += it.ntiles;
    cells += (long long)it.g.nx * it.g.ny * it.g.nz;
  }
  HCK(s, hipMemcpyAsync(s->items_d, s->items_h, sizeof(BatchItem) * n, hipMemcpyHostToDevice, s->stream));
  const size_t rec0 = s->recs.size();
  int m = 0;
  bool first = true;
  for (;;) {
    const int chunk = first ? std::min(std::max(pred + 2, 4), max_budget + 1) : std::max(4, pred / 4);
    first = false;
    for (int c = 0; c < chunk && m < max_budget + 1; c++) {
      m++;
      Timed t(s, NS_T_SOR, 2000000 + m, bpc * cells);
      HCK(s, launch_sor_batched<T>(s->stream, s->items_d, n, nblocks, s->batch_ty, m, 1,
                                   zero_first && m == 1));
    }
    ns_status e = poll_all(s);
    if (e != NS_OK) return e;
    bool all = true;
    for (int q = 0; q < n; q++) all &= s->hctl[idx_of_item[q]].done != 0;
    if (all) break;
    if (m >= max_budget + 1) return fail(s, NS_E_DEVICE, "batched solve ended without a decision");
  }
  // algorithmic bytes of each launch: the domains that still swept in it
  for (size_t q = rec0; q < s->recs.size(); q++) {
    EvRec& rc = s->recs[q];
    if (rc.stage != NS_T_SOR || rc.m < 2000000) continue;
    const int mm = rc.m - 2000000;
    long long by = 0;
    for (int it = 0; it < n; it++) {
      const BatchItem& bi = s->items_h[it];
      if (s->hctl[idx_of_item[it]].final_ + 1 >= mm) by += bpc * (long long)bi.g.nx * bi.g.ny * bi.g.nz;
    }
    if (by == 0) rc.stage = NS_T_COUNT - 1;  // every domain had returned on its flag
    else rc.bytes = by;
  }
  fbuf.resize(n);
  for (int q = 0; q < n; q++) fbuf[q] = (s->items_h[q].cur + s->hctl[idx_of_item[q]].final_) & 1;
  return NS_OK;
}

template <class T>
ns_status run_batched(ns_solver* s, int n, int max_budget, int pred, int zero_first, long long bpc,
                      const std::vector<int>& idx_of_item, std::vector<int>& fbuf) {
  const bool pass = s->batch_ty >= 16;
  if (pass)
    for (int q = 0; q < n; q++) pass_item_shape(s->items_h[q], s->batch_ty, s->batch_zc, 2);
  const std::vector<int> ord = order_longest_first(s->items_h, n);
  std::vector<int> idx(n), fb;
  for (int k = 0; k < n; k++) idx[k] = idx_of_item[ord[k]];
  const ns_status e = pass ? run_batched_pass<T>(s, n, max_budget, pred, zero_first, bpc, idx, fb)
                           : run_batched_sweeps<T>(s, n, max_budget, pred, zero_first, bpc, idx, fb);
  if (e != NS_OK) return e;
  fbuf.assign(n, 0);
  for (int k = 0; k < n; k++) fbuf[ord[k]] = fb[k];
  return NS_OK;
}

void fill_item(ns_solver* s, BatchItem& it, Inst& I, void* p0, void* p1, const void* rhs, int cur, int budget,
               int inner) {
  it.g = I.g;
  it.p[0] = p0;
  it.p[1] = p1;
  it.rhs = rhs;
  it.ctl = I.ctl;
  it.part = I.part;
  it.omega = I.prm.omega;
  it.cur = cur;
  it.budget = budget;
  it.inner = inner;
  batch_item_shape(it, s->batch_ty, s->batch_zc);
}

ns_status solve_batched_fp64(ns_solver* s, std::vector<int>& sweeps) {
  const int n = (int)s->in.size();
  int max_budget = 0, pred = 0;
  std::vector<int> ids(n);
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    fill_item(s, s->items_h[i], I, I.s.p[0], I.s.p[1], I.rhs, I.s.pcur, I.prm.itermax, 0);
    max_budget = std::max(max_budget, I.prm.itermax);
    pred = std::max(pred, I.pred);
    ids[i] = i;
  }
  std::vector<int> fbuf;
  ns_status e = run_batched<double>(s, n, max_budget, pred, 0, 24, ids, fbuf);
  if (e != NS_OK) return e;
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    const int f = s->hctl[i].final_;
    sweeps[i] = f;
    I.s.pcur = fbuf[i];
    I.pred = f;
  }
  return NS_OK;
}

ns_status solve_batched_mixed(ns_solver* s, std::vector<int>& sweeps, std::vector<int>& outer) {
  const int n = (int)s->in.size();
  const long long big = 1;
  (void)big;
  for (int i = 0; i < n; i++) {
    sweeps[i] = 0;
    outer[i] = 0;
  }
  long long cells_all = 0;
  for (auto& I : s->in) cells_all += (long long)I.g.nx * I.g.ny * I.g.nz;
  ns_status e0;
  {
    Timed t(s, NS_T_DEFECT, 0, 20LL * cells_all);
    e0 = stage_batched<float>(s, kStageDefect, all_ids(n), [&](int i, StageItem& it) {
      Inst& I = s->in[i];
      it.in[0] = I.s.p[I.s.pcur];
      it.in[2] = I.rhs;
      it.out[1] = I.r;
      it.ctl = I.ctl;
      it.part = I.part;
      it.s[0] = I.prm.eta;
    });
  }
  if (e0 != NS_OK) return e0;
  for (;;) {
    ns_status e = poll_all(s);
    if (e != NS_OK) return e;
    std::vector<int> ids;
    int max_budget = 0, pred = 0;
    for (int i = 0; i < n; i++) {
      Inst& I = s->in[i];
      const Ctl& h = s->hctl[i];
      if (h.outer_done || h.nonfinite || sweeps[i] >= I.prm.itermax) continue;
      const int budget = I.prm.itermax - sweeps[i];
      fill_item(s, s->items_h[ids.size()], I, I.e[0], I.e[1], I.r, 0, budget, 1);
      ids.push_back(i);
      outer[i]++;
      max_budget = std::max(max_budget, budget);
      pred = std::max(pred, I.pred);
    }
    if (ids.empty()) break;
    std::vector<int> fbuf;
    e = run_batched<float>(s, (int)ids.size(), max_budget, pred, 1, 12, ids, fbuf);
    if (e != NS_OK) return e;
    std::vector<int> fb_of(n, 0);
    for (int q = 0; q < (int)ids.size(); q++) fb_of[ids[q]] = fbuf[q];
    long long cells = 0;
    for (int i : ids) {
      Inst& I = s->in[i];
      const int f = s->hctl[i].final_;
      sweeps[i] += f;
      I.pred = f;
      cells += (long long)I.g.nx * I.g.ny * I.g.nz;
    }
    {
      Timed t(s, NS_T_DEFECT, 0, 40LL * cells);
      e = stage_batched<float>(s, kStageDefect, ids, [&](int i, StageItem& it) {
        Inst& I = s->in[i];
        it.in[0] = I.s.p[I.s.pcur];
        it.in[1] = I.e[fb_of[i]];
        it.in[2] = I.rhs;
        it.out[0] = I.s.p[I.s.pcur ^ 1];
        it.out[1] = I.r;
        it.ctl = I.ctl;
        it.part = I.part;
        it.s[0] = I.prm.eta;
      });
    }
    if (e != NS_OK) return e;
    for (int i : ids) s->in[i].s.pcur ^= 1;
  }
  return NS_OK;
}

template <class T>
ns_status step_batched(ns_solver* s) {
  const int n = (int)s->in.size();
  const std::vector<int> ids = all_ids(n);
  std::vector<int> adapt;
  for (int i = 0; i < n; i++)
    if (s->in[i].prm.dt <= 0) adapt.push_back(i);
  // The cell stages take one launch each for every domain (same arithmetic
  // as the single-domain step); the face launches of the boundary fill go
  // per domain to the library streams.
  auto bc_fill = [&](int i) {
    Inst& I = s->in[i];
    Timed t(s, NS_T_BC);
    HCK(s, launch_bc_vel<T>(s->stream, I.g, (T*)I.s.u, (T*)I.s.v, (T*)I.s.w, I.prm.wall_vel));
    return NS_OK;
  };
  ns_status e = NS_OK;
  if (!adapt.empty()) {
    Timed t(s, NS_T_OTHER);
    e = stage_batched<T>(s, kStageUmax, adapt, [&](int i, StageItem& it) {
      Inst& I = s->in[i];
      double wm[3];
      wall_speed_max(I.prm, wm);
      it.in[0] = I.s.u;
      it.in[1] = I.s.v;
      it.in[2] = I.s.w;
      it.ctl = I.ctl;
      it.part = I.part;
      it.s[0] = I.prm.re;
      it.s[1] = I.prm.tau;
      for (int c = 0; c < 3; c++) it.s[2 + c] = wm[c];
    });
    if (e != NS_OK) return e;
  }
  e = fan_out(s, ids, false, bc_fill);
  if (e != NS_OK) return e;
  {
    Timed t(s, NS_T_FGH);
    e = stage_batched<T>(s, kStageFgh, ids, [&](int i, StageItem& it) {
      Inst& I = s->in[i];
      it.in[0] = I.s.u;
      it.in[1] = I.s.v;
      it.in[2] = I.s.w;
      for (int c = 0; c < 3; c++) it.in[3 + c] = I.frc[c];
      it.out[0] = I.F;
      it.out[1] = I.G;
      it.out[2] = I.H;
      it.ctl = I.ctl;
      it.s[0] = 1.0 / I.prm.re;
      it.s[1] = I.prm.gamma;
      for (int c = 0; c < 3; c++) it.s[2 + c] = I.prm.g[c];
    });
    if (e != NS_OK) return e;
  }
  {
    Timed t(s, NS_T_RHS);
    e = stage_batched<T>(s, kStageRhs, ids, [&](int i, StageItem& it) {
      Inst& I = s->in[i];
      it.in[0] = I.F;
      it.in[1] = I.G;
      it.in[2] = I.H;
      it.out[0] = I.rhs;
      it.ctl = I.ctl;
      it.part = I.part;
      it.s[0] = I.prm.tol;
    });
    if (e != NS_OK) return e;
  }
  std::vector<int> sweeps(n, 0), outer(n, 0);
  e = s->in[0].mixed ? solve_batched_mixed(s, sweeps, outer) : solve_batched_fp64(s, sweeps);
  if (e != NS_OK) return e;
  ns_status ret = fan_out(s, ids, true, [&](int i) {
    Inst& I = s->in[i];
    Timed t(s, NS_T_PROJECT);
    HCK(s, launch_p_ghosts<double>(s->stream, I.g, I.s.p[I.s.pcur]));
    return NS_OK;
  });
  if (ret == NS_OK) {
    Timed t(s, NS_T_PROJECT);
    ret = stage_batched<T>(s, kStageProject, ids, [&](int i, StageItem& it) {
      Inst& I = s->in[i];
      it.in[0] = I.F;
      it.in[1] = I.G;
      it.in[2] = I.H;
      it.in[3] = I.s.p[I.s.pcur];
      it.out[0] = I.s.u;
      it.out[1] = I.s.v;
      it.out[2] = I.s.w;
      it.ctl = I.ctl;
    });
  }
  if (ret == NS_OK) ret = fan_out(s, ids, true, bc_fill);
  for (int i : ids) {
    const ns_status a = step_account(s, i, sweeps[i], outer[i], true);
    if (a != NS_OK && ret == NS_OK) ret = a;
  }
  if (s->timing) {
    HCK(s, hipStreamSynchronize(s->stream));
    harvest(s, 1 << 30);
  }
  return ret;
}

// ---- persistent batched launch ---------------------------------------------------
// Plane-steps the busiest workgroup of a team of `team` spends on one pass
// over a domain (two-sweep tiles of `rows` rows, each workgroup an equal
// share of the (plane-column, plane) space cut at column ends, as the
// kernel splits it): a z range of planes z0..z1 costs z1 - z0 + 7 steps
// (the pipeline runs 2 planes before and 4 after it).  A step's time is
// about the same for every tile, so this is the team's time per pass.
long pass_steps(const Geo& g, int team, int rows) {
  const int ntx = (g.nx + 55) / 56, nty = (g.ny + rows - 9) / (rows - 8);
  const long ptot = (long)ntx * nty * g.nz;
  long worst = 0;
  for (int r = 0; r < team; r++) {
    long q0 = ptot * r / team, st = 0;
    const long q1 = ptot * (r + 1) / team;
    while (q0 < q1) {
      const long col = q0 / g.nz;
      const long z0 = q0 - col * g.nz + 1;
      const long z1 = std::min((long)g.nz, z0 + (q1 - q0) - 1);
      st += z1 - z0 + 7;
      q0 += z1 - z0 + 1;
    }
    worst = std::max(worst, st);
  }
  return worst;
}

// Teams: the co-resident workgroups of the launch are split among the
// domains.  Workgroup b runs on XCD b mod 8; the domains are dealt to the
// XCDs longest-processing-time first by their pass work (tile columns x
// planes), and the workgroups of an XCD are handed out one at a time to the
// domain whose team currently has the longest pass (pass_steps), so a
// domain's team sits on one XCD (one L2) and the teams finish a pass at
// about the same time.  Returns false when some XCD would get more domains
// than workgroups.
bool persist_teams(const std::vector<Geo>& geo, int G, int rows, std::vector<PSlot>& slots,
                   std::vector<int>& team) {
  const int n = (int)geo.size();
  slots.assign(G, PSlot{-1, 0});
  team.assign(n, 0);
  int gx[8];
  for (int x = 0; x < 8; x++) gx[x] = G / 8 + (x < G % 8 ? 1 : 0);
  std::vector<long long> work(n);
  for (int d = 0; d < n; d++)
    work[d] = (long long)((geo[d].nx + 55) / 56) * ((geo[d].ny + rows - 9) / (rows - 8)) * geo[d].nz;
  std::vector<int> ord(n);
  for (int i = 0; i < n; i++) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work[a] > work[b]; });
  long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int> on[8];
  for (int d : ord) {
    int best = -1;
    for (int x = 0; x < 8; x++)
      if ((int)on[x].size() < gx[x] && (best < 0 || load[x] < load[best])) best = x;
    if (best < 0) return false;
    on[best].push_back(d);
    load[best] += work[d];
  }
  for (int x = 0; x < 8; x++) {
    if (on[x].empty()) continue;
    std::vector<long> cost(on[x].size());
    for (size_t q = 0; q < on[x].size(); q++) {
      team[on[x][q]] = 1;
      cost[q] = pass_steps(geo[on[x][q]], 1, rows);
    }
    for (int k = (int)on[x].size(); k < gx[x]; k++) {
      size_t q = 0;
      for (size_t c = 1; c < cost.size(); c++)
        if (cost[c] > cost[q]) q = c;
      const int d = on[x][q];
      team[d]++;
      cost[q] = pass_steps(geo[d], team[d], rows);
    }
    int slot = 0;
    for (int d : on[x])
      for (int r = 0; r < team[d]; r++, slot++) slots[x + 8 * slot] = PSlot{d, r};
  }
  return true;
}

// Sweeps per pass of a domain in the persistent launch: two (the pass
// tile's temporal blocking).  One-sweep tiles recompute less halo (60 of 64
// lanes, 12 of 16 rows against 56 and 8) but need twice the passes and
// team barriers; on the 64-cavity workload they measured slower (699
// against 748 Mcell-steps/s), as did a per-domain choice by tile cost.
int persist_sweeps_per_pass(const Geo&) { return 2; }

// Sets up the persistent launch of a batched handle; leaves s->persist
// false (and allocates nothing) when the handle does not qualify.
ns_status persist_setup(ns_solver* s) {
  const int n = (int)s->in.size();
  const bool f32 = s->in[0].mixed;
  if (s->in[0].prm.flags & NS_BATCH_LAUNCHES) return NS_OK;
  for (auto& I : s->in)
    if (I.prm.tile[0] != 0 || I.prm.checkpoint_every > 0 || !pass_grid_ok(I.g, I.esz)) return NS_OK;
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, s->device) != hipSuccess || !coop)
    return NS_OK;
  const int G = persistent_resident(f32);
  if (G < n) return NS_OK;
  std::vector<Geo> geo(n);
  for (int i = 0; i < n; i++) geo[i] = s->in[i].g;
  std::vector<PSlot> slots;
  std::vector<int> team;
  if (!persist_teams(geo, G, persist_rows(f32), slots, team)) return NS_OK;
  int rate = 0;
  HCK(s, hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, s->device));
  s->clock_khz = rate > 0 ? (double)rate : 100000.0;
  // a barrier wait longer than this gives up (a test lowers it to force
  // the give-up path); default 30 s
  double limit_us = 30e6;
  if (const char* e = getenv("NS_TEAM_WAIT_LIMIT_US")) limit_us = atof(e);
  s->persist_limit = (long long)(limit_us * s->clock_khz / 1000.0);
  // partial sums: two halves of 3 per team workgroup (the time step's three
  // maxima)
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    const size_t need = 6 * (size_t)team[i] + 8;
    if (need > reduce_blocks(I.g)) {
      dfree(I.part);
      I.part = nullptr;
      HCK(s, dmalloc((void**)&I.part, need * sizeof(double)));
    }
  }
  HCK(s, hipHostMalloc((void**)&s->pitems_h, sizeof(PItem) * n, hipHostMallocDefault));
  HCK(s, hipHostMalloc((void**)&s->pstats_h, sizeof(PStats) * n, hipHostMallocDefault));
  HCK(s, hipHostMalloc((void**)&s->perr_h, sizeof(int), hipHostMallocDefault));
  HCK(s, dmalloc((void**)&s->pitems_d, sizeof(PItem) * n));
  HCK(s, dmalloc((void**)&s->pstats_d, sizeof(PStats) * n));
  HCK(s, dmalloc((void**)&s->pslots_d, sizeof(PSlot) * G));
  HCK(s, dmalloc((void**)&s->pbar_d, sizeof(unsigned) * n));
  HCK(s, dmalloc((void**)&s->perr_d, sizeof(int)));
  HCK(s, hipMemcpy(s->pslots_d, slots.data(), sizeof(PSlot) * G, hipMemcpyHostToDevice));
  for (int i = 0; i < n; i++) {
    PItem& it = s->pitems_h[i];
    it = PItem{};
    it.team = team[i];
  }
  s->persist_blocks = G;
  s->persist = true;
  return NS_OK;
}

// nsteps steps of every domain in one launch.
// Persistent launches on one device take turns (held from the first copy to
// the final synchronisation): each grid fills every compute unit, and two
// grids dispatched side by side by handles on different streams could each
// hold part of the device while their team barriers wait for workgroups that
// only the other grid's exit would let in -- until the wait limit failed both.
std::mutex& persist_device_mutex(int device) {
  static std::mutex mu[64];
  return mu[device & 63];
}

ns_status persist_run(ns_solver* s, int nsteps) {
  std::lock_guard<std::mutex> turn(persist_device_mutex(s->device));
  const int n = (int)s->in.size();
  const bool f32 = s->in[0].mixed;
  std::vector<long long> sweeps0(n);
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    PItem& it = s->pitems_h[i];
    const int team = it.team;
    it = PItem{};
    it.team = team;
    it.g = I.g;
    it.u = I.s.u;
    it.v = I.s.v;
    it.w = I.s.w;
    it.F = I.F;
    it.G = I.G;
    it.H = I.H;
    it.rhs = I.rhs;
    for (int c = 0; c < 3; c++) it.frc[c] = I.frc[c];
    it.p[0] = I.s.p[0];
    it.p[1] = I.s.p[1];
    it.e[0] = I.e[0];
    it.e[1] = I.e[1];
    it.r = I.r;
    it.part = I.part;
    it.ctl = I.ctl;
    it.st = s->pstats_d + i;
    it.bar = s->pbar_d + i;
    for (int f = 0; f < 6; f++)
      for (int c = 0; c < 3; c++) it.wall[f][c] = I.prm.wall_vel[f][c];
    wall_speed_max(I.prm, it.wmax);
    for (int c = 0; c < 3; c++) it.gforce[c] = I.prm.g[c];
    it.re = I.prm.re;
    it.tau = I.prm.tau;
    it.gamma = I.prm.gamma;
    it.omega = I.prm.omega;
    it.tol = I.prm.tol;
    it.eta = I.prm.eta;
    it.adaptive = I.prm.dt <= 0;
    it.itermax = I.prm.itermax;
    it.ns_max = persist_sweeps_per_pass(I.g);
    it.cgx = (I.g.nx + kCellX - 1) / kCellX;
    it.cgy = (I.g.ny + persist_waves(f32) - 1) / persist_waves(f32);
    it.cgz = (I.g.nz + kPersistZr - 1) / kPersistZr;
    PStats& ps = s->pstats_h[i];
    ps = PStats{};
    ps.t = I.st.t;
    ps.dt_last = I.st.dt_last;
    ps.res_last = I.st.res_last;
    ps.sweeps_total = I.st.sweeps_total;
    ps.steps = I.st.steps;
    ps.sweeps_max = I.st.sweeps_max;
    ps.steps_unconverged = I.st.steps_unconverged;
    ps.outer_max = I.st.outer_max;
    ps.pcur = I.s.pcur;
    sweeps0[i] = I.st.sweeps_total;
  }
  HCK(s, hipMemcpyAsync(s->pitems_d, s->pitems_h, sizeof(PItem) * n, hipMemcpyHostToDevice, s->stream));
  HCK(s, hipMemcpyAsync(s->pstats_d, s->pstats_h, sizeof(PStats) * n, hipMemcpyHostToDevice, s->stream));
  HCK(s, hipMemsetAsync(s->pbar_d, 0, sizeof(unsigned) * n, s->stream));
  HCK(s, hipMemsetAsync(s->perr_d, 0, sizeof(int), s->stream));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (s->timing) {
    HCK(s, hipEventCreate(&ea));
    HCK(s, hipEventCreate(&eb));
    HCK(s, hipEventRecord(ea, s->stream));
  }
  HCK(s, launch_persistent(s->stream, f32, s->pitems_d, s->pslots_d, s->persist_blocks, nsteps, s->perr_d,
                           s->persist_limit));
  if (s->timing) HCK(s, hipEventRecord(eb, s->stream));
  HCK(s, hipMemcpyAsync(s->pstats_h, s->pstats_d, sizeof(PStats) * n, hipMemcpyDeviceToHost, s->stream));
  HCK(s, hipMemcpyAsync(s->perr_h, s->perr_d, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HCK(s, hipStreamSynchronize(s->stream));
  bool nonfinite = false;
  double sweep_ms = 0.0;
  long long sweep_bytes = 0;
  for (int i = 0; i < n; i++) {
    Inst& I = s->in[i];
    const PStats& ps = s->pstats_h[i];
    I.st.t = ps.t;
    I.st.dt_last = ps.dt_last;
    I.st.res_last = ps.res_last;
    I.st.sweeps_total = ps.sweeps_total;
    I.st.steps = ps.steps;
    I.st.sweeps_max = ps.sweeps_max;
    I.st.steps_unconverged = ps.steps_unconverged;
    I.st.outer_max = ps.outer_max;
    I.s.pcur = ps.pcur;
    nonfinite |= ps.nonfinite != 0;
    sweep_ms = std::max(sweep_ms, ps.sweep_ticks / s->clock_khz);
    sweep_bytes += (long long)(f32 ? 12 : 24) * I.g.nx * I.g.ny * I.g.nz * (ps.sweeps_total - sweeps0[i]);
  }
  if (s->timing) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ea, eb) == hipSuccess) {
      s->tm.ms[NS_T_SOR] += std::min((double)ms, sweep_ms);
      s->tm.ms[NS_T_OTHER] += std::max(0.0, (double)ms - sweep_ms);
      s->tm.launches[NS_T_SOR] += 1;
      s->tm.sor_bytes += sweep_bytes;
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
  }
  if (*s->perr_h) return fail(s, NS_E_DEVICE, "persistent batch: a team barrier wait exceeded its time limit");
  if (nonfinite) return fail(s, NS_E_NONFINITE, "non-finite residual in the pressure solve");
  return NS_OK;
}

ns_status copy_in(ns_solver* s, Inst& I, void* dst, bool dst_f32, const double* src, int on_device) {
  const long n = I.g.ntot;
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (!dst_f32) {
    HCK(s, hipMemcpyAsync(dst, src, n * sizeof(double), kind, s->stream));
  } else {
    const double* from = src;
    if (!on_device) {
      HCK(s, hipMemcpyAsync(s->stage, src, n * sizeof(double), kind, s->stream));
      from = s->stage;
    }
    k_to_f32<<<conv_grid(n), 256, 0, s->stream>>>(from, (float*)dst, n);
    HCK(s, hipGetLastError());
  }
  HCK(s, hipStreamSynchronize(s->stream));
  return NS_OK;
}

ns_status copy_out(ns_solver* s, const Inst& I, const void* src, bool src_f32, double* dst, int on_device) {
  const long n = I.g.ntot;
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (!src_f32) {
    HCK(s, hipMemcpyAsync(dst, src, n * sizeof(double), kind, s->stream));
  } else {
    double* to = on_device ? dst : s->stage;
    k_to_f64<<<conv_grid(n), 256, 0, s->stream>>>((const float*)src, to, n);
    HCK(s, hipGetLastError());
    if (!on_device) HCK(s, hipMemcpyAsync(dst, s->stage, n * sizeof(double), kind, s->stream));
  }
  HCK(s, hipStreamSynchronize(s->stream));
  return NS_OK;
}

ns_status save_state(ns_solver* s, Inst& I, const State& from, State& to) {
  HCK(s, hipMemcpyAsync(to.u, from.u, I.bytes, hipMemcpyDeviceToDevice, s->stream));
  HCK(s, hipMemcpyAsync(to.v, from.v, I.bytes, hipMemcpyDeviceToDevice, s->stream));
  HCK(s, hipMemcpyAsync(to.w, from.w, I.bytes, hipMemcpyDeviceToDevice, s->stream));
  HCK(s, hipMemcpyAsync(to.p[0], from.p[from.pcur], I.pbytes, hipMemcpyDeviceToDevice, s->stream));
  to.pcur = 0;
  return NS_OK;
}

// ---- allocation-free step -------------------------------------------------------
// ns_step_noalloc keeps everything beyond the caller's fields in one static
// device array: the predictor fields F, G, H, the right-hand side and the
// second pressure buffer (kNaEntries FP64 entries each, padded layout), the
// partial sums of the reductions and one control block.  Each device the
// library runs on holds its own copy until the process ends.
constexpr long kNaEntries = 1L << 19;  // padded entries (nx+2)(ny+2)(nz+2) per field
constexpr long kNaPartials = 1L << 16;
constexpr long kNaCtl = (long)(sizeof(Ctl) / sizeof(double));
constexpr long kNaDoubles = 5 * kNaEntries + kNaPartials + kNaCtl;
static_assert(sizeof(Ctl) % sizeof(double) == 0, "control block is a whole number of doubles");
static __device__ __align__(256) double scratch[kNaDoubles];

// Host side, per device: the device address of `scratch` (from
// hipGetSymbolAddress; the array's name is only a host stand-in), a solver
// shell whose single instance is pointed at the caller's fields and the
// scratch on every call, and the lock that keeps calls on one device from
// overlapping.
struct NaDevice {
  bool ready = false;
  double* ptr = nullptr;
  ns_solver* shell = nullptr;
  Ctl hctl{};
  std::mutex mu;
};
constexpr int kNaMaxDevices = 64;
NaDevice g_na[kNaMaxDevices];
std::mutex g_na_setup_mu;

// Clears the scratch fields and partial sums (the state a freshly created
// handle starts from) and writes the control block's initial dt.
__global__ void k_na_init(double* __restrict__ q, long n, Ctl* __restrict__ ctl, double dt) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) q[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl c{};
    c.dt = dt;
    *ctl = c;
  }
}

ns_status na_setup(int dev, NaDevice** out) {
  std::lock_guard<std::mutex> lk(g_na_setup_mu);
  NaDevice& D = g_na[dev];
  if (!D.ready) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, NS_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    D.ptr = (double*)ptr;
    D.shell = new ns_solver();
    D.shell->in.resize(1);
    D.shell->launch_log.reserve(4096);
    D.shell->hctl = &D.hctl;
    D.shell->device = dev;
    D.ready = true;
  }
  *out = &D;
  return NS_OK;
}

// NS_OK when q points into device memory of device dev.
ns_status is_device_memory(const void* q, int dev) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, q) != hipSuccess) {
    (void)hipGetLastError();
    return NS_E_INVALID;
  }
  return a.type == hipMemoryTypeDevice && a.device == dev ? NS_OK : NS_E_INVALID;
}

}  // namespace

// ============================================================================
// C ABI

extern "C" {

ns_status ns_params_default(ns_params* p) {
  if (!p) return NS_E_INVALID;
  memset(p, 0, sizeof *p);
  p->struct_size = sizeof(ns_params);
  p->nx = p->ny = p->nz = 16;
  p->lx = p->ly = p->lz = 1.0;
  p->re = 100.0;
  p->dt = 0.01;
  p->tau = 0.5;
  p->gamma = 0.5;
  p->omega = 1.7;
  p->tol = 1e-6;
  p->itermax = 200;
  p->wall_vel[5][0] = 1.0;
  p->eta = 1e-2;
  p->precision = NS_FP64;
  return NS_OK;
}

ns_status ns_create(const ns_params* params, int32_t n_instances, void* hip_stream, ns_solver** out) {
  if (!out) return fail(nullptr, NS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!params || n_instances < 1) return fail(nullptr, NS_E_INVALID, "need params[n_instances], n_instances >= 1");
  for (int i = 0; i < n_instances; i++) {
    ns_status st = validate(params[i], i);
    if (st != NS_OK) return st;
    if ((params[i].flags & (NS_GENERATED | NS_ADVECTIVE | NS_RK2)) && n_instances > 1)
      return fail(nullptr, NS_E_INVALID, "NS_GENERATED, NS_ADVECTIVE and NS_RK2 need a handle of one instance");
  }
  ns_solver* s = new ns_solver();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(nullptr, NS_E_DEVICE, "no HIP device");
  }
  s->stream = (hipStream_t)hip_stream;
  s->in.resize(n_instances);
  s->timing = (params[0].flags & NS_TIMING) != 0;
  auto bail = [&](ns_status code, const std::string& m) {
    g_create_err = m;
    (void)hipGetLastError();  // the failure is reported here, not by a later call
    ns_destroy(s);
    return code;
  };
  if (hipHostMalloc((void**)&s->hctl, sizeof(Ctl) * n_instances, hipHostMallocDefault) != hipSuccess)
    return bail(NS_E_OOM, "pinned control block allocation failed");
  memset(s->hctl, 0, sizeof(Ctl) * n_instances);
  if (dmalloc((void**)&s->ctl_all, sizeof(Ctl) * n_instances) != hipSuccess)
    return bail(NS_E_OOM, "control block allocation failed");
  size_t max_ntot = 0;
  for (int i = 0; i < n_instances; i++) {
    Inst& I = s->in[i];
    I.prm = params[i];
    I.g = make_geo(I.prm);
    I.mixed = I.prm.precision == NS_MIXED;
    I.esz = I.mixed ? 4 : 8;
    I.bytes = (size_t)I.g.ntot * I.esz;
    I.pbytes = (size_t)I.g.ntot * 8;
    max_ntot = std::max(max_ntot, (size_t)I.g.ntot);
    hipError_t e = alloc_state(I.s, I);
    if (e == hipSuccess) e = dmalloc(&I.F, I.bytes);
    if (e == hipSuccess) e = dmalloc(&I.G, I.bytes);
    if (e == hipSuccess) e = dmalloc(&I.H, I.bytes);
    if (e == hipSuccess) e = dmalloc(&I.rhs, I.bytes);
    if (e == hipSuccess && I.mixed) {
      e = dmalloc((void**)&I.e[0], (size_t)I.g.ntot * 4);
      if (e == hipSuccess) e = dmalloc((void**)&I.e[1], (size_t)I.g.ntot * 4);
      if (e == hipSuccess) e = dmalloc((void**)&I.r, (size_t)I.g.ntot * 4);
    }
    if (e == hipSuccess) e = dmalloc((void**)&I.part, reduce_blocks(I.g) * sizeof(double));
    if (I.prm.flags & NS_RK2)
      for (int c = 0; c < 3 && e == hipSuccess; c++) e = dmalloc(&I.save[c], I.bytes);
    I.ctl = s->ctl_all + i;
    if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? NS_E_OOM : NS_E_DEVICE,
                                     std::string("allocation failed: ") + hipGetErrorString(e));
    Ctl c{};
    c.dt = I.prm.dt > 0 ? I.prm.dt : 0.0;
    if (hipMemcpy(I.ctl, &c, sizeof c, hipMemcpyHostToDevice) != hipSuccess)
      return bail(NS_E_DEVICE, "control block upload failed");
    I.rec_valid = I.prm.checkpoint_every > 0;
    I.shape = pick_shape(I.prm, I.g, I.esz);
  }
  // staging buffer for FP32 conversions of host data
  bool any_mixed = false;
  for (auto& I : s->in) any_mixed |= I.mixed;
  if (any_mixed) {
    if (dmalloc((void**)&s->stage, max_ntot * sizeof(double)) != hipSuccess)
      return bail(NS_E_OOM, "staging buffer allocation failed");
    s->stage_n = max_ntot;
  }
  for (int i = 0; i < n_instances; i++) {
    Inst& I = s->in[i];
    hipError_t e = I.mixed ? launch_bc_vel<float>(s->stream, I.g, (float*)I.s.u, (float*)I.s.v, (float*)I.s.w,
                                                  I.prm.wall_vel)
                           : launch_bc_vel<double>(s->stream, I.g, (double*)I.s.u, (double*)I.s.v,
                                                   (double*)I.s.w, I.prm.wall_vel);
    if (e != hipSuccess) return bail(NS_E_DEVICE, std::string("boundary fill failed: ") + hipGetErrorString(e));
  }
  if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(NS_E_DEVICE, "stream synchronisation failed");
  // several instances of one precision: one launch per sweep for all of them
  {
    bool same = n_instances > 1;
    // (the batched sweeps are fused or pass tiles: every plane within their offsets)
    for (auto& I : s->in) same &= I.mixed == s->in[0].mixed && I.prm.tile[0] >= 0 && fused_grid_ok(I.g, I.esz);
    s->batched = same;
  }
  if (s->batched) {
    for (int k = 0; k < ns_solver::kAux; k++)
      if (hipStreamCreateWithFlags(&s->aux[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&s->ev_join[k], hipEventDisableTiming) != hipSuccess)
        return bail(NS_E_DEVICE, "stream creation failed");
    if (hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess)
      return bail(NS_E_DEVICE, "event creation failed");
    // room for a full table and a table of re-sweeps behind it
    if (hipHostMalloc((void**)&s->items_h, 2 * sizeof(BatchItem) * n_instances, hipHostMallocDefault) !=
            hipSuccess ||
        dmalloc((void**)&s->items_d, 2 * sizeof(BatchItem) * n_instances) != hipSuccess ||
        hipHostMalloc((void**)&s->stage_h, sizeof(StageItem) * kStageKinds * n_instances, hipHostMallocDefault) !=
            hipSuccess ||
        dmalloc((void**)&s->stage_d, sizeof(StageItem) * kStageKinds * n_instances) != hipSuccess)
      return bail(NS_E_OOM, "batch table allocation failed");
    if (persist_setup(s) != NS_OK) return bail(NS_E_DEVICE, "persistent launch set-up: " + s->err);
    if (s->persist) {
      s->batch_ty = 16;
      s->batch_zc = 0;
    } else if (params[0].tile[0] > 0) {
      s->batch_ty = params[0].tile[0];
      s->batch_zc = params[0].tile[1];
      if (s->batch_ty >= 16)
        for (auto& I : s->in)
          if (!pass_grid_ok(I.g, I.esz))
            return bail(NS_E_INVALID, "tile: the two-sweep pass needs periodic axes of at least 4 cells");
    } else if (autotune_batch(s) != NS_OK) {
      return bail(NS_E_DEVICE, "batch autotune: " + s->err);
    }
  } else {
    for (auto& I : s->in) {
      if (autotune(s, I) != NS_OK) return bail(NS_E_DEVICE, "autotune: " + s->err);
    }
  }
  // the trial sweeps wrote the second pressure buffer: clear it again
  for (auto& I : s->in)
    if (hipMemsetAsync(I.s.p[1], 0, I.pbytes, s->stream) != hipSuccess ||
        (I.mixed && hipMemsetAsync(I.e[1], 0, (size_t)I.g.ntot * 4, s->stream) != hipSuccess))
      return bail(NS_E_DEVICE, "buffer clear failed");
  if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(NS_E_DEVICE, "stream synchronisation failed");
  *out = s;
  return NS_OK;
}

ns_status ns_set_state(ns_solver* s, int32_t inst, int32_t field, const double* src, int32_t on_device) {
  if (!s) return fail(nullptr, NS_E_INVALID, "NULL handle");
  if (inst < 0 || inst >= (int)s->in.size()) return fail(s, NS_E_INVALID, "instance out of range");
  if (!src) return fail(s, NS_E_INVALID, "src is NULL");
  DevGuard dg(s->device);
  Inst& I = s->in[inst];
  void* dst = nullptr;
  bool f32 = I.mixed;
  switch (field) {
    case NS_U: dst = I.s.u; break;
    case NS_V: dst = I.s.v; break;
    case NS_W: dst = I.s.w; break;
    case NS_P: dst = I.s.p[I.s.pcur]; f32 = false; break;
    case NS_FX: case NS_FY: case NS_FZ: {
      // the three force fields exist together (zero where never set): the
      // predictor reads all of them or none
      for (int c = 0; c < 3; c++)
        if (!I.frc[c]) HCK(s, dmalloc(&I.frc[c], I.bytes));
      dst = I.frc[field - NS_FX];
      break;
    }
    case NS_F: dst = I.F; break;
    case NS_G: dst = I.G; break;
    case NS_H: dst = I.H; break;
    case NS_RHS: dst = I.rhs; break;
    default: return fail(s, NS_E_INVALID, "unknown field id");
  }
  ns_status e = copy_in(s, I, dst, f32, src, on_device);
  if (e != NS_OK) return e;
  if (field <= NS_P) {
    I.rec_steps = 0;
    I.rec_valid = I.prm.checkpoint_every > 0;
  }
  return NS_OK;
}

ns_status ns_get_state(const ns_solver* cs, int32_t inst, int32_t field, double* dst, int32_t on_device) {
  ns_solver* s = const_cast<ns_solver*>(cs);
  if (!s) return fail(nullptr, NS_E_INVALID, "NULL handle");
  if (inst < 0 || inst >= (int)s->in.size()) return fail(s, NS_E_INVALID, "instance out of range");
  if (!dst) return fail(s, NS_E_INVALID, "dst is NULL");
  DevGuard dg(s->device);
  const Inst& I = s->in[inst];
  const void* src = nullptr;
  bool f32 = I.mixed;
  switch (field) {
    case NS_U: src = I.s.u; break;
    case NS_V: src = I.s.v; break;
    case NS_W: src = I.s.w; break;
    case NS_P: src = I.s.p[I.s.pcur]; f32 = false; break;
    case NS_FX: case NS_FY: case NS_FZ:
      src = I.frc[field - NS_FX];
      if (!src) {  // never set: zero
        if (on_device) HCK(s, hipMemsetAsync(dst, 0, I.g.ntot * sizeof(double), s->stream));
        else memset(dst, 0, I.g.ntot * sizeof(double));
        HCK(s, hipStreamSynchronize(s->stream));
        return NS_OK;
      }
      break;
    case NS_F: src = I.F; break;
    case NS_G: src = I.G; break;
    case NS_H: src = I.H; break;
    case NS_RHS: src = I.rhs; break;
    default: return fail(s, NS_E_INVALID, "unknown field id");
  }
  return copy_out(s, I, src, f32, dst, on_device);
}

ns_status ns_step(ns_solver* s, int32_t nsteps, ns_stats* stats) {
  if (!s) return fail(nullptr, NS_E_INVALID, "NULL handle");
  if (nsteps < 0) return fail(s, NS_E_INVALID, "nsteps must be >= 0");
  DevGuard dg(s->device);
  ns_status ret = NS_OK;
  auto checkpoint = [&](Inst& I) -> ns_status {
    const int k = I.prm.checkpoint_every;
    if (!(k > 0 && I.rec_valid && I.rec_steps % k == 0)) return NS_OK;
    const size_t slot = I.rec_steps / k;
    while (I.ck.size() <= slot) {
      I.ck.emplace_back();
      hipError_t e = alloc_state(I.ck.back(), I);
      if (e != hipSuccess) return fail_hip(s, "checkpoint allocation", e);
    }
    return save_state(s, I, I.s, I.ck[slot]);
  };
  if (s->batched && s->persist) {
    ret = nsteps > 0 ? persist_run(s, nsteps) : NS_OK;
    if (stats)
      for (size_t i = 0; i < s->in.size(); i++) stats[i] = s->in[i].st;
    return ret;
  }
  for (int n = 0; n < nsteps && ret == NS_OK; n++) {
    if (s->batched) {
      for (auto& I : s->in)
        if (ret == NS_OK) ret = checkpoint(I);
      if (ret == NS_OK) ret = s->in[0].mixed ? step_batched<float>(s) : step_batched<double>(s);
      for (auto& I : s->in) {
        if (ret == NS_OK && I.prm.checkpoint_every > 0 && I.rec_valid) I.rec_steps++;
        if (ret != NS_OK) I.rec_valid = false;
      }
      continue;
    }
    for (int i = 0; i < (int)s->in.size() && ret == NS_OK; i++) {
      Inst& I = s->in[i];
      const int k = I.prm.checkpoint_every;
      ret = checkpoint(I);
      if (ret != NS_OK) break;
      ret = I.mixed ? step_inst<float>(s, i, I.s, true) : step_inst<double>(s, i, I.s, true);
      if (ret == NS_OK && k > 0 && I.rec_valid) I.rec_steps++;
      if (ret != NS_OK) I.rec_valid = false;
    }
  }
  if (stats)
    for (size_t i = 0; i < s->in.size(); i++) stats[i] = s->in[i].st;
  return ret;
}

ns_status ns_get_timing(const ns_solver* s, ns_timing* out) {
  if (!s || !out) return fail(const_cast<ns_solver*>(s), NS_E_INVALID, "NULL argument");
  *out = s->tm;
  out->sor_tile[0] = s->batched ? s->batch_ty : s->in[0].shape.ty;
  out->sor_tile[1] = s->batched ? s->batch_zc : s->in[0].shape.zc;
  return NS_OK;
}

ns_status ns_backward(ns_solver* s, int32_t inst, const double* const g_final[3], double* const g_init[3],
                      int32_t on_device) {
  if (!s) return fail(nullptr, NS_E_INVALID, "NULL handle");
  if (inst < 0 || inst >= (int)s->in.size()) return fail(s, NS_E_INVALID, "instance out of range");
  if (!g_final || !g_init) return fail(s, NS_E_INVALID, "NULL gradient array");
  for (int c = 0; c < 3; c++)
    if (!g_final[c] || !g_init[c]) return fail(s, NS_E_INVALID, "NULL gradient field");
  Inst& I = s->in[inst];
  if (I.prm.checkpoint_every <= 0 || I.mixed || I.prm.dt <= 0)
    return fail(s, NS_E_INVALID, "ns_backward needs checkpoint_every > 0, NS_FP64 and a fixed dt");
  if (!I.rec_valid || I.rec_steps < 1)
    return fail(s, NS_E_STATE, "no recorded steps since the velocity was last set");
  DevGuard dg(s->device);
  const Geo& g = I.g;
  const int N = I.rec_steps, k = I.prm.checkpoint_every;
  const size_t pb = I.pbytes;
  // lazily allocate the adjoint work space
  if (!I.R.u) HCK(s, alloc_state(I.R, I));
  for (int c = 0; c < 3; c++) {
    if (!I.lam[c]) HCK(s, dmalloc((void**)&I.lam[c], pb));
    if (!I.z[c]) HCK(s, dmalloc((void**)&I.z[c], pb));
  }
  for (int b = 0; b < 2; b++)
    if (!I.q[b]) HCK(s, dmalloc((void**)&I.q[b], pb));
  while ((int)I.hist.size() < 3 * k) {
    double* h = nullptr;
    HCK(s, dmalloc((void**)&h, pb));
    I.hist.push_back(h);
  }
  const bool timing = s->timing;
  s->timing = false;
  const int saved_pred = I.pred;
  for (int c = 0; c < 3; c++) {
    ns_status e = copy_in(s, I, I.lam[c], false, g_final[c], on_device);
    if (e != NS_OK) { s->timing = timing; return e; }
    HCK(s, launch_mask_unknowns(s->stream, g, I.lam[c], c));
  }
  ns_status ret = NS_OK;
  I.qcur = 0;
  HCK(s, hipMemsetAsync(I.q[0], 0, pb, s->stream));
  const int nseg = (N + k - 1) / k;
  for (int seg = nseg - 1; seg >= 0 && ret == NS_OK; seg--) {
    const int s0 = seg * k, s1 = std::min(N, s0 + k);
    // recompute the segment from its checkpoint, keeping u^n (boundary-filled)
    ret = save_state(s, I, I.ck[seg], I.R);
    for (int n = s0; n < s1 && ret == NS_OK; n++) {
      double* hu = I.hist[3 * (n - s0)];
      double* hv = I.hist[3 * (n - s0) + 1];
      double* hw = I.hist[3 * (n - s0) + 2];
      HCK(s, launch_bc_vel<double>(s->stream, g, (double*)I.R.u, (double*)I.R.v, (double*)I.R.w, I.prm.wall_vel));
      HCK(s, hipMemcpyAsync(hu, I.R.u, pb, hipMemcpyDeviceToDevice, s->stream));
      HCK(s, hipMemcpyAsync(hv, I.R.v, pb, hipMemcpyDeviceToDevice, s->stream));
      HCK(s, hipMemcpyAsync(hw, I.R.w, pb, hipMemcpyDeviceToDevice, s->stream));
      if (n + 1 < s1) ret = step_inst<double>(s, inst, I.R, false);
    }
    // reverse sweep over the segment
    for (int n = s1 - 1; n >= s0 && ret == NS_OK; n--) {
      // mu = P lambda: rhs = D lambda, A q = rhs, mu = lambda - G q (dt = 1)
      for (int c = 0; c < 3; c++) {
        HCK(s, launch_mask_unknowns(s->stream, g, I.lam[c], c));
        for (int a = 0; a < 3; a++)
          if (g.per[a]) HCK(s, launch_periodic<double>(s->stream, g, I.lam[c], a));
      }
      HCK(s, launch_rhs<double>(s->stream, g, I.lam[0], I.lam[1], I.lam[2], (double*)I.rhs, I.ctl, I.part,
                                I.prm.tol, 1.0));
      int sw = 0;
      ret = solve_fp64(s, inst, I.q, &I.qcur, &sw);
      if (ret != NS_OK) break;
      if (s->hctl[inst].nonfinite) { ret = fail(s, NS_E_NONFINITE, "non-finite adjoint residual"); break; }
      HCK(s, launch_p_ghosts<double>(s->stream, g, I.q[I.qcur]));
      HCK(s, launch_project<double>(s->stream, g, I.lam[0], I.lam[1], I.lam[2], I.q[I.qcur], I.lam[0], I.lam[1],
                                    I.lam[2], I.ctl, 1.0));
      for (int c = 0; c < 3; c++) HCK(s, launch_mask_unknowns(s->stream, g, I.lam[c], c));
      // lambda^n = B^T J(u^n)^T mu
      const double* hu = I.hist[3 * (n - s0)];
      const double* hv = I.hist[3 * (n - s0) + 1];
      const double* hw = I.hist[3 * (n - s0) + 2];
      HCK(s, launch_adj_fgh(s->stream, g, hu, hv, hw, I.lam[0], I.lam[1], I.lam[2], I.z[0], I.z[1], I.z[2],
                            I.prm.dt, I.prm.re, I.prm.gamma));
      HCK(s, launch_adj_fold(s->stream, g, I.z[0], I.z[1], I.z[2]));
      for (int c = 0; c < 3; c++) std::swap(I.lam[c], I.z[c]);
    }
  }
  I.pred = saved_pred;
  s->timing = timing;
  if (ret != NS_OK) return ret;
  for (int c = 0; c < 3; c++) {
    ns_status e = copy_out(s, I, I.lam[c], false, g_init[c], on_device);
    if (e != NS_OK) return e;
  }
  return NS_OK;
}

void ns_destroy(ns_solver* s) {
  if (!s) return;
  DevGuard dg(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  for (auto& I : s->in) free_inst(I);
  for (auto e : s->pool) (void)hipEventDestroy(e);
  if (s->hctl) (void)hipHostFree(s->hctl);
  if (s->items_h) (void)hipHostFree(s->items_h);
  dfree(s->items_d);
  if (s->stage_h) (void)hipHostFree(s->stage_h);
  dfree(s->stage_d);
  for (int k = 0; k < ns_solver::kAux; k++) {
    if (s->aux[k]) (void)hipStreamDestroy(s->aux[k]);
    if (s->ev_join[k]) (void)hipEventDestroy(s->ev_join[k]);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  dfree(s->ctl_all);
  dfree(s->stage);
  if (s->pitems_h) (void)hipHostFree(s->pitems_h);
  if (s->pstats_h) (void)hipHostFree(s->pstats_h);
  if (s->perr_h) (void)hipHostFree(s->perr_h);
  dfree(s->pitems_d);
  dfree(s->pstats_d);
  dfree(s->pslots_d);
  dfree(s->pbar_d);
  dfree(s->perr_d);
  delete s;
}

int64_t ns_guard_check(int32_t self_test) {
  if (self_test && guard_on()) {
    void* q = nullptr;
    if (dmalloc(&q, 1000) == hipSuccess) {
      (void)hipMemset((char*)q + 1000, 0x5A, 1);  // one byte past the end, by a host-side fill
      dfree(q);
    }
  }
  std::lock_guard<std::mutex> lk(g_guard_mu);
  (void)hipDeviceSynchronize();
  long long bad = g_guard_bad;
  for (const auto& kv : g_guard) bad += guard_scan(kv.second);
  return bad;
}

ns_status ns_step_noalloc(const ns_params* params, double* u, double* v, double* w, double* p, int32_t nsteps,
                          void* hip_stream, ns_stats* stats) {
  if (!params) return fail(nullptr, NS_E_INVALID, "params is NULL");
  ns_status st = validate(*params, 0);
  if (st != NS_OK) return st;
  if (params->precision != NS_FP64) return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: NS_FP64 only");
  if (params->checkpoint_every != 0) return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: no recording");
  if (params->flags & NS_TIMING) return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: no stage timers");
  if (params->flags & NS_RK2) return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: Euler steps only");
  if (nsteps < 0) return fail(nullptr, NS_E_INVALID, "nsteps must be >= 0");
  if (!u || !v || !w || !p) return fail(nullptr, NS_E_INVALID, "u, v, w and p must be device pointers");
  const Geo g = make_geo(*params);
  if (g.ntot > kNaEntries)
    return fail(nullptr, NS_E_INVALID,
                "ns_step_noalloc: (nx+2)(ny+2)(nz+2) exceeds the static scratch (524288 entries per field)");
  if ((long)reduce_blocks(g) > kNaPartials)
    return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: too many partial sums for the static scratch");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(nullptr, NS_E_DEVICE, "no HIP device");
  if (dev >= kNaMaxDevices) return fail(nullptr, NS_E_INVALID, "device index beyond the supported range");
  double* const fields[4] = {u, v, w, p};
  for (double* q : fields)
    if (is_device_memory(q, dev) != NS_OK)
      return fail(nullptr, NS_E_INVALID, "ns_step_noalloc: u, v, w and p must be memory of the current device");
  NaDevice* D = nullptr;
  st = na_setup(dev, &D);
  if (st != NS_OK) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  ns_solver* s = D->shell;
  s->stream = (hipStream_t)hip_stream;
  Inst& I = s->in[0];
  I = Inst{};
  I.prm = *params;
  I.g = g;
  I.mixed = false;
  I.esz = 8;
  I.bytes = I.pbytes = (size_t)g.ntot * 8;
  double* base = D->ptr;
  I.F = base;
  I.G = base + kNaEntries;
  I.H = base + 2 * kNaEntries;
  I.rhs = base + 3 * kNaEntries;
  I.part = base + 5 * kNaEntries;
  I.ctl = (Ctl*)(base + 5 * kNaEntries + kNaPartials);
  I.s.u = u;
  I.s.v = v;
  I.s.w = w;
  I.s.p[0] = p;
  I.s.p[1] = base + 4 * kNaEntries;
  I.s.pcur = 0;
  I.shape = pick_shape(I.prm, g, 8);
  auto done = [&](ns_status code) {
    if (code != NS_OK) g_create_err = s->err;
    if (stats) *stats = I.st;
    return code;
  };
  k_na_init<<<conv_grid(5 * kNaEntries + kNaPartials), 256, 0, s->stream>>>(
      base, 5 * kNaEntries + kNaPartials, I.ctl, I.prm.dt > 0 ? I.prm.dt : 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return done(fail_hip(s, "scratch clear", e));
  ns_status ret = NS_OK;
  for (int n = 0; n < nsteps && ret == NS_OK; n++) ret = step_inst<double>(s, 0, I.s, true);
  if (ret == NS_OK && I.s.pcur == 1) {
    e = hipMemcpyAsync(p, I.s.p[1], I.pbytes, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) ret = fail_hip(s, "pressure copy", e);
  }
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess && ret == NS_OK) ret = fail_hip(s, "stream synchronisation", e);
  return done(ret);
}

const char* ns_last_error(const ns_solver* s) {
  return s ? s->err.c_str() : g_create_err.c_str();
}

}  // extern "C"
