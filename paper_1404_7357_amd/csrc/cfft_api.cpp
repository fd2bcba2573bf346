// C-ABI layer of the contour-FFT library: argument validation, plans,
// workspace and geometry management, and launch sequencing.  All arithmetic
// of the method runs in the HIP kernels; this file only decides what to
// launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cfft.h"
#include "cfft_internal.h"

using namespace cfft;

constexpr int kProfClasses = 10;

namespace {

thread_local std::string g_last_error;

cfft_status_t fail(cfft_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

cfft_status_t hip_fail(hipError_t e, const char* what) {
  return fail(CFFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool env_flag(const char* name) {
  const char* v = std::getenv(name);
  return v && v[0] && std::strcmp(v, "0") != 0;
}

long long env_ll(const char* name, long long dflt) {
  const char* v = std::getenv(name);
  if (!v || !v[0]) return dflt;
  char* end = nullptr;
  long long r = std::strtoll(v, &end, 10);
  return (end && *end == 0) ? r : dflt;
}

// Cap of the pass workspace (the intermediates of one pair chunk), MiB:
// CFFT_WORKSPACE_MB, else 64 GiB, which lets every benchmark grid run all
// its pairs in one launch on a 288 GB device (4096^2 FP64, 36 pairs:
// 38.7 GB).  cfft_tabulate takes smaller chunks when the allocation fails.
long long workspace_limit_mb() { return env_ll("CFFT_WORKSPACE_MB", 65536); }

// Device allocation with the test hook CFFT_TEST_FAIL_ALLOC=1.
cfft_status_t dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (env_flag("CFFT_TEST_FAIL_ALLOC")) return fail(CFFT_ERR_ALLOC, "%s: allocation refused (CFFT_TEST_FAIL_ALLOC)", what);
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(CFFT_ERR_ALLOC, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  return CFFT_OK;
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

struct GeomHost {
  std::vector<GeomGroup> groups;
  std::vector<double> xs, ys;
  std::vector<int> index;
  int total_p = 0, total_r = 0, total_idx = 0, ppad = 0, ngroups_x = 0;
};

// Group bases by (kind, a, b); inside a group place each basis on the grid of
// distinct centres.  A second basis on an occupied slot opens another group.
bool build_geometry(const cfft_basis_t* basis, int nb, GeomHost& out) {
  std::vector<int> pending(nb);
  for (int i = 0; i < nb; ++i) pending[i] = i;
  while (!pending.empty()) {
    std::map<std::tuple<int, double, double>, std::vector<int>> by_shape;
    for (int j : pending) by_shape[std::make_tuple(basis[j].kind, basis[j].a, basis[j].b)].push_back(j);
    std::vector<int> overflow;
    for (auto& kv : by_shape) {
      const auto& mem = kv.second;
      std::vector<double> xs, ys;
      for (int j : mem) {
        xs.push_back(basis[j].cx);
        ys.push_back(basis[j].cy);
      }
      std::sort(xs.begin(), xs.end());
      xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
      std::sort(ys.begin(), ys.end());
      ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
      GeomGroup g;
      g.kind = std::get<0>(kv.first);
      g.a = std::get<1>(kv.first);
      g.b = std::get<2>(kv.first);
      g.np = (int)xs.size();
      g.nr = (int)ys.size();
      g.xoff = (int)out.xs.size();
      g.yoff = (int)out.ys.size();
      g.ioff = (int)out.index.size();
      g.uoff = g.poff = 0;   // set below, once the group order is final
      auto spacing = [](const std::vector<double>& v, double& step) {
        step = v.size() > 1 ? (v.back() - v.front()) / (double)(v.size() - 1) : 0.0;
        const double tol = 1e-12 * std::max(std::fabs(v.front()) + std::fabs(v.back()), std::fabs(step));
        for (size_t i = 0; i < v.size(); ++i)
          if (std::fabs(v[i] - (v.front() + (double)i * step)) > tol) return false;
        return true;
      };
      const bool ux = spacing(xs, g.dxc), uy = spacing(ys, g.dyc);
      g.uniform = ux && uy ? 1 : 0;
      std::vector<int> idx((size_t)g.np * g.nr, -1);
      for (int j : mem) {
        const int p = (int)(std::lower_bound(xs.begin(), xs.end(), basis[j].cx) - xs.begin());
        const int r = (int)(std::lower_bound(ys.begin(), ys.end(), basis[j].cy) - ys.begin());
        int& slot = idx[(size_t)p * g.nr + r];
        if (slot < 0) slot = j;
        else overflow.push_back(j);
      }
      out.xs.insert(out.xs.end(), xs.begin(), xs.end());
      out.ys.insert(out.ys.end(), ys.begin(), ys.end());
      out.index.insert(out.index.end(), idx.begin(), idx.end());
      out.total_r += g.nr;
      out.total_idx += g.np * g.nr;
      out.groups.push_back(g);
      if ((int)out.groups.size() > kMaxGroups) return false;
    }
    pending.swap(overflow);
  }
  // x-directed groups first (the spectra kernel accumulates one current
  // component at a time), then the per-group row offsets in that order.
  std::stable_sort(out.groups.begin(), out.groups.end(), [](const GeomGroup& a, const GeomGroup& b) {
    return (a.kind == CFFT_ROOFTOP_Y || a.kind == CFFT_COSINE_Y) < (b.kind == CFFT_ROOFTOP_Y || b.kind == CFFT_COSINE_Y);
  });
  out.total_p = 0;
  out.ppad = 0;
  out.ngroups_x = 0;
  for (GeomGroup& g : out.groups) {
    g.uoff = out.total_p;
    g.poff = out.ppad;
    out.total_p += g.np;
    out.ppad += (g.np + kSpecPChunk - 1) / kSpecPChunk * kSpecPChunk;
    if (!(g.kind == CFFT_ROOFTOP_Y || g.kind == CFFT_COSINE_Y)) ++out.ngroups_x;
  }
  return true;
}

uint64_t hash_bytes(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

// Device scratch of the allocation-free entry point (cfft_tabulate_noalloc):
// the intermediates between the row and column passes of one pair chunk.
// Each device the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, not a device
// address: c_fft_plan resolves the device address with hipGetSymbolAddress
// once per device (with that device current), and only that address is
// ever handed to kernels.
constexpr size_t kNoAllocScratchBytes = CFFT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), resolved on
// the first call for that device.
cfft_status_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(CFFT_ERR_UNSUPPORTED, "device index %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return CFFT_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(CFFT_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                e != hipSuccess ? hipGetErrorString(e) : "null address");
  }
  g_scratch_ptr[device] = ptr;
  return CFFT_OK;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

struct GridState {
  cfft_grid_desc_t d;
  Axis x, y;
  void* tw64x = nullptr;
  void* tw64y = nullptr;
  void* tw32x = nullptr;
  void* tw32y = nullptr;
  double2* utab = nullptr;       // spectra tables for the current geometry
  uint64_t utab_geo = 0;
  size_t utab_bytes = 0;
  int band = 0;                  // x2 zero-padded grid (CFFT_FLAG_ZERO_PAD2)
};

struct cfft_plan_s {
  int device = 0;
  int max_mbf = 0;
  int flags = 0;
  std::vector<GridState> grids;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* ws2 = nullptr;
  size_t ws2_bytes = 0;
  void* ws3 = nullptr;      // spectra scratch (per-row contractions over y-centres)
  size_t ws3_bytes = 0;
  void* ws4 = nullptr;      // interpolation adjoints: sort keys, runs and sort scratch
  size_t ws4_bytes = 0;
  // geometry cache (one basis set at a time)
  uint64_t geo_hash = 0;
  int geo_nbasis = 0;
  GeomHost geo_host;
  GeomDevice geo_dev{};
  void* geo_mem = nullptr;
  int* flag_dev = nullptr;
  int* flag_host = nullptr;
  // instrumentation: recorded (start, stop) event pairs per kernel class
  bool profiling = false;
  struct Schedule {
    long long chunk;   // pairs per row/column launch
    int lanes;         // 1, or 2 plan-owned streams taking alternate chunks
    int tile;          // kColTile*: column tile of the column pass
  };
  std::map<long long, Schedule> tuned;   // (grid, npairs) -> the autotuner's choice
  hipStream_t lane[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_row0 = nullptr, ev_join[2] = {nullptr, nullptr};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof[kProfClasses];
};

namespace {

std::mutex g_plans_mu;
std::set<cfft_plan_s*> g_plans;

bool plan_live(cfft_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  return g_plans.count(p) != 0;
}

void free_geometry(cfft_plan_s* p) {
  if (p->geo_mem) (void)hipFree(p->geo_mem);
  p->geo_mem = nullptr;
  p->geo_hash = 0;
  p->geo_nbasis = 0;
  p->geo_dev = GeomDevice{};
}

cfft_status_t make_twiddles(int n, void** d64, void** d32) {
  std::vector<double2> t64(n);
  std::vector<float2> t32(n);
  for (int j = 0; j < n; ++j) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
    const long double c = cosl(ang), s = sinl(ang);
    t64[j] = make_double2((double)c, (double)s);
    t32[j] = make_float2((float)c, (float)s);
  }
  cfft_status_t st = dev_alloc(d64, sizeof(double2) * n, "twiddles");
  if (st != CFFT_OK) return st;
  st = dev_alloc(d32, sizeof(float2) * n, "twiddles");
  if (st != CFFT_OK) return st;
  hipError_t e = hipMemcpy(*d64, t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(*d32, t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "twiddle upload");
  return CFFT_OK;
}

cfft_status_t check_plan(cfft_plan_t plan, int grid) {
  if (!plan) return fail(CFFT_ERR_INVALID_ARG, "plan is NULL");
  if (!plan_live(plan)) return fail(CFFT_ERR_INVALID_ARG, "unknown or destroyed plan");
  if (grid < 0 || grid >= (int)plan->grids.size())
    return fail(CFFT_ERR_INVALID_ARG, "grid index %d out of range [0, %zu)", grid, plan->grids.size());
  hipError_t e = hipSetDevice(plan->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return CFFT_OK;
}

// Largest factor by which the Taylor recombination of eq. fftarry can
// amplify the rounding of a transform over the table.  A transform of term
// (a, b) is weighted by (gamma kx)^a (gamma ky)^b before it and by
// Dx^a Dy^b / (a! b!) after it; with |k| <= k_max and |D| <= n pi / (2 k_max)
// per axis the product is at most x^a y^b / (a! b!), x = gamma nx pi / 2,
// y = gamma ny pi / 2, whatever the spectral span.  Summed over the terms:
// sum_{c <= P} (x + y)^c / c! for the total-degree truncation, and
// (sum_a x^a / a!)(sum_b y^b / b!) for the tensor truncation.  The parabolic
// contour's ratio never exceeds gamma, so the same bound holds there.
double taylor_amplification(const cfft_grid_desc_t& d) {
  const double x = d.gamma * d.nx * M_PI / 2.0, y = d.gamma * d.ny * M_PI / 2.0;
  auto poly = [&](double v) {
    double s = 0.0, t = 1.0;
    for (int c = 0; c <= d.order; ++c) {
      if (c > 0) t *= v / c;
      s += t;
    }
    return s;
  };
  return d.truncation == CFFT_TRUNC_TENSOR ? poly(x) * poly(y) : poly(x + y);
}

// Pairs per launch when npairs go in launches of at most `chunk`: the same
// number of launches, in chunks that differ by at most one pair (81 pairs in
// launches of at most 64 run as 41 + 40, not 64 + 17).
long long balanced_chunk(long long npairs, long long chunk) {
  const long long launches = (npairs + chunk - 1) / chunk;
  return (npairs + launches - 1) / launches;
}

// The row pass streams its intermediates past the caches (non-temporal
// stores) when the intermediates in flight between a row pass and its column
// pass exceed what the 256 MB memory-side cache can keep: then they return
// from HBM anyway, and the caches stay with the inputs that the pairs of a
// row share (4096^2 FP64, 36 pairs: row pass 18.6 -> 16.5 ms).
bool stream_out(size_t inter_bytes) { return inter_bytes > ((size_t)192 << 20); }

// Mixed grids run their transforms in FP32 up to this amplification and in
// FP64 (on the same FP32-stored data) beyond it.  Measured FP32-transform
// errors against the FP64 oracle: <= 5.4e-7 up to an amplification of 4.4e3
// (every mixed workload up to 2048-point axes), 1.1e-5 at 2.1e4 (a
// 4096-point axis), above the mixed path's 1e-5 target.
constexpr double kFp32MaxAmplification = 8000.0;

PassParams pass_params(const GridState& gs) {
  PassParams p;
  p.x = gs.x;
  p.y = gs.y;
  p.gamma = gs.d.gamma;
  p.order = gs.d.order;
  p.tensor = gs.d.truncation == CFFT_TRUNC_TENSOR ? 1 : 0;
  p.parabolic = gs.d.contour == CFFT_CONTOUR_PARABOLIC ? 1 : 0;
  p.beta_end = gs.d.beta_end;
  p.band = gs.band;
  p.precision = gs.d.precision;
  p.hi_compute = gs.d.precision == CFFT_MIXED && taylor_amplification(gs.d) > kFp32MaxAmplification ? 1 : 0;
  p.col_tile = kColTileDefault;
  p.stream_out = 0;
  return p;
}

GreenParams green_params(const GridState& gs, double eps_r, double tan_delta, double h) {
  return GreenParams{gs.x, gs.y, gs.d.gamma, gs.d.k0, eps_r, tan_delta, h,
                     gs.d.contour == CFFT_CONTOUR_PARABOLIC ? 1 : 0, gs.d.beta_end};
}

cfft_status_t ensure_ws(void** ws, size_t* have, size_t need, const char* what) {
  if (*have >= need) return CFFT_OK;
  if (*ws) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise before workspace growth");
    (void)hipFree(*ws);
    *ws = nullptr;
    *have = 0;
  }
  cfft_status_t st = dev_alloc(ws, need, what);
  if (st != CFFT_OK) return st;
  *have = need;
  return CFFT_OK;
}

cfft_status_t validate_basis(const cfft_basis_t* basis, int nbasis) {
  if (!basis) return fail(CFFT_ERR_INVALID_ARG, "basis is NULL");
  if (nbasis < 1 || nbasis > 65536) return fail(CFFT_ERR_INVALID_ARG, "nbasis %d outside [1, 65536]", nbasis);
  for (int j = 0; j < nbasis; ++j) {
    const cfft_basis_t& b = basis[j];
    if (b.kind < CFFT_ROOFTOP_X || b.kind > CFFT_COSINE_Y)
      return fail(CFFT_ERR_INVALID_ARG, "basis %d: unknown kind %d", j, b.kind);
    if (b.pad != 0) return fail(CFFT_ERR_INVALID_ARG, "basis %d: pad must be 0", j);
    if (!(std::isfinite(b.cx) && std::isfinite(b.cy) && b.a > 0 && b.b > 0 && std::isfinite(b.a) &&
          std::isfinite(b.b)))
      return fail(CFFT_ERR_INVALID_ARG, "basis %d: non-finite centre or non-positive size", j);
  }
  return CFFT_OK;
}

// Upload (or reuse) the separable geometry of a basis set and make sure the
// grid's spectra tables match it.
cfft_status_t ensure_geometry(cfft_plan_s* plan, GridState& gs, const cfft_basis_t* basis, int nbasis,
                              hipStream_t s) {
  const uint64_t h = hash_bytes(basis, sizeof(cfft_basis_t) * (size_t)nbasis, (uint64_t)nbasis * 0x9e3779b97f4a7c15ull);
  if (!(plan->geo_mem && plan->geo_hash == h && plan->geo_nbasis == nbasis)) {
    GeomHost gh;
    if (!build_geometry(basis, nbasis, gh))
      return fail(CFFT_ERR_UNSUPPORTED, "basis set needs more than %d shape groups", kMaxGroups);
    GeomDevice probe{};
    probe.ngroups = (int)gh.groups.size();
    probe.total_r = gh.total_r;
    if (spectra_lds_bytes(probe, plan->max_mbf) > kMaxDynamicLds)
      return fail(CFFT_ERR_UNSUPPORTED, "%d distinct y-centres: too many for the per-row LDS tables", gh.total_r);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "synchronise before geometry upload");
    free_geometry(plan);
    const size_t bg = sizeof(GeomGroup) * gh.groups.size();
    const size_t bx = sizeof(double) * gh.xs.size();
    const size_t by = sizeof(double) * gh.ys.size();
    const size_t bi = sizeof(int) * gh.index.size();
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t total = al(bg) + al(bx) + al(by) + al(bi);
    cfft_status_t st = dev_alloc(&plan->geo_mem, total, "geometry");
    if (st != CFFT_OK) return st;
    char* base = (char*)plan->geo_mem;
    GeomDevice gd;
    gd.ngroups = (int)gh.groups.size();
    gd.nbasis = nbasis;
    gd.total_p = gh.total_p;
    gd.total_r = gh.total_r;
    gd.total_idx = gh.total_idx;
    gd.ppad = gh.ppad;
    gd.ngroups_x = gh.ngroups_x;
    gd.groups = (GeomGroup*)base;
    gd.xs = (double*)(base + al(bg));
    gd.ys = (double*)(base + al(bg) + al(bx));
    gd.index = (int*)(base + al(bg) + al(bx) + al(by));
    e = hipMemcpy(gd.groups, gh.groups.data(), bg, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gd.xs, gh.xs.data(), bx, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gd.ys, gh.ys.data(), by, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gd.index, gh.index.data(), bi, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_geometry(plan);
      return hip_fail(e, "geometry upload");
    }
    plan->geo_dev = gd;
    plan->geo_host = gh;
    plan->geo_hash = h;
    plan->geo_nbasis = nbasis;
    for (auto& g : plan->grids) g.utab_geo = 0;
  }
  if (gs.utab_geo != plan->geo_hash) {
    const size_t need = sizeof(double2) * spectra_tables_len(gs.x, gs.y, plan->geo_dev);
    if (gs.utab_bytes < need) {
      if (gs.utab) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "synchronise before table growth");
        (void)hipFree(gs.utab);
        gs.utab = nullptr;
        gs.utab_bytes = 0;
      }
      cfft_status_t st = dev_alloc((void**)&gs.utab, need, "spectra tables");
      if (st != CFFT_OK) return st;
      gs.utab_bytes = need;
    }
    hipError_t e = launch_spectra_tables(gs.x, gs.y, gs.d.gamma, plan->geo_dev, gs.utab, s);
    if (e != hipSuccess) return hip_fail(e, "spectra tables launch");
    gs.utab_geo = plan->geo_hash;
  }
  return CFFT_OK;
}

cfft_status_t validate_pairs(const int32_t* pairs, int npairs, int nmbf) {
  if (!pairs) return fail(CFFT_ERR_INVALID_ARG, "pairs is NULL");
  if (npairs < 1 || npairs > 4096) return fail(CFFT_ERR_INVALID_ARG, "npairs %d outside [1, 4096]", npairs);
  for (int i = 0; i < npairs; ++i) {
    if (pairs[2 * i] < 0 || pairs[2 * i] >= nmbf || pairs[2 * i + 1] < 0 || pairs[2 * i + 1] >= nmbf)
      return fail(CFFT_ERR_INVALID_ARG, "pair %d = (%d, %d) outside [0, %d)", i, pairs[2 * i], pairs[2 * i + 1], nmbf);
  }
  return CFFT_OK;
}

__global__ void nonfinite_kernel(const double* v, size_t n, int* flag) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) {
      *flag = 1;
      return;
    }
}
__global__ void nonfinite_kernel_f(const float* v, size_t n, int* flag) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) {
      *flag = 1;
      return;
    }
}

cfft_status_t check_finite(cfft_plan_s* plan, const void* data, size_t nreal, bool fp32, hipStream_t s) {
  if (!(plan->flags & CFFT_FLAG_CHECK_FINITE)) return CFFT_OK;
  hipError_t e = hipMemsetAsync(plan->flag_dev, 0, sizeof(int), s);
  if (e != hipSuccess) return hip_fail(e, "flag reset");
  if (fp32)
    hipLaunchKernelGGL(nonfinite_kernel_f, dim3(1024), dim3(256), 0, s, (const float*)data, nreal, plan->flag_dev);
  else
    hipLaunchKernelGGL(nonfinite_kernel, dim3(1024), dim3(256), 0, s, (const double*)data, nreal, plan->flag_dev);
  e = hipMemcpyAsync(plan->flag_host, plan->flag_dev, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "non-finite check");
  if (*plan->flag_host) return fail(CFFT_ERR_NONFINITE, "output contains NaN or Inf");
  return CFFT_OK;
}

// Bracket a launch with events when profiling is on.
struct ProfScope {
  cfft_plan_s* plan;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(cfft_plan_s* p, int c, hipStream_t st) : plan(p), cls(c), s(st) {
    if (!plan->profiling) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      (void)hipGetLastError();
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    plan->prof[cls].emplace_back(a, b);
  }
};

// Two plan-owned streams at default priority plus the fork/join events of the
// two-lane schedule, created on first use.
hipError_t ensure_lanes(cfft_plan_s* plan) {
  if (plan->lane[0]) return hipSuccess;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&plan->lane[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_row0, hipEventDisableTiming);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&plan->ev_join[i], hipEventDisableTiming);
  return e;
}

void release_plan(cfft_plan_s* plan) {
  (void)hipSetDevice(plan->device);
  (void)hipDeviceSynchronize();
  for (int i = 0; i < 2; ++i)
    if (plan->lane[i]) (void)hipStreamDestroy(plan->lane[i]);
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_row0) (void)hipEventDestroy(plan->ev_row0);
  for (int i = 0; i < 2; ++i)
    if (plan->ev_join[i]) (void)hipEventDestroy(plan->ev_join[i]);
  for (auto& g : plan->grids) {
    if (g.tw64x) (void)hipFree(g.tw64x);
    if (g.tw64y) (void)hipFree(g.tw64y);
    if (g.tw32x) (void)hipFree(g.tw32x);
    if (g.tw32y) (void)hipFree(g.tw32y);
    if (g.utab) (void)hipFree(g.utab);
  }
  if (plan->ws) (void)hipFree(plan->ws);
  if (plan->ws2) (void)hipFree(plan->ws2);
  if (plan->ws3) (void)hipFree(plan->ws3);
  if (plan->ws4) (void)hipFree(plan->ws4);
  if (plan->flag_dev) (void)hipFree(plan->flag_dev);
  if (plan->flag_host) (void)hipHostFree(plan->flag_host);
  for (auto& v : plan->prof)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  free_geometry(plan);
  delete plan;
}

}  // namespace

extern "C" {

const char* cfft_last_error(void) { return g_last_error.c_str(); }

cfft_status_t cfft_profile(cfft_plan_t plan, int32_t enable) {
  g_last_error.clear();
  if (!plan || !plan_live(plan)) return fail(CFFT_ERR_INVALID_ARG, "unknown or destroyed plan");
  plan->profiling = enable != 0;
  return CFFT_OK;
}

cfft_status_t cfft_profile_read(cfft_plan_t plan, int32_t kernel_class, double* total_ms, int64_t* launches) {
  g_last_error.clear();
  if (!plan || !plan_live(plan)) return fail(CFFT_ERR_INVALID_ARG, "unknown or destroyed plan");
  if (kernel_class < 0 || kernel_class >= kProfClasses)
    return fail(CFFT_ERR_INVALID_ARG, "kernel class %d outside [0, %d)", kernel_class, kProfClasses);
  if (!total_ms || !launches) return fail(CFFT_ERR_INVALID_ARG, "total_ms or launches is NULL");
  double acc = 0.0;
  int64_t cnt = 0;
  hipError_t err = hipSuccess;
  for (auto& pr : plan->prof[kernel_class]) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess && err == hipSuccess) err = e;
    acc += ms;
    ++cnt;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  plan->prof[kernel_class].clear();
  *total_ms = acc;
  *launches = cnt;
  if (err != hipSuccess) return hip_fail(err, "profile read");
  return CFFT_OK;
}

const char* cfft_version(void) { return "cfft-mi355x 0.1 (gfx950)"; }

cfft_status_t c_fft_plan(const cfft_grid_desc_t* grids, int32_t ngrids, int32_t max_mbf, int32_t flags,
                         cfft_plan_t* out) {
  g_last_error.clear();
  if (!out) return fail(CFFT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grids) return fail(CFFT_ERR_INVALID_ARG, "grids is NULL");
  if (ngrids < 1 || ngrids > 64) return fail(CFFT_ERR_INVALID_ARG, "ngrids %d outside [1, 64]", ngrids);
  if (max_mbf < 1 || max_mbf > 16) return fail(CFFT_ERR_INVALID_ARG, "max_mbf %d outside [1, 16]", max_mbf);
  if (flags & ~(CFFT_FLAG_CHECK_FINITE | CFFT_FLAG_AUTOTUNE | CFFT_FLAG_ZERO_PAD2))
    return fail(CFFT_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  for (int i = 0; i < ngrids; ++i) {
    const cfft_grid_desc_t& g = grids[i];
    if (!pow2_in(g.nx, 16, 4096) || !pow2_in(g.ny, 16, 4096))
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: nx, ny = %d, %d must be powers of two in [16, 4096]", i, g.nx, g.ny);
    if (!(g.kx_max > 0 && g.ky_max > 0 && std::isfinite(g.kx_max) && std::isfinite(g.ky_max)))
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: kx_max, ky_max must be finite and > 0", i);
    if (!(g.k0 > 0 && std::isfinite(g.k0))) return fail(CFFT_ERR_INVALID_ARG, "grid %d: k0 must be finite and > 0", i);
    if (!(g.gamma > 0 && std::isfinite(g.gamma))) return fail(CFFT_ERR_INVALID_ARG, "grid %d: gamma must be > 0", i);
    if (g.order < 0 || g.order > kMaxOrder)
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: order %d outside [0, %d]", i, g.order, kMaxOrder);
    if (g.precision != CFFT_FP64 && g.precision != CFFT_MIXED)
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: unknown precision %d", i, g.precision);
    if (g.truncation != CFFT_TRUNC_TOTAL && g.truncation != CFFT_TRUNC_TENSOR)
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: truncation %d is neither TOTAL nor TENSOR", i, g.truncation);
    if (g.contour != CFFT_CONTOUR_RAY && g.contour != CFFT_CONTOUR_PARABOLIC)
      return fail(CFFT_ERR_INVALID_ARG, "grid %d: unknown contour %d", i, g.contour);
    if (g.contour == CFFT_CONTOUR_PARABOLIC) {
      if (!(std::isfinite(g.beta_end) && g.beta_end > 0.0))
        return fail(CFFT_ERR_INVALID_ARG, "grid %d: the parabolic contour needs a finite beta_end > 0", i);
      if (g.truncation == CFFT_TRUNC_TENSOR)
        return fail(CFFT_ERR_UNSUPPORTED, "grid %d: tensor-product truncation needs the ray contour", i);
    }
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(CFFT_ERR_HIP, "no HIP device available (%s)", e == hipSuccess ? "0 devices" : hipGetErrorString(e));
  }
  cfft_plan_s* p = new (std::nothrow) cfft_plan_s();
  if (!p) return fail(CFFT_ERR_ALLOC, "host allocation of the plan failed");
  e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  {
    cfft_status_t sst = resolve_scratch(p->device);
    if (sst != CFFT_OK) {
      delete p;
      return sst;
    }
  }
  p->max_mbf = max_mbf;
  p->flags = flags;
  p->grids.resize(ngrids);
  for (int i = 0; i < ngrids; ++i) {
    GridState& gs = p->grids[i];
    gs.d = grids[i];
    gs.band = (flags & CFFT_FLAG_ZERO_PAD2) ? 1 : 0;
    const double xm = gs.d.nx * M_PI / (2.0 * gs.d.kx_max);
    const double ym = gs.d.ny * M_PI / (2.0 * gs.d.ky_max);
    gs.x = Axis{gs.d.nx, -gs.d.kx_max, 2.0 * gs.d.kx_max / gs.d.nx, -xm, M_PI / gs.d.kx_max};
    gs.y = Axis{gs.d.ny, -gs.d.ky_max, 2.0 * gs.d.ky_max / gs.d.ny, -ym, M_PI / gs.d.ky_max};
    cfft_status_t st = make_twiddles(gs.d.nx, &gs.tw64x, &gs.tw32x);
    if (st == CFFT_OK) st = make_twiddles(gs.d.ny, &gs.tw64y, &gs.tw32y);
    if (st != CFFT_OK) {
      release_plan(p);
      return st;
    }
  }
  cfft_status_t st = dev_alloc((void**)&p->flag_dev, sizeof(int), "flag");
  if (st != CFFT_OK) {
    release_plan(p);
    return st;
  }
  e = hipHostMalloc((void**)&p->flag_host, sizeof(int), hipHostMallocDefault);
  if (e != hipSuccess) {
    p->flag_host = nullptr;
    release_plan(p);
    return fail(CFFT_ERR_ALLOC, "pinned flag allocation failed: %s", hipGetErrorString(e));
  }
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(p);
  }
  *out = p;
  return CFFT_OK;
}

cfft_status_t c_fft_plan_destroy(cfft_plan_t plan) {
  g_last_error.clear();
  if (!plan) return CFFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!g_plans.erase(plan)) return fail(CFFT_ERR_INVALID_ARG, "unknown or already destroyed plan");
  }
  release_plan(plan);
  return CFFT_OK;
}

cfft_status_t slab_green_eval(cfft_plan_t plan, int32_t grid, double eps_r, double tan_delta, double h, void* g,
                              void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!g) return fail(CFFT_ERR_INVALID_ARG, "g is NULL");
  if (!(std::isfinite(eps_r) && eps_r >= 1.0)) return fail(CFFT_ERR_INVALID_ARG, "eps_r must be finite and >= 1");
  if (!(std::isfinite(tan_delta) && tan_delta >= 0.0))
    return fail(CFFT_ERR_INVALID_ARG, "tan_delta must be finite and >= 0");
  if (!(std::isfinite(h) && h > 0.0)) return fail(CFFT_ERR_INVALID_ARG, "h must be finite and > 0");
  GridState& gs = plan->grids[grid];
  const GreenParams p = green_params(gs, eps_r, tan_delta, h);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps(plan, 0, s);
    e = launch_green(p, (double2*)g, s);
  }
  if (e != hipSuccess) return hip_fail(e, "slab_green_eval launch");
  return check_finite(plan, g, (size_t)6 * gs.x.n * gs.y.n, false, s);
}

cfft_status_t mbf_spectra(cfft_plan_t plan, int32_t grid, const cfft_basis_t* basis, int32_t nbasis, const void* q,
                          int32_t nmbf, void* spec, void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!q || !spec) return fail(CFFT_ERR_INVALID_ARG, "q or spec is NULL");
  if (nmbf < 1 || nmbf > plan->max_mbf)
    return fail(CFFT_ERR_INVALID_ARG, "nmbf %d outside [1, max_mbf = %d]", nmbf, plan->max_mbf);
  st = validate_basis(basis, nbasis);
  if (st != CFFT_OK) return st;
  GridState& gs = plan->grids[grid];
  hipStream_t s = (hipStream_t)stream;
  st = ensure_geometry(plan, gs, basis, nbasis, s);
  if (st != CFFT_OK) return st;
  hipError_t e;
  if (gs.d.contour == CFFT_CONTOUR_PARABOLIC) {
    st = ensure_ws(&plan->ws3, &plan->ws3_bytes, sizeof(double2) * spectra_direct_scratch_len(plan->geo_dev, nmbf),
                   "spectra scratch");
    if (st != CFFT_OK) return st;
    const Contour c{gs.d.gamma, 1, gs.d.beta_end};
    ProfScope ps(plan, 1, s);
    e = launch_spectra_direct(gs.x, gs.y, c, plan->geo_dev, (const double2*)q, nmbf, (double2*)plan->ws3, spec,
                              gs.d.precision, s);
  } else {
    st = ensure_ws(&plan->ws3, &plan->ws3_bytes, sizeof(double2) * spectra_scratch_len(gs.y, plan->geo_dev, nmbf),
                   "spectra scratch");
    if (st != CFFT_OK) return st;
    ProfScope ps(plan, 1, s);
    e = launch_spectra(gs.x, gs.y, gs.d.gamma, plan->geo_dev, gs.utab, (const double2*)q, nmbf, (double2*)plan->ws3,
                       spec, gs.d.precision, s);
  }
  if (e != hipSuccess) return hip_fail(e, "mbf_spectra launch");
  return check_finite(plan, spec, (size_t)8 * nmbf * gs.x.n * gs.y.n, gs.d.precision != CFFT_FP64, s);
}

cfft_status_t cfft_tabulate(cfft_plan_t plan, int32_t grid, const void* spec, int32_t nmbf, const void* g,
                            const int32_t* pairs, int32_t npairs, void* z, void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!spec || !g || !z) return fail(CFFT_ERR_INVALID_ARG, "spec, g or z is NULL");
  if (nmbf < 1 || nmbf > plan->max_mbf)
    return fail(CFFT_ERR_INVALID_ARG, "nmbf %d outside [1, max_mbf = %d]", nmbf, plan->max_mbf);
  st = validate_pairs(pairs, npairs, nmbf);
  if (st != CFFT_OK) return st;
  GridState& gs = plan->grids[grid];
  PassParams pp = pass_params(gs);
  const size_t n = (size_t)gs.x.n * gs.y.n;
  const size_t cbytes = pp.precision == CFFT_FP64 ? 16 : 8;
  const size_t per_pair = (size_t)inter_slots(pp) * n * cbytes;
  long long chunk = std::max<long long>(1, (workspace_limit_mb() << 20) / (long long)per_pair);
  chunk = std::min<long long>(chunk, std::min<long long>(npairs, kMaxPairsPerLaunch));
  const long long forced = env_ll("CFFT_PAIR_CHUNK", 0);
  if (forced > 0) chunk = std::min<long long>(chunk, forced);
  hipStream_t s = (hipStream_t)stream;
  // a workspace that does not fit the device's free memory takes fewer pairs per launch
  while ((st = ensure_ws(&plan->ws, &plan->ws_bytes, per_pair * (size_t)chunk, "pass workspace")) == CFFT_ERR_ALLOC &&
         chunk > 1 && !env_flag("CFFT_TEST_FAIL_ALLOC"))
    chunk /= 2;
  if (st != CFFT_OK) return st;
  if (forced <= 0) chunk = balanced_chunk(npairs, chunk);
  // twiddles in the transforms' compute precision
  const bool c64 = pp.precision == CFFT_FP64 || pp.hi_compute;
  const void* twx = c64 ? gs.tw64x : gs.tw32x;
  const void* twy = c64 ? gs.tw64y : gs.tw32y;
  std::vector<int> pm(npairs), pn(npairs);
  for (int i = 0; i < npairs; ++i) {
    pm[i] = pairs[2 * i];
    pn[i] = pairs[2 * i + 1];
  }
  // Schedules: `ck` pairs per chunk; with two lanes, even chunks run on one
  // plan-owned stream and odd chunks on the other, each with its own half of
  // the workspace, so that one lane's column pass overlaps the other lane's
  // row pass (the second lane starts once the first row pass is done).  The
  // lanes fork from and join back into the caller's stream through events,
  // which keeps the call capturable in a HIP graph.
  auto run_passes = [&](long long ck, int lanes, int tile) -> hipError_t {
    pp.col_tile = tile;
    pp.stream_out = stream_out(per_pair * (size_t)ck * (size_t)lanes);
    hipStream_t ls[2] = {s, s};
    if (lanes == 2) {
      hipError_t e = ensure_lanes(plan);
      if (e != hipSuccess) return e;
      ls[0] = plan->lane[0];
      ls[1] = plan->lane[1];
      e = hipEventRecord(plan->ev_fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(ls[0], plan->ev_fork, 0);
      if (e != hipSuccess) return e;
    }
    int chunk_id = 0;
    for (int p0 = 0; p0 < npairs; p0 += (int)ck, ++chunk_id) {
      const int np = (int)std::min<long long>(ck, npairs - p0);
      const int lane = lanes == 2 ? (chunk_id & 1) : 0;
      hipStream_t st2 = ls[lane];
      void* wsl = (char*)plan->ws + (size_t)lane * per_pair * (size_t)ck;
      hipError_t e;
      {
        ProfScope ps(plan, 2, st2);
        e = launch_row_pass(pp, (const double2*)g, spec, pm.data() + p0, pn.data() + p0, np, wsl,
                            twx, st2);
      }
      if (e != hipSuccess) return e;
      if (lanes == 2 && chunk_id == 0) {
        e = hipEventRecord(plan->ev_row0, st2);
        if (e == hipSuccess) e = hipStreamWaitEvent(ls[1], plan->ev_row0, 0);
        if (e != hipSuccess) return e;
      }
      {
        ProfScope ps(plan, 3, st2);
        e = launch_col_pass(pp, wsl, np, (char*)z + (size_t)p0 * n * cbytes, twy, st2);
      }
      if (e != hipSuccess) return e;
    }
    if (lanes == 2) {
      hipError_t e = hipEventRecord(plan->ev_join[0], ls[0]);
      if (e == hipSuccess) e = hipEventRecord(plan->ev_join[1], ls[1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->ev_join[0], 0);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->ev_join[1], 0);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // schedules forced from the environment (values outside the ranges are ignored)
  int lanes = 1;
  const long long env_lanes = env_ll("CFFT_LANES", 0);
  const bool forced_lanes = env_lanes == 1 || env_lanes == 2;
  if (forced_lanes) lanes = (int)env_lanes;
  int tile = kColTileDefault;
  const long long env_tile = env_ll("CFFT_COL_TILE", -1);
  const bool forced_tile = env_tile == kColTileDefault || env_tile == kColTileHalf ||
                           (env_tile == kColTileAltR && pp.y.n >= 1024);
  if (forced_tile) tile = (int)env_tile;
  auto lanes_ok = [&](long long ck) { return (npairs + ck - 1) / ck >= 2; };
  // With CFFT_FLAG_AUTOTUNE the first call per (grid, npairs) times every
  // (pair chunk, lanes, column tile) candidate (synchronously) and the plan
  // keeps the fastest.  Smaller chunks keep a chunk's intermediates resident
  // in the memory-side cache between the two passes; narrower column tiles
  // trade row-piece length for more, smaller blocks; the other number of
  // points per thread trades threads per transform for work per thread and
  // changes the widest tile that fits the LDS.
  if ((plan->flags & CFFT_FLAG_AUTOTUNE) && forced <= 0 && !forced_lanes && !forced_tile) {
    const long long key = (long long)grid * 1000003LL + npairs;
    auto it = plan->tuned.find(key);
    if (it == plan->tuned.end()) {
      std::vector<cfft_plan_s::Schedule> cands;
      for (long long c0 : {chunk, 32LL, 16LL, 8LL, 4LL, 2LL}) {
        if (c0 > chunk) continue;
        const long long c = balanced_chunk(npairs, c0);
        for (int l : {1, 2}) {
          if (l == 2 && !lanes_ok(c)) continue;
          if (l == 2 && per_pair * (size_t)c * 2 > plan->ws_bytes) {
            // a two-lane workspace that does not fit leaves the candidate out
            st = ensure_ws(&plan->ws, &plan->ws_bytes, per_pair * (size_t)c * 2, "pass workspace");
            if (st == CFFT_ERR_ALLOC) {
              st = ensure_ws(&plan->ws, &plan->ws_bytes, per_pair * (size_t)chunk, "pass workspace");
              if (st != CFFT_OK) return st;
              continue;
            }
            if (st != CFFT_OK) return st;
          }
          for (int w : {kColTileDefault, kColTileHalf, kColTileAltR}) {
            if (w == kColTileAltR && pp.y.n < 1024) continue;
            bool dup = false;
            for (const auto& x : cands) dup = dup || (x.chunk == c && x.lanes == l && x.tile == w);
            if (!dup) cands.push_back({c, l, w});
          }
        }
      }
      hipEvent_t ea, eb;
      hipError_t e = hipEventCreate(&ea);
      if (e == hipSuccess) e = hipEventCreate(&eb);
      if (e != hipSuccess) return hip_fail(e, "autotune events");
      cfft_plan_s::Schedule best{chunk, 1, kColTileDefault};
      float best_ms = 3.4e38f;
      for (const auto& c : cands) {
        e = run_passes(c.chunk, c.lanes, c.tile);  // warm-up
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventRecord(ea, s);
        if (e == hipSuccess) e = run_passes(c.chunk, c.lanes, c.tile);
        if (e == hipSuccess) e = run_passes(c.chunk, c.lanes, c.tile);
        if (e == hipSuccess) e = hipEventRecord(eb, s);
        if (e == hipSuccess) e = hipEventSynchronize(eb);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
        if (e != hipSuccess) break;
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
      (void)hipEventDestroy(ea);
      (void)hipEventDestroy(eb);
      if (e != hipSuccess) return hip_fail(e, "autotune");
      it = plan->tuned.emplace(key, best).first;
    }
    chunk = it->second.chunk;
    lanes = it->second.lanes;
    tile = it->second.tile;
  }
  if (lanes == 2 && !lanes_ok(chunk)) lanes = 1;
  if (lanes == 2) {
    st = ensure_ws(&plan->ws, &plan->ws_bytes, per_pair * (size_t)chunk * 2, "pass workspace");
    if (st != CFFT_OK) return st;
  }
  {
    hipError_t e = run_passes(chunk, lanes, tile);
    if (e != hipSuccess) return hip_fail(e, "pass launch");
  }
  return check_finite(plan, z, 2 * n * (size_t)npairs, pp.precision != CFFT_FP64, s);
}

cfft_status_t cfft_tabulate_noalloc(cfft_plan_t plan, int32_t grid, const void* spec, int32_t nmbf, const void* g,
                                    const int32_t* pairs, int32_t npairs, void* z, void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!spec || !g || !z) return fail(CFFT_ERR_INVALID_ARG, "spec, g or z is NULL");
  if (nmbf < 1 || nmbf > plan->max_mbf)
    return fail(CFFT_ERR_INVALID_ARG, "nmbf %d outside [1, max_mbf = %d]", nmbf, plan->max_mbf);
  st = validate_pairs(pairs, npairs, nmbf);
  if (st != CFFT_OK) return st;
  GridState& gs = plan->grids[grid];
  PassParams pp = pass_params(gs);
  const size_t n = (size_t)gs.x.n * gs.y.n;
  const size_t cbytes = pp.precision == CFFT_FP64 ? 16 : 8;
  const size_t per_pair = (size_t)inter_slots(pp) * n * cbytes;
  if (per_pair > kNoAllocScratchBytes)
    return fail(CFFT_ERR_UNSUPPORTED,
                "grid %d needs %zu bytes of intermediates per pair; the allocation-free entry point holds %zu",
                grid, per_pair, kNoAllocScratchBytes);
  void* ws = scratch_of(plan->device);
  if (!ws) return fail(CFFT_ERR_HIP, "scratch address of device %d not resolved", plan->device);
  const int chunk = (int)balanced_chunk(
      npairs, (long long)std::min<size_t>(kNoAllocScratchBytes / per_pair, (size_t)kMaxPairsPerLaunch));
  pp.stream_out = stream_out(per_pair * (size_t)std::min(chunk, (int)npairs));
  const bool c64 = pp.precision == CFFT_FP64 || pp.hi_compute;
  const void* twx = c64 ? gs.tw64x : gs.tw32x;
  const void* twy = c64 ? gs.tw64y : gs.tw32y;
  hipStream_t s = (hipStream_t)stream;
  // every intermediate the column pass reads is written by the row pass of
  // the same chunk first, so the scratch needs no clearing
  int pm[kMaxPairsPerLaunch], pn[kMaxPairsPerLaunch];
  for (int p0 = 0; p0 < npairs; p0 += chunk) {
    const int np = std::min(chunk, npairs - p0);
    for (int i = 0; i < np; ++i) {
      pm[i] = pairs[2 * (p0 + i)];
      pn[i] = pairs[2 * (p0 + i) + 1];
    }
    hipError_t e;
    {
      ProfScope ps(plan, 2, s);
      e = launch_row_pass(pp, (const double2*)g, spec, pm, pn, np, ws, twx, s);
    }
    if (e == hipSuccess) {
      ProfScope ps(plan, 3, s);
      e = launch_col_pass(pp, ws, np, (char*)z + (size_t)p0 * n * cbytes, twy, s);
    }
    if (e != hipSuccess) return hip_fail(e, "pass launch");
  }
  return check_finite(plan, z, 2 * n * (size_t)npairs, pp.precision != CFFT_FP64, s);
}

static cfft_status_t lookup_common(cfft_plan_t plan, int32_t grid, const void* z, int32_t npairs, const double* pts,
                                   int32_t npts, void* out, void* stream, bool quadratic) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!z || !pts || !out) return fail(CFFT_ERR_INVALID_ARG, "z, pts or out is NULL");
  if (npairs < 1 || npairs > 4096) return fail(CFFT_ERR_INVALID_ARG, "npairs %d outside [1, 4096]", npairs);
  if (npts < 1 || (long long)npts * npairs > (1LL << 31) - 1)
    return fail(CFFT_ERR_INVALID_ARG, "npts %d invalid", npts);
  GridState& gs = plan->grids[grid];
  hipError_t e;
  {
    ProfScope ps(plan, 4, (hipStream_t)stream);
    e = quadratic ? launch_lookup_quadratic(pass_params(gs), z, npairs, pts, npts, (double2*)out, (hipStream_t)stream)
                  : launch_lookup(pass_params(gs), z, npairs, pts, npts, (double2*)out, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "lookup launch");
  return CFFT_OK;
}

cfft_status_t cfft_lookup_quadratic(cfft_plan_t plan, int32_t grid, const void* z, int32_t npairs, const double* pts,
                                    int32_t npts, void* out, void* stream) {
  return lookup_common(plan, grid, z, npairs, pts, npts, out, stream, true);
}

cfft_status_t cfft_lookup(cfft_plan_t plan, int32_t grid, const void* z, int32_t npairs, const double* pts,
                          int32_t npts, void* out, void* stream) {
  return lookup_common(plan, grid, z, npairs, pts, npts, out, stream, false);
}

static cfft_status_t fill_common(cfft_plan_t plan, int32_t grid, const void* z, const int32_t* pairs, int32_t npairs,
                                 int32_t nmbf, const double* pos, int32_t nelem, int32_t order, void* out,
                                 const void* dout, void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!pos || !out || (!dout && !z)) return fail(CFFT_ERR_INVALID_ARG, "a table, pos or output pointer is NULL");
  if (nmbf < 1 || nmbf > kFillMaxMbf) return fail(CFFT_ERR_INVALID_ARG, "nmbf %d outside [1, %d]", nmbf, kFillMaxMbf);
  if (order != 1 && order != 2) return fail(CFFT_ERR_INVALID_ARG, "order %d is not 1 or 2", order);
  if (nelem < 1 || (long long)nelem * nmbf > 65535)
    return fail(CFFT_ERR_INVALID_ARG, "nelem %d invalid (nelem * nmbf must be <= 65535)", nelem);
  st = validate_pairs(pairs, npairs, nmbf);
  if (st != CFFT_OK) return st;
  short slot[kFillMaxMbf * kFillMaxMbf];
  for (short& v : slot) v = -1;
  for (int k = 0; k < npairs; ++k) {
    short& v = slot[pairs[2 * k] * kFillMaxMbf + pairs[2 * k + 1]];
    if (v >= 0) return fail(CFFT_ERR_INVALID_ARG, "pair (%d, %d) listed twice", pairs[2 * k], pairs[2 * k + 1]);
    v = (short)k;
  }
  GridState& gs = plan->grids[grid];
  if (dout && gs.d.precision != CFFT_FP64) return fail(CFFT_ERR_UNSUPPORTED, "the fill adjoint needs an FP64 grid");
  if (nelem == 1) return CFFT_OK;   // only the self block, which is not written
  hipError_t e;
  if (dout) {
    const size_t need = scatter_workspace_bytes((long long)nelem * nelem);
    if (need == 0) return fail(CFFT_ERR_UNSUPPORTED, "fill adjoint of %d elements: too many element pairs", nelem);
    st = ensure_ws(&plan->ws4, &plan->ws4_bytes, need, "scatter workspace");
    if (st != CFFT_OK) return st;
    int pm[kScatterMaxPairs], pn[kScatterMaxPairs];
    for (int k = 0; k < npairs; ++k) {
      pm[k] = pairs[2 * k];
      pn[k] = pairs[2 * k + 1];
    }
    ProfScope ps(plan, 4, (hipStream_t)stream);
    e = launch_fill_backward(pass_params(gs), pm, pn, npairs, nmbf, pos, nelem, order, (const double2*)dout,
                             (double2*)out, plan->ws4, (hipStream_t)stream);
  } else {
    ProfScope ps(plan, 4, (hipStream_t)stream);
    e = launch_fill(pass_params(gs), z, slot, nmbf, pos, nelem, order, (double2*)out, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "fill launch");
  return CFFT_OK;
}

cfft_status_t cfft_fill(cfft_plan_t plan, int32_t grid, const void* z, const int32_t* pairs, int32_t npairs,
                        int32_t nmbf, const double* pos, int32_t nelem, int32_t order, void* out, void* stream) {
  if (!z) {
    g_last_error.clear();
    return fail(CFFT_ERR_INVALID_ARG, "z is NULL");
  }
  return fill_common(plan, grid, z, pairs, npairs, nmbf, pos, nelem, order, out, nullptr, stream);
}

cfft_status_t cfft_fill_backward(cfft_plan_t plan, int32_t grid, const void* dout, const int32_t* pairs,
                                 int32_t npairs, int32_t nmbf, const double* pos, int32_t nelem, int32_t order,
                                 void* dz, void* stream) {
  if (!dout) {
    g_last_error.clear();
    return fail(CFFT_ERR_INVALID_ARG, "dout is NULL");
  }
  return fill_common(plan, grid, nullptr, pairs, npairs, nmbf, pos, nelem, order, dz, dout, stream);
}

static cfft_status_t lookup_backward_common(cfft_plan_t plan, int32_t grid, const void* dout, int32_t npairs,
                                            const double* pts, int32_t npts, void* dz, void* stream, bool quadratic) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!dout || !pts || !dz) return fail(CFFT_ERR_INVALID_ARG, "dout, pts or dz is NULL");
  if (npairs < 1 || npairs > 4096) return fail(CFFT_ERR_INVALID_ARG, "npairs %d outside [1, 4096]", npairs);
  if (npts < 1 || (long long)npts * npairs > (1LL << 31) - 1)
    return fail(CFFT_ERR_INVALID_ARG, "npts %d invalid", npts);
  GridState& gs = plan->grids[grid];
  if (gs.d.precision != CFFT_FP64) return fail(CFFT_ERR_UNSUPPORTED, "lookup adjoint needs an FP64 grid");
  const size_t need = scatter_workspace_bytes(npts);
  if (need == 0) return fail(CFFT_ERR_UNSUPPORTED, "lookup adjoint of %d points: too many points", npts);
  st = ensure_ws(&plan->ws4, &plan->ws4_bytes, need, "scatter workspace");
  if (st != CFFT_OK) return st;
  hipError_t e = launch_lookup_backward(pass_params(gs), (const double2*)dout, npairs, pts, npts, (double2*)dz,
                                        quadratic, plan->ws4, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lookup adjoint launch");
  return CFFT_OK;
}

cfft_status_t cfft_lookup_backward(cfft_plan_t plan, int32_t grid, const void* dout, int32_t npairs,
                                   const double* pts, int32_t npts, void* dz, void* stream) {
  return lookup_backward_common(plan, grid, dout, npairs, pts, npts, dz, stream, false);
}

cfft_status_t cfft_lookup_quadratic_backward(cfft_plan_t plan, int32_t grid, const void* dout, int32_t npairs,
                                             const double* pts, int32_t npts, void* dz, void* stream) {
  return lookup_backward_common(plan, grid, dout, npairs, pts, npts, dz, stream, true);
}

cfft_status_t cfft_backward(cfft_plan_t plan, int32_t grid, const void* dz, double eps_r, double tan_delta, double h,
                            const cfft_basis_t* basis, int32_t nbasis, const void* q, int32_t nmbf,
                            const int32_t* pairs, int32_t npairs, const void* g, const void* spec, double* grad_sub,
                            void* grad_q, void* stream) {
  g_last_error.clear();
  cfft_status_t st = check_plan(plan, grid);
  if (st != CFFT_OK) return st;
  if (!dz || !q || !g || !spec || !grad_sub || !grad_q)
    return fail(CFFT_ERR_INVALID_ARG, "dz, q, g, spec, grad_sub or grad_q is NULL");
  if (!(std::isfinite(eps_r) && eps_r >= 1.0)) return fail(CFFT_ERR_INVALID_ARG, "eps_r must be finite and >= 1");
  if (!(std::isfinite(tan_delta) && tan_delta >= 0.0))
    return fail(CFFT_ERR_INVALID_ARG, "tan_delta must be finite and >= 0");
  if (!(std::isfinite(h) && h > 0.0)) return fail(CFFT_ERR_INVALID_ARG, "h must be finite and > 0");
  if (nmbf < 1 || nmbf > plan->max_mbf)
    return fail(CFFT_ERR_INVALID_ARG, "nmbf %d outside [1, max_mbf = %d]", nmbf, plan->max_mbf);
  st = validate_basis(basis, nbasis);
  if (st != CFFT_OK) return st;
  st = validate_pairs(pairs, npairs, nmbf);
  if (st != CFFT_OK) return st;
  GridState& gs = plan->grids[grid];
  if (gs.d.precision != CFFT_FP64) return fail(CFFT_ERR_UNSUPPORTED, "the adjoint needs an FP64 grid");
  if (gs.d.contour != CFFT_CONTOUR_RAY) return fail(CFFT_ERR_UNSUPPORTED, "the adjoint needs the ray contour");
  hipStream_t s = (hipStream_t)stream;
  st = ensure_geometry(plan, gs, basis, nbasis, s);
  if (st != CFFT_OK) return st;
  if (adj_spectra_lds_bytes(plan->geo_dev, nmbf) > kMaxDynamicLds)
    return fail(CFFT_ERR_UNSUPPORTED,
                "the spectra adjoint keeps %d MBFs x %d distinct x-centres in LDS: %zu bytes, more than %zu", nmbf,
                plan->geo_dev.total_p, adj_spectra_lds_bytes(plan->geo_dev, nmbf), kMaxDynamicLds);
  const PassParams pp = pass_params(gs);
  const size_t n = (size_t)gs.x.n * gs.y.n;
  const size_t per_pair = (size_t)inter_slots(pp) * n * 16 + n * 16;   // intermediates + gH
  long long chunk = std::max<long long>(1, (workspace_limit_mb() << 20) / (long long)per_pair);
  chunk = std::min<long long>(chunk, std::min<long long>(npairs, kMaxPairsPerLaunch));
  const long long forced = env_ll("CFFT_PAIR_CHUNK", 0);
  if (forced > 0) chunk = std::min<long long>(chunk, forced);
  else chunk = balanced_chunk(npairs, chunk);
  const GreenParams gp = green_params(gs, eps_r, tan_delta, h);
  const int green_blocks = std::min(1024, (green_threads(gp) + 255) / 256);
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t b_gg = al(3 * n * 16), b_gs = al((size_t)nmbf * 4 * n * 16);
  const size_t b_row = al(adj_spectra_scratch(gs.y, plan->geo_dev, nmbf));
  const size_t b_part = al(sizeof(double) * 2 * green_blocks);
  st = ensure_ws(&plan->ws, &plan->ws_bytes, per_pair * (size_t)chunk, "adjoint workspace");
  if (st != CFFT_OK) return st;
  st = ensure_ws(&plan->ws2, &plan->ws2_bytes, b_gg + b_gs + b_row + b_part, "adjoint scratch");
  if (st != CFFT_OK) return st;
  char* w2 = (char*)plan->ws2;
  double2* gg = (double2*)w2;
  double2* gspec = (double2*)(w2 + b_gg);
  double2* rowacc = (double2*)(w2 + b_gg + b_gs);
  double* partial = (double*)(w2 + b_gg + b_gs + b_row);
  double2* inter = (double2*)plan->ws;
  double2* gi = (double2*)((char*)plan->ws + (size_t)inter_slots(pp) * n * 16 * chunk);
  std::vector<int> pm(npairs), pn(npairs);
  for (int i = 0; i < npairs; ++i) {
    pm[i] = pairs[2 * i];
    pn[i] = pairs[2 * i + 1];
  }
  for (int p0 = 0; p0 < npairs; p0 += (int)chunk) {
    const int np = (int)std::min<long long>(chunk, npairs - p0);
    hipError_t e;
    {
      ProfScope ps(plan, 5, s);
      e = launch_adj_col_pass(pp, (const double2*)dz + (size_t)p0 * n, np, inter, gs.tw64y, s);
    }
    if (e == hipSuccess) {
      ProfScope ps(plan, 6, s);
      e = launch_adj_row_pass(pp, inter, np, gi, gs.tw64x, s);
    }
    if (e == hipSuccess) {
      ProfScope ps(plan, 7, s);
      e = launch_adj_integrand(pp, gi, (const double2*)g, (const double2*)spec, pm.data() + p0, pn.data() + p0, np,
                               nmbf, gg, gspec, p0 > 0 ? 1 : 0, s);
    }
    if (e != hipSuccess) return hip_fail(e, "adjoint pass launch");
  }
  hipError_t e;
  {
    ProfScope ps(plan, 8, s);
    e = launch_adj_green(gp, gg, partial, green_blocks, s);
    if (e == hipSuccess) e = launch_reduce_sum(partial, green_blocks, 2, grad_sub, s);
  }
  if (e == hipSuccess) {
    ProfScope ps(plan, 9, s);
    e = launch_adj_spectra(gs.x, gs.y, plan->geo_dev, gs.utab, gspec, nmbf, rowacc, (double2*)grad_q, s);
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint reduction launch");
  return CFFT_OK;
}

}  // extern "C"
