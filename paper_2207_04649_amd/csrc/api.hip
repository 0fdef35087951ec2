// The C ABI (include/dpc.h): argument checks, the exact cut-off, the grid plan,
// the workspace layout and the launch sequence of each call.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"
#include "prof.h"

#include <mutex>
#include <vector>

namespace dpc {

// ---- optional kernel timing ----
namespace {
struct ProfRec {
  int kernel;
  hipEvent_t begin, end;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;
std::vector<ProfRec> g_prof_open;  // begins awaiting their end, per kernel id
int g_prof_level = 0;
// work counters of the last dependent search (profiling level 2)
int64_t g_work[4] = {0, 0, 0, 0};
const char *kProfNames[kProfCount] = {"grid_build", "density", "rank_keys", "rank_sort", "search",
                                      "ringk", "peaks", "finish", "label"};
}  // namespace

bool prof_on() { return g_prof_level > 0; }

void prof_mark(hipStream_t s, int kernel, bool begin) {
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (begin) {
    g_prof_open.push_back({kernel, e, nullptr});
    return;
  }
  for (size_t i = g_prof_open.size(); i-- > 0;) {
    if (g_prof_open[i].kernel == kernel) {
      ProfRec r = g_prof_open[i];
      r.end = e;
      g_prof_open.erase(g_prof_open.begin() + long(i));
      g_prof_recs.push_back(r);
      return;
    }
  }
  hipEventDestroy(e);
}

namespace {

thread_local std::string g_last_error;

dpc_status fail(dpc_status code, const char *msg) {
  g_last_error = msg;
  return code;
}

dpc_status device_fail(hipError_t e, const char *where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return DPC_EDEVICE;
}

// ceil(d^2) without rounding error: d*d = h + l exactly (error-free product).
int64_t cutoff_square(double d) {
  if (!std::isfinite(d) || !(d > 0.0)) return -1;
  if (d >= 524288.0) return int64_t(1) << 38;  // beyond every in-range squared distance
  const double h = d * d;
  const double l = std::fma(d, d, -h);
  int64_t R;
  if (h == std::floor(h))
    R = int64_t(h) + (l > 0.0 ? 1 : 0);
  else
    R = int64_t(std::ceil(h));
  return R < 1 ? 1 : R;
}

int64_t isqrt64(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = int64_t(std::sqrt(double(v)));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Largest c with c^d <= cap.
int64_t iroot(int64_t cap, int d) {
  int64_t c = int64_t(std::pow(double(cap), 1.0 / d));
  auto fits = [&](int64_t v) {
    __int128 r = 1;
    for (int i = 0; i < d; ++i) r *= v;
    return r <= cap;
  };
  while (c > 1 && !fits(c)) --c;
  while (fits(c + 1)) ++c;
  return c;
}

// Largest window extent E per dimension for which the packed 16-bit path is exact:
// |dx| <= E - 1 < 2^15 and d * (E - 1)^2 <= 2^31 - 1.
int64_t p16_extent(int d) {
  int64_t m = isqrt64(((int64_t(1) << 31) - 1) / d);
  if (m > 32767) m = 32767;
  return m + 1;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Cells per ball half-extent for each dimension (finer cells clip the windows
// closer to the d_cut-ball; the table grows as their d-th power).
int default_subdivision(int d) { return d <= 2 ? 4 : (d == 3 ? 2 : 1); }

bool make_plan(int64_t n, int32_t d, double d_cut, Plan *out) {
  if (n < 1 || n >= DPC_MAX_POINTS || d < 1 || d > DPC_MAX_DIM) return false;
  const int64_t R = cutoff_square(d_cut);
  if (R < 1) return false;
  Plan p;
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  p.d = d;
  p.words = (d + 1) / 2;
  p.R = R;
  int64_t L0 = isqrt64(R - 1);
  if (L0 < 1) L0 = 1;
  if (L0 > DPC_COORD_LIMIT) L0 = DPC_COORD_LIMIT;
  p.L0 = int32_t(L0);
  int S = default_subdivision(d);
  if (const char *env = std::getenv("DPC_SUBDIV")) {  // tuning override
    const int v = std::atoi(env);
    if (v >= 1 && v <= 16) S = v;
  }
  const int64_t nc_max = iroot(kTableMax, d);
  int64_t L = 1, nc = 1;
  for (;; --S) {
    L = (L0 + S - 1) / S;
    if (L < 1) L = 1;
    nc = (DPC_COORD_LIMIT + L - 1) / L;
    if (nc <= nc_max || S == 1) break;
  }
  if (nc > nc_max) {  // coarsen: any side >= floor(sqrt(R - 1)) stays exact
    L = (DPC_COORD_LIMIT + nc_max - 1) / nc_max;
    nc = (DPC_COORD_LIMIT + L - 1) / L;
  }
  p.L = int32_t(L);
  p.nc = int32_t(nc);
  p.K0 = int32_t((L0 + L - 1) / L);
  // Strip width: a window of radius K around a strip spans at most (wc + 2K)
  // cells in the last dimension; the packed 16-bit path needs that below E.
  const int64_t E = p16_extent(d);
  auto p16_ok = [&](int64_t K, int64_t wc) { return wc >= 1 && (wc + 2 * K) * L <= E && (2 * K + 1) * L <= E; };
  const int64_t wc16 = E / L - 2 * int64_t(p.K0);
  if (p16_ok(p.K0, wc16)) {
    p.mode = kModeP16;
    p.wc = int32_t(wc16 < nc ? wc16 : nc);
  } else {
    p.mode = kModeI64;
    p.wc = int32_t(nc);
  }
  if (const char *env = std::getenv("DPC_STRIP_CELLS")) {  // tuning override (narrower only)
    int64_t v = std::atoll(env);
    if (v >= 1 && v < p.wc) p.wc = int32_t(v);
  }
  // Dependent-search stages: window radii in cells and tasks gathered per wave
  // (more as fewer points stay open); a later stage is dropped when its window
  // has more than 4096 rows.
  int radii[4] = {1, 3, 0, 0}, groups[4] = {1, 4, 0, 0}, nst = 2;
  if (const char *env = std::getenv("DPC_STAGES")) {  // tuning override: "K:group,K:group,..."
    int k = 0;
    for (const char *c = env; *c && k < 4;) {
      int K = 0, g = 1;
      if (std::sscanf(c, "%d:%d", &K, &g) < 1 || K < 1 || K > 64 || g < 1 || g > 64) break;
      radii[k] = K;
      groups[k] = g;
      ++k;
      c = std::strchr(c, ',');
      if (!c) break;
      ++c;
    }
    if (k > 0) nst = k;
  }
  p.nstages = 0;
  for (int st = 0; st < nst; ++st) {
    const int K = radii[st];
    int64_t rows = 1;
    for (int t = 0; t < d - 1; ++t) rows *= 2 * K + 1;
    if (st > 0 && rows > 4096) break;
    p.stageK[p.nstages] = K;
    p.stageGroup[p.nstages] = groups[st];
    p.stageMode[p.nstages] = p16_ok(K, p.wc) ? kModeP16 : kModeI64;
    ++p.nstages;
  }
  p.ring_cap = kRingCostCap;
  if (const char *env = std::getenv("DPC_RING_CAP")) {  // tuning override
    const int v = std::atoi(env);
    if (v >= 1 && v <= 1 << 20) p.ring_cap = v;
  }
  p.nsx = int32_t((nc + p.wc - 1) / p.wc);
  p.ncells = ipow(nc, d);
  p.nrows = ipow(nc, d - 1);
  p.nstrips = p.nrows * p.nsx;
  p.max_tasks = n / kQueryChunk + p.nstrips + 1;

  const int64_t scan_max = std::max(std::max(p.ncells + 1, p.nstrips + 1), n + 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  p.o_hdr = take(sizeof(DevHeader));
  p.o_cnt = take(size_t(p.ncells + 1) * 4);
  p.o_bsum = take(size_t(scan_max / kScanTile + 2) * 4);
  p.o_key = take(size_t(n) * 4);
  p.o_slot = take(size_t(n) * 4);
  p.o_spts = take(size_t(n) * d * 4);
  p.o_spk = take(size_t(n) * p.words * 4);
  p.o_sid = take(size_t(n) * 4);
  p.o_sK = take(size_t(n) * 8);
  p.o_tcnt = take(size_t(p.nstrips + 1) * 4);
  p.o_tasks = take(size_t(p.max_tasks) * 16);
  p.o_rcnt = take(size_t(n + 1) * 4);
  p.o_rpts = take(size_t(n) * d * 4);
  p.o_rid = take(size_t(n) * 4);
  p.o_best = take(size_t(n) * 8);
  p.o_unres = take(size_t(n + 1) * 4);  // + a spare slot for lanes that append nothing
  p.o_peaks = take(size_t(n + 1) * 4);
  p.o_flag = take(size_t(n));
  p.total = o;
  *out = p;
  return true;
}

dpc_status check_common(const int32_t *pts, int64_t n, int32_t d, double d_cut, void *ws, size_t ws_bytes,
                        Plan *p) {
  if (!pts || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (n < 1 || n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (d < 1 || d > DPC_MAX_DIM) return fail(DPC_EINVAL, "d must be in [1, 8]");
  if (!std::isfinite(d_cut) || !(d_cut > 0.0)) return fail(DPC_EINVAL, "d_cut must be finite and > 0");
  if (!make_plan(n, d, d_cut, p)) return fail(DPC_EINVAL, "no plan for these sizes");
  if (ws_bytes < p->total) return fail(DPC_EWORKSPACE, "workspace smaller than dpc_workspace_bytes()");
  return DPC_OK;
}

dpc_status run_density(const Plan &p, const Ws &w, const int32_t *pts, int32_t *rho, hipStream_t s) {
  hipError_t e;
  {
    ProfScope ps(s, kProfGrid);
    e = build_grid(p, w, pts, s);
  }
  if (e != hipSuccess) return device_fail(e, "grid build");
  ProfScope ps(s, kProfDensity);
  e = launch_density(p, w, rho, s);
  if (e != hipSuccess) return device_fail(e, "density kernel");
  return DPC_OK;
}

// Profiling level 2: tasks, points left open by the search stages, points sent
// to the prefix scan and the candidates those scans cover (synchronises).
hipError_t record_work(const Plan &p, const Ws &w, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  DevHeader h;
  if ((e = hipMemcpy(&h, w.hdr, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  std::vector<uint32_t> peaks(h.n_peaks), rstart(size_t(p.n) + 1);
  std::vector<uint64_t> sK(size_t(p.n));
  if (h.n_peaks && (e = hipMemcpy(peaks.data(), w.peaks, h.n_peaks * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return e;
  if ((e = hipMemcpy(sK.data(), w.sK, sK.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if ((e = hipMemcpy(rstart.data(), w.rcnt, rstart.size() * 4, hipMemcpyDeviceToHost)) != hipSuccess) return e;
  int64_t prefix = 0;
  for (uint32_t q : peaks) prefix += rstart[size_t(p.n - int64_t(sK[q] >> 32) + 1)];
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_work[0] = h.ntasks;
  g_work[1] = h.n_unres;
  g_work[2] = h.n_peaks;
  g_work[3] = prefix;
  return hipSuccess;
}

dpc_status run_dependent(const Plan &p, const Ws &w, const int32_t *pts, const int32_t *rho, int32_t *dep,
                         double *delta, bool reuse, hipStream_t s) {
  hipError_t e;
  if (!reuse) {
    ProfScope ps(s, kProfGrid);
    if ((e = build_grid(p, w, pts, s)) != hipSuccess) return device_fail(e, "grid build");
  } else if ((e = reset_counters(w.hdr, false, s)) != hipSuccess) {
    return device_fail(e, "reset");
  }
  {
    ProfScope ps(s, kProfRankKeys);
    if ((e = gather_rank_keys(p, w, rho, s)) != hipSuccess) return device_fail(e, "rank keys");
  }
  {
    ProfScope ps(s, kProfRankSort);
    if ((e = rank_sort(p, w, s)) != hipSuccess) return device_fail(e, "rank sort");
  }
  if ((e = launch_dependent(p, w, dep, delta, s)) != hipSuccess) return device_fail(e, "dependent kernels");
  if (g_prof_level >= 2 && (e = record_work(p, w, s)) != hipSuccess) return device_fail(e, "work counters");
  return DPC_OK;
}

}  // namespace
}  // namespace dpc

using namespace dpc;

extern "C" {

int32_t dpc_version(void) { return 100; }

const char *dpc_last_error(void) { return g_last_error.c_str(); }

int64_t dpc_cutoff_square(double d_cut) { return cutoff_square(d_cut); }

size_t dpc_workspace_bytes(int64_t n, int32_t d, double d_cut) {
  Plan p;
  return make_plan(n, d, d_cut, &p) ? p.total : 0;
}

dpc_status dpc_plan(int64_t n, int32_t d, double d_cut, dpc_plan_info *out) {
  Plan p;
  if (!out) return fail(DPC_EINVAL, "null pointer argument");
  if (!make_plan(n, d, d_cut, &p)) return fail(DPC_EINVAL, "no plan for these sizes");
  out->R = p.R;
  out->cell_side = p.L;
  out->cells_per_dim = p.nc;
  out->cells = p.ncells;
  out->strip_cells = p.wc;
  out->strips = p.nstrips;
  out->max_tasks = p.max_tasks;
  out->mode = p.mode;
  out->workspace_bytes = int64_t(p.total);
  out->window_radius = p.K0;
  out->stages = p.nstages;
  return DPC_OK;
}

dpc_status dpc_density(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t *rho, void *ws,
                       size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!rho) return fail(DPC_EINVAL, "null pointer argument");
  const Ws w = resolve(p, ws);
  hipError_t e = clear_status(w.hdr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "status reset");
  return run_density(p, w, pts, rho, static_cast<hipStream_t>(stream));
}

dpc_status dpc_dependent(const int32_t *pts, int64_t n, int32_t d, double d_cut, const int32_t *rho,
                         int32_t *dep, double *delta, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!rho || !dep || !delta) return fail(DPC_EINVAL, "null pointer argument");
  if (flags & ~DPC_REUSE_GRID) return fail(DPC_EINVAL, "unknown flag");
  const Ws w = resolve(p, ws);
  hipError_t e = clear_status(w.hdr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "status reset");
  return run_dependent(p, w, pts, rho, dep, delta, (flags & DPC_REUSE_GRID) != 0, static_cast<hipStream_t>(stream));
}

dpc_status dpc_label(int64_t n, const int32_t *rho, const int32_t *dep, const double *delta, int32_t rho_min,
                     double delta_min, int32_t *label, int64_t *ncenters, void *ws, size_t ws_bytes,
                     void *stream) {
  if (!rho || !dep || !delta || !label || !ncenters || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (n < 1 || n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(delta_min)) return fail(DPC_EINVAL, "delta_min is NaN");
  if (ws_bytes < DPC_LABEL_WS_BYTES) return fail(DPC_EWORKSPACE, "workspace smaller than DPC_LABEL_WS_BYTES");
  hipError_t e = clear_status(static_cast<DevHeader *>(ws), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "status reset");
  ProfScope ps(static_cast<hipStream_t>(stream), kProfLabel);
  e = launch_label(n, rho, dep, delta, rho_min, delta_min, label, ncenters, static_cast<DevHeader *>(ws),
                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "label kernels");
  return DPC_OK;
}

dpc_status dpc_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                   int32_t *rho, int32_t *dep, double *delta, int32_t *label, int64_t *ncenters, void *ws,
                   size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!rho || !dep || !delta || !label || !ncenters) return fail(DPC_EINVAL, "null pointer argument");
  if (rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(delta_min) || !(delta_min > d_cut)) return fail(DPC_EINVAL, "delta_min must exceed d_cut");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = resolve(p, ws);
  hipError_t e0 = clear_status(w.hdr, s);
  if (e0 != hipSuccess) return device_fail(e0, "status reset");
  if ((st = run_density(p, w, pts, rho, s)) != DPC_OK) return st;
  if ((st = run_dependent(p, w, pts, rho, dep, delta, true, s)) != DPC_OK) return st;
  ProfScope ps(s, kProfLabel);
  hipError_t e = launch_label(n, rho, dep, delta, rho_min, delta_min, label, ncenters, w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "label kernels");
  return DPC_OK;
}

void dpc_profile_enable(int32_t level) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_level = level < 0 ? 0 : level;
}

int32_t dpc_profile_report(char *buf, size_t len) {
  double ms[kProfCount] = {0};
  int64_t calls[kProfCount] = {0};
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof_recs);
  }
  for (const ProfRec &r : recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.end) == hipSuccess && hipEventElapsedTime(&t, r.begin, r.end) == hipSuccess) {
      ms[r.kernel] += t;
      calls[r.kernel] += 1;
    }
    hipEventDestroy(r.begin);
    hipEventDestroy(r.end);
  }
  std::string out = "{";
  for (int k = 0; k < kProfCount; ++k) {
    char item[128];
    std::snprintf(item, sizeof(item), "%s\"%s\": [%lld, %.6f]", k ? ", " : "", kProfNames[k],
                  static_cast<long long>(calls[k]), ms[k]);
    out += item;
  }
  {
    char item[192];
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::snprintf(item, sizeof(item), ", \"work\": {\"tasks\": %lld, \"open\": %lld, \"peaks\": %lld, "
                  "\"peak_prefix\": %lld}", static_cast<long long>(g_work[0]), static_cast<long long>(g_work[1]),
                  static_cast<long long>(g_work[2]), static_cast<long long>(g_work[3]));
    out += item;
  }
  out += "}";
  if (buf && len) {
    std::strncpy(buf, out.c_str(), len - 1);
    buf[len - 1] = 0;
  }
  return int32_t(out.size());
}

dpc_status dpc_sync_status(void *ws, void *stream) {
  if (!ws) return fail(DPC_EINVAL, "null pointer argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(e, "stream synchronize");
  uint32_t status = 0;
  e = hipMemcpy(&status, ws, sizeof(status), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(e, "status read");
  if (status) {
    const uint32_t zero = 0;
    e = hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "status clear");
  }
  if (status & 1u) return fail(DPC_ERANGE, "a coordinate was outside [0, 2^17) and was clamped");
  if (status & 2u) return fail(DPC_EINVAL, "inconsistent rho or dep input (clamped or cut)");
  g_last_error.clear();
  return DPC_OK;
}

}  // extern "C"
