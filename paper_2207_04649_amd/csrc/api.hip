// The C ABI (include/dpc.h): argument checks, the exact cut-off, the grid plan,
// the workspace layout and the launch sequence of each call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
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
int64_t g_work[5] = {0, 0, 0, 0, 0};
// candidate distance tests of the last call's density, window search, ring search and prefix scan
int64_t g_tests[4] = {0, 0, 0, 0};
const char *kProfNames[kProfCount] = {"grid_build", "density", "rank_keys", "rank_sort", "search",
                                      "open_search", "ringk", "peaks", "finish", "label", "approx"};
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

// Cells per cut-off distance for each number of grid dimensions (finer cells
// clip the windows closer to the d_cut-ball; the table grows as their power).
int default_subdivision(int d) { return d <= 3 ? 2 : 1; }

bool valid_stages(const dpc_tuning &t) {
  if (t.nstages < 1 || t.nstages > 4) return false;
  for (int k = 0; k < t.nstages; ++k)
    if (t.stage_radius[k] < 0 || t.stage_radius[k] > 64 || t.stage_group[k] < 1 || t.stage_group[k] > 64)
      return false;
  return true;
}

// Dense-table cap: at most kTableMax cells, and at most `per_point` per point
// (4096 at least), so a small problem does not scan a table far larger than itself.
int64_t table_cap(int64_t n, int64_t per_point) {
  const int64_t c = std::max<int64_t>(4096, per_point * n);
  return std::min<int64_t>(kTableMax, c);
}

// Lane form (one query per lane) by default where data is sparse per cell:
// measured on 4-D random walks, where a strip of cells holds a few points and a
// 64-query task leaves most lanes idle.
bool default_lanes(int d, int gm) { return d == 4 && gm == d; }

bool make_plan(int64_t n, int32_t d, double d_cut, const dpc_tuning *opt, Plan *out) {
  if (n < 1 || n >= DPC_MAX_POINTS || d < 1 || d > DPC_MAX_DIM) return false;
  const int64_t R = cutoff_square(d_cut);
  if (R < 1) return false;
  if (opt && (opt->lanes < 0 || opt->lanes > 2)) return false;
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
  // Grid dimensions: the first gm coordinates are indexed.  In many dimensions a
  // full grid leaves most rows with a point or two, so tasks run nearly empty
  // waves and windows and rings grow as 3^(d-1); past four dimensions three
  // indexed ones keep rows full (measured on blob and random-walk data).
  int gm = d <= 4 ? d : 3;
  {
    const int v = opt ? opt->grid_dims : 0;
    if (v >= 1) gm = v < d ? v : d;  // more than d: all of them
  }
  p.gm = gm;
  p.lanes = opt && opt->lanes ? (opt->lanes == 2 ? 1 : 0) : (default_lanes(d, gm) ? 1 : 0);
  // A partial grid runs the exact int64 distance path with cells one cut-off
  // wide; a full one subdivides the cut-off (finer cells clip windows closer to
  // the ball, the table grows as their power).  In lane form cells are one
  // cut-off wide: a lane's window then has 3^gm cells, and each row lookup is
  // paid per query.
  int S = (gm < d || p.lanes) ? 1 : default_subdivision(gm);
  {
    const int v = opt ? opt->subdiv : 0;
    if (v >= 1 && v <= 16) S = v;
  }
  const int64_t nc_max = iroot(table_cap(n, p.lanes ? 16 : 8), gm);
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
  p.ext16 = int32_t(E);
  auto p16_ok = [&](int64_t K, int64_t wc) { return wc >= 1 && (wc + 2 * K) * L <= E && (2 * K + 1) * L <= E; };
  const int64_t wc16 = E / L - 2 * int64_t(p.K0);
  // The packed path needs every coordinate difference bounded by the window,
  // so every coordinate must be indexed.
  if (gm == d && p16_ok(p.K0, wc16)) {
    p.mode = kModeP16;
    p.wc = int32_t(wc16 < nc ? wc16 : nc);
  } else {
    p.mode = kModeI64;
    p.wc = int32_t(nc);
  }
  // Without the packed path's width limit, a strip spans a whole row, and
  // tasks of sparse rows spread over many cells; four-cell strips keep each
  // task's window narrow.
  if (gm < d && p.wc > 4) p.wc = 4;
  {
    const int64_t v = opt ? opt->strip_cells : 0;
    if (v >= 1 && v < p.wc) p.wc = int32_t(v);  // narrower only
  }
  if (p.lanes) {  // the packed path needs each lane's window within E, no strips
    p.mode = (gm == d && (int64_t(p.K0) + 1) * L <= E) ? kModeP16 : kModeI64;
    p.wc = int32_t(nc);
  }
  // Dependent-search stages: window radii in cells (0: the ball stage) and, in
  // task form, tasks gathered per wave (more as fewer points stay open); a later
  // stage is dropped when its window has more than 4096 rows.  Lane form runs
  // one stage (by default a block of one cell: the ring search continues from it).
  dpc_tuning st;
  std::memset(&st, 0, sizeof(st));
  st.nstages = 1;  // one window stage, then the ring search (measured best on 2-D to 6-D data)
  st.stage_radius[0] = 1;
  st.stage_group[0] = 1;
  if (opt && opt->nstages) {
    if (!valid_stages(*opt)) return false;
    st = *opt;
  }
  if (p.lanes) st.nstages = 1;
  p.nstages = 0;
  for (int k = 0; k < st.nstages; ++k) {
    const int K = st.stage_radius[k] == 0 ? p.K0 : st.stage_radius[k];  // 0: the ball stage
    int64_t rows = 1;
    for (int t = 0; t < gm - 1; ++t) rows *= 2 * K + 1;
    if (k > 0 && rows > 4096) break;
    p.stageK[p.nstages] = st.stage_radius[k];
    p.stageGroup[p.nstages] = st.stage_group[k];
    // a lane's candidates lie within (K + 1) L - 1 of it in every coordinate; a
    // task's within its strip's window
    const bool p16 = p.lanes ? (K + 1) * L <= E : p16_ok(K, p.wc);
    p.stageMode[p.nstages] = (gm == d && p16) ? kModeP16 : kModeI64;
    ++p.nstages;
  }
  // Lane form, on request: a second window stage over the points the first
  // leaves open; the ring search then grows from its block.  Off by default:
  // on 4M 4-D random walks it took as long as the ring-search passes it saves
  // (0.40 + 0.87 ms against 1.27 ms), and longer in the many-job form.
  p.openK = 0;
  p.openMode = kModeI64;
  {
    const int v = opt ? opt->open_radius : 0;
    if (v < 0 || v > 16) return false;
    if (v > 0) {
      if (!p.lanes || p.stageK[0] < 1 || v <= p.stageK[0]) return false;
      int64_t rows = 1;  // the stage's rows stay below 2^20
      for (int t = 0; t < gm - 1; ++t) rows *= 2 * v + 1;
      if (rows > (int64_t(1) << 20)) return false;
      p.openK = v;
      p.openMode = (gm == d && (int64_t(v) + 1) * L <= E) ? kModeP16 : kModeI64;
    }
  }
  // Ring steps before the prefix scan: more in more dimensions, where rings
  // stay cheap longer than scanning a long density prefix.
  p.ring_cap = d <= 2 ? kRingCostCap : kRingCostCapWide;
  {
    const int v = opt ? opt->ring_cap : 0;
    if (v >= 1 && v <= 1 << 20) p.ring_cap = v;
  }
  p.nsx = int32_t((nc + p.wc - 1) / p.wc);
  p.ncells = ipow(nc, gm);
  p.nrows = ipow(nc, gm - 1);
  p.nstrips = p.lanes ? 0 : p.nrows * p.nsx;  // lane form builds no strip tasks
  p.max_tasks = p.lanes ? 0 : n / kQueryChunk + p.nstrips + 1;

  const int64_t scan_max = std::max(std::max(p.ncells + 1, p.nstrips + 1), n + 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  p.o_hdr = take(sizeof(DevHeader));
  // the cell table, with three slack entries after it: a radius-1 lane window
  // reads start[x - 1 .. x + 2] of a row in one load (start[-1] is the last word
  // of the header slot just before the table; neither slack value is used)
  p.o_cnt = take(size_t(p.ncells + 1 + 3) * 4);
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
  p.o_srec = 0;
  if (p.lanes && d <= 4 && p.stageMode[0] == kModeP16) p.o_srec = take(size_t(n) * 16);
  // one bit per 8 cells, written whole by the table scan (every word of every
  // 4096-cell scan tile)
  p.o_occ = take(size_t((p.ncells + 1 + kScanTile - 1) / kScanTile) * (kScanTile / 256) * 4);
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
  if (!make_plan(n, d, d_cut, nullptr, p)) return fail(DPC_EINVAL, "no plan for these sizes");
  if (ws_bytes < p->total) return fail(DPC_EWORKSPACE, "workspace smaller than dpc_workspace_bytes()");
  p->count_work = g_prof_level >= 2 ? 1 : 0;
  return DPC_OK;
}

// 64-bit FNV-1a of a plan's bytes (the struct is zero-filled before its fields
// are set, so equal plans hash equally).
uint64_t plan_hash(const Plan &plan) {
  Plan p = plan;
  p.count_work = 0;  // profiling does not change the grid
  const unsigned char *b = reinterpret_cast<const unsigned char *>(&p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < sizeof(Plan); ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// The identity of the grid a call on these inputs builds.
GridStamp grid_stamp(const Plan &p, const int32_t *pts) {
  GridStamp st;
  st.w[0] = kStampMagic;
  st.w[1] = uint64_t(reinterpret_cast<uintptr_t>(pts));
  st.w[2] = uint64_t(p.n);
  st.w[3] = uint64_t(p.R);
  st.w[4] = plan_hash(p);
  st.w[5] = uint64_t(p.d) | (uint64_t(p.gm) << 8) | (uint64_t(p.lanes) << 16) | (uint64_t(uint32_t(p.L)) << 32);
  return st;
}

// Grid and local density; the density stays in the workspace's rank keys.
dpc_status run_density(const Plan &p, const Ws &w, const int32_t *pts, hipStream_t s) {
  hipError_t e;
  {
    ProfScope ps(s, kProfGrid);
    e = build_grid(p, w, pts, grid_stamp(p, pts), s);
  }
  if (e != hipSuccess) return device_fail(e, "grid build");
  ProfScope ps(s, kProfDensity);
  e = launch_density(p, w, s);
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
  g_work[4] = p.openK ? h.n_ring : h.n_unres;
  for (int k = 0; k < 4; ++k) g_tests[k] = int64_t(h.work[k]);
  return hipSuccess;
}

// Dependent points.  `rho_in` (caller's densities, id order) fills the rank keys,
// or, when null, the keys the density kernel left in the workspace are used and
// `rho_out` receives the densities in id order.  The grid is built (kGridBuild),
// taken from a previous dpc_density call on the same workspace after checking
// its stamp on the device (kGridReuse), or built earlier in the same call
// (kGridOwn).
enum GridSource { kGridBuild, kGridReuse, kGridOwn };

dpc_status run_dependent(const Plan &p, const Ws &w, const int32_t *pts, const int32_t *rho_in, int32_t *dep,
                         double *delta, int32_t *rho_out, GridSource grid, hipStream_t s) {
  hipError_t e;
  if (grid == kGridBuild) {
    ProfScope ps(s, kProfGrid);
    if ((e = build_grid(p, w, pts, grid_stamp(p, pts), s)) != hipSuccess) return device_fail(e, "grid build");
  } else if (grid == kGridReuse) {
    if ((e = check_grid(w.hdr, grid_stamp(p, pts), s)) != hipSuccess) return device_fail(e, "grid check");
  } else if ((e = reset_counters(w.hdr, false, s)) != hipSuccess) {
    return device_fail(e, "reset");
  }
  if (rho_in) {
    ProfScope ps(s, kProfRankKeys);
    if ((e = gather_rank_keys(p, w, rho_in, s)) != hipSuccess) return device_fail(e, "rank keys");
  }
  {
    ProfScope ps(s, kProfRankSort);
    if ((e = rank_sort(p, w, s)) != hipSuccess) return device_fail(e, "rank sort");
  }
  if ((e = launch_dependent(p, w, dep, delta, rho_out, s)) != hipSuccess) return device_fail(e, "dependent kernels");
  if (g_prof_level >= 2 && (e = record_work(p, w, s)) != hipSuccess) return device_fail(e, "work counters");
  return DPC_OK;
}

void fill_plan_info(const Plan &p, dpc_plan_info *out) {
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
  out->grid_dims = p.gm;
  out->lanes = p.lanes;
  out->open_radius = p.openK;
}

// ---- the static scratch array of dpc_run_static ----
//
// One array per GPU (each device holds its own copy of a __device__ variable),
// kept until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: the device address comes from hipGetSymbolAddress, looked up
// once per device with that device current, and only that address is ever handed
// to kernels.
constexpr size_t kStaticScratchBytes = size_t(DPC_STATIC_SCRATCH_BYTES);
static_assert(kStaticScratchBytes % 256 == 0, "whole 256-byte slots");
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on first use).
dpc_status static_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DPC_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u)) return fail(DPC_EDEVICE, "static scratch misaligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DPC_OK;
}

// The device status word of a workspace, copied to the caller's memory.
__global__ void k_copy_status(const DevHeader *hdr, uint32_t *out) {
  if (threadIdx.x == 0) *out = hdr->status;
}

dpc_status check_job(const dpc_job &j) {
  if (!j.pts || !j.rho || !j.dep || !j.delta || !j.label || !j.ncenters) return fail(DPC_EINVAL, "null pointer");
  if (j.n < 1 || j.n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (j.d < 1 || j.d > DPC_MAX_DIM) return fail(DPC_EINVAL, "d must be in [1, 8]");
  if (!std::isfinite(j.d_cut) || !(j.d_cut > 0.0)) return fail(DPC_EINVAL, "d_cut must be finite and > 0");
  if (j.rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(j.delta_min) || !(j.delta_min > j.d_cut)) return fail(DPC_EINVAL, "delta_min must exceed d_cut");
  return DPC_OK;
}

// Gathers every job's device status word (sorted job order).
__global__ void k_batch_status(const JobDev *jobs, int32_t njobs, uint32_t *out) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < njobs; k += int64_t(gridDim.x) * blockDim.x)
    out[k] = jobs[k].w.hdr->status;
}

}  // namespace
}  // namespace dpc

// Host-side plan of a many-job launch.
struct dpc_batch {
  struct Map {
    std::vector<uint32_t> vjob, vfirst, vcount;
  };
  int32_t njobs = 0;
  std::vector<int32_t> order;   // order[k]: caller index of the k-th job (launch order)
  std::vector<int32_t> pos;     // pos[i]: launch position of caller job i
  std::vector<dpc_job> jobs;    // caller order
  std::vector<dpc::Plan> plans; // caller order
  std::vector<size_t> ws_off;   // launch order: offset of each job's workspace
  Map maps[5];                  // one, pts, cells, strips, work
  size_t o_status = 0, o_jobs = 0, o_map[5][3] = {}, total = 0;
  int32_t ngroups = 0, gdim[DPC_MAX_DIM] = {}, max_stages = 0, any_open = 0;
  uint32_t gwork0[DPC_MAX_DIM] = {}, gwork1[DPC_MAX_DIM] = {};
  void *bound = nullptr;
};

namespace dpc {
namespace {

enum { kMapOne = 0, kMapPts, kMapCells, kMapStrips, kMapWork };

void add_blocks(dpc_batch::Map &m, uint32_t k, int64_t count) {
  const uint32_t c = uint32_t(std::max<int64_t>(1, std::min<int64_t>(count, 1 << 20)));
  m.vfirst.push_back(uint32_t(m.vjob.size()));
  m.vcount.push_back(c);
  m.vjob.insert(m.vjob.end(), c, k);
}

BatchMaps batch_maps(const dpc_batch &b, void *ws) {
  char *base = static_cast<char *>(ws);
  BatchMaps B;
  std::memset(&B, 0, sizeof(B));
  B.jobs = reinterpret_cast<const JobDev *>(base + b.o_jobs);
  B.njobs = b.njobs;
  VMap *vm[5] = {&B.one, &B.pts, &B.cells, &B.strips, &B.work};
  for (int m = 0; m < 5; ++m) {
    vm[m]->vjob = reinterpret_cast<const uint32_t *>(base + b.o_map[m][0]);
    vm[m]->vfirst = reinterpret_cast<const uint32_t *>(base + b.o_map[m][1]);
    vm[m]->vcount = reinterpret_cast<const uint32_t *>(base + b.o_map[m][2]);
    vm[m]->v0 = 0;
    vm[m]->v1 = uint32_t(b.maps[m].vjob.size());
  }
  B.ngroups = b.ngroups;
  for (int g = 0; g < b.ngroups; ++g) {
    B.gdim[g] = b.gdim[g];
    B.gwork0[g] = b.gwork0[g];
    B.gwork1[g] = b.gwork1[g];
  }
  B.max_stages = b.max_stages;
  B.any_open = b.any_open;
  return B;
}

}  // namespace
// Approx-DPC's second grid and its workspace after the exact path's (which it
// uses as dpc_run does).
ApproxPlan make_approx_plan(const Plan &p, double d_cut) {
  ApproxPlan a{};
  a.La = int32_t(1 + isqrt64((p.R - 1) / p.d));
  uint64_t slots = 256;
  while (slots < 2 * uint64_t(p.n)) slots <<= 1;
  a.mask = uint32_t(slots - 1);
  a.d_cut = d_cut;
  size_t o = align_up(p.total);
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  a.o_cnt = take(256);
  a.o_rep = take(slots * 4);
  a.o_top = take(slots * 8);
  a.o_minrho = take(slots * 4);
  a.o_ent = take(size_t(p.n) * 4);
  a.o_plist = take(size_t(p.n) * 4);
  a.total = o;
  return a;
}

// ceil(e^2) for e = eps * d_cut rounded to a double (one IEEE product), exactly as
// for d_cut itself; 1 when the product underflows to zero.
int64_t eps_cutoff_square(double d_cut, double eps) {
  const double e = eps * d_cut;
  return e > 0.0 ? cutoff_square(e) : 1;
}

SApproxPlan make_sapprox_plan(const Plan &p, double d_cut, double eps) {
  SApproxPlan a{};
  const int64_t Re = eps_cutoff_square(d_cut, eps);
  a.Le = int32_t(1 + isqrt64((Re - 1) / p.d));
  uint64_t slots = 256;
  while (slots < 2 * uint64_t(p.n)) slots <<= 1;
  a.mask = uint32_t(slots - 1);
  size_t o = align_up(p.total);
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  a.o_cnt = take(256);
  a.o_rep = take(slots * 4);
  a.o_pick = take(slots * 4);
  a.o_ppos = take(slots * 4);
  a.o_prho = take(slots * 4);
  a.o_ent = take(size_t(p.n) * 4);
  a.o_plist = take(size_t(p.n) * 4);
  a.total = o;
  return a;
}

}  // namespace dpc

using namespace dpc;

extern "C" {

int32_t dpc_version(void) { return 100; }

const char *dpc_last_error(void) { return g_last_error.c_str(); }

int64_t dpc_cutoff_square(double d_cut) { return cutoff_square(d_cut); }

size_t dpc_workspace_bytes(int64_t n, int32_t d, double d_cut) {
  Plan p;
  return make_plan(n, d, d_cut, nullptr, &p) ? p.total : 0;
}

dpc_status dpc_plan(int64_t n, int32_t d, double d_cut, dpc_plan_info *out) {
  return dpc_plan_tuned(n, d, d_cut, nullptr, out);
}

dpc_status dpc_plan_tuned(int64_t n, int32_t d, double d_cut, const dpc_tuning *tuning, dpc_plan_info *out) {
  Plan p;
  if (!out) return fail(DPC_EINVAL, "null pointer argument");
  if (!make_plan(n, d, d_cut, tuning, &p)) return fail(DPC_EINVAL, "no plan for these sizes or options");
  fill_plan_info(p, out);
  return DPC_OK;
}

dpc_status dpc_batch_plan(const dpc_job *jobs, int32_t njobs, const dpc_tuning *tuning, dpc_batch **out,
                          size_t *ws_bytes) {
  if (!jobs || !out || !ws_bytes || njobs < 1) return fail(DPC_EINVAL, "null pointer argument or no jobs");
  *out = nullptr;
  dpc_batch *b = new dpc_batch;
  b->njobs = njobs;
  b->jobs.assign(jobs, jobs + njobs);
  b->plans.resize(njobs);
  for (int32_t i = 0; i < njobs; ++i) {
    dpc_status st = check_job(jobs[i]);
    if (st == DPC_OK && !make_plan(jobs[i].n, jobs[i].d, jobs[i].d_cut, tuning ? tuning + i : nullptr, &b->plans[i]))
      st = fail(DPC_EINVAL, "no plan for these sizes or options");
    if (st != DPC_OK) {
      g_last_error = "job " + std::to_string(i) + ": " + g_last_error;
      delete b;
      return st;
    }
  }
  // Launch order: by dimension (one launch per dimension for the templated
  // kernels), then largest first so the long jobs start early.
  b->order.resize(njobs);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) {
    if (jobs[x].d != jobs[y].d) return jobs[x].d < jobs[y].d;
    return jobs[x].n > jobs[y].n;
  });
  b->pos.resize(njobs);
  for (int32_t k = 0; k < njobs; ++k) b->pos[b->order[k]] = k;
  for (int32_t k = 0; k < njobs; ++k) {
    const Plan &p = b->plans[b->order[k]];
    add_blocks(b->maps[kMapOne], uint32_t(k), 1);
    add_blocks(b->maps[kMapPts], uint32_t(k), (p.n + kBatchPoints - 1) / kBatchPoints);
    add_blocks(b->maps[kMapCells], uint32_t(k), (p.ncells + kBatchCells) / kBatchCells);
    add_blocks(b->maps[kMapStrips], uint32_t(k), (p.nstrips + kBatchPoints) / kBatchPoints);
    const uint32_t w0 = uint32_t(b->maps[kMapWork].vjob.size());
    // persistent work: about kBatchTasks tasks per virtual block, or in lane form
    // kBatchLanePoints points (one per lane)
    add_blocks(b->maps[kMapWork], uint32_t(k),
               p.lanes ? (p.n + kBatchLanePoints - 1) / kBatchLanePoints
                       : std::min<int64_t>(2048, (p.max_tasks + kBatchTasks - 1) / kBatchTasks));
    if (b->ngroups == 0 || b->gdim[b->ngroups - 1] != p.d) {
      b->gdim[b->ngroups] = p.d;
      b->gwork0[b->ngroups] = w0;
      ++b->ngroups;
    }
    b->gwork1[b->ngroups - 1] = uint32_t(b->maps[kMapWork].vjob.size());
    b->max_stages = std::max(b->max_stages, p.nstages);
    if (p.openK) b->any_open = 1;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  b->o_status = take(size_t(njobs) * 4);
  b->o_jobs = take(size_t(njobs) * sizeof(JobDev));
  for (int m = 0; m < 5; ++m) {
    b->o_map[m][0] = take(b->maps[m].vjob.size() * 4);
    b->o_map[m][1] = take(b->maps[m].vfirst.size() * 4);
    b->o_map[m][2] = take(b->maps[m].vcount.size() * 4);
  }
  b->ws_off.resize(njobs);
  for (int32_t k = 0; k < njobs; ++k) b->ws_off[k] = take(b->plans[b->order[k]].total);
  b->total = o;
  *ws_bytes = o;
  *out = b;
  return DPC_OK;
}

dpc_status dpc_batch_bind(dpc_batch *b, void *ws, size_t ws_bytes) {
  if (!b || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (ws_bytes < b->total) return fail(DPC_EWORKSPACE, "workspace smaller than the batch needs");
  char *base = static_cast<char *>(ws);
  const size_t head = b->ws_off.empty() ? b->total : b->ws_off[0];
  std::vector<char> host(head, 0);
  JobDev *jd = reinterpret_cast<JobDev *>(host.data() + b->o_jobs);
  for (int32_t k = 0; k < b->njobs; ++k) {
    const int32_t i = b->order[k];
    const dpc_job &j = b->jobs[i];
    JobDev &J = jd[k];
    std::memset(&J, 0, sizeof(J));
    J.p = b->plans[i];
    J.w = resolve(J.p, base + b->ws_off[k]);
    J.pts = j.pts;
    J.rho = j.rho;
    J.dep = j.dep;
    J.delta = j.delta;
    J.label = j.label;
    J.ncenters = j.ncenters;
    J.rho_min = j.rho_min;
    J.delta_min = j.delta_min;
  }
  for (int m = 0; m < 5; ++m) {
    const auto &M = b->maps[m];
    std::memcpy(host.data() + b->o_map[m][0], M.vjob.data(), M.vjob.size() * 4);
    std::memcpy(host.data() + b->o_map[m][1], M.vfirst.data(), M.vfirst.size() * 4);
    std::memcpy(host.data() + b->o_map[m][2], M.vcount.data(), M.vcount.size() * 4);
  }
  hipError_t e = hipMemcpy(base, host.data(), head, hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(e, "batch table upload");
  b->bound = ws;
  return DPC_OK;
}

dpc_status dpc_batch_run(const dpc_batch *b, void *ws, void *stream) {
  if (!b || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (b->bound != ws) return fail(DPC_EINVAL, "workspace not bound to this batch (dpc_batch_bind)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const BatchMaps B = batch_maps(*b, ws);
  hipError_t e;
  if ((e = batch_start(B, s)) != hipSuccess) return device_fail(e, "batch start");
  {
    ProfScope ps(s, kProfGrid);
    if ((e = batch_build_grid(B, s)) != hipSuccess) return device_fail(e, "batch grid build");
  }
  {
    ProfScope ps(s, kProfDensity);
    if ((e = batch_density(B, s)) != hipSuccess) return device_fail(e, "batch density");
  }
  {
    ProfScope ps(s, kProfRankSort);
    if ((e = batch_rank(B, s)) != hipSuccess) return device_fail(e, "batch rank");
  }
  if ((e = batch_dependent(B, s)) != hipSuccess) return device_fail(e, "batch dependent");
  ProfScope ps(s, kProfLabel);
  if ((e = batch_label(B, s)) != hipSuccess) return device_fail(e, "batch label");
  return DPC_OK;
}

dpc_status dpc_batch_sync_status(const dpc_batch *b, void *ws, void *stream, int32_t *first_bad) {
  if (!b || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (first_bad) *first_bad = -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  uint32_t *dst = reinterpret_cast<uint32_t *>(base + b->o_status);
  DPC_LAUNCH((k_batch_status), blocks_for(b->njobs, kBlock), kBlock, s,
             reinterpret_cast<const JobDev *>(base + b->o_jobs), b->njobs, dst);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(e, "stream synchronize");
  std::vector<uint32_t> st(b->njobs);
  e = hipMemcpy(st.data(), dst, st.size() * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(e, "status read");
  uint32_t all = 0;
  int32_t bad = -1;
  for (int32_t i = 0; i < b->njobs; ++i) {
    const uint32_t v = st[b->pos[i]];
    all |= v;
    if (v && bad < 0) bad = i;
  }
  if (first_bad) *first_bad = bad;
  if (all & 1u) return fail(DPC_ERANGE, "a coordinate was outside [0, 2^17) and was clamped");
  if (all & 2u) return fail(DPC_EINVAL, "inconsistent rho or dep input (clamped or cut)");
  g_last_error.clear();
  return DPC_OK;
}

dpc_status dpc_batch_job_plan(const dpc_batch *b, int32_t i, dpc_plan_info *out) {
  if (!b || !out) return fail(DPC_EINVAL, "null pointer argument");
  if (i < 0 || i >= b->njobs) return fail(DPC_EINVAL, "job index out of range");
  fill_plan_info(b->plans[i], out);
  return DPC_OK;
}

void dpc_batch_free(dpc_batch *b) { delete b; }

dpc_status dpc_density(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t *rho, void *ws,
                       size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!rho) return fail(DPC_EINVAL, "null pointer argument");
  const Ws w = resolve(p, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = clear_status(w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "status reset");
  if ((st = run_density(p, w, pts, s)) != DPC_OK) return st;
  e = write_rho(p, w, rho, s);
  return e == hipSuccess ? DPC_OK : device_fail(e, "density output");
}

dpc_status dpc_dependent(const int32_t *pts, int64_t n, int32_t d, double d_cut, const int32_t *rho,
                         int32_t *dep, double *delta, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!rho || !dep || !delta) return fail(DPC_EINVAL, "null pointer argument");
  if (flags & ~DPC_REUSE_GRID) return fail(DPC_EINVAL, "unknown flag");
  const Ws w = resolve(p, ws);
  const bool reuse = (flags & DPC_REUSE_GRID) != 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // A reused grid keeps the status of its build (a clamped coordinate); the grid
  // check clears the rest.
  if (!reuse) {
    hipError_t e = clear_status(w.hdr, s);
    if (e != hipSuccess) return device_fail(e, "status reset");
  }
  return run_dependent(p, w, pts, rho, dep, delta, nullptr, reuse ? kGridReuse : kGridBuild, s);
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
  if ((st = run_density(p, w, pts, s)) != DPC_OK) return st;
  if ((st = run_dependent(p, w, pts, nullptr, dep, delta, rho, kGridOwn, s)) != DPC_OK) return st;
  ProfScope ps(s, kProfLabel);
  hipError_t e = launch_label(n, rho, dep, delta, rho_min, delta_min, label, ncenters, w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "label kernels");
  return DPC_OK;
}

size_t dpc_approx_workspace_bytes(int64_t n, int32_t d, double d_cut) {
  Plan p;
  return make_plan(n, d, d_cut, nullptr, &p) ? make_approx_plan(p, d_cut).total : 0;
}

dpc_status dpc_approx_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                          double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                          int64_t *ncenters, uint8_t *approx, void *ws, size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  const ApproxPlan a = make_approx_plan(p, d_cut);
  if (ws_bytes < a.total) return fail(DPC_EWORKSPACE, "workspace smaller than dpc_approx_workspace_bytes()");
  if (!rho || !dep || !delta || !label || !ncenters) return fail(DPC_EINVAL, "null pointer argument");
  if (rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(delta_min) || !(delta_min > d_cut)) return fail(DPC_EINVAL, "delta_min must exceed d_cut");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = resolve(p, ws);
  hipError_t e = clear_status(w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "status reset");
  if ((st = run_density(p, w, pts, s)) != DPC_OK) return st;
  if ((e = reset_counters(w.hdr, false, s)) != hipSuccess) return device_fail(e, "reset");
  {
    ProfScope ps(s, kProfRankSort);
    if ((e = rank_sort(p, w, s)) != hipSuccess) return device_fail(e, "rank sort");
  }
  if ((e = launch_approx(p, w, a, ws, dep, delta, rho, approx, s)) != hipSuccess)
    return device_fail(e, "approximate dependent kernels");
  ProfScope ps(s, kProfLabel);
  e = launch_label(n, rho, dep, delta, rho_min, delta_min, label, ncenters, w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "label kernels");
  return DPC_OK;
}

size_t dpc_sapprox_workspace_bytes(int64_t n, int32_t d, double d_cut, double eps) {
  Plan p;
  if (!(eps > 0.0 && eps <= 1.0)) return 0;
  return make_plan(n, d, d_cut, nullptr, &p) ? make_sapprox_plan(p, d_cut, eps).total : 0;
}

dpc_status dpc_sapprox_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, double eps, int32_t rho_min,
                           double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                           int64_t *ncenters, uint8_t *picked, void *ws, size_t ws_bytes, void *stream) {
  Plan p;
  dpc_status st = check_common(pts, n, d, d_cut, ws, ws_bytes, &p);
  if (st != DPC_OK) return st;
  if (!(eps > 0.0 && eps <= 1.0)) return fail(DPC_EINVAL, "eps must be in (0, 1]");
  const SApproxPlan a = make_sapprox_plan(p, d_cut, eps);
  if (ws_bytes < a.total) return fail(DPC_EWORKSPACE, "workspace smaller than dpc_sapprox_workspace_bytes()");
  if (!rho || !dep || !delta || !label || !ncenters) return fail(DPC_EINVAL, "null pointer argument");
  if (rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(delta_min) || !(delta_min > d_cut)) return fail(DPC_EINVAL, "delta_min must exceed d_cut");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = resolve(p, ws);
  hipError_t e = clear_status(w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "status reset");
  if ((st = run_density(p, w, pts, s)) != DPC_OK) return st;
  if ((e = launch_sapprox(p, w, a, ws, dep, delta, rho, picked, s)) != hipSuccess)
    return device_fail(e, "S-Approx-DPC kernels");
  ProfScope ps(s, kProfLabel);
  e = launch_label(n, rho, dep, delta, rho_min, delta_min, label, ncenters, w.hdr, s);
  if (e != hipSuccess) return device_fail(e, "label kernels");
  return DPC_OK;
}

dpc_status dpc_decision_top(int64_t n, const int32_t *rho, const double *delta, int32_t rho_min, int32_t k,
                            int32_t *ids, double *deltas, int32_t *rhos, int64_t *count, void *ws,
                            size_t ws_bytes, void *stream) {
  if (!rho || !delta || !ids || !deltas || !count || !ws) return fail(DPC_EINVAL, "null pointer argument");
  if (n < 1 || n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (k < 1 || k > DPC_DECISION_TOP_MAX) return fail(DPC_EINVAL, "k must be in [1, DPC_DECISION_TOP_MAX]");
  if (ws_bytes < DPC_DECISION_WS_BYTES) return fail(DPC_EWORKSPACE, "workspace smaller than DPC_DECISION_WS_BYTES");
  hipError_t e = launch_decision_top(n, rho, delta, rho_min, k, ids, deltas, rhos, count, ws,
                                     static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPC_OK : device_fail(e, "decision top-k kernels");
}

dpc_status dpc_decision_histogram(int64_t n, const int32_t *rho, const double *delta, const double *rho_edges,
                                  int32_t n_rho_bins, const double *delta_edges, int32_t n_delta_bins,
                                  int64_t *counts, void *stream) {
  if (!rho || !delta || !rho_edges || !delta_edges || !counts) return fail(DPC_EINVAL, "null pointer argument");
  if (n < 1 || n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (n_rho_bins < 1 || n_delta_bins < 1 || int64_t(n_rho_bins) * n_delta_bins > (int64_t(1) << 24))
    return fail(DPC_EINVAL, "bins must be >= 1 on each axis and at most 2^24 in all");
  hipError_t e = launch_decision_hist(n, rho, delta, rho_edges, n_rho_bins, delta_edges, n_delta_bins, counts,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPC_OK : device_fail(e, "decision histogram kernels");
}

dpc_status dpc_decision_suggest(const double *top_deltas, const int64_t *count, double d_cut, double *delta_min,
                                int64_t *centers, void *stream) {
  if (!top_deltas || !count || !delta_min || !centers) return fail(DPC_EINVAL, "null pointer argument");
  if (!std::isfinite(d_cut) || !(d_cut > 0.0)) return fail(DPC_EINVAL, "d_cut must be finite and > 0");
  hipError_t e = launch_decision_suggest(top_deltas, count, d_cut, delta_min, centers,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPC_OK : device_fail(e, "decision suggestion kernel");
}

dpc_status dpc_run_static(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                          double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                          int64_t *ncenters, uint32_t *status, void *stream) {
  // Every check dpc_run makes, and the size check, come before any HIP call.
  if (!pts) return fail(DPC_EINVAL, "null pointer argument");
  Plan p;
  if (n < 1 || n >= DPC_MAX_POINTS) return fail(DPC_EINVAL, "n must be in [1, 2^27)");
  if (d < 1 || d > DPC_MAX_DIM) return fail(DPC_EINVAL, "d must be in [1, 8]");
  if (!std::isfinite(d_cut) || !(d_cut > 0.0)) return fail(DPC_EINVAL, "d_cut must be finite and > 0");
  if (!make_plan(n, d, d_cut, nullptr, &p)) return fail(DPC_EINVAL, "no plan for these sizes");
  if (!rho || !dep || !delta || !label || !ncenters) return fail(DPC_EINVAL, "null pointer argument");
  if (rho_min < 0) return fail(DPC_EINVAL, "rho_min must be >= 0");
  if (std::isnan(delta_min) || !(delta_min > d_cut)) return fail(DPC_EINVAL, "delta_min must exceed d_cut");
  if (p.total > kStaticScratchBytes)
    return fail(DPC_EWORKSPACE, ("problem needs " + std::to_string(p.total) + " bytes of scratch; the static array "
                                 "holds " + std::to_string(kStaticScratchBytes)).c_str());
  void *ws = nullptr;
  dpc_status st = static_scratch(&ws);
  if (st != DPC_OK) return st;
  st = dpc_run(pts, n, d, d_cut, rho_min, delta_min, rho, dep, delta, label, ncenters, ws, p.total, stream);
  if (st != DPC_OK || !status) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DPC_LAUNCH((k_copy_status), 1, kWave, s, static_cast<const DevHeader *>(ws), status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DPC_OK : device_fail(e, "status copy");
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
    char item[512];
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::snprintf(item, sizeof(item), ", \"work\": {\"tasks\": %lld, \"open\": %lld, \"ring\": %lld, "
                  "\"peaks\": %lld, \"peak_prefix\": %lld, \"tests_density\": %lld, \"tests_search\": %lld, "
                  "\"tests_ring\": %lld, \"tests_peaks\": %lld}", static_cast<long long>(g_work[0]),
                  static_cast<long long>(g_work[1]), static_cast<long long>(g_work[4]),
                  static_cast<long long>(g_work[2]), static_cast<long long>(g_work[3]),
                  static_cast<long long>(g_tests[0]), static_cast<long long>(g_tests[1]),
                  static_cast<long long>(g_tests[2]), static_cast<long long>(g_tests[3]));
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
