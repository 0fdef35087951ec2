// Shared definitions of the HIP library: the launch plan, the workspace layout,
// the device header and small wave-level helpers.  Internal; the public ABI is
// include/dpc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dpc.h"

namespace dpc {

constexpr int kWave = 64;
constexpr int kBlock = 256;              // threads per workgroup of the wave-task kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kQueryChunk = 64;          // queries per task: one per lane
constexpr int64_t kTableMax = int64_t(1) << 26;   // cells of the dense cell table
constexpr int kIdBits = 27;              // packed key = (D2 << 27) | id
constexpr uint64_t kIdMask = (uint64_t(1) << kIdBits) - 1;
constexpr uint64_t kNoKey = ~uint64_t(0);
constexpr int kScanItems = 16;           // items per thread in the block scan
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kBatchPoints = 4096;       // points (or strips) per virtual block of a many-job launch
constexpr int kBatchCells = 8192;        // table cells per virtual block of a many-job launch
constexpr int kBatchTasks = 8;           // tasks per virtual block of the persistent kernels
constexpr int kBatchLanePoints = 256;    // points per virtual block of lane-form kernels (one per lane)
enum WorkCounter { kWorkDensity = 0, kWorkSearch, kWorkRing, kWorkPeaks };
constexpr int kPeakChunk = 256;          // rank-order candidates per prefix-scan work unit
constexpr int64_t kGridCap = 32768;      // most workgroups of a wave-task launch (16 x the resident 2048)
constexpr int kRingCostCap = 48;         // default of Plan::ring_cap up to 2-D
#ifndef DPC_RING_CAP_WIDE
#define DPC_RING_CAP_WIDE 192
#endif
constexpr int kRingCostCapWide = DPC_RING_CAP_WIDE;  // and beyond 2-D

enum DistMode : int32_t {
  kModeP16 = 0,  // low 16 bits of each coordinate, packed two per word; exact while the
                 // search window keeps |dx| < 2^15 and D2 < 2^31
  kModeI64 = 1,  // exact int64 squared distances on full coordinates
};

// Identity of the grid a workspace holds: written by the grid build, checked by a
// dependent-point search that reuses the grid (DPC_REUSE_GRID).
constexpr int kStampWords = 6;
constexpr uint64_t kStampMagic = 0x44504347524944ull;  // "DPCGRID"

// Device-side scalars of one workspace.  Counters are reset by the call that uses them.
struct DevHeader {
  uint32_t status;        // errors of the current call: bit 0 coordinate out of range, bit 1 inconsistent input
  uint32_t ntasks;        // tasks of the density and search kernels (written by the task builder)
  uint32_t n_unres;       // points left open by the search stages
  uint32_t n_peaks;       // points left to the rank-prefix scan
  uint32_t skip;          // 1: the workspace holds no grid of this call's inputs; grid kernels do nothing
  uint32_t n_ring;        // points left to the ring search by the open-point stage (Plan::openK)
  uint64_t stamp[kStampWords];  // the grid's identity (grid_stamp)
  uint64_t work[4];       // with Plan::count_work: candidate (query, point) distance tests of the
                          // density, window search, ring search and prefix scan kernels
  uint32_t rank_end;      // ranks the prefix scan reads: the largest bucket end of a deferred point
  uint32_t pad[37];
};
static_assert(sizeof(DevHeader) == 256, "header is one 256-byte slot");

// Everything a kernel needs to know about one problem and its workspace.
struct Plan {
  int64_t n;
  int32_t d;
  int32_t words;     // packed 16-bit words per point, (d + 1) / 2
  int64_t R;         // ceil(d_cut^2)
  int32_t L0;        // floor(sqrt(R - 1)): largest coordinate gap inside the d_cut-ball
  int32_t K0;        // density window radius in cells: K0 * L >= L0
  int32_t L;         // cell side
  int32_t nc;        // cells per dimension
  int32_t wc;        // strip width in cells along the last grid dimension
  int32_t nsx;       // strips per row, ceil(nc / wc)
  int32_t mode;      // DistMode of the density kernel
  int32_t nstages;   // dependent-search stages
  int32_t stageK[4];     // window radius (cells) of each stage
  int32_t stageGroup[4]; // tasks gathered per wave in each stage
  int32_t stageMode[4];  // DistMode of each stage
  int32_t ring_cap;  // most ring-search steps per point before the prefix scan
  int32_t gm;        // grid dimensions: the cells index the first gm coordinates (1..d)
  int32_t lanes;     // 1: one query per lane with its own window (sparse data); 0: tasks of 64
                     // queries of one strip sharing a window's candidates (dense data)
  int32_t count_work; // 1: the kernels count their distance tests into DevHeader::work (profiling)
  int32_t openK;     // lane form: radius of an optional second window stage over the points the
                     // first left open (0: none; the ring search then starts from the first block)
  int32_t openMode;  // DistMode of that stage
  int32_t ext16;     // E: the packed 16-bit distance path is exact while every coordinate
                     // difference is below E (E - 1 <= 32767, d (E - 1)^2 < 2^31)
  int64_t ncells;    // nc^gm
  int64_t nrows;     // nc^(gm-1)
  int64_t nstrips;   // nrows * nsx
  int64_t max_tasks;
  // workspace byte offsets
  size_t o_hdr, o_cnt, o_bsum, o_key, o_slot, o_spts, o_spk, o_sid, o_sK, o_tcnt, o_tasks, o_rcnt,
      o_rpts, o_rid, o_best, o_unres, o_peaks, o_flag, o_srec, o_occ, total;
};

// Approx-DPC's second grid (cells of side La) and its part of the workspace,
// which follows the exact path's.
struct ApproxPlan {
  int32_t La;        // cell side: 1 + floor(sqrt((R - 1) / d))
  uint32_t mask;     // hash table slots - 1 (slots: a power of two >= 2n)
  double d_cut;      // dependent distance given to an approximate dependent point
  size_t o_cnt, o_rep, o_top, o_minrho, o_ent, o_plist, total;
};

// S-Approx-DPC's grid G' (cells of side Le) and its part of the workspace, which
// follows the exact path's.
struct SApproxPlan {
  int32_t Le;        // cell side: 1 + floor(sqrt((Re - 1) / d)), Re = ceil((eps d_cut)^2)
  uint32_t mask;     // hash table slots - 1 (slots: a power of two >= 2n)
  size_t o_cnt, o_rep, o_pick, o_ppos, o_prho, o_ent, o_plist, total;
};

// Pointers into one workspace, resolved from a Plan.
struct Ws {
  DevHeader *hdr;
  uint32_t *cnt;     // [ncells + 1] cell counts, then cell starts (exclusive scan)
  uint32_t *bsum;    // scan block sums
  uint32_t *key;     // [n] cell key per id; after the id scatter, the id's cell-order position
  uint32_t *slot;    // [n] slot within the cell (later: slot within the rho bucket; after the rank
                     // sort, the points the open-point stage leaves to the ring search)
  int32_t *spts;     // [n][d] clamped coordinates in cell order
  uint32_t *spk;     // [n][words] packed low 16 bits of the coordinates, cell order
  int32_t *sid;      // [n] id at each cell-order position
  uint64_t *sK;      // [n] (rho << 32) | ~id at each cell-order position (written by the
                     // density kernels, or gathered from a caller's rho)
  uint32_t *tcnt;    // [nstrips + 1] tasks per strip, then task offsets
  uint4 *tasks;      // [max_tasks] {first query, end query, strip, 0}
  uint32_t *rcnt;    // [n + 1] rho histogram by (n - rho), then bucket starts
  int32_t *rpts;     // [n][d] coordinates in rank order
  int32_t *rid;      // [n] cell-order position at each rank position; up to DevHeader::rank_end,
                     // rewritten with the id there when the rank-order points are gathered
  uint64_t *best;    // [n] packed (D2 << 27 | dep) per cell-order position, kNoKey if none
  uint32_t *unres;   // [n + 1] cell-order positions open after the search stages (+ spare slot)
  uint32_t *peaks;   // [n + 1] cell-order positions left to the rank-prefix scan (+ spare slot)
  uint8_t *flag;     // [n] 1 while the cell-order position's dependent point is open
  uint32_t *occ;     // [ceil(ncells / 256)] cell occupancy: bit g (word g / 32) is set when one of
                     // the 8 cells 8g .. 8g + 7 (flat table index) holds a point
  uint4 *srec;       // [n] lane form with packed coordinates of d <= 4: per cell-order position
                     // {packed words (one or two), rank key low, rank key high}, what a lane
                     // search reads of a candidate in one 16-byte load (null otherwise)
};

inline Ws resolve(const Plan &p, void *base) {
  char *b = static_cast<char *>(base);
  Ws w;
  w.hdr = reinterpret_cast<DevHeader *>(b + p.o_hdr);
  w.cnt = reinterpret_cast<uint32_t *>(b + p.o_cnt);
  w.bsum = reinterpret_cast<uint32_t *>(b + p.o_bsum);
  w.key = reinterpret_cast<uint32_t *>(b + p.o_key);
  w.slot = reinterpret_cast<uint32_t *>(b + p.o_slot);
  w.spts = reinterpret_cast<int32_t *>(b + p.o_spts);
  w.spk = reinterpret_cast<uint32_t *>(b + p.o_spk);
  w.sid = reinterpret_cast<int32_t *>(b + p.o_sid);
  w.sK = reinterpret_cast<uint64_t *>(b + p.o_sK);
  w.tcnt = reinterpret_cast<uint32_t *>(b + p.o_tcnt);
  w.tasks = reinterpret_cast<uint4 *>(b + p.o_tasks);
  w.rcnt = reinterpret_cast<uint32_t *>(b + p.o_rcnt);
  w.rpts = reinterpret_cast<int32_t *>(b + p.o_rpts);
  w.rid = reinterpret_cast<int32_t *>(b + p.o_rid);
  w.best = reinterpret_cast<uint64_t *>(b + p.o_best);
  w.unres = reinterpret_cast<uint32_t *>(b + p.o_unres);
  w.peaks = reinterpret_cast<uint32_t *>(b + p.o_peaks);
  w.flag = reinterpret_cast<uint8_t *>(b + p.o_flag);
  w.srec = p.o_srec ? reinterpret_cast<uint4 *>(b + p.o_srec) : nullptr;
  w.occ = reinterpret_cast<uint32_t *>(b + p.o_occ);
  return w;
}

// One job of a many-job launch, as the kernels read it (device memory).
struct JobDev {
  Plan p;
  Ws w;
  const int32_t *pts;
  int32_t *rho, *dep;
  double *delta;
  int32_t *label;
  int64_t *ncenters;
  int32_t rho_min, pad;
  double delta_min;
};

// Virtual blocks of a many-job launch: vjob[v] is the job of virtual block v,
// and job j owns the vcount[j] virtual blocks from vfirst[j].  A launch covers
// virtual blocks [v0, v1) (jobs of one dimension for the templated kernels).
struct VMap {
  const uint32_t *vjob, *vfirst, *vcount;
  uint32_t v0, v1;
};

// Host description of a many-job launch: the device job table and the virtual
// block maps of each kind of phase.  Jobs are ordered by dimension, so the jobs
// of one dimension own one contiguous range of every map.
struct BatchMaps {
  const JobDev *jobs;
  int32_t njobs;
  VMap one;     // one virtual block per job
  VMap pts;     // about kBatchPoints points per virtual block
  VMap cells;   // about kBatchCells table cells per virtual block
  VMap strips;  // about kBatchPoints strips per virtual block
  VMap work;    // persistent kernels: about kBatchTasks tasks per virtual block
  int32_t ngroups;
  int32_t gdim[DPC_MAX_DIM];                       // dimension of each group
  uint32_t gwork0[DPC_MAX_DIM], gwork1[DPC_MAX_DIM];  // its work virtual blocks
  int32_t max_stages;
  int32_t any_open;  // some job runs the open-point stage (Plan::openK)
};

// Blocks of a many-job launch over m (0: nothing to launch).
inline unsigned vgrid(const VMap &m) {
  const uint32_t v = m.v1 > m.v0 ? m.v1 - m.v0 : 0u;
  return v < uint32_t(kGridCap) ? v : uint32_t(kGridCap);
}

// The identity a grid build stamps into its workspace header.
struct GridStamp {
  uint64_t w[kStampWords];
};

// Host-side launch helpers (implemented in the .hip files).
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_scan(uint32_t *data, int64_t count, uint32_t *bsum, hipStream_t s, uint32_t *occ = nullptr);
// Grid: cell keys, counting sort into cells, cell-order copies, strip tasks; stamps the header.
hipError_t build_grid(const Plan &p, const Ws &w, const int32_t *pts, const GridStamp &stamp, hipStream_t s);
// Checks the header's stamp against `stamp` (a reused grid): on a mismatch every grid kernel
// of the call does nothing and the status gets the inconsistent-input bit.
hipError_t check_grid(DevHeader *hdr, const GridStamp &stamp, hipStream_t s);
// Rank keys of the cell-order positions from a caller's densities (id order).
hipError_t gather_rank_keys(const Plan &p, const Ws &w, const int32_t *rho, hipStream_t s);
// Local density into the rank keys (cell order); write_rho copies it to the caller's id order.
hipError_t launch_density(const Plan &p, const Ws &w, hipStream_t s);
hipError_t write_rho(const Plan &p, const Ws &w, int32_t *rho, hipStream_t s);
hipError_t rank_sort(const Plan &p, const Ws &w, hipStream_t s);
hipError_t launch_rank_gather(const Plan &p, const Ws &w, hipStream_t s);  // after the ring search
// Dependent points; the outputs (and rho, if not null) are written in id order.
hipError_t launch_dependent(const Plan &p, const Ws &w, int32_t *dep, double *delta, int32_t *rho, hipStream_t s);
// The ring search from an empty window, then the prefix scan, over the list
// w.unres (DevHeader::n_unres entries) a caller filled; each listed position's
// best key must be kNoKey.
hipError_t launch_exact_remainder(const Plan &p, const Ws &w, hipStream_t s);
// The list w.unres of the cell-order positions whose w.flag is set (appended to
// DevHeader::n_unres).
hipError_t launch_collect(const Plan &p, const Ws &w, hipStream_t s);
// Approx-DPC's dependent points after the density kernels and the rank sort:
// the second grid, the approximation rules, the exact remainder, and the outputs
// in id order (approx, if not null, gets 1 where the dependent point is approximate).
hipError_t launch_approx(const Plan &p, const Ws &w, const ApproxPlan &a, void *base, int32_t *dep,
                         double *delta, int32_t *rho, uint8_t *approx, hipStream_t s);
// S-Approx-DPC after the grid build: G', the picks' densities, both phases, the
// outputs in id order (picked, if not null, gets 1 for the picked points).
hipError_t launch_sapprox(const Plan &p, const Ws &w, const SApproxPlan &a, void *base, int32_t *dep,
                          double *delta, int32_t *rho, uint8_t *picked, hipStream_t s);
hipError_t launch_label(int64_t n, const int32_t *rho, const int32_t *dep, const double *delta,
                        int32_t rho_min, double delta_min, int32_t *label, int64_t *ncenters,
                        DevHeader *hdr, hipStream_t s);
hipError_t reset_counters(DevHeader *hdr, bool grid, hipStream_t s);
// Decision-graph summaries (decision.hip): top-k by delta, <rho, delta> histogram,
// suggested delta_min.
hipError_t launch_decision_top(int64_t n, const int32_t *rho, const double *delta, int32_t rho_min, int32_t k,
                               int32_t *ids, double *deltas, int32_t *rhos, int64_t *count, void *ws,
                               hipStream_t s);
hipError_t launch_decision_hist(int64_t n, const int32_t *rho, const double *delta, const double *re, int nr,
                                const double *de, int nd, int64_t *counts, hipStream_t s);
hipError_t launch_decision_suggest(const double *top, const int64_t *count, double d_cut, double *delta_min,
                                   int64_t *centers, hipStream_t s);

// Many-job launches (every phase for all jobs of a BatchMaps, one launch each).
hipError_t batch_start(const BatchMaps &B, hipStream_t s);
hipError_t batch_build_grid(const BatchMaps &B, hipStream_t s);
hipError_t batch_density(const BatchMaps &B, hipStream_t s);
hipError_t batch_rank(const BatchMaps &B, hipStream_t s);
hipError_t batch_rank_gather(const BatchMaps &B, hipStream_t s);  // after the ring search
hipError_t batch_dependent(const BatchMaps &B, hipStream_t s);
hipError_t batch_label(const BatchMaps &B, hipStream_t s);
hipError_t clear_status(DevHeader *hdr, hipStream_t s);
unsigned persistent_blocks(int64_t max_waves);

inline unsigned blocks_for(int64_t items, int per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace dpc

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
#define DPC_DEVICE_HELPERS 1
#endif

// Kernel launch on a stream: DPC_LAUNCH((kernel<T...>), grid, block, stream, args...).
// The kernel name is parenthesised so template argument commas survive the macro.
#define DPC_STRIP(...) __VA_ARGS__
#ifndef DPC_LAUNCH
#define DPC_LAUNCH(K, G, B, S, ...) DPC_STRIP K<<<(G), (B), 0, (S)>>>(__VA_ARGS__)
#endif

// Fewest waves per SIMD a kernel is compiled for (the compiler caps its
// registers to fit them).
#ifndef DPC_WAVES
#define DPC_WAVES(n) __attribute__((amdgpu_waves_per_eu(n)))
#endif
#ifndef DPC_DENSITY_WAVES
#define DPC_DENSITY_WAVES 1
#endif
#ifndef DPC_SEARCH_WAVES
#define DPC_SEARCH_WAVES 1
#endif
#ifndef DPC_RING_WAVES
#define DPC_RING_WAVES 8
#endif

// Read-only global memory seen through the constant address space: uniform loads
// from it become scalar (SMEM) loads.  Only for data no kernel writes while it runs.
#ifndef DPC_CONST
#define DPC_CONST(T) const __attribute__((address_space(4))) T
#endif

template <typename T>
__device__ __forceinline__ DPC_CONST(T) * as_const(const T *p) {
  return (DPC_CONST(T) *)(p);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (dpc::kWave - 1); }

// 64-bit minimum over the wave.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off, dpc::kWave);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, dpc::kWave);
  return v;
}

// Exclusive prefix sum over the wave; *total gets the wave total.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, uint32_t *total) {
  const int lane = lane_id();
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < dpc::kWave; off <<= 1) {
    uint32_t y = __shfl_up(x, off, dpc::kWave);
    x += lane >= off ? y : 0u;
  }
  *total = __shfl(x, dpc::kWave - 1, dpc::kWave);
  return x - v;
}

// Work item / list slot helpers for persistent loops.  They contain no
// lane-divergent branch: a divergent `if (lane == 0)` around an atomic inside a
// loop lets the compiler's control-flow structurizer split the loop so that lane
// 0 falls an iteration behind the others, and the next cross-lane read (a
// shuffle without lane 0) then never sees a new work item.  Every lane issues the
// atomic, adding 0 or 1, and the first lane's result is broadcast.

// Slot in a list for each lane with `take` set (distinct, dense from the
// counter's old value); lanes without `take` get an unspecified value.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool take) {
  return atomicAdd(counter, take ? 1u : 0u);
}

// Block-wide list append: each thread offers up to 32 items (bit k of `mask`: item k
// taken) and gets the list slot of its first taken item; a thread's items follow
// each other, and threads follow thread order.  One atomic per block on `counter`
// (a counter bumped by every wave serialises in L2).  Every thread of the block
// calls it, with uniform control flow.
__device__ __forceinline__ uint32_t block_append(uint32_t mask, uint32_t *counter) {
  __shared__ uint32_t wave_tot[dpc::kWavesPerBlock];
  __shared__ uint32_t base;
  uint32_t tot;
  const uint32_t off = wave_exclusive_scan(uint32_t(__popc(mask)), &tot);
  const int wv = threadIdx.x / dpc::kWave;
  if (lane_id() == 0) wave_tot[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sum = 0;
    for (int k = 0; k < dpc::kWavesPerBlock; ++k) sum += wave_tot[k];
    base = sum ? atomicAdd(counter, sum) : 0u;
  }
  __syncthreads();
  uint32_t at = base + off;
  for (int k = 0; k < wv; ++k) at += wave_tot[k];
  __syncthreads();  // the shared words are reused by the next call
  return at;
}

// A job's share of a launch: block b of nb blocks.  For a single-job call it
// is the whole grid; in a many-job launch each job gets a run of virtual blocks
// that the launch's blocks take in turn.  Kernels are written against Blk, so
// both kinds of launch run the same code.
struct Blk {
  uint32_t b, nb;
};

__device__ __forceinline__ Blk grid_blk() { return Blk{blockIdx.x, gridDim.x}; }

// The launch's blocks renumbered so that the blocks of each XCD cover one
// contiguous run: the dispatcher hands workgroups to the 8 XCDs in turn (block b
// to XCD b % 8), and each XCD has its own L2, so work that reads neighbouring
// cell-order data shares that cache when it runs on one XCD.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ Blk xcd_blk() {
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t per = nb / kXcds, rem = nb % kXcds, x = b % kXcds, i = b / kXcds;
  return Blk{x * per + (x < rem ? x : rem) + i, nb};
}

// Adds a lane's count of distance tests to a work counter (profiling): a wave
// sum, then one atomic by the first lane.  Call it where every lane of the wave
// is active (after the kernel's work loop), and only when the count is wanted.
__device__ __forceinline__ void add_work(dpc::DevHeader *hdr, int which, uint64_t lane_count) {
  uint64_t v = lane_count;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, dpc::kWave);
  if (lane_id() == 0 && v) atomicAdd(reinterpret_cast<unsigned long long *>(&hdr->work[which]), (unsigned long long)v);
}

// True when the call found no grid of its inputs in the workspace (check_grid):
// the kernels that index the grid's arrays then return at once.
__device__ __forceinline__ bool grid_skipped(const dpc::DevHeader *hdr) {
  return uniform(uint32_t(as_const(&hdr->skip)[0])) != 0u;
}

// Index of the calling wave among the job's waves, and their number: wave loops
// take items wave_index(k), wave_index(k) + grid_waves(k), ...  A static
// interleave needs no shared counter: one returning atomic per work item on a
// single address serialises (about 12-16 ns each, measured; a ticket counter
// made the density kernel 2.2x slower).  The balance comes from grids larger
// than the resident set instead (kGridCap).
__device__ __forceinline__ uint32_t wave_index(Blk k) {
  return uniform(uint32_t(k.b * dpc::kWavesPerBlock + threadIdx.x / dpc::kWave));
}
__device__ __forceinline__ uint32_t grid_waves(Blk k) { return k.nb * uint32_t(dpc::kWavesPerBlock); }
__device__ __forceinline__ int64_t thread_index(Blk k) { return int64_t(k.b) * dpc::kBlock + threadIdx.x; }
__device__ __forceinline__ int64_t grid_threads(Blk k) { return int64_t(k.nb) * dpc::kBlock; }

// a - b on two packed signed 16-bit halves (wrapping), as a 32-bit word.
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t b) {
#ifndef DPC_HOST_DOT2
  typedef short s2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(s2, a) - __builtin_bit_cast(s2, b));
#else
  const uint32_t lo = (a - b) & 0xFFFFu, hi = ((a >> 16) - (b >> 16)) & 0xFFFFu;
  return lo | (hi << 16);
#endif
}

// lo*lo + hi*hi + acc on packed signed 16-bit halves (VOP3P v_dot2_i32_i16, acc may be scalar).
#ifndef DPC_HOST_DOT2
__device__ __forceinline__ int32_t dot2_self_s(uint32_t a, int32_t acc_uniform) {
  int32_t r;
  asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(r) : "v"(a), "s"(acc_uniform));
  return r;
}
__device__ __forceinline__ int32_t dot2_self_v(uint32_t a, int32_t acc) {
  int32_t r;
  asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(r) : "v"(a), "v"(acc));
  return r;
}
#else
__device__ __forceinline__ int32_t dot2_self_v(uint32_t a, int32_t acc) {
  const int32_t lo = int16_t(a & 0xFFFFu), hi = int16_t(a >> 16);
  return int32_t(uint32_t(acc) + uint32_t(lo * lo) + uint32_t(hi * hi));
}
__device__ __forceinline__ int32_t dot2_self_s(uint32_t a, int32_t acc) { return dot2_self_v(a, acc); }
#endif

// Copy of a read-only struct through the constant address space: with a
// wave-uniform address its words become scalar loads, and words that are never
// used are never loaded.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *src) {
  static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
  T out;
  uint32_t *o = reinterpret_cast<uint32_t *>(&out);
  DPC_CONST(uint32_t) *s = as_const(reinterpret_cast<const uint32_t *>(src));
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) o[i] = s[i];
  return out;
}

// Job and block coordinates of virtual block v of a many-job launch.
__device__ __forceinline__ uint32_t vjob_of(const dpc::VMap &m, uint32_t v) {
  return uniform(uint32_t(as_const(m.vjob)[v]));
}
__device__ __forceinline__ Blk vblk_of(const dpc::VMap &m, uint32_t v, uint32_t j) {
  return Blk{v - uniform(uint32_t(as_const(m.vfirst)[j])), uniform(uint32_t(as_const(m.vcount)[j]))};
}
