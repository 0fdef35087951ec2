// Grid construction (counting sort of points into cells), the density-rank
// sort, and the exclusive scan both use.
//
// The cells replace the paper's kd-tree (Section 3) as the range-search index:
// with cell side L, every point closer than d_cut to p lies in the cells within
// ceil(floor(sqrt(R - 1)) / L) cells of p's cell, R = ceil(d_cut^2) (Def. 1).
//
// Every kernel is a body over Blk (a job's share of the launch) with two
// wrappers: k_* runs one job on the whole grid, kb_* runs the jobs of a
// many-job launch, each virtual block calling the body for its job.
#include "common.h"

namespace dpc {
namespace {

// ---- bodies ----

__device__ __forceinline__ void fill_u32(Blk k, uint32_t *p, uint32_t v, int64_t count) {
  for (int64_t i = thread_index(k); i < count; i += grid_threads(k)) p[i] = v;
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[kBlock / kWave];
  const int wave = threadIdx.x / kWave;
  uint32_t wt;
  uint32_t x = wave_exclusive_scan(v, &wt);
  wsum[wave] = wt;  // every lane stores the same wave total
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    uint32_t s = wsum[i];
    before += i < wave ? s : 0u;
    all += s;
  }
  __syncthreads();
  *total = all;
  return x + before;
}

static_assert(kScanItems % 4 == 0, "the scan moves whole tiles in 16-byte vectors");

// Bit i of x at bit 2i (16 bits spread over 32).
__device__ __forceinline__ uint32_t spread_bits16(uint32_t x) {
  x &= 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Exclusive scan of u32 in three passes over tiles of kScanTile items:
// tile-local scans with each tile's total written to bsum ...  With `occ`, the
// pass also writes the occupancy bits of the counts it scans: bit g set when one
// of the 8 counts 8g .. 8g + 7 is nonzero (a lane's 16 counts are two groups, a
// wave's 1024 counts four whole words, each written once).
__device__ __forceinline__ void scan_tiles(Blk k, uint32_t *data, int64_t count, uint32_t *bsum,
                                           uint32_t *occ = nullptr) {
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  for (int64_t t = k.b; t < tiles; t += k.nb) {
    const int64_t base = t * kScanTile + int64_t(threadIdx.x) * kScanItems;
    // A whole tile of a 16-byte aligned array moves in 16-byte vectors (four
    // per lane instead of sixteen 4-byte accesses); the ragged last tile and
    // unaligned arrays take the element-wise path.
    const bool vec = (t + 1) * kScanTile <= count && (reinterpret_cast<uintptr_t>(data) & 15u) == 0;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
    if (vec) {
      const uint4 *src = reinterpret_cast<const uint4 *>(data + base);
#pragma unroll
      for (int q = 0; q < kScanItems / 4; ++q) {
        const uint4 a = src[q];
        v[4 * q] = a.x;
        v[4 * q + 1] = a.y;
        v[4 * q + 2] = a.z;
        v[4 * q + 3] = a.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        v[j] = i < count ? data[i] : 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) sum += v[j];
    if (occ) {
      static_assert(kScanItems == 16, "two 8-cell groups per lane");
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        lo |= v[j];
        hi |= v[8 + j];
      }
      const uint64_t m0 = __ballot(lo != 0), m1 = __ballot(hi != 0);
      const int lane = lane_id();
      if (lane < 4) {  // word `lane` of the wave: groups 32 lane .. 32 lane + 31
        const uint32_t e0 = uint32_t(m0 >> (16 * lane)), e1 = uint32_t(m1 >> (16 * lane));
        const int64_t word = (t * kScanTile + int64_t(threadIdx.x / kWave) * (kWave * kScanItems)) / 256 + lane;
        occ[word] = spread_bits16(e0) | (spread_bits16(e1) << 1);
      }
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, &total);
    if (vec) {
      uint4 *dst = reinterpret_cast<uint4 *>(data + base);
#pragma unroll
      for (int q = 0; q < kScanItems / 4; ++q) {
        uint4 o;
        o.x = run;
        run += v[4 * q];
        o.y = run;
        run += v[4 * q + 1];
        o.z = run;
        run += v[4 * q + 2];
        o.w = run;
        run += v[4 * q + 3];
        dst[q] = o;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < count) data[i] = run;
        run += v[j];
      }
    }
    if (threadIdx.x == 0) bsum[t] = total;
  }
}

// ... one workgroup scans the tile totals in place (in rounds of kScanTile) ...
__device__ __forceinline__ void scan_sums(uint32_t *bsum, int64_t count) {
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  uint32_t carry = 0;
  for (int64_t round = 0; round < tiles; round += kScanTile) {
    const int64_t base = round + int64_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = base + j;
      v[j] = i < tiles ? bsum[i] : 0u;
      sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, &total) + carry;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = base + j;
      if (i < tiles) bsum[i] = run;
      run += v[j];
    }
    carry += total;
  }
}

// ... and every tile adds its offset.
__device__ __forceinline__ void scan_add(Blk k, uint32_t *data, int64_t count, const uint32_t *bsum) {
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  for (int64_t t = k.b; t < tiles; t += k.nb) {
    const uint32_t add = bsum[t];
    for (int j = threadIdx.x; j < kScanTile; j += kBlock) {
      const int64_t i = t * kScanTile + j;
      if (i < count) data[i] += add;
    }
  }
}

// Cell key of every point (row-major over the cell coordinates of its first gm
// coordinates, the last of them fastest) and its slot in the cell.  Out-of-range coordinates are clamped and flagged.
__device__ __forceinline__ void cell_keys(Blk k, const int32_t *__restrict__ pts, const Plan &p,
                                          uint32_t *__restrict__ cnt, uint32_t *__restrict__ key,
                                          uint32_t *__restrict__ slot, DevHeader *__restrict__ hdr) {
  for (int64_t i = thread_index(k); i < p.n; i += grid_threads(k)) {
    uint32_t kk = 0;
    bool bad = false;
    for (int t = 0; t < p.d; ++t) {
      int32_t x = pts[i * p.d + t];
      if (x < 0 || x >= DPC_COORD_LIMIT) {
        bad = true;
        x = x < 0 ? 0 : DPC_COORD_LIMIT - 1;
      }
      if (t < p.gm) kk = kk * uint32_t(p.nc) + uint32_t(x / p.L);
    }
    if (bad) atomicOr(&hdr->status, 1u);
    key[i] = kk;
    slot[i] = atomicAdd(&cnt[kk], 1u);
  }
}

// Place every point's id at its cell-order position start[key] + slot: one
// scattered 4-byte store per point.  The position replaces the key (a
// contiguous store), so the id-order outputs can later be read from cell-order
// arrays with contiguous stores.  The coordinates follow in cell order in
// gather_pts, so that their stores are contiguous and only the reads of the
// (cache-resident) input scatter.
__device__ __forceinline__ void scatter_ids(Blk k, const Plan &p, const uint32_t *__restrict__ start,
                                            uint32_t *__restrict__ key, const uint32_t *__restrict__ slot,
                                            int32_t *__restrict__ sid) {
  for (int64_t i = thread_index(k); i < p.n; i += grid_threads(k)) {
    const uint32_t pos = start[key[i]] + slot[i];
    sid[pos] = int32_t(i);
    key[i] = pos;
  }
}

__device__ __forceinline__ int32_t clamp_coord(int32_t x) {
  return x < 0 ? 0 : (x >= DPC_COORD_LIMIT ? DPC_COORD_LIMIT - 1 : x);
}

// Cell-ordered copies of the point at each position: clamped coordinates and
// their packed low 16 bits.
__device__ __forceinline__ void gather_pts(Blk k, const int32_t *__restrict__ pts, const Plan &p,
                                           const int32_t *__restrict__ sid, int32_t *__restrict__ spts,
                                           uint32_t *__restrict__ spk) {
  // Four-coordinate rows of 16-byte aligned arrays move as one 16-byte vector.
  const bool v4 = p.d == 4 && ((reinterpret_cast<uintptr_t>(pts) | reinterpret_cast<uintptr_t>(spts)) & 15u) == 0;
  for (int64_t pos = thread_index(k); pos < p.n; pos += grid_threads(k)) {
    const int64_t i = sid[pos];
    if (v4) {
      uint4 a = reinterpret_cast<const uint4 *>(pts)[i];
      a.x = uint32_t(clamp_coord(int32_t(a.x)));
      a.y = uint32_t(clamp_coord(int32_t(a.y)));
      a.z = uint32_t(clamp_coord(int32_t(a.z)));
      a.w = uint32_t(clamp_coord(int32_t(a.w)));
      reinterpret_cast<uint4 *>(spts)[pos] = a;
      spk[pos * p.words] = (a.x & 0xFFFFu) | (a.y << 16);
      spk[pos * p.words + 1] = (a.z & 0xFFFFu) | (a.w << 16);
      continue;
    }
    uint32_t w = 0;
    for (int t = 0; t < p.d; ++t) {
      const int32_t x = clamp_coord(pts[i * p.d + t]);
      spts[pos * p.d + t] = x;
      w |= (uint32_t(x) & 0xFFFFu) << (16 * (t & 1));
      if (t & 1) {
        spk[pos * p.words + (t >> 1)] = w;
        w = 0;
      }
    }
    if (p.d & 1) spk[pos * p.words + (p.d >> 1)] = w;
  }
}

// A strip is wc consecutive cells of one row (all coordinates but the last fixed).
// Tasks cut each strip's points into chunks of kQueryChunk.
__device__ __forceinline__ void strip_range(const Plan &p, int64_t s, const uint32_t *start, uint32_t *b,
                                            uint32_t *e) {
  const int64_t row = s / p.nsx;
  const int32_t xb = int32_t(s % p.nsx);
  const int64_t k0 = row * p.nc + int64_t(xb) * p.wc;
  int64_t k1 = row * p.nc + min(int64_t(xb + 1) * p.wc, int64_t(p.nc));
  *b = start[k0];
  *e = start[k1];
}

// Tasks per strip; the entry past the last strip is cleared for the scan.
__device__ __forceinline__ void strip_count(Blk k, const Plan &p, const uint32_t *__restrict__ start,
                                            uint32_t *__restrict__ tcnt) {
  for (int64_t s = thread_index(k); s <= p.nstrips; s += grid_threads(k)) {
    uint32_t c = 0;
    if (s < p.nstrips) {
      uint32_t b, e;
      strip_range(p, s, start, &b, &e);
      c = (e - b + kQueryChunk - 1) / kQueryChunk;
    }
    tcnt[s] = c;
  }
}

__device__ __forceinline__ void strip_tasks(Blk k, const Plan &p, const uint32_t *__restrict__ start,
                                            const uint32_t *__restrict__ toff, uint4 *__restrict__ tasks,
                                            DevHeader *__restrict__ hdr) {
  for (int64_t s = thread_index(k); s < p.nstrips; s += grid_threads(k)) {
    if (s == 0) hdr->ntasks = toff[p.nstrips];
    uint32_t b, e;
    strip_range(p, s, start, &b, &e);
    uint32_t t = toff[s];
    for (uint32_t q = b; q < e; q += kQueryChunk, ++t)
      tasks[t] = make_uint4(q, min(q + uint32_t(kQueryChunk), e), uint32_t(s), 0u);
  }
}

// (rho << 32) | ~id for every cell-order position, from the caller's rho.  A
// density outside [1, n] (not produced by dpc_density) is clamped and flagged,
// so every bucket index stays in range.
__device__ __forceinline__ void gather_keys(Blk k, const Plan &p, const Ws &w, const int32_t *__restrict__ rho) {
  if (grid_skipped(w.hdr)) return;
  for (int64_t q = thread_index(k); q < p.n; q += grid_threads(k)) {
    const int32_t id = w.sid[q];
    int64_t r = rho[id];
    if (r < 1 || r > p.n) {
      atomicOr(&w.hdr->status, 2u);
      r = r < 1 ? 1 : p.n;
    }
    const uint64_t key = (uint64_t(r) << 32) | uint32_t(~uint32_t(id));
    w.sK[q] = key;
    if (w.srec) {  // lane form, packed coordinates of d <= 4 (one or two words)
      const uint32_t a = w.spk[q * p.words], b = p.words == 2 ? w.spk[q * p.words + 1] : 0u;
      w.srec[q] = make_uint4(a, b, uint32_t(key), uint32_t(key >> 32));
    }
  }
}

// ---- density-rank sort: order by rho descending; equal rho share a bucket ----

// Bucket slots of the density-rank sort.  Most densities are small and many
// points share one, so a block first counts a chunk's small densities in LDS and
// then claims each bucket's slots with one global atomic; densities of kRankBins
// or more take a global atomic each.
constexpr int kRankBins = 2048;
constexpr int kRankItems = 4;  // points per thread and chunk
constexpr int64_t kRankChunk = int64_t(kBlock) * kRankItems;

__device__ __forceinline__ void rank_hist(Blk k, const Plan &p, const uint64_t *__restrict__ sK,
                                          uint32_t *__restrict__ rcnt, uint32_t *__restrict__ slot) {
  __shared__ uint32_t bins[kRankBins];
  const int64_t chunks = (p.n + kRankChunk - 1) / kRankChunk;
  for (int64_t c = k.b; c < chunks; c += k.nb) {
    for (int b = threadIdx.x; b < kRankBins; b += kBlock) bins[b] = 0;
    __syncthreads();
    const int64_t base = c * kRankChunk;
    uint32_t local[kRankItems];
    int64_t rho[kRankItems];
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
      const int64_t q = base + int64_t(j) * kBlock + threadIdx.x;
      rho[j] = 0;
      local[j] = 0;
      if (q < p.n) {
        int64_t r = int64_t(sK[q] >> 32);
        r = r < 1 ? 1 : (r > p.n ? p.n : r);
        rho[j] = r;
        if (r <= kRankBins)
          local[j] = atomicAdd(&bins[r - 1], 1u);
        else
          slot[q] = atomicAdd(&rcnt[p.n - r], 1u);
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kRankBins; b += kBlock) {
      const uint32_t cnt = bins[b];
      if (cnt && b + 1 <= p.n) bins[b] = atomicAdd(&rcnt[p.n - (b + 1)], cnt);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
      const int64_t q = base + int64_t(j) * kBlock + threadIdx.x;
      if (q < p.n && rho[j] <= kRankBins) slot[q] = bins[rho[j] - 1] + local[j];
    }
    __syncthreads();
  }
}

// Rank order in two passes, like the grid: each cell-order position q stores
// itself at its rank position in rid (one scattered 4-byte store) ...
__device__ __forceinline__ void rank_scatter(Blk k, const Plan &p, const Ws &w) {
  if (grid_skipped(w.hdr)) return;
  for (int64_t q = thread_index(k); q < p.n; q += grid_threads(k)) {
    int64_t rho = int64_t(w.sK[q] >> 32);
    rho = rho < 1 ? 1 : (rho > p.n ? p.n : rho);
    w.rid[int64_t(w.rcnt[p.n - rho]) + w.slot[q]] = int32_t(q);
  }
}

// ... and, once the ring search has deferred its points, every rank position
// the prefix scan will read (below DevHeader::rank_end, usually a short run of
// the densest ranks) copies its point and id from there (contiguous stores,
// gathered reads; in place in rid).
__device__ __forceinline__ void rank_gather(Blk k, const Plan &p, const Ws &w) {
  if (grid_skipped(w.hdr)) return;
  const int64_t end = int64_t(uniform(as_const(&w.hdr->rank_end)[0]));
  const bool v4 = p.d == 4;  // 16-byte rows (the arrays are 256-byte aligned)
  for (int64_t r = thread_index(k); r < end; r += grid_threads(k)) {
    const uint32_t q = uint32_t(w.rid[r]);
    if (v4) {
      reinterpret_cast<int4 *>(w.rpts)[r] = reinterpret_cast<const int4 *>(w.spts)[q];
    } else {
      for (int t = 0; t < p.d; ++t) w.rpts[r * p.d + t] = w.spts[int64_t(q) * p.d + t];
    }
    w.rid[r] = w.sid[q];
  }
}

// Work counters of one call; `grid` also clears the task count of the grid build
// and marks the grid as the call's own.
__device__ __forceinline__ void reset_hdr(DevHeader *hdr, int grid) {
  if (threadIdx.x == 0) {
    if (grid) {
      hdr->ntasks = 0;
      hdr->skip = 0;
    }
    hdr->n_unres = 0;
    hdr->n_peaks = 0;
    hdr->n_ring = 0;
    hdr->rank_end = 0;
  }
}

// ---- single-job kernels ----

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t count) {
  fill_u32(grid_blk(), p, v, count);
}
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *data, int64_t count, uint32_t *bsum, uint32_t *occ) {
  scan_tiles(grid_blk(), data, count, bsum, occ);
}
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t *bsum, int64_t count) { scan_sums(bsum, count); }
__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *data, int64_t count, const uint32_t *bsum) {
  scan_add(grid_blk(), data, count, bsum);
}
__global__ __launch_bounds__(kBlock) void k_cell_keys(const int32_t *pts, Plan p, Ws w) {
  cell_keys(grid_blk(), pts, p, w.cnt, w.key, w.slot, w.hdr);
}
__global__ __launch_bounds__(kBlock) void k_scatter(Plan p, Ws w) {
  scatter_ids(grid_blk(), p, w.cnt, w.key, w.slot, w.sid);
}
__global__ __launch_bounds__(kBlock) void k_gather_pts(const int32_t *pts, Plan p, Ws w) {
  gather_pts(grid_blk(), pts, p, w.sid, w.spts, w.spk);
}
__global__ __launch_bounds__(kBlock) void k_strip_count(Plan p, Ws w) { strip_count(grid_blk(), p, w.cnt, w.tcnt); }
__global__ __launch_bounds__(kBlock) void k_strip_tasks(Plan p, Ws w) {
  strip_tasks(grid_blk(), p, w.cnt, w.tcnt, w.tasks, w.hdr);
}
__global__ __launch_bounds__(kBlock) void k_gather_rank_keys(Plan p, const int32_t *rho, Ws w) {
  gather_keys(grid_blk(), p, w, rho);
}
__global__ __launch_bounds__(kBlock) void k_rank_hist(Plan p, Ws w) { rank_hist(grid_blk(), p, w.sK, w.rcnt, w.slot); }
__global__ __launch_bounds__(kBlock) void k_rank_scatter(Plan p, Ws w) { rank_scatter(grid_blk(), p, w); }
__global__ __launch_bounds__(kBlock) void k_rank_gather(Plan p, Ws w) { rank_gather(grid_blk(), p, w); }
__global__ void k_clear_status(DevHeader *hdr) {
  if (threadIdx.x == 0) hdr->status = 0;
}
__global__ void k_reset_counters(DevHeader *hdr, int grid) { reset_hdr(hdr, grid); }

// A grid build starts: counters cleared, the grid marked as built for `stamp`.
__global__ void k_stamp_grid(DevHeader *hdr, GridStamp stamp) {
  reset_hdr(hdr, 1);
  if (threadIdx.x < kStampWords) hdr->stamp[threadIdx.x] = stamp.w[threadIdx.x];
  if (threadIdx.x < 4) hdr->work[threadIdx.x] = 0;
}

// A reused grid: counters cleared; the grid kernels are skipped (and the input
// flagged as inconsistent) unless the stamp is the one this call's inputs give.
__global__ void k_check_grid(DevHeader *hdr, GridStamp stamp) {
  reset_hdr(hdr, 0);
  if (threadIdx.x < 4) hdr->work[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    bool same = true;
    for (int i = 0; i < kStampWords; ++i) same = same && hdr->stamp[i] == stamp.w[i];
    hdr->skip = same ? 0u : 1u;
    if (!same) {
      hdr->ntasks = 0;
      hdr->status |= 2u;
    }
  }
}

// ---- many-job kernels: virtual block v of map m runs the body for its job ----

#define DPC_FOR_VBLOCKS(m)                                             \
  for (uint32_t v = (m).v0 + blockIdx.x; v < (m).v1; v += gridDim.x) { \
    const uint32_t j = vjob_of((m), v);                                \
    const Blk k = vblk_of((m), v, j);                                  \
    const Plan p = load_uniform(&jobs[j].p);                                \
    const Ws w = load_uniform(&jobs[j].w);

// The arrays the batched scans and fills work on.
enum ScanArr { kArrCells = 0, kArrStrips = 1, kArrRank = 2 };

template <int A>
__device__ __forceinline__ void scan_target(const Plan &p, const Ws &w, uint32_t **data, int64_t *count) {
  if (A == kArrCells) {
    *data = w.cnt;
    *count = p.ncells + 1;
  } else if (A == kArrStrips) {
    *data = w.tcnt;
    *count = p.nstrips + 1;
  } else {
    *data = w.rcnt;
    *count = p.n + 1;
  }
}

__global__ __launch_bounds__(kBlock) void kb_start(const JobDev *jobs, VMap m, int grid) {
  DPC_FOR_VBLOCKS(m)
  (void)k;
  (void)p;
  if (threadIdx.x == 0) w.hdr->status = 0;
  reset_hdr(w.hdr, grid);
}
}

template <int A>
__global__ __launch_bounds__(kBlock) void kb_fill(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  uint32_t *data;
  int64_t count;
  scan_target<A>(p, w, &data, &count);
  fill_u32(k, data, 0u, count);
}
}

template <int A>
__global__ __launch_bounds__(kBlock) void kb_scan_tiles(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  uint32_t *data;
  int64_t count;
  scan_target<A>(p, w, &data, &count);
  scan_tiles(k, data, count, w.bsum, A == kArrCells ? w.occ : nullptr);
}
}

template <int A>
__global__ __launch_bounds__(kBlock) void kb_scan_sums(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  (void)k;
  uint32_t *data;
  int64_t count;
  scan_target<A>(p, w, &data, &count);
  scan_sums(w.bsum, count);
}
}

template <int A>
__global__ __launch_bounds__(kBlock) void kb_scan_add(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  uint32_t *data;
  int64_t count;
  scan_target<A>(p, w, &data, &count);
  scan_add(k, data, count, w.bsum);
}
}

__global__ __launch_bounds__(kBlock) void kb_cell_keys(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  cell_keys(k, as_const(jobs)[j].pts, p, w.cnt, w.key, w.slot, w.hdr);
}
}

__global__ __launch_bounds__(kBlock) void kb_scatter(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  scatter_ids(k, p, w.cnt, w.key, w.slot, w.sid);
}
}

__global__ __launch_bounds__(kBlock) void kb_gather_pts(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  gather_pts(k, as_const(jobs)[j].pts, p, w.sid, w.spts, w.spk);
}
}

__global__ __launch_bounds__(kBlock) void kb_strip_count(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  strip_count(k, p, w.cnt, w.tcnt);
}
}

__global__ __launch_bounds__(kBlock) void kb_strip_tasks(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  strip_tasks(k, p, w.cnt, w.tcnt, w.tasks, w.hdr);
}
}

__global__ __launch_bounds__(kBlock) void kb_rank_hist(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  rank_hist(k, p, w.sK, w.rcnt, w.slot);
}
}

__global__ __launch_bounds__(kBlock) void kb_rank_scatter(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  rank_scatter(k, p, w);
}
}

__global__ __launch_bounds__(kBlock) void kb_rank_gather(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  rank_gather(k, p, w);
}
}

#undef DPC_FOR_VBLOCKS

template <int A>
void batch_scan(const BatchMaps &B, const VMap &tiles, hipStream_t s) {
  if (vgrid(tiles)) DPC_LAUNCH((kb_scan_tiles<A>), vgrid(tiles), kBlock, s, B.jobs, tiles);
  if (vgrid(B.one)) DPC_LAUNCH((kb_scan_sums<A>), vgrid(B.one), kBlock, s, B.jobs, B.one);
  if (vgrid(tiles)) DPC_LAUNCH((kb_scan_add<A>), vgrid(tiles), kBlock, s, B.jobs, tiles);
}

}  // namespace

// ---- single-job host side ----

hipError_t launch_fill_u32(uint32_t *ptr, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  unsigned blocks = blocks_for(count, kBlock);
  if (blocks > 65536u) blocks = 65536u;
  DPC_LAUNCH((k_fill_u32), blocks, kBlock, s, ptr, value, count);
  return hipGetLastError();
}

hipError_t launch_scan(uint32_t *data, int64_t count, uint32_t *bsum, hipStream_t s, uint32_t *occ) {
  if (count <= 0) return hipSuccess;
  const unsigned tiles = blocks_for(count, kScanTile);
  DPC_LAUNCH((k_scan_tiles), tiles, kBlock, s, data, count, bsum, occ);
  DPC_LAUNCH((k_scan_sums), 1, kBlock, s, bsum, count);
  DPC_LAUNCH((k_scan_add), tiles, kBlock, s, data, count, bsum);
  return hipGetLastError();
}

hipError_t clear_status(DevHeader *hdr, hipStream_t s) {
  DPC_LAUNCH((k_clear_status), 1, kWave, s, hdr);
  return hipGetLastError();
}

hipError_t reset_counters(DevHeader *hdr, bool grid, hipStream_t s) {
  DPC_LAUNCH((k_reset_counters), 1, kWave, s, hdr, grid ? 1 : 0);
  return hipGetLastError();
}

hipError_t check_grid(DevHeader *hdr, const GridStamp &stamp, hipStream_t s) {
  DPC_LAUNCH((k_check_grid), 1, kWave, s, hdr, stamp);
  return hipGetLastError();
}

hipError_t build_grid(const Plan &p, const Ws &w, const int32_t *pts, const GridStamp &stamp, hipStream_t s) {
  hipError_t e;
  DPC_LAUNCH((k_stamp_grid), 1, kWave, s, w.hdr, stamp);
  if ((e = launch_fill_u32(w.cnt, 0u, p.ncells + 1, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_cell_keys), blocks_for(p.n, kBlock), kBlock, s, pts, p, w);
  if ((e = launch_scan(w.cnt, p.ncells + 1, w.bsum, s, w.occ)) != hipSuccess) return e;
  DPC_LAUNCH((k_scatter), blocks_for(p.n, kBlock), kBlock, s, p, w);
  DPC_LAUNCH((k_gather_pts), blocks_for(p.n, kBlock), kBlock, s, pts, p, w);
  if (p.lanes) return hipGetLastError();  // one query per lane: no strip tasks
  DPC_LAUNCH((k_strip_count), blocks_for(p.nstrips + 1, kBlock), kBlock, s, p, w);
  if ((e = launch_scan(w.tcnt, p.nstrips + 1, w.bsum, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_strip_tasks), blocks_for(p.nstrips, kBlock), kBlock, s, p, w);
  return hipGetLastError();
}

hipError_t gather_rank_keys(const Plan &p, const Ws &w, const int32_t *rho, hipStream_t s) {
  DPC_LAUNCH((k_gather_rank_keys), blocks_for(p.n, kBlock), kBlock, s, p, rho, w);
  return hipGetLastError();
}

hipError_t rank_sort(const Plan &p, const Ws &w, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32(w.rcnt, 0u, p.n + 1, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_rank_hist), blocks_for(p.n, int(kRankChunk)), kBlock, s, p, w);
  if ((e = launch_scan(w.rcnt, p.n + 1, w.bsum, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_rank_scatter), blocks_for(p.n, kBlock), kBlock, s, p, w);
  return hipGetLastError();
}

hipError_t launch_rank_gather(const Plan &p, const Ws &w, hipStream_t s) {
  DPC_LAUNCH((k_rank_gather), blocks_for(p.n, kBlock * 8), kBlock, s, p, w);
  return hipGetLastError();
}

// ---- many-job host side ----

hipError_t batch_start(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.one)) DPC_LAUNCH((kb_start), vgrid(B.one), kBlock, s, B.jobs, B.one, 1);
  return hipGetLastError();
}

hipError_t batch_build_grid(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.cells)) DPC_LAUNCH((kb_fill<kArrCells>), vgrid(B.cells), kBlock, s, B.jobs, B.cells);
  if (vgrid(B.pts)) DPC_LAUNCH((kb_cell_keys), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  batch_scan<kArrCells>(B, B.cells, s);
  if (vgrid(B.pts)) DPC_LAUNCH((kb_scatter), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  if (vgrid(B.pts)) DPC_LAUNCH((kb_gather_pts), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  // (jobs in lane mode own no strip virtual blocks)
  if (vgrid(B.strips)) DPC_LAUNCH((kb_strip_count), vgrid(B.strips), kBlock, s, B.jobs, B.strips);
  batch_scan<kArrStrips>(B, B.strips, s);
  if (vgrid(B.strips)) DPC_LAUNCH((kb_strip_tasks), vgrid(B.strips), kBlock, s, B.jobs, B.strips);
  return hipGetLastError();
}

// (the density kernels left each job's rank keys in its workspace)
hipError_t batch_rank(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.pts)) {
    DPC_LAUNCH((kb_fill<kArrRank>), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
    DPC_LAUNCH((kb_rank_hist), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  }
  batch_scan<kArrRank>(B, B.pts, s);
  if (vgrid(B.pts)) DPC_LAUNCH((kb_rank_scatter), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  return hipGetLastError();
}

hipError_t batch_rank_gather(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.pts)) DPC_LAUNCH((kb_rank_gather), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  return hipGetLastError();
}

}  // namespace dpc
