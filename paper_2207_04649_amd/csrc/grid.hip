// Grid construction (counting sort of points into d_cut-sized cells), the
// density-rank sort, and the device-wide exclusive scan both use.
//
// The cells replace the paper's kd-tree (Section 3) as the range-search index:
// with cell side L >= floor(sqrt(R - 1)), R = ceil(d_cut^2), every point closer
// than d_cut to p lies in the 3^d cells around p's cell (Def. 1).
#include "common.h"

namespace dpc {
namespace {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

// ---- exclusive scan of u32, three passes over tiles of kScanTile items ----

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[kBlock / kWave];
  const int lane = lane_id(), wave = threadIdx.x / kWave;
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

// Tile-local exclusive scan; writes each tile's total to bsum.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *data, int64_t count, uint32_t *bsum) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < count ? data[i] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < count) data[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup scans the tile totals in place (any count, in rounds of kScanTile).
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t *bsum, int64_t count) {
  uint32_t carry = 0;
  for (int64_t round = 0; round < count; round += kScanTile) {
    const int64_t base = round + int64_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      v[k] = i < count ? bsum[i] : 0u;
      sum += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, &total) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      if (i < count) bsum[i] = run;
      run += v[k];
    }
    carry += total;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *data, int64_t count, const uint32_t *bsum) {
  const uint32_t add = bsum[blockIdx.x];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
    int64_t i = base + k;
    if (i < count) data[i] += add;
  }
}

// ---- grid build ----

// Cell key of every point (row-major over the cell coordinates, last dimension
// fastest) and its slot in the cell.  Out-of-range coordinates are clamped and flagged.
__global__ void k_cell_keys(const int32_t *__restrict__ pts, Plan p, uint32_t *__restrict__ cnt,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ slot,
                            DevHeader *__restrict__ hdr) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  uint32_t k = 0;
  bool bad = false;
  for (int t = 0; t < p.d; ++t) {
    int32_t x = pts[i * p.d + t];
    if (x < 0 || x >= DPC_COORD_LIMIT) {
      bad = true;
      x = x < 0 ? 0 : DPC_COORD_LIMIT - 1;
    }
    k = k * uint32_t(p.nc) + uint32_t(x / p.L);
  }
  if (bad) atomicOr(&hdr->status, 1u);
  key[i] = k;
  slot[i] = atomicAdd(&cnt[k], 1u);
}

// Place every point at start[key] + slot: clamped coordinates, their packed low
// 16 bits, and the id.
__global__ void k_scatter(const int32_t *__restrict__ pts, Plan p, const uint32_t *__restrict__ start,
                          const uint32_t *__restrict__ key, const uint32_t *__restrict__ slot,
                          int32_t *__restrict__ spts, uint32_t *__restrict__ spk, int32_t *__restrict__ sid) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int64_t pos = int64_t(start[key[i]]) + slot[i];
  uint32_t w = 0;
  for (int t = 0; t < p.d; ++t) {
    int32_t x = pts[i * p.d + t];
    x = x < 0 ? 0 : (x >= DPC_COORD_LIMIT ? DPC_COORD_LIMIT - 1 : x);
    spts[pos * p.d + t] = x;
    w |= (uint32_t(x) & 0xFFFFu) << (16 * (t & 1));
    if (t & 1) {
      spk[pos * p.words + (t >> 1)] = w;
      w = 0;
    }
  }
  if (p.d & 1) spk[pos * p.words + (p.d >> 1)] = w;
  sid[pos] = int32_t(i);
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

__global__ void k_strip_count(Plan p, const uint32_t *__restrict__ start, uint32_t *__restrict__ tcnt) {
  int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= p.nstrips) return;
  uint32_t b, e;
  strip_range(p, s, start, &b, &e);
  tcnt[s] = (e - b + kQueryChunk - 1) / kQueryChunk;
}

__global__ void k_strip_tasks(Plan p, const uint32_t *__restrict__ start, const uint32_t *__restrict__ toff,
                              uint4 *__restrict__ tasks, DevHeader *__restrict__ hdr) {
  int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s == 0) hdr->ntasks = toff[p.nstrips];
  if (s >= p.nstrips) return;
  uint32_t b, e;
  strip_range(p, s, start, &b, &e);
  uint32_t t = toff[s];
  for (uint32_t q = b; q < e; q += kQueryChunk, ++t)
    tasks[t] = make_uint4(q, min(q + uint32_t(kQueryChunk), e), uint32_t(s), 0u);
}

// (rho << 32) | ~id for every cell-order position, from the caller's rho.  A
// density outside [1, n] (not produced by dpc_density) is clamped and flagged,
// so every bucket index stays in range.
__global__ void k_gather_rank_keys(Plan p, const int32_t *__restrict__ rho, const int32_t *__restrict__ sid,
                                   uint64_t *__restrict__ sK, DevHeader *__restrict__ hdr) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= p.n) return;
  const int32_t id = sid[q];
  int64_t r = rho[id];
  if (r < 1 || r > p.n) {
    atomicOr(&hdr->status, 2u);
    r = r < 1 ? 1 : p.n;
  }
  sK[q] = (uint64_t(r) << 32) | uint32_t(~uint32_t(id));
}

// ---- density-rank sort: order by rho descending; equal rho share a bucket ----

// Bucket slots of the density-rank sort.  Most densities are small and many
// points share one, so a block first counts its small densities in LDS and then
// claims each bucket's slots with one global atomic; densities of kRankBins or
// more take a global atomic each.
constexpr int kRankBins = 2048;
constexpr int kRankItems = 4;  // points per thread

__global__ __launch_bounds__(kBlock) void k_rank_hist(Plan p, const uint64_t *__restrict__ sK,
                                                      uint32_t *__restrict__ rcnt, uint32_t *__restrict__ slot) {
  __shared__ uint32_t bins[kRankBins];
  for (int b = threadIdx.x; b < kRankBins; b += kBlock) bins[b] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kBlock * kRankItems;
  uint32_t local[kRankItems];
  int64_t rho[kRankItems];
#pragma unroll
  for (int k = 0; k < kRankItems; ++k) {
    const int64_t q = base + int64_t(k) * kBlock + threadIdx.x;
    rho[k] = 0;
    local[k] = 0;
    if (q < p.n) {
      int64_t r = int64_t(sK[q] >> 32);
      r = r < 1 ? 1 : (r > p.n ? p.n : r);
      rho[k] = r;
      if (r <= kRankBins)
        local[k] = atomicAdd(&bins[r - 1], 1u);
      else
        slot[q] = atomicAdd(&rcnt[p.n - r], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kRankBins; b += kBlock) {
    const uint32_t c = bins[b];
    if (c && b + 1 <= p.n) bins[b] = atomicAdd(&rcnt[p.n - (b + 1)], c);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRankItems; ++k) {
    const int64_t q = base + int64_t(k) * kBlock + threadIdx.x;
    if (q < p.n && rho[k] <= kRankBins) slot[q] = bins[rho[k] - 1] + local[k];
  }
}

__global__ void k_rank_scatter(Plan p, const uint64_t *__restrict__ sK, const uint32_t *__restrict__ rstart,
                               const uint32_t *__restrict__ slot, const int32_t *__restrict__ spts,
                               const int32_t *__restrict__ sid, int32_t *__restrict__ rpts,
                               int32_t *__restrict__ rid) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= p.n) return;
  int64_t rho = int64_t(sK[q] >> 32);
  rho = rho < 1 ? 1 : (rho > p.n ? p.n : rho);
  const int64_t r = int64_t(rstart[p.n - rho]) + slot[q];
  for (int t = 0; t < p.d; ++t) rpts[r * p.d + t] = spts[q * p.d + t];
  rid[r] = sid[q];
}

__global__ void k_clear_status(DevHeader *hdr) {
  if (threadIdx.x == 0) hdr->status = 0;
}

// Work counters of one call; `grid` also clears the task count of the grid build.
__global__ void k_reset_counters(DevHeader *hdr, int grid) {
  if (threadIdx.x == 0) {
    if (grid) hdr->ntasks = 0;
    hdr->n_unres = 0;
    hdr->n_peaks = 0;
  }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *ptr, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  unsigned blocks = blocks_for(count, kBlock);
  if (blocks > 65536u) blocks = 65536u;
  DPC_LAUNCH((k_fill_u32), blocks, kBlock, s, ptr, value, count);
  return hipGetLastError();
}

hipError_t launch_scan(uint32_t *data, int64_t count, uint32_t *bsum, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned tiles = blocks_for(count, kScanTile);
  DPC_LAUNCH((k_scan_tiles), tiles, kBlock, s, data, count, bsum);
  DPC_LAUNCH((k_scan_sums), 1, kBlock, s, bsum, tiles);
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

hipError_t build_grid(const Plan &p, const Ws &w, const int32_t *pts, hipStream_t s) {
  hipError_t e;
  if ((e = reset_counters(w.hdr, true, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(w.cnt, 0u, p.ncells + 1, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_cell_keys), blocks_for(p.n, kBlock), kBlock, s, pts, p, w.cnt, w.key, w.slot, w.hdr);
  if ((e = launch_scan(w.cnt, p.ncells + 1, w.bsum, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_scatter), blocks_for(p.n, kBlock), kBlock, s, pts, p, w.cnt, w.key, w.slot, w.spts, w.spk, w.sid);
  DPC_LAUNCH((k_strip_count), blocks_for(p.nstrips, kBlock), kBlock, s, p, w.cnt, w.tcnt);
  if ((e = launch_fill_u32(w.tcnt + p.nstrips, 0u, 1, s)) != hipSuccess) return e;
  if ((e = launch_scan(w.tcnt, p.nstrips + 1, w.bsum, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_strip_tasks), blocks_for(p.nstrips, kBlock), kBlock, s, p, w.cnt, w.tcnt, w.tasks, w.hdr);
  return hipGetLastError();
}

hipError_t gather_rank_keys(const Plan &p, const Ws &w, const int32_t *rho, hipStream_t s) {
  DPC_LAUNCH((k_gather_rank_keys), blocks_for(p.n, kBlock), kBlock, s, p, rho, w.sid, w.sK, w.hdr);
  return hipGetLastError();
}

hipError_t rank_sort(const Plan &p, const Ws &w, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32(w.rcnt, 0u, p.n + 1, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_rank_hist), blocks_for(p.n, kBlock * kRankItems), kBlock, s, p, w.sK, w.rcnt, w.slot);
  if ((e = launch_scan(w.rcnt, p.n + 1, w.bsum, s)) != hipSuccess) return e;
  DPC_LAUNCH((k_rank_scatter), blocks_for(p.n, kBlock), kBlock, s, p, w.sK, w.rcnt, w.slot, w.spts, w.sid, w.rpts,
                                                           w.rid);
  return hipGetLastError();
}

}  // namespace dpc
