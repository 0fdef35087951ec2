// Wave-cooperative range scan over the exact grid, for the approximate methods'
// per-point searches of radius d_cut.
#pragma once

#include "common.h"

namespace dpc {

// Runs of equal keys among consecutive lanes (points in cell order often share a
// cell of a coarser grid): the first lane of the calling lane's run, and whether
// the calling lane ends its run.  Every lane of the wave calls it.
struct WaveRun {
  int start;
  bool tail;
};

__device__ __forceinline__ WaveRun wave_run(uint32_t key) {
  const int lane = lane_id();
  const uint32_t prev = __shfl_up(key, 1, kWave), next = __shfl(key, (lane + 1) & (kWave - 1), kWave);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(start, off, kWave);
    if (lane >= off) start = max(start, o);
  }
  return WaveRun{start, lane == kWave - 1 || next != key};
}

// The combination by `op` of v over the lanes start .. lane of the calling lane's
// run (inclusive); at the run's tail, over the whole run.  Every lane calls it.
template <class T, class Op>
__device__ __forceinline__ T run_reduce(T v, int start, Op op) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const T o = __shfl_up(v, off, kWave);
    if (lane - off >= start) v = op(v, o);
  }
  return v;
}

// Calls f(j) on the calling lane for every cell-order position j of the exact
// grid's rows that can hold a point within d_cut of xq (the lane's own query):
// the same box as wave_near, row by row with an odometer.  For sparse data, where
// a query has few candidates and a wave's setup would cost more than its scan.
template <int D, class F>
__device__ __forceinline__ void lane_near(const Plan &p, const Ws &w, const int32_t *xq, F &&f) {
  const int32_t L = p.L, nc = p.nc, gm = p.gm, r0 = p.L0;
  const int last = gm - 1;
  int32_t lo[D], hi[D], cur[D];
  int32_t lo_l = 0, hi_l = 0;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    lo[t] = t < gm ? max(xq[t] - r0, 0) / L : 0;
    hi[t] = t < gm ? min(xq[t] + r0, DPC_COORD_LIMIT - 1) / L : 0;
    cur[t] = lo[t];
    if (t == last) {
      lo_l = lo[t];
      hi_l = hi[t];
    }
  }
  for (;;) {
    int64_t row = 0;
#pragma unroll
    for (int t = 0; t < D; ++t)
      if (t < last) row = row * nc + cur[t];
    const int64_t c0 = row * nc + lo_l;
    const uint32_t j0 = w.cnt[c0], j1 = w.cnt[c0 + (hi_l - lo_l) + 1];
    for (uint32_t j = j0; j < j1; ++j) f(j);
    bool carry = true;  // next row: an odometer over the dimensions before the last
#pragma unroll
    for (int t = D - 1; t >= 0; --t) {
      if (t < last && carry) {
        if (cur[t] < hi[t]) {
          ++cur[t];
          carry = false;
        } else {
          cur[t] = lo[t];
        }
      }
    }
    if (carry) break;
  }
}

// Per-wave LDS of wave_near: one group of up to 64 rows at a time.
struct NearLds {
  uint32_t off[kWave];  // exclusive prefix of the rows' point counts
  uint32_t j0[kWave];   // first cell-order position of each row
};

// Calls f(j) once, on some lane of the calling wave, for every cell-order position
// j of the exact grid's rows that can hold a point within d_cut of xq (the same for
// every lane): the box of radius floor(sqrt(R - 1)) over the first gm coordinates,
// whose cells along the last grid dimension form one run of positions per row.
// The rows are taken 64 at a time, one per lane; their runs are flattened by a
// prefix sum so that consecutive lanes read consecutive positions.
template <int D, class F>
__device__ __forceinline__ void wave_near(const Plan &p, const Ws &w, const int32_t *xq, NearLds &lds, F &&f) {
  const int lane = lane_id();
  const int32_t L = p.L, nc = p.nc, gm = p.gm, r0 = p.L0;
  const int last = gm - 1;
  int32_t lo[D], ext[D];
  int32_t lo_l = 0, ext_l = 1;
  uint32_t nrows = 1;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    lo[t] = 0;
    ext[t] = 1;
    if (t < gm) {
      const int32_t a = max(xq[t] - r0, 0) / L, b = min(xq[t] + r0, DPC_COORD_LIMIT - 1) / L;
      if (t == last) {
        lo_l = a;
        ext_l = b - a + 1;
      } else {
        lo[t] = a;
        ext[t] = b - a + 1;
        nrows *= uint32_t(ext[t]);
      }
    }
  }
  for (uint32_t g = 0; g < nrows; g += kWave) {
    const uint32_t r = g + uint32_t(lane);
    uint32_t len = 0, j0 = 0;
    if (r < nrows) {
      // row r in row-major order of the dimensions before the last
      uint32_t rem = r;
      int64_t row = 0, scale = 1;
#pragma unroll
      for (int t = D - 1; t >= 0; --t) {
        if (t < last) {
          const uint32_t dig = rem % uint32_t(ext[t]);
          rem /= uint32_t(ext[t]);
          row += int64_t(lo[t] + int32_t(dig)) * scale;
          scale *= nc;
        }
      }
      const int64_t c0 = row * nc + lo_l;
      j0 = w.cnt[c0];
      len = w.cnt[c0 + ext_l] - j0;
    }
    uint32_t total;
    const uint32_t off = wave_exclusive_scan(len, &total);
    lds.off[lane] = off;
    lds.j0[lane] = j0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t k = uint32_t(lane); k < total; k += kWave) {
      // the row holding flattened index k: the last with off <= k
      uint32_t a = 0, b = kWave - 1;
      while (a < b) {
        const uint32_t m = (a + b + 1) >> 1;
        if (lds.off[m] <= k) a = m;
        else b = m - 1;
      }
      f(lds.j0[a] + (k - lds.off[a]));
    }
    __builtin_amdgcn_wave_barrier();  // every lane has read the group before it is overwritten
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

}  // namespace dpc
