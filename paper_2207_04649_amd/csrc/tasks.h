// Task geometry shared by the density and dependent-search kernels.
//
// The cells index the first gm coordinates of a point (gm <= d, a plan value);
// a row fixes the first gm - 1 cell coordinates, and a strip is a run of cells
// of one row along grid dimension gm - 1.  A task is up to 64 cell-order points
// of one strip.  Its search window of radius K cells is, in every row within K
// of the task's row ((2K+1)^(gm-1) rows), the contiguous cell range
// [x0 - K, x1 + K], where x0..x1 are the cells of the task's points along the
// strip dimension.  Cells are keyed row-major, so each row range is one
// contiguous run of the cell-ordered arrays.  Coordinates past gm are not
// indexed: the projection onto the grid dimensions never increases a distance,
// so the windows still hold every point they must, and distances are always
// computed over all d coordinates.
//
// Rows and row ranges are clipped to a radius when one is known: a row whose
// nearest coordinate is farther than the radius from the task's row is
// skipped, and the cell range is cut to the cells within the radius of the
// task's span along the strip dimension.  With the cut-off distance as the
// radius (local density, Def. 1) the window follows the d_cut-ball instead of
// its bounding box.
//
// Loops over grid dimensions run over all D - 1 (or D) indices, fully
// unrolled, with a guard on gm, so register arrays are indexed by constants.
#pragma once

#include "common.h"

namespace dpc {

template <int D>
struct TaskGeom {
  int32_t c[D > 1 ? D - 1 : 1];  // cell coordinates of the task's row (first gm - 1 used)
  int32_t x0, x1;                // strip-dimension cells of the task's points
  int32_t xlo, xhi;              // strip-dimension coordinate span of the task's points
};

// Row coordinates of strip `strip`.
template <int D>
__device__ __forceinline__ void strip_row(const Plan &p, uint32_t strip, TaskGeom<D> &g) {
  int64_t row = int64_t(strip) / p.nsx;
#pragma unroll
  for (int t = D - 2; t >= 0; --t) {
    g.c[t] = 0;
    if (t < p.gm - 1) {
      g.c[t] = int32_t(row % p.nc);
      row /= p.nc;
    }
  }
}

// Squared distance from the task's row to row offset o of a window (0 for the
// row itself): the gap between the row cells, per dimension, summed.
__device__ __forceinline__ int64_t row_gap(int32_t o, int32_t L) {
  const int32_t a = o < 0 ? -o : o;
  return a == 0 ? 0 : int64_t(a - 1) * L + 1;
}

// Rows of a window of radius K: (2K+1)^(gm-1).
__device__ __forceinline__ int64_t window_rows(const Plan &p, int K) {
  int64_t r = 1;
  for (int t = 0; t < p.gm - 1; ++t) r *= 2 * K + 1;
  return r;
}

// Largest r with r * r <= v (v < 2^62).
__device__ __forceinline__ int64_t isqrt_floor(uint64_t v) {
  int64_t r = int64_t(__builtin_sqrt(double(v)));
  while (r > 0 && uint64_t(r) * uint64_t(r) > v) --r;
  while (uint64_t(r + 1) * uint64_t(r + 1) <= v) ++r;
  return r;
}

// Candidate range [b, e) of row r (0 <= r < window_rows(p, K)) of the window of
// radius K, clipped to squared radius `clip2` (no clipping when clip2 is
// UINT64_MAX).  Empty if the row is outside the grid or beyond the radius.
template <int D>
__device__ __forceinline__ void window_row(const Plan &p, const TaskGeom<D> &g, int K, int r, uint64_t clip2,
                                           const uint32_t *start, uint32_t *b, uint32_t *e) {
  *b = 0;
  *e = 0;
  int64_t rowk = 0, dy2 = 0;
  bool ok = true;
  const int side = 2 * K + 1;
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    if (t < p.gm - 1) {
      const int32_t o = r % side - K;
      r /= side;
      const int32_t nb = g.c[t] + o;
      ok = ok && nb >= 0 && nb < p.nc;
      rowk = rowk * p.nc + nb;
      const int64_t gy = row_gap(o, p.L);
      dy2 += gy * gy;
    }
  }
  if (!ok) return;
  int32_t lo = max(g.x0 - K, 0), hi = min(g.x1 + K, p.nc - 1);
  if (clip2 != ~uint64_t(0)) {
    if (uint64_t(dy2) > clip2) return;
    const int64_t hw = isqrt_floor(clip2 - uint64_t(dy2));
    // clamped into [0, 2^17) first, so the divisions are 32-bit
    const int32_t a = int32_t(max(int64_t(g.xlo) - hw, int64_t(0)));
    const int32_t c = int32_t(min(int64_t(g.xhi) + hw, int64_t(DPC_COORD_LIMIT - 1)));
    lo = max(lo, a / p.L);
    hi = min(hi, c / p.L);
    if (lo > hi) return;
  }
  *b = start[rowk * p.nc + lo];
  *e = start[rowk * p.nc + hi + 1];
}

// Squared distance from a point to the outside of the unclipped window of
// radius K: every point outside has D2 >= the returned value, since its gap in
// one grid dimension alone is that large (UINT64_MAX when the window reaches the
// grid boundary on every side).
template <int D>
__device__ __forceinline__ uint64_t window_exterior_d2(const Plan &p, const TaskGeom<D> &g, int K, const int32_t *x) {
  int64_t gap = INT64_MAX;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    if (t < p.gm) {
      const bool last = t == p.gm - 1;
      const int32_t lo = last ? g.x0 - K : g.c[t < D - 1 ? t : 0] - K;
      const int32_t hi = last ? g.x1 + K : g.c[t < D - 1 ? t : 0] + K;
      if (lo >= 1) gap = min(gap, int64_t(x[t]) - int64_t(lo) * p.L + 1);
      if (hi <= p.nc - 2) gap = min(gap, int64_t(hi + 1) * p.L - int64_t(x[t]));
    }
  }
  return gap == INT64_MAX ? ~uint64_t(0) : uint64_t(gap) * uint64_t(gap);
}

// Wave-wide minimum / maximum of a 32-bit value.
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off, kWave);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Finish a task's geometry from its points' strip-dimension coordinates (lanes
// holding a valid point pass valid = true; all 64 lanes call this).
template <int D>
__device__ __forceinline__ void task_span(const Plan &p, TaskGeom<D> &g, int32_t xlast, bool valid) {
  g.xlo = uniform(wave_min_i32(valid ? xlast : INT32_MAX));
  g.xhi = uniform(wave_max_i32(valid ? xlast : INT32_MIN));
  g.x0 = g.xlo / p.L;
  g.x1 = g.xhi / p.L;
}

}  // namespace dpc
