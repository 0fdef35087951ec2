// Task geometry shared by the density and ring-1 kernels.
//
// A task is up to 64 consecutive cell-order points of one strip (cells x0..x1 of
// one row).  Its search window is, in every row adjacent to the query row
// (3^(d-1) rows), the contiguous cell range [x0 - 1, x1 + 1]: it contains the
// 3^d cells around every query's own cell, so it holds every point closer than
// d_cut to any query (Def. 1).  Cells are keyed row-major, so each of those row
// ranges is one contiguous run of the cell-ordered arrays.
#pragma once

#include "common.h"

namespace dpc {

template <int D>
struct Pow3 {
  static constexpr int value = 3 * Pow3<D - 1>::value;
};
template <>
struct Pow3<0> {
  static constexpr int value = 1;
};

template <int D>
struct TaskGeom {
  uint32_t qb, qe;     // query positions [qb, qe)
  int32_t c[D > 1 ? D - 1 : 1];  // cell coordinates of the query row
  int32_t x0, x1;      // last-dimension cells of the first and last query
};

// Decode task t (all values uniform across the wave).
template <int D>
__device__ __forceinline__ TaskGeom<D> decode_task(const Plan &p, const uint4 *tasks, const int32_t *spts,
                                                   uint32_t t) {
  TaskGeom<D> g;
  DPC_CONST(uint32_t) *tc = as_const(reinterpret_cast<const uint32_t *>(tasks));
  g.qb = uniform(uint32_t(tc[4 * int64_t(t)]));
  g.qe = uniform(uint32_t(tc[4 * int64_t(t) + 1]));
  int64_t row = int64_t(uniform(uint32_t(tc[4 * int64_t(t) + 2]))) / p.nsx;
#pragma unroll
  for (int t2 = D - 2; t2 >= 0; --t2) {
    g.c[t2] = int32_t(row % p.nc);
    row /= p.nc;
  }
  DPC_CONST(int32_t) *sp = as_const(spts);
  g.x0 = uniform(sp[int64_t(g.qb) * D + (D - 1)] / p.L);
  g.x1 = uniform(sp[int64_t(g.qe - 1) * D + (D - 1)] / p.L);
  return g;
}

// Candidate range of row offset r (0 <= r < 3^(D-1)) of a task's window; empty
// if the row lies outside the grid.
template <int D>
__device__ __forceinline__ void window_row(const Plan &p, const TaskGeom<D> &g, int r, const uint32_t *start,
                                           uint32_t *b, uint32_t *e) {
  int64_t rowk = 0;
  bool ok = true;
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    const int32_t nb = g.c[t] + (r % 3) - 1;
    r /= 3;
    ok = ok && nb >= 0 && nb < p.nc;
    rowk = rowk * p.nc + nb;
  }
  *b = 0;
  *e = 0;
  if (ok) {
    const int64_t klo = rowk * p.nc + max(g.x0 - 1, 0);
    const int64_t khi = rowk * p.nc + min(g.x1 + 1, p.nc - 1);
    *b = start[klo];
    *e = start[khi + 1];
  }
}

// Squared distance from a query to the outside of its task window, as a bound:
// every point outside the window has D2 >= the returned value (kNoKey-like
// UINT64_MAX when the window reaches the grid boundary on every side).
template <int D>
__device__ __forceinline__ uint64_t window_exterior_d2(const Plan &p, const TaskGeom<D> &g, const int32_t *x) {
  int64_t gap = INT64_MAX;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const int32_t lo = (t == D - 1) ? g.x0 - 1 : g.c[t] - 1;
    const int32_t hi = (t == D - 1) ? g.x1 + 1 : g.c[t] + 1;
    if (lo >= 1) gap = min(gap, int64_t(x[t]) - int64_t(lo) * p.L + 1);
    if (hi <= p.nc - 2) gap = min(gap, int64_t(hi + 1) * p.L - int64_t(x[t]));
  }
  return gap == INT64_MAX ? ~uint64_t(0) : uint64_t(gap) * uint64_t(gap);
}

}  // namespace dpc
