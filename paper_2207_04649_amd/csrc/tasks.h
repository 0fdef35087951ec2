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

// ---------------------------------------------------------------- one query per lane
//
// In lane form every lane walks its own window: the rows within K of its cell
// (the first gm - 1 cell coordinates), and in each row the strip-dimension cells
// within K, clipped to a squared radius.  The row offsets are the same for every
// lane (a wave-uniform walk); the cell ranges differ per lane.

constexpr int kLaneRowChunk = 8;  // window rows whose cell ranges a lane loads before scanning them (K > 1)

template <int D>
struct LaneGeom {
  int32_t x[D];  // the query's coordinates
  int32_t c[D];  // its cell coordinates (first gm used)
  int32_t xs;    // the coordinate along the strip dimension (gm - 1), and its cell
  int32_t cs;
};

template <int D>
__device__ __forceinline__ void lane_geom(const Plan &p, const int32_t *src, LaneGeom<D> &g) {
  if (D == 4) {
    const int4 v = *reinterpret_cast<const int4 *>(src);  // rows of 16 bytes, 16-byte aligned
    g.x[0] = v.x;
    g.x[1] = v.y;
    g.x[2 % D] = v.z;
    g.x[3 % D] = v.w;
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) g.x[k] = src[k];
  }
#pragma unroll
  for (int t = 0; t < D; ++t) g.c[t] = t < p.gm ? g.x[t] / p.L : 0;
  // read again from memory: indexing x by the run-time gm would move the
  // register arrays to scratch memory
  g.xs = src[p.gm - 1];
  g.cs = g.xs / p.L;
}

// Row offsets of a window of radius K, as an odometer over the first gm - 1
// grid dimensions.  With `zigzag` each digit runs 0, -1, +1, -2, +2, ..., so the
// query's own row comes first and nearer rows early (a search clipped to its
// best distance then skips more rows).
template <int D>
struct RowWalk {
  int32_t i[D > 1 ? D - 1 : 1];
  bool zigzag;
  __device__ __forceinline__ RowWalk(int K, bool zz) : zigzag(zz) {
#pragma unroll
    for (int t = 0; t < (D > 1 ? D - 1 : 1); ++t) i[t] = 0;
    (void)K;
  }
  __device__ __forceinline__ int32_t offset(int t, int K) const {
    if (!zigzag) return i[t] - K;
    return (i[t] & 1) ? -((i[t] + 1) >> 1) : (i[t] >> 1);
  }
  __device__ __forceinline__ void next(const Plan &p, int K) {
#pragma unroll
    for (int t = 0; t < D - 1; ++t) {
      if (t < p.gm - 1) {
        if (++i[t] <= 2 * K) return;
        i[t] = 0;
      }
    }
  }
  // `step` rows on (a carry through the digits).
  __device__ __forceinline__ void advance(const Plan &p, int K, int step) {
    const int side = 2 * K + 1;
    int carry = step;
#pragma unroll
    for (int t = 0; t < D - 1; ++t) {
      if (t < p.gm - 1 && carry) {
        i[t] += carry;
        carry = 0;
        while (i[t] >= side) {
          i[t] -= side;
          ++carry;
        }
      }
    }
  }
};

// Gap from coordinate x to cell cc along a grid dimension (0 inside the cell).
__device__ __forceinline__ int64_t cell_gap(int32_t x, int32_t cc, int32_t L) {
  const int64_t lo = int64_t(cc) * L, hi = lo + L - 1;
  return x < lo ? lo - x : (x > hi ? int64_t(x) - hi : 0);
}

// Candidate range [b, e) of the walk's current row for one lane, clipped to
// squared radius `clip` (cells whose nearest point is farther are left out).
// False when the row is outside the grid, beyond the radius, or empty.
template <int D>
__device__ __forceinline__ bool lane_row(const Plan &p, const LaneGeom<D> &g, const RowWalk<D> &rw, int K, int64_t clip,
                                         const uint32_t *__restrict__ start, uint32_t *b, uint32_t *e) {
  int64_t rowk = 0, dy2 = 0;
  bool ok = true;
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    if (t < p.gm - 1) {
      const int32_t nb = g.c[t] + rw.offset(t, K);
      ok = ok && nb >= 0 && nb < p.nc;
      rowk = rowk * p.nc + nb;
      const int64_t gp = cell_gap(g.x[t], nb, p.L);
      dy2 += gp * gp;
    }
  }
  if (!ok || dy2 > clip) return false;
  const int s = p.gm - 1;
  const int32_t xs = g.xs, cs = g.cs;
  int32_t lo = cs - K, hi = cs + K;
  while (lo < cs) {
    const int64_t gp = cell_gap(xs, lo, p.L);
    if (gp * gp + dy2 <= clip) break;
    ++lo;
  }
  while (hi > cs) {
    const int64_t gp = cell_gap(xs, hi, p.L);
    if (gp * gp + dy2 <= clip) break;
    --hi;
  }
  lo = max(lo, 0);
  hi = min(hi, p.nc - 1);
  if (K == 1) {
    // The four entries start[cs - 1 .. cs + 2] of the row hold both ends of any
    // range within one cell of cs: one 16-byte load (dword-aligned loads of several
    // dwords are allowed on this target; the table has a slack entry on each side).
    uint4 v;
    __builtin_memcpy(&v, start + (rowk * p.nc + cs - 1), 16);
    const int ib = lo - (cs - 1), ie = hi + 1 - (cs - 1);  // 0..3
    *b = ib == 0 ? v.x : (ib == 1 ? v.y : (ib == 2 ? v.z : v.w));
    *e = ie == 0 ? v.x : (ie == 1 ? v.y : (ie == 2 ? v.z : v.w));
  } else {
    *b = start[rowk * p.nc + lo];
    *e = start[rowk * p.nc + hi + 1];
  }
  return *b < *e;
}

// Square root of a float >= 0 by the hardware instruction (not correctly
// rounded; callers add a margin).
__device__ __forceinline__ float sqrt_approx(float v) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_sqrtf(v);
#else
  return __builtin_sqrtf(v);
#endif
}

// A bound r >= sqrt(v) (v < 2^40) from the float square root: the conversion and
// the root are each within a relative 2^-23 of exact, so a 2^-20 margin and one
// unit cover them.
__device__ __forceinline__ int32_t sqrt_ceil_bound(uint64_t v) {
  const float f = __builtin_sqrtf(float(v));
  return int32_t(f * (1.0f + 0x1p-20f)) + 1;
}

// Gap from coordinate x to cell cc (side L) along one dimension, 32-bit and
// branch-free (at most one of the two differences is positive).
__device__ __forceinline__ uint32_t cell_gap32(int32_t x, int32_t cc, int32_t L) {
  const int32_t lo = cc * L, hi = lo + L - 1;
  return uint32_t(max(max(lo - x, x - hi), 0));
}

// Exact squared distance: each |dx| < 2^31, its square formed as a 32 x 32 -> 64
// bit product.
template <int D>
__device__ __forceinline__ uint64_t exact_d2_u(const int32_t *a, const int32_t *b) {
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int32_t df = a[k] - b[k];
    const uint32_t ad = uint32_t(df < 0 ? -df : df);
    s += uint64_t(ad) * uint64_t(ad);
  }
  return s;
}

// False when none of the table cells c0 .. c1 (flat indices, c0 <= c1) holds a
// point, by the occupancy bits (one per 8 cells): a row piece of empty cells then
// needs no table lookup.  Pieces wider than 32 groups are taken as occupied.
__device__ __forceinline__ bool cells_occupied(const uint32_t *__restrict__ occ, int32_t c0, int32_t c1) {
  const uint32_t ga = uint32_t(c0) >> 3, gb = uint32_t(c1) >> 3;
  if (gb - ga >= 32u) return true;
  const uint32_t w0 = occ[ga >> 5], w1 = occ[gb >> 5];
  const uint64_t bits = ((uint64_t(w1) << 32) | w0) >> (ga & 31u);  // w1 == w0 when one word holds both
  const uint64_t mask = (uint64_t(2) << (gb - ga)) - 1u;
  return (((ga >> 5) == (gb >> 5) ? uint64_t(w0 >> (ga & 31u)) : bits) & mask) != 0u;
}

constexpr int ipow3(int e) { return e <= 0 ? 1 : 3 * ipow3(e - 1); }

// Rows of a radius-1 window whose candidate ranges one lane queues in LDS before
// testing them as one stream (a plane of the window when D = 4).
template <int D>
constexpr int walk_chunk() {
  return ipow3(D - 1) < 9 ? ipow3(D - 1) : 9;
}
constexpr int kWalkQueue = 9;  // LDS queue entries per lane (walk_chunk<D>() <= this)



// The radius-1 window of a lane's cell when every coordinate is indexed (gm ==
// D), with compile-time row offsets: 3^(D-1) rows, the lane's own row first
// (digits run 0, -1, +1).  A chunk of walk_chunk<D>() rows has its cell ranges
// loaded together (two words of start[x - 1 .. x + 2] per row); the non-empty
// ranges go to the lane's LDS queue (entries `queue[k * kBlock]`, k <
// kWalkQueue) and their candidates are then tested as one stream, so a wave
// runs as many test steps as its busiest lane has candidates in the chunk (not
// the sum over rows of each row's busiest lane); with PAIR two candidates per
// step, their loads in flight together.  `clip()` gives the squared
// radius, read once per chunk (a smaller one later only leaves extra
// candidates); `test(j, take)` tests candidate j and keeps the result only when
// `take` (its loads run either way, on a valid j).  Returns the candidates tested.
// T holds squared gaps and radii: 32 bits when they are known to stay below
// 2^31 (the packed path's windows), else 64.
template <int D, class T, bool PAIR, class ClipF, class TestF>
__device__ __forceinline__ uint32_t walk_k1(const Plan &p, const LaneGeom<D> &g, const uint32_t *__restrict__ start,
                                            uint2 *queue, ClipF clip_fn, TestF test) {
  constexpr int RD = D - 1;          // row dimensions
  constexpr int NR = ipow3(RD);      // rows
  constexpr int RA = RD > 0 ? RD : 1;
  constexpr int CH = walk_chunk<D>();
  static_assert(CH <= kWalkQueue, "queue too short for a chunk");
  const int32_t L = p.L, nc = p.nc;
  T gy[RA][3];
  int32_t part[RA][3];
  bool okd[RA][3];
  int32_t stride = nc;  // the table index of row digits is sum(part) + x: row-major, x fastest
#pragma unroll
  for (int t = RD - 1; t >= 0; --t) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int32_t nb = g.c[t] + (i == 0 ? 0 : (i == 1 ? -1 : 1));
      okd[t][i] = nb >= 0 && nb < nc;
      const T gp = T(cell_gap(g.x[t], nb, L));
      gy[t][i] = gp * gp;
      part[t][i] = nb * stride;
    }
    stride *= nc;
  }
  const int32_t xs = g.x[D - 1], cs = g.c[D - 1];
  const T gl = T(cell_gap(xs, cs - 1, L)), gh = T(cell_gap(xs, cs + 1, L));
  const T gsl = gl * gl, gsh = gh * gh;
  const bool lo_in = cs >= 1, hi_in = cs + 1 < nc;
  const uint32_t *base = start + (cs - 1);
  uint32_t tested = 0;
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += CH) {
    const T clip = clip_fn();
    uint32_t vb[CH], ve[CH];
    T dy2[CH];
    bool ok[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int r = r0 + c;
      T dy = 0;
      bool in = true;
      int32_t rowk = 0;
#pragma unroll
      for (int t = 0; t < RD; ++t) {
        const int i = (r / ipow3(t)) % 3;
        dy += gy[t][i];
        in = in && okd[t][i];
        rowk += part[t][i];
      }
      dy2[c] = dy;
      ok[c] = in && dy <= clip;
      // the row's range: from start[x - 1] when cell x - 1 is within the radius
      // (else start[x]) to start[x + 2] when cell x + 1 is (else start[x + 1])
      const int bo = (lo_in && gsl + dy <= clip) ? 0 : 1, eo = (hi_in && gsh + dy <= clip) ? 3 : 2;
      vb[c] = ve[c] = 0;
      if (ok[c]) {
        vb[c] = base[rowk + bo];
        ve[c] = base[rowk + eo];
      }
    }
    uint32_t m = 0, total = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const uint32_t b = vb[c], e = ve[c];
      if (ok[c] && b < e) {
        queue[m * kBlock] = make_uint2(b, e);
        ++m;
        total += e - b;
      }
    }
    if (PAIR) {
      // two candidates per step (both loads in flight together); the next queued
      // range is read one refill ahead
      uint32_t j = 0, e = 0, k = 1;
      uint2 nx = make_uint2(0u, 0u);
      if (m > 0) nx = queue[0];
      for (uint32_t t = 0; t < total; t += 2) {
        if (j == e) {
          j = nx.x;
          e = nx.y;
          if (k < m) nx = queue[k * kBlock];
          ++k;
        }
        const uint32_t j0 = j++;
        const bool two = t + 1 < total;
        if (two && j == e) {
          j = nx.x;
          e = nx.y;
          if (k < m) nx = queue[k * kBlock];
          ++k;
        }
        const uint32_t j1 = two ? j : j0;
        j += two ? 1u : 0u;
        test(j0, true);
        test(j1, two);
      }
    } else {
      uint32_t j = 0, e = 0, k = 0;
      for (uint32_t t = 0; t < total; ++t) {
        if (j == e) {  // the next queued range (never empty)
          const uint2 r = queue[k * kBlock];
          ++k;
          j = r.x;
          e = r.y;
        }
        test(j, true);
        ++j;
      }
    }
    tested += total;
  }
  return tested;
}

// Squared distance from x to the outside of the block of cells within K of its
// own cell (UINT64_MAX when the block covers the grid): every point outside has
// D2 >= this, since its gap in one grid dimension alone is that large.
template <int D>
__device__ __forceinline__ uint64_t lane_exterior_d2(const Plan &p, const LaneGeom<D> &g, int K) {
  int64_t gap = INT64_MAX;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    if (t < p.gm) {
      if (g.c[t] - K >= 1) gap = min(gap, int64_t(g.x[t]) - int64_t(g.c[t] - K) * p.L + 1);
      if (g.c[t] + K <= p.nc - 2) gap = min(gap, int64_t(g.c[t] + K + 1) * p.L - int64_t(g.x[t]));
    }
  }
  return gap == INT64_MAX ? ~uint64_t(0) : uint64_t(gap) * uint64_t(gap);
}

// W consecutive 32-bit words (one vector load when aligned: W = 2 or 4 words of
// an array with W-word elements from a 256-byte aligned base).
template <int W>
__device__ __forceinline__ void load_words(const uint32_t *src, uint32_t *c) {
  if (W == 2) {
    const uint2 v = *reinterpret_cast<const uint2 *>(src);
    c[0] = v.x;
    c[1 % W] = v.y;
  } else if (W == 4) {
    const uint4 v = *reinterpret_cast<const uint4 *>(src);
    c[0] = v.x;
    c[1 % W] = v.y;
    c[2 % W] = v.z;
    c[3 % W] = v.w;
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) c[k] = src[k];
  }
}

}  // namespace dpc
