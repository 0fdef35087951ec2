// Approx-DPC (Section 4) on top of the exact path's grid and density kernels.
//
// The local densities are exact (Section 4.2); the exact path's kernels
// compute them.  A second grid of cells of side La (Section 4.1; for integer
// coordinates La = 1 + floor(sqrt((R - 1) / d)), the largest side that keeps
// every two points of a cell strictly within d_cut) is built as an open-
// addressing hash table over the occupied cells: each cell keeps its densest
// point p*(c) (the largest rank key (rho << 32 | ~id)) and its smallest
// density.  The rules of Section 4.3 then give most points a dependent point
// in O(1) or one range search:
//
//   * a point that is not its cell's p* takes p*(c);
//   * p*(c) takes p*(c') of a cell c' that holds a point strictly within d_cut
//     of it and whose points all have a higher density (the qualifying cell with
//     the smallest cell coordinates, first dimension most significant);
//
// both with the dependent distance d_cut.  The p* points no cell qualifies for
// go to the exact path's ring search and prefix scan, which start from an empty
// window (Defs. 2-3).  The paper's own exact step (density-sorted subsets with
// one kd-tree each, Section 4.3) is replaced by that search: both return the
// exact dependent point.
#include "common.h"
#include "near.h"
#include "prof.h"

namespace dpc {
namespace {

constexpr uint32_t kEmpty = 0xffffffffu;
// D2 field of a packed (D2 << kIdBits | id) key that marks an approximate
// dependent point: no two in-range points are that far apart
// (8 (2^17 - 1)^2 < 2^37 - 2), and it differs from kNoKey's.
constexpr uint64_t kApproxD2 = (uint64_t(1) << (64 - kIdBits)) - 2;

struct AxWs {
  uint32_t *cnt;    // [4] counters: p* points
  uint32_t *rep;    // [slots] cell-order position of the point that opened the slot, kEmpty if free
  uint64_t *top;    // [slots] largest rank key of the cell (its p*), 0 before any point
  uint32_t *minrho; // [slots] smallest density of the cell
  uint32_t *ent;    // [n] table slot of each cell-order position
  uint32_t *plist;  // [n] cell-order positions of the p* points
};

AxWs ax_resolve(const ApproxPlan &a, void *base) {
  char *b = static_cast<char *>(base);
  AxWs x;
  x.cnt = reinterpret_cast<uint32_t *>(b + a.o_cnt);
  x.rep = reinterpret_cast<uint32_t *>(b + a.o_rep);
  x.top = reinterpret_cast<uint64_t *>(b + a.o_top);
  x.minrho = reinterpret_cast<uint32_t *>(b + a.o_minrho);
  x.ent = reinterpret_cast<uint32_t *>(b + a.o_ent);
  x.plist = reinterpret_cast<uint32_t *>(b + a.o_plist);
  return x;
}

// Slot hash of a cell's coordinates (multiply-xorshift rounds).
template <int D>
__device__ __forceinline__ uint32_t cell_hash(const int32_t *c) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    h = (h ^ uint32_t(c[t])) * 0xFF51AFD7ED558CCDull;
    h ^= h >> 29;
  }
  return uint32_t(h ^ (h >> 32));
}

__global__ __launch_bounds__(kBlock) void k_ax_clear(AxWs x, uint32_t slots) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < 4) x.cnt[i] = 0;
  if (i < slots) {
    x.rep[i] = kEmpty;
    x.top[i] = 0;
    x.minrho[i] = kEmpty;
  }
}

// Each point finds (or opens) its cell's slot, then raises the slot's top key
// and lowers its smallest density.  Slots only ever go from free to taken, so a
// stale free slot read is settled by the compare-and-swap, and a taken one is
// final.  The table has more slots than points, so a free slot always exists.
// Consecutive lanes of one cell (cell order keeps a cell's points together)
// combine their keys first, and the last of them updates the slot: one pair of
// atomics per run instead of per point.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ax_insert(Plan p, Ws w, ApproxPlan a, AxWs x) {
  if (grid_skipped(w.hdr)) return;
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool valid = q < p.n;
  uint32_t h = kEmpty;  // (no slot has this index)
  uint64_t K = 0;
  if (valid) {
    int32_t c[D];
#pragma unroll
    for (int t = 0; t < D; ++t) c[t] = w.spts[q * D + t] / a.La;
    h = cell_hash<D>(c) & a.mask;
    for (uint32_t probe = 0; probe <= a.mask; ++probe) {
      uint32_t r = x.rep[h];
      if (r == kEmpty) {
        r = atomicCAS(&x.rep[h], kEmpty, uint32_t(q));
        if (r == kEmpty) break;  // opened by this point
      }
      bool same = true;
#pragma unroll
      for (int t = 0; t < D; ++t) same = same && w.spts[int64_t(r) * D + t] / a.La == c[t];
      if (same) break;
      h = (h + 1) & a.mask;
    }
    K = w.sK[q];
    x.ent[q] = h;
  }
  const WaveRun run = wave_run(h);
  const uint64_t top = run_reduce(K, run.start, [](uint64_t u, uint64_t v) { return u > v ? u : v; });
  const uint32_t low = run_reduce(valid ? uint32_t(K >> 32) : kEmpty, run.start,
                                  [](uint32_t u, uint32_t v) { return u < v ? u : v; });
  if (valid && run.tail) {
    atomicMax(reinterpret_cast<unsigned long long *>(&x.top[h]), static_cast<unsigned long long>(top));
    atomicMin(&x.minrho[h], low);
  }
}

// First rule: a point other than its cell's p* takes p*(c).  The p* points are
// listed for the range search (kSplitPer consecutive positions per thread, one
// atomic per block).
constexpr int kSplitPer = 16;

__global__ __launch_bounds__(kBlock) void k_ax_split(Plan p, Ws w, AxWs x) {
  if (grid_skipped(w.hdr)) return;
  const int64_t q0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) * kSplitPer;
  uint32_t mask = 0;
  for (int k = 0; k < kSplitPer; ++k) {
    const int64_t q = q0 + k;
    if (q >= p.n) break;
    const uint64_t top = x.top[x.ent[q]];
    if (top == w.sK[q]) {
      mask |= 1u << k;
    } else {
      w.best[q] = (kApproxD2 << kIdBits) | (~uint32_t(top) & kIdMask);
      w.flag[q] = 0;
    }
  }
  uint32_t at = block_append(mask, &x.cnt[0]);
  for (int k = 0; k < kSplitPer; ++k)
    if (mask & (1u << k)) x.plist[at++] = uint32_t(q0 + k);
}

// Second rule: a range search of radius d_cut around each p* point over the
// exact grid's rows, keeping the qualifying cell with the smallest coordinates.
// A point no cell qualifies for gets kNoKey and its open flag, which puts it on
// the ring search's list.
template <int D>
__device__ __forceinline__ bool lex_less(const int32_t *a, const int32_t *b) {
  bool less = false, eq = true;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    less = less || (eq && a[t] < b[t]);
    eq = eq && a[t] == b[t];
  }
  return less;
}

// One candidate j of p*'s range search: a point strictly within d_cut, of higher
// density, in another cell whose points all have a higher density, updates the
// best qualifying cell (bc, be) when its cell's coordinates are smaller.
template <int D>
__device__ __forceinline__ void ax_visit(const Plan &p, const Ws &w, const ApproxPlan &a, const AxWs &x,
                                         const int32_t *xq, uint32_t e, uint32_t rho, uint32_t j, int &found,
                                         int32_t *bc, uint32_t &be) {
  if (uint32_t(w.sK[j] >> 32) <= rho) return;  // cheapest test first
  int64_t d2 = 0;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const int64_t df = int64_t(w.spts[int64_t(j) * D + t]) - xq[t];
    d2 += df * df;
  }
  if (d2 >= p.R) return;
  const uint32_t e2 = x.ent[j];
  if (e2 == e || x.minrho[e2] <= rho) return;
  int32_t cc[D];
#pragma unroll
  for (int t = 0; t < D; ++t) cc[t] = w.spts[int64_t(j) * D + t] / a.La;
  if (!found || lex_less<D>(cc, bc)) {
#pragma unroll
    for (int t = 0; t < D; ++t) bc[t] = cc[t];
    be = e2;
    found = 1;
  }
}

__device__ __forceinline__ uint64_t ax_key(const AxWs &x, int found, uint32_t be) {
  return found ? (kApproxD2 << kIdBits) | (~uint32_t(x.top[be]) & kIdMask) : kNoKey;
}

// Dense data (task-form plans): one wave per p* point, each lane keeping its own
// best cell, then a reduction over the wave.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ax_near(Plan p, Ws w, ApproxPlan a, AxWs x) {
  __shared__ NearLds lds_all[kWavesPerBlock];
  NearLds &lds = lds_all[threadIdx.x / kWave];
  if (grid_skipped(w.hdr)) return;
  const Blk blk = grid_blk();
  const uint32_t nstar = uniform(x.cnt[0]);
  const uint32_t nw = grid_waves(blk);
  for (uint32_t u = wave_index(blk); u < nstar; u += nw) {
    const uint32_t q = uniform(x.plist[u]);
    int32_t xq[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xq[t] = uniform(w.spts[int64_t(q) * D + t]);
    const uint32_t e = uniform(x.ent[q]);
    const uint32_t rho = uniform(uint32_t(w.sK[q] >> 32));
    int32_t bc[D];
#pragma unroll
    for (int t = 0; t < D; ++t) bc[t] = 0;
    uint32_t be = 0;
    int found = 0;
    wave_near<D>(p, w, xq, lds, [&](uint32_t j) { ax_visit<D>(p, w, a, x, xq, e, rho, j, found, bc, be); });
    for (int off = kWave / 2; off > 0; off >>= 1) {
      int32_t oc[D];
#pragma unroll
      for (int t = 0; t < D; ++t) oc[t] = __shfl_xor(bc[t], off, kWave);
      const uint32_t oe = __shfl_xor(be, off, kWave);
      const int of = __shfl_xor(found, off, kWave);
      if (of && (!found || lex_less<D>(oc, bc))) {
#pragma unroll
        for (int t = 0; t < D; ++t) bc[t] = oc[t];
        be = oe;
        found = 1;
      }
    }
    if (lane_id() == 0) {  // every lane holds the same winner
      w.best[q] = ax_key(x, found, be);
      w.flag[q] = found ? 0 : 1;  // open for the exact remainder
    }
  }
}

// Sparse data (lane-form plans): one lane per p* point.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ax_near_lanes(Plan p, Ws w, ApproxPlan a, AxWs x) {
  if (grid_skipped(w.hdr)) return;
  const uint32_t u = blockIdx.x * kBlock + threadIdx.x;
  if (u >= x.cnt[0]) return;
  const uint32_t q = x.plist[u];
  int32_t xq[D];
#pragma unroll
  for (int t = 0; t < D; ++t) xq[t] = w.spts[int64_t(q) * D + t];
  const uint32_t e = x.ent[q];
  const uint32_t rho = uint32_t(w.sK[q] >> 32);
  int32_t bc[D];
#pragma unroll
  for (int t = 0; t < D; ++t) bc[t] = 0;
  uint32_t be = 0;
  int found = 0;
  lane_near<D>(p, w, xq, [&](uint32_t j) { ax_visit<D>(p, w, a, x, xq, e, rho, j, found, bc, be); });
  w.best[q] = ax_key(x, found, be);
  w.flag[q] = found ? 0 : 1;  // open for the exact remainder
}

// Outputs in id order: the exact keys as the exact path's finish writes them,
// approximate ones as (p*, d_cut) with the flag set.
__global__ __launch_bounds__(kBlock) void k_ax_finish(Plan p, Ws w, double d_cut, int32_t *__restrict__ dep,
                                                      double *__restrict__ delta, int32_t *__restrict__ rho,
                                                      uint8_t *__restrict__ approx) {
  if (grid_skipped(w.hdr)) return;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t q = w.key[i];
  const uint64_t key = w.best[q];
  bool ax = false;
  if (key == kNoKey) {
    dep[i] = -1;
    delta[i] = __builtin_huge_val();
  } else if ((key >> kIdBits) == kApproxD2) {
    dep[i] = int32_t(key & kIdMask);
    delta[i] = d_cut;
    ax = true;
  } else {
    dep[i] = int32_t(key & kIdMask);
    delta[i] = __builtin_sqrt(double(key >> kIdBits));  // correctly rounded (IEEE sqrt)
  }
  rho[i] = int32_t(w.sK[q] >> 32);
  if (approx) approx[i] = ax ? 1 : 0;
}

template <int D>
hipError_t launch_cells_d(const Plan &p, const Ws &w, const ApproxPlan &a, const AxWs &x, hipStream_t s) {
  DPC_LAUNCH((k_ax_insert<D>), blocks_for(p.n, kBlock), kBlock, s, p, w, a, x);
  DPC_LAUNCH((k_ax_split), blocks_for(p.n, kBlock * kSplitPer), kBlock, s, p, w, x);
  if (p.lanes)
    DPC_LAUNCH((k_ax_near_lanes<D>), blocks_for(p.n, kBlock), kBlock, s, p, w, a, x);
  else
    DPC_LAUNCH((k_ax_near<D>), persistent_blocks(p.n), kBlock, s, p, w, a, x);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_collect(p, w, s);
}

}  // namespace

hipError_t launch_approx(const Plan &p, const Ws &w, const ApproxPlan &a, void *base, int32_t *dep,
                         double *delta, int32_t *rho, uint8_t *approx, hipStream_t s) {
  const AxWs x = ax_resolve(a, base);
  hipError_t e;
  {
    ProfScope ps(s, kProfApprox);
    DPC_LAUNCH((k_ax_clear), blocks_for(int64_t(a.mask) + 1, kBlock), kBlock, s, x, a.mask + 1);
    switch (p.d) {
      case 1: e = launch_cells_d<1>(p, w, a, x, s); break;
      case 2: e = launch_cells_d<2>(p, w, a, x, s); break;
      case 3: e = launch_cells_d<3>(p, w, a, x, s); break;
      case 4: e = launch_cells_d<4>(p, w, a, x, s); break;
      case 5: e = launch_cells_d<5>(p, w, a, x, s); break;
      case 6: e = launch_cells_d<6>(p, w, a, x, s); break;
      case 7: e = launch_cells_d<7>(p, w, a, x, s); break;
      case 8: e = launch_cells_d<8>(p, w, a, x, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  if ((e = launch_exact_remainder(p, w, s)) != hipSuccess) return e;
  ProfScope ps(s, kProfFinish);
  DPC_LAUNCH((k_ax_finish), blocks_for(p.n, kBlock), kBlock, s, p, w, a.d_cut, dep, delta, rho, approx);
  return hipGetLastError();
}

}  // namespace dpc
