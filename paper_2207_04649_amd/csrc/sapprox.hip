// S-Approx-DPC (Section 5): one picked point per cell of a grid G' of side about
// eps * d_cut / sqrt(d) stands for its cell.
//
//   * G' is an open-addressing hash table over the occupied cells (as in
//     Approx-DPC); integer side Le = 1 + floor(sqrt((Re - 1) / d)), Re = ceil(e^2)
//     for the double e = eps * d_cut, so the points of a cell lie strictly within e
//     of each other.  A cell's pick is its smallest id (an atomicMin per run of
//     same-cell lanes).
//   * Local density of the picks (Def. 1, against all points).  The section
//     computes it for the picks only; here the exact path's density kernels run
//     over every point, which on this hardware costs less than a range search
//     per pick, and the picks read theirs.
//   * A point that was not picked takes its cell's pick (true distance, below
//     eps * d_cut) and reports the pick's density.
//   * First phase: a pick takes the nearest higher-ranked pick among the picks of
//     the cells that hold a point strictly within d_cut of it (N(c)).
//   * Second phase: the picks left take their nearest higher-ranked pick through
//     the exact path's ring search and prefix scan.  Their rank keys rank every
//     pick above every other point (a point that was not picked gets density key
//     1, a pick its density plus one when no point has density n, else its
//     density: a point of density n is within d_cut of every point, so then no
//     pick has density 1), so that search only ever returns picks.  The section's
//     temporary clusters prune this same search; its result does not depend on
//     them.
#include "common.h"
#include "near.h"
#include "prof.h"

namespace dpc {
namespace {

constexpr uint32_t kEmpty = 0xffffffffu;

struct SaWs {
  uint32_t *cnt;    // [4] counters: picks, largest density of all points
  uint32_t *rep;    // [slots] cell-order position of the point that opened the slot, kEmpty if free
  uint32_t *pick;   // [slots] smallest id of the cell (its pick), kEmpty before any point
  uint32_t *ppos;   // [slots] cell-order position of the pick
  uint32_t *prho;   // [slots] density of the pick
  uint32_t *ent;    // [n] table slot of each cell-order position
  uint32_t *plist;  // [n] cell-order positions of the picks
};

SaWs sa_resolve(const SApproxPlan &a, void *base) {
  char *b = static_cast<char *>(base);
  SaWs x;
  x.cnt = reinterpret_cast<uint32_t *>(b + a.o_cnt);
  x.rep = reinterpret_cast<uint32_t *>(b + a.o_rep);
  x.pick = reinterpret_cast<uint32_t *>(b + a.o_pick);
  x.ppos = reinterpret_cast<uint32_t *>(b + a.o_ppos);
  x.prho = reinterpret_cast<uint32_t *>(b + a.o_prho);
  x.ent = reinterpret_cast<uint32_t *>(b + a.o_ent);
  x.plist = reinterpret_cast<uint32_t *>(b + a.o_plist);
  return x;
}

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

template <int D>
__device__ __forceinline__ int64_t d2_of(const int32_t *__restrict__ spts, uint32_t a, const int32_t *xq) {
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const int64_t df = int64_t(spts[int64_t(a) * D + t]) - xq[t];
    s += df * df;
  }
  return s;
}

__global__ __launch_bounds__(kBlock) void k_sa_clear(SaWs x, uint32_t slots) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < 4) x.cnt[i] = 0;
  if (i < slots) {
    x.rep[i] = kEmpty;
    x.pick[i] = kEmpty;
  }
}

// Each point finds (or opens) its cell's slot and lowers the slot's pick id;
// consecutive lanes of one cell combine first (one atomic per run).
template <int D>
__global__ __launch_bounds__(kBlock) void k_sa_insert(Plan p, Ws w, SApproxPlan a, SaWs x) {
  if (grid_skipped(w.hdr)) return;
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool valid = q < p.n;
  uint32_t h = kEmpty;  // (no slot has this index)
  uint32_t id = kEmpty;
  if (valid) {
    int32_t c[D];
#pragma unroll
    for (int t = 0; t < D; ++t) c[t] = w.spts[q * D + t] / a.Le;
    h = cell_hash<D>(c) & a.mask;
    for (uint32_t probe = 0; probe <= a.mask; ++probe) {
      uint32_t r = x.rep[h];
      if (r == kEmpty) {
        r = atomicCAS(&x.rep[h], kEmpty, uint32_t(q));
        if (r == kEmpty) break;
      }
      bool same = true;
#pragma unroll
      for (int t = 0; t < D; ++t) same = same && w.spts[int64_t(r) * D + t] / a.Le == c[t];
      if (same) break;
      h = (h + 1) & a.mask;
    }
    x.ent[q] = h;
    id = uint32_t(w.sid[q]);
  }
  const WaveRun run = wave_run(h);
  const uint32_t low = run_reduce(id, run.start, [](uint32_t u, uint32_t v) { return u < v ? u : v; });
  if (valid && run.tail) atomicMin(&x.pick[h], low);
}

// The picks: their positions and densities per slot, and as a list
// (kSplitPer consecutive positions per thread, one atomic per block); the
// largest density of all points (one atomic per block).
constexpr int kSplitPer = 16;

__global__ __launch_bounds__(kBlock) void k_sa_split(Plan p, Ws w, SaWs x) {
  __shared__ uint32_t wave_max[kWavesPerBlock];
  if (grid_skipped(w.hdr)) return;
  const int64_t q0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) * kSplitPer;
  uint32_t mask = 0, top = 0;
  for (int k = 0; k < kSplitPer; ++k) {
    const int64_t q = q0 + k;
    if (q >= p.n) break;
    const uint32_t e = x.ent[q];
    const uint32_t rho = uint32_t(w.sK[q] >> 32);
    top = max(top, rho);
    if (x.pick[e] == uint32_t(w.sid[q])) {
      mask |= 1u << k;
      x.ppos[e] = uint32_t(q);
      x.prho[e] = rho;
    } else {
      w.flag[q] = 0;
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) top = max(top, uint32_t(__shfl_xor(top, off, kWave)));
  if (lane_id() == 0) wave_max[threadIdx.x / kWave] = top;
  uint32_t at = block_append(mask, &x.cnt[0]);  // (synchronises the block)
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) m = max(m, wave_max[k]);
    atomicMax(&x.cnt[1], m);
  }
  for (int k = 0; k < kSplitPer; ++k)
    if (mask & (1u << k)) x.plist[at++] = uint32_t(q0 + k);
}

// Rank keys: every pick above every other point (see the file comment; the
// shift is decided on the largest density of all points: if some point is within
// d_cut of every point, every pick has density >= 2), and the dependent point of
// each point that was not picked: its cell's pick.
__global__ __launch_bounds__(kBlock) void k_sa_keys(Plan p, Ws w, SaWs x) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= p.n || grid_skipped(w.hdr)) return;
  const uint32_t e = x.ent[q];
  const uint32_t id = uint32_t(w.sid[q]);
  const uint32_t shift = uint64_t(x.cnt[1]) < uint64_t(p.n) ? 1u : 0u;
  const uint32_t pp = x.ppos[e];
  const bool star = pp == uint32_t(q);
  const uint64_t r = star ? uint64_t(x.prho[e]) + shift : 1u;
  const uint64_t key = (r << 32) | uint32_t(~id);
  w.sK[q] = key;
  if (w.srec) {  // the ring search's packed records carry the rank key
    const uint32_t a0 = w.spk[q * p.words], a1 = p.words == 2 ? w.spk[q * p.words + 1] : 0u;
    w.srec[q] = make_uint4(a0, a1, uint32_t(key), uint32_t(key >> 32));
  }
  if (!star) {
    int64_t s = 0;
    for (int t = 0; t < p.d; ++t) {
      const int64_t df = int64_t(w.spts[q * p.d + t]) - w.spts[int64_t(pp) * p.d + t];
      s += df * df;
    }
    w.best[q] = (uint64_t(s) << kIdBits) | x.pick[e];
  }
}

// First phase: the nearest higher-ranked pick of the cells that hold a point
// strictly within d_cut; picks without one keep no key and their open flag, which
// puts them on the ring search's list.  One candidate j:
template <int D>
__device__ __forceinline__ void sa_visit_d(const Plan &p, const Ws &w, const SaWs &x, const int32_t *xq,
                                           uint32_t e, uint32_t rho, uint32_t id, uint32_t j, uint32_t &last_e,
                                           uint64_t &best) {
  const uint32_t e2 = x.ent[j];
  if (e2 == e || e2 == last_e) return;  // consecutive positions often share a cell
  if (d2_of<D>(w.spts, j, xq) >= p.R) return;
  last_e = e2;
  const uint32_t r2 = x.prho[e2], id2 = x.pick[e2];
  if (!(r2 > rho || (r2 == rho && id2 < id))) return;
  const uint64_t key = (uint64_t(d2_of<D>(w.spts, x.ppos[e2], xq)) << kIdBits) | id2;
  best = key < best ? key : best;
}

// Dense data (task-form plans): one wave per pick, then the wave's minimum.
template <int D>
__global__ __launch_bounds__(kBlock) void k_sa_phase1(Plan p, Ws w, SaWs x) {
  __shared__ NearLds lds_all[kWavesPerBlock];
  NearLds &lds = lds_all[threadIdx.x / kWave];
  if (grid_skipped(w.hdr)) return;
  const Blk blk = grid_blk();
  const uint32_t npick = uniform(x.cnt[0]);
  const uint32_t nw = grid_waves(blk);
  for (uint32_t u = wave_index(blk); u < npick; u += nw) {
    const uint32_t q = uniform(x.plist[u]);
    int32_t xq[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xq[t] = uniform(w.spts[int64_t(q) * D + t]);
    const uint32_t e = uniform(x.ent[q]);
    const uint32_t rho = uniform(x.prho[e]), id = uniform(uint32_t(w.sid[q]));
    uint64_t best = kNoKey;
    uint32_t last_e = e;
    wave_near<D>(p, w, xq, lds, [&](uint32_t j) { sa_visit_d<D>(p, w, x, xq, e, rho, id, j, last_e, best); });
    best = wave_min_u64(best);
    if (lane_id() == 0) {
      w.best[q] = best;
      w.flag[q] = best == kNoKey ? 1 : 0;  // open for the second phase
    }
  }
}

// Sparse data (lane-form plans): one lane per pick.
template <int D>
__global__ __launch_bounds__(kBlock) void k_sa_phase1_lanes(Plan p, Ws w, SaWs x) {
  if (grid_skipped(w.hdr)) return;
  const uint32_t u = blockIdx.x * kBlock + threadIdx.x;
  if (u >= x.cnt[0]) return;
  const uint32_t q = x.plist[u];
  int32_t xq[D];
#pragma unroll
  for (int t = 0; t < D; ++t) xq[t] = w.spts[int64_t(q) * D + t];
  const uint32_t e = x.ent[q];
  const uint32_t rho = x.prho[e], id = uint32_t(w.sid[q]);
  uint64_t best = kNoKey;
  uint32_t last_e = e;
  lane_near<D>(p, w, xq, [&](uint32_t j) { sa_visit_d<D>(p, w, x, xq, e, rho, id, j, last_e, best); });
  w.best[q] = best;
  w.flag[q] = best == kNoKey ? 1 : 0;  // open for the second phase
}

// Outputs in id order: dep and the true distance from the key, the pick's density,
// the picked flag.
__global__ __launch_bounds__(kBlock) void k_sa_finish(Plan p, Ws w, SaWs x, int32_t *__restrict__ dep,
                                                      double *__restrict__ delta, int32_t *__restrict__ rho,
                                                      uint8_t *__restrict__ picked) {
  if (grid_skipped(w.hdr)) return;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t q = w.key[i];
  const uint64_t key = w.best[q];
  if (key == kNoKey) {
    dep[i] = -1;
    delta[i] = __builtin_huge_val();
  } else {
    dep[i] = int32_t(key & kIdMask);
    delta[i] = __builtin_sqrt(double(key >> kIdBits));  // correctly rounded (IEEE sqrt)
  }
  const uint32_t e = x.ent[q];
  rho[i] = int32_t(x.prho[e]);
  if (picked) picked[i] = x.ppos[e] == q ? 1 : 0;
}

template <int D>
void launch_sa_d(const Plan &p, const Ws &w, const SApproxPlan &a, const SaWs &x, hipStream_t s) {
  DPC_LAUNCH((k_sa_insert<D>), blocks_for(p.n, kBlock), kBlock, s, p, w, a, x);
  DPC_LAUNCH((k_sa_split), blocks_for(p.n, kBlock * kSplitPer), kBlock, s, p, w, x);
  DPC_LAUNCH((k_sa_keys), blocks_for(p.n, kBlock), kBlock, s, p, w, x);
  if (p.lanes)
    DPC_LAUNCH((k_sa_phase1_lanes<D>), blocks_for(p.n, kBlock), kBlock, s, p, w, x);
  else
    DPC_LAUNCH((k_sa_phase1<D>), persistent_blocks(p.n), kBlock, s, p, w, x);
}

}  // namespace

hipError_t launch_sapprox(const Plan &p, const Ws &w, const SApproxPlan &a, void *base, int32_t *dep,
                          double *delta, int32_t *rho, uint8_t *picked, hipStream_t s) {
  const SaWs x = sa_resolve(a, base);
  hipError_t e;
  {
    ProfScope ps(s, kProfApprox);
    DPC_LAUNCH((k_sa_clear), blocks_for(int64_t(a.mask) + 1, kBlock), kBlock, s, x, a.mask + 1);
    switch (p.d) {
      case 1: launch_sa_d<1>(p, w, a, x, s); break;
      case 2: launch_sa_d<2>(p, w, a, x, s); break;
      case 3: launch_sa_d<3>(p, w, a, x, s); break;
      case 4: launch_sa_d<4>(p, w, a, x, s); break;
      case 5: launch_sa_d<5>(p, w, a, x, s); break;
      case 6: launch_sa_d<6>(p, w, a, x, s); break;
      case 7: launch_sa_d<7>(p, w, a, x, s); break;
      case 8: launch_sa_d<8>(p, w, a, x, s); break;
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_collect(p, w, s)) != hipSuccess) return e;
  }
  {
    ProfScope ps(s, kProfRankSort);
    if ((e = rank_sort(p, w, s)) != hipSuccess) return e;
  }
  if ((e = launch_exact_remainder(p, w, s)) != hipSuccess) return e;
  ProfScope ps(s, kProfFinish);
  DPC_LAUNCH((k_sa_finish), blocks_for(p.n, kBlock), kBlock, s, p, w, x, dep, delta, rho, picked);
  return hipGetLastError();
}

}  // namespace dpc
