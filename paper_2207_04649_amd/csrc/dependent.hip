// Dependent point and dependent distance (Defs. 2-3).
//
// q_i is the point with the smallest (D2, id) among the points ranked above i in
// the order (rho descending, id ascending); delta_i = sqrt(D2).  Ex-DPC finds it
// with a kd-tree grown in density order (Section 3); here it takes exact passes,
// all keyed by the packed u64 (D2 << 27 | id), whose minimum is unique, so every
// reduction order gives the same answer:
//
//  1. search stages: windows of radius K = 1 and 3 cells (by default) around
//     groups of up to 64 open points of one strip.  A point whose best candidate
//     is strictly closer than its window's exterior is final.  Most points end
//     in the first stage, since most dependent distances are far below d_cut
//     (the paper makes the same observation, Section 3, after Lemma 2); later
//     stages gather the open points of several tasks into full waves and clip
//     their windows to the largest best distance found so far;
//  2. ring search: one wave per still-open point grows the searched cell block
//     by annuli, until the best is strictly closer than the block's exterior or
//     the work would exceed a scan of the point's density prefix;
//  3. peaks: a scan of the density prefix (the points of higher rank, contiguous
//     in the rank-sorted copy, as in the straightforward algorithm of Section 2.2,
//     step 3), 64 points per wave, split over waves in chunks and merged with a
//     64-bit atomic minimum.
#include "prof.h"
#include "tasks.h"

namespace dpc {
namespace {

// -------------------------------------------------------------------- search stages

// One window search for up to 64 open points of one strip (lane = point; lanes
// with valid = false repeat a valid lane's point and store the same values).
//
// K >= 1: the window of radius K cells; a point is final when its best is
// strictly closer than the window's exterior.  K == 0 (ball stage): the density
// window (radius K0, clipped to the d_cut-balls), which holds every point closer
// than d_cut to each query; a point is final when its best is inside its ball.
template <int D, int MODE>
__device__ __forceinline__ void search_batch(const Plan &p, const Ws &w, int Kin, bool first, uint32_t strip,
                                             uint32_t q, bool valid, uint64_t *work) {
  const bool ball = Kin == 0;
  const int K = ball ? p.K0 : Kin;
  constexpr int W = (D + 1) / 2;
  const int lane = lane_id();
  DPC_CONST(uint32_t) *spk = as_const(w.spk);
  DPC_CONST(int32_t) *spc = as_const(w.spts);
  DPC_CONST(uint64_t) *sKc = as_const(w.sK);
  DPC_CONST(int32_t) *sidc = as_const(w.sid);
  TaskGeom<D> g;
  strip_row<D>(p, strip, g);
  int32_t qx[D];
#pragma unroll
  for (int k = 0; k < D; ++k) qx[k] = w.spts[int64_t(q) * D + k];
  task_span<D>(p, g, w.spts[int64_t(q) * D + (p.gm - 1)], valid);  // strip-dimension coordinate
  const uint64_t Ki = w.sK[q];
  uint64_t best = first ? kNoKey : w.best[q];
  // Clip the window to the largest best distance when every point has one.
  const bool all_have = __ballot(valid && best == kNoKey) == 0;
  uint64_t clip2 = ball ? uint64_t(p.R - 1) : ~uint64_t(0);
  if (all_have) {
    const uint64_t c = uniform(wave_max_u64(valid ? (best >> kIdBits) : uint64_t(0)));
    clip2 = c < clip2 ? c : clip2;
  }
  uint32_t qk[W];
  if (MODE == kModeP16) {
#pragma unroll
    for (int k = 0; k < W; ++k) qk[k] = w.spk[int64_t(q) * W + k];
    // inner-loop key: (D2 << 32) | id, D2 < 2^31 on this path
    if (best != kNoKey) best = ((best >> kIdBits) << 32) | (best & kIdMask);
  }
  const int nrow = int(window_rows(p, K));
  const uint32_t nvalid = uint32_t(__popcll(__ballot(valid)));
  for (int rb = 0; rb < nrow; rb += kWave) {
    uint32_t sb = 0, se = 0;
    if (rb + lane < nrow) window_row<D>(p, g, K, rb + lane, clip2, w.cnt, &sb, &se);
    const int nr = min(kWave, nrow - rb);
    for (int r = 0; r < nr; ++r) {
      const uint32_t b = __builtin_amdgcn_readlane(sb, r);
      const uint32_t e = __builtin_amdgcn_readlane(se, r);
      *work += uint64_t(e - b) * nvalid;
      uint32_t j = b;
      if (MODE == kModeP16) {
        constexpr int B = 8 / W > 0 ? 8 / W : 1;
        for (; j + B <= e; j += B) {
          // one scalar load per array for B candidates (uniform base, constant offsets)
          DPC_CONST(uint32_t) *cb = spk + int64_t(j) * W;
          DPC_CONST(uint64_t) *kb = sKc + j;
          DPC_CONST(int32_t) *ib = sidc + j;
          uint32_t c[B * W], idj[B];
          uint64_t kj[B];
#pragma unroll
          for (int u = 0; u < B * W; ++u) c[u] = cb[u];
#pragma unroll
          for (int u = 0; u < B; ++u) {
            kj[u] = kb[u];
            idj[u] = uint32_t(ib[u]);
          }
#pragma unroll
          for (int u = 0; u < B; ++u) {
            int32_t d2 = dot2_self_s(pk_sub16(qk[0], c[u * W]), 0);
#pragma unroll
            for (int k = 1; k < W; ++k) d2 = dot2_self_v(pk_sub16(qk[k], c[u * W + k]), d2);
            const uint64_t key = (uint64_t(uint32_t(d2)) << 32) | idj[u];
            best = (kj[u] > Ki && key < best) ? key : best;
          }
        }
        for (; j < e; ++j) {
          const uint64_t kj = sKc[j];
          int32_t d2 = dot2_self_s(pk_sub16(qk[0], spk[int64_t(j) * W]), 0);
#pragma unroll
          for (int k = 1; k < W; ++k) d2 = dot2_self_v(pk_sub16(qk[k], spk[int64_t(j) * W + k]), d2);
          const uint64_t key = (uint64_t(uint32_t(d2)) << 32) | uint32_t(sidc[j]);
          best = (kj > Ki && key < best) ? key : best;
        }
      } else {
        for (; j < e; ++j) {
          const uint64_t kj = sKc[j];
          int64_t d2 = 0;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const int64_t df = int64_t(qx[k] - spc[int64_t(j) * D + k]);
            d2 += df * df;
          }
          const uint64_t key = (uint64_t(d2) << kIdBits) | uint32_t(sidc[j]);
          best = (kj > Ki && key < best) ? key : best;
        }
      }
    }
  }
  if (MODE == kModeP16 && best != kNoKey) best = ((best >> 32) << kIdBits) | (best & 0xFFFFFFFFu);
  const uint64_t ext = window_exterior_d2<D>(p, g, K, qx);
  const uint64_t bound = ball ? uint64_t(p.R) : ext;  // every point closer than this was searched
  const bool resolved = ext == kNoKey || (best != kNoKey && (best >> kIdBits) < bound);
  w.best[q] = best;
  w.flag[q] = resolved ? 0 : 1;
}

// ------------------------------------------------------------ lane form
//
// One query per lane, each with its own window around its cell, for the point
// ranked above it with the smallest (D2, id).  Rows and cells are clipped to the
// best distance found so far (a cell whose nearest point is farther cannot hold
// a better candidate), the lane's own row first.  Two kinds of stage:
//  * a block of K >= 1 cells: the best is final when strictly closer than the
//    block's exterior; the ring search then grows the block from K;
//  * the ball (K = 0): the density window, clipped to the d_cut-ball as well;
//    the best is final when D2 <= R - 1, since every point that close was seen
//    (most dependent points lie within d_cut, the observation the paper makes
//    after Lemma 2); the ring search then starts from nothing.
template <int D, int MODE>
__device__ __forceinline__ void search_lanes(Blk blk, const Plan &p, const Ws &w, int Kin) {
  constexpr int W = (D + 1) / 2;
  if (grid_skipped(w.hdr)) return;
  const bool ball = Kin == 0;
  const int K = ball ? p.K0 : Kin;
  const int shift = MODE == kModeP16 ? 32 : kIdBits;
  // the ball's bound, or no bound (a block is clipped by the best alone)
  const int64_t C = ball ? p.R - 1 : INT64_MAX;
  const int nrow = int(window_rows(p, K));
  const uint4 *srec = w.srec;
  __shared__ uint2 queue_all[kWalkQueue * kBlock];  // each lane's queue of row ranges
  uint2 *queue = queue_all + threadIdx.x;
  uint64_t work = 0;  // the lane's candidate tests (profiling)
  for (int64_t q = thread_index(blk); q < p.n; q += grid_threads(blk)) {
    LaneGeom<D> geo;
    lane_geom<D>(p, w.spts + q * D, geo);
    const uint64_t Ki = w.sK[q];
    uint32_t qk[W];
    if (MODE == kModeP16) {
#pragma unroll
      for (int k = 0; k < W; ++k) qk[k] = w.spk[q * W + k];
    }
    // p16: key (D2 << 32) | id while searching; i64: (D2 << 27) | id throughout
    uint64_t best = kNoKey;
    // one candidate: the rank test and the (D2, id) minimum
    auto consider = [&](uint32_t j, bool take) {
      uint64_t kj, key;
      uint32_t cw[W];
      if (MODE == kModeP16 && W <= 2 && srec) {  // words and rank key in one load
        const uint4 rec = srec[j];
        cw[0] = rec.x;
        cw[W - 1] = W == 2 ? rec.y : rec.x;
        kj = (uint64_t(rec.w) << 32) | rec.z;
      } else {
        kj = w.sK[j];
        if (MODE == kModeP16) load_words<W>(w.spk + int64_t(j) * W, cw);
      }
      if (MODE == kModeP16) {
        int32_t d2 = dot2_self_v(pk_sub16(qk[0], cw[0]), 0);
#pragma unroll
        for (int k = 1; k < W; ++k) d2 = dot2_self_v(pk_sub16(qk[k], cw[k]), d2);
        key = (uint64_t(uint32_t(d2)) << 32) | uint32_t(~uint32_t(kj));
      } else {
        int64_t d2 = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const int64_t df = int64_t(geo.x[k] - w.spts[int64_t(j) * D + k]);
          d2 += df * df;
        }
        key = (uint64_t(d2) << kIdBits) | uint32_t(~uint32_t(kj));
      }
      best = (take && kj > Ki && key < best) ? key : best;
    };
    bool done = false;
    if constexpr (D <= 4) {
      if (K == 1 && p.gm == D) {  // compile-time rows
        if (MODE == kModeP16) {  // squared gaps of a packed-path window stay below 2^31
          auto clip = [&]() {
            return uint32_t(best == kNoKey ? (ball ? uint64_t(C) : uint64_t(UINT32_MAX)) : min(uint64_t(C), best >> 32));
          };
          work += walk_k1<D, uint32_t, false>(p, geo, w.cnt, queue, clip, consider);
        } else {
          auto clip = [&]() { return best == kNoKey ? C : min(C, int64_t(best >> kIdBits)); };
          work += walk_k1<D, int64_t, false>(p, geo, w.cnt, queue, clip, consider);
        }
        done = true;
      }
    }
    if (!done) {
      RowWalk<D> rw(K, true);
      for (int r0 = 0; r0 < nrow; r0 += kLaneRowChunk) {
        // cell ranges of the chunk's rows first (independent loads), then their candidates
        const int64_t clip = best == kNoKey ? C : min(C, int64_t(best >> shift));
        uint32_t bb[kLaneRowChunk], ee[kLaneRowChunk];
#pragma unroll
        for (int c = 0; c < kLaneRowChunk; ++c) {
          bb[c] = ee[c] = 0;
          if (r0 + c < nrow) lane_row<D>(p, geo, rw, K, clip, w.cnt, &bb[c], &ee[c]);
          rw.next(p, K);
        }
#pragma unroll
        for (int c = 0; c < kLaneRowChunk; ++c) {
          work += ee[c] - bb[c];
          for (uint32_t j = bb[c]; j < ee[c]; ++j) consider(j, true);
        }
      }
    }
    if (MODE == kModeP16 && best != kNoKey) best = ((best >> 32) << kIdBits) | (best & 0xFFFFFFFFu);
    bool resolved;
    if (ball) {
      resolved = best != kNoKey && int64_t(best >> kIdBits) <= C;
    } else {
      const uint64_t ext = lane_exterior_d2<D>(p, geo, K);
      resolved = ext == kNoKey || (best != kNoKey && (best >> kIdBits) < ext);
    }
    w.best[q] = best;
    w.flag[q] = resolved ? 0 : 1;
  }
  if (p.count_work) add_work(w.hdr, kWorkSearch, work);
}

// Second window stage in lane form, over the points the first stage left open
// (the list of k_collect): kOpenLanes lanes per open point, which split the rows
// of the cells within K of its cell (outside the block within kprev that the
// first stage searched) and then take the minimum of their bests.  Rows and
// strip-dimension cells are clipped to the lane's best distance so far (float
// bounds rounded outwards, so a clip only ever keeps extra cells).  The
// candidate ranges of kOpenChunk rows are queued in LDS and tested as one
// stream, two at a time.  A point stays open, listed for the ring search,
// unless its best is strictly closer than the exterior of the block.
constexpr int kOpenLanes = 4;                // lanes per open point (a power of two)
constexpr int kOpenChunk = 5;                // rows per queue fill
constexpr int kOpenQueue = 2 * kOpenChunk;   // two pieces per row at most
#ifndef DPC_OPEN_CAP
#define DPC_OPEN_CAP 256
#endif
constexpr uint32_t kOpenCap = DPC_OPEN_CAP;  // candidates per lane before the point goes to the ring search
constexpr uint32_t kRingFromFirst = 1u << 31;  // ring-list flag: start from the first stage's block

template <int D, int MODE>
__device__ __forceinline__ void search_open(Blk blk, const Plan &p, const Ws &w, int K, int kprev) {
  constexpr int W = (D + 1) / 2;
  constexpr int RA = D > 1 ? D - 1 : 1;
  if (grid_skipped(w.hdr)) return;
  __shared__ uint2 queue_all[kOpenQueue * kBlock];  // each lane's queue of candidate ranges
  uint2 *queue = queue_all + threadIdx.x;
  const uint32_t nopen = uniform(as_const(&w.hdr->n_unres)[0]);
  const int nr = p.gm - 1;
  const int32_t L = p.L, nc = p.nc;
  const int side = 2 * K + 1;
  const int nrow = int(window_rows(p, K));
  const int nchunk = (nrow + kOpenChunk - 1) / kOpenChunk;
  const float inv_l = 1.0f / float(L), inv_side = 1.0f / float(side);
  const uint4 *srec = w.srec;
  const int sub = int(threadIdx.x) & (kOpenLanes - 1);
  uint64_t work = 0;  // the lane's candidate tests (profiling)
  // Every lane of a point's group runs the same iterations (the shuffles below).
  const int64_t ngroups = grid_threads(blk) / kOpenLanes;
  for (int64_t i = thread_index(blk) / kOpenLanes; i < int64_t(nopen); i += ngroups) {
    const uint32_t q = w.unres[i];
    LaneGeom<D> geo;
    lane_geom<D>(p, w.spts + int64_t(q) * D, geo);
    const uint64_t Ki = w.sK[q];
    uint32_t qk[W];
    if (MODE == kModeP16) {
#pragma unroll
      for (int k = 0; k < W; ++k) qk[k] = w.spk[int64_t(q) * W + k];
    }
    uint64_t best = w.best[q];  // (D2 << kIdBits) | id, kNoKey if none
    // candidate j's key, or kNoKey when it does not rank above the point
    auto key_of = [&](uint32_t j) -> uint64_t {
      uint64_t kj, d2;
      if constexpr (MODE == kModeP16) {
        uint32_t cw[W];
        if (W <= 2 && srec) {  // words and rank key in one load
          const uint4 rec = srec[j];
          cw[0] = rec.x;
          cw[W - 1] = W == 2 ? rec.y : rec.x;
          kj = (uint64_t(rec.w) << 32) | rec.z;
        } else {
          kj = w.sK[j];
          load_words<W>(w.spk + int64_t(j) * W, cw);
        }
        int32_t a = dot2_self_v(pk_sub16(qk[0], cw[0]), 0);
#pragma unroll
        for (int k = 1; k < W; ++k) a = dot2_self_v(pk_sub16(qk[k], cw[k]), a);
        d2 = uint32_t(a);
      } else {
        kj = w.sK[j];
        int32_t y[D];
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = w.spts[int64_t(j) * D + k];
        d2 = exact_d2_u<D>(geo.x, y);
      }
      return kj > Ki ? (d2 << kIdBits) | uint32_t(~uint32_t(kj)) : kNoKey;
    };
    const int32_t xs = geo.xs, cs = geo.cs;
    // the queued ranges' candidates, two per step (the next queued range is read
    // one refill ahead)
    uint32_t spent = 0;  // the lane's candidates so far
    bool over = false;   // the lane gave up: past kOpenCap candidates
    auto stream = [&](const uint32_t *pb, const uint32_t *pe) {
      uint32_t m = 0, total = 0;
#pragma unroll
      for (int k = 0; k < kOpenQueue; ++k) {
        if (pb[k] < pe[k]) {
          queue[m * kBlock] = make_uint2(pb[k], pe[k]);
          ++m;
          total += pe[k] - pb[k];
        }
      }
      // A dense neighbourhood would hold the whole wave back: the point goes to
      // the ring search (a wave per point) instead.
      over = over || spent + total > kOpenCap;
      if (over) return;
      spent += total;
      // two candidates per step; the next queued range is read one refill ahead
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
        const uint64_t k0 = key_of(j0), k1 = key_of(j1);
        best = k0 < best ? k0 : best;
        best = (two && k1 < best) ? k1 : best;
      }
      work += total;
    };
    if (side <= kOpenChunk && nr >= 1) {
      // A chunk is one line of the window: the rows of every value of the first
      // row digit, whose gaps, cells and flags are set once per point; the other
      // digits' share is set once per line.  A strip-dimension cell is kept when
      // its gap and the row's, squared and summed, can be within the best (float
      // bounds rounded outwards); no square root.
      constexpr int kHalf = kOpenChunk / 2;
      float g0[kOpenChunk], gl[kHalf + 1], gr[kHalf + 1];
      int32_t nb0s[kOpenChunk];
      bool ok0[kOpenChunk], in0[kOpenChunk], okl[kHalf + 1], okr[kHalf + 1];
      int32_t stride0 = 1;
      for (int t = 1; t < nr; ++t) stride0 *= nc;
#pragma unroll
      for (int c = 0; c < kOpenChunk; ++c) {
        const int32_t o = c - K;
        const int32_t nb = geo.c[0] + o;
        ok0[c] = c < side && nb >= 0 && nb < nc;
        in0[c] = o <= kprev && o >= -kprev;
        const float a0 = float(cell_gap32(geo.x[0], nb, L));
        g0[c] = a0 * a0;
        nb0s[c] = nb * stride0;
      }
      // strip cells cs - u and cs + u (u <= K), squared gaps lowered a little
#pragma unroll
      for (int u = 1; u <= kHalf; ++u) {
        okl[u] = u <= K && cs - u >= 0;
        okr[u] = u <= K && cs + u < nc;
        const float al = float(cell_gap32(xs, cs - u, L)), ar = float(cell_gap32(xs, cs + u, L));
        gl[u] = al * al * (1.0f - 0x1p-20f);
        gr[u] = ar * ar * (1.0f - 0x1p-20f);
      }
      const int nlines = nrow / side;
      for (int ln = sub; ln < nlines; ln += kOpenLanes) {
        float part = 0.0f;
        int32_t rk = 0;
        bool ok12 = true, in12 = kprev >= 0;
        {
          int32_t r = ln;  // the other digits, the second fastest first
#pragma unroll
          for (int t = 1; t < RA; ++t) {
            if (t < nr) {
              const int32_t qd = int32_t((float(r) + 0.5f) * inv_side);  // exact: r < 2^20
              const int32_t o = r - qd * side - K;
              r = qd;
              const int32_t nb = geo.c[t] + o;
              ok12 = ok12 && nb >= 0 && nb < nc;
              in12 = in12 && o <= kprev && o >= -kprev;
              rk = rk * nc + nb;
              const float gp = float(cell_gap32(geo.x[t], nb, L));
              part = __builtin_fmaf(gp, gp, part);
            }
          }
        }
        const bool clip = best != kNoKey;
        const float bf = clip ? float(best >> kIdBits) * (1.0f + 0x1p-20f) + 1.0f : 0.0f;
        uint32_t pb[kOpenQueue], pe[kOpenQueue];
#pragma unroll
        for (int c = 0; c < kOpenChunk; ++c) {
          pb[2 * c] = pe[2 * c] = pb[2 * c + 1] = pe[2 * c + 1] = 0;
          const float mdf = (part + g0[c]) * (1.0f - 0x1p-20f);
          if (ok12 && ok0[c] && (!clip || mdf <= bf)) {
            // strip cells cs + lo .. cs + hi: the gaps grow away from cs
            int32_t lo = 0, hi = 0;
#pragma unroll
            for (int u = 1; u <= kHalf; ++u) {
              if (okl[u] && (!clip || gl[u] + mdf <= bf)) lo = -u;
              if (okr[u] && (!clip || gr[u] + mdf <= bf)) hi = u;
            }
            const int32_t base = nb0s[c] + rk;  // row index
            const int32_t row0 = base * nc + cs;
            if (ok12 && in12 && in0[c]) {  // two pieces: left and right of the first block
              if (lo <= -kprev - 1) {
                pb[2 * c] = w.cnt[row0 + lo];
                pe[2 * c] = w.cnt[row0 - kprev];
              }
              if (hi >= kprev + 1) {
                pb[2 * c + 1] = w.cnt[row0 + kprev + 1];
                pe[2 * c + 1] = w.cnt[row0 + hi + 1];
              }
            } else {
              pb[2 * c] = w.cnt[row0 + lo];
              pe[2 * c] = w.cnt[row0 + hi + 1];
            }
          }
        }
        stream(pb, pe);
      }
    } else {
      for (int ch = sub; ch < nchunk; ch += kOpenLanes) {
        // digits of the chunk's first row (each in [0, 2K], the first fastest)
        // (r / side in float: exact, as r < 2^20 keeps the rounding far below the
        // 1 / (2 side) that (r + 1/2) / side keeps from an integer)
        int32_t dg[RA];
        {
          int32_t r = ch * kOpenChunk;
#pragma unroll
          for (int t = 0; t < RA; ++t) {
            dg[t] = 0;
            if (t < nr) {
              const int32_t qd = int32_t((float(r) + 0.5f) * inv_side);
              dg[t] = r - qd * side;
              r = qd;
            }
          }
        }
        const uint64_t bestd2 = best >> kIdBits;
        const bool clip = best != kNoKey;
        const float bf = clip ? float(bestd2) * (1.0f + 0x1p-20f) + 1.0f : 0.0f;
        uint32_t pb[kOpenQueue], pe[kOpenQueue];
#pragma unroll
        for (int c = 0; c < kOpenChunk; ++c) {
          pb[2 * c] = pe[2 * c] = pb[2 * c + 1] = pe[2 * c + 1] = 0;
          if (ch * kOpenChunk + c < nrow) {
            int32_t rowk = 0;
            float mdf = 0.0f;
            bool ok = true, inner = kprev >= 0;
#pragma unroll
            for (int t = 0; t < RA; ++t) {
              if (t < nr) {
                const int32_t o = dg[t] - K;
                const int32_t nb = geo.c[t] + o;
                ok = ok && nb >= 0 && nb < nc;
                inner = inner && o <= kprev && o >= -kprev;
                rowk = rowk * nc + nb;
                const float gp = float(cell_gap32(geo.x[t], nb, L));
                mdf = __builtin_fmaf(gp, gp, mdf);
              }
            }
            mdf *= 1.0f - 0x1p-20f;
            if (ok && (!clip || mdf <= bf)) {
              int32_t lo = max(cs - K, 0), hi = min(cs + K, nc - 1);
              if (clip) {
                const float rr = sqrt_approx(bf - mdf) * (1.0f + 0x1p-20f) + 1.0f;
                const float xa = float(xs) - rr, xz = float(xs) + rr;
                if (xa > 0.0f) lo = max(lo, int32_t(xa * inv_l * (1.0f - 0x1p-20f)));
                if (xz < float(DPC_COORD_LIMIT)) hi = min(hi, int32_t(xz * inv_l * (1.0f + 0x1p-20f)));
              }
              const int32_t base = rowk * nc;
              const int32_t l_hi = inner ? min(hi, cs - kprev - 1) : hi;
              const int32_t r_lo = inner ? max(lo, cs + kprev + 1) : hi + 1;
              if (lo <= l_hi) {
                pb[2 * c] = w.cnt[base + lo];
                pe[2 * c] = w.cnt[base + l_hi + 1];
              }
              if (r_lo <= hi) {
                pb[2 * c + 1] = w.cnt[base + r_lo];
                pe[2 * c + 1] = w.cnt[base + hi + 1];
              }
            }
          }
          bool carry = true;  // the next row
#pragma unroll
          for (int t = 0; t < RA; ++t) {
            if (t < nr && carry) {
              carry = dg[t] == 2 * K;
              dg[t] = carry ? 0 : dg[t] + 1;
            }
          }
        }
        stream(pb, pe);
      }
    }
    // the group's best, and whether a lane gave up
    uint32_t gave_up = over ? 1u : 0u;
#pragma unroll
    for (int off = 1; off < kOpenLanes; off <<= 1) {
      const uint64_t o = __shfl_xor(best, off, kWave);
      best = o < best ? o : best;
      gave_up |= uint32_t(__shfl_xor(int(gave_up), off, kWave));
    }
    if (sub == 0) {
      // A point whose block was not searched whole keeps its best (a bound from
      // real candidates) and is listed with kRingFromFirst: the ring search then
      // grows from the first stage's block.
      const uint64_t ext = lane_exterior_d2<D>(p, geo, K);
      const bool resolved = !gave_up && (ext == kNoKey || (best != kNoKey && (best >> kIdBits) < ext));
      w.best[q] = best;
      if (!resolved) w.slot[wave_append(&w.hdr->n_ring, true)] = q | (gave_up ? kRingFromFirst : 0u);
    }
  }
  if (p.count_work) add_work(w.hdr, kWorkSearch, work);
}

// One search stage.  Each wave takes `group` consecutive tasks, gathers their
// open points (all points in the first stage) into batches of 64 per strip
// through an LDS queue, and searches each batch's window of radius K.
template <int D, int MODE>
__device__ __forceinline__ void search_body(Blk blk, const Plan &p, const Ws &w, int K, int group, int first) {
  if (grid_skipped(w.hdr)) return;
  __shared__ uint32_t queue_all[kWavesPerBlock][2 * kWave + 1];  // + a spare slot
  uint32_t *queue = queue_all[threadIdx.x / kWave];
  const int lane = lane_id();
  DPC_CONST(uint32_t) *tc = as_const(reinterpret_cast<const uint32_t *>(w.tasks));
  const uint32_t ntasks = uniform(as_const(&w.hdr->ntasks)[0]);
  const uint32_t ngroups = (ntasks + uint32_t(group) - 1) / uint32_t(group);
  const uint64_t below = (uint64_t(1) << lane) - 1;
  uint64_t work = 0;  // candidate tests of valid queries (wave-uniform; profiling)

  const uint32_t nw = grid_waves(blk);
  for (uint32_t gi = wave_index(blk); gi < ngroups; gi += nw) {
    uint32_t pending = 0, cur = 0;
    const uint32_t t_end = min((gi + 1) * uint32_t(group), ntasks);
    for (uint32_t t = gi * uint32_t(group); t < t_end; ++t) {
      const uint32_t qb = uniform(uint32_t(tc[4 * int64_t(t)]));
      const uint32_t qe = uniform(uint32_t(tc[4 * int64_t(t) + 1]));
      const uint32_t strip = uniform(uint32_t(tc[4 * int64_t(t) + 2]));
      if (pending != 0 && strip != cur) {  // a batch never spans two strips
        const uint32_t qv = queue[min(uint32_t(lane), pending - 1)];
        search_batch<D, MODE>(p, w, K, first != 0, cur, qv, uint32_t(lane) < pending, &work);
        pending = 0;
      }
      cur = strip;
      const uint32_t q = qb + uint32_t(lane);
      const bool take = q < qe && (first != 0 || w.flag[min(q, qe - 1)] != 0);
      const uint64_t m = __ballot(take);
      queue[take ? pending + uint32_t(__popcll(m & below)) : uint32_t(2 * kWave)] = q;
      pending += uint32_t(__popcll(m));
      __builtin_amdgcn_wave_barrier();
      if (pending >= uint32_t(kWave)) {
        search_batch<D, MODE>(p, w, K, first != 0, cur, queue[lane], true, &work);
        const uint32_t moved = queue[kWave + lane];  // entries kWave.. move to the front
        __builtin_amdgcn_wave_barrier();
        queue[lane] = moved;
        __builtin_amdgcn_wave_barrier();
        pending -= uint32_t(kWave);
      }
    }
    if (pending != 0) {
      const uint32_t qv = queue[min(uint32_t(lane), pending - 1)];
      search_batch<D, MODE>(p, w, K, first != 0, cur, qv, uint32_t(lane) < pending, &work);
    }
  }
  if (p.count_work) add_work(w.hdr, kWorkSearch, lane == 0 ? work : 0);
}

// Open points after the search stages, as a list in cell order.  Each thread
// reads kCollectPer flags; a block counts its open points, takes its slice of
// the list with one atomic and writes it in order (one atomic per block: a
// counter that every wave bumps serialises in L2).
constexpr int kCollectPer = 16;

__device__ __forceinline__ void collect_body(Blk blk, const Plan &p, const uint8_t *__restrict__ flag,
                                             uint32_t *__restrict__ unres, DevHeader *__restrict__ hdr) {
  __shared__ uint32_t wave_tot[kWavesPerBlock];
  __shared__ uint32_t base;
  constexpr int64_t kChunk = int64_t(kBlock) * kCollectPer;
  const int64_t chunks = (p.n + kChunk - 1) / kChunk;
  for (int64_t c = blk.b; c < chunks; c += blk.nb) {
    const int64_t i0 = c * kChunk + int64_t(threadIdx.x) * kCollectPer;
    uint32_t open = 0;
#pragma unroll
    for (int k = 0; k < kCollectPer; ++k) {
      const int64_t i = i0 + k;
      open |= (i < p.n && flag[i < p.n ? i : 0] != 0) ? (1u << k) : 0u;
    }
    uint32_t tot;
    const uint32_t off = wave_exclusive_scan(uint32_t(__popc(open)), &tot);
    const int wv = threadIdx.x / kWave;
    wave_tot[wv] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t sum = 0;
      for (int k = 0; k < kWavesPerBlock; ++k) sum += wave_tot[k];
      base = atomicAdd(&hdr->n_unres, sum);
    }
    __syncthreads();
    uint32_t at = base + off;
    for (int k = 0; k < wv; ++k) at += wave_tot[k];
#pragma unroll
    for (int k = 0; k < kCollectPer; ++k) {
      if (open & (1u << k)) unres[at++] = uint32_t(i0 + k);
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------- ring k

__device__ __forceinline__ int64_t gap_to(int32_t x, int64_t lo, int64_t hi) {
  return x < lo ? lo - x : (x > hi ? x - hi : 0);
}

template <int D>
__device__ __forceinline__ uint64_t exact_d2(const int32_t *a, DPC_CONST(int32_t) * b) {
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int64_t df = int64_t(a[k] - b[k]);
    s += df * df;
  }
  return uint64_t(s);
}

template <int D>
__device__ __forceinline__ uint64_t exact_d2_v(const int32_t *a, const int32_t *b) {
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int64_t df = int64_t(a[k] - b[k]);
    s += df * df;
  }
  return uint64_t(s);
}

// Ring search for the points the search stages left open, one wave per point.
// Each pass grows the searched block from the cells within k0 of the point's
// cell (the last stage's radius) to k1 = 2 k0 (an annulus per pass, so a sparse
// neighbourhood needs a logarithmic number of passes); the point is final once
// its best candidate is strictly closer than the exterior of the block.  With a
// candidate at squared distance b, a pass also leaves out the cells farther than
// sqrt(b) from the point in some dimension; when that bound is tighter than the
// block on every side, the pass has seen every cell within sqrt(b) of the point,
// so every point closer than the best, and the point is final too.  In every
// row the cell range is clipped to the cells that can still hold a point within
// the best distance so far, and a row farther than that is skipped.  A
// pass takes its rows kRingRows per lane at a time (their cell ranges loaded
// together), flattens their candidates over the wave and tests two per lane at
// a time.  The point goes to the prefix scan when the passes have cost more than
// that scan would.
#ifndef DPC_RING_ROWS
#define DPC_RING_ROWS 2
#endif
constexpr int kRingRows = DPC_RING_ROWS;  // rows per lane per round

struct SegLds {
  uint32_t off[kWave];                // exclusive prefix of the lanes' candidate counts
  uint2 seg[kWave][2 * kRingRows];    // each lane's row pieces: {first position, count}
};

template <int D>
__device__ __forceinline__ void ringk_body(Blk blk, const Plan &p, const Ws &w, int k_start) {
  __shared__ SegLds lds_all[kWavesPerBlock];
  SegLds &lds = lds_all[threadIdx.x / kWave];
  constexpr int RA = D > 1 ? D - 1 : 1;
  const int lane = lane_id();
  if (grid_skipped(w.hdr)) return;
  // the open-point stage's list when it ran, else the first stage's
  const uint32_t nunres = uniform(as_const(p.openK ? &w.hdr->n_ring : &w.hdr->n_unres)[0]);
  if (p.openK) k_start = p.openK;
  DPC_CONST(int32_t) *spc = as_const(w.spts);
  DPC_CONST(uint64_t) *sKc = as_const(w.sK);
  DPC_CONST(uint32_t) *unres = as_const(p.openK ? w.slot : w.unres);
  DPC_CONST(uint32_t) *rstart = as_const(w.rcnt);
  const int32_t L = p.L, nc = p.nc;
  const int nr = p.gm - 1;  // row dimensions
  constexpr int W = (D + 1) / 2;
  // packed candidate records (lane form with the packed path, d <= 4, every
  // coordinate indexed)
  const bool use_rec = W <= 2 && w.srec != nullptr && p.gm == D;

  uint64_t work = 0;  // candidate tests (wave-uniform; profiling)
  const uint32_t nw = grid_waves(blk);
  for (uint32_t u = wave_index(blk); u < nunres; u += nw) {
    const uint32_t entry = uniform(unres[u]);
    const uint32_t q = entry & ~kRingFromFirst;
    int32_t x[D], c[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      x[k] = uniform(spc[int64_t(q) * D + k]);
      c[k] = x[k] / L;
    }
    const int32_t xs = uniform(spc[int64_t(q) * D + nr]);  // coordinate along the strip dimension
    uint32_t qk[W];  // its packed words, for the packed candidate records
#pragma unroll
    for (int k = 0; k < W; ++k) qk[k] = use_rec ? uniform(as_const(w.spk)[int64_t(q) * W + k]) : 0u;
    const int32_t cl = xs / L;
    const uint64_t Ki = uniform(sKc[q]);
    const int64_t rho = int64_t(Ki >> 32);
    uint64_t best = uniform(w.best[q]);
    const uint32_t prefix = uniform(rstart[p.n - rho + 1]);
    const int64_t budget = min(int64_t(prefix / kWave) + 2, int64_t(p.ring_cap));
    int64_t cost = 0;
    bool defer = false;
    // -1: nothing searched yet
    int32_t k0 = (entry & kRingFromFirst) ? (p.stageK[0] == 0 ? -1 : p.stageK[0]) : k_start;

    for (;;) {
      // This pass: the cells of the box [lo, lo + ext) (row dimensions) x [sa, sb]
      // (strip dimension) outside the block within k0 of the point's cell.
      const bool has_best = best != kNoKey;
      const int32_t k1 = k0 < 1 ? 1 : min(2 * k0, nc);
      const int32_t rb = has_best ? sqrt_ceil_bound(best >> kIdBits) : 0;
      bool covered = has_best;  // the radius bound is the tighter one on every side
      auto box = [&](int32_t xt, int32_t ct, int32_t *a, int32_t *b) {
        *a = max(ct - k1, 0);
        *b = min(ct + k1, nc - 1);
        if (has_best) {
          const int32_t ra = max(xt - rb, 0) / L, rz = min(xt + rb, DPC_COORD_LIMIT - 1) / L;
          covered = covered && (ra >= *a || *a == 0) && (rz <= *b || *b == nc - 1);
          *a = max(*a, ra);
          *b = min(*b, rz);
        }
      };
      int32_t lo[RA], ext[RA];
      uint64_t nrows = 1;
#pragma unroll
      for (int t = 0; t < RA; ++t) {
        lo[t] = 0;
        ext[t] = 1;
        if (t < nr) {
          int32_t a, b;
          box(x[t], c[t], &a, &b);
          lo[t] = a;
          ext[t] = b - a + 1;
          nrows *= uint64_t(ext[t]);
        }
      }
      int32_t sa, sb;
      box(xs, cl, &sa, &sb);
      // The packed 16-bit records serve while every candidate of the block lies
      // within (k1 + 1) L - 1 of the point in each coordinate, all of them indexed.
      const bool packed = use_rec && (int64_t(k1) + 1) * L <= int64_t(p.ext16);
      // A pass costs at least kRingRows per round: one that cannot end within the
      // budget defers the point at once.
      constexpr uint32_t kStride = kWave * kRingRows;  // rows per round
      if (cost + int64_t(kRingRows) * int64_t((nrows + kStride - 1) / kStride) >= budget) {
        defer = true;
        break;
      }
      // Rows are visited as mixed-radix numbers (digit t in [0, ext[t])): each lane
      // keeps the digits of its kRingRows rows and adds the round stride to them
      // with carries.  nrows < 2^26 here (the budget is at most 2^20).
      uint32_t sd[RA], dd[kRingRows][RA], rl[kRingRows];
      {
        // r / e as a high product with m = ceil(2^32 / e): exact while r * e < 2^32
        // (here r < kStride and e <= nc < 2^18)
        uint32_t m[RA];
#pragma unroll
        for (int t = 0; t < RA; ++t) m[t] = ext[t] > 1 ? 0xFFFFFFFFu / uint32_t(ext[t]) + 1u : 0u;
        auto digits = [&](uint32_t r, uint32_t *dg) {
#pragma unroll
          for (int t = 0; t < RA; ++t) {
            const uint32_t q = ext[t] > 1 ? __umulhi(r, m[t]) : r;
            dg[t] = r - q * uint32_t(ext[t]);
            r = q;
          }
        };
        digits(kStride, sd);
#pragma unroll
        for (int i = 0; i < kRingRows; ++i) {
          rl[i] = uint32_t(i * kWave + lane);
          digits(rl[i], dd[i]);
        }
      }
      const float inv_l = 1.0f / float(L);
      for (uint32_t r0b = 0; r0b < uint32_t(nrows); r0b += kStride) {
        const uint64_t bestd2 = best >> kIdBits;  // huge when there is no best yet
        // the best distance as a float a little above it (no clipping without one)
        const bool clip = bestd2 < (uint64_t(1) << 40);
        const float bf = clip ? float(bestd2) * (1.0f + 0x1p-20f) + 1.0f : 0.0f;
        uint2 sg[2 * kRingRows];
        uint32_t mine = 0;  // this lane's candidates in the round
#pragma unroll
        for (int i = 0; i < kRingRows; ++i) {
          sg[2 * i] = make_uint2(0u, 0u);
          sg[2 * i + 1] = make_uint2(0u, 0u);
          if (rl[i] < uint32_t(nrows)) {
            float mdf = 0.0f;  // squared gap of the row, a little below the exact value
            int32_t rowk = 0;  // row index of the cell table (ncells < 2^31)
            bool outer = k0 < 0;
#pragma unroll
            for (int t = 0; t < RA; ++t) {
              if (t < nr) {
                const int32_t nb = lo[t] + int32_t(dd[i][t]);
                const int32_t o = nb - c[t];
                outer = outer || o > k0 || o < -k0;
                rowk = rowk * nc + nb;
                const float gp = float(cell_gap32(x[t], nb, L));  // exact: below 2^24
                mdf = __builtin_fmaf(gp, gp, mdf);
              }
            }
            mdf *= 1.0f - 0x1p-20f;
            // A row is skipped only when it is surely farther than the best.
            if (!clip || mdf <= bf) {
              // strip-dimension cells that can hold a point within the best distance:
              // a bound above sqrt(best - gap^2), and cell indices rounded outwards
              int32_t lo_s = sa, hi_s = sb;
              if (clip) {
                // the hardware root (within a few ulp; the margin is 8 ulp)
                const float rr = sqrt_approx(bf - mdf) * (1.0f + 0x1p-20f) + 1.0f;
                const float xa = float(xs) - rr, xz = float(xs) + rr;
                if (xa > 0.0f) lo_s = max(lo_s, int32_t(xa * inv_l * (1.0f - 0x1p-20f)));
                if (xz < float(DPC_COORD_LIMIT)) hi_s = min(hi_s, int32_t(xz * inv_l * (1.0f + 0x1p-20f)));
              }
              // (in lane form, meant for sparse data, a piece of empty cells, the
              // common case in a sparse annulus, is skipped by its occupancy bits
              // without touching the table)
              const int32_t base = rowk * nc;
              auto occupied = [&](int32_t a, int32_t b) { return !p.lanes || cells_occupied(w.occ, base + a, base + b); };
              if (outer) {  // the whole row lies outside the block searched so far
                if (lo_s <= hi_s && occupied(lo_s, hi_s)) {
                  const uint32_t b = w.cnt[base + lo_s];
                  sg[2 * i] = make_uint2(b, w.cnt[base + hi_s + 1] - b);
                }
              } else {  // two pieces: left and right of the searched block
                const int32_t l_hi = min(hi_s, cl - k0 - 1), r_lo = max(lo_s, cl + k0 + 1);
                if (lo_s <= l_hi && occupied(lo_s, l_hi)) {
                  const uint32_t b = w.cnt[base + lo_s];
                  sg[2 * i] = make_uint2(b, w.cnt[base + l_hi + 1] - b);
                }
                if (r_lo <= hi_s && occupied(r_lo, hi_s)) {
                  const uint32_t b = w.cnt[base + r_lo];
                  sg[2 * i + 1] = make_uint2(b, w.cnt[base + hi_s + 1] - b);
                }
              }
            }
          }
          // the lane's row in the next round
          uint32_t carry = 0;
#pragma unroll
          for (int t = 0; t < RA; ++t) {
            const uint32_t v = dd[i][t] + sd[t] + carry;
            carry = v >= uint32_t(ext[t]) ? 1u : 0u;
            dd[i][t] = carry ? v - uint32_t(ext[t]) : v;
          }
          rl[i] += kStride;
        }
#pragma unroll
        for (int i = 0; i < 2 * kRingRows; ++i) mine += sg[i].y;
        uint32_t total;
        const uint32_t off = wave_exclusive_scan(mine, &total);
        total = uniform(total);
        cost += kRingRows + (total + kWave - 1) / kWave;
        // Stop before a round that would cost more than scanning the density
        // prefix (a dense neighbourhood around a density peak).
        if (cost >= budget) break;
        work += total;
        lds.off[lane] = off;
#pragma unroll
        for (int i = 0; i < 2 * kRingRows; ++i) lds.seg[lane][i] = sg[i];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        uint64_t lbest = kNoKey;
        for (uint32_t fb = 0; fb < total; fb += 2 * kWave) {
          // two candidates per lane: both positions first, then both loads
          uint32_t pos[2];
          bool have[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint32_t f = fb + uint32_t(h * kWave + lane);
            have[h] = f < total;
            int s = 0;  // last lane whose offset is <= f
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
              if (lds.off[s + step] <= f) s += step;
            uint32_t rel = f - lds.off[s], at = 0;
            bool found = false;
#pragma unroll
            for (int i = 0; i < 2 * kRingRows; ++i) {
              const uint2 g = lds.seg[s][i];
              const bool in = !found && rel < g.y;
              at = in ? g.x + rel : at;
              rel = (found || in) ? rel : rel - g.y;
              found = found || in;
            }
            pos[h] = have[h] ? at : 0u;
          }
          uint64_t kj[2], d2[2];
          if (packed) {  // one 16-byte record per candidate
            uint4 rec[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) rec[h] = w.srec[pos[h]];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              kj[h] = (uint64_t(rec[h].w) << 32) | rec[h].z;
              int32_t a = dot2_self_v(pk_sub16(qk[0], rec[h].x), 0);
              if (W == 2) a = dot2_self_v(pk_sub16(qk[W - 1], rec[h].y), a);
              d2[h] = uint32_t(a);
            }
          } else {
            int32_t y[2][D];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              kj[h] = w.sK[pos[h]];
#pragma unroll
              for (int t = 0; t < D; ++t) y[h][t] = w.spts[int64_t(pos[h]) * D + t];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) d2[h] = exact_d2_u<D>(x, y[h]);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint64_t key = (d2[h] << kIdBits) | uint32_t(~uint32_t(kj[h]));
            lbest = (have[h] && kj[h] > Ki && key < lbest) ? key : lbest;
          }
        }
        __builtin_amdgcn_wave_barrier();
        const uint64_t wb = uniform(wave_min_u64(lbest));
        best = wb < best ? wb : best;
      }
      if (cost >= budget) {  // the pass is incomplete: only the prefix scan is exact now
        defer = true;
        break;
      }
      // Every cell within the starting best distance has been seen.
      if (covered) break;
      // The searched block is now every cell within k1 of the point's cell (in
      // the grid dimensions; a gap in one of them bounds the full distance).
      int64_t gap = INT64_MAX;
#pragma unroll
      for (int t = 0; t < D; ++t) {
        if (t < p.gm) {
          if (c[t] - k1 >= 1) gap = min(gap, int64_t(x[t]) - int64_t(c[t] - k1) * L + 1);
          if (c[t] + k1 <= nc - 2) gap = min(gap, int64_t(c[t] + k1 + 1) * L - int64_t(x[t]));
        }
      }
      if (gap == INT64_MAX) break;  // the block covers the whole grid
      if (best != kNoKey && (best >> kIdBits) < uint64_t(gap) * uint64_t(gap)) break;
      k0 = k1;
    }
    // Every lane stores the same values (no lane-divergent branch in the loop);
    // `defer` is wave-uniform, so its branch is a scalar one.
    w.best[q] = best;
    if (uniform(defer ? 1u : 0u) != 0u) {
      const uint32_t slot = uniform(wave_append(&w.hdr->n_peaks, lane == 0));
      w.peaks[slot] = q;
      if (lane == 0) atomicMax(&w.hdr->rank_end, prefix);  // the ranks its prefix scan reads
    }
  }
  if (p.count_work) add_work(w.hdr, kWorkRing, lane == 0 ? work : 0);
}

// -------------------------------------------------------------------- peaks

// Prefix scan for the points the ring search deferred.  A work unit is 64
// deferred points (one per lane) and one chunk of kPeakChunk positions of the
// rank-sorted copy; the wave streams the chunk with scalar loads, so each
// candidate is loaded once for 64 points.  Lane i takes candidate r when r ranks
// above it: r before its density bucket, or in its bucket with a smaller id
// (buckets are unordered inside).  Units are spread over all waves, and each
// lane merges its chunk minimum into best[] with a 64-bit atomic minimum.
template <int D>
__device__ __forceinline__ void peak_batch_load(DPC_CONST(int32_t) * rpc, DPC_CONST(int32_t) * ridc, uint32_t r,
                                                int32_t *c, int32_t *idr) {
  constexpr int B = 16 / D > 0 ? 16 / D : 1;
  DPC_CONST(int32_t) *cb = rpc + int64_t(r) * D;
  DPC_CONST(int32_t) *ib = ridc + r;
#pragma unroll
  for (int v = 0; v < B * D; ++v) c[v] = cb[v];
#pragma unroll
  for (int v = 0; v < B; ++v) idr[v] = ib[v];
}

template <int D>
__device__ __forceinline__ void peaks_body(Blk blk, const Plan &p, const Ws &w) {
  constexpr int B = 16 / D > 0 ? 16 / D : 1;  // candidates per scalar-load batch
  const int lane = lane_id();
  if (grid_skipped(w.hdr)) return;
  const uint32_t npeaks = uniform(as_const(&w.hdr->n_peaks)[0]);
  const uint32_t ngroups = (npeaks + kWave - 1) / kWave;
  const uint32_t nchunks = uint32_t((p.n + kPeakChunk - 1) / kPeakChunk);
  const uint64_t units = uint64_t(ngroups) * nchunks;
  DPC_CONST(int32_t) *rpc = as_const(w.rpts);
  DPC_CONST(int32_t) *ridc = as_const(w.rid);
  uint64_t work = 0;  // candidate tests of owned points (wave-uniform; profiling)

  const uint32_t nw = grid_waves(blk);
  for (uint64_t u = wave_index(blk); u < units; u += nw) {
    const uint32_t g = uint32_t(u % ngroups);
    const uint32_t ch = uint32_t(u / ngroups);
    const uint32_t q = w.peaks[min(g * uint32_t(kWave) + uint32_t(lane), npeaks - 1u)];
    const uint64_t Ki = w.sK[q];
    const int32_t id = int32_t(~uint32_t(Ki));
    const int64_t rho = int64_t(Ki >> 32);
    const uint32_t bstart = w.rcnt[p.n - rho];
    const uint32_t bend = w.rcnt[p.n - rho + 1];
    const uint32_t r0 = ch * uint32_t(kPeakChunk);
    const uint32_t r1 = min(r0 + uint32_t(kPeakChunk), uint32_t(uniform(wave_max_i32(int32_t(bend)))));
    if (r0 >= r1) continue;  // wave-uniform: the chunk lies past every lane's prefix
    work += uint64_t(r1 - r0) * min(uint32_t(kWave), npeaks - g * uint32_t(kWave));
    int32_t x[D];
#pragma unroll
    for (int t = 0; t < D; ++t) x[t] = w.spts[int64_t(q) * D + t];
    uint64_t lbest = kNoKey;
    uint32_t r = r0;
    if (r + B <= r1) {
      int32_t c[B * D], idr[B];
      peak_batch_load<D>(rpc, ridc, r, c, idr);
      for (;;) {
        // Load the next batch (or this one again at the end) before using this one.
        const uint32_t rn = r + B;
        const bool more = rn + B <= r1;
        int32_t cn[B * D], idn[B];
        peak_batch_load<D>(rpc, ridc, more ? rn : r, cn, idn);
#pragma unroll
        for (int v = 0; v < B; ++v) {
          const uint32_t rv = r + uint32_t(v);
          // rank above: before the bucket, or inside it with a smaller id (no short circuit)
          const bool above = (rv < bstart) | ((rv < bend) & (idr[v] < id));
          const uint64_t key = (exact_d2_v<D>(x, c + v * D) << kIdBits) | uint32_t(idr[v]);
          lbest = (above & (key < lbest)) ? key : lbest;
        }
        r = rn;
        if (!more) break;
#pragma unroll
        for (int v = 0; v < B * D; ++v) c[v] = cn[v];
#pragma unroll
        for (int v = 0; v < B; ++v) idr[v] = idn[v];
      }
    }
    for (; r < r1; ++r) {
      int32_t c[D];
#pragma unroll
      for (int t = 0; t < D; ++t) c[t] = rpc[int64_t(r) * D + t];
      const int32_t idr = ridc[r];
      const bool above = (r < bstart) | ((r < bend) & (idr < id));
      const uint64_t key = (exact_d2_v<D>(x, c) << kIdBits) | uint32_t(idr);
      lbest = (above & (key < lbest)) ? key : lbest;
    }
    // Only lanes that hold a point of the list and found a candidate merge: lanes
    // past the end repeat the last point, and atomics of many lanes on one
    // address serialise in L2.  (A plain if-region: no loop depends on it.)
    const bool own = g * uint32_t(kWave) + uint32_t(lane) < npeaks;
    if (own && lbest != kNoKey)
      atomicMin(reinterpret_cast<unsigned long long *>(&w.best[q]), static_cast<unsigned long long>(lbest));
  }
  if (p.count_work) add_work(w.hdr, kWorkPeaks, lane_id() == 0 ? work : 0);
}

// -------------------------------------------------------------------- finish

// The outputs in id order: each id reads its cell-order position (contiguous
// stores, cache-friendly gathered reads); rho too when `rho` is not null.
__device__ __forceinline__ void finish_body(Blk blk, const Plan &p, const Ws &w, int32_t *__restrict__ dep,
                                            double *__restrict__ delta, int32_t *__restrict__ rho) {
  if (grid_skipped(w.hdr)) return;
  for (int64_t i = thread_index(blk); i < p.n; i += grid_threads(blk)) {
    const uint32_t q = w.key[i];
    const uint64_t key = w.best[q];
    if (key == kNoKey) {
      dep[i] = -1;
      delta[i] = __builtin_huge_val();
    } else {
      dep[i] = int32_t(key & kIdMask);
      delta[i] = __builtin_sqrt(double(key >> kIdBits));  // correctly rounded (IEEE sqrt)
    }
    if (rho) rho[i] = int32_t(w.sK[q] >> 32);
  }
}

// -------------------------------------------------------------------- kernels

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_search(Plan p, Ws w, int K, int group, int first) {
  search_body<D, MODE>(grid_blk(), p, w, K, group, first);
}
// The lane-form stage covers every point with a grid sized to them, its blocks
// renumbered per XCD (neighbouring points share an L2).
template <int D, int MODE>
__global__ __launch_bounds__(kBlock) DPC_WAVES(DPC_SEARCH_WAVES) void k_search_lanes(Plan p, Ws w, int K) {
  search_lanes<D, MODE>(xcd_blk(), p, w, K);
}
__global__ __launch_bounds__(kBlock) void k_collect(Plan p, Ws w) { collect_body(grid_blk(), p, w.flag, w.unres, w.hdr); }
template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_search_open(Plan p, Ws w) {
  search_open<D, MODE>(grid_blk(), p, w, p.openK, p.stageK[0]);
}
template <int D>
__global__ __launch_bounds__(kBlock) DPC_WAVES(DPC_RING_WAVES) void k_ringk(Plan p, Ws w, int k_start) {
  ringk_body<D>(grid_blk(), p, w, k_start);
}
template <int D>
__global__ __launch_bounds__(kBlock) void k_peaks(Plan p, Ws w) {
  peaks_body<D>(grid_blk(), p, w);
}
__global__ __launch_bounds__(kBlock) void k_finish(Plan p, Ws w, int32_t *dep, double *delta, int32_t *rho) {
  finish_body(grid_blk(), p, w, dep, delta, rho);
}

// Many-job forms: virtual block v of map m runs the body for its job.
#define DPC_FOR_VBLOCKS(m)                                             \
  for (uint32_t v = (m).v0 + blockIdx.x; v < (m).v1; v += gridDim.x) { \
    const uint32_t j = vjob_of((m), v);                                \
    const Blk k = vblk_of((m), v, j);                                  \
    const Plan p = load_uniform(&jobs[j].p);                                \
    const Ws w = load_uniform(&jobs[j].w);

// Stage st of every job that has one (the mode is per job).
template <int D>
__global__ __launch_bounds__(kBlock) void kb_search(const JobDev *jobs, VMap m, int st) {
  DPC_FOR_VBLOCKS(m)
  if (st < p.nstages) {
    // stage parameters straight from the job table (scalar loads; indexing the
    // local copy with a run-time stage would put it in scratch memory)
    const int K = uniform(int32_t(as_const(jobs)[j].p.stageK[st]));
    const int group = uniform(int32_t(as_const(jobs)[j].p.stageGroup[st]));
    const int mode = uniform(int32_t(as_const(jobs)[j].p.stageMode[st]));
    if (p.lanes) {
      if (mode == kModeP16)
        search_lanes<D, kModeP16>(k, p, w, K);
      else
        search_lanes<D, kModeI64>(k, p, w, K);
    } else if (mode == kModeP16)
      search_body<D, kModeP16>(k, p, w, K, group, st == 0 ? 1 : 0);
    else
      search_body<D, kModeI64>(k, p, w, K, group, st == 0 ? 1 : 0);
  }
}
}

__global__ __launch_bounds__(kBlock) void kb_collect(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  collect_body(k, p, w.flag, w.unres, w.hdr);
}
}

template <int D>
__global__ __launch_bounds__(kBlock) void kb_search_open(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  if (p.openK) {
    if (p.openMode == kModeP16)
      search_open<D, kModeP16>(k, p, w, p.openK, p.stageK[0]);
    else
      search_open<D, kModeI64>(k, p, w, p.openK, p.stageK[0]);
  }
}
}

template <int D>
__global__ __launch_bounds__(kBlock) void kb_ringk(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  const int kl = uniform(int32_t(as_const(jobs)[j].p.stageK[p.nstages - 1]));
  ringk_body<D>(k, p, w, kl == 0 ? -1 : kl);  // after a ball stage no cell block is known searched
}
}

template <int D>
__global__ __launch_bounds__(kBlock) void kb_peaks(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  peaks_body<D>(k, p, w);
}
}

__global__ __launch_bounds__(kBlock) void kb_finish(const JobDev *jobs, VMap m) {
  DPC_FOR_VBLOCKS(m)
  finish_body(k, p, w, as_const(jobs)[j].dep, as_const(jobs)[j].delta, as_const(jobs)[j].rho);
}
}

#undef DPC_FOR_VBLOCKS

template <int D>
hipError_t launch_dep_d(const Plan &p, const Ws &w, int32_t *dep, double *delta, int32_t *rho, hipStream_t s) {
  if (p.lanes) {  // one stage in lane form
    ProfScope ps(s, kProfSearch);
    const unsigned blocks = blocks_for(p.n, kBlock);
    if (p.stageMode[0] == kModeP16)
      DPC_LAUNCH((k_search_lanes<D, kModeP16>), blocks, kBlock, s, p, w, p.stageK[0]);
    else
      DPC_LAUNCH((k_search_lanes<D, kModeI64>), blocks, kBlock, s, p, w, p.stageK[0]);
  } else {
    ProfScope ps(s, kProfSearch);
    for (int st = 0; st < p.nstages; ++st) {
      const int K = p.stageK[st], group = p.stageGroup[st];
      const unsigned blocks = persistent_blocks((p.max_tasks + group - 1) / group);
      if (p.stageMode[st] == kModeP16)
        DPC_LAUNCH((k_search<D, kModeP16>), blocks, kBlock, s, p, w, K, group, st == 0 ? 1 : 0);
      else
        DPC_LAUNCH((k_search<D, kModeI64>), blocks, kBlock, s, p, w, K, group, st == 0 ? 1 : 0);
    }
  }
  const unsigned rb = persistent_blocks(p.n);
  {
    ProfScope ps(s, kProfSearch);  // the open points' list closes the window search
    DPC_LAUNCH((k_collect), blocks_for(p.n, kBlock * kCollectPer), kBlock, s, p, w);
  }
  if (p.openK) {  // kOpenLanes lanes per open point: up to 16 points each if all were open
    ProfScope ps(s, kProfOpen);
    const unsigned ob = blocks_for(p.n, kBlock * 16 / kOpenLanes);
    if (p.openMode == kModeP16)
      DPC_LAUNCH((k_search_open<D, kModeP16>), ob, kBlock, s, p, w);
    else
      DPC_LAUNCH((k_search_open<D, kModeI64>), ob, kBlock, s, p, w);
  }
  {
    ProfScope ps(s, kProfRingK);
    const int kl = p.stageK[p.nstages - 1];
    DPC_LAUNCH((k_ringk<D>), rb, kBlock, s, p, w, kl == 0 ? -1 : kl);  // after a ball stage: nothing
  }
  {
    ProfScope ps(s, kProfPeaks);
    hipError_t e = launch_rank_gather(p, w, s);
    if (e != hipSuccess) return e;
    DPC_LAUNCH((k_peaks<D>), rb, kBlock, s, p, w);
  }
  ProfScope ps(s, kProfFinish);
  DPC_LAUNCH((k_finish), blocks_for(p.n, kBlock), kBlock, s, p, w, dep, delta, rho);
  return hipGetLastError();
}

template <int D>
hipError_t remainder_d(const Plan &p, const Ws &w, hipStream_t s) {
  const unsigned rb = persistent_blocks(p.n);
  {
    ProfScope ps(s, kProfRingK);
    DPC_LAUNCH((k_ringk<D>), rb, kBlock, s, p, w, -1);  // nothing searched yet
  }
  ProfScope ps(s, kProfPeaks);
  hipError_t e = launch_rank_gather(p, w, s);
  if (e != hipSuccess) return e;
  DPC_LAUNCH((k_peaks<D>), rb, kBlock, s, p, w);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dependent(const Plan &p, const Ws &w, int32_t *dep, double *delta, int32_t *rho, hipStream_t s) {
  switch (p.d) {
    case 1: return launch_dep_d<1>(p, w, dep, delta, rho, s);
    case 2: return launch_dep_d<2>(p, w, dep, delta, rho, s);
    case 3: return launch_dep_d<3>(p, w, dep, delta, rho, s);
    case 4: return launch_dep_d<4>(p, w, dep, delta, rho, s);
    case 5: return launch_dep_d<5>(p, w, dep, delta, rho, s);
    case 6: return launch_dep_d<6>(p, w, dep, delta, rho, s);
    case 7: return launch_dep_d<7>(p, w, dep, delta, rho, s);
    case 8: return launch_dep_d<8>(p, w, dep, delta, rho, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_collect(const Plan &p, const Ws &w, hipStream_t s) {
  DPC_LAUNCH((k_collect), blocks_for(p.n, kBlock * kCollectPer), kBlock, s, p, w);
  return hipGetLastError();
}

hipError_t launch_exact_remainder(const Plan &p, const Ws &w, hipStream_t s) {
  if (p.openK) return hipErrorInvalidValue;  // the ring search would read the open stage's list
  switch (p.d) {
    case 1: return remainder_d<1>(p, w, s);
    case 2: return remainder_d<2>(p, w, s);
    case 3: return remainder_d<3>(p, w, s);
    case 4: return remainder_d<4>(p, w, s);
    case 5: return remainder_d<5>(p, w, s);
    case 6: return remainder_d<6>(p, w, s);
    case 7: return remainder_d<7>(p, w, s);
    case 8: return remainder_d<8>(p, w, s);
    default: return hipErrorInvalidValue;
  }
}

// Search stages, ring search and prefix scan of every dimension group, then
// finish.  The open points are gathered (kb_collect) after the stages of every
// group, so the groups' stages go first.
template <int DD>
void batch_dep_group(const BatchMaps &B, const VMap &m, int what, int st, hipStream_t s) {
  if (what == 0) {
    DPC_LAUNCH((kb_search<DD>), vgrid(m), kBlock, s, B.jobs, m, st);
  } else if (what == 2) {
    ProfScope ps(s, kProfOpen);
    DPC_LAUNCH((kb_search_open<DD>), vgrid(m), kBlock, s, B.jobs, m);
  } else if (what == 1) {
    ProfScope ps(s, kProfRingK);
    DPC_LAUNCH((kb_ringk<DD>), vgrid(m), kBlock, s, B.jobs, m);
  } else {
    ProfScope ps(s, kProfPeaks);
    DPC_LAUNCH((kb_peaks<DD>), vgrid(m), kBlock, s, B.jobs, m);
  }
}

hipError_t batch_groups(const BatchMaps &B, int what, int st, hipStream_t s) {
  for (int g = 0; g < B.ngroups; ++g) {
    VMap m = B.work;
    m.v0 = B.gwork0[g];
    m.v1 = B.gwork1[g];
    if (!vgrid(m)) continue;
    switch (B.gdim[g]) {
      case 1: batch_dep_group<1>(B, m, what, st, s); break;
      case 2: batch_dep_group<2>(B, m, what, st, s); break;
      case 3: batch_dep_group<3>(B, m, what, st, s); break;
      case 4: batch_dep_group<4>(B, m, what, st, s); break;
      case 5: batch_dep_group<5>(B, m, what, st, s); break;
      case 6: batch_dep_group<6>(B, m, what, st, s); break;
      case 7: batch_dep_group<7>(B, m, what, st, s); break;
      case 8: batch_dep_group<8>(B, m, what, st, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t batch_dependent(const BatchMaps &B, hipStream_t s) {
  hipError_t e;
  {
    ProfScope ps(s, kProfSearch);
    for (int st = 0; st < B.max_stages; ++st)
      if ((e = batch_groups(B, 0, st, s)) != hipSuccess) return e;
  }
  {
    ProfScope ps(s, kProfSearch);
    if (vgrid(B.pts)) DPC_LAUNCH((kb_collect), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  }
  if (B.any_open && (e = batch_groups(B, 2, 0, s)) != hipSuccess) return e;
  if ((e = batch_groups(B, 1, 0, s)) != hipSuccess) return e;
  {
    ProfScope ps(s, kProfPeaks);
    if ((e = batch_rank_gather(B, s)) != hipSuccess) return e;
  }
  if ((e = batch_groups(B, 3, 0, s)) != hipSuccess) return e;
  ProfScope ps(s, kProfFinish);
  if (vgrid(B.pts)) DPC_LAUNCH((kb_finish), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  return hipGetLastError();
}

}  // namespace dpc
