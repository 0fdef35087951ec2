// Local density (Def. 1, Eq. 1): rho_i = #{ j : D2(i, j) < R }, the point itself
// included, R = ceil(d_cut^2).  The count goes into the rank key (rho << 32) | ~id
// of the point's cell-order position (contiguous stores); write_rho copies it to
// the caller's id order, reading the cell-order array at each id's position.
//
// Two forms, picked by the plan:
//
// * tasks (dense data): one wave per task (64 queries of one strip, one per
//   lane).  The window holds the cells within K0 of the task's cells (K0 * L >=
//   floor(sqrt(R - 1)), so it covers every d_cut-ball) and is clipped to the
//   balls' union row by row.  The wave walks its candidate runs with scalar
//   loads, so every candidate reaches all 64 lanes as a scalar operand: no LDS,
//   no barriers.  Waves take tasks in a static interleave (see wave_index); the
//   paper balances its per-point range searches with dynamic OpenMP scheduling
//   (Section 3);
// * lanes (sparse data, where a strip holds a few points and a task would leave
//   most lanes idle): one query per lane, each with its own window of radius K0
//   around its cell, clipped to its own ball row by row; candidates are read with
//   per-lane vector loads.
#include "tasks.h"

namespace dpc {
namespace {

template <int D, int MODE>
__device__ __forceinline__ void density_body(Blk blk, const Plan &p, const Ws &w) {
  constexpr int W = (D + 1) / 2;
  const int lane = lane_id();
  DPC_CONST(uint32_t) *spk = as_const(w.spk);
  DPC_CONST(int32_t) *spc = as_const(w.spts);
  DPC_CONST(uint32_t) *tc = as_const(reinterpret_cast<const uint32_t *>(w.tasks));
  const uint32_t ntasks = uniform(as_const(&w.hdr->ntasks)[0]);
  const int32_t negR = -int32_t(p.R < INT32_MAX ? p.R : INT32_MAX);
  const int K = p.K0;
  const uint64_t clip2 = uint64_t(p.R - 1);  // D2 <= R - 1 is inside the ball
  const int nrow = int(window_rows(p, K));

  uint64_t work = 0;  // candidate tests of the wave's valid queries (profiling)
  const uint32_t nw = grid_waves(blk);
  for (uint32_t t = wave_index(blk); t < ntasks; t += nw) {
    const int r_lo = 0, r_hi = nrow;
    const uint32_t qb = uniform(uint32_t(tc[4 * int64_t(t)]));
    const uint32_t qe = uniform(uint32_t(tc[4 * int64_t(t) + 1]));
    TaskGeom<D> g;
    strip_row<D>(p, uniform(uint32_t(tc[4 * int64_t(t) + 2])), g);
    const uint32_t q = min(qb + uint32_t(lane), qe - 1u);
    int32_t qx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) qx[k] = w.spts[int64_t(q) * D + k];
    task_span<D>(p, g, w.spts[int64_t(q) * D + (p.gm - 1)], true);  // strip-dimension coordinate
    uint32_t qk[W];
    if (MODE == kModeP16) {
#pragma unroll
      for (int k = 0; k < W; ++k) qk[k] = w.spk[int64_t(q) * W + k];
    }
    uint32_t count = 0;
    for (int rb = r_lo; rb < r_hi; rb += kWave) {
      uint32_t sb = 0, se = 0;
      if (rb + lane < r_hi) window_row<D>(p, g, K, rb + lane, clip2, w.cnt, &sb, &se);
      const int nr = min(kWave, r_hi - rb);
      for (int r = 0; r < nr; ++r) {
        const uint32_t b = __builtin_amdgcn_readlane(sb, r);
        const uint32_t e = __builtin_amdgcn_readlane(se, r);
        work += uint64_t(e - b) * (qe - qb);
        uint32_t j = b;
        if (MODE == kModeP16) {
          // B candidates per batch: one scalar load per 16 words.  (Double
          // buffering the loads needs half-size batches for the SGPRs and was
          // measured slower; 8 resident waves per SIMD hide the latency.)
          constexpr int B = 16 / W;
          for (; j + B <= e; j += B) {
            DPC_CONST(uint32_t) *cb = spk + int64_t(j) * W;
            uint32_t c[B * W];
#pragma unroll
            for (int u = 0; u < B * W; ++u) c[u] = cb[u];
#pragma unroll
            for (int u = 0; u < B; ++u) {
              int32_t acc = dot2_self_s(pk_sub16(qk[0], c[u * W]), negR);
#pragma unroll
              for (int k = 1; k < W; ++k) acc = dot2_self_v(pk_sub16(qk[k], c[u * W + k]), acc);
              count += uint32_t(acc) >> 31;
            }
          }
          for (; j < e; ++j) {
            int32_t acc = dot2_self_s(pk_sub16(qk[0], spk[int64_t(j) * W]), negR);
#pragma unroll
            for (int k = 1; k < W; ++k) acc = dot2_self_v(pk_sub16(qk[k], spk[int64_t(j) * W + k]), acc);
            count += uint32_t(acc) >> 31;
          }
        } else {
          for (; j < e; ++j) {
            int64_t d2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
              const int64_t df = int64_t(qx[k] - spc[int64_t(j) * D + k]);
              d2 += df * df;
            }
            count += d2 < p.R ? 1u : 0u;
          }
        }
      }
    }
    // Lanes past the end of the task repeat its last query: they store the same
    // value, so no lane-divergent branch surrounds the store.
    w.sK[q] = (uint64_t(count) << 32) | uint32_t(~uint32_t(w.sid[q]));
  }
  if (p.count_work) add_work(w.hdr, kWorkDensity, lane == 0 ? work : 0);
}


// One query per lane: the cells within K0 of the query's own cell, clipped to
// its ball row by row (a row farther than d_cut is skipped; in the strip
// dimension a cell is kept when its nearest coordinate is within d_cut).
template <int D, int MODE>
__device__ __forceinline__ void density_lanes(Blk blk, const Plan &p, const Ws &w) {
  constexpr int W = (D + 1) / 2;
  const int32_t negR = -int32_t(p.R < INT32_MAX ? p.R : INT32_MAX);
  const int64_t R1 = p.R - 1;  // D2 <= R - 1 is inside the ball
  const int K = p.K0;
  const int nrow = int(window_rows(p, K));
  __shared__ uint2 queue_all[kWalkQueue * kBlock];  // each lane's queue of row ranges
  uint2 *queue = queue_all + threadIdx.x;
  uint64_t work = 0;  // the lane's candidate tests (profiling)
  for (int64_t q = thread_index(blk); q < p.n; q += grid_threads(blk)) {
    LaneGeom<D> g;
    lane_geom<D>(p, w.spts + q * D, g);
    uint32_t qk[W];
    if (MODE == kModeP16) {
#pragma unroll
      for (int k = 0; k < W; ++k) qk[k] = w.spk[q * W + k];
    }
    uint32_t count = 0;
    // one candidate: inside the ball or not
    auto test = [&](uint32_t j, bool take) {
      if (MODE == kModeP16) {
        uint32_t cw[W];
        load_words<W>(w.spk + int64_t(j) * W, cw);
        int32_t acc = dot2_self_v(pk_sub16(qk[0], cw[0]), negR);
#pragma unroll
        for (int k = 1; k < W; ++k) acc = dot2_self_v(pk_sub16(qk[k], cw[k]), acc);
        count += take ? uint32_t(acc) >> 31 : 0u;
      } else {
        int64_t d2 = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const int64_t df = int64_t(g.x[k] - w.spts[int64_t(j) * D + k]);
          d2 += df * df;
        }
        count += (take && d2 <= R1) ? 1u : 0u;
      }
    };
    bool done = false;
    if constexpr (D <= 4) {
      if (K == 1 && p.gm == D) {  // compile-time rows (3^(D-1) of them)
        if (MODE == kModeP16)
          work += walk_k1<D, uint32_t, true>(p, g, w.cnt, queue, [&]() { return uint32_t(R1); }, test);
        else
          work += walk_k1<D, int64_t, true>(p, g, w.cnt, queue, [&]() { return R1; }, test);
        done = true;
      }
    }
    if (!done) {
      RowWalk<D> rw(K, false);
      for (int r0 = 0; r0 < nrow; r0 += kLaneRowChunk) {
        // cell ranges of the chunk's rows first (independent loads), then their candidates
        uint32_t bb[kLaneRowChunk], ee[kLaneRowChunk];
#pragma unroll
        for (int c = 0; c < kLaneRowChunk; ++c) {
          bb[c] = ee[c] = 0;
          if (r0 + c < nrow) lane_row<D>(p, g, rw, K, R1, w.cnt, &bb[c], &ee[c]);
          rw.next(p, K);
        }
#pragma unroll
        for (int c = 0; c < kLaneRowChunk; ++c) {
          work += ee[c] - bb[c];
          for (uint32_t j = bb[c]; j < ee[c]; ++j) test(j, true);
        }
      }
    }
    const uint64_t key = (uint64_t(count) << 32) | uint32_t(~uint32_t(w.sid[q]));
    w.sK[q] = key;
    if (MODE == kModeP16 && W <= 2 && w.srec)
      w.srec[q] = make_uint4(qk[0], W == 2 ? qk[W - 1] : 0u, uint32_t(key), uint32_t(key >> 32));
  }
  if (p.count_work) add_work(w.hdr, kWorkDensity, work);
}

// The caller's rho in id order: each id reads its cell-order position's key.
__device__ __forceinline__ void rho_out(Blk blk, const Plan &p, const Ws &w, int32_t *__restrict__ rho) {
  for (int64_t i = thread_index(blk); i < p.n; i += grid_threads(blk)) rho[i] = int32_t(w.sK[w.key[i]] >> 32);
}

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_density(Plan p, Ws w) {
  density_body<D, MODE>(grid_blk(), p, w);
}

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) DPC_WAVES(DPC_DENSITY_WAVES) void k_density_lanes(Plan p, Ws w) {
  density_lanes<D, MODE>(xcd_blk(), p, w);
}

__global__ __launch_bounds__(kBlock) void k_rho_out(Plan p, Ws w, int32_t *rho) { rho_out(grid_blk(), p, w, rho); }

// Many-job form: the jobs of one dimension, each on its own virtual blocks.
template <int D>
__global__ __launch_bounds__(kBlock) void kb_density(const JobDev *jobs, VMap m) {
  for (uint32_t v = m.v0 + blockIdx.x; v < m.v1; v += gridDim.x) {
    const uint32_t j = vjob_of(m, v);
    const Blk k = vblk_of(m, v, j);
    const Plan p = load_uniform(&jobs[j].p);
    const Ws w = load_uniform(&jobs[j].w);
    if (p.lanes) {
      if (p.mode == kModeP16)
        density_lanes<D, kModeP16>(k, p, w);
      else
        density_lanes<D, kModeI64>(k, p, w);
    } else if (p.mode == kModeP16) {
      density_body<D, kModeP16>(k, p, w);
    } else {
      density_body<D, kModeI64>(k, p, w);
    }
  }
}

template <int D>
hipError_t launch_d(const Plan &p, const Ws &w, hipStream_t s) {
  if (p.lanes) {
    const unsigned blocks = blocks_for(p.n, kBlock);
    if (p.mode == kModeP16)
      DPC_LAUNCH((k_density_lanes<D, kModeP16>), blocks, kBlock, s, p, w);
    else
      DPC_LAUNCH((k_density_lanes<D, kModeI64>), blocks, kBlock, s, p, w);
    return hipGetLastError();
  }
  const unsigned blocks = persistent_blocks(p.max_tasks);
  if (p.mode == kModeP16)
    DPC_LAUNCH((k_density<D, kModeP16>), blocks, kBlock, s, p, w);
  else
    DPC_LAUNCH((k_density<D, kModeI64>), blocks, kBlock, s, p, w);
  return hipGetLastError();
}

}  // namespace

unsigned persistent_blocks(int64_t max_items) {
  // One wave per item up to kGridCap blocks, 16 times the 2048 workgroups of 4
  // waves that the 256 CUs hold at once (fewer when there is less work).  Work
  // per item varies several-fold (a task's window holds tens to thousands of
  // candidates), and a grid larger than the resident set lets the hardware
  // dispatcher start a new workgroup wherever one has finished: a dynamic
  // balance with no shared counter.
  int64_t waves = max_items < 1 ? 1 : max_items;
  int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  return static_cast<unsigned>(blocks < kGridCap ? blocks : kGridCap);
}

hipError_t launch_density(const Plan &p, const Ws &w, hipStream_t s) {
  switch (p.d) {
    case 1: return launch_d<1>(p, w, s);
    case 2: return launch_d<2>(p, w, s);
    case 3: return launch_d<3>(p, w, s);
    case 4: return launch_d<4>(p, w, s);
    case 5: return launch_d<5>(p, w, s);
    case 6: return launch_d<6>(p, w, s);
    case 7: return launch_d<7>(p, w, s);
    case 8: return launch_d<8>(p, w, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t write_rho(const Plan &p, const Ws &w, int32_t *rho, hipStream_t s) {
  DPC_LAUNCH((k_rho_out), blocks_for(p.n, kBlock), kBlock, s, p, w, rho);
  return hipGetLastError();
}

hipError_t batch_density(const BatchMaps &B, hipStream_t s) {
  for (int g = 0; g < B.ngroups; ++g) {
    VMap m = B.work;
    m.v0 = B.gwork0[g];
    m.v1 = B.gwork1[g];
    if (!vgrid(m)) continue;
    switch (B.gdim[g]) {
      case 1: DPC_LAUNCH((kb_density<1>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 2: DPC_LAUNCH((kb_density<2>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 3: DPC_LAUNCH((kb_density<3>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 4: DPC_LAUNCH((kb_density<4>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 5: DPC_LAUNCH((kb_density<5>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 6: DPC_LAUNCH((kb_density<6>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 7: DPC_LAUNCH((kb_density<7>), vgrid(m), kBlock, s, B.jobs, m); break;
      case 8: DPC_LAUNCH((kb_density<8>), vgrid(m), kBlock, s, B.jobs, m); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace dpc
