// Local density (Def. 1, Eq. 1): rho_i = #{ j : D2(i, j) < R }, the point itself
// included, R = ceil(d_cut^2).
//
// One wave per task (64 queries, one per lane).  The wave walks its window's
// candidate runs with scalar loads, so every candidate reaches all 64 lanes as a
// scalar operand; no LDS, no barriers.  Tasks are handed out by a global work
// counter, so the cost spread between dense and sparse cells balances
// dynamically (the paper's dynamic per-point scheduling, Section 3, in
// wave-sized units).  Waves take tasks in a static interleave (see wave_index).
#include "tasks.h"

namespace dpc {
namespace {

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_density(Plan p, Ws w, int32_t *__restrict__ rho) {
  constexpr int W = (D + 1) / 2;
  const int lane = lane_id();
  DPC_CONST(uint32_t) *spk = as_const(w.spk);
  DPC_CONST(int32_t) *spc = as_const(w.spts);
  DPC_CONST(uint32_t) *start = as_const(w.cnt);
  const uint32_t ntasks = uniform(as_const(&w.hdr->ntasks)[0]);
  const int32_t negR = -int32_t(p.R < INT32_MAX ? p.R : INT32_MAX);

  const uint32_t nw = grid_waves();
  for (uint32_t t = wave_index(); t < ntasks; t += nw) {
    const TaskGeom<D> g = decode_task<D>(p, w.tasks, w.spts, t);
    const uint32_t q = min(g.qb + uint32_t(lane), g.qe - 1u);
    uint32_t qk[W];
    int32_t qx[D];
    if (MODE == kModeP16) {
#pragma unroll
      for (int k = 0; k < W; ++k) qk[k] = w.spk[int64_t(q) * W + k];
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) qx[k] = w.spts[int64_t(q) * D + k];
    }
    uint32_t count = 0;
    constexpr int NROW = Pow3<D - 1>::value;
    for (int rb = 0; rb < NROW; rb += kWave) {
      uint32_t sb = 0, se = 0;
      if (rb + lane < NROW) window_row<D>(p, g, rb + lane, w.cnt, &sb, &se);
      const int nr = min(kWave, NROW - rb);
      for (int r = 0; r < nr; ++r) {
        const uint32_t b = __builtin_amdgcn_readlane(sb, r);
        const uint32_t e = __builtin_amdgcn_readlane(se, r);
        uint32_t j = b;
        if (MODE == kModeP16) {
          constexpr int B = 16 / W;
          for (; j + B <= e; j += B) {
            uint32_t c[B * W];
#pragma unroll
            for (int u = 0; u < B * W; ++u) c[u] = spk[int64_t(j) * W + u];
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
    // Lanes past the end of the task repeat its last query, so they store the
    // same values to the same places: no lane-divergent branch in the loop.
    const int32_t id = w.sid[q];
    rho[id] = int32_t(count);
    w.sK[q] = (uint64_t(count) << 32) | uint32_t(~uint32_t(id));
  }
}

template <int D>
hipError_t launch_d(const Plan &p, const Ws &w, int32_t *rho, hipStream_t s, unsigned blocks) {
  if (p.mode == kModeP16)
    DPC_LAUNCH((k_density<D, kModeP16>), blocks, kBlock, s, p, w, rho);
  else
    DPC_LAUNCH((k_density<D, kModeI64>), blocks, kBlock, s, p, w, rho);
  return hipGetLastError();
}

}  // namespace

unsigned persistent_blocks(int64_t max_items) {
  // 256 CUs x 8 resident workgroups of 4 waves; fewer when there is less work.
  int64_t waves = max_items < 1 ? 1 : max_items;
  int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  const int64_t cap = 256 * 8;
  return static_cast<unsigned>(blocks < cap ? blocks : cap);
}

hipError_t launch_density(const Plan &p, const Ws &w, int32_t *rho, hipStream_t s) {
  const unsigned blocks = persistent_blocks(p.max_tasks);
  switch (p.d) {
    case 1: return launch_d<1>(p, w, rho, s, blocks);
    case 2: return launch_d<2>(p, w, rho, s, blocks);
    case 3: return launch_d<3>(p, w, rho, s, blocks);
    case 4: return launch_d<4>(p, w, rho, s, blocks);
    case 5: return launch_d<5>(p, w, rho, s, blocks);
    case 6: return launch_d<6>(p, w, rho, s, blocks);
    case 7: return launch_d<7>(p, w, rho, s, blocks);
    case 8: return launch_d<8>(p, w, rho, s, blocks);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpc
