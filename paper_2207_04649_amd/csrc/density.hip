// Local density (Def. 1, Eq. 1): rho_i = #{ j : D2(i, j) < R }, the point itself
// included, R = ceil(d_cut^2).
//
// One wave per task (64 queries, one per lane).  The window holds the cells
// within K0 of the task's cells (K0 * L >= floor(sqrt(R - 1)), so it covers every
// d_cut-ball) and is clipped to the balls' union row by row.  The wave walks its
// candidate runs with scalar loads, so every candidate reaches all 64 lanes as a
// scalar operand: no LDS, no barriers.
//
// Work units are (task, part of its window rows): a dense task's window holds
// thousands of candidates, so whole tasks leave a few waves with several times
// the average work.  With more than one part per task, every part adds its
// counts into rho with an atomic add (rho cleared first); with one, the count is
// stored.  Waves take units in a static interleave (see wave_index); the paper
// balances the per-point range searches with dynamic OpenMP scheduling
// (Section 3), the interleave does it in these smaller units.
#include "tasks.h"

namespace dpc {
namespace {

template <int D, int MODE>
__device__ __forceinline__ void density_body(Blk blk, const Plan &p, const Ws &w, int32_t *__restrict__ rho) {
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

  const uint32_t parts = uint32_t(p.row_split);
  const int rows_per = (nrow + int(parts) - 1) / int(parts);
  const uint64_t units = uint64_t(ntasks) * parts;

  const uint32_t nw = grid_waves(blk);
  for (uint64_t u = wave_index(blk); u < units; u += nw) {
    const uint32_t t = uint32_t(u / parts);
    const int r_lo = int(u % parts) * rows_per;
    const int r_hi = min(nrow, r_lo + rows_per);
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
    // value, or add 0, so no lane-divergent branch surrounds the store.
    const int32_t id = w.sid[q];
    if (parts == 1)
      rho[id] = int32_t(count);
    else
      atomicAdd(&rho[id], qb + uint32_t(lane) < qe ? int32_t(count) : 0);
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t *__restrict__ v, int64_t n) {
  for (int64_t i = thread_index(grid_blk()); i < n; i += grid_threads(grid_blk())) v[i] = 0;
}

// rho of every job that splits its density tasks, cleared for the atomic adds.
__global__ __launch_bounds__(kBlock) void kb_zero_rho(const JobDev *jobs, VMap m) {
  for (uint32_t v = m.v0 + blockIdx.x; v < m.v1; v += gridDim.x) {
    const uint32_t j = vjob_of(m, v);
    const Blk k = vblk_of(m, v, j);
    if (uniform(int32_t(as_const(jobs)[j].p.row_split)) > 1) {
      const int64_t n = as_const(jobs)[j].p.n;
      int32_t *rho = as_const(jobs)[j].rho;
      for (int64_t i = thread_index(k); i < n; i += grid_threads(k)) rho[i] = 0;
    }
  }
}

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_density(Plan p, Ws w, int32_t *__restrict__ rho) {
  density_body<D, MODE>(grid_blk(), p, w, rho);
}

// Many-job form: the jobs of one dimension, each on its own virtual blocks.
template <int D>
__global__ __launch_bounds__(kBlock) void kb_density(const JobDev *jobs, VMap m) {
  for (uint32_t v = m.v0 + blockIdx.x; v < m.v1; v += gridDim.x) {
    const uint32_t j = vjob_of(m, v);
    const Blk k = vblk_of(m, v, j);
    const Plan p = load_uniform(&jobs[j].p);
    const Ws w = load_uniform(&jobs[j].w);
    int32_t *rho = as_const(jobs)[j].rho;
    if (p.mode == kModeP16)
      density_body<D, kModeP16>(k, p, w, rho);
    else
      density_body<D, kModeI64>(k, p, w, rho);
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

hipError_t launch_density(const Plan &p, const Ws &w, int32_t *rho, hipStream_t s) {
  if (p.row_split > 1) DPC_LAUNCH((k_zero_i32), blocks_for(p.n, kBlock * 4), kBlock, s, rho, p.n);
  const unsigned blocks = persistent_blocks(p.max_tasks * p.row_split);
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

hipError_t batch_density(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.pts)) DPC_LAUNCH((kb_zero_rho), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
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
