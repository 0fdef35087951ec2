// Noise, cluster centers and labels (Defs. 4-6).
//
// Every non-noise point that is not a center points at its dependent point; a
// center points at itself (the paper takes a center's dependent point to be
// itself, Section 2.1).  The dependent point always ranks higher, so the links
// form a forest whose roots are the centers, and a point's label is its root.
// The paper propagates labels by depth-first search from the centers (Section
// 2.2, step 4); here three rounds of in-place pointer jumping shorten the chains
// and a final pass follows each chain to its root.
#include "common.h"

namespace dpc {
namespace {

__device__ __forceinline__ bool ranks_above(int32_t rho_j, int32_t j, int32_t rho_i, int32_t i) {
  return rho_j > rho_i || (rho_j == rho_i && j < i);
}

// parent = -1 (noise), self (center) or dep.  A dep that does not rank above the
// point (inputs not produced by dpc_dependent) is cut and flagged, which keeps
// every chain finite.  Each lane counts its centers; after the loop one lane of
// each wave adds the wave's total (a plain if-region: no loop depends on it).
__device__ __forceinline__ void label_init(Blk k, int64_t n, const int32_t *__restrict__ rho,
                                           const int32_t *__restrict__ dep, const double *__restrict__ delta,
                                           int32_t rho_min, double delta_min, int32_t *__restrict__ parent,
                                           unsigned long long *__restrict__ ncenters, DevHeader *__restrict__ hdr) {
  uint32_t centers = 0;
  for (int64_t i = thread_index(k); i < n; i += grid_threads(k)) {
    const int32_t r = rho[i];
    const bool noise = r < rho_min;
    const bool center = !noise && delta[i] >= delta_min;
    int32_t par = -1;
    if (center) {
      par = int32_t(i);
    } else if (!noise) {
      const int32_t q = dep[i];
      if (q >= 0 && q < n && ranks_above(rho[q], q, r, int32_t(i))) {
        par = q;
      } else {
        atomicOr(&hdr->status, 2u);
      }
    }
    parent[i] = par;
    centers += center ? 1u : 0u;
  }
  const uint32_t total = uniform(wave_sum_u32(centers));
  if (lane_id() == 0 && total != 0) atomicAdd(ncenters, static_cast<unsigned long long>(total));
}

// One round of in-place pointer jumping: parent[i] <- parent[parent[i]].  Reads
// racing with writes see either value, both ancestors of i, so the result is the
// same forest with shorter chains.
__device__ __forceinline__ void jump(Blk k, int64_t n, int32_t *parent) {
  for (int64_t i = thread_index(k); i < n; i += grid_threads(k)) {
    const int32_t a = parent[i];
    if (a < 0 || a == i) continue;
    const int32_t b = parent[a];
    if (b != a) parent[i] = b < 0 ? -1 : b;
  }
}

// Follow each chain to its root: a center (self-parent) or a cut link (-1).
// Parents rank strictly above their children, so every walk ends.
__device__ __forceinline__ void root(Blk k, int64_t n, int32_t *parent) {
  for (int64_t i = thread_index(k); i < n; i += grid_threads(k)) {
    int32_t a = parent[i];
    if (a < 0 || a == i) continue;
    for (;;) {
      const int32_t b = parent[a];
      if (b < 0) {
        a = -1;
        break;
      }
      if (b == a) break;
      a = b;
    }
    parent[i] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_label_init(int64_t n, const int32_t *rho, const int32_t *dep,
                                                       const double *delta, int32_t rho_min, double delta_min,
                                                       int32_t *parent, unsigned long long *ncenters,
                                                       DevHeader *hdr) {
  label_init(grid_blk(), n, rho, dep, delta, rho_min, delta_min, parent, ncenters, hdr);
}

__global__ void k_zero_count(unsigned long long *c) {
  if (threadIdx.x == 0) *c = 0;
}

__global__ __launch_bounds__(kBlock) void k_jump(int64_t n, int32_t *parent) { jump(grid_blk(), n, parent); }
__global__ __launch_bounds__(kBlock) void k_root(int64_t n, int32_t *parent) { root(grid_blk(), n, parent); }

// Many-job forms over the jobs' own rho, dep, delta, thresholds and outputs.
__global__ __launch_bounds__(kBlock) void kb_zero_count(const JobDev *jobs, VMap m) {
  for (uint32_t v = m.v0 + blockIdx.x; v < m.v1; v += gridDim.x) {
    const uint32_t j = vjob_of(m, v);
    if (threadIdx.x == 0) *reinterpret_cast<unsigned long long *>(as_const(jobs)[j].ncenters) = 0;
  }
}

template <int STEP>  // 0: init, 1: jump, 2: root
__global__ __launch_bounds__(kBlock) void kb_label(const JobDev *jobs, VMap m) {
  for (uint32_t v = m.v0 + blockIdx.x; v < m.v1; v += gridDim.x) {
    const uint32_t j = vjob_of(m, v);
    const Blk k = vblk_of(m, v, j);
    const int64_t n = as_const(jobs)[j].p.n;
    int32_t *label = as_const(jobs)[j].label;
    if (STEP == 0)
      label_init(k, n, as_const(jobs)[j].rho, as_const(jobs)[j].dep, as_const(jobs)[j].delta,
                 as_const(jobs)[j].rho_min, as_const(jobs)[j].delta_min, label,
                 reinterpret_cast<unsigned long long *>(as_const(jobs)[j].ncenters), as_const(jobs)[j].w.hdr);
    else if (STEP == 1)
      jump(k, n, label);
    else
      root(k, n, label);
  }
}

}  // namespace

hipError_t launch_label(int64_t n, const int32_t *rho, const int32_t *dep, const double *delta,
                        int32_t rho_min, double delta_min, int32_t *label, int64_t *ncenters,
                        DevHeader *hdr, hipStream_t s) {
  unsigned long long *nc = reinterpret_cast<unsigned long long *>(ncenters);
  DPC_LAUNCH((k_zero_count), 1, kWave, s, nc);
  const unsigned blocks = blocks_for(n, kBlock);
  DPC_LAUNCH((k_label_init), blocks, kBlock, s, n, rho, dep, delta, rho_min, delta_min, label, nc, hdr);
  constexpr int kJumps = 3;  // then the root walk follows the (short) remaining chains
  for (int k = 0; k < kJumps; ++k) DPC_LAUNCH((k_jump), blocks, kBlock, s, n, label);
  DPC_LAUNCH((k_root), blocks, kBlock, s, n, label);
  return hipGetLastError();
}

hipError_t batch_label(const BatchMaps &B, hipStream_t s) {
  if (vgrid(B.one)) DPC_LAUNCH((kb_zero_count), vgrid(B.one), kBlock, s, B.jobs, B.one);
  if (vgrid(B.pts)) {
    DPC_LAUNCH((kb_label<0>), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
    DPC_LAUNCH((kb_label<1>), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
    DPC_LAUNCH((kb_label<1>), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
    DPC_LAUNCH((kb_label<2>), vgrid(B.pts), kBlock, s, B.jobs, B.pts);
  }
  return hipGetLastError();
}

}  // namespace dpc
