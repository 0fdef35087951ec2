// Noise, cluster centers and labels (Defs. 4-6).
//
// Every non-noise point that is not a center points at its dependent point; a
// center points at itself (the paper takes a center's dependent point to be
// itself, Section 2.1).  The dependent point always ranks higher, so the links
// form a forest whose roots are the centers, and a point's label is its root.
// The paper propagates labels by depth-first search from the centers (Section
// 2.2, step 4); here two rounds of in-place pointer jumping shorten the chains
// and a final pass follows each chain to its root.
#include "common.h"

namespace dpc {
namespace {

__device__ __forceinline__ bool ranks_above(int32_t rho_j, int32_t j, int32_t rho_i, int32_t i) {
  return rho_j > rho_i || (rho_j == rho_i && j < i);
}

// parent = -1 (noise), self (center) or dep.  A dep that does not rank above the
// point (inputs not produced by dpc_dependent) is cut and flagged, which keeps
// every chain finite.
__global__ void k_label_init(int64_t n, const int32_t *__restrict__ rho, const int32_t *__restrict__ dep,
                             const double *__restrict__ delta, int32_t rho_min, double delta_min,
                             int32_t *__restrict__ parent, unsigned long long *__restrict__ ncenters,
                             DevHeader *__restrict__ hdr) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool center = false;
  if (i < n) {
    const int32_t r = rho[i];
    const bool noise = r < rho_min;
    center = !noise && delta[i] >= delta_min;
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
  }
  const uint64_t m = __ballot(center);
  if (lane_id() == 0 && m) atomicAdd(ncenters, static_cast<unsigned long long>(__popcll(m)));
}

__global__ void k_zero_count(unsigned long long *c) {
  if (threadIdx.x == 0) *c = 0;
}

// One round of in-place pointer jumping: parent[i] <- parent[parent[i]].  Reads
// racing with writes see either value, both ancestors of i, so the result is the
// same forest with shorter chains.
__global__ void k_jump(int64_t n, int32_t *parent) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = parent[i];
  if (a < 0 || a == i) return;
  const int32_t b = parent[a];
  if (b != a) parent[i] = b < 0 ? -1 : b;
}

// Follow each chain to its root: a center (self-parent) or a cut link (-1).
// Parents rank strictly above their children, so every walk ends.
__global__ void k_root(int64_t n, int32_t *parent) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t a = parent[i];
  if (a < 0 || a == i) return;
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

}  // namespace

hipError_t launch_label(int64_t n, const int32_t *rho, const int32_t *dep, const double *delta,
                        int32_t rho_min, double delta_min, int32_t *label, int64_t *ncenters,
                        DevHeader *hdr, hipStream_t s) {
  unsigned long long *nc = reinterpret_cast<unsigned long long *>(ncenters);
  DPC_LAUNCH((k_zero_count), 1, kWave, s, nc);
  const unsigned blocks = blocks_for(n, kBlock);
  DPC_LAUNCH((k_label_init), blocks, kBlock, s, n, rho, dep, delta, rho_min, delta_min, label, nc, hdr);
  DPC_LAUNCH((k_jump), blocks, kBlock, s, n, label);
  DPC_LAUNCH((k_jump), blocks, kBlock, s, n, label);
  DPC_LAUNCH((k_root), blocks, kBlock, s, n, label);
  return hipGetLastError();
}

}  // namespace dpc
