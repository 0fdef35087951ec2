// Decision-graph summaries (Section 2.1): the <rho, delta> pairs a user reads to
// choose rho_min and delta_min, computed on the device from resident outputs.
//
// Top-k by delta.  Each non-noise point gets a 96-bit key: the bits of its delta
// (a non-negative double, whose bit pattern orders as its value, +inf highest),
// then 2^32 - 1 - id, so that larger keys are larger deltas and, among equal
// deltas, smaller ids.  A radix select over eight 12-bit digits, most significant
// first, finds the k-th largest key T: each pass counts the digit of the keys that
// match the digits decided so far (an LDS histogram per block, 4096 bins), and one
// block picks the digit where the running count from the top reaches the number
// still needed.  Keys are distinct, so exactly min(k, eligible) keys are >= T;
// they are gathered and sorted by one block (bitonic sort in LDS).
//
// Histogram.  Each point finds its bin on both axes by binary search over the
// caller's edges (half-open bins, the last one closed) and counts into an LDS
// histogram per block when the grid of bins fits, else straight into HBM.
//
// Suggested delta_min.  Over the sorted top list, the consecutive pair with the
// largest ratio delta_j / delta_{j+1} among those with delta_j finite and above
// d_cut; delta_min = delta_j.
#include "common.h"

namespace dpc {
namespace {

constexpr int kDigitBits = 12;
constexpr int kBins = 1 << kDigitBits;
constexpr int kDigits = 96 / kDigitBits;
constexpr int kTopMax = DPC_DECISION_TOP_MAX;
constexpr int kSortThreads = 1024;

struct TopState {
  uint32_t pre[3];   // decided key bits (word 0: least significant 32 bits)
  uint32_t mask[3];  // which bits are decided
  uint32_t need;     // keys still to take among those matching the decided bits
  uint32_t done;     // 1: every matching key is taken (no digit left to decide)
  uint32_t taken;    // candidates gathered
  uint32_t pad[55];
  uint32_t hist[kBins];
  uint64_t cand_key[kTopMax];  // delta bits of each candidate
  uint32_t cand_id[kTopMax];
};
static_assert(sizeof(TopState) <= DPC_DECISION_WS_BYTES, "top-k state fits the documented workspace");

struct Key {
  uint32_t w[3];  // w[2] most significant
};

__device__ __forceinline__ Key make_key(double delta, int64_t id) {
  const uint64_t b = __double_as_longlong(delta);
  return Key{{0xffffffffu - uint32_t(id), uint32_t(b), uint32_t(b >> 32)}};
}

// Digit t (0: most significant) of a key.
__device__ __forceinline__ uint32_t digit(const Key &k, int t) {
  const int s = 96 - kDigitBits * (t + 1);  // lowest bit of the digit
  const int wi = s >> 5, bi = s & 31;
  uint32_t v = k.w[wi] >> bi;
  if (bi + kDigitBits > 32) v |= k.w[wi + 1] << (32 - bi);
  return v & (kBins - 1);
}

__device__ __forceinline__ bool matches(const Key &k, const TopState *st) {
  return ((k.w[0] & st->mask[0]) == st->pre[0]) && ((k.w[1] & st->mask[1]) == st->pre[1]) &&
         ((k.w[2] & st->mask[2]) == st->pre[2]);
}

// k >= threshold (the decided bits, the others zero)
__device__ __forceinline__ bool at_least(const Key &k, const TopState *st) {
  for (int i = 2; i >= 0; --i) {
    if (k.w[i] != st->pre[i]) return k.w[i] > st->pre[i];
  }
  return true;
}

__global__ void k_top_init(TopState *st, uint32_t k) {
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) st->hist[i] = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < 3; ++i) st->pre[i] = st->mask[i] = 0;
    st->need = k;
    st->done = 0;
    st->taken = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_top_hist(int64_t n, const int32_t *__restrict__ rho,
                                                     const double *__restrict__ delta, int32_t rho_min,
                                                     TopState *st, int t) {
  __shared__ uint32_t h[kBins];
  if (st->done) return;  // uniform: written by the previous launch
  for (int i = threadIdx.x; i < kBins; i += kBlock) h[i] = 0;
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    if (rho[i] < rho_min) continue;
    const Key k = make_key(delta[i], i);
    if (matches(k, st)) atomicAdd(&h[digit(k, t)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += kBlock)
    if (h[i]) atomicAdd(&st->hist[i], h[i]);
}

// One block: the digit where the count from the top reaches `need`, then the
// histogram is cleared for the next pass.  When all matching keys are needed the
// selection is complete (done).
__global__ __launch_bounds__(kSortThreads) void k_top_pick(TopState *st, int t) {
  __shared__ uint32_t part[kSortThreads];
  __shared__ uint32_t pick_digit, pick_above;
  constexpr int kPer = kBins / kSortThreads;  // bins per thread, from the top
  if (st->done) return;
  const int tid = threadIdx.x;
  // thread tid holds bins kBins-1-tid*kPer .. down, so that thread order is digit order from the top
  uint32_t c[kPer], sum = 0;
  for (int j = 0; j < kPer; ++j) {
    c[j] = st->hist[kBins - 1 - (tid * kPer + j)];
    sum += c[j];
  }
  part[tid] = sum;
  __syncthreads();
  // inclusive scan of the thread sums (Hillis-Steele in LDS)
  for (int off = 1; off < kSortThreads; off <<= 1) {
    const uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const uint32_t total = part[kSortThreads - 1];
  const uint32_t need = st->need;
  if (tid == 0) pick_digit = kBins;  // none
  __syncthreads();
  if (total > need) {
    uint32_t run = tid ? part[tid - 1] : 0u;  // keys in higher digits than this thread's
    for (int j = 0; j < kPer; ++j) {
      if (run < need && run + c[j] >= need) {
        pick_digit = uint32_t(kBins - 1 - (tid * kPer + j));
        pick_above = run;
      }
      run += c[j];
    }
  }
  __syncthreads();
  for (int i = tid; i < kBins; i += kSortThreads) st->hist[i] = 0;
  if (tid == 0) {
    if (total <= need) {
      st->done = 1;  // every matching key is needed: keys >= the decided prefix
    } else {
      const int s = 96 - kDigitBits * (t + 1);
      const int wi = s >> 5, bi = s & 31;
      const uint32_t v = pick_digit;
      st->pre[wi] |= v << bi;
      st->mask[wi] |= uint32_t(kBins - 1) << bi;
      if (bi + kDigitBits > 32) {
        st->pre[wi + 1] |= v >> (32 - bi);
        st->mask[wi + 1] |= uint32_t(kBins - 1) >> (32 - bi);
      }
      st->need = need - pick_above;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_top_gather(int64_t n, const int32_t *__restrict__ rho,
                                                       const double *__restrict__ delta, int32_t rho_min,
                                                       TopState *st) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    if (rho[i] < rho_min) continue;
    const double dl = delta[i];
    const Key k = make_key(dl, i);
    if (!at_least(k, st)) continue;
    const uint32_t at = atomicAdd(&st->taken, 1u);
    if (at < uint32_t(kTopMax)) {
      st->cand_key[at] = __double_as_longlong(dl);
      st->cand_id[at] = uint32_t(i);
    }
  }
}

// (key, id) a before b in the output order: larger delta first, then smaller id
__device__ __forceinline__ bool before(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(kSortThreads) void k_top_sort(const TopState *st, uint32_t k,
                                                           const int32_t *__restrict__ rho,
                                                           int32_t *__restrict__ ids, double *__restrict__ deltas,
                                                           int32_t *__restrict__ rhos, int64_t *__restrict__ count) {
  __shared__ uint64_t key[kTopMax];
  __shared__ uint32_t id[kTopMax];
  const uint32_t m = min(min(st->taken, k), uint32_t(kTopMax));
  uint32_t size = 1;
  while (size < m) size <<= 1;
  for (uint32_t i = threadIdx.x; i < size; i += kSortThreads) {
    key[i] = i < m ? st->cand_key[i] : 0ull;
    id[i] = i < m ? st->cand_id[i] : 0xffffffffu;  // padding sorts last
  }
  __syncthreads();
  for (uint32_t len = 2; len <= size; len <<= 1) {
    for (uint32_t stride = len >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < size; i += kSortThreads) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & len) == 0;  // this run ascends in output order
          const bool swap = up ? before(key[j], id[j], key[i], id[i]) : before(key[i], id[i], key[j], id[j]);
          if (swap) {
            const uint64_t tk = key[i];
            key[i] = key[j];
            key[j] = tk;
            const uint32_t ti = id[i];
            id[i] = id[j];
            id[j] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < m; i += kSortThreads) {
    ids[i] = int32_t(id[i]);
    deltas[i] = __longlong_as_double(key[i]);
    if (rhos) rhos[i] = rho[id[i]];
  }
  if (threadIdx.x == 0) *count = int64_t(m);
}

// Bin of v: half-open bins [e_i, e_{i+1}), the last one closed; -1 outside.
__device__ __forceinline__ int find_bin(double v, const double *__restrict__ e, int nb) {
  int lo = 0, hi = nb + 1;  // first edge index whose edge > v, in [lo, hi)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (e[mid] > v) hi = mid;
    else lo = mid + 1;
  }
  const int b = lo - 1;
  if (b >= 0 && b < nb) return b;
  if (nb > 0 && v == e[nb]) return nb - 1;
  return -1;
}

constexpr int kHistLds = 8192;  // bins counted in LDS per block (32 KB)

__global__ __launch_bounds__(kBlock) void k_hist(int64_t n, const int32_t *__restrict__ rho,
                                                 const double *__restrict__ delta, const double *__restrict__ re,
                                                 int nr, const double *__restrict__ de, int nd,
                                                 unsigned long long *__restrict__ counts) {
  __shared__ uint32_t h[kHistLds];
  const int nbins = nr * nd;
  const bool lds = nbins <= kHistLds;
  if (lds) {
    for (int i = threadIdx.x; i < nbins; i += kBlock) h[i] = 0;
    __syncthreads();
  }
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const int a = find_bin(double(rho[i]), re, nr);
    if (a < 0) continue;
    const int b = find_bin(delta[i], de, nd);
    if (b < 0) continue;
    if (lds) atomicAdd(&h[a * nd + b], 1u);
    else atomicAdd(&counts[int64_t(a) * nd + b], 1ull);
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += kBlock)
      if (h[i]) atomicAdd(&counts[i], (unsigned long long)h[i]);
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_i64(int64_t *p, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += int64_t(gridDim.x) * kBlock) p[i] = 0;
}

__global__ __launch_bounds__(kSortThreads) void k_suggest(const double *__restrict__ top, const int64_t *count,
                                                          double d_cut, double *delta_min, int64_t *centers) {
  __shared__ double best_r[kSortThreads];
  __shared__ int best_j[kSortThreads];
  __shared__ uint32_t ncent[kSortThreads];
  const int m = int(min(*count, int64_t(kTopMax)));
  double br = -1.0;
  int bj = -1;
  for (int j = threadIdx.x; j + 1 < m; j += kSortThreads) {
    const double a = top[j], b = top[j + 1];
    if (!(a <= __DBL_MAX__ && a > d_cut)) continue;  // finite and above d_cut
    const double r = b == 0.0 ? __builtin_huge_val() : a / b;
    if (r > br) {  // j ascends within a thread: ties keep the first
      br = r;
      bj = j;
    }
  }
  best_r[threadIdx.x] = br;
  best_j[threadIdx.x] = bj;
  __syncthreads();
  for (int off = kSortThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double r2 = best_r[threadIdx.x + off];
      const int j2 = best_j[threadIdx.x + off];
      const double r1 = best_r[threadIdx.x];
      const int j1 = best_j[threadIdx.x];
      if (j2 >= 0 && (j1 < 0 || r2 > r1 || (r2 == r1 && j2 < j1))) {
        best_r[threadIdx.x] = r2;
        best_j[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  const int j = best_j[0];
  const double dmin = j >= 0 ? top[j] : __builtin_nan("");
  uint32_t c = 0;
  if (j >= 0)
    for (int i = threadIdx.x; i < m; i += kSortThreads) c += top[i] >= dmin ? 1u : 0u;
  ncent[threadIdx.x] = c;
  __syncthreads();
  for (int off = kSortThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) ncent[threadIdx.x] += ncent[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *delta_min = dmin;
    *centers = int64_t(ncent[0]);
  }
}

unsigned scan_blocks(int64_t n) {
  const int64_t b = (n + int64_t(kBlock) * 8 - 1) / (int64_t(kBlock) * 8);
  return unsigned(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

}  // namespace

hipError_t launch_decision_top(int64_t n, const int32_t *rho, const double *delta, int32_t rho_min, int32_t k,
                               int32_t *ids, double *deltas, int32_t *rhos, int64_t *count, void *ws,
                               hipStream_t s) {
  TopState *st = static_cast<TopState *>(ws);
  const unsigned nb = scan_blocks(n);
  DPC_LAUNCH((k_top_init), 1, kBlock, s, st, uint32_t(k));
  for (int t = 0; t < kDigits; ++t) {
    DPC_LAUNCH((k_top_hist), nb, kBlock, s, n, rho, delta, rho_min, st, t);
    DPC_LAUNCH((k_top_pick), 1, kSortThreads, s, st, t);
  }
  DPC_LAUNCH((k_top_gather), nb, kBlock, s, n, rho, delta, rho_min, st);
  DPC_LAUNCH((k_top_sort), 1, kSortThreads, s, st, uint32_t(k), rho, ids, deltas, rhos, count);
  return hipGetLastError();
}

hipError_t launch_decision_hist(int64_t n, const int32_t *rho, const double *delta, const double *re, int nr,
                                const double *de, int nd, int64_t *counts, hipStream_t s) {
  const int64_t nbins = int64_t(nr) * nd;
  DPC_LAUNCH((k_zero_i64), blocks_for(nbins, kBlock), kBlock, s, counts, nbins);
  DPC_LAUNCH((k_hist), scan_blocks(n), kBlock, s, n, rho, delta, re, nr, de, nd,
             reinterpret_cast<unsigned long long *>(counts));
  return hipGetLastError();
}

hipError_t launch_decision_suggest(const double *top, const int64_t *count, double d_cut, double *delta_min,
                                   int64_t *centers, hipStream_t s) {
  DPC_LAUNCH((k_suggest), 1, kSortThreads, s, top, count, d_cut, delta_min, centers);
  return hipGetLastError();
}

}  // namespace dpc
