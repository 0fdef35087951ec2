// CPU stand-in for <hip/hip_runtime.h>, used only to build the library's kernel
// sources as a host program for tests (bounds checking with AddressSanitizer,
// hang and deadlock detection).  Every GPU thread runs as a fiber; a workgroup's
// fibers are scheduled round-robin on one OS thread, and wave-level intrinsics
// (shuffles, ballot, readlane) exchange values through a per-wave rendezvous
// that all live lanes of the wave must reach, as they would in lockstep.  A
// round in which no fiber makes progress is reported as a deadlock.
#pragma once

#include <ucontext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#define DPC_HOST_DOT2 1
#define DPC_CONST(T) const T

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define DPC_WAVES(n)
#define __shared__ static
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };

struct uint4 {
  unsigned x, y, z, w;
};
struct alignas(16) int4 {
  int x, y, z, w;
};
struct alignas(8) uint2 {
  unsigned x, y;
};
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return uint4{x, y, z, w}; }
inline uint2 make_uint2(unsigned x, unsigned y) { return uint2{x, y}; }
inline unsigned __umulhi(unsigned a, unsigned b) { return unsigned((static_cast<unsigned long long>(a) * b) >> 32); }

template <class T>
inline T min(T a, T b) {
  return a < b ? a : b;
}
template <class T>
inline T max(T a, T b) {
  return a < b ? b : a;
}

namespace emu {

constexpr int kWaveLanes = 64;

struct Fiber {
  ucontext_t ctx;
  unsigned tid = 0;
  bool done = false;
};

struct Wave {
  unsigned live = 0;
  unsigned arrived = 0;
  uint64_t gen = 0;
  uint64_t slot[2][kWaveLanes] = {};
  uint64_t present[2] = {0, 0};  // lanes that took part in each rendezvous
};

struct Block {
  unsigned nthreads = 0, live = 0;
  std::vector<Fiber> fibers;
  std::vector<Wave> waves;
  ucontext_t sched;
  int cur = -1;
  unsigned bar_count = 0;
  uint64_t bar_gen = 0;
  uint64_t progress = 0;
  std::function<void()> body;
};

inline Block *&blk() {
  static Block *b = nullptr;
  return b;
}
inline unsigned &block_idx() {
  static unsigned v = 0;
  return v;
}
inline unsigned &grid_dim() {
  static unsigned v = 0;
  return v;
}
inline unsigned &block_dim() {
  static unsigned v = 0;
  return v;
}
inline std::vector<std::vector<char>> &stacks() {
  static std::vector<std::vector<char>> s;
  return s;
}
inline uint64_t &watchdog() {  // rounds without progress before a deadlock is declared
  static uint64_t v = 4;
  return v;
}

inline void yield() {
  Block *b = blk();
  swapcontext(&b->fibers[b->cur].ctx, &b->sched);
}

inline unsigned tid() { return blk()->fibers[blk()->cur].tid; }

inline void trampoline() {
  Block *b = blk();
  b->body();
  Fiber &f = b->fibers[b->cur];
  f.done = true;
  b->live--;
  Wave &w = b->waves[f.tid / kWaveLanes];
  w.live--;
  b->progress++;
  if (w.live && w.arrived == w.live) {  // the rest of the wave waits on this lane
    w.arrived = 0;
    w.gen++;
  }
  if (b->live && b->bar_count == b->live) {
    b->bar_count = 0;
    b->bar_gen++;
  }
  swapcontext(&f.ctx, &b->sched);
}

inline void launch(unsigned grid, unsigned block, const std::function<void()> &body) {
  const size_t stack_bytes = 256 * 1024;
  if (stacks().size() < block) stacks().resize(block);
  for (auto &s : stacks())
    if (s.size() < stack_bytes) s.resize(stack_bytes);
  grid_dim() = grid;
  block_dim() = block;
  for (unsigned bi = 0; bi < grid; ++bi) {
    Block b;
    b.nthreads = b.live = block;
    b.fibers.resize(block);
    b.waves.resize((block + kWaveLanes - 1) / kWaveLanes);
    for (unsigned t = 0; t < block; ++t) b.waves[t / kWaveLanes].live++;
    b.body = body;
    blk() = &b;
    block_idx() = bi;
    for (unsigned t = 0; t < block; ++t) {
      Fiber &f = b.fibers[t];
      f.tid = t;
      getcontext(&f.ctx);
      f.ctx.uc_stack.ss_sp = stacks()[t].data();
      f.ctx.uc_stack.ss_size = stacks()[t].size();
      f.ctx.uc_link = nullptr;
      makecontext(&f.ctx, trampoline, 0);
    }
    uint64_t idle_rounds = 0;
    while (b.live) {
      const uint64_t before = b.progress;
      for (unsigned t = 0; t < block; ++t) {
        if (b.fibers[t].done) continue;
        b.cur = int(t);
        swapcontext(&b.sched, &b.fibers[t].ctx);
      }
      idle_rounds = b.progress == before ? idle_rounds + 1 : 0;
      if (idle_rounds > watchdog()) {
        std::fprintf(stderr, "emu: deadlock in block %u (%u live threads)\n", bi, b.live);
        std::abort();
      }
    }
    blk() = nullptr;
  }
}

// Rendezvous of the live lanes of the calling lane's wave; returns the slot row
// holding every lane's value.
inline const uint64_t *wave_exchange(uint64_t v) {
  Block *b = blk();
  const unsigned t = tid();
  Wave &w = b->waves[t / kWaveLanes];
  const uint64_t my = w.gen;
  if (w.arrived == 0) w.present[my & 1] = 0;
  w.slot[my & 1][t % kWaveLanes] = v;
  w.present[my & 1] |= uint64_t(1) << (t % kWaveLanes);
  if (++w.arrived == w.live) {
    w.arrived = 0;
    w.gen++;
    b->progress++;
  } else {
    while (w.gen == my) yield();
  }
  return w.slot[my & 1];
}

inline unsigned lane() { return tid() % kWaveLanes; }

// Lanes present at the rendezvous whose values `row` holds.
inline uint64_t present_mask(const uint64_t *row) {
  Wave &w = blk()->waves[tid() / kWaveLanes];
  return row == w.slot[0] ? w.present[0] : w.present[1];
}

template <class T>
inline uint64_t bits(T v) {
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <class T>
inline T from_bits(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}

}  // namespace emu

struct emu_dim3 {
  unsigned x;
};
#define threadIdx (emu_dim3{emu::tid()})
#define blockIdx (emu_dim3{emu::block_idx()})
#define blockDim (emu_dim3{emu::block_dim()})
#define gridDim (emu_dim3{emu::grid_dim()})

inline void __syncthreads() {
  emu::Block *b = emu::blk();
  const uint64_t my = b->bar_gen;
  if (++b->bar_count == b->live) {
    b->bar_count = 0;
    b->bar_gen++;
    b->progress++;
  } else {
    while (b->bar_gen == my) emu::yield();
  }
}

template <class T>
inline T __shfl(T v, int src, int width = 64) {
  (void)width;
  return emu::from_bits<T>(emu::wave_exchange(emu::bits(v))[src & 63]);
}
template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  (void)width;
  const uint64_t *s = emu::wave_exchange(emu::bits(v));
  const unsigned l = emu::lane();
  return l >= delta ? emu::from_bits<T>(s[l - delta]) : v;
}
template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  return emu::from_bits<T>(emu::wave_exchange(emu::bits(v))[(emu::lane() ^ unsigned(mask)) & 63]);
}
inline uint64_t __ballot(int pred) {
  const uint64_t *s = emu::wave_exchange(pred ? 1 : 0);
  const uint64_t live = emu::present_mask(s);
  uint64_t m = 0;
  for (unsigned l = 0; l < 64; ++l)
    if (((live >> l) & 1) && s[l]) m |= uint64_t(1) << l;
  return m;
}
template <class T>
inline T emu_readfirstlane(T v) {
  const uint64_t *s = emu::wave_exchange(emu::bits(v));
  return emu::from_bits<T>(s[__builtin_ctzll(emu::present_mask(s))]);
}
template <class T>
inline T emu_readlane(T v, int l) {
  return emu::from_bits<T>(emu::wave_exchange(emu::bits(v))[l & 63]);
}
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane(v)
#define __builtin_amdgcn_readlane(v, l) emu_readlane((v), (l))
// Lanes of a real wave run in lockstep, so LDS written by one lane is visible to
// the others at the next instruction; here the lanes meet at the wave barrier.
#define __builtin_amdgcn_wave_barrier() ((void)emu::wave_exchange(0))
#define __builtin_amdgcn_fence(...) ((void)0)
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline long long __double_as_longlong(double v) {
  long long r;
  std::memcpy(&r, &v, 8);
  return r;
}
inline double __longlong_as_double(long long v) {
  double r;
  std::memcpy(&r, &v, 8);
  return r;
}
inline int __ffsll(long long v) { return __builtin_ffsll(v); }

template <class T>
inline T atomicAdd(T *p, T v) {
  T old = *p;
  *p = old + v;
  return old;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
  unsigned long long old = *p;
  *p = old + v;
  return old;
}
inline unsigned atomicOr(unsigned *p, unsigned v) {
  unsigned old = *p;
  *p = old | v;
  return old;
}
inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v) {
  unsigned long long old = *p;
  if (v < old) *p = v;
  return old;
}
inline unsigned atomicMax(unsigned *p, unsigned v) {
  unsigned old = *p;
  if (v > old) *p = v;
  return old;
}
inline unsigned long long atomicMax(unsigned long long *p, unsigned long long v) {
  unsigned long long old = *p;
  if (v > old) *p = v;
  return old;
}
inline unsigned atomicMin(unsigned *p, unsigned v) {
  unsigned old = *p;
  if (v < old) *p = v;
  return old;
}
inline unsigned atomicCAS(unsigned *p, unsigned cmp, unsigned v) {
  unsigned old = *p;
  if (old == cmp) *p = v;
  return old;
}

// Runtime calls used by the host side of the library: memory is host memory.
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emulated"; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t *e) {
  *e = nullptr;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *t, hipEvent_t, hipEvent_t) {
  *t = 0.f;
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
  *p = const_cast<void *>(sym);
  return hipSuccess;
}

#define DPC_LAUNCH(K, G, B, S, ...) ::emu::launch((G), (B), [&]() { DPC_STRIP K(__VA_ARGS__); })
