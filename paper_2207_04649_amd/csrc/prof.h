// Optional per-kernel timing with HIP events on the launching stream (off by
// default; dpc_profile_enable turns it on, dpc_profile_report reads and resets it).
#pragma once

#include <hip/hip_runtime.h>

namespace dpc {

enum ProfKernel : int {
  kProfGrid = 0,   // cell keys, scans, scatter, strips and tasks
  kProfDensity,
  kProfRankKeys,
  kProfRankSort,
  kProfSearch,
  kProfOpen,       // the second window stage over the open points (lane form)
  kProfRingK,
  kProfPeaks,
  kProfFinish,
  kProfLabel,
  kProfApprox,     // Approx-DPC's second grid and approximation rules
  kProfCount
};

bool prof_on();
void prof_mark(hipStream_t s, int kernel, bool begin);

// Records a begin event now and an end event when it goes out of scope.
struct ProfScope {
  hipStream_t s;
  int k;
  bool on;
  ProfScope(hipStream_t s_, int k_) : s(s_), k(k_), on(prof_on()) {
    if (on) prof_mark(s, k, true);
  }
  ~ProfScope() {
    if (on) prof_mark(s, k, false);
  }
};

}  // namespace dpc
