// Kernel-class timing hooks (see profile.hip).
#pragma once

#include "common.h"

namespace mlpcp {

enum KernelClass {
  KC_INIT = 0,
  KC_GRAM,
  KC_COARSE,
  KC_JACOBI_PAIRS,
  KC_JACOBI_APPLY,
  KC_JACOBI_MISC,
  KC_SVT,
  KC_EPILOGUE,
  KC_REDUCE,
  KC_FINAL,
  KC_COARSE_SMALL,
  KC_FW_PASS,
  KC_FW_POWER,
  KC_FW_SMALL,
  KC_FW_TOP,
  KC_MSVT,
  KC_RECON,
  KC_OTHER,
  KC_COUNT
};

void prof_begin(int cls, hipStream_t s);
void prof_end(int cls, hipStream_t s);
void prof_drain();

// RAII helper: times the launches issued in its scope as one kernel class.
struct ProfScope {
  int cls;
  hipStream_t s;
  ProfScope(int c, hipStream_t st) : cls(c), s(st) { prof_begin(cls, s); }
  ~ProfScope() { prof_end(cls, s); }
};

// Events for one kernel of class cls launched by hipExtLaunchKernelGGL, which records
// them at the kernel's own start and end (the dispatch gap that events recorded
// around a launch take in stays out); both null when the class is not being timed.
struct ProfKernel {
  int cls;
  hipEvent_t start = nullptr, stop = nullptr;
  explicit ProfKernel(int c);
  ~ProfKernel();   // queues the pair for accumulation
};

}  // namespace mlpcp
