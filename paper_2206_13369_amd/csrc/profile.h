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

}  // namespace mlpcp
