// ntt_internal.hpp -- host-side plan object and helpers shared by the library's
// translation units (never exposed through the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "../../include/ntt.h"
#include "modarith.hpp"

struct ntt_plan_s {
  int device = 0;
  uint32_t N = 0, log_n = 0, L = 0, word_bits = 0, flags = 0;
  uint32_t log_n1 = 0;                // column stages (0: single pass)
  std::vector<uint64_t> moduli, psi;
  std::vector<uint32_t> cls;          // arithmetic class per limb
  nttk::LimbDev* d_limbs = nullptr;   // device [L]
  void* d_tables = nullptr;           // device twiddle tables
  uint32_t* d_cls_limbs = nullptr;    // device limb lists, concatenated per class
  uint32_t cls_off[3] = {0, 0, 0};
  uint32_t cls_cnt[3] = {0, 0, 0};
};

namespace nttk {

ntt_status fail(ntt_status st, const char* fmt, ...);
ntt_status hip_fail(hipError_t e, const char* what);

// Split chosen by the tuning cache for this shape, or `fallback`.
uint32_t tuned_split(uint32_t N, uint32_t L, uint32_t word_bits, uint32_t fallback);

}  // namespace nttk
