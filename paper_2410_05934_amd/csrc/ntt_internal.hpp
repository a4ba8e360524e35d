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

// Column stages used by polymul.  The fused row kernel holds two operands in
// registers; at 2^14-word rows (1024 threads, at most 128 VGPRs) it would
// spill, so such plans multiply with a 2^13-word row pass instead.
inline uint32_t polymul_split(const ntt_plan_s* p) {
  return (p->log_n1 == 0 && p->log_n == 14) ? 1u : p->log_n1;
}

ntt_status fail(ntt_status st, const char* fmt, ...);
ntt_status hip_fail(hipError_t e, const char* what);

// Per-launch timing (enabled through ntt_stats_enable).  When enabled, the
// launch is bracketed by two events on its own stream.
bool stats_enabled();
class LaunchTimer {
 public:
  LaunchTimer(const char* kind, const char* cls, int size_log, bool inv, bool two_pass,
              uint64_t words, hipStream_t s);
  ~LaunchTimer();
  LaunchTimer(const LaunchTimer&) = delete;
  LaunchTimer& operator=(const LaunchTimer&) = delete;

 private:
  bool on_ = false;
  int slot_ = -1;
  hipStream_t s_ = nullptr;
};

// Split chosen by the tuning cache for this shape, or `fallback`.
uint32_t tuned_split(uint32_t N, uint32_t L, uint32_t word_bits, uint32_t fallback);

}  // namespace nttk
