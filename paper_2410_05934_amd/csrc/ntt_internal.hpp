// ntt_internal.hpp -- host-side plan object and helpers shared by the library's
// translation units (never exposed through the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "../../include/ntt.h"
#include "modarith.hpp"

namespace nttk {
// A device-resident twiddle table pair (forward, inverse) for one prime and
// arithmetic class, of length 2^log_len; shared by reference count.
struct PrimeTable {
  int device = 0;
  uint64_t q = 0;
  uint32_t cls = 0;
  uint32_t log_len = 0;
  void* mem = nullptr;
  const void* twf = nullptr;
  const void* twi = nullptr;
  int refs = 0;
  size_t bytes = 0;
};
}  // namespace nttk

struct ntt_plan_s {
  int device = 0;
  uint32_t N = 0, log_n = 0, L = 0, word_bits = 0, flags = 0;
  uint32_t log_n1 = 0;                // default column stages (0: single pass)
  int forced_split = -1;              // NTT_FLAG_SPLIT, or -1
  int row_rb = 0;                     // forced log2 values per thread in row passes (0: choose)
  uint32_t col_block = 0;             // forced column-pass workgroup size (0: choose)
  std::vector<uint64_t> moduli, psi;
  std::vector<uint32_t> cls;          // arithmetic class per limb
  nttk::LimbDev* d_limbs = nullptr;   // device [L]
  std::vector<nttk::LimbDev> h_limbs; // host copy of the same constants
  std::vector<const nttk::PrimeTable*> tables;  // shared tables, one per limb
  uint32_t* d_cls_limbs = nullptr;    // device limb lists, concatenated per class
  std::vector<uint32_t> h_cls_limbs;  // host copy of the same lists
  uint32_t cls_off[3] = {0, 0, 0};
  uint32_t cls_cnt[3] = {0, 0, 0};
};

namespace nttk {

// Column stages used by polymul (and forward-and-multiply) for a transform
// split of n1 column stages.  The fused row kernel holds two operands in
// registers and is built for rows of at most 2^13 words (at 2^14-word rows,
// 1024 threads with at most 128 VGPRs, it would spill), so any split whose
// rows would be longer -- the single pass at N = 2^14, or n1 = log2 N - 14 at
// N = 2^15 and 2^16 -- takes just enough column stages for 2^13-word rows.
inline uint32_t polymul_split_log(uint32_t log_n, uint32_t n1) {
  if (n1 == 0) return log_n <= 13 ? 0u : log_n - 13;
  return (log_n > 13 && log_n - n1 > 13) ? log_n - 13 : n1;
}
inline uint32_t polymul_split(const ntt_plan_s* p, uint32_t n1) {
  return polymul_split_log(p->log_n, n1);
}

// Bounded waits of the single-launch form: polls before a wait gives up, and
// the testing switch that makes every wait's target unreachable (set through
// ntt_debug_wait_limit).
uint32_t fused_spin_limit();
bool fused_force_expire();

ntt_status fail(ntt_status st, const char* fmt, ...);
// NTT_FLAG_VALIDATE: check that `polys` polynomials [polys][L][N] at `data` hold
// canonical words (device-side check; waits for the stream).  NTT_OK when the
// plan does not have the flag.
ntt_status validate_words(const ntt_plan_s* p, const void* data, uint64_t polys, hipStream_t s,
                          const char* name);
ntt_status hip_fail(hipError_t e, const char* what);
void clear_error();  // empties the calling thread's last-error message

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

// Shared twiddle tables (twiddles.cpp).
uint32_t table_log_len(uint64_t q);
ntt_status acquire_table(int device, uint64_t q, uint32_t cls, const PrimeTable** out);
void release_table(const PrimeTable* t);
size_t resident_table_bytes();

// Tuning table (tune.cpp).
uint32_t tuned_split_for(uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback);
uint32_t tuned_ragged_row_log(uint32_t log_n, uint32_t fallback);
bool split_valid(int log_n, int n1);

// Values per thread (log2) of row passes: forced by NTT_FLAG_ROW_RADIX8 or
// NTT_FLAG_ROW_RADIX4, else the tuning table, else radix-4 for forward and
// inverse rows of calls in the 64-bit integer class with at most kLatencyChunks
// row chunks, radix-8 for inverse rows, forward rows of 2^10..2^11 words and
// single-pass polymul rows, and radix-16 for the rest.
uint32_t tuned_row_rb(uint32_t kind, uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback);
inline int dominant_class(const ntt_plan_s* p) {
  uint32_t best = 0, cnt = 0;
  for (uint32_t c = 0; c < 3; ++c)
    if (p->cls_cnt[c] > cnt) { cnt = p->cls_cnt[c]; best = c; }
  return (int)best;
}
// Row lengths each radix is built for: radix-16 2^4..2^14, radix-8 2^10..2^13,
// radix-4 2^8..2^12 (at most 1024 threads per chunk).
inline bool row_rb_ok(int rb, int n2) {
  if (rb == 4) return n2 >= 4 && n2 <= 14;
  if (rb == 3) return n2 >= 10 && n2 <= 13;
  if (rb == 2) return n2 >= 8 && n2 <= 12;
  return false;
}
// Up to one row chunk per compute unit, a thread's chain of dependent
// butterflies bounds the pass, not the work per compute unit.  That matters for
// the integer class, whose butterfly is several times longer than the fp64
// ones (measured on one 56-bit prime: N = 2^12 forward 10.3 us with radix-16
// rows, 7.0 us with radix-4; fp64 classes gain nothing).
constexpr uint64_t kLatencyChunks = 256;
inline int row_rb_for(const ntt_plan_s* p, bool inv, uint32_t split, uint32_t batch) {
  const int n2 = (int)p->log_n - (int)split;
  if (p->row_rb) return row_rb_ok(p->row_rb, n2) ? p->row_rb : 4;
  const uint64_t chunks = ((uint64_t)batch * p->L) << split;
  const int cls = dominant_class(p);
  uint32_t fallback = 4;
  if (cls == 2 && chunks <= kLatencyChunks && row_rb_ok(2, n2)) fallback = 2;
  else if ((inv || n2 <= 11) && row_rb_ok(3, n2)) fallback = 3;
  const int rb = (int)tuned_row_rb(inv ? 3u : 2u, p->log_n, (uint32_t)cls, (uint64_t)batch * p->L,
                                   fallback);
  return row_rb_ok(rb, n2) ? rb : 4;
}

// Columns (threads) per workgroup of column passes: forced by the plan (the
// tuner's measurements), else the tuning table, else 256.  One thread per column,
// so this is both the waves per workgroup (1, 2, 4) and the transforms' columns
// a workgroup holds.
uint32_t tuned_col_block(uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback);
inline uint32_t col_block_for(const ntt_plan_s* p, uint32_t batch) {
  if (p->col_block) return p->col_block;
  return tuned_col_block(p->log_n, (uint32_t)dominant_class(p), (uint64_t)batch * p->L, 256u);
}

inline int polymul_rb_for(const ntt_plan_s* p, uint32_t split, uint32_t batch) {
  const int n2 = (int)p->log_n - (int)split;
  if (!row_rb_ok(3, n2)) return 4;
  if (p->row_rb == 3 || p->row_rb == 4) return p->row_rb;
  // measured on 2 x 36 x 2^16: radix-16 rows 46 us, radix-8 52 us (two-pass)
  const uint32_t fallback = split ? 4u : 3u;
  const int rb = (int)tuned_row_rb(4u, p->log_n, (uint32_t)dominant_class(p),
                                   (uint64_t)batch * p->L, fallback);
  return rb == 3 ? 3 : 4;
}

// Single-launch two-pass form (both passes in one persistent launch): for
// splits with 2^12-word rows and 2..16 columns per transform; forced by
// NTT_FLAG_FUSED, else off.
inline bool fused_shape_ok(const ntt_plan_s* p, uint32_t split) {
  return split >= 1 && split <= 4 && p->log_n == split + 12;
}
inline bool fused_for(const ntt_plan_s* p, bool inv, uint32_t split, uint32_t batch) {
  (void)inv;
  (void)batch;
  if (!fused_shape_ok(p, split)) return false;
  return (p->flags & NTT_FLAG_FUSED) != 0;
}

// Fused external product (one launch per class): N = 2^4 .. 2^12, cols <= rows,
// at most 1024 threads (rows * N/16) and 64 KiB of LDS (rows * (N + N/16)
// values) per workgroup, key 16-byte aligned.
inline bool xprod_fits(const ntt_plan_s* p, uint32_t rows, uint32_t cols, const void* key) {
  if (p->log_n < 4 || p->log_n > 12 || cols > rows) return false;
  const uint64_t n = 1ull << p->log_n;
  if ((uint64_t)rows * (n / 16) > 1024) return false;
  if ((uint64_t)rows * (n + n / 16) * 8 > 65536) return false;
  return (reinterpret_cast<uintptr_t>(key) & 15u) == 0;
}

// Split used by one call over `batch` polynomials.
inline uint32_t call_split(const ntt_plan_s* p, uint32_t batch) {
  if (p->forced_split >= 0) return (uint32_t)p->forced_split;
  return tuned_split_for(p->log_n, (uint32_t)dominant_class(p), (uint64_t)batch * p->L, p->log_n1);
}

// Polymul with a caller-provided workspace of polymul_ws_bytes(p, batch) bytes
// (none needed when that is 0): the same launches as ntt_polymul without its
// stream-ordered allocation.  No argument checks beyond the workspace.
size_t polymul_ws_bytes(const ntt_plan_s* p, uint32_t batch);
ntt_status polymul_into(const ntt_plan_s* p, void* out, const void* a, const void* b,
                        uint32_t batch, void* ws, hipStream_t s);

// Polymul of `batch` polynomials whose limb-rows live anywhere: row
// poly * L + limb of a, b and out is at a_rows / b_rows / out_rows[row] (device
// arrays of byte addresses, batch * L each).  o and ws are two contiguous
// scratch buffers of batch * L * N words.  Only for calls whose polymul split
// has both passes (polymul_rows_ok); the words are those of polymul_into.
bool polymul_rows_ok(const ntt_plan_s* p, uint32_t batch);
ntt_status polymul_rows_into(const ntt_plan_s* p, const uint64_t* out_rows, const uint64_t* a_rows,
                             const uint64_t* b_rows, uint32_t batch, void* o, void* ws,
                             hipStream_t s);

}  // namespace nttk
