// ntt_lib.hip -- plan construction, kernel dispatch and the C ABI of libntt.so.
//
// Host number theory here (primality, non-residue, root choice, inverses) is
// this library's own; it shares nothing with any checking code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ntt.h"
#include "decompose.hpp"
#include "modarith.hpp"
#include "ntt_internal.hpp"

using namespace nttk;

// ---------------------------------------------------------------------------
// Errors

static thread_local std::string g_last_error;

ntt_status nttk::fail(ntt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

ntt_status nttk::hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? NTT_ENOMEM : NTT_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

void nttk::clear_error() { g_last_error.clear(); }

#include "numtheory.hpp"

static ntt_status check_modulus(uint32_t N, uint64_t q, uint32_t word_bits) {
  if (N < 2 || N > (1u << 16) || (N & (N - 1)))
    return fail(NTT_EINVAL, "N=%u is not a power of two in [2, 65536]", N);
  if (word_bits != 32 && word_bits != 64) return fail(NTT_EINVAL, "word_bits=%u", word_bits);
  if (word_bits == 32 && q >= (1ull << 32))
    return fail(NTT_ERANGE, "q=%llu does not fit 32-bit words", (unsigned long long)q);
  if (word_bits == 64 && q >= (1ull << 62))
    return fail(NTT_ERANGE, "q=%llu >= 2^62", (unsigned long long)q);
  if (!nt_is_prime(q)) return fail(NTT_ENOTPRIME, "q=%llu is not prime", (unsigned long long)q);
  if ((q - 1) % (2ull * N) != 0)
    return fail(NTT_ENOROOT, "q=%llu is not 1 mod 2N=%u", (unsigned long long)q, 2 * N);
  return NTT_OK;
}

static uint64_t root_of(uint32_t N, uint64_t q) {
  const uint64_t g = nt_smallest_nonresidue(q);
  return nt_pow(g, (q - 1) / (2ull * N), q);
}

// ---------------------------------------------------------------------------
// Plan

static uint32_t default_split(int log_n) {
  if (log_n < 4) return (uint32_t)log_n;   // whole transform in the column kernel
  if (log_n <= 12) return 0;               // single on-chip pass
  return (uint32_t)(log_n - 12);           // column pass + 4096-word rows
}

bool nttk::split_valid(int log_n, int n1) {
  if (n1 == 0) return log_n >= 4 && log_n <= 14;
  if (n1 == log_n) return log_n <= 5;
  return n1 >= 1 && n1 <= 5 && (log_n - n1) >= 4 && (log_n - n1) <= 14;
}

static double centred(uint64_t w, uint64_t q) {
  return w > q / 2 ? -(double)(q - w) : (double)w;
}

static ntt_status build_plan(ntt_plan_s* p, const uint64_t* moduli) {
  const uint32_t N = p->N;
  const int n = p->log_n;
  std::vector<LimbDev> limbs(p->L);
  p->tables.assign(p->L, nullptr);
  for (uint32_t l = 0; l < p->L; ++l) {
    const uint64_t q = moduli[l];
    uint32_t c;
    if (p->word_bits == 32) c = 0;
    else if (!(p->flags & NTT_FLAG_FORCE_INT64) && q < kF64LBound) c = 1;
    else c = 2;
    p->cls[l] = c;
    const PrimeTable* t = nullptr;
    ntt_status st = acquire_table(p->device, q, c, &t);
    if (st != NTT_OK) return st;
    p->tables[l] = t;
    // psi_N = psi_table^(2^(log_len - n)); the table prefix of length N is T_N.
    const uint64_t psi = root_of(N, q);
    const uint64_t psi_inv = nt_pow(psi, q - 2, q);
    p->psi[l] = psi;
    const uint64_t ninv = nt_pow(N % q, q - 2, q);
    // last inverse stage twiddle: psi^-brv(1) = psi^-(N/2)
    const uint64_t w1inv = nt_pow(psi_inv, N / 2, q);
    const uint64_t ninvw = nt_mul(ninv, w1inv, q);
    LimbDev& d = limbs[l];
    std::memset(&d, 0, sizeof(d));
    d.q = q;
    d.qd = (double)q;
    d.qinv = 1.0 / (double)q;
    d.cls = c;
    d.qbits = 64 - __builtin_clzll(q);
    d.bmu = (uint64_t)(((u128)1 << (2 * d.qbits)) / q);
    d.ninv_d = centred(ninv, q);
    d.ninvw_d = centred(ninvw, q);
    d.ninv = ninv;
    d.ninv_s = (uint64_t)(((u128)ninv << 64) / q);
    d.ninvw = ninvw;
    d.ninvw_s = (uint64_t)(((u128)ninvw << 64) / q);
    d.twf = t->twf;
    d.twi = t->twi;
    (void)n;
  }
  hipError_t e = hipMalloc(&p->d_limbs, sizeof(LimbDev) * p->L);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(limb constants)");
  e = hipMemcpy(p->d_limbs, limbs.data(), sizeof(LimbDev) * p->L, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(limb constants)");
  p->h_limbs = limbs;
  // Limb lists per arithmetic class.
  std::vector<uint32_t> lists;
  for (int c = 0; c < 3; ++c) {
    p->cls_off[c] = (uint32_t)lists.size();
    for (uint32_t l = 0; l < p->L; ++l)
      if (p->cls[l] == (uint32_t)c) lists.push_back(l);
    p->cls_cnt[c] = (uint32_t)lists.size() - p->cls_off[c];
  }
  e = hipMalloc(&p->d_cls_limbs, sizeof(uint32_t) * lists.size());
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(limb lists)");
  e = hipMemcpy(p->d_cls_limbs, lists.data(), sizeof(uint32_t) * lists.size(),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(limb lists)");
  p->h_cls_limbs = lists;
  return NTT_OK;
}

static void free_plan(ntt_plan_s* p) {
  if (!p) return;
  for (const PrimeTable* t : p->tables) release_table(t);
  if (p->d_limbs) (void)hipFree(p->d_limbs);
  if (p->d_cls_limbs) (void)hipFree(p->d_cls_limbs);
  delete p;
}

// Launchers, instantiated per arithmetic class in inst_*.hip.
namespace nttk {
template <class A>
hipError_t transform_cls(const ntt_plan_s* p, int c, void* data, uint32_t batch, bool inv,
                         uint32_t split, uint32_t* work, hipStream_t s);
template <class A>
hipError_t pointwise_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* b,
                         uint32_t batch, hipStream_t s);
template <class A>
hipError_t polymul_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* b,
                       void* ws, uint32_t batch, uint32_t split, hipStream_t s);
template <class A>
hipError_t polymul_rows_cls(const ntt_plan_s* p, int c, const uint64_t* out_rows,
                            const uint64_t* a_rows, const uint64_t* b_rows, void* o, void* ws,
                            uint32_t batch, uint32_t split, hipStream_t s);
template <class A>
hipError_t mac_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* key,
                   uint32_t rows, uint32_t cols, uint32_t num_operands, hipStream_t s);
template <class A>
hipError_t fwdmul_cls(const ntt_plan_s* p, int c, void* out, void* a, void* b, uint32_t batch,
                      uint32_t split, hipStream_t s);
template <class A>
hipError_t xprod_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* key,
                     uint32_t rows, uint32_t cols, uint32_t num_operands, hipStream_t s,
                     uint32_t comps, uint32_t levels, uint32_t log_base, const uint32_t* rot);
#define NTT_EXTERN_CLASS(A)                                                                   \
  extern template hipError_t transform_cls<A>(const ntt_plan_s*, int, void*, uint32_t, bool,  \
                                              uint32_t, uint32_t*, hipStream_t);              \
  extern template hipError_t pointwise_cls<A>(const ntt_plan_s*, int, void*, const void*,     \
                                              const void*, uint32_t, hipStream_t);            \
  extern template hipError_t polymul_cls<A>(const ntt_plan_s*, int, void*, const void*,       \
                                            const void*, void*, uint32_t, uint32_t,           \
                                            hipStream_t);                                     \
  extern template hipError_t mac_cls<A>(const ntt_plan_s*, int, void*, const void*,           \
                                        const void*, uint32_t, uint32_t, uint32_t, hipStream_t); \
  extern template hipError_t xprod_cls<A>(const ntt_plan_s*, int, void*, const void*,         \
                                          const void*, uint32_t, uint32_t, uint32_t, hipStream_t, \
                                          uint32_t, uint32_t, uint32_t, const uint32_t*);
#define NTT_EXTERN_FWDMUL(A)                                                             \
  extern template hipError_t fwdmul_cls<A>(const ntt_plan_s*, int, void*, void*, void*, uint32_t, \
                                           uint32_t, hipStream_t);                              \
  extern template hipError_t polymul_rows_cls<A>(const ntt_plan_s*, int, const uint64_t*,      \
                                                 const uint64_t*, const uint64_t*, void*, void*, \
                                                 uint32_t, uint32_t, hipStream_t);
NTT_EXTERN_FWDMUL(ArF64S)
NTT_EXTERN_FWDMUL(ArF64L)
NTT_EXTERN_FWDMUL(ArI64)
NTT_EXTERN_CLASS(ArF64S)
NTT_EXTERN_CLASS(ArF64L)
NTT_EXTERN_CLASS(ArI64)
}  // namespace nttk

// Run F<A>(...) for every arithmetic class present in the plan.
#define NTT_FOR_CLASSES(p, CALL)                                                 \
  do {                                                                           \
    for (int c_ = 0; c_ < 3; ++c_) {                                             \
      if ((p)->cls_cnt[c_] == 0) continue;                                       \
      hipError_t e_;                                                             \
      if (c_ == 0) { using A = ArF64S; const int c = c_; e_ = CALL; }            \
      else if (c_ == 1) { using A = ArF64L; const int c = c_; e_ = CALL; }       \
      else { using A = ArI64; const int c = c_; e_ = CALL; }                     \
      if (e_ != hipSuccess) return hip_fail(e_, "kernel launch");                \
    }                                                                            \
  } while (0)

// Digits of ciphertexts [num_ct][comps][L][N] into operands
// [num_ct][comps * levels][L][N] (operand c * levels + j = digit j of component c).
struct DecArgs {
  void* out;
  const void* ct;
  const LimbDev* limbs;
  uint32_t L, log_n, comps, levels, log_base;
  uint32_t total;  // output words, < 2^32
  uint64_t offset;  // digit_offset(levels, log_base)
};

template <class W>
static __global__ void __launch_bounds__(256) decompose_kernel(DecArgs d) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= d.total) return;
  const uint32_t n = e & ((1u << d.log_n) - 1u);
  uint32_t rest = e >> d.log_n;
  const uint32_t l = rest % d.L;
  rest /= d.L;
  const uint32_t rows = d.comps * d.levels;
  const uint32_t r = rest % rows;
  const uint32_t g = rest / rows;
  const uint32_t comp = r / d.levels;
  const uint32_t j = r - comp * d.levels;
  const W x = static_cast<const W*>(d.ct)[((((uint64_t)g * d.comps + comp) * d.L + l) << d.log_n) + n];
  static_cast<W*>(d.out)[e] = signed_digit<W>(x, j, d.levels, d.log_base, d.offset, d.limbs[l].q);
}

// X^rot[g] acc[g] - acc[g] for acc [num_ct][comps][L][N] (rot taken mod 2N).
struct RotArgs {
  void* out;
  const void* acc;
  const uint32_t* rot;
  const LimbDev* limbs;
  uint32_t L, log_n, comps;
  uint32_t total;  // words, < 2^32
};

template <class W>
static __global__ void __launch_bounds__(256) rotdiff_kernel(RotArgs d) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= d.total) return;
  const uint32_t nmask = (1u << d.log_n) - 1u;
  const uint32_t pos = e & nmask;
  const uint32_t row = e >> d.log_n;  // (g * comps + c) * L + l
  const uint32_t l = row % d.L;
  const uint32_t g = row / d.L / d.comps;
  const uint64_t q = d.limbs[l].q;
  const W* src = static_cast<const W*>(d.acc) + ((uint64_t)row << d.log_n);
  uint32_t r = d.rot[g] & (2u * nmask + 1u);
  const bool flip = r > nmask;
  r &= nmask;
  const bool wrap = pos < r;
  const uint64_t rv = (uint64_t)src[(pos - r) & nmask], av = (uint64_t)src[pos];
  const uint64_t sv = (flip != wrap) ? (rv == 0 ? 0 : q - rv) : rv;
  static_cast<W*>(d.out)[e] = (W)(sv >= av ? sv - av : sv + q - av);
}

// out += acc elementwise mod q (same [num][comps][L][N] layout).
template <class W>
static __global__ void __launch_bounds__(256) addmod_kernel(RotArgs d) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= d.total) return;
  const uint32_t l = (e >> d.log_n) % d.L;
  const uint64_t q = d.limbs[l].q;
  W* o = static_cast<W*>(d.out);
  const uint64_t s2 = (uint64_t)o[e] + (uint64_t)static_cast<const W*>(d.acc)[e];
  o[e] = (W)(s2 >= q ? s2 - q : s2);
}

static __global__ void fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Range check of NTT_FLAG_VALIDATE: the smallest flat index of a word that is
// not below its limb's modulus goes to *first (kept at 0xffffffff otherwise).
struct CheckArgs {
  const void* data;      // [polys][L][N]
  const LimbDev* limbs;  // [L]
  uint32_t L, log_n;
  uint32_t total;        // polys * L * N words, < 2^32
  uint32_t* first;
};

template <class W>
static __global__ void __launch_bounds__(256) range_check_kernel(CheckArgs c) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= c.total) return;
  const uint32_t l = (e >> c.log_n) % c.L;
  if ((uint64_t)static_cast<const W*>(c.data)[e] >= c.limbs[l].q) atomicMin(c.first, e);
}

// With NTT_FLAG_VALIDATE: check `polys` polynomials of the plan's layout at
// `data` before anything is launched on them; waits for the stream.  NTT_ERANGE
// names the first word outside [0, q).
ntt_status nttk::validate_words(const ntt_plan_s* p, const void* data, uint64_t polys,
                                hipStream_t s, const char* name) {
  if (!(p->flags & NTT_FLAG_VALIDATE)) return NTT_OK;
  const uint64_t total = polys * p->L << p->log_n;
  if (total >= (1ull << 32)) return fail(NTT_EINVAL, "%s: 2^32 words or more", name);
  uint32_t* first = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&first), 4, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(range check)");
  hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, s, first, 1u, 0xffffffffu);
  CheckArgs c;
  c.data = data;
  c.limbs = p->d_limbs;
  c.L = p->L;
  c.log_n = p->log_n;
  c.total = (uint32_t)total;
  c.first = first;
  const dim3 grid((uint32_t)((total + 255) / 256));
  if (p->word_bits == 32) hipLaunchKernelGGL(range_check_kernel<uint32_t>, grid, dim3(256), 0, s, c);
  else hipLaunchKernelGGL(range_check_kernel<uint64_t>, grid, dim3(256), 0, s, c);
  e = hipGetLastError();
  uint32_t bad = 0xffffffffu;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, first, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFreeAsync(first, s);
  if (e != hipSuccess) return hip_fail(e, "range check");
  if (bad != 0xffffffffu) {
    const uint32_t idx = bad & ((1u << p->log_n) - 1u);
    const uint32_t row = bad >> p->log_n;
    return fail(NTT_ERANGE, "%s: word %u of polynomial %u, limb %u is not below q = %llu", name,
                idx, row / p->L, row % p->L, (unsigned long long)p->moduli[row % p->L]);
  }
  return NTT_OK;
}

static std::atomic<uint32_t> g_spin_limit{1u << 20};
static std::atomic<uint32_t> g_force_expire{0};
uint32_t nttk::fused_spin_limit() { return g_spin_limit.load(std::memory_order_relaxed); }
bool nttk::fused_force_expire() { return g_force_expire.load(std::memory_order_relaxed) != 0; }

// Forward or inverse over every class of the plan.  The single-launch form
// needs 1 + batch * cls_cnt[c] zeroed counters per class and one expiry flag
// (one stream-ordered allocation, cleared by a fill kernel); it waits for the
// stream and reads the flag back, so that an expired wait is reported.
static ntt_status transform_entry(ntt_plan_t plan, void* data, uint32_t batch, bool inv,
                                  hipStream_t s) {
  const uint32_t split = call_split(plan, batch);
  uint32_t* work = nullptr;
  const uint32_t n = batch * plan->L + 4;
  if (fused_for(plan, inv, split, batch)) {
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&work), (size_t)n * 4, s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(single-launch counters)");
    hipLaunchKernelGGL(fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, work, n, 0u);
    e = hipGetLastError();
    if (e != hipSuccess) {
      (void)hipFreeAsync(work, s);
      return hip_fail(e, "counter fill");
    }
  }
  ntt_status rc = [&]() -> ntt_status {
    NTT_FOR_CLASSES(plan, (transform_cls<A>(plan, c, data, batch, inv, split, work, s)));
    return NTT_OK;
  }();
  if (work) {
    uint32_t expired = 0;
    hipError_t e = hipMemcpyAsync(&expired, work + (n - 1), 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc == NTT_OK && e != hipSuccess) rc = hip_fail(e, "single-launch expiry flag");
    if (rc == NTT_OK && expired)
      rc = fail(NTT_ETIMEOUT, "a wait of the single-launch transform gave up after %u polls; "
                "the output is unspecified", fused_spin_limit());
    (void)hipFreeAsync(work, s);
  }
  return rc;
}

namespace nttk {
size_t polymul_ws_bytes(const ntt_plan_s* p, uint32_t batch) {
  const uint32_t split = polymul_split(p, call_split(p, batch));
  return split ? ((size_t)batch * p->L << p->log_n) * (p->word_bits / 8) : 0;
}

ntt_status polymul_into(const ntt_plan_s* plan, void* out, const void* a, const void* b,
                        uint32_t batch, void* ws, hipStream_t s) {
  const uint32_t split = polymul_split(plan, call_split(plan, batch));
  if (split && !ws) return fail(NTT_EINVAL, "polymul workspace missing");
  NTT_FOR_CLASSES(plan, (polymul_cls<A>(plan, c, out, a, b, ws, batch, split, s)));
  return NTT_OK;
}

bool polymul_rows_ok(const ntt_plan_s* p, uint32_t batch) {
  const uint32_t split = polymul_split(p, call_split(p, batch));
  return split > 0 && split < p->log_n;
}

ntt_status polymul_rows_into(const ntt_plan_s* plan, const uint64_t* out_rows, const uint64_t* a_rows,
                             const uint64_t* b_rows, uint32_t batch, void* o, void* ws,
                             hipStream_t s) {
  if (!polymul_rows_ok(plan, batch)) return fail(NTT_EINVAL, "polymul through row tables needs two passes");
  if (!o || !ws || !out_rows || !a_rows || !b_rows) return fail(NTT_EINVAL, "null argument");
  const uint32_t split = polymul_split(plan, call_split(plan, batch));
  NTT_FOR_CLASSES(plan, (polymul_rows_cls<A>(plan, c, out_rows, a_rows, b_rows, o, ws, batch, split, s)));
  return NTT_OK;
}
}  // namespace nttk

static ntt_status check_plan_batch(ntt_plan_t p, uint32_t batch) {
  if (!p) return fail(NTT_EINVAL, "null plan");
  if (batch == 0) return fail(NTT_EINVAL, "batch must be >= 1");
  const uint64_t words = (uint64_t)batch * p->L << p->log_n;
  if (words >= (1ull << 32)) return fail(NTT_EINVAL, "batch * L * N must be < 2^32 words");
  return NTT_OK;
}

// ArF64S only instantiates with 32-bit words and the others with 64-bit words;
// a plan never mixes word widths, so the unused pairings are never launched.

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* ntt_last_error(void) { return g_last_error.c_str(); }

const char* ntt_version(void) { return "mi355x-ntt 0.1 (gfx950)"; }

ntt_status ntt_debug_wait_limit(uint32_t polls, uint32_t force_expire) {
  clear_error();
  g_spin_limit.store(polls ? polls : (1u << 20), std::memory_order_relaxed);
  g_force_expire.store(force_expire ? 1u : 0u, std::memory_order_relaxed);
  return NTT_OK;
}

ntt_status ntt_check_modulus(uint32_t N, uint64_t q, uint32_t word_bits) {
  clear_error();
  return check_modulus(N, q, word_bits);
}

ntt_status ntt_find_root(uint32_t N, uint64_t q, uint64_t* psi) {
  clear_error();
  if (!psi) return fail(NTT_EINVAL, "null psi");
  ntt_status st = check_modulus(N, q, 64);
  if (st != NTT_OK) return st;
  *psi = root_of(N, q);
  return NTT_OK;
}

ntt_status ntt_plan_create(ntt_plan_t* out, uint32_t N, const uint64_t* moduli,
                           uint32_t num_moduli, uint32_t word_bits, uint32_t flags) {
  clear_error();
  if (!out || !moduli) return fail(NTT_EINVAL, "null argument");
  *out = nullptr;
  if (num_moduli == 0 || num_moduli > 4096) return fail(NTT_EINVAL, "num_moduli=%u", num_moduli);
  for (uint32_t l = 0; l < num_moduli; ++l) {
    ntt_status st = check_modulus(N, moduli[l], word_bits);
    if (st != NTT_OK) return st;
  }
  if ((flags & NTT_FLAG_ROW_RADIX8) && (flags & NTT_FLAG_ROW_RADIX4))
    return fail(NTT_EINVAL, "NTT_FLAG_ROW_RADIX8 and NTT_FLAG_ROW_RADIX4 are exclusive");
  const int log_n = ilog2(N);
  uint32_t n1 = default_split(log_n);
  if (flags & NTT_FLAG_SPLIT_MASK) {
    const int forced = (int)((flags & NTT_FLAG_SPLIT_MASK) >> 8) - 1;
    if (!split_valid(log_n, forced)) return fail(NTT_EINVAL, "split n1=%d invalid for N=%u", forced, N);
    n1 = (uint32_t)forced;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  ntt_plan_s* p = new (std::nothrow) ntt_plan_s();
  if (!p) return fail(NTT_ENOMEM, "host allocation");
  p->device = dev;
  p->N = N;
  p->log_n = (uint32_t)log_n;
  p->L = num_moduli;
  p->word_bits = word_bits;
  p->flags = flags;
  p->log_n1 = n1;
  p->forced_split = (flags & NTT_FLAG_SPLIT_MASK) ? (int)n1 : -1;
  p->row_rb = (flags & NTT_FLAG_ROW_RADIX8) ? 3 : (flags & NTT_FLAG_ROW_RADIX4) ? 2 : 0;
  p->moduli.assign(moduli, moduli + num_moduli);
  p->psi.resize(num_moduli);
  p->cls.resize(num_moduli);
  ntt_status st = build_plan(p, moduli);
  if (st != NTT_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return NTT_OK;
}

ntt_status ntt_plan_destroy(ntt_plan_t plan) {
  clear_error();
  if (!plan) return fail(NTT_EINVAL, "null plan");
  free_plan(plan);
  return NTT_OK;
}

ntt_status ntt_plan_root(ntt_plan_t plan, uint32_t limb, uint64_t* psi) {
  clear_error();
  if (!plan || !psi) return fail(NTT_EINVAL, "null argument");
  if (limb >= plan->L) return fail(NTT_EINVAL, "limb %u out of range", limb);
  *psi = plan->psi[limb];
  return NTT_OK;
}

ntt_status ntt_plan_split(ntt_plan_t plan, uint32_t* log_n1) {
  clear_error();
  if (!plan || !log_n1) return fail(NTT_EINVAL, "null argument");
  *log_n1 = plan->forced_split >= 0 ? (uint32_t)plan->forced_split : plan->log_n1;
  return NTT_OK;
}

ntt_status ntt_plan_split_for(ntt_plan_t plan, uint32_t batch, uint32_t* log_n1) {
  clear_error();
  if (!plan || !log_n1) return fail(NTT_EINVAL, "null argument");
  *log_n1 = call_split(plan, batch);
  return NTT_OK;
}

ntt_status ntt_plan_limb_class(ntt_plan_t plan, uint32_t limb, uint32_t* cls) {
  clear_error();
  if (!plan || !cls) return fail(NTT_EINVAL, "null argument");
  if (limb >= plan->L) return fail(NTT_EINVAL, "limb %u out of range", limb);
  *cls = plan->cls[limb];
  return NTT_OK;
}

ntt_status ntt_forward(ntt_plan_t plan, void* data, uint32_t batch, void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, batch);
  if (st != NTT_OK) return st;
  if (!data) return fail(NTT_EINVAL, "null data");
  st = validate_words(plan, data, batch, static_cast<hipStream_t>(stream), "data");
  if (st != NTT_OK) return st;
  return transform_entry(plan, data, batch, false, static_cast<hipStream_t>(stream));
}

ntt_status ntt_inverse(ntt_plan_t plan, void* data, uint32_t batch, void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, batch);
  if (st != NTT_OK) return st;
  if (!data) return fail(NTT_EINVAL, "null data");
  st = validate_words(plan, data, batch, static_cast<hipStream_t>(stream), "data");
  if (st != NTT_OK) return st;
  return transform_entry(plan, data, batch, true, static_cast<hipStream_t>(stream));
}

ntt_status ntt_pointwise_mul(ntt_plan_t plan, void* out, const void* a, const void* b,
                             uint32_t batch, void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, batch);
  if (st != NTT_OK) return st;
  if (!out || !a || !b) return fail(NTT_EINVAL, "null data");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = validate_words(plan, a, batch, s, "a")) != NTT_OK) return st;
  if ((st = validate_words(plan, b, batch, s, "b")) != NTT_OK) return st;
  NTT_FOR_CLASSES(plan, (pointwise_cls<A>(plan, c, out, a, b, batch, s)));
  return NTT_OK;
}

ntt_status ntt_mac(ntt_plan_t plan, void* out, const void* a, const void* key, uint32_t rows,
                   uint32_t cols, uint32_t num_operands, void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, num_operands);
  if (st != NTT_OK) return st;
  if (!out || !a || !key) return fail(NTT_EINVAL, "null data");
  if (rows == 0 || cols == 0) return fail(NTT_EINVAL, "rows and cols must be >= 1");
  {
    const uint64_t groups = ((uint64_t)num_operands + rows - 1) / rows;
    const uint64_t poly = (uint64_t)plan->L << plan->log_n;
    if (groups * cols * poly >= (1ull << 32) || (uint64_t)rows * cols * poly >= (1ull << 32))
      return fail(NTT_EINVAL, "out and key must each hold < 2^32 words");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = validate_words(plan, a, num_operands, s, "a")) != NTT_OK) return st;
  if ((st = validate_words(plan, key, (uint64_t)rows * cols, s, "key")) != NTT_OK) return st;
  NTT_FOR_CLASSES(plan, (mac_cls<A>(plan, c, out, a, key, rows, cols, num_operands, s)));
  return NTT_OK;
}

ntt_status ntt_pointwise_mac(ntt_plan_t plan, void* acc, const void* a, const void* key,
                             uint32_t rows, uint32_t cols, uint32_t groups, uint32_t batch_tail,
                             void* stream) {
  clear_error();
  if (groups == 0 || rows == 0) return fail(NTT_EINVAL, "groups and rows must be >= 1");
  if (batch_tail > rows) return fail(NTT_EINVAL, "batch_tail=%u exceeds rows=%u", batch_tail, rows);
  const uint64_t ops = (uint64_t)(groups - 1) * rows + (batch_tail ? batch_tail : rows);
  if (ops >= (1ull << 32)) return fail(NTT_EINVAL, "too many operands");
  return ntt_mac(plan, acc, a, key, rows, cols, (uint32_t)ops, stream);
}

ntt_status ntt_external_product(ntt_plan_t plan, void* out, const void* a, const void* key,
                                uint32_t rows, uint32_t cols, uint32_t num_operands, void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, num_operands);
  if (st != NTT_OK) return st;
  if (!out || !a || !key) return fail(NTT_EINVAL, "null data");
  if (rows == 0 || cols == 0) return fail(NTT_EINVAL, "rows and cols must be >= 1");
  if (out == a || out == key) return fail(NTT_EINVAL, "out must not alias a or key");
  const uint64_t groups = ((uint64_t)num_operands + rows - 1) / rows;
  const uint64_t poly = (uint64_t)plan->L << plan->log_n;
  if (groups * cols * poly >= (1ull << 32) || (uint64_t)rows * cols * poly >= (1ull << 32))
    return fail(NTT_EINVAL, "out and key must each hold < 2^32 words");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = validate_words(plan, a, num_operands, s, "a")) != NTT_OK) return st;
  if ((st = validate_words(plan, key, (uint64_t)rows * cols, s, "key")) != NTT_OK) return st;
  if (xprod_fits(plan, rows, cols, key)) {
    NTT_FOR_CLASSES(plan, (xprod_cls<A>(plan, c, out, a, key, rows, cols, num_operands, s, 0u, 0u, 0u,
                                        nullptr)));
    return NTT_OK;
  }
  // Other shapes: forward a copy of the operands, MAC, inverse.
  const size_t bytes = (size_t)num_operands * poly * (plan->word_bits / 8);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, bytes, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(external-product workspace)");
  e = hipMemcpyAsync(ws, a, bytes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync");
  if (st == NTT_OK) st = ntt_forward(plan, ws, num_operands, stream);
  if (st == NTT_OK) st = ntt_mac(plan, out, ws, key, rows, cols, num_operands, stream);
  if (st == NTT_OK) st = ntt_inverse(plan, out, (uint32_t)(groups * cols), stream);
  (void)hipFreeAsync(ws, s);
  return st;
}

ntt_status ntt_external_product_decomposed(ntt_plan_t plan, void* out, const void* ct,
                                           const void* key, uint32_t num_ct, uint32_t comps,
                                           uint32_t levels, uint32_t log_base, uint32_t cols,
                                           void* stream) {
  clear_error();
  if (!plan) return fail(NTT_EINVAL, "null plan");
  if (!out || !ct || !key) return fail(NTT_EINVAL, "null data");
  if (num_ct == 0 || comps == 0 || levels == 0 || cols == 0)
    return fail(NTT_EINVAL, "num_ct, comps, levels and cols must be >= 1");
  if (log_base == 0 || log_base > 32) return fail(NTT_EINVAL, "log_base=%u not in 1..32", log_base);
  if (out == ct || out == key) return fail(NTT_EINVAL, "out must not alias ct or key");
  const uint64_t span = (uint64_t)levels * log_base;  // digits cover 2^(span - 1)
  if (span > 64) return fail(NTT_EINVAL, "levels * log_base = %llu exceeds 64",
                             (unsigned long long)span);
  for (uint32_t l = 0; l < plan->L; ++l) {
    if (span < 64 && plan->moduli[l] > (1ull << (span - 1)))
      return fail(NTT_EINVAL, "levels * log_base = %llu too small for q=%llu (need q <= 2^%llu)",
                  (unsigned long long)span, (unsigned long long)plan->moduli[l],
                  (unsigned long long)(span - 1));
  }
  const uint64_t rows = (uint64_t)comps * levels;
  const uint64_t poly = (uint64_t)plan->L << plan->log_n;
  const uint64_t num_operands = (uint64_t)num_ct * rows;
  if (num_operands * poly >= (1ull << 32) || (uint64_t)num_ct * cols * poly >= (1ull << 32) ||
      rows * cols * poly >= (1ull << 32))
    return fail(NTT_EINVAL, "operands, out and key must each hold < 2^32 words");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ntt_status vst = validate_words(plan, ct, (uint64_t)num_ct * comps, s, "ct");
  if (vst == NTT_OK) vst = validate_words(plan, key, rows * cols, s, "key");
  if (vst != NTT_OK) return vst;
  if (xprod_fits(plan, (uint32_t)rows, cols, key)) {
    NTT_FOR_CLASSES(plan, (xprod_cls<A>(plan, c, out, ct, key, (uint32_t)rows, cols,
                                        (uint32_t)num_operands, s, comps, levels, log_base,
                                        nullptr)));
    return NTT_OK;
  }
  // Other shapes: the digits into a stream-ordered workspace, then the external
  // product of those operands.
  const size_t bytes = (size_t)(num_operands * poly) * (plan->word_bits / 8);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, bytes, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(decomposition workspace)");
  DecArgs d;
  d.out = ws;
  d.ct = ct;
  d.limbs = plan->d_limbs;
  d.L = plan->L;
  d.log_n = plan->log_n;
  d.comps = comps;
  d.levels = levels;
  d.log_base = log_base;
  d.total = (uint32_t)(num_operands * poly);
  d.offset = digit_offset(levels, log_base);
  const uint32_t blocks = (uint32_t)(((uint64_t)d.total + 255) / 256);
  if (plan->word_bits == 32)
    hipLaunchKernelGGL(decompose_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL(decompose_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s, d);
  e = hipGetLastError();
  ntt_status st = NTT_OK;
  if (e != hipSuccess) st = hip_fail(e, "kernel launch");
  if (st == NTT_OK) st = ntt_external_product(plan, out, ws, key, (uint32_t)rows, cols,
                                              (uint32_t)num_operands, stream);
  (void)hipFreeAsync(ws, s);
  return st;
}

ntt_status ntt_cmux(ntt_plan_t plan, void* out, const void* acc, const uint32_t* rot,
                    const void* key, uint32_t num_ct, uint32_t comps, uint32_t levels,
                    uint32_t log_base, void* stream) {
  clear_error();
  if (!plan) return fail(NTT_EINVAL, "null plan");
  if (!out || !acc || !rot || !key) return fail(NTT_EINVAL, "null data");
  if (num_ct == 0 || comps == 0 || levels == 0)
    return fail(NTT_EINVAL, "num_ct, comps and levels must be >= 1");
  if (log_base == 0 || log_base > 32) return fail(NTT_EINVAL, "log_base=%u not in 1..32", log_base);
  if (out == acc || out == key) return fail(NTT_EINVAL, "out must not alias acc or key");
  const uint64_t span = (uint64_t)levels * log_base;
  if (span > 64) return fail(NTT_EINVAL, "levels * log_base = %llu exceeds 64", (unsigned long long)span);
  for (uint32_t l = 0; l < plan->L; ++l) {
    if (span < 64 && plan->moduli[l] > (1ull << (span - 1)))
      return fail(NTT_EINVAL, "levels * log_base = %llu too small for q=%llu",
                  (unsigned long long)span, (unsigned long long)plan->moduli[l]);
  }
  const uint64_t rows = (uint64_t)comps * levels;
  const uint64_t poly = (uint64_t)plan->L << plan->log_n;
  const uint64_t acc_words = (uint64_t)num_ct * comps * poly;
  if ((uint64_t)num_ct * rows * poly >= (1ull << 32) || rows * comps * poly >= (1ull << 32))
    return fail(NTT_EINVAL, "operands and key must each hold < 2^32 words");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ntt_status vst = validate_words(plan, acc, (uint64_t)num_ct * comps, s, "acc");
  if (vst == NTT_OK) vst = validate_words(plan, key, rows * comps, s, "key");
  if (vst != NTT_OK) return vst;
  if (xprod_fits(plan, (uint32_t)rows, comps, key)) {
    NTT_FOR_CLASSES(plan, (xprod_cls<A>(plan, c, out, acc, key, (uint32_t)rows, comps,
                                        (uint32_t)(num_ct * rows), s, comps, levels, log_base,
                                        rot)));
    return NTT_OK;
  }
  // Other shapes: the rotated difference into a workspace, its decomposed
  // external product into out, then out += acc.
  const size_t bytes = (size_t)acc_words * (plan->word_bits / 8);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, bytes, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(CMux workspace)");
  RotArgs d;
  d.out = ws;
  d.acc = acc;
  d.rot = rot;
  d.limbs = plan->d_limbs;
  d.L = plan->L;
  d.log_n = plan->log_n;
  d.comps = comps;
  d.total = (uint32_t)acc_words;
  const uint32_t blocks = (uint32_t)(((uint64_t)d.total + 255) / 256);
  if (plan->word_bits == 32) hipLaunchKernelGGL(rotdiff_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s, d);
  else hipLaunchKernelGGL(rotdiff_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s, d);
  e = hipGetLastError();
  ntt_status st = e == hipSuccess ? NTT_OK : hip_fail(e, "kernel launch");
  if (st == NTT_OK)
    st = ntt_external_product_decomposed(plan, out, ws, key, num_ct, comps, levels, log_base,
                                         comps, stream);
  if (st == NTT_OK) {
    d.out = out;
    if (plan->word_bits == 32) hipLaunchKernelGGL(addmod_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s, d);
    else hipLaunchKernelGGL(addmod_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s, d);
    e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "kernel launch");
  }
  (void)hipFreeAsync(ws, s);
  return st;
}

ntt_status ntt_forward_mul(ntt_plan_t plan, void* out, void* a, void* b, uint32_t batch,
                           void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, batch);
  if (st != NTT_OK) return st;
  if (!out || !a || !b) return fail(NTT_EINVAL, "null data");
  if (out == a || out == b || a == b) return fail(NTT_EINVAL, "out, a and b must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = validate_words(plan, a, batch, s, "a")) != NTT_OK) return st;
  if ((st = validate_words(plan, b, batch, s, "b")) != NTT_OK) return st;
  // the split of a forward over all 2 * batch polynomials, restricted as polymul's
  const uint32_t split = polymul_split(plan, call_split(plan, 2 * batch));
  NTT_FOR_CLASSES(plan, (fwdmul_cls<A>(plan, c, out, a, b, batch, split, s)));
  return NTT_OK;
}

ntt_status ntt_polymul(ntt_plan_t plan, void* out, const void* a, const void* b, uint32_t batch,
                       void* stream) {
  clear_error();
  ntt_status st = check_plan_batch(plan, batch);
  if (st != NTT_OK) return st;
  if (!out || !a || !b) return fail(NTT_EINVAL, "null data");
  if (out == a || out == b) return fail(NTT_EINVAL, "out must not alias a or b");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = validate_words(plan, a, batch, s, "a")) != NTT_OK) return st;
  if ((st = validate_words(plan, b, batch, s, "b")) != NTT_OK) return st;
  void* ws = nullptr;
  const size_t bytes = polymul_ws_bytes(plan, batch);
  if (bytes) {
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(polymul workspace)");
  }
  const ntt_status rc = polymul_into(plan, out, a, b, batch, ws, s);
  if (ws) (void)hipFreeAsync(ws, s);
  return rc;
}

}  // extern "C"
