// automorph.hip -- the automorphism sigma_k of R_q = Z_q[x]/(x^N+1),
// b(x) = a(x^k) for odd k (Sec. III lists Automorph among the CKKS operators
// around the NTT; Sec. IV-B builds repacking on it).
//
// It moves words and negates some of them; no modular products.
//   coefficient domain: the term a_i x^i becomes a_i x^(i k mod 2N), negated
//     when that exponent is N or more (x^N = -1).  Either thread i reads a_i
//     and scatters it to i k mod 2N (SCATTER), or thread t gathers output t
//     from i = t k^-1 mod 2N (negated, from i - N, when i >= N).  The host takes
//     the form whose lane-to-lane stride (k or k^-1, taken mod 2N either way
//     round) is smaller: rotations by small powers of the generator have small
//     k and large k^-1 (k = 5: 5 against 52429 at N = 2^16).
//   transform domain (the forward transform's output order): slot j holds the
//     value at psi^(2 brv(j) + 1), and b evaluated there is a evaluated at
//     psi^((2 brv(j) + 1) k), i.e. slot brv(((2 brv(j) + 1) k mod 2N - 1) / 2)
//     of the input: a pure permutation, gathered.  Low bits of j stay low bits
//     of the source slot (j and j ^ 1 read neighbours), so its reads are nearly
//     as local as its writes.
// Rows are dealt to the XCDs in contiguous ranges, so the scattered accesses of
// a row meet in one L2.
#include <hip/hip_runtime.h>

#include "ntt_internal.hpp"
#include "ntt_kernels.hpp"

namespace nttk {

struct AutoArgs {
  void* out;
  const void* in;
  const LimbDev* limbs;  // q of each limb (coefficient domain only)
  uint32_t L;
  uint32_t log_n;
  uint32_t k;            // odd, < 2N
  uint32_t kinv;         // k^-1 mod 2N
  uint32_t total;        // batch * L * N < 2^32
};

constexpr uint32_t kAutoBlock = 256;

__device__ __forceinline__ uint32_t brv_bits(uint32_t x, uint32_t bits) {
  return __builtin_bitreverse32(x) >> (32u - bits);  // bits >= 1
}

template <class W, bool TRANSFORMED, bool SCATTER>
__global__ void __launch_bounds__(kAutoBlock) automorph_kernel(AutoArgs a) {
  const uint32_t e = xcd_block(blockIdx.x, gridDim.x) * kAutoBlock + threadIdx.x;
  if (e >= a.total) return;
  const uint32_t n = 1u << a.log_n;
  const uint32_t mask2n = 2u * n - 1u;
  const uint32_t row = e >> a.log_n;
  const uint32_t t = e & (n - 1u);
  if constexpr (SCATTER) {
    // thread t holds the term a_t x^t of its row
    W* dst = static_cast<W*>(a.out) + ((uint64_t)row << a.log_n);
    const W v = static_cast<const W*>(a.in)[e];
    const uint32_t ex = (uint32_t)(((uint64_t)t * a.k) & mask2n);
    if (ex < n) {
      dst[ex] = v;
    } else {
      const W q = (W)a.limbs[row % a.L].q;
      dst[ex - n] = v == 0 ? v : (W)(q - v);
    }
    return;
  }
  const W* src = static_cast<const W*>(a.in) + ((uint64_t)row << a.log_n);
  W x;
  if constexpr (TRANSFORMED) {
    const uint32_t ex = (uint32_t)(((uint64_t)(2u * brv_bits(t, a.log_n) + 1u) * a.k) & mask2n);
    x = src[brv_bits((ex - 1u) >> 1, a.log_n)];
  } else {
    const uint32_t i = (uint32_t)(((uint64_t)t * a.kinv) & mask2n);
    if (i < n) {
      x = src[i];
    } else {
      const W v = src[i - n];
      const W q = (W)a.limbs[row % a.L].q;
      x = v == 0 ? v : (W)(q - v);
    }
  }
  static_cast<W*>(a.out)[e] = x;
}

// Distance of x from 0 mod m, either way round.
static uint32_t ring_dist(uint32_t x, uint32_t m) { return x < m - x ? x : m - x; }

template <class W>
static hipError_t launch_automorph(const AutoArgs& a, bool transformed, hipStream_t s) {
  const uint32_t blocks = (uint32_t)(((uint64_t)a.total + kAutoBlock - 1) / kAutoBlock);
  const uint32_t two_n = 2u << a.log_n;
  LaunchTimer t("automorph", sizeof(W) == 4 ? "u32" : "u64", (int)a.log_n, false, transformed,
                a.total, s);
  if (transformed)
    hipLaunchKernelGGL((automorph_kernel<W, true, false>), dim3(blocks), dim3(kAutoBlock), 0, s, a);
  else if (ring_dist(a.k, two_n) < ring_dist(a.kinv, two_n))
    hipLaunchKernelGGL((automorph_kernel<W, false, true>), dim3(blocks), dim3(kAutoBlock), 0, s, a);
  else
    hipLaunchKernelGGL((automorph_kernel<W, false, false>), dim3(blocks), dim3(kAutoBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace nttk

using namespace nttk;

extern "C" {

ntt_status ntt_automorph(ntt_plan_t plan, void* out, const void* in, uint32_t batch, uint32_t k,
                         uint32_t flags, void* stream) {
  clear_error();
  if (!plan) return fail(NTT_EINVAL, "null plan");
  if (batch == 0) return fail(NTT_EINVAL, "batch must be >= 1");
  if (!out || !in) return fail(NTT_EINVAL, "null data");
  if (flags & ~NTT_AUTOMORPH_TRANSFORMED) return fail(NTT_EINVAL, "unknown flags 0x%x", flags);
  const uint64_t two_n = 2ull << plan->log_n;
  if ((k & 1u) == 0 || k >= two_n)
    return fail(NTT_EINVAL, "k=%u must be odd and below 2N=%llu", k, (unsigned long long)two_n);
  const uint64_t words = (uint64_t)batch * plan->L << plan->log_n;
  if (words >= (1ull << 32)) return fail(NTT_EINVAL, "batch * L * N must be < 2^32 words");
  const uint64_t bytes = words * (plan->word_bits / 8);
  const uintptr_t o = reinterpret_cast<uintptr_t>(out), i = reinterpret_cast<uintptr_t>(in);
  if (o < i + bytes && i < o + bytes) return fail(NTT_EINVAL, "out must not overlap in");
  // k^-1 mod 2N: Newton's iteration x <- x (2 - k x) doubles the correct low
  // bits each step (k x = 1 mod 2^3 for x = k, k odd), so five steps give 96.
  uint32_t kinv = k;
  for (int it = 0; it < 5; ++it) kinv *= 2u - k * kinv;
  AutoArgs a;
  a.out = out;
  a.in = in;
  a.limbs = plan->d_limbs;
  a.L = plan->L;
  a.log_n = plan->log_n;
  a.k = k;
  a.kinv = kinv & (uint32_t)(two_n - 1);
  a.total = (uint32_t)words;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ntt_status vst = validate_words(plan, in, batch, s, "in");
  if (vst != NTT_OK) return vst;
  const bool tr = (flags & NTT_AUTOMORPH_TRANSFORMED) != 0;
  const hipError_t e = plan->word_bits == 32 ? launch_automorph<uint32_t>(a, tr, s)
                                             : launch_automorph<uint64_t>(a, tr, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return NTT_OK;
}

}  // extern "C"
