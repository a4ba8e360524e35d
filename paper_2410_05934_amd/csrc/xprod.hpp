// xprod.hpp -- fused external product for single-pass transform lengths.
//
// The TFHE external product (Sec. II-B, Sec. IV-A) transforms the decomposed
// operands, multiplies-and-accumulates them against a key already in the
// transform domain, and inverse-transforms the accumulators.  For N <= 2^12
// one workgroup does all of it for one group of `rows` operands and one limb:
//   slot s (N/16 threads each) forward-transforms operand g*rows + s in
//   registers/LDS, leaves the result in its LDS region, then slot c < cols
//   accumulates sum_r F_r (.) key[r][c] at its 16 positions per thread and
//   inverse-transforms the accumulator (its first inverse round holds the same
//   positions as the forward's last round).  The operands are read once and
//   only the accumulators are written: the same words as ntt_forward on a
//   copy, ntt_mac and ntt_inverse, with one launch and no intermediate in HBM.
#pragma once

#include "decompose.hpp"
#include "ntt_kernels.hpp"

namespace nttk {

struct XpArgs {
  void* dst;                  // [groups][cols][L][N], natural order
  const void* a;              // [num_operands][L][N], natural order, not modified
                              // (decomposing: [groups][comps][L][N] ciphertexts)
  const void* key;            // [rows][cols][L][N], transform domain
  const LimbDev* limbs;
  const uint32_t* cls_limbs;  // limbs of this launch's class
  uint32_t n_cls;
  uint32_t L;
  uint32_t rows, cols, num_operands;
  uint32_t comps, levels, log_base;  // decomposing: rows = comps * levels
  uint64_t dec_offset;               // digit_offset(levels, log_base)
  const uint32_t* rot;               // CMux: rotation of each ciphertext (taken mod 2N)
};

// What the kernel's operands are.
enum XpMode : int {
  kXpOperands = 0,  // the operands themselves, in `a`
  kXpDecompose = 1, // the gadget digits of the ciphertexts in `a`
  kXpCmux = 2,      // the digits of X^rot acc - acc (acc in `a`); acc is added to the result
};

// Grid: groups * n_cls workgroups of rows * (N / 2^RB) threads (radix-2^RB
// rounds); dynamic LDS of rows regions of N + N/16 values (the padded chunk,
// also for N = 16 where the row pass itself needs no LDS).  Requires
// cols <= rows.
// kXpDecompose: the operands are not in memory; slot s = c * levels + j computes
// digit j of component c of ciphertext `grp` as it loads (Decompose, fused).
// kXpCmux: one CMux of blind rotation (Sec. II-B, Sec. IV-A): the digits are
// those of X^r acc - acc (r = rot[grp]), and the stored result is acc plus the
// inverse transform, i.e. acc + ExtProd(key, X^r acc - acc); cols = comps.
template <class A, int LOGN2, int MODE = kXpOperands, int RB = 4>
__global__ void __launch_bounds__(1024)
xprod_kernel(XpArgs args) {
  using S = RowShape<LOGN2, RB>;
  using V = typename A::V;
  using W = typename A::W;
  constexpr int R = S::R;
  constexpr uint32_t kRegion = (1u << LOGN2) + (1u << LOGN2) / 16;
  extern __shared__ double xp_lds[];
  V* lds_all = reinterpret_cast<V*>(xp_lds);
  const uint32_t slot = threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x % S::TPC;
  const uint32_t grp = blockIdx.x / args.n_cls;
  const uint32_t limb = args.cls_limbs[blockIdx.x % args.n_cls];
  const LimbDev& ld = args.limbs[limb];
  const A ar(ld);
  const uint64_t poly_words = (uint64_t)args.L << LOGN2;
  const uint64_t limb_off = (uint64_t)limb << LOGN2;
  const uint32_t first = grp * args.rows;
  const uint32_t nr = min(args.rows, args.num_operands - first);
  V* lds = lds_all + slot * kRegion;
  constexpr int H0 = S::hb(0);

  // Column c = slot; thread tt reads key positions tt*R + u.  The key words of
  // the first row are requested before the forward transform and those of row
  // r + 1 before the products of row r, so their latency overlaps work.
  const uint32_t c = slot < args.cols ? slot : 0;
  const W* key = reinterpret_cast<const W*>(args.key) + limb_off + ((uint64_t)tt << RB);
  constexpr int kVec = 16 / (int)sizeof(W);
  auto load_key = [&](W (&kw)[R], uint32_t r) {
    const W* kr = key + ((uint64_t)r * args.cols + c) * poly_words;
#pragma unroll
    for (int u = 0; u < R; u += kVec) {
      W part[kVec];
      load_words<W, kVec>(part, kr + u);
#pragma unroll
      for (int k = 0; k < kVec; ++k) kw[u + k] = part[k];
    }
  };
  W kcur[R];
  load_key(kcur, 0);

  // Forward transform of operand `slot` (a slot past the group's end
  // transforms the group's first operand and its result is never read).
  const uint32_t op = slot < nr ? slot : 0;
  V v[R];
  if constexpr (MODE == kXpDecompose) {
    const uint32_t comp = op / args.levels;
    const uint32_t digit = op - comp * args.levels;
    const W* src = reinterpret_cast<const W*>(args.a) +
                   ((uint64_t)grp * args.comps + comp) * poly_words + limb_off;
#pragma unroll
    for (int u = 0; u < R; ++u)
      v[u] = ar.from_word(signed_digit<W>(src[ins_bits<RB>(tt, u, H0)], digit, args.levels,
                                          args.log_base, args.dec_offset, ld.q));
  } else if constexpr (MODE == kXpCmux) {
    const uint32_t comp = op / args.levels;
    const uint32_t digit = op - comp * args.levels;
    const W* src = reinterpret_cast<const W*>(args.a) +
                   ((uint64_t)grp * args.comps + comp) * poly_words + limb_off;
    constexpr uint32_t kN = 1u << LOGN2;
    // X^r = -X^(r - N) for r >= N; then coefficient pos of X^r' a is a[pos - r'],
    // negated once more when pos - r' wraps below zero.
    uint32_t r = args.rot[grp] & (2u * kN - 1u);
    const bool flip = r >= kN;
    r &= kN - 1u;
    const uint64_t q = ld.q;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t pos = ins_bits<RB>(tt, u, H0);
      const bool wrap = pos < r;
      const uint64_t rv = (uint64_t)src[(pos - r) & (kN - 1u)];
      const uint64_t av = (uint64_t)src[pos];
      const uint64_t sv = (flip != wrap) ? (rv == 0 ? 0 : q - rv) : rv;  // X^r acc at pos
      const uint64_t dv = sv >= av ? sv - av : sv + q - av;             // minus acc
      v[u] = ar.from_word(signed_digit<W>((W)dv, digit, args.levels, args.log_base,
                                          args.dec_offset, q));
    }
  } else {
    const W* src = reinterpret_cast<const W*>(args.a) + (uint64_t)(first + op) * poly_words +
                   limb_off;
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = ar.from_word(src[ins_bits<RB>(tt, u, H0)]);
  }
  // One limb per workgroup: the tables are wave-uniform (scalar first-round twiddles).
  const typename A::TW* twf = uniform_ptr(reinterpret_cast<const typename A::TW*>(ld.twf));
  const typename A::TW* twi = uniform_ptr(reinterpret_cast<const typename A::TW*>(ld.twi));
  row_forward_from<A, LOGN2, RB, 0>(ar, v, twf, 1u, tt, lds);
  // Publish F_slot: thread tt holds positions tt*R + u (the last round's layout).
  using MB = LdsMap<RB, 0>;
  const uint32_t bb = MB::base(tt);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < R; ++u) lds[MB::slot(tt, bb, u)] = v[u];
  __syncthreads();

  // acc = sum over the group's rows of F_r (.) key[r][c].  When a slot spans
  // whole waves (N >= 2^10), `busy` is wave-uniform and the slots without a
  // column skip the products and the inverse arithmetic; they still take part
  // in every barrier of the inverse's LDS exchanges.
  constexpr bool kWaveSlots = S::TPC % 64 == 0;
  const bool busy = !kWaveSlots || __builtin_amdgcn_readfirstlane(slot) < args.cols;
  V acc[R];
#pragma unroll
  for (int u = 0; u < R; ++u) acc[u] = V{};
  for (uint32_t r = 0; busy && r < nr; ++r) {
    W knext[R];
    if (r + 1 < nr) load_key(knext, r + 1);
    const V* fr = lds_all + r * kRegion;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const V prod = ar.mul(fr[MB::slot(tt, bb, u)], ar.from_word(kcur[u]));
      acc[u] = r == 0 ? prod : ar.add(acc[u], prod);
    }
#pragma unroll
    for (int u = 0; u < R; ++u) kcur[u] = knext[u];
  }
#pragma unroll
  for (int u = 0; u < R; ++u) ar.center(acc[u]);
  __syncthreads();  // every slot has read the F regions before they are reused

  // Inverse transform of the accumulator; only the first `cols` slots store.
  if (busy) {
    row_inverse_from<A, LOGN2, RB, S::K - 1, true>(ar, acc, twi, 1u, tt, lds, ld);
  } else {
    // the barriers of the K - 1 exchanges (two each) in row_inverse_from
#pragma unroll
    for (int i = 0; i < 2 * (S::K - 1); ++i) __syncthreads();
  }
  if (slot < args.cols) {
    W* dst = reinterpret_cast<W*>(args.dst) + ((uint64_t)grp * args.cols + slot) * poly_words +
             limb_off;
    if constexpr (MODE == kXpCmux) {
      // acc + ExtProd: component `slot` of this ciphertext, same positions
      const W* a0 = reinterpret_cast<const W*>(args.a) +
                    ((uint64_t)grp * args.comps + slot) * poly_words + limb_off;
      const uint64_t q = ld.q;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const uint32_t pos = ins_bits<RB>(tt, u, H0);
        const uint64_t s2 = (uint64_t)ar.to_word(acc[u]) + (uint64_t)a0[pos];
        dst[pos] = (W)(s2 >= q ? s2 - q : s2);
      }
    } else {
#pragma unroll
      for (int u = 0; u < R; ++u) dst[ins_bits<RB>(tt, u, H0)] = ar.to_word(acc[u]);
    }
  }
}

}  // namespace nttk
