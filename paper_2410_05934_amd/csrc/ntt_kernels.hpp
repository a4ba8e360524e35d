// ntt_kernels.hpp -- gfx950 kernels for the negacyclic NTT over RNS limbs.
//
// Transform structure (Chameleon, Sec. II-D, Eq. (1)): the forward transform is
// the Cooley-Tukey network taking natural order to bit-reversed order with
// twiddles psi^brv(m+i); the inverse is the Gentleman-Sande network taking
// bit-reversed order back to natural order with psi^-brv(m+i), followed by
// N^-1 (folded here into the last stage).  Stage s (s = 0 .. log2 N - 1) has
// m = 2^s groups; element x pairs with x + N/2^(s+1), twiddle index
// 2^s + (x >> (log2 N - s)).
//
// Splitting N = N1 * N2 (the paper's two-phase hybrid, Sec. V-C/V-D):
//   column pass   stages 0 .. log2 N1 - 1.  For a fixed r in [0, N2) the
//                 elements {r + k*N2} are closed under these stages.  One
//                 thread owns one column: it loads its N1 elements (lanes own
//                 consecutive r, so every load is coalesced), runs all of the
//                 column's stages in registers and stores them back.  The
//                 twiddles psi^brv(1 .. N1-1) are the same for every column.
//   row pass      stages log2 N1 .. log2 N - 1.  Each contiguous chunk of N2
//                 words is closed under these stages.  One chunk is owned by
//                 N2/16 threads holding 16 values each; rounds of four fused
//                 stages run in registers (radix-16), and the values are
//                 re-dealt between rounds through padded LDS.  The first
//                 forward round deals out the top four index bits, so global
//                 loads are coalesced; the last round holds the bottom four
//                 bits, i.e. 16 consecutive words per thread (one 128-byte line
//                 for 64-bit words).
// N <= 2^14 runs as a single row pass (N1 = 1).  Tiny N < 16 runs as a single
// column pass (N2 = 1).  The split is a plan parameter (autotuned).
//
// This replaces the paper's butterfly decomposition / thread aggregation /
// coefficient shuffling with the wave64 form of the same ideas: a thread owns
// whole radix-16 sub-transforms (thread aggregation), the data layout keeps
// every dependent value inside one workgroup (coefficient shuffling), and the
// only global synchronisation is the pass boundary.
#pragma once

#include "modarith.hpp"

namespace nttk {

// Row-pass workgroups hold whole chunks and at least one wave: a chunk of 64 or
// more threads is a workgroup of its own, so a single 2^10 transform is one
// 64-thread workgroup and a batch spreads over as many workgroups as chunks
// (measured: 2^10 forward + inverse latency 7.1 against 8.1 us with four
// chunks per 256-thread workgroup).
constexpr int kRowThreadsMin = 64;

struct RowArgs {
  void* dst;                 // output (row pass writes here)
  const void* src;           // input (may equal dst)
  const void* src2;          // second input (fused polymul only)
  const LimbDev* limbs;      // [L]
  const uint32_t* cls_limbs; // limb indices handled by this launch
  uint32_t n_cls;            // number of entries in cls_limbs
  uint32_t L;                // limbs per polynomial in the data layout
  uint32_t log_n;            // log2 N
  uint32_t log_n1;           // column stages before this pass (0: single pass)
  uint32_t total_chunks;     // batch * n_cls * N1
  uint32_t batch;            // polynomials
  void* dst2;                // forward-and-multiply rows: the product a (.) b
  // When the launch's class holds one limb (n_cls == 1): that limb's index and
  // constants, so that short launches read them from their arguments instead of
  // through two dependent global loads (limb list, then constants).
  uint32_t limb0;
  LimbDev one;
};

struct ColArgs {
  void* dst;
  const void* src;
  const LimbDev* limbs;
  const uint32_t* cls_limbs;
  uint32_t n_cls;
  uint32_t L;
  uint32_t log_n;
  uint32_t log_n2;           // row stages after this pass (0: whole transform)
  uint32_t total_cols;       // batch * n_cls * N2
  void* dst2;                // optional second operand of the same shape (polymul's b):
  const void* src2;          //   threads total_cols .. 2*total_cols-1 take it
  uint32_t limb0;            // n_cls == 1: the limb and its constants (as in RowArgs)
  LimbDev one;
  uint32_t block;            // launch: threads (columns) per workgroup, 64..kColBlock
  // Optional row tables (kernels built with ROWS): the byte address of limb-row
  // poly * L + limb of src / src2 / dst, in place of base + row * N words; a
  // null table means the contiguous layout.  Lets one launch read and write
  // operands that live in separate buffers.
  const uint64_t* src_rows;
  const uint64_t* src2_rows;
  const uint64_t* dst_rows;
};

struct EltArgs {
  void* dst;
  const void* a;
  const void* b;
  const LimbDev* limbs;
  const uint32_t* cls_limbs;
  uint32_t n_cls;
  uint32_t L;
  uint32_t log_n;
  uint64_t total;            // batch * n_cls * N elements
};

struct MacArgs {
  void* dst;                 // [groups][cols][L][N]
  const void* a;             // [num_operands][L][N]
  const void* key;           // [rows][cols][L][N]
  const LimbDev* limbs;
  const uint32_t* cls_limbs;
  uint32_t n_cls;
  uint32_t L;
  uint32_t log_n;
  uint32_t rows, cols, num_operands, groups;
  uint64_t total;            // groups * cols * n_cls * N
};

// Padded LDS index: one spare slot after every 16 (spreads strided accesses
// over the banks).
__device__ __forceinline__ uint32_t lds_pad(uint32_t y) { return y + (y >> 4); }

// Row-chunk geometry: 2^LOGN2 words, R = 2^RB values per thread (radix-R
// rounds of RB fused stages).
template <int LOGN2, int RB = 4>
struct RowShape {
  static constexpr int R = 1 << RB;
  static constexpr int N2 = 1 << LOGN2;
  static constexpr int TPC = N2 / R;  // threads per chunk
  static constexpr int CPW = TPC >= kRowThreadsMin ? 1 : kRowThreadsMin / TPC;
  static constexpr int BLOCK = TPC * CPW;
  static constexpr int K = (LOGN2 + RB - 1) / RB;  // rounds
  static constexpr int LAST = LOGN2 - RB * (K - 1);  // stages in the last round
  static constexpr int CHUNK_LDS = K > 1 ? N2 + N2 / 16 : 1;
  // slot of word tt + u*TPC in the padded chunk (linear in u when TPC % 16 == 0)
  __device__ __forceinline__ static uint32_t tail_slot(uint32_t tt, uint32_t u) {
    if constexpr (TPC % 16 == 0) return lds_pad(tt) + u * (TPC + TPC / 16);
    else return lds_pad(tt + u * TPC);
  }
  static constexpr int LDS_ELEMS = CPW * CHUNK_LDS;
  // held-bit offset of round j (forward numbering)
  static constexpr int hb(int j) { return j < K - 1 ? LOGN2 - RB - RB * j : 0; }
  static constexpr int nst(int j) { return j < K - 1 ? RB : LAST; }
};

#define NTT_GLOBAL __attribute__((address_space(1)))

// Tables live in device global memory; saying so lets the compiler use global
// (not flat) loads for pointers that come out of the limb constants.
template <class T>
__device__ __forceinline__ const NTT_GLOBAL T* gptr(const T* p) {
  return (const NTT_GLOBAL T*)p;
}

// A pointer every lane of the wave holds, moved to scalar registers (so that
// loads through it at uniform offsets can be scalar loads).
template <class T>
__device__ __forceinline__ const T* uniform_ptr(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// Local index of value u of thread tt when the thread holds the RB bits at hb.
template <int RB = 4>
__device__ __forceinline__ uint32_t ins_bits(uint32_t tt, uint32_t u, int hb) {
  return ((tt >> hb) << (hb + RB)) | (u << hb) | (tt & ((1u << hb) - 1u));
}

// Padded LDS slot of value u of thread tt in a round holding RB bits at HB.
// When the value bits sit at or above bit 4 (HB >= 4), or at the bottom with
// RB <= 4 (HB == 0), the slot is base(tt) + u * STRIDE with a compile-time
// stride, which the compiler folds into the ds instruction's offset field;
// otherwise it is computed per value.
template <int RB, int HB>
struct LdsMap {
  static constexpr bool kLinear = HB >= 4 || HB == 0;
  static constexpr uint32_t kStride = HB >= 4 ? ((1u << HB) + (1u << (HB - 4))) : 1u;
  __device__ __forceinline__ static uint32_t base(uint32_t tt) {
    return lds_pad(ins_bits<RB>(tt, 0, HB));
  }
  __device__ __forceinline__ static uint32_t slot(uint32_t tt, uint32_t bse, uint32_t u) {
    if constexpr (kLinear) return bse + u * kStride;
    else return lds_pad(ins_bits<RB>(tt, u, HB));
  }
};

// One table entry from global memory (fp64 entry or Shoup pair).
template <class TW>
__device__ __forceinline__ TW load1(const NTT_GLOBAL TW* p) {
  if constexpr (sizeof(TW) == 16) {
    typedef uint64_t uvec2 __attribute__((ext_vector_type(2)));
    const uvec2 t = *reinterpret_cast<const NTT_GLOBAL uvec2*>(p);
    TW w;
    w.w = t.x;
    w.ws = t.y;
    return w;
  } else {
    return *p;
  }
}

// Load G consecutive twiddles starting at an index that is a multiple of G.
template <class TW, int G>
__device__ __forceinline__ void load_tw(TW (&w)[G], const TW* __restrict__ tab_in, uint32_t idx) {
  const NTT_GLOBAL TW* tab = gptr(tab_in);
  if constexpr (sizeof(TW) == 8 && G >= 2) {
    typedef double dvec2 __attribute__((ext_vector_type(2)));
    const NTT_GLOBAL dvec2* p = reinterpret_cast<const NTT_GLOBAL dvec2*>(tab + idx);
#pragma unroll
    for (int i = 0; i < G / 2; ++i) {
      const dvec2 t = p[i];
      w[2 * i] = t.x;
      w[2 * i + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < G; ++i) w[i] = load1<TW>(tab + idx + i);
  }
}

// One forward (CT) stage on the R registers: local stage SP acts on u-bit B.
// ZT: every thread of the chunk has tt >> HB == 0 (the chunk's first round),
// so the twiddle index depends on the chunk alone -- a scalar load when the
// caller made `base` and the table pointer wave-uniform.
template <class A, int RB, int B, int SP, int HB, bool ZT = false>
__device__ __forceinline__ void fwd_stage(const A& ar, typename A::V (&v)[1 << RB],
                                          const typename A::TW* __restrict__ tw, uint32_t base,
                                          uint32_t tt) {
  constexpr int G = 1 << (RB - 1 - B);
  typename A::TW w[G];
  const uint32_t tg = (base << SP) + (ZT ? 0u : ((tt >> HB) << (RB - 1 - B)));
  load_tw<typename A::TW, G>(w, tw, tg);
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int i = 0; i < (1 << B); ++i) {
      const int lo = (g << (B + 1)) | i;
      ar.ct(v[lo], v[lo | (1 << B)], w[g]);
    }
  }
}

// One inverse (GS) stage; FOLD applies N^-1 (only for global stage 0); ZT as
// for fwd_stage.
template <class A, int RB, int B, int SP, int HB, bool FOLD, bool ZT = false>
__device__ __forceinline__ void inv_stage(const A& ar, typename A::V (&v)[1 << RB],
                                          const typename A::TW* __restrict__ tw, uint32_t base,
                                          uint32_t tt, const LimbDev& ld) {
  constexpr int G = 1 << (RB - 1 - B);
  if constexpr (FOLD) {
    static_assert(G == 1, "fold only at the single-group stage");
#pragma unroll
    for (int i = 0; i < (1 << B); ++i) {
      typename A::TW w{};
      ar.gs_fold(v[i], v[i | (1 << B)], w, ld);
    }
  } else {
    typename A::TW w[G];
    const uint32_t tg = (base << SP) + (ZT ? 0u : ((tt >> HB) << (RB - 1 - B)));
    load_tw<typename A::TW, G>(w, tw, tg);
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int i = 0; i < (1 << B); ++i) {
        const int lo = (g << (B + 1)) | i;
        ar.gs(v[lo], v[lo | (1 << B)], w[g]);
      }
    }
  }
}

template <class A, int LOGN2, int RB, int J, int ST>
__device__ __forceinline__ void fwd_round_stages(const A& ar, typename A::V (&v)[1 << RB],
                                                 const typename A::TW* __restrict__ tw,
                                                 uint32_t base, uint32_t tt) {
  using S = RowShape<LOGN2, RB>;
  if constexpr (ST < S::nst(J)) {
    constexpr int HB = S::hb(J);
    constexpr int SP = RB * J + ST;
    constexpr int B = (LOGN2 - 1 - SP) - HB;
    fwd_stage<A, RB, B, SP, HB, (HB >= LOGN2 - RB)>(ar, v, tw, base, tt);
    fwd_round_stages<A, LOGN2, RB, J, ST + 1>(ar, v, tw, base, tt);
  }
}

// Inverse stages of round J run from the highest local stage down.
template <class A, int LOGN2, int RB, int J, int ST, bool FOLD>
__device__ __forceinline__ void inv_round_stages(const A& ar, typename A::V (&v)[1 << RB],
                                                 const typename A::TW* __restrict__ tw,
                                                 uint32_t base, uint32_t tt, const LimbDev& ld) {
  using S = RowShape<LOGN2, RB>;
  if constexpr (ST < S::nst(J)) {
    constexpr int HB = S::hb(J);
    constexpr int SP = RB * J + S::nst(J) - 1 - ST;
    constexpr int B = (LOGN2 - 1 - SP) - HB;
    if constexpr (FOLD && SP == 0) {
      inv_stage<A, RB, B, SP, HB, true>(ar, v, tw, base, tt, ld);
    } else {
      inv_stage<A, RB, B, SP, HB, false, (HB >= LOGN2 - RB)>(ar, v, tw, base, tt, ld);
    }
    inv_round_stages<A, LOGN2, RB, J, ST + 1, FOLD>(ar, v, tw, base, tt, ld);
  }
}

// Re-deal R values per thread from the layout of round JF to round JT.
template <class A, int LOGN2, int RB, int JF, int JT>
__device__ __forceinline__ void lds_exchange(typename A::V (&v)[1 << RB], typename A::V* lds,
                                             uint32_t tt) {
  using S = RowShape<LOGN2, RB>;
  constexpr int HF = S::hb(JF), HT = S::hb(JT);
  using MF = LdsMap<RB, HF>;
  using MT = LdsMap<RB, HT>;
  const uint32_t bf = MF::base(tt), bt = MT::base(tt);
#pragma unroll
  for (int u = 0; u < S::R; ++u) lds[MF::slot(tt, bf, u)] = v[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < S::R; ++u) v[u] = lds[MT::slot(tt, bt, u)];
  __syncthreads();
}

template <class A, int LOGN2, int RB, int J>
__device__ __forceinline__ void row_forward_from(const A& ar, typename A::V (&v)[1 << RB],
                                                 const typename A::TW* __restrict__ tw,
                                                 uint32_t base, uint32_t tt, typename A::V* lds) {
  using S = RowShape<LOGN2, RB>;
  if constexpr (J < S::K) {
    fwd_round_stages<A, LOGN2, RB, J, 0>(ar, v, tw, base, tt);
    if constexpr (J + 1 < S::K) {
      if constexpr (A::kCenterRounds) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) ar.center(v[u]);
      }
      lds_exchange<A, LOGN2, RB, J, J + 1>(v, lds, tt);
      row_forward_from<A, LOGN2, RB, J + 1>(ar, v, tw, base, tt, lds);
    }
  }
}

template <class A, int LOGN2, int RB, int J, bool FOLD>
__device__ __forceinline__ void row_inverse_from(const A& ar, typename A::V (&v)[1 << RB],
                                                 const typename A::TW* __restrict__ tw,
                                                 uint32_t base, uint32_t tt, typename A::V* lds,
                                                 const LimbDev& ld) {
  if constexpr (J >= 0) {
    inv_round_stages<A, LOGN2, RB, J, 0, FOLD>(ar, v, tw, base, tt, ld);
    if constexpr (J > 0) {
      if constexpr (A::kCenterRounds) {
#pragma unroll
        for (int u = 0; u < (1 << RB); ++u) ar.center(v[u]);
      }
      lds_exchange<A, LOGN2, RB, J, J - 1>(v, lds, tt);
      row_inverse_from<A, LOGN2, RB, J - 1, FOLD>(ar, v, tw, base, tt, lds, ld);
    }
  }
}

// Forward stages of two operands of the same chunk (polymul's a and b): each
// stage's twiddles are loaded once and applied to both, and the two butterfly
// streams interleave.
template <class A, int RB, int B, int SP, int HB, bool ZT>
__device__ __forceinline__ void fwd_stage2(const A& ar, typename A::V (&va)[1 << RB],
                                           typename A::V (&vb)[1 << RB],
                                           const typename A::TW* __restrict__ tw, uint32_t base,
                                           uint32_t tt) {
  constexpr int G = 1 << (RB - 1 - B);
  typename A::TW w[G];
  const uint32_t tg = (base << SP) + (ZT ? 0u : ((tt >> HB) << (RB - 1 - B)));
  load_tw<typename A::TW, G>(w, tw, tg);
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int i = 0; i < (1 << B); ++i) {
      const int lo = (g << (B + 1)) | i;
      ar.ct(va[lo], va[lo | (1 << B)], w[g]);
      ar.ct(vb[lo], vb[lo | (1 << B)], w[g]);
    }
  }
}

template <class A, int LOGN2, int RB, int J, int ST>
__device__ __forceinline__ void fwd_round_stages2(const A& ar, typename A::V (&va)[1 << RB],
                                                  typename A::V (&vb)[1 << RB],
                                                  const typename A::TW* __restrict__ tw,
                                                  uint32_t base, uint32_t tt) {
  using S = RowShape<LOGN2, RB>;
  if constexpr (ST < S::nst(J)) {
    constexpr int HB = S::hb(J);
    constexpr int SP = RB * J + ST;
    constexpr int B = (LOGN2 - 1 - SP) - HB;
    fwd_stage2<A, RB, B, SP, HB, (HB >= LOGN2 - RB)>(ar, va, vb, tw, base, tt);
    fwd_round_stages2<A, LOGN2, RB, J, ST + 1>(ar, va, vb, tw, base, tt);
  }
}

template <class A, int LOGN2, int RB, int J>
__device__ __forceinline__ void row_forward2_from(const A& ar, typename A::V (&va)[1 << RB],
                                                  typename A::V (&vb)[1 << RB],
                                                  const typename A::TW* __restrict__ tw,
                                                  uint32_t base, uint32_t tt, typename A::V* lds) {
  using S = RowShape<LOGN2, RB>;
  if constexpr (J < S::K) {
    fwd_round_stages2<A, LOGN2, RB, J, 0>(ar, va, vb, tw, base, tt);
    if constexpr (J + 1 < S::K) {
      if constexpr (A::kCenterRounds) {
#pragma unroll
        for (int u = 0; u < S::R; ++u) {
          ar.center(va[u]);
          ar.center(vb[u]);
        }
      }
      // one LDS region: the two re-deals take turns
      lds_exchange<A, LOGN2, RB, J, J + 1>(va, lds, tt);
      lds_exchange<A, LOGN2, RB, J, J + 1>(vb, lds, tt);
      row_forward2_from<A, LOGN2, RB, J + 1>(ar, va, vb, tw, base, tt, lds);
    }
  }
}

// Chunk bookkeeping shared by the row kernels.
struct ChunkPos {
  uint64_t off;     // word offset of the chunk
  uint32_t limb;
  uint32_t base;    // (N1 + c): twiddle base of this chunk
  bool valid;
};

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD x runs a contiguous range of chunk indices:
// chunks are ordered polynomial-fastest, so the polynomials that share a
// modulus (and its twiddle table) run on one XCD back to back, and each XCD
// needs the tables of only 1/8 of the limbs.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
  const uint32_t per = nblocks / kXcds;
  if (b >= per * kXcds) return b;
  return (b % kXcds) * per + b / kXcds;
}

// ONE: the launch's class holds one limb, given in the arguments (a.limb0).
template <bool ONE = false>
__device__ __forceinline__ ChunkPos chunk_pos(const RowArgs& a, uint32_t gc, int log_n2) {
  ChunkPos p;
  p.valid = gc < a.total_chunks;
  const uint32_t g = p.valid ? gc : 0;
  const uint32_t n1 = 1u << a.log_n1;
  const uint32_t poly = g % a.batch;
  const uint32_t rest = g / a.batch;
  const uint32_t c = rest & (n1 - 1);
  const uint32_t li = rest >> a.log_n1;
  p.limb = ONE ? a.limb0 : a.cls_limbs[li];
  p.off = ((uint64_t)poly * a.L + p.limb) << a.log_n;
  p.off += (uint64_t)c << log_n2;
  p.base = n1 + c;
  return p;
}

// ---------------------------------------------------------------------------
// Row pass on one chunk of N2 = 2^LOGN2 words.  `dst`/`src` point at the
// chunk (always a readable one: threads without a chunk of their own pass
// chunk 0 and valid = false, so loads need no guard and only stores are
// skipped); `base` = N1 + c is its twiddle base, `tt` the thread's index within
// the chunk's N2/R threads (R = 2^RB values each), `lds` the chunk's LDS
// region.  All threads of the workgroup must call it together (it
// synchronises the workgroup).
// INV selects the direction; TWO_PASS says whether a column pass precedes
// (forward) or follows (inverse): then the pass reads/writes the raw
// intermediate format instead of canonical words, and the inverse leaves the
// N^-1 scaling to the column pass.
template <class A, int LOGN2, bool INV, bool TWO_PASS, int RB = 4>
__device__ __forceinline__ void row_chunk(typename A::W* __restrict__ dst,
                                          const typename A::W* __restrict__ src, const LimbDev& ld,
                                          uint32_t base, uint32_t tt, typename A::V* lds,
                                          bool valid) {
  using S = RowShape<LOGN2, RB>;
  constexpr int R = S::R;
  using V = typename A::V;
  using W = typename A::W;
  const A ar(ld);
  // When a chunk spans whole waves (N2/R a multiple of 64), the chunk's twiddle
  // base and tables are the same in every lane of a wave; say so, so the first
  // round's twiddles are scalar loads.
  const typename A::TW* twf = reinterpret_cast<const typename A::TW*>(ld.twf);
  const typename A::TW* twi = reinterpret_cast<const typename A::TW*>(ld.twi);
  if constexpr (S::TPC % 64 == 0) {
    base = __builtin_amdgcn_readfirstlane(base);
    twf = uniform_ptr(twf);
    twi = uniform_ptr(twi);
  }
  V v[R];
  if constexpr (!INV) {
    constexpr int H0 = S::hb(0);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const W x = src[ins_bits<RB>(tt, u, H0)];
      v[u] = TWO_PASS ? ar.from_raw(x) : ar.from_word(x);
    }
    const auto* tw = twf;
    row_forward_from<A, LOGN2, RB, 0>(ar, v, tw, base, tt, lds);
    if constexpr (S::K > 1) {
      // The last round holds R consecutive words per thread; re-deal them
      // through LDS so that each store instruction writes contiguous words.
      using MB = LdsMap<RB, 0>;
      const uint32_t bb = MB::base(tt);
#pragma unroll
      for (int u = 0; u < R; ++u) lds[MB::slot(tt, bb, u)] = v[u];
      __syncthreads();
      if (valid) {
#pragma unroll
        for (int u = 0; u < R; ++u) dst[tt + u * S::TPC] = ar.to_word(lds[S::tail_slot(tt, u)]);
      }
      __syncthreads();
    } else if (valid) {
#pragma unroll
      for (int u = 0; u < R; ++u) dst[u] = ar.to_word(v[u]);
    }
  } else {
    if constexpr (S::K > 1) {
      // Contiguous loads into LDS, then each thread takes R consecutive words.
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const W x = src[tt + u * S::TPC];
        V t = ar.from_word(x);
        ar.center(t);
        lds[S::tail_slot(tt, u)] = t;
      }
      __syncthreads();
      using MB = LdsMap<RB, 0>;
      const uint32_t bb = MB::base(tt);
#pragma unroll
      for (int u = 0; u < R; ++u) v[u] = lds[MB::slot(tt, bb, u)];
      __syncthreads();
    } else {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const W x = src[u];
        v[u] = ar.from_word(x);
        ar.center(v[u]);
      }
    }
    const auto* tw = twi;
    row_inverse_from<A, LOGN2, RB, S::K - 1, !TWO_PASS>(ar, v, tw, base, tt, lds, ld);
    constexpr int H0 = S::hb(0);
    if (valid) {
#pragma unroll
      for (int u = 0; u < R; ++u)
        dst[ins_bits<RB>(tt, u, H0)] = TWO_PASS ? ar.to_raw(v[u]) : ar.to_word(v[u]);
    }
  }
}

// Radix-16 rows: ask for four waves per SIMD (<= 128 VGPRs); the LDS of four
// workgroups per CU allows no more anyway.
template <class A, int LOGN2, bool INV, bool TWO_PASS, int RB = 4>
__global__ void __launch_bounds__((RowShape<LOGN2, RB>::BLOCK), (RB == 4 ? 4 : 1))
row_kernel(RowArgs args) {
  using S = RowShape<LOGN2, RB>;
  using V = typename A::V;
  using W = typename A::W;
  __shared__ V lds_all[S::LDS_ELEMS];
  const uint32_t ci = S::CPW == 1 ? 0u : threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
  const uint32_t gc = xcd_block(blockIdx.x, gridDim.x) * S::CPW + ci;
  if constexpr (RB == 2) {
    // Radix-4 rows serve short launches, where the dependent loads of the limb
    // list and constants are a visible part of the launch: one limb comes from
    // the arguments.
    if (args.n_cls == 1) {
      const ChunkPos cp = chunk_pos<true>(args, gc, LOGN2);
      row_chunk<A, LOGN2, INV, TWO_PASS, RB>(reinterpret_cast<W*>(args.dst) + cp.off,
                                         reinterpret_cast<const W*>(args.src) + cp.off, args.one,
                                         cp.base, tt, lds_all + ci * S::CHUNK_LDS, cp.valid);
      return;
    }
  }
  const ChunkPos cp = chunk_pos(args, gc, LOGN2);
  row_chunk<A, LOGN2, INV, TWO_PASS, RB>(reinterpret_cast<W*>(args.dst) + cp.off,
                                     reinterpret_cast<const W*>(args.src) + cp.off,
                                     args.limbs[cp.limb], cp.base, tt,
                                     lds_all + ci * S::CHUNK_LDS, cp.valid);
}

// Second half of the fused product on one row chunk: the pointwise product of
// the two forward-transformed register sets, then the inverse rounds, then the
// store (raw intermediate format with TWO_PASS, canonical words otherwise).
template <class A, int LOGN2, bool TWO_PASS, int RB>
__device__ __forceinline__ void product_inverse(const A& ar, typename A::V (&va)[1 << RB],
                                                const typename A::V (&vb)[1 << RB],
                                                typename A::W* __restrict__ dst,
                                                const LimbDev& ld,
                                                const typename A::TW* __restrict__ twi,
                                                uint32_t base, uint32_t tt, typename A::V* lds,
                                                bool valid) {
  using S = RowShape<LOGN2, RB>;
  constexpr int R = S::R;
  constexpr int H0 = S::hb(0);
#pragma unroll
  for (int u = 0; u < R; ++u) {
    va[u] = ar.mul(va[u], vb[u]);
    ar.center(va[u]);
  }
  row_inverse_from<A, LOGN2, RB, S::K - 1, !TWO_PASS>(ar, va, twi, base, tt, lds, ld);
  if (valid) {
#pragma unroll
    for (int u = 0; u < R; ++u)
      dst[ins_bits<RB>(tt, u, H0)] = TWO_PASS ? ar.to_raw(va[u]) : ar.to_word(va[u]);
  }
}

// The whole fused product on one row chunk (the body of polymul_row_kernel for
// callers that place chunks themselves): sa, sb and dst point at the chunk
// (dst may equal sa); `base`, `tt`, `lds` and `valid` as for row_chunk.
template <class A, int LOGN2, bool TWO_PASS, int RB = 4>
__device__ __forceinline__ void polymul_chunk(typename A::W* __restrict__ dst,
                                              const typename A::W* sa, const typename A::W* sb,
                                              const LimbDev& ld, uint32_t base, uint32_t tt,
                                              typename A::V* lds, bool valid) {
  using S = RowShape<LOGN2, RB>;
  constexpr int R = S::R;
  using V = typename A::V;
  using W = typename A::W;
  const A ar(ld);
  const auto* twf = reinterpret_cast<const typename A::TW*>(ld.twf);
  const auto* twi = reinterpret_cast<const typename A::TW*>(ld.twi);
  if constexpr (S::TPC % 64 == 0) {
    base = __builtin_amdgcn_readfirstlane(base);
    twf = uniform_ptr(twf);
    twi = uniform_ptr(twi);
  }
  constexpr int H0 = S::hb(0);
  V va[R], vb[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const W x = sa[ins_bits<RB>(tt, u, H0)];
    const W y = sb[ins_bits<RB>(tt, u, H0)];
    va[u] = TWO_PASS ? ar.from_raw(x) : ar.from_word(x);
    vb[u] = TWO_PASS ? ar.from_raw(y) : ar.from_word(y);
  }
  row_forward2_from<A, LOGN2, RB, 0>(ar, va, vb, twf, base, tt, lds);
  product_inverse<A, LOGN2, TWO_PASS, RB>(ar, va, vb, dst, ld, twi, base, tt, lds, valid);
}

// Fused negacyclic product on one row chunk: forward(a), forward(b), pointwise
// product, inverse -- Eq. (1) without leaving registers/LDS.  With TWO_PASS
// the inputs are column-pass outputs and the result still needs the inverse
// column pass.
// FWDMUL: forward-and-multiply rows instead: a (src, in place through dst) and b
// (src2, in place) are written back transformed and their elementwise product
// goes to dst2, all in the forward's output order (no inverse).
template <class A, int LOGN2, bool TWO_PASS, int RB = 4, bool FWDMUL = false>
__global__ void __launch_bounds__((RowShape<LOGN2, RB>::BLOCK))
polymul_row_kernel(RowArgs args) {
  using S = RowShape<LOGN2, RB>;
  constexpr int R = S::R;
  using V = typename A::V;
  using W = typename A::W;
  __shared__ V lds_all[S::LDS_ELEMS];
  const uint32_t ci = S::CPW == 1 ? 0u : threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
  ChunkPos cp = chunk_pos(args, xcd_block(blockIdx.x, gridDim.x) * S::CPW + ci, LOGN2);
  const LimbDev& ld = args.limbs[cp.limb];
  const A ar(ld);
  V* lds = lds_all + ci * S::CHUNK_LDS;
  const W* __restrict__ sa = reinterpret_cast<const W*>(args.src) + cp.off;
  const W* __restrict__ sb = reinterpret_cast<const W*>(args.src2) + cp.off;
  W* __restrict__ dst = reinterpret_cast<W*>(args.dst) + cp.off;
  const auto* twf = reinterpret_cast<const typename A::TW*>(ld.twf);
  const auto* twi = reinterpret_cast<const typename A::TW*>(ld.twi);
  if constexpr (S::TPC % 64 == 0) {  // a chunk spans whole waves: wave-uniform base and tables
    cp.base = __builtin_amdgcn_readfirstlane(cp.base);
    twf = uniform_ptr(twf);
    twi = uniform_ptr(twi);
  }
  constexpr int H0 = S::hb(0);
  V va[R], vb[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const W x = sa[ins_bits<RB>(tt, u, H0)];
    const W y = sb[ins_bits<RB>(tt, u, H0)];
    va[u] = TWO_PASS ? ar.from_raw(x) : ar.from_word(x);
    vb[u] = TWO_PASS ? ar.from_raw(y) : ar.from_word(y);
  }
  row_forward2_from<A, LOGN2, RB, 0>(ar, va, vb, twf, cp.base, tt, lds);
  if constexpr (FWDMUL) {
    // Thread tt holds positions tt*R + u; each of the three results goes through
    // the (free) LDS region once so that every store instruction is contiguous.
    W* __restrict__ da = reinterpret_cast<W*>(args.dst) + cp.off;
    W* __restrict__ db = reinterpret_cast<W*>(const_cast<void*>(args.src2)) + cp.off;
    W* __restrict__ dp = reinterpret_cast<W*>(args.dst2) + cp.off;
    auto put = [&](W* __restrict__ d, const V (&x)[R]) {
      if constexpr (S::K > 1) {
        using MB = LdsMap<RB, 0>;
        const uint32_t bb = MB::base(tt);
#pragma unroll
        for (int u = 0; u < R; ++u) lds[MB::slot(tt, bb, u)] = x[u];
        __syncthreads();
        if (cp.valid) {
#pragma unroll
          for (int u = 0; u < R; ++u) d[tt + u * S::TPC] = ar.to_word(lds[S::tail_slot(tt, u)]);
        }
        __syncthreads();
      } else if (cp.valid) {
#pragma unroll
        for (int u = 0; u < R; ++u) d[u] = ar.to_word(x[u]);
      }
    };
    put(da, va);
    put(db, vb);
#pragma unroll
    for (int u = 0; u < R; ++u) va[u] = ar.mul(va[u], vb[u]);  // a is written; reuse
    put(dp, va);
    return;
  }
  product_inverse<A, LOGN2, TWO_PASS, RB>(ar, va, vb, dst, ld, twi, cp.base, tt, lds, cp.valid);
}

// ---------------------------------------------------------------------------
// Column pass: one thread owns one column of N1 = 2^LOGN1 elements; a
// workgroup holds 64, 128 or kColBlock columns (the launch chooses).
constexpr int kColBlock = 256;

// One column of N1 = 2^LOGN1 words at src[k << log_n2], k < N1, written to the
// same positions of dst.  Runs all of the column's stages in registers.
template <class A, int LOGN1, bool INV, bool TWO_PASS>
__device__ __forceinline__ void col_one(typename A::W* __restrict__ dst,
                                        const typename A::W* __restrict__ src, const LimbDev& ld,
                                        uint32_t log_n2, bool valid) {
  using V = typename A::V;
  using W = typename A::W;
  using TW = typename A::TW;
  constexpr int N1 = 1 << LOGN1;
  const A ar(ld);
  V v[N1];
  if constexpr (!INV) {
    const NTT_GLOBAL TW* tw = gptr(reinterpret_cast<const TW*>(ld.twf));
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const W x = src[(uint64_t)k << log_n2];
      v[k] = ar.from_word(x);
    }
#pragma unroll
    for (int s = 0; s < LOGN1; ++s) {
      const int t = N1 >> (s + 1);
#pragma unroll
      for (int i = 0; i < (1 << s); ++i) {
        const TW w = load1<TW>(tw + (1 << s) + i);
#pragma unroll
        for (int j = 0; j < t; ++j) ar.ct(v[2 * i * t + j], v[2 * i * t + j + t], w);
      }
      if constexpr (A::kCenterRounds) {
        if ((s & 3) == 3 && s + 1 < LOGN1) {
#pragma unroll
          for (int k = 0; k < N1; ++k) ar.center(v[k]);
        }
      }
    }
    if (valid) {
#pragma unroll
      for (int k = 0; k < N1; ++k)
        dst[(uint64_t)k << log_n2] = TWO_PASS ? ar.to_raw(v[k]) : ar.to_word(v[k]);
    }
  } else {
    const NTT_GLOBAL TW* tw = gptr(reinterpret_cast<const TW*>(ld.twi));
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const W x = src[(uint64_t)k << log_n2];
      v[k] = TWO_PASS ? ar.from_raw(x) : ar.from_word(x);
      ar.center(v[k]);
    }
#pragma unroll
    for (int s = LOGN1 - 1; s >= 0; --s) {
      const int t = N1 >> (s + 1);
      if (s == 0) {
        TW w{};
#pragma unroll
        for (int j = 0; j < t; ++j) ar.gs_fold(v[j], v[j + t], w, ld);
      } else {
#pragma unroll
        for (int i = 0; i < (1 << s); ++i) {
          const TW w = load1<TW>(tw + (1 << s) + i);
#pragma unroll
          for (int j = 0; j < t; ++j) ar.gs(v[2 * i * t + j], v[2 * i * t + j + t], w);
        }
      }
      if constexpr (A::kCenterRounds) {
        if (((LOGN1 - 1 - s) & 3) == 3 && s > 0) {
#pragma unroll
          for (int k = 0; k < N1; ++k) ar.center(v[k]);
        }
      }
    }
    if (valid) {
#pragma unroll
      for (int k = 0; k < N1; ++k) dst[(uint64_t)k << log_n2] = ar.to_word(v[k]);
    }
  }
}

// ONE: the launch's class holds one limb (n_cls == 1), whose index and constants
// come from the arguments; its twiddles are then wave-uniform loads.
// ROWS: the launch may carry row tables (ColArgs::src_rows and the others).
template <class A, int LOGN1, bool INV, bool TWO_PASS, bool ONE = false, bool ROWS = false>
__global__ void __launch_bounds__(kColBlock)
col_kernel(ColArgs args) {
  using W = typename A::W;
  uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  void* dst_base = args.dst;
  const void* src_base = args.src;
  const uint64_t* src_rows = ROWS ? args.src_rows : nullptr;
  const uint64_t* dst_rows = ROWS ? args.dst_rows : nullptr;
  if ((args.src2 || (ROWS && args.src2_rows)) && gid >= args.total_cols) {
    gid -= args.total_cols;
    dst_base = args.dst2;
    src_base = args.src2;
    src_rows = ROWS ? args.src2_rows : nullptr;
    dst_rows = nullptr;
  }
  const bool valid = gid < args.total_cols;
  const uint32_t g = valid ? gid : 0;
  const uint32_t n2 = 1u << args.log_n2;
  const uint32_t r = g & (n2 - 1);
  const uint32_t rest = g >> args.log_n2;
  // the column's words in its limb-row (poly * L + limb) of src and dst
  auto at = [&](uint64_t row, W** d, const W** sp) {
    *d = reinterpret_cast<W*>(dst_base) + (row << args.log_n) + r;
    *sp = reinterpret_cast<const W*>(src_base) + (row << args.log_n) + r;
    if constexpr (ROWS) {
      if (dst_rows) *d = reinterpret_cast<W*>(dst_rows[row]) + r;
      if (src_rows) *sp = reinterpret_cast<const W*>(src_rows[row]) + r;
    }
  };
  W* d;
  const W* sp;
  if constexpr (ONE) {
    at((uint64_t)rest * args.L + args.limb0, &d, &sp);
    col_one<A, LOGN1, INV, TWO_PASS>(d, sp, args.one, args.log_n2, valid);
  } else {
    const uint32_t li = rest % args.n_cls;
    const uint32_t poly = rest / args.n_cls;
    const uint32_t limb = args.cls_limbs[li];
    at((uint64_t)poly * args.L + limb, &d, &sp);
    col_one<A, LOGN1, INV, TWO_PASS>(d, sp, args.limbs[limb], args.log_n2, valid);
  }
}

// ---------------------------------------------------------------------------
// VEC consecutive words at p: one 16-byte access when VEC words make 16 bytes
// (the caller guarantees 16-byte alignment then), else VEC word accesses.
template <class W, int VEC>
__device__ __forceinline__ void load_words(W (&x)[VEC], const W* p_in) {
  if constexpr (VEC * sizeof(W) == 16) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = *(const NTT_GLOBAL u32x4*)p_in;
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      if constexpr (sizeof(W) == 8) x[k] = (W)d[2 * k] | ((W)d[2 * k + 1] << 32);
      else x[k] = (W)d[k];
    }
  } else {
    const NTT_GLOBAL W* p = (const NTT_GLOBAL W*)p_in;
#pragma unroll
    for (int k = 0; k < VEC; ++k) x[k] = p[k];
  }
}

template <class W, int VEC>
__device__ __forceinline__ void store_words(W* p_out, const W (&x)[VEC]) {
  if constexpr (VEC * sizeof(W) == 16) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    uint32_t d[4];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      if constexpr (sizeof(W) == 8) {
        d[2 * k] = (uint32_t)x[k];
        d[2 * k + 1] = (uint32_t)(x[k] >> 32);
      } else {
        d[k] = (uint32_t)x[k];
      }
    }
    u32x4 v;
    v.x = d[0];
    v.y = d[1];
    v.z = d[2];
    v.w = d[3];
    *(NTT_GLOBAL u32x4*)p_out = v;
  } else {
    NTT_GLOBAL W* p = (NTT_GLOBAL W*)p_out;
#pragma unroll
    for (int k = 0; k < VEC; ++k) p[k] = x[k];
  }
}

// Elementwise product c = a (.) b on [batch][L][N] (NTT domain).  Each thread
// takes VEC consecutive words of one limb-row: VEC = 16 / sizeof(word) gives one
// 16-byte load per operand and one 16-byte store (the host picks VEC = 1 when N
// is shorter or a pointer is not 16-byte aligned).
constexpr int kEltBlock = 256;

template <class A, int VEC>
__global__ void __launch_bounds__(kEltBlock)
pointwise_kernel(EltArgs args) {
  using W = typename A::W;
  const uint32_t e = (blockIdx.x * kEltBlock + threadIdx.x) * VEC;
  if (e >= args.total) return;
  const uint32_t row = e >> args.log_n;
  const uint32_t li = row % args.n_cls;
  const uint32_t poly = row / args.n_cls;
  const uint32_t limb = args.cls_limbs[li];
  const A ar(args.limbs[limb]);
  const uint64_t off = (((uint64_t)poly * args.L + limb) << args.log_n) +
                       (e & ((1u << args.log_n) - 1u));
  W x[VEC], y[VEC], z[VEC];
  load_words<W, VEC>(x, reinterpret_cast<const W*>(args.a) + off);
  load_words<W, VEC>(y, reinterpret_cast<const W*>(args.b) + off);
#pragma unroll
  for (int k = 0; k < VEC; ++k) z[k] = ar.to_word(ar.mul(ar.from_word(x[k]), ar.from_word(y[k])));
  store_words<W, VEC>(reinterpret_cast<W*>(args.dst) + off, z);
}

// Grouped multiply-accumulate (external-product MAC in the NTT domain):
// out[g][c] = sum over rows r present in group g of a[g*rows + r] (.) key[r][c].
// One thread per VEC consecutive words of one (group, column, limb) row.  Rows
// are taken kMacRows at a time with every load issued before the products (the
// rows beyond the group's end are computed and dropped by a select, so no
// branch holds a load back).
constexpr int kMacRows = 8;

template <class A, int VEC>
__global__ void __launch_bounds__(kEltBlock)
mac_kernel(MacArgs args) {
  using W = typename A::W;
  using V = typename A::V;
  const uint32_t e = (blockIdx.x * kEltBlock + threadIdx.x) * VEC;
  if (e >= args.total) return;
  const uint32_t row = e >> args.log_n;  // (group * cols + c) * n_cls + li
  const uint32_t li = row % args.n_cls;
  const uint32_t gc = row / args.n_cls;
  const uint32_t c = gc % args.cols;
  const uint32_t grp = gc / args.cols;
  const uint32_t limb = args.cls_limbs[li];
  const A ar(args.limbs[limb]);
  const uint64_t poly_words = (uint64_t)args.L << args.log_n;
  const uint64_t limb_off = ((uint64_t)limb << args.log_n) + (e & ((1u << args.log_n) - 1u));
  const uint32_t first = grp * args.rows;
  const uint32_t nr = min(args.rows, args.num_operands - first);
  const W* a = reinterpret_cast<const W*>(args.a);
  const W* key = reinterpret_cast<const W*>(args.key);
  V acc[VEC];
  for (uint32_t r0 = 0; r0 < nr; r0 += kMacRows) {
    W x[kMacRows][VEC], k[kMacRows][VEC];
#pragma unroll
    for (int i = 0; i < kMacRows; ++i) {
      const uint32_t r = r0 + i < nr ? r0 + i : r0;  // in range; dropped below
      load_words<W, VEC>(x[i], a + (uint64_t)(first + r) * poly_words + limb_off);
      load_words<W, VEC>(k[i], key + ((uint64_t)r * args.cols + c) * poly_words + limb_off);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load above the products
#pragma unroll
    for (int i = 0; i < kMacRows; ++i) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const V prod = ar.mul(ar.from_word(x[i][v]), ar.from_word(k[i][v]));
        const V sum = (r0 + i == 0) ? prod : ar.add(acc[v], prod);
        acc[v] = (r0 + i < nr) ? sum : acc[v];
      }
    }
  }
  W z[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) z[v] = ar.to_word(acc[v]);
  store_words<W, VEC>(reinterpret_cast<W*>(args.dst) + (uint64_t)gc * poly_words + limb_off, z);
}

}  // namespace nttk
