// bconv.hip -- RNS basis conversion (BConv; Sec. III lists it among the CKKS
// operators around the NTT, the other half of key switching's ModUp/ModDown).
//
// x[batch][L][N] holds residues of X modulo q_0..q_(L-1); the output
// y[batch][M][N] holds, modulo each p_j,
//     sum_i [x_i (Q/q_i)^-1 mod q_i] * (Q/q_i mod p_j)         (Q = prod q_i)
// which is X + alpha Q for one integer 0 <= alpha < L (fast conversion, alpha
// not corrected).
//
// One thread per (polynomial, coefficient).  Output moduli go in chunks of
// kBconvChunk: for each chunk the thread walks the L source residues of its
// coefficient (lanes with consecutive coefficients read consecutive words),
// forms t_i = x_i w_i mod q_i and adds t_i (Q/q_i mod p_j) into the chunk's
// accumulators, then stores one coalesced word per output modulus.  Every
// constant is the same for all lanes (scalar loads) and every product has a
// constant operand, so all products are Shoup products with precomputed
// companions.  Re-forming t_i per chunk costs L products per chunk on top of
// the L M of the sum (+1/8) and keeps the registers to the chunk's accumulators
// whatever L and M are.  The work is VALU-bound for dozens of limbs, not
// HBM-bound.
//
// When every modulus is below 2^50 - 2^10 the products run on the fp64 FMA
// units instead (the exact product of the fp64 arithmetic classes: high part,
// FMA error term, rounded quotient): a handful of full-rate fp64 operations
// against some ten quarter-rate 32-bit multiplies for a 64-bit Shoup product.
// Each term lies in (-7/8 p, 7/8 p), so eight of them are summed exactly in a
// double before the sum is centred again.
//
// In that case the sum itself, a dense L x M contraction per coefficient, goes
// to the int8 matrix cores.  Every t_i < 2^50 is written in balanced base-256
// digits d_0..d_6 (d_a in [-128, 128) below the top, t = sum_a d_a 256^a), and
// so is every constant m'_(i,a),j = (Q/q_i mod p_j) 256^a mod p_j (digits
// e_0..e_6).  Then for each output modulus
//     sum_i t_i (Q/q_i mod p_j) = sum_c 256^c D_c (mod p_j),
//     D_c = sum_(i,a) d_a(t_i) e_c(m'_(i,a),j),
// and the D_c are products of int8 matrices with exact int32 sums
// (|D_c| <= 512 * 128 * 128 = 2^23).  The digits of t_i are one byte each of
// z_i = (t_i + 128 (1 + 256 + ... + 256^5)) XOR 0x808080808080: eight bytes per
// limb, the eighth zero, so one 64-bit word is one MFMA operand.  With
// coefficients as the MFMA's columns and (output, digit c) as its rows, a lane
// ends up with four D_c of four outputs for its own coefficient; four fp64
// products with 256^c mod p_j, one exchange with the lane 32 away, and a
// coalesced store finish the conversion.  The matrix work is 64 L M int8 MACs
// per coefficient (about 10 us for 36 -> 36 limbs on 2^18 coefficients at the
// dense int8 rate); the rest is the L x N reads and M x N writes.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "ntt_internal.hpp"
#include "numtheory.hpp"

struct ntt_bconv_s {
  int device = 0;
  uint32_t N = 0, log_n = 0, L = 0, M = 0, word_bits = 0;
  uint64_t* d_c1 = nullptr;  // [L][3]: q_i, w_i = (Q/q_i)^-1 mod q_i, floor(w_i 2^64 / q_i)
  uint64_t* d_c2 = nullptr;  // [L][M][2]: (Q/q_i) mod p_j and its Shoup companion
  uint64_t* d_p = nullptr;   // [M]
  bool f64 = false;          // every modulus < 2^50 - 2^10: fp64 products
  double* d_f1 = nullptr;    // [L][4]: q_i, 1/q_i, w_i, w_i/q_i
  double* d_f2 = nullptr;    // [L][M][2]: (Q/q_i) mod p_j, that over p_j
  double* d_fp = nullptr;    // [M][2]: p_j, 1/p_j
  bool mfma = false;         // fp64-eligible, N >= 32, not switched off: int8 MFMA form
  uint64_t* d_kop = nullptr; // MFMA constant operands [ceil(M/4)][ceil(L/2)][64 lanes]
  double* d_om = nullptr;    // [M][8][2]: 256^c mod p_j and that over p_j
  double* d_om2 = nullptr;   // [M][4]: p_j, 1/p_j, 2^32 mod p_j, that over p_j
  uint32_t ws_grid = 0;      // workgroups of the weights-stationary kernel (0: not used)
};

// The two conversions of key switching between Q = prod q_i and the special
// modulus P = prod p_k, with the scale of ModDown.
struct ntt_basis_ext_s {
  uint32_t N = 0, log_n = 0, L = 0, K = 0, word_bits = 0;
  ntt_bconv_s* up = nullptr;    // Q -> P
  ntt_bconv_s* down = nullptr;  // P -> Q
  uint64_t* d_sc = nullptr;     // [L][2]: s_i = P^-1 mod q_i, floor(s_i 2^64 / q_i)
  double* d_sf = nullptr;       // [L][2]: s_i, s_i / q_i (fp64 classes)
};

namespace nttk {

struct BconvArgs {
  void* out;
  const void* in;
  const uint64_t* c1;
  const uint64_t* c2;
  const uint64_t* p;
  const double* f1;
  const double* f2;
  const double* fp;
  const uint64_t* kop;
  const double* om;
  const double* om2;
  uint32_t L, M, log_n;
  uint32_t total;        // batch * N threads
  uint64_t in_stride;    // words from one polynomial of `in` to the next
  uint64_t out_stride;   // words from one polynomial of `out` to the next
  // ModUp: every source residue the kernel reads is also written to
  // copy[b * aux_stride + i N + n].  ModDown: output j becomes
  // (sub[b * aux_stride + j N + n] - y_j) s_j mod p_j.
  void* copy;
  const void* sub;
  uint64_t aux_stride;
  const uint64_t* sc;    // [M][2]: s_j and floor(s_j 2^64 / p_j)   (ModDown)
  const double* sf;      // [M][2]: s_j and s_j / p_j               (ModDown)
};

// What a conversion kernel does around the sum (the template argument MODE).
constexpr int kBconvPlain = 0;  // y_j
constexpr int kBconvUp = 1;     // y_j, and the source residues copied beside them
constexpr int kBconvDown = 2;   // (x_j - y_j) s_j mod p_j

constexpr uint32_t kBconvBlock = 256;

// y w mod q up to one q: y w - floor(y ws / 2^64) q lies in [0, 2q) for any
// 64-bit y when w < q < 2^63 and ws = floor(w 2^64 / q).
__device__ __forceinline__ uint64_t shoup2(uint64_t y, uint64_t w, uint64_t ws, uint64_t q) {
  return y * w - __umul64hi(y, ws) * q;
}

constexpr int kBconvChunk = 8;

template <class W, int MODE>
__global__ void __launch_bounds__(kBconvBlock) bconv_kernel(BconvArgs a) {
  constexpr int JB = kBconvChunk;
  const uint32_t gid = blockIdx.x * kBconvBlock + threadIdx.x;
  if (gid >= a.total) return;
  const uint32_t n = gid & ((1u << a.log_n) - 1u);
  const uint32_t b = gid >> a.log_n;
  const W* x = static_cast<const W*>(a.in) + (uint64_t)b * a.in_stride + n;
  W* y = static_cast<W*>(a.out) + (uint64_t)b * a.out_stride + n;
  for (uint32_t j0 = 0; j0 < a.M; j0 += JB) {
    const uint32_t jn = a.M - j0 < (uint32_t)JB ? a.M - j0 : (uint32_t)JB;
    uint64_t acc[JB];  // each < 2p_j (p < 2^62: acc + product < 4p < 2^64)
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) acc[jj] = 0;
    for (uint32_t i = 0; i < a.L; ++i) {
      const uint64_t q = a.c1[3 * i], w = a.c1[3 * i + 1], ws = a.c1[3 * i + 2];
      const W xi = x[(uint64_t)i << a.log_n];
      if (MODE == kBconvUp && j0 == 0)
        static_cast<W*>(a.copy)[(uint64_t)b * a.aux_stride + ((uint64_t)i << a.log_n) + n] = xi;
      uint64_t t = shoup2((uint64_t)xi, w, ws, q);
      t = t >= q ? t - q : t;
      const uint64_t* ci = a.c2 + 2 * ((uint64_t)i * a.M + j0);
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        if ((uint32_t)jj < jn) {
          const uint64_t p2 = 2 * a.p[j0 + jj];
          acc[jj] += shoup2(t, ci[2 * jj], ci[2 * jj + 1], p2 >> 1);
          acc[jj] = acc[jj] >= p2 ? acc[jj] - p2 : acc[jj];
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      if ((uint32_t)jj < jn) {
        const uint32_t j = j0 + jj;
        const uint64_t p = a.p[j];
        uint64_t r = acc[jj] >= p ? acc[jj] - p : acc[jj];
        if (MODE == kBconvDown) {
          const uint64_t xs = static_cast<const W*>(a.sub)[(uint64_t)b * a.aux_stride +
                                                           ((uint64_t)j << a.log_n) + n];
          const uint64_t d = xs >= r ? xs - r : xs + (p - r);
          r = shoup2(d, a.sc[2 * j], a.sc[2 * j + 1], p);
          r = r >= p ? r - p : r;
        }
        y[(uint64_t)j << a.log_n] = (W)r;
      }
    }
  }
}

// x w mod q for x, w < q < 2^50 - 2^10 given wq = w/q: the exact value of
// x w - c q with c the rounded quotient, in (-7/8 q, 7/8 q).
__device__ __forceinline__ double f64_mulmod_pre(double x, double w, double wq, double q) {
  const double h = x * w;
  const double l = __builtin_fma(x, w, -h);
  const double c = __builtin_rint(x * wq);
  return __builtin_fma(-c, q, h) + l;
}

// The ModDown step on a reduced sum r in [0, p): (x - r) s mod p for the
// residue x in [0, p), with s < p < 2^50 - 2^10 and sq = s / p.  |x - r| < p,
// so the product is exact as for non-negative operands.
__device__ __forceinline__ double f64_sub_scale(double x, double r, double s, double sq, double p) {
  const double v = f64_mulmod_pre(x - r, s, sq, p);
  return v < 0.0 ? v + p : v;
}

template <class W, int MODE>
__global__ void __launch_bounds__(kBconvBlock) bconv_f64_kernel(BconvArgs a) {
  constexpr int JB = kBconvChunk;
  const uint32_t gid = blockIdx.x * kBconvBlock + threadIdx.x;
  if (gid >= a.total) return;
  const uint32_t n = gid & ((1u << a.log_n) - 1u);
  const uint32_t b = gid >> a.log_n;
  const W* x = static_cast<const W*>(a.in) + (uint64_t)b * a.in_stride + n;
  W* y = static_cast<W*>(a.out) + (uint64_t)b * a.out_stride + n;
  for (uint32_t j0 = 0; j0 < a.M; j0 += JB) {
    const uint32_t jn = a.M - j0 < (uint32_t)JB ? a.M - j0 : (uint32_t)JB;
    double acc[JB];  // |acc| < p/2 + 2 after each centring, < 2^53 between
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) acc[jj] = 0.0;
    for (uint32_t i = 0; i < a.L; ++i) {
      const double* f = a.f1 + 4 * i;
      const W xi = x[(uint64_t)i << a.log_n];
      if (MODE == kBconvUp && j0 == 0)
        static_cast<W*>(a.copy)[(uint64_t)b * a.aux_stride + ((uint64_t)i << a.log_n) + n] = xi;
      double t = f64_mulmod_pre((double)xi, f[2], f[3], f[0]);
      t = t < 0.0 ? t + f[0] : t;  // [x_i w_i]_(q_i) in [0, q_i)
      const double* fi = a.f2 + 2 * ((uint64_t)i * a.M + j0);
      const bool recentre = (i & 7u) == 7u;
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        if ((uint32_t)jj < jn) {
          const double p = a.fp[2 * (j0 + jj)];
          acc[jj] += f64_mulmod_pre(t, fi[2 * jj], fi[2 * jj + 1], p);
          if (recentre)
            acc[jj] = __builtin_fma(-__builtin_rint(acc[jj] * a.fp[2 * (j0 + jj) + 1]), p, acc[jj]);
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      if ((uint32_t)jj < jn) {
        const uint32_t j = j0 + jj;
        const double p = a.fp[2 * j], pinv = a.fp[2 * j + 1];
        double r = __builtin_fma(-__builtin_rint(acc[jj] * pinv), p, acc[jj]);
        r = r < 0.0 ? r + p : r;
        r = r >= p ? r - p : r;
        if (MODE == kBconvDown) {
          const W xs = static_cast<const W*>(a.sub)[(uint64_t)b * a.aux_stride +
                                                    ((uint64_t)j << a.log_n) + n];
          r = f64_sub_scale((double)xs, r, a.sf[2 * j], a.sf[2 * j + 1], p);
        }
        y[(uint64_t)j << a.log_n] = (W)(uint64_t)r;
      }
    }
  }
}

typedef int bconv_v16i __attribute__((ext_vector_type(16)));
constexpr uint64_t kDigitOffset = 0x808080808080ull;  // 128 at digits 0..5

// One wave per 32 coefficients of one polynomial (N >= 32); four waves per block.
// SMAX bounds the k-steps (two limbs each) so that the digit words and two sets
// of constant operands stay in registers.
template <class W, int SMAX, int MODE>
__global__ void __launch_bounds__(256) bconv_mfma_kernel(BconvArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t h = lane >> 5;    // which limb of a k-step / which digit half
  const uint32_t col = lane & 31u; // the lane's coefficient within the tile
  const uint32_t tile = (blockIdx.x * 4u + (threadIdx.x >> 6));
  const uint64_t g = (uint64_t)tile * 32u + col;
  if (tile * 32u >= a.total) return;  // whole waves leave together
  const uint32_t n = (uint32_t)(g & ((1u << a.log_n) - 1u));
  const uint64_t b = g >> a.log_n;
  const uint32_t steps = (a.L + 1u) >> 1;
  const W* x = static_cast<const W*>(a.in) + b * a.in_stride + n;
  // Digits of t_i = [x_i w_i]_(q_i) for the limbs i = 2s + h of this lane.
  uint64_t z[SMAX];
#pragma unroll
  for (int st = 0; st < SMAX; ++st) {
    z[st] = 0;
    const uint32_t i = 2u * st + h;
    if ((uint32_t)st < steps && i < a.L) {
      const double* f = a.f1 + 4 * i;
      const W xi = x[(uint64_t)i << a.log_n];
      if (MODE == kBconvUp)
        static_cast<W*>(a.copy)[b * a.aux_stride + ((uint64_t)i << a.log_n) + n] = xi;
      double t = f64_mulmod_pre((double)xi, f[2], f[3], f[0]);
      t = t < 0.0 ? t + f[0] : t;
      z[st] = ((uint64_t)t + kDigitOffset) ^ kDigitOffset;
    }
  }
  W* y = static_cast<W*>(a.out) + b * a.out_stride + n;
  const uint32_t row_tiles = (a.M + 3u) >> 2;
  const uint64_t* kop = a.kop + lane;
  // Indices are clamped into the table, so no load can leave it whatever the
  // compiler hoists; the unused words are zeroed.
  auto load_k = [&](uint64_t (&k)[SMAX], uint32_t rt) {
    const uint32_t rc = rt < row_tiles ? rt : row_tiles - 1u;
    const uint64_t* kr = kop + ((uint64_t)rc * steps) * 64u;
#pragma unroll
    for (int st = 0; st < SMAX; ++st) {
      const uint32_t sc = (uint32_t)st < steps ? (uint32_t)st : steps - 1u;
      if (rt < row_tiles && (uint32_t)st < steps) k[st] = kr[(uint64_t)sc * 64u];
      else k[st] = 0;
    }
  };
  auto products = [&](const uint64_t (&k)[SMAX]) {
    bconv_v16i acc = {};
#pragma unroll
    for (int st = 0; st < SMAX; ++st) {
      if ((uint32_t)st < steps)
        acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)k[st], (long)z[st], acc, 0, 0, 0);
    }
    return acc;
  };
  // Pipeline: the products of row tile rt + 1 and the operand loads of rt + 2
  // are issued before the vector work that finishes row tile rt.
  uint64_t ka[SMAX], kb[SMAX];
  load_k(ka, 0);
  bconv_v16i acc = products(ka);
  load_k(kb, 1);
  for (uint32_t rt = 0; rt < row_tiles; ++rt) {
    bconv_v16i acc2 = {};
    if (rt + 1 < row_tiles) acc2 = products(kb);
    load_k(ka, rt + 2);
    // acc[4 j' + c4] = D_(4h + c4) of output J = 4 rt + j' for this coefficient.
#pragma unroll
    for (int jp = 0; jp < 4; ++jp) {
      const uint32_t J = 4u * rt + jp;
      const uint32_t Jc = J < a.M ? J : a.M - 1u;  // in-table index for rows past M
      const double* om = a.om + 16 * (uint64_t)Jc + 8 * h;
      const double p = a.fp[2 * Jc], pinv = a.fp[2 * Jc + 1];
      double part = 0.0;
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4)
        part += f64_mulmod_pre((double)acc[4 * jp + c4], om[2 * c4], om[2 * c4 + 1], p);
      const double sum = part + __shfl_xor(part, 32);
      if (J < a.M && (uint32_t)(jp >> 1) == h) {
        double r = __builtin_fma(-__builtin_rint(sum * pinv), p, sum);
        r = r < 0.0 ? r + p : r;
        r = r >= p ? r - p : r;
        if (MODE == kBconvDown) {
          const W xs = static_cast<const W*>(a.sub)[b * a.aux_stride + ((uint64_t)J << a.log_n) + n];
          r = f64_sub_scale((double)xs, r, a.sf[2 * J], a.sf[2 * J + 1], p);
        }
        y[(uint64_t)J << a.log_n] = (W)(uint64_t)r;
      }
    }
    acc = acc2;
#pragma unroll
    for (int st = 0; st < SMAX; ++st) kb[st] = ka[st];
  }
}

// The weights-stationary form of the int8 matrix-core conversion, for at most
// 48 source and 48 target moduli (up to 12 row tiles).  A workgroup walks a
// contiguous run of tiles of 32 coefficients with two kinds of waves:
//   - owner wave w < row_tiles keeps the constant operands of row tile w
//     (outputs 4w .. 4w + 3, one 64-bit word per k-step) in registers for the
//     whole launch; per tile it runs its chain of k-step MFMAs on the tile's
//     digit words (from LDS) and finishes its four outputs: the four digit sums
//     D_(4h+c) a lane holds are combined exactly in fp64 (S = sum_c D_(4h+c)
//     256^c, |S| < 2^47.01); one swap of register halves between lanes 32
//     apart gives each half both sums of two of the outputs, and each lane
//     finishes two outputs as lo + hi 2^32 mod p (one exact product);
//   - the four helper waves load the source words three tiles ahead (two words
//     per load) and form the digit words of tile t + 2 into a third LDS buffer
//     while the owners work on tile t.
// So the matrix work of the owners and the vector work of the helpers run at
// the same time on each SIMD; one barrier per tile separates the buffers.
// Measured on 36 -> 36 limbs of 4 x 2^16 coefficients: 57 us, against 151 us
// for the streaming form above (bconv_mfma_kernel, which reloads the constant
// operands per row tile); ModUp 61 us, ModDown 81-88 us.
constexpr int kWsMaxTiles = 12;
constexpr uint32_t kWsMaxLimbs = 48;  // 24 k-steps of constant operands in registers
constexpr uint32_t kWsHelpers = 4;

// Exact conversions of integers below 2^52 between words and doubles (through
// the 2^52 exponent: two operations each way instead of a general conversion).
__device__ __forceinline__ double small_to_f64(uint64_t x) {
  return __builtin_bit_cast(double, x | 0x4330000000000000ull) - 4503599627370496.0;
}
__device__ __forceinline__ uint64_t f64_to_small(double r) {
  return __builtin_bit_cast(uint64_t, r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// IPT: coefficient pairs per helper thread (2 * steps * 16 over 256).
template <class W, int SMAX, int IPT, int MODE>
__global__ void __launch_bounds__(1024) bconv_ws_kernel(BconvArgs a) {
  extern __shared__ uint64_t zbuf[];  // [3][2 * steps][32] digit words, then [L][4] doubles
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
  const uint32_t steps = (a.L + 1u) >> 1, lp = 2u * steps;
  const uint32_t row_tiles = (a.M + 3u) >> 2;
  const uint32_t nmask = (1u << a.log_n) - 1u;
  const uint32_t tiles = a.total >> 5;
  // Workgroup b takes the contiguous tiles [b T, (b + 1) T), T = ceil(tiles / G):
  // each row of the input and output is then read and written in runs.
  const uint32_t per = (tiles + gridDim.x - 1u) / gridDim.x;
  const uint32_t first = blockIdx.x * per;
  const uint32_t end = first + per < tiles ? first + per : tiles;
  if (first >= end) return;  // the whole workgroup: no barrier is left waiting
  // Three LDS buffers: at step t the owners read the digits of tile t while
  // the helpers write those of tile t + 2.  After them, a copy of the source
  // limbs' constants (4 doubles each).
  auto buffer = [&](uint32_t t) { return zbuf + (t % 3u) * (lp * 32u); };
  {
    double* f1s = reinterpret_cast<double*>(zbuf + 3u * lp * 32u);
    for (uint32_t j = threadIdx.x; j < 4u * a.L; j += blockDim.x) f1s[j] = a.f1[j];
  }
  __syncthreads();

  if (wave < row_tiles) {
    // ---- owner wave: row tile `wave`
    const uint32_t h = lane >> 5, col = lane & 31u;
    uint64_t k[SMAX];
#pragma unroll
    for (int st = 0; st < SMAX; ++st)
      k[st] = (uint32_t)st < steps ? a.kop[((uint64_t)wave * steps + st) * 64u + lane] : 0ull;
    const uint32_t J0 = 4u * wave;
    // Every k-step runs: past the last one the constant operand is zero, and
    // the digit row read is clamped into the buffer.
    auto products = [&](const uint64_t* buf) {
      bconv_v16i acc = {};
#pragma unroll
      for (int st = 0; st < SMAX; ++st) {
        const uint32_t r2 = 2u * st < lp ? 2u * st : lp - 2u;
        const uint64_t zz = buf[(r2 + h) * 32u + col];
        acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)k[st], (long)zz, acc, 0, 0, 0);
      }
      return acc;
    };
    // Output J0 + 2h + s (s = 0, 1) is finished by the lanes of half h; its
    // constants stay in registers for the whole launch.
    double cp[2], cpinv[2], cw[2], cwq[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const uint32_t J = J0 + 2u * h + sl;
      const double* o = a.om2 + 4u * (uint64_t)(J < a.M ? J : a.M - 1u);
      cp[sl] = o[0];
      cpinv[sl] = o[1];
      cw[sl] = o[2];
      cwq[sl] = o[3];
    }
    // ModDown: the residues x_J of the two outputs this lane finishes, loaded
    // before the products so that their latency hides behind the MFMA chain.
    auto load_sub = [&](uint32_t tile, W (&xs)[2]) {
      const uint64_t g = (uint64_t)tile * 32u + col;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const uint32_t J = J0 + 2u * h + sl;
        const uint32_t Jc = J < a.M ? J : a.M - 1u;
        xs[sl] = static_cast<const W*>(a.sub)[(g >> a.log_n) * a.aux_stride + ((uint64_t)Jc << a.log_n) +
                                              (uint32_t)(g & nmask)];
      }
    };
    auto finish = [&](const bconv_v16i& acc, uint32_t tile, const W (&xs)[2]) {
      // S[jp]: this half's digit sums of output J0 + jp combined exactly
      // (|D_c| <= 2^23, so every partial sum is an integer below 2^48).
      double S[4];
#pragma unroll
      for (int jp = 0; jp < 4; ++jp) {
        double sm = __builtin_fma((double)acc[4 * jp + 3], 256.0, (double)acc[4 * jp + 2]);
        sm = __builtin_fma(sm, 256.0, (double)acc[4 * jp + 1]);
        S[jp] = __builtin_fma(sm, 256.0, (double)acc[4 * jp]);
      }
      const uint64_t g = (uint64_t)tile * 32u + col;
      const uint32_t n = (uint32_t)(g & nmask);
      const uint64_t b = g >> a.log_n;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        // Swap the upper half of S[sl] with the lower half of S[sl + 2]: then
        // half h holds the low (digits 0..3) and high (4..7) sums of output
        // J0 + 2h + sl, and the value is lo + hi 2^32 mod p.
        const uint64_t x = __builtin_bit_cast(uint64_t, S[sl]), y = __builtin_bit_cast(uint64_t, S[sl + 2]);
        const auto l32 = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)y, false, false);
        const auto h32 = __builtin_amdgcn_permlane32_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
        const double lo = __builtin_bit_cast(double, ((uint64_t)h32[0] << 32) | l32[0]);
        const double hi = __builtin_bit_cast(double, ((uint64_t)h32[1] << 32) | l32[1]);
        const double v = lo + f64_mulmod_pre(hi, cw[sl], cwq[sl], cp[sl]);  // |v| < 2^47.02 + p
        double r = __builtin_fma(-__builtin_rint(v * cpinv[sl]), cp[sl], v);
        r = r < 0.0 ? r + cp[sl] : r;
        const uint32_t J = J0 + 2u * h + sl;
        if (J < a.M) {
          if (MODE == kBconvDown) {
            r = f64_sub_scale(small_to_f64((uint64_t)xs[sl]), r, a.sf[2 * J], a.sf[2 * J + 1], cp[sl]);
          }
          static_cast<W*>(a.out)[b * a.out_stride + ((uint64_t)J << a.log_n) + n] = (W)f64_to_small(r);
        }
      }
    };
    __syncthreads();  // the digits of the first two tiles
    for (uint32_t t = 0; first + t < end; ++t) {
      W xs[2] = {0, 0};
      if (MODE == kBconvDown) load_sub(first + t, xs);
      finish(products(buffer(t)), first + t, xs);
      __syncthreads();
    }
    return;
  }

  // ---- helper waves: thread ht of 256 takes the coefficient pairs ht + 256 m
  // (pair index = limb * 16 + coefficient / 2), one 2-word load each.
  typedef W W2 __attribute__((ext_vector_type(2)));
  const uint32_t ht = threadIdx.x - 64u * row_tiles;
  // Loads are unconditional, from indices clamped into the input (pairs past
  // the run or the limbs read valid words that the digit step ignores).
  auto load_tile = [&](W2 (&xr)[IPT], uint32_t tile) {
    const uint32_t tc = tile < end ? tile : end - 1u;
#pragma unroll
    for (int m = 0; m < IPT; ++m) {
      const uint32_t pidx = ht + m * 64u * kWsHelpers;
      const uint32_t i = pidx >> 4 < a.L ? pidx >> 4 : a.L - 1u, cp = pidx & 15u;
      const uint64_t g = (uint64_t)tc * 32u + 2u * cp;
      xr[m] = *reinterpret_cast<const W2*>(static_cast<const W*>(a.in) + (g >> a.log_n) * a.in_stride +
                                           ((uint64_t)i << a.log_n) + (uint32_t)(g & nmask));
    }
  };
  // The limb constants come from an LDS copy (made before the first tile), so
  // that the only vector loads of the loop are the words loaded ahead (a vector
  // load of a constant would wait behind them).
  const double* f1 = reinterpret_cast<const double*>(zbuf + 3u * lp * 32u);
  auto digit_word = [&](W x, double q, double w, double wq) {
    double t = f64_mulmod_pre(small_to_f64((uint64_t)x), w, wq, q);
    t = t < 0.0 ? t + q : t;
    return (f64_to_small(t) + kDigitOffset) ^ kDigitOffset;
  };
  auto digits = [&](const W2 (&xr)[IPT], uint32_t tile, uint64_t* buf) {
    typedef uint64_t U2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int m = 0; m < IPT; ++m) {
      const uint32_t pidx = ht + m * 64u * kWsHelpers;
      const uint32_t i = pidx >> 4, cp = pidx & 15u;
      const double* f = f1 + 4u * (i < a.L ? i : a.L - 1u);
      const double q = f[0], w = f[2], wq = f[3];
      if (pidx < lp * 16u) {
        U2 z = {0, 0};
        if (i < a.L) {
          if (MODE == kBconvUp) {
            const uint64_t g = (uint64_t)tile * 32u + 2u * cp;
            *reinterpret_cast<W2*>(static_cast<W*>(a.copy) + (g >> a.log_n) * a.aux_stride +
                                   ((uint64_t)i << a.log_n) + (uint32_t)(g & nmask)) = xr[m];
          }
          z.x = digit_word(xr[m].x, q, w, wq);
          z.y = digit_word(xr[m].y, q, w, wq);
        }
        *reinterpret_cast<U2*>(buf + i * 32u + 2u * cp) = z;
      }
    }
  };
  // Before step t (t = 0, 1, ...) the digits of tiles t and t + 1 are in LDS;
  // during step t the helpers form those of tile t + 2 and load the words of
  // tile t + 5: four register sets in turn (so the loop body appears four
  // times), each load three steps ahead of its use.  One barrier per step, as
  // the owners.
  W2 x0[IPT], x1[IPT], x2[IPT], x3[IPT];
  load_tile(x0, first);
  load_tile(x1, first + 1u);
  load_tile(x2, first + 2u);
  load_tile(x3, first + 3u);
  digits(x0, first, buffer(0));
  if (first + 1u < end) digits(x1, first + 1u, buffer(1));
  load_tile(x0, first + 4u);
  __syncthreads();
  uint32_t t = 0;
  auto step = [&](W2 (&ld)[IPT], const W2 (&use)[IPT]) {
    load_tile(ld, first + t + 5u);
    if (first + t + 2u < end) digits(use, first + t + 2u, buffer(t + 2u));
    __syncthreads();
    ++t;
  };
  while (true) {
    step(x1, x2);
    if (first + t >= end) break;
    step(x2, x3);
    if (first + t >= end) break;
    step(x3, x0);
    if (first + t >= end) break;
    step(x0, x1);
    if (first + t >= end) break;
  }
}

template <class W, int SMAX, int IPT, int MODE>
static hipError_t launch_ws(const BconvArgs& a, uint32_t grid, uint32_t block, hipStream_t s) {
  const uint32_t lds = 3u * ((a.L + 1u) & ~1u) * 32u * 8u + 32u * a.L;
  hipLaunchKernelGGL((bconv_ws_kernel<W, SMAX, IPT, MODE>), dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

// Threads of a weights-stationary workgroup: one wave per row tile and the helpers.
inline uint32_t ws_block(uint32_t M) { return 64u * (((M + 3u) >> 2) + kWsHelpers); }
// Coefficient pairs per helper thread: at most 48 limbs (768 pairs) over 256 threads.
inline uint32_t ws_ipt(uint32_t L, uint32_t M) {
  (void)M;
  const uint32_t per = (((L + 1u) & ~1u) * 16u + 64u * kWsHelpers - 1u) / (64u * kWsHelpers);
  return per <= 2u ? 2u : 3u;
}

template <class W, int SMAX, int MODE>
static hipError_t launch_ws_ipt(const BconvArgs& a, uint32_t grid, hipStream_t s) {
  const uint32_t block = ws_block(a.M), ipt = ws_ipt(a.L, a.M);
  if (ipt == 2) return launch_ws<W, SMAX, 2, MODE>(a, grid, block, s);
  return launch_ws<W, SMAX, 3, MODE>(a, grid, block, s);
}

template <class W, int MODE>
static hipError_t launch_bconv_mode(const BconvArgs& a, bool f64, bool mfma, uint32_t ws_grid,
                                    hipStream_t s) {
  static const char* const kNames[3][3] = {{"bconv", "bconv_f64", "bconv_mfma"},
                                           {"modup", "modup_f64", "modup_mfma"},
                                           {"moddown", "moddown_f64", "moddown_mfma"}};
  const char* cls = sizeof(W) == 4 ? "u32" : "u64";
  if (mfma && ws_grid) {
    LaunchTimer t(kNames[MODE][2], cls, (int)a.log_n, false, false, (uint64_t)a.total * a.M, s);
    const uint32_t steps = (a.L + 1u) / 2u;
    if (steps <= 8) return launch_ws_ipt<W, 8, MODE>(a, ws_grid, s);
    if (steps <= 16) return launch_ws_ipt<W, 16, MODE>(a, ws_grid, s);
    if (steps <= 18) return launch_ws_ipt<W, 18, MODE>(a, ws_grid, s);
    return launch_ws_ipt<W, 24, MODE>(a, ws_grid, s);
  }
  if (mfma) {
    const uint32_t tiles = a.total / 32u;  // N >= 32: tiles never straddle polynomials
    LaunchTimer t(kNames[MODE][2], cls, (int)a.log_n, false, false, (uint64_t)a.total * a.M, s);
    const dim3 grid((tiles + 3u) / 4u), block(256);
    const uint32_t steps = (a.L + 1u) / 2u;
    if (steps <= 8) hipLaunchKernelGGL((bconv_mfma_kernel<W, 8, MODE>), grid, block, 0, s, a);
    else if (steps <= 12) hipLaunchKernelGGL((bconv_mfma_kernel<W, 12, MODE>), grid, block, 0, s, a);
    else if (steps <= 16) hipLaunchKernelGGL((bconv_mfma_kernel<W, 16, MODE>), grid, block, 0, s, a);
    else if (steps <= 20) hipLaunchKernelGGL((bconv_mfma_kernel<W, 20, MODE>), grid, block, 0, s, a);
    else if (steps <= 24) hipLaunchKernelGGL((bconv_mfma_kernel<W, 24, MODE>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((bconv_mfma_kernel<W, 32, MODE>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  const uint32_t blocks = (uint32_t)(((uint64_t)a.total + kBconvBlock - 1) / kBconvBlock);
  LaunchTimer t(kNames[MODE][f64 ? 1 : 0], cls, (int)a.log_n, false, false, (uint64_t)a.total * a.M, s);
  if (f64)
    hipLaunchKernelGGL((bconv_f64_kernel<W, MODE>), dim3(blocks), dim3(kBconvBlock), 0, s, a);
  else
    hipLaunchKernelGGL((bconv_kernel<W, MODE>), dim3(blocks), dim3(kBconvBlock), 0, s, a);
  return hipGetLastError();
}

template <class W>
static hipError_t launch_bconv(const BconvArgs& a, int mode, bool f64, bool mfma, uint32_t ws_grid,
                               hipStream_t s) {
  if (mode == kBconvUp) return launch_bconv_mode<W, kBconvUp>(a, f64, mfma, ws_grid, s);
  if (mode == kBconvDown) return launch_bconv_mode<W, kBconvDown>(a, f64, mfma, ws_grid, s);
  return launch_bconv_mode<W, kBconvPlain>(a, f64, mfma, ws_grid, s);
}

// Workgroups of the weights-stationary kernel resident per CU (any grid is
// correct: workgroups share nothing; this one fills the chip once).
template <class W, int SMAX>
static int ws_occ(uint32_t L, uint32_t M, uint32_t lds) {
  int nb = 0;
  const uint32_t block = ws_block(M), ipt = ws_ipt(L, M);
  hipError_t e;
  if (ipt == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bconv_ws_kernel<W, SMAX, 2, 2>, block, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bconv_ws_kernel<W, SMAX, 3, 2>, block, lds);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

// Workgroups of the weights-stationary kernel resident per CU (any grid is
// correct: workgroups share nothing; this one fills the chip once).
template <class W>
static int ws_blocks_per_cu(uint32_t L, uint32_t M, uint32_t lds) {
  const uint32_t steps = (L + 1u) / 2u;
  if (steps <= 8) return ws_occ<W, 8>(L, M, lds);
  if (steps <= 16) return ws_occ<W, 16>(L, M, lds);
  if (steps <= 18) return ws_occ<W, 18>(L, M, lds);
  return ws_occ<W, 24>(L, M, lds);
}

static void free_bconv(ntt_bconv_s* h) {
  if (!h) return;
  if (h->d_c1) (void)hipFree(h->d_c1);
  if (h->d_c2) (void)hipFree(h->d_c2);
  if (h->d_p) (void)hipFree(h->d_p);
  if (h->d_f1) (void)hipFree(h->d_f1);
  if (h->d_f2) (void)hipFree(h->d_f2);
  if (h->d_fp) (void)hipFree(h->d_fp);
  if (h->d_kop) (void)hipFree(h->d_kop);
  if (h->d_om) (void)hipFree(h->d_om);
  if (h->d_om2) (void)hipFree(h->d_om2);
  delete h;
}

}  // namespace nttk

using namespace nttk;

extern "C" {

// Balanced base-256 digit c (c < 7) of v < 2^50 as an int8 bit pattern; digit 7 is 0.
static uint8_t digit256(uint64_t v, uint32_t c) {
  const uint64_t z = (v + kDigitOffset) ^ kDigitOffset;
  return (uint8_t)(z >> (8 * c));
}

// Checks the arguments of one conversion and puts its constants on the current
// device; *out owns them (free_bconv).
static ntt_status bconv_build(ntt_bconv_s** out, uint32_t N, const uint64_t* src_moduli, uint32_t L,
                              const uint64_t* dst_moduli, uint32_t M, uint32_t word_bits,
                              uint32_t flags) {
  if (flags & ~(NTT_BCONV_NO_MFMA | NTT_BCONV_MFMA | NTT_BCONV_NO_WS))
    return fail(NTT_EINVAL, "unknown flags 0x%x", flags);
  if ((flags & NTT_BCONV_NO_MFMA) && (flags & NTT_BCONV_MFMA))
    return fail(NTT_EINVAL, "NTT_BCONV_NO_MFMA and NTT_BCONV_MFMA are exclusive");
  if (!out || !src_moduli || !dst_moduli) return fail(NTT_EINVAL, "null argument");
  *out = nullptr;
  if (N < 2 || N > (1u << 16) || (N & (N - 1)))
    return fail(NTT_EINVAL, "N=%u is not a power of two in [2, 65536]", N);
  if (L == 0 || L > 64) return fail(NTT_EINVAL, "L=%u source moduli (1 .. 64)", L);
  if (M == 0 || M > 4096) return fail(NTT_EINVAL, "M=%u target moduli (1 .. 4096)", M);
  if (word_bits != 32 && word_bits != 64) return fail(NTT_EINVAL, "word_bits=%u", word_bits);
  const uint64_t bound = word_bits == 32 ? (1ull << 32) : (1ull << 62);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = src_moduli[i];
    if (q >= bound) return fail(NTT_ERANGE, "source q=%llu too wide", (unsigned long long)q);
    if (!nt_is_prime(q)) return fail(NTT_ENOTPRIME, "source q=%llu is not prime", (unsigned long long)q);
    for (uint32_t k = 0; k < i; ++k)
      if (src_moduli[k] == q) return fail(NTT_EINVAL, "source moduli must be distinct");
  }
  for (uint32_t j = 0; j < M; ++j) {
    const uint64_t p = dst_moduli[j];
    if (p < 2 || p >= bound) return fail(NTT_ERANGE, "target p=%llu out of range", (unsigned long long)p);
  }
  std::vector<uint64_t> c1(3 * (size_t)L), c2(2 * (size_t)L * M);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = src_moduli[i];
    uint64_t qhat = 1;  // (Q/q_i) mod q_i
    for (uint32_t k = 0; k < L; ++k)
      if (k != i) qhat = nt_mul(qhat, src_moduli[k] % q, q);
    const uint64_t w = nt_pow(qhat, q - 2, q);  // q prime
    c1[3 * i] = q;
    c1[3 * i + 1] = w;
    c1[3 * i + 2] = (uint64_t)(((u128)w << 64) / q);
    for (uint32_t j = 0; j < M; ++j) {
      const uint64_t p = dst_moduli[j];
      uint64_t m = 1 % p;  // (Q/q_i) mod p_j
      for (uint32_t k = 0; k < L; ++k)
        if (k != i) m = nt_mul(m, src_moduli[k] % p, p);
      c2[2 * ((size_t)i * M + j)] = m;
      c2[2 * ((size_t)i * M + j) + 1] = (uint64_t)(((u128)m << 64) / p);
    }
  }
  ntt_bconv_s* h = new (std::nothrow) ntt_bconv_s();
  if (!h) return fail(NTT_ENOMEM, "host allocation");
  hipError_t e = hipGetDevice(&h->device);
  h->N = N;
  h->log_n = 0;
  while ((1u << h->log_n) < N) ++h->log_n;
  h->L = L;
  h->M = M;
  h->word_bits = word_bits;
  if (e == hipSuccess) e = hipMalloc(&h->d_c1, c1.size() * 8);
  if (e == hipSuccess) e = hipMalloc(&h->d_c2, c2.size() * 8);
  if (e == hipSuccess) e = hipMalloc(&h->d_p, (size_t)M * 8);
  if (e == hipSuccess) e = hipMemcpy(h->d_c1, c1.data(), c1.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_c2, c2.data(), c2.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_p, dst_moduli, (size_t)M * 8, hipMemcpyHostToDevice);
  // fp64 products when every modulus fits the exact fp64 arithmetic
  constexpr uint64_t kF64Bound = kF64LBound;
  h->f64 = true;
  for (uint32_t i = 0; i < L; ++i) h->f64 = h->f64 && src_moduli[i] < kF64Bound;
  for (uint32_t j = 0; j < M; ++j) h->f64 = h->f64 && dst_moduli[j] < kF64Bound;
  if (h->f64 && e == hipSuccess) {
    std::vector<double> f1(4 * (size_t)L), f2(2 * (size_t)L * M), fp(2 * (size_t)M);
    for (uint32_t i = 0; i < L; ++i) {
      const double q = (double)c1[3 * i], w = (double)c1[3 * i + 1];
      f1[4 * i] = q;
      f1[4 * i + 1] = 1.0 / q;
      f1[4 * i + 2] = w;
      f1[4 * i + 3] = w * (1.0 / q);
      for (uint32_t j = 0; j < M; ++j) {
        const double m = (double)c2[2 * ((size_t)i * M + j)];
        f2[2 * ((size_t)i * M + j)] = m;
        f2[2 * ((size_t)i * M + j) + 1] = m * (1.0 / (double)dst_moduli[j]);
      }
    }
    for (uint32_t j = 0; j < M; ++j) {
      fp[2 * j] = (double)dst_moduli[j];
      fp[2 * j + 1] = 1.0 / (double)dst_moduli[j];
    }
    e = hipMalloc(&h->d_f1, f1.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&h->d_f2, f2.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&h->d_fp, fp.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(h->d_f1, f1.data(), f1.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_f2, f2.data(), f2.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_fp, fp.data(), fp.size() * 8, hipMemcpyHostToDevice);
  }
  // The matrix cores pay off for dense conversions (measured: 36 -> 36 limbs on
  // one 2^16 polynomial 50 us against 173 us on the vector units); with fewer
  // than 16 source or target moduli the vector form is faster.
  h->mfma = h->f64 && N >= 32 && !(flags & NTT_BCONV_NO_MFMA) &&
            ((flags & NTT_BCONV_MFMA) || (L >= 16 && M >= 16));
  if (h->mfma && e == hipSuccess) {
    // Constant operands: for row tile rt (outputs 4 rt .. 4 rt + 3), k-step s
    // (limbs 2s, 2s + 1) and lane l, byte e of the operand is digit c = l mod 8
    // of (Q/q_i mod p_J) 256^e mod p_J, J = 4 rt + (l mod 32) / 8, i = 2s + l / 32.
    const uint32_t steps = (L + 1) / 2, row_tiles = (M + 3) / 4;
    std::vector<uint64_t> kop((size_t)row_tiles * steps * 64, 0);
    for (uint32_t rt = 0; rt < row_tiles; ++rt)
      for (uint32_t st = 0; st < steps; ++st)
        for (uint32_t l = 0; l < 64; ++l) {
          const uint32_t J = 4 * rt + (l % 32) / 8, c = l % 8, i = 2 * st + l / 32;
          if (J >= M || i >= L) continue;
          const uint64_t p = dst_moduli[J], m = c2[2 * ((size_t)i * M + J)];
          uint64_t word = 0, scaled = m;  // scaled = m 256^e mod p
          for (uint32_t e8 = 0; e8 < 7; ++e8) {
            word |= (uint64_t)digit256(scaled, c) << (8 * e8);
            scaled = nt_mul(scaled, 256 % p, p);
          }
          kop[((size_t)rt * steps + st) * 64 + l] = word;
        }
    std::vector<double> om((size_t)M * 16);
    for (uint32_t j = 0; j < M; ++j) {
      const uint64_t p = dst_moduli[j];
      uint64_t w = 1 % p;
      for (uint32_t c = 0; c < 8; ++c) {
        om[16 * (size_t)j + 2 * c] = (double)w;
        om[16 * (size_t)j + 2 * c + 1] = (double)w * (1.0 / (double)p);
        w = nt_mul(w, 256 % p, p);
      }
    }
    // weights-stationary form: p_j, 1/p_j, 2^32 mod p_j and that over p_j
    std::vector<double> om2((size_t)M * 4);
    for (uint32_t j = 0; j < M; ++j) {
      const uint64_t p = dst_moduli[j];
      const uint64_t w32 = nt_mul(65536 % p, 65536 % p, p);
      om2[4 * (size_t)j] = (double)p;
      om2[4 * (size_t)j + 1] = 1.0 / (double)p;
      om2[4 * (size_t)j + 2] = (double)w32;
      om2[4 * (size_t)j + 3] = (double)w32 * (1.0 / (double)p);
    }
    e = hipMalloc(&h->d_kop, kop.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&h->d_om, om.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&h->d_om2, om2.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(h->d_kop, kop.data(), kop.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_om, om.data(), om.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_om2, om2.data(), om2.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && row_tiles <= (uint32_t)kWsMaxTiles && L <= kWsMaxLimbs &&
        !(flags & NTT_BCONV_NO_WS)) {
      int cus = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
      const uint32_t lds = 3u * (2u * steps) * 32u * 8u + 32u * L;
      const int per_cu = word_bits == 32 ? ws_blocks_per_cu<uint32_t>(L, M, lds)
                                         : ws_blocks_per_cu<uint64_t>(L, M, lds);
      h->ws_grid = (uint32_t)((cus > 0 ? cus : 1) * per_cu);
    }
  }
  if (e != hipSuccess) {
    free_bconv(h);
    return hip_fail(e, "basis conversion constants");
  }
  *out = h;
  return NTT_OK;
}

// One launch of conversion h over `batch` polynomials in the given mode; the
// caller has checked pointers, sizes and overlaps.
static ntt_status bconv_run(const ntt_bconv_s* h, int mode, void* out, uint64_t out_stride,
                            const void* in, uint64_t in_stride, void* copy, const void* sub,
                            uint64_t aux_stride, const uint64_t* sc, const double* sf,
                            uint32_t batch, void* stream) {
  BconvArgs a;
  a.out = out;
  a.in = in;
  a.c1 = h->d_c1;
  a.c2 = h->d_c2;
  a.p = h->d_p;
  a.f1 = h->d_f1;
  a.f2 = h->d_f2;
  a.fp = h->d_fp;
  a.kop = h->d_kop;
  a.om = h->d_om;
  a.om2 = h->d_om2;
  a.L = h->L;
  a.M = h->M;
  a.log_n = h->log_n;
  a.total = (uint32_t)((uint64_t)batch << h->log_n);
  a.in_stride = in_stride;
  a.out_stride = out_stride;
  a.copy = copy;
  a.sub = sub;
  a.aux_stride = aux_stride;
  a.sc = sc;
  a.sf = sf;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // weights-stationary grid: every workgroup that fits at once, at most one per tile
  const uint32_t tiles = a.total >> 5;
  const uint32_t ws_grid = h->ws_grid ? (tiles < h->ws_grid ? tiles : h->ws_grid) : 0u;
  const hipError_t e = h->word_bits == 32
                           ? launch_bconv<uint32_t>(a, mode, h->f64, h->mfma, ws_grid, s)
                           : launch_bconv<uint64_t>(a, mode, h->f64, h->mfma, ws_grid, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return NTT_OK;
}

static bool overlaps(const void* a, uint64_t a_bytes, const void* b, uint64_t b_bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + b_bytes && y < x + a_bytes;
}

ntt_status ntt_bconv_create(ntt_bconv_t* out, uint32_t N, const uint64_t* src_moduli, uint32_t L,
                            const uint64_t* dst_moduli, uint32_t M, uint32_t word_bits,
                            uint32_t flags) {
  clear_error();
  return bconv_build(out, N, src_moduli, L, dst_moduli, M, word_bits, flags);
}

ntt_status ntt_bconv(ntt_bconv_t h, void* out, const void* in, uint32_t batch, void* stream) {
  clear_error();
  if (!h) return fail(NTT_EINVAL, "null basis conversion");
  if (!out || !in) return fail(NTT_EINVAL, "null data");
  if (batch == 0) return fail(NTT_EINVAL, "batch must be >= 1");
  const uint64_t in_words = ((uint64_t)batch * h->L) << h->log_n;
  const uint64_t out_words = ((uint64_t)batch * h->M) << h->log_n;
  if (in_words >= (1ull << 32) || out_words >= (1ull << 32))
    return fail(NTT_EINVAL, "batch * L * N and batch * M * N must be < 2^32 words");
  const uint64_t wb = h->word_bits / 8;
  if (overlaps(out, out_words * wb, in, in_words * wb))
    return fail(NTT_EINVAL, "out must not overlap in");
  return bconv_run(h, kBconvPlain, out, (uint64_t)h->M << h->log_n, in,
                   (uint64_t)h->L << h->log_n, nullptr, nullptr, 0, nullptr, nullptr, batch, stream);
}

ntt_status ntt_bconv_destroy(ntt_bconv_t h) {
  clear_error();
  if (!h) return fail(NTT_EINVAL, "null basis conversion");
  free_bconv(h);
  return NTT_OK;
}

static void free_ext(ntt_basis_ext_s* h) {
  if (!h) return;
  free_bconv(h->up);
  free_bconv(h->down);
  if (h->d_sc) (void)hipFree(h->d_sc);
  if (h->d_sf) (void)hipFree(h->d_sf);
  delete h;
}

ntt_status ntt_basis_ext_create(ntt_basis_ext_t* out, uint32_t N, const uint64_t* q_moduli,
                                uint32_t L, const uint64_t* p_moduli, uint32_t K,
                                uint32_t word_bits, uint32_t flags) {
  clear_error();
  if (!out || !q_moduli || !p_moduli) return fail(NTT_EINVAL, "null argument");
  *out = nullptr;
  if (L == 0 || L > 64 || K == 0 || K > 64)
    return fail(NTT_EINVAL, "L=%u, K=%u moduli (1 .. 64 each)", L, K);
  for (uint32_t i = 0; i < L; ++i)
    for (uint32_t k = 0; k < K; ++k)
      if (q_moduli[i] == p_moduli[k])
        return fail(NTT_EINVAL, "q and p moduli must be distinct (%llu in both)",
                    (unsigned long long)q_moduli[i]);
  // The first build checks the q_i in full and the p_k only for range; the p_k
  // are the second build's sources, checked here so that nothing is allocated
  // for a basis that would fail.
  if (word_bits != 32 && word_bits != 64) return fail(NTT_EINVAL, "word_bits=%u", word_bits);
  const uint64_t bound = word_bits == 32 ? (1ull << 32) : (1ull << 62);
  for (uint32_t k = 0; k < K; ++k) {
    if (p_moduli[k] >= bound)
      return fail(NTT_ERANGE, "p=%llu too wide", (unsigned long long)p_moduli[k]);
    if (!nt_is_prime(p_moduli[k]))
      return fail(NTT_ENOTPRIME, "p=%llu is not prime", (unsigned long long)p_moduli[k]);
    for (uint32_t j = 0; j < k; ++j)
      if (p_moduli[j] == p_moduli[k]) return fail(NTT_EINVAL, "p moduli must be distinct");
  }
  ntt_basis_ext_s* h = new (std::nothrow) ntt_basis_ext_s();
  if (!h) return fail(NTT_ENOMEM, "host allocation");
  // Each build checks N, word_bits and flags, and that its source moduli are
  // distinct primes that fit the word: together, that every q_i and p_k is.
  ntt_status st = bconv_build(&h->up, N, q_moduli, L, p_moduli, K, word_bits, flags);
  if (st == NTT_OK) st = bconv_build(&h->down, N, p_moduli, K, q_moduli, L, word_bits, flags);
  if (st != NTT_OK) {
    free_ext(h);
    return st;
  }
  h->N = N;
  h->log_n = h->up->log_n;
  h->L = L;
  h->K = K;
  h->word_bits = word_bits;
  std::vector<uint64_t> sc(2 * (size_t)L);
  std::vector<double> sf(2 * (size_t)L);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = q_moduli[i];
    uint64_t pm = 1;  // P mod q_i, nonzero: the moduli are distinct primes
    for (uint32_t k = 0; k < K; ++k) pm = nt_mul(pm, p_moduli[k] % q, q);
    const uint64_t s = nt_pow(pm, q - 2, q);
    sc[2 * i] = s;
    sc[2 * i + 1] = (uint64_t)(((u128)s << 64) / q);
    sf[2 * i] = (double)s;
    sf[2 * i + 1] = (double)s * (1.0 / (double)q);
  }
  hipError_t e = hipMalloc(&h->d_sc, sc.size() * 8);
  if (e == hipSuccess) e = hipMalloc(&h->d_sf, sf.size() * 8);
  if (e == hipSuccess) e = hipMemcpy(h->d_sc, sc.data(), sc.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_sf, sf.data(), sf.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_ext(h);
    return hip_fail(e, "key-switching basis constants");
  }
  *out = h;
  return NTT_OK;
}

// Sizes and overlap of one ModUp / ModDown call: `narrow` has L limbs per
// polynomial, `wide` L + K.
static ntt_status ext_check(const ntt_basis_ext_s* h, const void* narrow, const void* wide,
                            uint32_t batch) {
  if (!h) return fail(NTT_EINVAL, "null key-switching basis");
  if (!narrow || !wide) return fail(NTT_EINVAL, "null data");
  if (batch == 0) return fail(NTT_EINVAL, "batch must be >= 1");
  const uint64_t wide_words = ((uint64_t)batch * (h->L + h->K)) << h->log_n;
  if (wide_words >= (1ull << 32)) return fail(NTT_EINVAL, "batch * (L + K) * N must be < 2^32 words");
  const uint64_t wb = h->word_bits / 8;
  if (overlaps(narrow, (((uint64_t)batch * h->L) << h->log_n) * wb, wide, wide_words * wb))
    return fail(NTT_EINVAL, "out must not overlap in");
  return NTT_OK;
}

ntt_status ntt_mod_up(ntt_basis_ext_t h, void* out, const void* in, uint32_t batch, void* stream) {
  clear_error();
  const ntt_status st = ext_check(h, in, out, batch);
  if (st != NTT_OK) return st;
  const uint64_t nq = (uint64_t)h->L << h->log_n, nw = (uint64_t)(h->L + h->K) << h->log_n;
  char* o = static_cast<char*>(out);
  return bconv_run(h->up, kBconvUp, o + nq * (h->word_bits / 8), nw, in, nq, out, nullptr, nw,
                   nullptr, nullptr, batch, stream);
}

ntt_status ntt_mod_down(ntt_basis_ext_t h, void* out, const void* in, uint32_t batch, void* stream) {
  clear_error();
  const ntt_status st = ext_check(h, out, in, batch);
  if (st != NTT_OK) return st;
  const uint64_t nq = (uint64_t)h->L << h->log_n, nw = (uint64_t)(h->L + h->K) << h->log_n;
  const char* x = static_cast<const char*>(in);
  return bconv_run(h->down, kBconvDown, out, nq, x + nq * (h->word_bits / 8), nw, nullptr, in, nw,
                   h->d_sc, h->d_sf, batch, stream);
}

ntt_status ntt_basis_ext_destroy(ntt_basis_ext_t h) {
  clear_error();
  if (!h) return fail(NTT_EINVAL, "null key-switching basis");
  free_ext(h);
  return NTT_OK;
}

}  // extern "C"
