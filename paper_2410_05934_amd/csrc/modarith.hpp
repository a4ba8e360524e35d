// modarith.hpp -- exact modular arithmetic for the gfx950 NTT kernels.
//
// Three arithmetic classes, chosen per modulus when a plan is built:
//
//   ArF64S  q < 2^32, 32-bit words.  Values are held in fp64 registers as
//           exact integers.  A product x*w is split exactly into h + l with
//           one multiply and one FMA; the quotient c = rint(x * (w/q)) is
//           estimated in fp64 and r = (h - c*q) + l is then exact (all terms
//           are integers below 2^53).  Inputs may be lazily reduced: for
//           q < 2^32 the bounds stay far below 2^53 for any N <= 2^16, so no
//           intermediate reduction is needed inside a transform.
//   ArF64L  q < 2^50 - 2^10, 64-bit words, the same fp64 scheme.  A group of
//           up to four butterfly stages keeps every value below 2^53 when its
//           inputs are centred (|x| <= q/2 + 2); a centred reduction
//           x - q*rint(x/q) follows every such group.
//   ArI64   q < 2^62, 64-bit words: Shoup multiplication with a precomputed
//           companion w' = floor(w * 2^64 / q) and Harvey's lazy butterflies
//           (forward values in [0, 4q), inverse values in [0, 2q)).
//
// fp64 is used because gfx950 runs fp64 FMA at full vector rate while 64-bit
// integer multiplies cost several quarter-rate 32-bit partial products.  The
// results are exact integers in every class; no floating-point rounding ever
// reaches an output.
//
// Everything here is __host__ __device__ so that the same code can be checked
// exhaustively on the CPU against 128-bit integer arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef __HIP_DEVICE_COMPILE__
#include <cmath>
#endif

namespace nttk {

#define NTT_HD __host__ __device__ __forceinline__

NTT_HD double fma_rn(double a, double b, double c) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_fma(a, b, c);
#else
  return std::fma(a, b, c);
#endif
}
NTT_HD double rint_rn(double a) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_rint(a);
#else
  return std::nearbyint(a);
#endif
}
NTT_HD double as_double(uint64_t x) {
  union { uint64_t u; double d; } c;
  c.u = x;
  return c.d;
}
NTT_HD uint64_t as_u64(double x) {
  union { uint64_t u; double d; } c;
  c.d = x;
  return c.u;
}
NTT_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

constexpr double kTwo52 = 4503599627370496.0;  // 2^52

// Largest modulus (exclusive) of the ArF64L class.  Four inverse (GS) stages
// double the sum side from centred inputs (|x| <= q/2 + 2) to 8q + 32, which
// must stay below 2^53; the forward chain (four CT stages from |x| < q, each
// adding at most q/2 + |x| (q/2) 3 2^-53) stays lower.  2^10 of margin below
// 2^50 covers the rounding terms.  Larger moduli take the integer class.
constexpr uint64_t kF64LBound = (1ull << 50) - (1ull << 10);

// x*w - c*q exactly, with c = rint(x * RN(w*qinv)).  |result| <= (1/2 + e)*q
// where e <= |x*w/q| * 3 * 2^-53 (see the bounds in the design notes).
NTT_HD double f64_mulmod(double x, double w, double q, double qinv) {
  const double h = x * w;
  const double l = fma_rn(x, w, -h);
  const double c = rint_rn(x * (w * qinv));
  const double r = fma_rn(-c, q, h);
  return r + l;
}

// General product of two lazily-reduced operands (neither is a table entry).
NTT_HD double f64_mulmod2(double x, double y, double q, double qinv) {
  const double h = x * y;
  const double l = fma_rn(x, y, -h);
  const double c = rint_rn(h * qinv);
  const double r = fma_rn(-c, q, h);
  return r + l;
}

// Centred representative: |result| <= q/2 + 2 for |x| < 2^53.
NTT_HD double f64_center(double x, double q, double qinv) {
  const double c = rint_rn(x * qinv);
  return fma_rn(-c, q, x);
}

// Canonical representative in [0, q) for |x| < 2^53.
NTT_HD double f64_canon(double x, double q, double qinv) {
  double r = f64_center(x, q, qinv);
  r = r < 0.0 ? r + q : r;
  return r;
}

// Shoup: y*w mod q in [0, 2q) for any y < 2^64, q < 2^63.
NTT_HD uint64_t shoup_mul(uint64_t y, uint64_t w, uint64_t ws, uint64_t q) {
  return y * w - mulhi64(y, ws) * q;
}

// Barrett-style product of two operands in [0, q), q < 2^62, b = bit length
// of q, mu = floor(2^(2b) / q).  Result in [0, q).
NTT_HD uint64_t barrett_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t mu, uint32_t qbits) {
  const uint64_t lo = a * b;
  const uint64_t hi = mulhi64(a, b);
  // t = floor(P / 2^(qbits-1)) < 2^(qbits+1)
  const uint32_t s1 = qbits - 1;
  const uint64_t t = (lo >> s1) | (hi << (64 - s1));
  // e = floor(t * mu / 2^(qbits+1))
  const uint64_t plo = t * mu;
  const uint64_t phi = mulhi64(t, mu);
  const uint32_t s2 = qbits + 1;
  const uint64_t e = (plo >> s2) | (phi << (64 - s2));
  uint64_t r = lo - e * q;  // in [0, 3q)
  r = r >= q ? r - q : r;
  r = r >= q ? r - q : r;
  return r;
}

// ---------------------------------------------------------------------------
// Per-modulus constants as the kernels see them.
struct LimbDev {
  uint64_t q;
  double qd, qinv;
  const void* twf;  // forward table, index k -> psi^brv(k)  (double or TwI64)
  const void* twi;  // inverse table, index k -> psi^-brv(k)
  // N^-1 folded into the last inverse stage: (u+v)*ninv, (u-v)*ninvw
  double ninv_d, ninvw_d;                  // centred, fp64 classes
  uint64_t ninv, ninv_s, ninvw, ninvw_s;   // Shoup pairs, ArI64
  uint64_t bmu;                            // Barrett constant, ArI64
  uint32_t qbits;
  uint32_t cls;
};

struct TwI64 {
  uint64_t w, ws;
};

// ---------------------------------------------------------------------------
// Arithmetic classes used as kernel template parameters.

struct ArF64S {
  using W = uint32_t;
  using V = double;
  using TW = double;
  static constexpr int kCls = 0;
  static constexpr const char* kName = "f64s";
  static constexpr bool kCenterRounds = false;
  double q, qinv;
  NTT_HD explicit ArF64S(const LimbDev& d) : q(d.qd), qinv(d.qinv) {}
  NTT_HD V from_word(W x) const { return (double)x; }
  NTT_HD W to_word(V x) const { return (W)f64_canon(x, q, qinv); }
  NTT_HD V from_raw(W x) const { return (double)(int32_t)x; }
  NTT_HD W to_raw(V x) const { return (W)(int32_t)f64_center(x, q, qinv); }
  NTT_HD void center(V& x) const { (void)x; }
  NTT_HD void ct(V& x, V& y, TW w) const {
    const double t = f64_mulmod(y, w, q, qinv);
    const double a = x;
    x = a + t;
    y = a - t;
  }
  NTT_HD void gs(V& x, V& y, TW w) const {
    const double a = x, b = y;
    x = a + b;
    y = f64_mulmod(a - b, w, q, qinv);
  }
  NTT_HD void gs_fold(V& x, V& y, TW w, const LimbDev& d) const {
    (void)w;
    const double a = x, b = y;
    x = f64_mulmod(a + b, d.ninv_d, q, qinv);
    y = f64_mulmod(a - b, d.ninvw_d, q, qinv);
  }
  NTT_HD V mul(V x, V y) const {
    return f64_mulmod2(f64_center(x, q, qinv), f64_center(y, q, qinv), q, qinv);
  }
  NTT_HD V add(V x, V y) const { return f64_center(x + y, q, qinv); }
};

struct ArF64L {
  using W = uint64_t;
  using V = double;
  using TW = double;
  static constexpr int kCls = 1;
  static constexpr const char* kName = "f64l";
  static constexpr bool kCenterRounds = true;
  double q, qinv;
  NTT_HD explicit ArF64L(const LimbDev& d) : q(d.qd), qinv(d.qinv) {}
  // Words below 2^52 become doubles exactly through the 2^52 exponent trick.
  NTT_HD V from_word(W x) const { return as_double(x | 0x4330000000000000ull) - kTwo52; }
  NTT_HD W to_word(V x) const {
    const double r = f64_canon(x, q, qinv);
    return as_u64(r + kTwo52) & 0x000FFFFFFFFFFFFFull;
  }
  NTT_HD V from_raw(W x) const { return as_double(x); }
  NTT_HD W to_raw(V x) const { return as_u64(f64_center(x, q, qinv)); }
  NTT_HD void center(V& x) const { x = f64_center(x, q, qinv); }
  NTT_HD void ct(V& x, V& y, TW w) const {
    const double t = f64_mulmod(y, w, q, qinv);
    const double a = x;
    x = a + t;
    y = a - t;
  }
  NTT_HD void gs(V& x, V& y, TW w) const {
    const double a = x, b = y;
    x = a + b;
    y = f64_mulmod(a - b, w, q, qinv);
  }
  NTT_HD void gs_fold(V& x, V& y, TW w, const LimbDev& d) const {
    (void)w;
    const double a = x, b = y;
    x = f64_mulmod(a + b, d.ninv_d, q, qinv);
    y = f64_mulmod(a - b, d.ninvw_d, q, qinv);
  }
  NTT_HD V mul(V x, V y) const {
    return f64_mulmod2(f64_center(x, q, qinv), f64_center(y, q, qinv), q, qinv);
  }
  NTT_HD V add(V x, V y) const { return f64_center(x + y, q, qinv); }
};

struct ArI64 {
  using W = uint64_t;
  using V = uint64_t;
  using TW = TwI64;
  static constexpr int kCls = 2;
  static constexpr const char* kName = "i64";
  static constexpr bool kCenterRounds = false;
  uint64_t q, q2, mu;
  uint32_t qbits;
  NTT_HD explicit ArI64(const LimbDev& d) : q(d.q), q2(2 * d.q), mu(d.bmu), qbits(d.qbits) {}
  NTT_HD V from_word(W x) const { return x; }
  NTT_HD W to_word(V x) const {
    x = x >= q2 ? x - q2 : x;
    x = x >= q ? x - q : x;
    return x;
  }
  NTT_HD V from_raw(W x) const { return x; }
  NTT_HD W to_raw(V x) const { return x; }
  NTT_HD void center(V& x) const { (void)x; }
  // Forward (Harvey): x, y in [0, 4q) -> outputs in [0, 4q).
  NTT_HD void ct(V& x, V& y, TW w) const {
    uint64_t a = x >= q2 ? x - q2 : x;
    const uint64_t t = shoup_mul(y, w.w, w.ws, q);
    x = a + t;
    y = a - t + q2;
  }
  // Inverse (Harvey): x, y in [0, 2q) -> outputs in [0, 2q).
  NTT_HD void gs(V& x, V& y, TW w) const {
    const uint64_t a = x, b = y;
    uint64_t s = a + b;
    s = s >= q2 ? s - q2 : s;
    x = s;
    y = shoup_mul(a - b + q2, w.w, w.ws, q);
  }
  NTT_HD void gs_fold(V& x, V& y, TW w, const LimbDev& d) const {
    (void)w;
    const uint64_t a = x, b = y;
    x = shoup_mul(a + b, d.ninv, d.ninv_s, q);
    y = shoup_mul(a - b + q2, d.ninvw, d.ninvw_s, q);
  }
  NTT_HD V mul(V x, V y) const { return barrett_mul(to_word(x), to_word(y), q, mu, qbits); }
  // Operands in [0, q) (products of mul) -> sum in [0, q).
  NTT_HD V add(V x, V y) const {
    const uint64_t s = x + y;
    return s >= q ? s - q : s;
  }
};

}  // namespace nttk
