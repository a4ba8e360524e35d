"""Host checks of the device arithmetic (csrc/modarith.hpp, csrc/decompose.hpp),
compiled with g++ as plain host code (the same functions the kernels inline,
with -ffp-contract=off as in the library build) and checked against 128-bit
integer arithmetic at the worst cases the kernels can reach.

What is pinned (Sec. II-D, Eq. (1): every butterfly of the transform is a
modular product and a sum; exactness of each is what makes the GPU words equal
the oracle's):
  * the fp64 product x*w - c*q is exact and congruent, with |r| within the
    analytic bound q/2 + |x| |w| 4 2^-53, for |x| up to the largest value a
    group of stages can reach, and w = +-(q-1)/2;
  * the growth chains of the kernels' stage groups stay below 2^53 for the
    largest modulus the fp64 class admits (forward: four CT stages from
    canonical inputs; inverse: four GS stages from centred inputs; the 32-bit
    class: sixteen stages without reduction), and the same chains would break
    for a modulus twice as large -- so the class bound cannot be raised;
  * centring, canonical conversion and the raw intermediate format;
  * the integer class: Shoup products in [0, 2q), Barrett products exact,
    Harvey butterflies closed on [0, 4q) (forward) and [0, 2q) (inverse);
  * the signed gadget digits read off x + offset against the digit-by-digit
    definition (exhaustively on small bases, and for eight (q, levels, base)
    combinations including the TFHE shape);
  * a CPU emulation of the kernels' schedule for N = 2^16 (column pass of four
    stages, row rounds of four, centring between groups, N^-1 folded into the
    last inverse stage), word for word against a plain 128-bit transform.
"""
import os
import shutil
import subprocess

import pytest

from paper_2410_05934_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2410_05934_amd", "csrc")
ROCM_INC = "/opt/rocm/include"

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include "modarith.hpp"
#include "decompose.hpp"
using namespace nttk;
typedef __int128 i128;
typedef unsigned __int128 u128;

static long fails = 0, checks = 0;
#define CHECK(cond, ...)                                                        \
  do {                                                                          \
    ++checks;                                                                   \
    if (!(cond)) {                                                              \
      if (fails++ < 12) { std::printf("FAIL line %d: ", __LINE__);              \
                          std::printf(__VA_ARGS__); std::printf("\n"); }        \
    }                                                                           \
  } while (0)

static const long double U = 1.0L / 9007199254740992.0L;  // 2^-53
static const long double TWO53 = 9007199254740992.0L;

static bool int53(double v) { return std::fabs(v) < 9007199254740992.0 && v == std::nearbyint(v); }
static i128 md(i128 a, i128 q) { i128 r = a % q; return r < 0 ? r + q : r; }
static uint64_t powm(uint64_t b, uint64_t e, uint64_t q) {
  u128 r = 1, x = b % q;
  while (e) { if (e & 1) r = r * x % q; x = x * x % q; e >>= 1; }
  return (uint64_t)r;
}
static double centred(uint64_t w, uint64_t q) { return w > q / 2 ? -(double)(q - w) : (double)w; }
static int brv(int x, int bits) { int r = 0; for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i); return r; }

// Analytic bound of |x w - c q| for |x| <= B, |w| <= W (rounding of q^-1, of
// w q^-1 and of the product: relative error below 4 2^-53 in all).
static long double R(long double B, long double W, long double q) { return q / 2 + B * W * 4 * U; }

// ---- fp64 product, centring, conversions ---------------------------------
static void check_f64_product(uint64_t qi, long double B, std::mt19937_64& rng) {
  B = floorl(B);  // the largest integer magnitude the chain admits
  const double q = (double)qi, qinv = 1.0 / q;
  const long double W = (long double)((qi - 1) / 2);
  const double xs[] = {(double)B, -(double)B, (double)(B - 1), 1.0, -1.0, 0.0};
  const double ws[] = {(double)W, -(double)W, 1.0, -1.0, 0.0, (double)(W - 7)};
  std::vector<double> xv(xs, xs + 6), wv(ws, ws + 6);
  std::uniform_int_distribution<int64_t> dx(-(int64_t)B, (int64_t)B), dw(-(int64_t)W, (int64_t)W);
  for (int i = 0; i < 200; ++i) { xv.push_back((double)dx(rng)); wv.push_back((double)dw(rng)); }
  for (double x : xv)
    for (double w : wv) {
      const double r = f64_mulmod(x, w, q, qinv);
      CHECK(int53(r), "mulmod not an integer q=%llu x=%.0f w=%.0f", (unsigned long long)qi, x, w);
      CHECK(md((i128)r - (i128)x * (i128)w, qi) == 0, "mulmod not congruent x=%.0f w=%.0f", x, w);
      CHECK(std::fabs((long double)r) <= R(std::fabs((long double)x), std::fabs((long double)w), q),
            "mulmod bound x=%.0f w=%.0f r=%.0f", x, w, r);
    }
}

static void check_center_canon(uint64_t qi, std::mt19937_64& rng) {
  const double q = (double)qi, qinv = 1.0 / q;
  std::vector<double> xv = {9007199254740991.0, -9007199254740991.0, 0.0, 1.0, -1.0,
                            (double)(qi / 2), -(double)(qi / 2), (double)(qi / 2 + 1), (double)qi,
                            -(double)qi, 8.0 * q + 32.0, -(8.0 * q + 32.0)};
  std::uniform_int_distribution<int64_t> d(-9007199254740991LL, 9007199254740991LL);
  for (int i = 0; i < 4000; ++i) xv.push_back((double)d(rng));
  for (double x : xv) {
    const double c = f64_center(x, q, qinv);
    CHECK(int53(c) && md((i128)c - (i128)x, qi) == 0, "center not congruent x=%.0f", x);
    CHECK(std::fabs(c) <= (double)((qi - 1) / 2 + 2), "center bound x=%.0f c=%.0f", x, c);
    const double k = f64_canon(x, q, qinv);
    CHECK(k >= 0 && k < q && md((i128)k - (i128)x, qi) == 0, "canon x=%.0f k=%.0f", x, k);
  }
}

// fp64 product of two centred operands (pointwise, MAC).
static void check_f64_product2(uint64_t qi, std::mt19937_64& rng) {
  const double q = (double)qi, qinv = 1.0 / q;
  const int64_t C = (int64_t)((qi - 1) / 2 + 2);
  std::vector<double> v = {(double)C, -(double)C, 0.0, 1.0, -1.0};
  std::uniform_int_distribution<int64_t> d(-C, C);
  for (int i = 0; i < 300; ++i) v.push_back((double)d(rng));
  for (double x : v)
    for (double y : v) {
      const double r = f64_mulmod2(x, y, q, qinv);
      CHECK(int53(r) && md((i128)r - (i128)x * (i128)y, qi) == 0, "mulmod2 x=%.0f y=%.0f", x, y);
      // |xy - cq| <= q/2 + |xy| 4 2^-53 (h = RN(xy), q^-1 and h q^-1 rounded): about 0.6 q at
      // q near 2^50; the callers centre or canonicalise the product afterwards
      CHECK(std::fabs((long double)r) <= R(std::fabs((long double)x), std::fabs((long double)y), q),
            "mulmod2 bound x=%.0f y=%.0f r=%.0f", x, y, r);
    }
}

// Growth chains of the stage groups; returns the largest magnitude reached.
//   forward (CT): x' = a + t, y' = a - t with |t| <= R(B): B <- B + R(B)
//   inverse (GS): x' = a + b (B <- 2B), y' = product of a - b (|a - b| <= 2B)
static long double fwd_chain(long double B0, int stages, long double q) {
  long double B = B0;
  for (int s = 0; s < stages; ++s) B = B + R(B, (q - 1) / 2, q);
  return B;
}
static long double inv_chain(long double B0, int stages, long double q, long double* prod_in) {
  long double B = B0, pin = 0;
  for (int s = 0; s < stages; ++s) {
    pin = std::max(pin, 2 * B);
    const long double p = R(2 * B, (q - 1) / 2, q);
    B = std::max(2 * B, p);
  }
  *prod_in = pin;
  return B;
}

// ---- CPU emulation of the kernels' schedule (ArF64L / ArF64S) ------------
// Forward: stages 0..3 (column pass, from canonical words), raw intermediate
// (centred), rounds of stages 4..7, 8..11, 12..15 with centring between them,
// canonical words out.  Inverse: words in, centred, rounds 15..12, 11..8, 7..4
// with centring between them, raw intermediate, centred, stages 3..1, stage 0
// with N^-1 folded, canonical words out.  Checked against plain 128-bit loops.
template <class A>
static void emulate(uint64_t qi, int logn, int pattern, std::mt19937_64& rng, long double* maxabs) {
  const int N = 1 << logn;
  const uint64_t g = [&] { for (uint64_t c = 2;; ++c) if (powm(c, (qi - 1) / 2, qi) == qi - 1) return c; }();
  const uint64_t psi = powm(g, (qi - 1) / (2 * (uint64_t)N), qi), psii = powm(psi, qi - 2, qi);
  std::vector<uint64_t> T(N), Ti(N);
  for (int k = 0; k < N; ++k) { T[k] = powm(psi, brv(k, logn), qi); Ti[k] = powm(psii, brv(k, logn), qi); }
  LimbDev ld;
  std::memset(&ld, 0, sizeof(ld));
  ld.qd = (double)qi;
  ld.qinv = 1.0 / (double)qi;
  const uint64_t ninv = powm(N % qi, qi - 2, qi), ninvw = (uint64_t)((u128)ninv * Ti[1] % qi);
  ld.ninv_d = centred(ninv, qi);
  ld.ninvw_d = centred(ninvw, qi);
  const A ar(ld);
  std::vector<uint64_t> a(N);
  std::uniform_int_distribution<uint64_t> du(0, qi - 1);
  for (int i = 0; i < N; ++i)
    a[i] = pattern == 0 ? du(rng) : pattern == 1 ? qi - 1 : pattern == 2 ? (i & 1 ? qi - 1 : 0)
         : (i % 3 == 0 ? qi - 1 : i % 3 == 1 ? qi / 2 : qi / 2 + 1);
  // plain 128-bit reference
  std::vector<uint64_t> ref = a;
  for (int m = 1, t = N / 2; m < N; m <<= 1, t >>= 1)
    for (int i = 0; i < m; ++i)
      for (int j = 2 * i * t; j < 2 * i * t + t; ++j) {
        const uint64_t u = ref[j], v = (uint64_t)((u128)ref[j + t] * T[m + i] % qi);
        ref[j] = (u + v) % qi;
        ref[j + t] = (u + qi - v) % qi;
      }
  auto track = [&](const std::vector<double>& v) {
    for (double x : v) {
      *maxabs = std::max(*maxabs, (long double)std::fabs(x));
      CHECK(int53(x), "intermediate not an exact integer (q=%llu)", (unsigned long long)qi);
    }
  };
  std::vector<double> v(N);
  for (int i = 0; i < N; ++i) v[i] = ar.from_word((typename A::W)a[i]);
  for (int s = 0, m = 1, t = N / 2; m < N; ++s, m <<= 1, t >>= 1) {
    for (int i = 0; i < m; ++i)
      for (int j = 2 * i * t; j < 2 * i * t + t; ++j) ar.ct(v[j], v[j + t], centred(T[m + i], qi));
    track(v);
    if (s == 3) for (auto& x : v) x = ar.from_raw(ar.to_raw(x));  // column pass -> row pass
    else if ((s & 3) == 3 && s + 1 < logn) for (auto& x : v) ar.center(x);
  }
  std::vector<uint64_t> got(N);
  for (int i = 0; i < N; ++i) got[i] = (uint64_t)ar.to_word(v[i]);
  int bad = 0;
  for (int i = 0; i < N; ++i) bad += got[i] != ref[i];
  CHECK(bad == 0, "emulated forward differs in %d words (q=%llu pattern %d)", bad, (unsigned long long)qi, pattern);
  // inverse of the reference back to a
  for (int i = 0; i < N; ++i) { v[i] = ar.from_word((typename A::W)ref[i]); ar.center(v[i]); }
  for (int s = logn - 1, m = N / 2, t = 1; s >= 0; --s, m >>= 1, t <<= 1) {
    for (int i = 0; i < m; ++i)
      for (int j = 2 * i * t; j < 2 * i * t + t; ++j) {
        if (s == 0) ar.gs_fold(v[j], v[j + t], 0.0, ld);
        else ar.gs(v[j], v[j + t], centred(Ti[m + i], qi));
      }
    track(v);
    if (s == 4) for (auto& x : v) { x = ar.from_raw(ar.to_raw(x)); ar.center(x); }  // row -> column
    else if (s > 0 && ((logn - 1 - s) & 3) == 3) for (auto& x : v) ar.center(x);
  }
  bad = 0;
  for (int i = 0; i < N; ++i) bad += (uint64_t)ar.to_word(v[i]) != a[i];
  CHECK(bad == 0, "emulated inverse differs in %d words (q=%llu pattern %d)", bad, (unsigned long long)qi, pattern);
}

// ---- integer class ---------------------------------------------------------
static void check_i64(uint64_t q, std::mt19937_64& rng) {
  LimbDev ld;
  std::memset(&ld, 0, sizeof(ld));
  ld.q = q;
  ld.qbits = 64 - __builtin_clzll(q);
  ld.bmu = (uint64_t)(((u128)1 << (2 * ld.qbits)) / q);
  std::uniform_int_distribution<uint64_t> dq(0, q - 1), d4(0, 4 * q - 1), d2(0, 2 * q - 1), d64;
  const uint64_t ni = dq(rng), nw = dq(rng);
  ld.ninv = ni; ld.ninv_s = (uint64_t)(((u128)ni << 64) / q);
  ld.ninvw = nw; ld.ninvw_s = (uint64_t)(((u128)nw << 64) / q);
  const ArI64 ar(ld);
  std::vector<uint64_t> ys = {0, 1, q - 1, q, 2 * q - 1, 2 * q, 4 * q - 1, ~0ull, ~0ull - q};
  std::vector<uint64_t> ws = {0, 1, q - 1, q / 2, q / 2 + 1};
  for (int i = 0; i < 300; ++i) { ys.push_back(d64(rng)); ws.push_back(dq(rng)); }
  for (uint64_t w : ws) {
    const uint64_t s = (uint64_t)(((u128)w << 64) / q);
    for (uint64_t y : ys) {
      const uint64_t r = shoup_mul(y, w, s, q);
      CHECK(r < 2 * q && (u128)r % q == (u128)y * w % q, "shoup q=%llu y=%llu w=%llu",
            (unsigned long long)q, (unsigned long long)y, (unsigned long long)w);
    }
  }
  std::vector<uint64_t> as = {0, 1, q - 1, q - 2, q / 2};
  for (int i = 0; i < 300; ++i) as.push_back(dq(rng));
  for (uint64_t x : as)
    for (uint64_t y : as)
      CHECK(barrett_mul(x, y, q, ld.bmu, ld.qbits) == (uint64_t)((u128)x * y % q), "barrett x=%llu y=%llu",
            (unsigned long long)x, (unsigned long long)y);
  // Harvey butterflies: forward closed on [0, 4q), inverse on [0, 2q)
  std::vector<uint64_t> f = {0, q - 1, q, 2 * q - 1, 2 * q, 3 * q, 4 * q - 1}, h = {0, q - 1, q, 2 * q - 1};
  for (int i = 0; i < 60; ++i) { f.push_back(d4(rng)); h.push_back(d2(rng)); }
  for (uint64_t w : {(uint64_t)0, (uint64_t)1, q - 1, dq(rng), dq(rng)}) {
    TwI64 tw;
    tw.w = w;
    tw.ws = (uint64_t)(((u128)w << 64) / q);
    for (uint64_t x : f)
      for (uint64_t y : f) {
        uint64_t X = x, Y = y;
        ar.ct(X, Y, tw);
        const i128 t = (i128)((u128)y * w % q);
        CHECK(X < 4 * q && Y < 4 * q && md((i128)X - x - t, q) == 0 && md((i128)Y - x + t, q) == 0,
              "harvey ct q=%llu x=%llu y=%llu", (unsigned long long)q, (unsigned long long)x,
              (unsigned long long)y);
        CHECK(ar.to_word(X) == (uint64_t)md((i128)x + t, q), "to_word");
      }
    for (uint64_t x : h)
      for (uint64_t y : h) {
        uint64_t X = x, Y = y;
        ar.gs(X, Y, tw);
        CHECK(X < 2 * q && Y < 2 * q && md((i128)X - x - y, q) == 0 &&
                  md((i128)Y - ((i128)x - (i128)y) * (i128)w, q) == 0,
              "harvey gs q=%llu x=%llu y=%llu", (unsigned long long)q, (unsigned long long)x,
              (unsigned long long)y);
        X = x; Y = y;
        ar.gs_fold(X, Y, tw, ld);
        CHECK(X < 2 * q && Y < 2 * q && md((i128)X - ((i128)x + y) * (i128)ni, q) == 0 &&
                  md((i128)Y - ((i128)x - (i128)y) * (i128)nw, q) == 0, "harvey gs_fold");
      }
  }
}

// ---- gadget digits -----------------------------------------------------------
// Digit-by-digit definition: lower digits r mod B moved to [-B/2, B/2), r <- (r - d)/B;
// the top digit is the last remainder.
static void digits_ref(uint64_t x, int levels, int beta, int64_t* d) {
  i128 r = x;
  const i128 B = (i128)1 << beta;
  for (int j = 0; j + 1 < levels; ++j) {
    i128 t = r % B;
    if (t >= B / 2) t -= B;
    d[j] = (int64_t)t;
    r = (r - t) / B;
  }
  d[levels - 1] = (int64_t)r;
}
static void check_digits(uint64_t q, int levels, int beta, uint64_t x) {
  int64_t d[64];
  digits_ref(x, levels, beta, d);
  const uint64_t off = digit_offset(levels, beta);
  i128 back = 0;
  for (int j = levels - 1; j >= 0; --j) {
    const uint64_t got = signed_digit<uint64_t>(x, j, levels, beta, off, q);
    const uint64_t want = d[j] < 0 ? (uint64_t)((i128)q + d[j]) : (uint64_t)d[j];
    CHECK(got == want, "digit %d of x=%llu (q=%llu, l=%d, b=%d): %llu vs %llu", j,
          (unsigned long long)x, (unsigned long long)q, levels, beta, (unsigned long long)got,
          (unsigned long long)want);
    back = back * ((i128)1 << beta) + d[j];
    if (j + 1 < levels) CHECK(d[j] >= -(1LL << (beta - 1)) && d[j] < (1LL << (beta - 1)), "lower digit range");
    else CHECK(d[j] >= 0 && d[j] <= (1LL << (beta - 1)), "top digit %lld out of [0, B/2]", (long long)d[j]);
  }
  CHECK(back == (i128)x, "digits do not reconstruct x=%llu", (unsigned long long)x);
}

int main(int argc, char** argv) {
  if (argc == 2 && !std::strcmp(argv[1], "bound")) {
    std::printf("%llu\n", (unsigned long long)kF64LBound);
    return 0;
  }
  // argv: qL (largest admitted fp64-class prime), qM, qS32 (largest 32-bit), qC3, q62, q56
  if (argc != 7) return 2;
  uint64_t Q[6];
  for (int i = 0; i < 6; ++i) Q[i] = std::strtoull(argv[i + 1], nullptr, 10);
  const uint64_t qL = Q[0], qM = Q[1], q32 = Q[2], qc3 = Q[3], q62 = Q[4], q56 = Q[5];
  std::mt19937_64 rng(12345);

  // 1. growth chains at the class bounds, and their failure just above
  for (uint64_t q : {qL, qM}) {
    const long double lq = (long double)q;
    const long double f4 = fwd_chain(lq - 1, 4, lq);           // from canonical words
    long double pin = 0;
    const long double i4 = inv_chain((lq - 1) / 2 + 2, 4, lq, &pin);
    CHECK(f4 < TWO53 && i4 < TWO53 && pin < TWO53, "chain q=%llu: fwd %.4Lf q, inv %.4Lf q",
          (unsigned long long)q, f4 / lq, i4 / lq);
    check_f64_product(q, f4, rng);
    check_f64_product(q, pin, rng);
    check_center_canon(q, rng);
    check_f64_product2(q, rng);
    if (q == qL) std::printf("fp64 class q=%llu: forward group %.3Lf q, inverse group %.3Lf q\n",
                             (unsigned long long)q, f4 / lq, i4 / lq);
  }
  {
    // a modulus twice the class bound breaks the inverse chain: the bound is tight
    const long double q2 = 2.0L * (long double)kF64LBound;
    long double pin = 0;
    CHECK(inv_chain((q2 - 1) / 2 + 2, 4, q2, &pin) >= TWO53, "inverse chain would still fit at 2x bound");
  }
  {
    // 32-bit class: sixteen stages with no reduction inside a transform
    const long double lq = (long double)q32;
    const long double f16 = fwd_chain(lq - 1, 16, lq);
    long double pin = 0;
    const long double i16 = inv_chain(lq - 1, 16, lq, &pin);
    CHECK(f16 < TWO53 && i16 < TWO53 && pin < TWO53, "32-bit chains: fwd %.3Le inv %.3Le", f16, i16);
    check_f64_product(q32, f16, rng);
    check_f64_product(q32, pin, rng);
    check_center_canon(q32, rng);
    check_f64_product2(q32, rng);
    // the raw intermediate of the 32-bit class is a centred int32
    ArF64S::W wmax = 0;
    LimbDev ld;
    std::memset(&ld, 0, sizeof(ld));
    ld.qd = (double)q32;
    ld.qinv = 1.0 / (double)q32;
    const ArF64S ar(ld);
    std::uniform_int_distribution<int64_t> d(-(int64_t)f16, (int64_t)f16);
    for (int i = 0; i < 20000; ++i) {
      const double x = i < 2 ? (i ? -(double)(int64_t)f16 : (double)(int64_t)f16) : (double)d(rng);
      const double back = ar.from_raw(ar.to_raw(x));
      CHECK(md((i128)back - (i128)x, q32) == 0 && std::fabs(back) <= (double)(q32 / 2),
            "32-bit raw format x=%.0f", x);
      wmax = std::max(wmax, ar.to_word(x));
    }
    CHECK(wmax < q32, "32-bit canonical words");
  }
  {
    // 64-bit fp64 class conversions: words below 2^52 through the exponent trick
    LimbDev ld;
    std::memset(&ld, 0, sizeof(ld));
    ld.qd = (double)qL;
    ld.qinv = 1.0 / (double)qL;
    const ArF64L ar(ld);
    std::uniform_int_distribution<uint64_t> du(0, qL - 1);
    for (int i = 0; i < 20000; ++i) {
      const uint64_t w = i == 0 ? 0 : i == 1 ? qL - 1 : du(rng);
      CHECK(ar.from_word(w) == (double)w && ar.to_word(ar.from_word(w)) == w, "f64l word %llu",
            (unsigned long long)w);
    }
  }
  // 2. the integer class
  for (uint64_t q : {q62, q56, qL}) check_i64(q, rng);
  // 3. gadget digits: exhaustive on small bases, then eight wide combinations
  for (int beta = 1; beta <= 4; ++beta)
    for (int levels = 1; levels <= 4; ++levels) {
      const uint64_t q = 1ull << (levels * beta - 1);
      for (uint64_t x = 0; x < q; ++x) check_digits(q, levels, beta, x);
    }
  struct Combo { uint64_t q; int levels, beta; } combos[] = {
      {qc3, 3, 11}, {q32, 3, 11}, {q32, 2, 17}, {q32, 4, 9},
      {qL, 5, 11}, {qL, 2, 26}, {q62, 4, 16}, {q62, 2, 32}};
  for (const Combo& c : combos) {
    CHECK(c.levels * c.beta <= 64 && (c.levels * c.beta == 64 || c.q <= (1ull << (c.levels * c.beta - 1))),
          "combination out of the admitted range");
    std::uniform_int_distribution<uint64_t> du(0, c.q - 1);
    for (uint64_t x : {(uint64_t)0, (uint64_t)1, c.q - 1, c.q / 2, c.q / 2 + 1}) check_digits(c.q, c.levels, c.beta, x);
    for (int i = 0; i < 20000; ++i) check_digits(c.q, c.levels, c.beta, du(rng));
  }
  // 4. the kernels' schedule emulated at N = 2^16
  long double mL = 0, mS = 0;
  for (int pattern = 0; pattern < 4; ++pattern) {
    emulate<ArF64L>(qL, 16, pattern, rng, &mL);
    emulate<ArF64S>(q32, 16, pattern, rng, &mS);
  }
  std::printf("emulated N=2^16: largest |intermediate| %.3Lf q (fp64 64-bit), %.3Lf q (32-bit)\n",
              mL / qL, mS / q32);
  std::printf("%s %ld checks, %ld failures\n", fails ? "FAILED" : "ok", checks, fails);
  return fails ? 1 : 0;
}
"""


def _build(tmp_path):
    src = tmp_path / "arith.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arith"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                           f"-I{ROCM_INC}", f"-I{CSRC}", str(src), "-o", str(exe)])
    return exe


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC),
                    reason="g++ or the HIP headers not available")
def test_device_arithmetic_is_exact_at_its_bounds(tmp_path):
    exe = _build(tmp_path)
    bound = int(subprocess.run([str(exe), "bound"], capture_output=True, text=True, check=True).stdout)
    assert bound <= (1 << 50)
    qL = synth.primes_below(bound, 1 << 17, 1)[0]           # largest modulus the fp64 class admits
    qM = synth.primes_below(1 << 45, 1 << 17, 1)[0]
    q32 = synth.primes_below(1 << 32, 1 << 17, 1)[0]
    qc3 = synth.c3_prime()
    q62 = synth.primes_below(1 << 62, 1 << 17, 1)[0]
    q56 = synth.latency_prime()
    out = subprocess.run([str(exe), str(qL), str(qM), str(q32), str(qc3), str(q62), str(q56)],
                         capture_output=True, text=True, timeout=600)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout
