// numtheory.hpp -- host number theory of the library (128-bit products; runs
// once per plan or table): primality, quadratic non-residue, roots, inverses.
#pragma once

#include <cstdint>

namespace nttk {
using u128 = unsigned __int128;

inline uint64_t nt_mul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

inline uint64_t nt_pow(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = nt_mul(r, b, q);
    b = nt_mul(b, b, q);
  }
  return r;
}

// Miller-Rabin with the first twelve prime bases: exact for all 64-bit n.
inline bool nt_is_prime(uint64_t n) {
  static const uint64_t P[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : P) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : P) {
    uint64_t x = nt_pow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int i = 1; i < s && composite; ++i) {
      x = nt_mul(x, x, n);
      if (x == n - 1) composite = false;
    }
    if (composite) return false;
  }
  return true;
}

inline uint64_t nt_smallest_nonresidue(uint64_t q) {
  for (uint64_t g = 2; g < q; ++g)
    if (nt_pow(g, (q - 1) / 2, q) == q - 1) return g;
  return 0;
}

inline int ilog2(uint32_t n) {
  int l = 0;
  while ((1u << l) < n) ++l;
  return l;
}

inline uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}


inline int two_adic(uint64_t x) { return x ? __builtin_ctzll(x) : 64; }

}  // namespace nttk
