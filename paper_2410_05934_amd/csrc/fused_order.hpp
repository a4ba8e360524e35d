// fused_order.hpp -- work-list order of the single-launch two-pass transform.
//
// A two-pass transform (N = N1 * N2, Sec. V-C/V-D) has one global
// synchronisation: every second-phase piece of a transform needs every
// first-phase piece of the same transform.  In the single-launch form the
// pieces of all n_tr transforms form one list that persistent workgroups take
// in order from an atomic counter.  Per transform t there are p1 first-phase
// items and p2 second-phase items.  The list is
//   head:  first-phase items of transforms 0 .. lag-1
//   body:  for k = 0 .. n_tr-lag-1: first-phase items of transform lag+k,
//          then second-phase items of transform k
//   tail:  second-phase items of transforms n_tr-lag .. n_tr-1
// so every second-phase item comes after all first-phase items of its
// transform, with about lag * (p1 + p2) items between them.  A workgroup that
// takes a second-phase item waits only for items that are earlier in the list,
// which running workgroups have already taken and finish without waiting:
// the wait always ends.
#pragma once

#include <cstdint>

#ifndef NTT_HD
#define NTT_HD __host__ __device__ __forceinline__
#endif

namespace nttk {

struct FusedItem {
  uint32_t phase;  // 0: first phase, 1: second phase
  uint32_t t;      // transform
  uint32_t sub;    // piece within the phase
};

// Item i of the list; requires 1 <= lag <= n_tr and i < n_tr * (p1 + p2).
NTT_HD FusedItem fused_item(uint32_t i, uint32_t n_tr, uint32_t lag, uint32_t p1, uint32_t p2) {
  FusedItem it;
  const uint32_t head = lag * p1;
  const uint32_t blk = p1 + p2;
  const uint32_t body = (n_tr - lag) * blk;
  if (i < head) {
    it.phase = 0;
    it.t = i / p1;
    it.sub = i % p1;
  } else if (i - head < body) {
    const uint32_t j = i - head;
    const uint32_t k = j / blk, r = j % blk;
    if (r < p1) {
      it.phase = 0;
      it.t = lag + k;
      it.sub = r;
    } else {
      it.phase = 1;
      it.t = k;
      it.sub = r - p1;
    }
  } else {
    const uint32_t j = i - head - body;
    it.phase = 1;
    it.t = n_tr - lag + j / p2;
    it.sub = j % p2;
  }
  return it;
}

}  // namespace nttk
