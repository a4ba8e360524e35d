// fused.hpp -- both passes of two-pass transforms in one persistent launch.
//
// The paper's hybrid NTT keeps one global synchronisation per transform
// between its two phases and runs it as a single kernel launch (Sec. V-D,
// Sec. VI-D).  Here persistent workgroups take pieces of all transforms of
// one launch from the work list of fused_order.hpp:
//   forward:  first phase = column pieces (BLOCK columns of N1 words),
//             second phase = row chunks (N2 words, the row pass);
//   inverse:  first phase = row chunks, second phase = column pieces.
// A finished first-phase piece makes its stores visible device-wide (release
// fence at agent scope: the stores leave the XCD's L2) and counts itself in the
// transform's counter; a second-phase piece waits until the counter reaches p1
// and acquires before it loads.  The intermediate of a transform is written
// and re-read while still in the caches, and the column pieces (memory bound)
// of some transforms run beside the row chunks (VALU bound) of others.
//
// The wait is bounded by `spin_limit` polls; by the list order it always ends
// long before (see fused_order.hpp), so the bound is a safeguard only.  A wait
// that gives up raises the launch's `expired` flag, which the host reads back
// and reports as NTT_ETIMEOUT; the piece then still runs (every address stays
// inside the transform), so the grid drains normally.
#pragma once

#include "ntt_kernels.hpp"
// after the kernels header, which brings the HIP runtime and NTT_HD
#include "fused_order.hpp"

namespace nttk {

struct FusedArgs {
  void* data;                 // [batch][L][N], transformed in place
  const LimbDev* limbs;       // [L]
  const uint32_t* cls_limbs;  // limbs of this launch's arithmetic class
  uint32_t L;
  uint32_t batch;
  uint32_t log_n;
  uint32_t n_tr;              // transforms: batch * (limbs of this class)
  uint32_t lag;               // list lag, 1 <= lag <= n_tr
  uint32_t p1, p2;            // pieces per transform in each phase
  uint32_t total;             // n_tr * (p1 + p2)
                              // forward: p1 = N2 / BLOCK column pieces, p2 = N1 row chunks;
                              // inverse: p1 = N1 row chunks, p2 = N2 / BLOCK column pieces
  uint32_t spin_limit;        // polls before a wait gives up
  uint32_t target_extra;      // added to every wait's target (testing: 1 = unreachable)
  uint32_t* work;             // [0] next item, [1 + t] first-phase pieces done of t
  uint32_t* expired;          // set to 1 when a wait gave up (zeroed by the host)
};

// At most 128 VGPRs (four waves per SIMD): the column piece of a 16-word
// column and a radix-16 row chunk each fit, and without the bound a radix-8
// (512-thread) instance takes more registers and fits one workgroup per CU.
template <class A, int LOGN1, int LOGN2, bool INV, int RB>
__global__ void __launch_bounds__((RowShape<LOGN2, RB>::BLOCK), 4)
fused_kernel(FusedArgs args) {
  using S = RowShape<LOGN2, RB>;
  static_assert(S::CPW == 1, "one row chunk per workgroup");
  using V = typename A::V;
  using W = typename A::W;
  __shared__ V lds[S::LDS_ELEMS];
  __shared__ uint32_t s_item;
  // Thread 0 does all counter traffic in one place, at the top of the loop:
  // it publishes the first-phase piece the workgroup has just finished (its
  // stores were released and the workgroup synchronised at the end of the
  // previous iteration) and fetches the next item.  Between two barriers
  // there is then a single thread-0 region, and the item index is read back
  // through readfirstlane so that every branch on it is uniform.  (With a
  // second thread-0 region at the end of the body the compiler nested the
  // loop so that, after a first-phase piece, the other waves went back to
  // the top without thread 0 and repeated the same item without end.)
  uint32_t done_t = 0xffffffffu;  // transform of the first-phase piece just finished
  for (;;) {
    if (threadIdx.x == 0) {
      if (done_t != 0xffffffffu) atomicAdd(args.work + 1 + done_t, 1u);
      s_item = atomicAdd(args.work, 1u);
    }
    __syncthreads();
    const uint32_t idx = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (idx >= args.total) break;
    const FusedItem it = fused_item(idx, args.n_tr, args.lag, args.p1, args.p2);
    const uint32_t poly = it.t % args.batch;
    const uint32_t limb = args.cls_limbs[it.t / args.batch];
    W* base = reinterpret_cast<W*>(args.data) + (((uint64_t)poly * args.L + limb) << args.log_n);
    const LimbDev& ld = args.limbs[limb];
    if (it.phase == 1) {
      if (threadIdx.x == 0) {
        const uint32_t target = args.p1 + args.target_extra;
        uint32_t polls = 0, seen;
        while ((seen = atomicAdd(args.work + 1 + it.t, 0u)) < target && polls < args.spin_limit) {
          __builtin_amdgcn_s_sleep(2);
          ++polls;
        }
        if (seen < target) atomicOr(args.expired, 1u);
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // Column pieces cover BLOCK of the N2 columns, row pieces one of the N1
    // rows; a piece index outside those ranges touches no memory.
    const bool columns = (it.phase == 0) != INV;
    if (columns) {
      if (it.sub < (1u << LOGN2) / S::BLOCK) {
        const uint32_t col = it.sub * S::BLOCK + threadIdx.x;
        col_one<A, LOGN1, INV, true>(base + col, base + col, ld, LOGN2, true);
      }
    } else if (it.sub < (1u << LOGN1)) {
      W* p = base + ((uint64_t)it.sub << LOGN2);
      row_chunk<A, LOGN2, INV, true, RB>(p, p, ld, (1u << LOGN1) + it.sub, threadIdx.x, lds, true);
    }
    if (it.phase == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    done_t = it.phase == 0 ? it.t : 0xffffffffu;
    __syncthreads();
  }
}

}  // namespace nttk
