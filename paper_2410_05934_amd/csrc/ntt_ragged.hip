// ntt_ragged.hip -- ragged batches of transforms in one persistent launch.
//
// A ragged batch mixes jobs of different N, limb counts and moduli: forward or
// inverse transforms in place, and negacyclic products out = a * b (Eq. (1)).
// The host turns it into a list of work items -- one limb-row of one job each,
// or up to 16 limb-rows of the same small N, arithmetic class and kind --
// sorted largest first.  One persistent kernel per word width is launched with as many
// workgroups as fit on the chip at once; each workgroup takes the next item
// from an atomic counter and transforms its row(s) completely:
//   N <= 2^12      one row pass in LDS/registers (several rows side by side);
//   N >= 2^13      column pass then row pass inside the same workgroup, the
//                  intermediate staying in the workgroup's own global memory
//                  view (written and re-read by the same CU, separated by a
//                  workgroup barrier).
// No item waits for another, so every workgroup exits once the counter passes
// the end of the list.  This is the paper's single-kernel-launch form of the
// hybrid NTT (Sec. V-D) applied to a batch: the one global synchronisation of
// each transform becomes a workgroup barrier because a workgroup owns the
// whole transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "ntt_internal.hpp"
#include "ntt_kernels.hpp"

namespace nttk {

constexpr int kRaggedBlock = 256;
constexpr int kRaggedRows = 16;
constexpr int kRaggedLds = 4096 + 256;  // one 2^12 chunk or several smaller ones, padded

// Job kinds (the op field of ntt_job).
constexpr uint32_t kOpFwd = NTT_OP_FORWARD, kOpInv = NTT_OP_INVERSE, kOpMul = NTT_OP_POLYMUL;

struct RaggedJobDev {
  void* data;        // transforms: the words transformed in place; polymul: the product
  const void* a;     // polymul operands (natural order, not modified)
  const void* b;
  void* ws;          // polymul with a column pass: b's intermediate, [batch][L][N]
  const LimbDev* limbs;
  uint32_t L;
  uint32_t log_n;
  uint32_t log_n2;  // row-pass length inside the workgroup (== log_n for one pass)
  uint32_t op;      // kOpFwd, kOpInv or kOpMul
};

struct RaggedItem {
  uint32_t job;
  uint32_t nrows;
  uint32_t cls;
  uint32_t log_n;
  uint32_t log_n2;
  uint32_t op;
  uint32_t rows[kRaggedRows];  // flattened row index b * L + l
};

template <class A, int LOGN, bool INV>
__device__ __noinline__ void ragged_single(const RaggedJobDev* jp, const RaggedItem* ip,
                                           typename A::V* lds) {
  using S = RowShape<LOGN>;
  using W = typename A::W;
  const uint32_t ci = threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
  const bool valid = ci < ip->nrows;
  const uint32_t row = ip->rows[valid ? ci : 0];
  W* p = reinterpret_cast<W*>(jp->data) + ((uint64_t)row << LOGN);
  row_chunk<A, LOGN, INV, false>(p, p, jp->limbs[row % jp->L], 1u, tt, lds + ci * S::CHUNK_LDS,
                                 valid);
}

template <class A, int LOGN1, int LOGN2, bool INV>
__device__ __noinline__ void ragged_two_pass(const RaggedJobDev* jp, const RaggedItem* ip,
                                             typename A::V* lds) {
  using S = RowShape<LOGN2>;
  using W = typename A::W;
  // Loop bounds are taken from the job at run time: with compile-time trip
  // counts the compiler interleaves iterations and doubles register use.
  const uint32_t N1 = 1u << (jp->log_n - jp->log_n2), N2 = 1u << jp->log_n2;
  const uint32_t row = ip->rows[0];
  W* p = reinterpret_cast<W*>(jp->data) + ((uint64_t)row << (LOGN1 + LOGN2));
  const LimbDev& ld = jp->limbs[row % jp->L];
  const uint32_t ci = threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
  auto columns = [&]() {
#pragma unroll 1
    for (uint32_t r = threadIdx.x; r < N2; r += kRaggedBlock)
      col_one<A, LOGN1, INV, true>(p + r, p + r, ld, LOGN2, true);
  };
  auto rows = [&]() {
    // the workgroup's kRaggedBlock threads hold kRaggedBlock / TPC chunks at a time
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < N1; c0 += kRaggedBlock / S::TPC) {
      const uint32_t c = c0 + ci;
      const bool valid = c < N1;
      W* q = p + ((uint64_t)(valid ? c : 0) << LOGN2);
      row_chunk<A, LOGN2, INV, true>(q, q, ld, N1 + c, tt, lds + ci * S::CHUNK_LDS, valid);
    }
  };
  if constexpr (!INV) {
    columns();
    __threadfence_block();
    __syncthreads();
    rows();
  } else {
    rows();
    __threadfence_block();
    __syncthreads();
    columns();
  }
  __threadfence_block();
  __syncthreads();
}

// Negacyclic products of up to kRaggedRows limb-rows of one small N side by
// side: each chunk forward-transforms a and b, multiplies and inverse-transforms
// in registers/LDS (the fused product of polymul), writing out.
template <class A, int LOGN>
__device__ __noinline__ void ragged_polymul_single(const RaggedJobDev* jp, const RaggedItem* ip,
                                                   typename A::V* lds) {
  using S = RowShape<LOGN>;
  using W = typename A::W;
  const uint32_t ci = threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
  const bool valid = ci < ip->nrows;
  const uint32_t row = ip->rows[valid ? ci : 0];
  const uint64_t off = (uint64_t)row << LOGN;
  polymul_chunk<A, LOGN, false>(reinterpret_cast<W*>(jp->data) + off,
                                reinterpret_cast<const W*>(jp->a) + off,
                                reinterpret_cast<const W*>(jp->b) + off, jp->limbs[row % jp->L], 1u,
                                tt, lds + ci * S::CHUNK_LDS, valid);
}

// One large negacyclic product in one workgroup: the column passes of a (into
// out) and b (into the job's workspace), the fused product rows over both
// intermediates, then the inverse column pass of out -- each phase separated by
// a workgroup barrier, as in ragged_two_pass.
template <class A, int LOGN1, int LOGN2>
__device__ __noinline__ void ragged_polymul_two_pass(const RaggedJobDev* jp, const RaggedItem* ip,
                                                     typename A::V* lds) {
  using S = RowShape<LOGN2>;
  using W = typename A::W;
  const uint32_t N1 = 1u << (jp->log_n - jp->log_n2), N2 = 1u << jp->log_n2;
  const uint32_t row = ip->rows[0];
  const uint64_t off = (uint64_t)row << (LOGN1 + LOGN2);
  W* po = reinterpret_cast<W*>(jp->data) + off;
  W* pw = reinterpret_cast<W*>(jp->ws) + off;
  const W* pa = reinterpret_cast<const W*>(jp->a) + off;
  const W* pb = reinterpret_cast<const W*>(jp->b) + off;
  const LimbDev& ld = jp->limbs[row % jp->L];
  const uint32_t ci = threadIdx.x / S::TPC;
  const uint32_t tt = threadIdx.x & (S::TPC - 1);
#pragma unroll 1
  for (uint32_t r = threadIdx.x; r < N2; r += kRaggedBlock) {
    col_one<A, LOGN1, false, true>(po + r, pa + r, ld, LOGN2, true);
    col_one<A, LOGN1, false, true>(pw + r, pb + r, ld, LOGN2, true);
  }
  __threadfence_block();
  __syncthreads();
#pragma unroll 1
  for (uint32_t c0 = 0; c0 < N1; c0 += kRaggedBlock / S::TPC) {
    const uint32_t c = c0 + ci;
    const bool valid = c < N1;
    const uint64_t co = (uint64_t)(valid ? c : 0) << LOGN2;
    polymul_chunk<A, LOGN2, true>(po + co, po + co, pw + co, ld, N1 + c, tt,
                                  lds + ci * S::CHUNK_LDS, valid);
  }
  __threadfence_block();
  __syncthreads();
#pragma unroll 1
  for (uint32_t r = threadIdx.x; r < N2; r += kRaggedBlock)
    col_one<A, LOGN1, true, true>(po + r, po + r, ld, LOGN2, true);
  __threadfence_block();
  __syncthreads();
}

template <class A>
__device__ void ragged_dispatch_pm(const RaggedJobDev& j, const RaggedItem& it, typename A::V* lds) {
  if (it.log_n2 == it.log_n) {
    switch (it.log_n) {
      case 4: ragged_polymul_single<A, 4>(&j, &it, lds); break;
      case 5: ragged_polymul_single<A, 5>(&j, &it, lds); break;
      case 6: ragged_polymul_single<A, 6>(&j, &it, lds); break;
      case 7: ragged_polymul_single<A, 7>(&j, &it, lds); break;
      case 8: ragged_polymul_single<A, 8>(&j, &it, lds); break;
      case 9: ragged_polymul_single<A, 9>(&j, &it, lds); break;
      case 10: ragged_polymul_single<A, 10>(&j, &it, lds); break;
      case 11: ragged_polymul_single<A, 11>(&j, &it, lds); break;
      case 12: ragged_polymul_single<A, 12>(&j, &it, lds); break;
      default: break;
    }
  } else if (it.log_n2 == 12) {
    switch (it.log_n) {
      case 13: ragged_polymul_two_pass<A, 1, 12>(&j, &it, lds); break;
      case 14: ragged_polymul_two_pass<A, 2, 12>(&j, &it, lds); break;
      case 15: ragged_polymul_two_pass<A, 3, 12>(&j, &it, lds); break;
      case 16: ragged_polymul_two_pass<A, 4, 12>(&j, &it, lds); break;
      default: break;
    }
  } else if (it.log_n2 == 11) {
    switch (it.log_n) {
      case 13: ragged_polymul_two_pass<A, 2, 11>(&j, &it, lds); break;
      case 14: ragged_polymul_two_pass<A, 3, 11>(&j, &it, lds); break;
      case 15: ragged_polymul_two_pass<A, 4, 11>(&j, &it, lds); break;
      case 16: ragged_polymul_two_pass<A, 5, 11>(&j, &it, lds); break;
      default: break;
    }
  }
}

template <class A, bool INV>
__device__ void ragged_dispatch_size(const RaggedJobDev& j, const RaggedItem& it,
                                     typename A::V* lds) {
  if (it.log_n2 == it.log_n) {
    switch (it.log_n) {
      case 4: ragged_single<A, 4, INV>(&j, &it, lds); break;
      case 5: ragged_single<A, 5, INV>(&j, &it, lds); break;
      case 6: ragged_single<A, 6, INV>(&j, &it, lds); break;
      case 7: ragged_single<A, 7, INV>(&j, &it, lds); break;
      case 8: ragged_single<A, 8, INV>(&j, &it, lds); break;
      case 9: ragged_single<A, 9, INV>(&j, &it, lds); break;
      case 10: ragged_single<A, 10, INV>(&j, &it, lds); break;
      case 11: ragged_single<A, 11, INV>(&j, &it, lds); break;
      case 12: ragged_single<A, 12, INV>(&j, &it, lds); break;
      default: break;
    }
  } else if (it.log_n2 == 12) {
    switch (it.log_n) {
      case 13: ragged_two_pass<A, 1, 12, INV>(&j, &it, lds); break;
      case 14: ragged_two_pass<A, 2, 12, INV>(&j, &it, lds); break;
      case 15: ragged_two_pass<A, 3, 12, INV>(&j, &it, lds); break;
      case 16: ragged_two_pass<A, 4, 12, INV>(&j, &it, lds); break;
      default: break;
    }
  } else if (it.log_n2 == 11) {
    switch (it.log_n) {
      case 13: ragged_two_pass<A, 2, 11, INV>(&j, &it, lds); break;
      case 14: ragged_two_pass<A, 3, 11, INV>(&j, &it, lds); break;
      case 15: ragged_two_pass<A, 4, 11, INV>(&j, &it, lds); break;
      case 16: ragged_two_pass<A, 5, 11, INV>(&j, &it, lds); break;
      default: break;
    }
  }
}

template <class A>
__device__ void ragged_dispatch(const RaggedJobDev& j, const RaggedItem& it, double* lds) {
  using V = typename A::V;
  V* l = reinterpret_cast<V*>(lds);
  if (it.op == kOpMul) ragged_dispatch_pm<A>(j, it, l);
  else if (it.op == kOpInv) ragged_dispatch_size<A, true>(j, it, l);
  else ragged_dispatch_size<A, false>(j, it, l);
}

struct RaggedArgs {
  const RaggedJobDev* jobs;
  const RaggedItem* items;
  uint32_t n_items;
  uint32_t* counter;
};

// WIDE = false: 32-bit words (class 0); WIDE = true: 64-bit words (classes 1, 2).
// Four waves per SIMD (at most 128 VGPRs): each tile shape alone fits, and the
// budget keeps the allocator from trading occupancy for the union of all shapes.
template <bool WIDE>
__global__ void __launch_bounds__(kRaggedBlock, 4) ragged_kernel(RaggedArgs args) {
  __shared__ double lds[kRaggedLds];
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(args.counter, 1u);
    __syncthreads();
    const uint32_t idx = s_item;
    __syncthreads();
    if (idx >= args.n_items) break;
    const RaggedItem& it = args.items[idx];
    const RaggedJobDev& j = args.jobs[it.job];
    if constexpr (WIDE) {
      if (it.cls == 1) ragged_dispatch<ArF64L>(j, it, lds);
      else ragged_dispatch<ArI64>(j, it, lds);
    } else {
      ragged_dispatch<ArF64S>(j, it, lds);
    }
  }
}

// ---------------------------------------------------------------------------
// Grouped two-pass launches for the large transforms of a batch (N >= 2^13):
// every limb-row of one (N, class, direction) goes into one row table, and one
// column launch plus one row launch (2^12-word rows) cover all of them, as the
// batched transform does for one plan.  Table rows are sorted by prime, and
// row chunks are ordered row-fastest, so neighbouring workgroups share twiddles.
struct RowRef {
  void* data;          // 2^log_n words of one limb-row (written)
  const void* src;     // the words read by a column pass that is not in place
  const LimbDev* ld;   // its modulus (device copy inside the owning plan)
};

struct GangArgs {
  const RowRef* rows;
  uint32_t n_rows;
  uint32_t log_n1;     // column stages; rows are 2^12 words
  uint32_t from_src;   // column pass reads rows[i].src (else rows[i].data, in place)
};

constexpr int kGangLogN2 = 12;

template <class A, int LOGN1, bool INV>
__global__ void __launch_bounds__(kColBlock) gang_col_kernel(GangArgs g) {
  using W = typename A::W;
  const uint32_t gid = blockIdx.x * kColBlock + threadIdx.x;
  const bool valid = gid < (g.n_rows << kGangLogN2);
  const uint32_t x = valid ? gid : 0;
  const RowRef rr = g.rows[x >> kGangLogN2];
  const uint32_t r = x & ((1u << kGangLogN2) - 1u);
  W* p = reinterpret_cast<W*>(rr.data) + r;
  const W* q = g.from_src ? reinterpret_cast<const W*>(rr.src) + r : p;
  col_one<A, LOGN1, INV, true>(p, q, *rr.ld, kGangLogN2, valid);
}

// Fused product rows of a polymul group: the table holds n_rows product rows
// (data = out, intermediate of a) followed by n_rows workspace rows (data =
// intermediate of b); chunk c of product row i reads both intermediates and
// writes the product's intermediate over out.
template <class A>
__global__ void __launch_bounds__((RowShape<kGangLogN2, 4>::BLOCK), 4) gang_pm_row_kernel(GangArgs g) {
  using S = RowShape<kGangLogN2, 4>;
  static_assert(S::CPW == 1, "one chunk per workgroup");
  using V = typename A::V;
  using W = typename A::W;
  __shared__ V lds[S::LDS_ELEMS];
  const uint32_t total = g.n_rows << g.log_n1;
  const uint32_t k0 = xcd_block(blockIdx.x, gridDim.x);
  const bool valid = k0 < total;
  const uint32_t k = valid ? k0 : 0;
  const uint32_t i = k % g.n_rows, c = k / g.n_rows;
  const RowRef ra = g.rows[i], rb = g.rows[i + g.n_rows];
  W* p = reinterpret_cast<W*>(ra.data) + ((uint64_t)c << kGangLogN2);
  const W* q = reinterpret_cast<const W*>(rb.data) + ((uint64_t)c << kGangLogN2);
  polymul_chunk<A, kGangLogN2, true, 4>(p, p, q, *ra.ld, (1u << g.log_n1) + c, threadIdx.x, lds,
                                        valid);
}

template <class A, bool INV>
__global__ void __launch_bounds__((RowShape<kGangLogN2, 4>::BLOCK), 4) gang_row_kernel(GangArgs g) {
  using S = RowShape<kGangLogN2, 4>;
  static_assert(S::CPW == 1, "one chunk per workgroup");
  using V = typename A::V;
  using W = typename A::W;
  __shared__ V lds[S::LDS_ELEMS];
  const uint32_t total = g.n_rows << g.log_n1;
  const uint32_t k0 = xcd_block(blockIdx.x, gridDim.x);
  const bool valid = k0 < total;
  const uint32_t k = valid ? k0 : 0;
  const uint32_t i = k % g.n_rows, c = k / g.n_rows;
  const RowRef rr = g.rows[i];
  W* p = reinterpret_cast<W*>(rr.data) + ((uint64_t)c << kGangLogN2);
  row_chunk<A, kGangLogN2, INV, true, 4>(p, p, *rr.ld, (1u << g.log_n1) + c, threadIdx.x, lds,
                                         valid);
}

template <class A, bool INV>
hipError_t launch_gang_col(const GangArgs& g, hipStream_t s, bool timed) {
  const uint32_t cols = g.n_rows << kGangLogN2;
  const uint64_t words = (uint64_t)g.n_rows << (g.log_n1 + kGangLogN2);
  LaunchTimer t(timed ? "gang_col" : nullptr, A::kName, (int)g.log_n1, INV, true, words, s);
  const dim3 grid((cols + kColBlock - 1) / kColBlock);
  switch (g.log_n1) {
    case 1: hipLaunchKernelGGL((gang_col_kernel<A, 1, INV>), grid, dim3(kColBlock), 0, s, g); break;
    case 2: hipLaunchKernelGGL((gang_col_kernel<A, 2, INV>), grid, dim3(kColBlock), 0, s, g); break;
    case 3: hipLaunchKernelGGL((gang_col_kernel<A, 3, INV>), grid, dim3(kColBlock), 0, s, g); break;
    case 4: hipLaunchKernelGGL((gang_col_kernel<A, 4, INV>), grid, dim3(kColBlock), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// A polymul group (table: n product rows, then n workspace rows): forward column
// passes of a and b over all 2n rows in one launch, the fused product rows, the
// inverse column pass of the product rows.
template <class A>
hipError_t launch_gang_pm(GangArgs g, hipStream_t s, bool timed) {
  GangArgs both = g;
  both.n_rows = 2 * g.n_rows;
  both.from_src = 1;
  hipError_t e = launch_gang_col<A, false>(both, s, timed);
  if (e != hipSuccess) return e;
  {
    const uint64_t words = (uint64_t)g.n_rows << (g.log_n1 + kGangLogN2);
    LaunchTimer t(timed ? "gang_polymul_row" : nullptr, A::kName, kGangLogN2, false, true, words, s);
    hipLaunchKernelGGL((gang_pm_row_kernel<A>), dim3(g.n_rows << g.log_n1),
                       dim3(RowShape<kGangLogN2, 4>::BLOCK), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  g.from_src = 0;
  return launch_gang_col<A, true>(g, s, timed);
}

template <class A, bool INV>
hipError_t launch_gang(const GangArgs& g, hipStream_t s, bool timed) {
  const uint32_t chunks = g.n_rows << g.log_n1;
  const uint64_t words = (uint64_t)g.n_rows << (g.log_n1 + kGangLogN2);
  auto col = [&]() -> hipError_t { return launch_gang_col<A, INV>(g, s, timed); };
  auto row = [&]() -> hipError_t {
    LaunchTimer t(timed ? "gang_row" : nullptr, A::kName, kGangLogN2, INV, true, words, s);
    hipLaunchKernelGGL((gang_row_kernel<A, INV>), dim3(chunks),
                       dim3(RowShape<kGangLogN2, 4>::BLOCK), 0, s, g);
    return hipGetLastError();
  };
  hipError_t e = INV ? row() : col();
  if (e == hipSuccess) e = INV ? col() : row();
  return e;
}

__global__ void zero_counters(uint32_t* c, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0;
}

}  // namespace nttk

using namespace nttk;

struct ntt_ragged_s {
  int device = 0;
  std::vector<RaggedJobDev> jobs;
  std::vector<RaggedItem> items;
  uint32_t n_items[2] = {0, 0};  // [narrow, wide]
  RaggedJobDev* d_jobs = nullptr;
  RaggedItem* d_items = nullptr;
  uint32_t* d_counter = nullptr;  // [2]
  uint32_t grid[2] = {0, 0};
  // grouped launches of the N >= 2^13 transforms
  struct Gang {
    uint32_t cls, log_n, op, off, n;  // polymul: table rows off .. off + 2n - 1
  };
  std::vector<Gang> gangs;
  RowRef* d_rows = nullptr;
  void* d_ws = nullptr;  // workspace of the polymul jobs with a column pass
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::mutex mu;
};

namespace {

uint32_t ragged_split_for(uint32_t log_n, uint32_t flags) {
  if (log_n <= 12) return log_n;
  const uint32_t forced = (flags >> 8) & 0xf;  // NTT_RAGGED_ROW_LOG(n2)
  if (forced == 11 || forced == 12) return forced;
  return tuned_ragged_row_log(log_n, 12);
}

// Launch everything on `s`; with `branches` (graph capture), each group of
// large transforms runs on its own stream forked from and joined back to `s`,
// so the captured graph has the groups and the persistent kernel as parallel
// branches (they touch disjoint data).
hipError_t launch_all(ntt_ragged_s* r, hipStream_t s, bool timed,
                      const std::vector<hipStream_t>* branches = nullptr) {
  hipError_t e = hipSuccess;
  std::vector<hipEvent_t> events;  // fork, then one join per branch
  auto cleanup = [&]() {
    for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
  };
  const bool fork = branches && !branches->empty() && !r->gangs.empty();
  if (fork) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) events.push_back(ev);
    if (e == hipSuccess) e = hipEventRecord(ev, s);
    for (size_t b = 0; e == hipSuccess && b < branches->size(); ++b)
      e = hipStreamWaitEvent((*branches)[b], ev, 0);
    if (e != hipSuccess) {
      cleanup();
      return e;
    }
  }
  hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, s, r->d_counter, 2u);
  e = hipGetLastError();
  if (e != hipSuccess) {
    cleanup();
    return e;
  }
  for (int w = 0; w < 2; ++w) {
    if (r->n_items[w] == 0) continue;
    RaggedArgs a;
    a.jobs = r->d_jobs;
    a.items = r->d_items + (w == 1 ? r->n_items[0] : 0);
    a.n_items = r->n_items[w];
    a.counter = r->d_counter + w;
    LaunchTimer t(timed ? "ragged" : nullptr, w ? "u64" : "u32", 0, false, false, 0, s);
    if (w) hipLaunchKernelGGL(ragged_kernel<true>, dim3(r->grid[w]), dim3(kRaggedBlock), 0, s, a);
    else hipLaunchKernelGGL(ragged_kernel<false>, dim3(r->grid[w]), dim3(kRaggedBlock), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) {
      cleanup();
      return e;
    }
  }
  for (size_t i = 0; i < r->gangs.size(); ++i) {
    const auto& gg = r->gangs[i];
    hipStream_t gs = fork ? (*branches)[i % branches->size()] : s;
    GangArgs g;
    g.rows = r->d_rows + gg.off;
    g.n_rows = gg.n;
    g.log_n1 = gg.log_n - kGangLogN2;
    g.from_src = 0;
    if (gg.op == kOpMul) {
      if (gg.cls == 0) e = launch_gang_pm<ArF64S>(g, gs, timed);
      else if (gg.cls == 1) e = launch_gang_pm<ArF64L>(g, gs, timed);
      else e = launch_gang_pm<ArI64>(g, gs, timed);
    } else {
      const bool inv = gg.op == kOpInv;
      if (gg.cls == 0) e = inv ? launch_gang<ArF64S, true>(g, gs, timed) : launch_gang<ArF64S, false>(g, gs, timed);
      else if (gg.cls == 1) e = inv ? launch_gang<ArF64L, true>(g, gs, timed) : launch_gang<ArF64L, false>(g, gs, timed);
      else e = inv ? launch_gang<ArI64, true>(g, gs, timed) : launch_gang<ArI64, false>(g, gs, timed);
    }
    if (e != hipSuccess) {
      cleanup();
      return e;
    }
  }
  if (fork) {
    for (size_t b = 0; e == hipSuccess && b < branches->size(); ++b) {
      hipEvent_t ev = nullptr;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) events.push_back(ev);
      if (e == hipSuccess) e = hipEventRecord(ev, (*branches)[b]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    }
  }
  cleanup();
  return e;
}

void free_ragged(ntt_ragged_s* r) {
  if (!r) return;
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  if (r->graph) (void)hipGraphDestroy(r->graph);
  if (r->d_jobs) (void)hipFree(r->d_jobs);
  if (r->d_items) (void)hipFree(r->d_items);
  if (r->d_counter) (void)hipFree(r->d_counter);
  if (r->d_rows) (void)hipFree(r->d_rows);
  if (r->d_ws) (void)hipFree(r->d_ws);
  delete r;
}

}  // namespace

extern "C" {

ntt_status ntt_ragged_create(ntt_ragged_t* out, const ntt_job* jobs, uint32_t n, uint32_t flags) {
  if (!out || !jobs || n == 0) return fail(NTT_EINVAL, "null argument or empty job list");
  *out = nullptr;
  ntt_ragged_s* r = new (std::nothrow) ntt_ragged_s();
  if (!r) return fail(NTT_ENOMEM, "host allocation");
  r->use_graph = !(flags & NTT_RAGGED_NO_GRAPH);
  hipError_t e = hipGetDevice(&r->device);
  if (e != hipSuccess) {
    free_ragged(r);
    return hip_fail(e, "hipGetDevice");
  }
  std::vector<RaggedItem> wide, narrow;
  const bool in_wg = (flags & NTT_RAGGED_IN_WORKGROUP) != 0;
  // (class, log_n, op) -> rows for the grouped launches: (twiddle table address,
  // row, companion row) -- the companion is the workspace row of a polymul
  struct GroupRow {
    uint64_t tw;
    RowRef r, r2;
  };
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::vector<GroupRow>> groups;
  // Workspace of the polymul jobs with a column pass (offsets into one
  // allocation, patched in once it exists): job index -> byte offset.
  std::vector<std::pair<uint32_t, size_t>> ws_jobs;
  size_t ws_bytes = 0;
  for (uint32_t ji = 0; ji < n; ++ji) {
    const ntt_job& jb = jobs[ji];
    if (!jb.plan || !jb.out || jb.batch == 0 || jb.op > kOpMul) {
      free_ragged(r);
      return fail(NTT_EINVAL, "job %u: null plan/out, zero batch or bad op", ji);
    }
    const ntt_plan_s* p = jb.plan;
    const size_t wbytes = p->word_bits / 8;
    const uint64_t words = (uint64_t)jb.batch * p->L << p->log_n;
    if (jb.op == kOpMul) {
      if (!jb.a || !jb.b) {
        free_ragged(r);
        return fail(NTT_EINVAL, "job %u: a polymul job needs a and b", ji);
      }
      const uintptr_t o = reinterpret_cast<uintptr_t>(jb.out), bytes = words * wbytes;
      for (const void* x : {jb.a, jb.b}) {
        const uintptr_t i = reinterpret_cast<uintptr_t>(x);
        if (o < i + bytes && i < o + bytes) {
          free_ragged(r);
          return fail(NTT_EINVAL, "job %u: out must not overlap a or b", ji);
        }
      }
    } else if ((jb.a && jb.a != jb.out) || (jb.b && jb.b != jb.out)) {
      free_ragged(r);
      return fail(NTT_EINVAL, "job %u: a transform job works in place on out (a, b NULL)", ji);
    }
    if (p->device != r->device) {
      free_ragged(r);
      return fail(NTT_EINVAL, "job %u: plan lives on another device", ji);
    }
    if (p->log_n < 4) {
      free_ragged(r);
      return fail(NTT_EINVAL, "job %u: ragged batches need N >= 16", ji);
    }
    RaggedJobDev jd;
    jd.data = jb.out;
    jd.a = jb.a;
    jd.b = jb.b;
    jd.ws = nullptr;
    jd.limbs = p->d_limbs;
    jd.L = p->L;
    jd.log_n = p->log_n;
    jd.log_n2 = ragged_split_for(p->log_n, flags);
    jd.op = jb.op;
    if (jb.op == kOpMul && p->log_n > 12) {
      ws_jobs.push_back({ji, ws_bytes});
      ws_bytes += (size_t)words * wbytes;
    }
    r->jobs.push_back(jd);
    if (p->log_n > 12 && !in_wg) {
      for (uint32_t b = 0; b < jb.batch; ++b)
        for (uint32_t l = 0; l < p->L; ++l) {
          const size_t off = (((uint64_t)b * p->L + l) << p->log_n) * wbytes;
          GroupRow gr;
          gr.tw = reinterpret_cast<uint64_t>(p->h_limbs[l].twf);
          gr.r.data = static_cast<unsigned char*>(jb.out) + off;
          gr.r.src = jb.op == kOpMul ? static_cast<const unsigned char*>(jb.a) + off : nullptr;
          gr.r.ld = p->d_limbs + l;
          // workspace row: an offset for now (patched once the workspace exists)
          gr.r2.data = reinterpret_cast<void*>(ws_bytes - (size_t)words * wbytes + off);
          gr.r2.src = jb.op == kOpMul ? static_cast<const unsigned char*>(jb.b) + off : nullptr;
          gr.r2.ld = gr.r.ld;
          groups[std::make_tuple((uint32_t)p->cls[l], p->log_n, jb.op)].push_back(gr);
        }
      continue;
    }
    const uint32_t per = p->log_n <= 12 ? std::min<uint32_t>(kRaggedRows, std::max<uint32_t>(1u, kRaggedBlock / ((1u << p->log_n) / 16)))
                                        : 1u;
    // Group rows of the same limb class; rows run b-major then l.
    for (uint32_t c = 0; c < 3; ++c) {
      RaggedItem it;
      std::memset(&it, 0, sizeof(it));
      it.job = ji;
      it.cls = c;
      it.log_n = p->log_n;
      it.log_n2 = jd.log_n2;
      it.op = jb.op;
      for (uint32_t b = 0; b < jb.batch; ++b) {
        for (uint32_t l = 0; l < p->L; ++l) {
          if (p->cls[l] != c) continue;
          it.rows[it.nrows++] = b * p->L + l;
          if (it.nrows == per) {
            (c == 0 ? narrow : wide).push_back(it);
            it.nrows = 0;
          }
        }
      }
      if (it.nrows) (c == 0 ? narrow : wide).push_back(it);
    }
  }
  // a product is three transforms' work
  auto cost = [](const RaggedItem& it) {
    return ((uint64_t)it.nrows * it.log_n << it.log_n) * (it.op == kOpMul ? 3u : 1u);
  };
  auto by_cost = [&](const RaggedItem& a, const RaggedItem& b) { return cost(a) > cost(b); };
  std::stable_sort(narrow.begin(), narrow.end(), by_cost);
  std::stable_sort(wide.begin(), wide.end(), by_cost);
  if (ws_bytes) {
    e = hipMalloc(&r->d_ws, ws_bytes);
    if (e != hipSuccess) {
      free_ragged(r);
      return hip_fail(e, "ragged polymul workspace");
    }
    for (const auto& jw : ws_jobs)
      r->jobs[jw.first].ws = static_cast<unsigned char*>(r->d_ws) + jw.second;
  }
  std::vector<RowRef> table;
  for (auto& kv : groups) {
    auto& v = kv.second;
    const uint32_t op = std::get<2>(kv.first);
    if (((uint64_t)v.size() << std::get<1>(kv.first)) * (op == kOpMul ? 2 : 1) >= (1ull << 32)) {
      free_ragged(r);
      return fail(NTT_EINVAL, "a group of 2^%u-word rows holds 2^32 words or more",
                  std::get<1>(kv.first));
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const GroupRow& x, const GroupRow& y) { return x.tw < y.tw; });
    ntt_ragged_s::Gang gg;
    gg.cls = std::get<0>(kv.first);
    gg.log_n = std::get<1>(kv.first);
    gg.op = op;
    gg.off = (uint32_t)table.size();
    gg.n = (uint32_t)v.size();
    for (const auto& x : v) table.push_back(x.r);
    if (op == kOpMul) {
      for (const auto& x : v) {
        RowRef w = x.r2;
        w.data = static_cast<unsigned char*>(r->d_ws) + reinterpret_cast<uintptr_t>(x.r2.data);
        table.push_back(w);
      }
    }
    r->gangs.push_back(gg);
  }
  r->n_items[0] = (uint32_t)narrow.size();
  r->n_items[1] = (uint32_t)wide.size();
  r->items = narrow;
  r->items.insert(r->items.end(), wide.begin(), wide.end());
  int cus = 0, per_cu[2] = {0, 0};
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[0], ragged_kernel<false>, kRaggedBlock, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[1], ragged_kernel<true>, kRaggedBlock, 0);
  if (e != hipSuccess) {
    free_ragged(r);
    return hip_fail(e, "occupancy query");
  }
  for (int w = 0; w < 2; ++w)
    r->grid[w] = std::max(1u, std::min<uint32_t>(r->n_items[w], (uint32_t)(cus * std::max(1, per_cu[w]))));
  e = hipMalloc(&r->d_jobs, sizeof(RaggedJobDev) * r->jobs.size());
  if (e == hipSuccess) e = hipMalloc(&r->d_items, sizeof(RaggedItem) * std::max<size_t>(1, r->items.size()));
  if (e == hipSuccess) e = hipMalloc(&r->d_counter, sizeof(uint32_t) * 2);
  if (e == hipSuccess)
    e = hipMemcpy(r->d_jobs, r->jobs.data(), sizeof(RaggedJobDev) * r->jobs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !r->items.empty())
    e = hipMemcpy(r->d_items, r->items.data(), sizeof(RaggedItem) * r->items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !table.empty()) {
    e = hipMalloc(&r->d_rows, sizeof(RowRef) * table.size());
    if (e == hipSuccess)
      e = hipMemcpy(r->d_rows, table.data(), sizeof(RowRef) * table.size(), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    free_ragged(r);
    return hip_fail(e, "ragged descriptors");
  }
  *out = r;
  return NTT_OK;
}

ntt_status ntt_ragged_run(ntt_ragged_t r, void* stream) {
  if (!r) return fail(NTT_EINVAL, "null ragged batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(r->mu);
  if (!r->use_graph) {
    hipError_t e = launch_all(r, s, true);
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ragged launch");
  }
  if (!r->exec) {
    // Capture the counter reset and the persistent launch(es) once.
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    // one capture branch per group of large transforms (at most 8)
    std::vector<hipStream_t> branches(std::min<size_t>(8, r->gangs.size()), nullptr);
    for (auto& b : branches)
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = launch_all(r, cap, false, &branches);
      e = hipStreamEndCapture(cap, &r->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
    for (hipStream_t b : branches)
      if (b) (void)hipStreamDestroy(b);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "ragged graph capture");
  }
  hipError_t e = hipGraphLaunch(r->exec, s);
  return e == hipSuccess ? NTT_OK : hip_fail(e, "hipGraphLaunch");
}

ntt_status ntt_ragged_info(ntt_ragged_t r, uint32_t* items, uint32_t* workgroups) {
  if (!r) return fail(NTT_EINVAL, "null ragged batch");
  uint32_t rows = 0;
  for (const auto& gg : r->gangs) rows += gg.n;  // limb-rows (products count once)
  if (items) *items = r->n_items[0] + r->n_items[1] + rows;
  if (workgroups) *workgroups = (r->n_items[0] ? r->grid[0] : 0) + (r->n_items[1] ? r->grid[1] : 0);
  return NTT_OK;
}

ntt_status ntt_ragged_destroy(ntt_ragged_t r) {
  if (!r) return fail(NTT_EINVAL, "null ragged batch");
  free_ragged(r);
  return NTT_OK;
}

ntt_status ntt_batch_ragged(const ntt_job* jobs, uint32_t n, void* stream) {
  ntt_ragged_t r = nullptr;
  ntt_status st = ntt_ragged_create(&r, jobs, n, NTT_RAGGED_NO_GRAPH);
  if (st != NTT_OK) return st;
  st = ntt_ragged_run(r, stream);
  // The descriptors must outlive the launch: wait for it before freeing them.
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  free_ragged(r);
  if (st != NTT_OK) return st;
  return e == hipSuccess ? NTT_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // extern "C"
