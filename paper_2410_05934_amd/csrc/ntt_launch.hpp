// ntt_launch.hpp -- host launchers for the kernels of one arithmetic class.
// Included by one translation unit per class (inst_*.hip), which instantiates
// them explicitly, so the three classes compile in parallel.
#pragma once

#include <algorithm>

#include "fused.hpp"
#include "ntt_internal.hpp"
#include "ntt_kernels.hpp"
#include "xprod.hpp"

namespace nttk {

// ---------------------------------------------------------------------------
// Launchers

template <class A, int LOGN2, bool INV, bool TWO, int RB = 4>
hipError_t launch_row_n(const RowArgs& a, hipStream_t s) {
  using S = RowShape<LOGN2, RB>;
  const uint32_t blocks = (a.total_chunks + S::CPW - 1) / S::CPW;
  LaunchTimer t(RB == 4 ? "row" : RB == 3 ? "row8" : "row4", A::kName, LOGN2, INV, TWO,
                (uint64_t)a.total_chunks << LOGN2, s);
  hipLaunchKernelGGL((row_kernel<A, LOGN2, INV, TWO, RB>), dim3(blocks), dim3(S::BLOCK), 0, s, a);
  return hipGetLastError();
}

template <class A, int LOGN2, bool TWO, int RB = 4>
hipError_t launch_pm_n(const RowArgs& a, hipStream_t s) {
  using S = RowShape<LOGN2, RB>;
  const uint32_t blocks = (a.total_chunks + S::CPW - 1) / S::CPW;
  LaunchTimer t(RB == 4 ? "polymul_row" : "polymul_row8", A::kName, LOGN2, false, TWO,
                (uint64_t)a.total_chunks << LOGN2, s);
  hipLaunchKernelGGL((polymul_row_kernel<A, LOGN2, TWO, RB>), dim3(blocks), dim3(S::BLOCK), 0, s, a);
  return hipGetLastError();
}

template <class A, int LOGN2, bool TWO, int RB = 4>
hipError_t launch_fm_n(const RowArgs& a, hipStream_t s) {
  using S = RowShape<LOGN2, RB>;
  const uint32_t blocks = (a.total_chunks + S::CPW - 1) / S::CPW;
  LaunchTimer t(RB == 4 ? "fwdmul_row" : "fwdmul_row8", A::kName, LOGN2, false, TWO,
                (uint64_t)a.total_chunks << LOGN2, s);
  hipLaunchKernelGGL((polymul_row_kernel<A, LOGN2, TWO, RB, true>), dim3(blocks), dim3(S::BLOCK), 0,
                     s, a);
  return hipGetLastError();
}

template <class A, int LOGN1, bool INV, bool TWO>
hipError_t launch_col_n(const ColArgs& a, hipStream_t s) {
  const uint64_t threads = (uint64_t)a.total_cols * ((a.src2 || a.src2_rows) ? 2 : 1);
  const uint32_t bs = (a.block == 64 || a.block == 128) ? a.block : (uint32_t)kColBlock;
  const uint32_t blocks = (uint32_t)((threads + bs - 1) / bs);
  LaunchTimer t("col", A::kName, LOGN1, INV, TWO, threads << LOGN1, s);
  if constexpr (TWO) {
    // row tables: built for the two-pass column launches only
    if (a.src_rows || a.src2_rows || a.dst_rows) {
      if (a.n_cls == 1)
        hipLaunchKernelGGL((col_kernel<A, LOGN1, INV, TWO, true, true>), dim3(blocks), dim3(bs), 0, s, a);
      else
        hipLaunchKernelGGL((col_kernel<A, LOGN1, INV, TWO, false, true>), dim3(blocks), dim3(bs), 0, s, a);
      return hipGetLastError();
    }
  } else {
    if (a.src_rows || a.src2_rows || a.dst_rows) return hipErrorInvalidValue;
  }
  if (a.n_cls == 1)
    hipLaunchKernelGGL((col_kernel<A, LOGN1, INV, TWO, true>), dim3(blocks), dim3(bs), 0, s, a);
  else
    hipLaunchKernelGGL((col_kernel<A, LOGN1, INV, TWO>), dim3(blocks), dim3(bs), 0, s, a);
  return hipGetLastError();
}

template <class A, bool INV, bool TWO>
hipError_t launch_row(int logn2, const RowArgs& a, hipStream_t s, int rb = 4) {
  if (rb == 2) {
    switch (logn2) {
      case 8: return launch_row_n<A, 8, INV, TWO, 2>(a, s);
      case 9: return launch_row_n<A, 9, INV, TWO, 2>(a, s);
      case 10: return launch_row_n<A, 10, INV, TWO, 2>(a, s);
      case 11: return launch_row_n<A, 11, INV, TWO, 2>(a, s);
      case 12: return launch_row_n<A, 12, INV, TWO, 2>(a, s);
      default: break;
    }
  }
  if (rb == 3) {
    switch (logn2) {
      case 10: return launch_row_n<A, 10, INV, TWO, 3>(a, s);
      case 11: return launch_row_n<A, 11, INV, TWO, 3>(a, s);
      case 12: return launch_row_n<A, 12, INV, TWO, 3>(a, s);
      case 13: return launch_row_n<A, 13, INV, TWO, 3>(a, s);
      default: break;
    }
  }
  switch (logn2) {
    case 4: return launch_row_n<A, 4, INV, TWO>(a, s);
    case 5: return launch_row_n<A, 5, INV, TWO>(a, s);
    case 6: return launch_row_n<A, 6, INV, TWO>(a, s);
    case 7: return launch_row_n<A, 7, INV, TWO>(a, s);
    case 8: return launch_row_n<A, 8, INV, TWO>(a, s);
    case 9: return launch_row_n<A, 9, INV, TWO>(a, s);
    case 10: return launch_row_n<A, 10, INV, TWO>(a, s);
    case 11: return launch_row_n<A, 11, INV, TWO>(a, s);
    case 12: return launch_row_n<A, 12, INV, TWO>(a, s);
    case 13: return launch_row_n<A, 13, INV, TWO>(a, s);
    case 14: return launch_row_n<A, 14, INV, TWO>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <class A, bool TWO>
hipError_t launch_pm(int logn2, const RowArgs& a, hipStream_t s, int rb = 4) {
  if (rb == 3) {
    switch (logn2) {
      case 10: return launch_pm_n<A, 10, TWO, 3>(a, s);
      case 11: return launch_pm_n<A, 11, TWO, 3>(a, s);
      case 12: return launch_pm_n<A, 12, TWO, 3>(a, s);
      case 13: return launch_pm_n<A, 13, TWO, 3>(a, s);
      default: break;
    }
  }
  switch (logn2) {
    case 4: return launch_pm_n<A, 4, TWO>(a, s);
    case 5: return launch_pm_n<A, 5, TWO>(a, s);
    case 6: return launch_pm_n<A, 6, TWO>(a, s);
    case 7: return launch_pm_n<A, 7, TWO>(a, s);
    case 8: return launch_pm_n<A, 8, TWO>(a, s);
    case 9: return launch_pm_n<A, 9, TWO>(a, s);
    case 10: return launch_pm_n<A, 10, TWO>(a, s);
    case 11: return launch_pm_n<A, 11, TWO>(a, s);
    case 12: return launch_pm_n<A, 12, TWO>(a, s);
    case 13: return launch_pm_n<A, 13, TWO>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <class A, bool INV, bool TWO>
hipError_t launch_col(int logn1, const ColArgs& a, hipStream_t s) {
  switch (logn1) {
    case 1: return launch_col_n<A, 1, INV, TWO>(a, s);
    case 2: return launch_col_n<A, 2, INV, TWO>(a, s);
    case 3: return launch_col_n<A, 3, INV, TWO>(a, s);
    case 4: return launch_col_n<A, 4, INV, TWO>(a, s);
    case 5: return launch_col_n<A, 5, INV, TWO>(a, s);
    default: return hipErrorInvalidValue;
  }
}

inline RowArgs row_args(const ntt_plan_s* p, int c, void* dst, const void* src, const void* src2,
                        uint32_t batch, int n1 = -1) {
  if (n1 < 0) n1 = (int)p->log_n1;
  RowArgs a;
  a.dst = dst;
  a.src = src;
  a.src2 = src2;
  a.limbs = p->d_limbs;
  a.cls_limbs = p->d_cls_limbs + p->cls_off[c];
  a.n_cls = p->cls_cnt[c];
  a.L = p->L;
  a.log_n = p->log_n;
  a.log_n1 = (uint32_t)n1;
  a.total_chunks = batch * p->cls_cnt[c] << n1;
  a.batch = batch;
  a.dst2 = nullptr;
  a.limb0 = p->cls_cnt[c] == 1 ? p->h_cls_limbs[p->cls_off[c]] : 0u;
  a.one = p->h_limbs[a.limb0];
  return a;
}

inline ColArgs col_args(const ntt_plan_s* p, int c, void* dst, const void* src, uint32_t batch,
                        int n1 = -1) {
  if (n1 < 0) n1 = (int)p->log_n1;
  ColArgs a;
  a.dst = dst;
  a.src = src;
  a.limbs = p->d_limbs;
  a.cls_limbs = p->d_cls_limbs + p->cls_off[c];
  a.n_cls = p->cls_cnt[c];
  a.L = p->L;
  a.log_n = p->log_n;
  a.log_n2 = p->log_n - (uint32_t)n1;
  a.total_cols = (batch * p->cls_cnt[c]) << a.log_n2;
  a.dst2 = nullptr;
  a.src2 = nullptr;
  a.limb0 = p->cls_cnt[c] == 1 ? p->h_cls_limbs[p->cls_off[c]] : 0u;
  a.one = p->h_limbs[a.limb0];
  a.block = col_block_for(p, batch);
  a.src_rows = a.src2_rows = a.dst_rows = nullptr;
  return a;
}

// Single-launch two-pass transform (row length 2^12): persistent grid of the
// workgroups resident at once, list lag from the grid.
template <class A, int LOGN1, bool INV, int RB>
hipError_t launch_fused_n(FusedArgs a, int device, hipStream_t s) {
  using S = RowShape<12, RB>;
  // resident workgroups per CU (one gfx950 build: the same on every device)
  static const int per_cu = []() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_kernel<A, LOGN1, 12, INV, RB>,
                                                     S::BLOCK, 0) != hipSuccess || nb < 1)
      nb = 1;
    return nb;
  }();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus < 1)
    cus = 1;
  // forward: columns first (pieces of BLOCK columns), then rows; inverse: rows
  // first, then columns
  const uint32_t col_pieces = (1u << 12) / S::BLOCK, row_pieces = 1u << LOGN1;
  a.p1 = INV ? row_pieces : col_pieces;
  a.p2 = INV ? col_pieces : row_pieces;
  a.total = a.n_tr * (a.p1 + a.p2);
  const uint32_t grid = std::min<uint32_t>(a.total, (uint32_t)(cus * per_cu));
  const uint32_t want = (3 * grid + 2 * (a.p1 + a.p2) - 1) / (2 * (a.p1 + a.p2));
  a.lag = std::max<uint32_t>(1u, std::min<uint32_t>(a.n_tr, want));
  LaunchTimer t(RB == 4 ? "fused" : "fused8", A::kName, LOGN1 + 12, INV, true,
                (uint64_t)a.n_tr << (LOGN1 + 12), s);
  hipLaunchKernelGGL((fused_kernel<A, LOGN1, 12, INV, RB>), dim3(grid), dim3(S::BLOCK), 0, s, a);
  return hipGetLastError();
}

template <class A, bool TWO>
hipError_t launch_fm(int logn2, const RowArgs& a, hipStream_t s, int rb = 4) {
  if (rb == 3) {
    switch (logn2) {
      case 10: return launch_fm_n<A, 10, TWO, 3>(a, s);
      case 11: return launch_fm_n<A, 11, TWO, 3>(a, s);
      case 12: return launch_fm_n<A, 12, TWO, 3>(a, s);
      case 13: return launch_fm_n<A, 13, TWO, 3>(a, s);
      default: break;
    }
  }
  switch (logn2) {
    case 4: return launch_fm_n<A, 4, TWO>(a, s);
    case 5: return launch_fm_n<A, 5, TWO>(a, s);
    case 6: return launch_fm_n<A, 6, TWO>(a, s);
    case 7: return launch_fm_n<A, 7, TWO>(a, s);
    case 8: return launch_fm_n<A, 8, TWO>(a, s);
    case 9: return launch_fm_n<A, 9, TWO>(a, s);
    case 10: return launch_fm_n<A, 10, TWO>(a, s);
    case 11: return launch_fm_n<A, 11, TWO>(a, s);
    case 12: return launch_fm_n<A, 12, TWO>(a, s);
    case 13: return launch_fm_n<A, 13, TWO>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <class A, bool INV>
hipError_t launch_fused(int n1, const FusedArgs& a, int device, hipStream_t s, int rb) {
  if (rb == 3) {
    switch (n1) {
      case 1: return launch_fused_n<A, 1, INV, 3>(a, device, s);
      case 2: return launch_fused_n<A, 2, INV, 3>(a, device, s);
      case 3: return launch_fused_n<A, 3, INV, 3>(a, device, s);
      case 4: return launch_fused_n<A, 4, INV, 3>(a, device, s);
      default: break;
    }
  } else {
    switch (n1) {
      case 1: return launch_fused_n<A, 1, INV, 4>(a, device, s);
      case 2: return launch_fused_n<A, 2, INV, 4>(a, device, s);
      case 3: return launch_fused_n<A, 3, INV, 4>(a, device, s);
      case 4: return launch_fused_n<A, 4, INV, 4>(a, device, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// `work` (nullptr: two launches) holds the counters of the single-launch form
// for every class of the plan: class c uses 1 + batch * cls_cnt[c] words at
// offset batch * cls_off[c] + c; the word after all of them is the expiry flag.
template <class A>
hipError_t transform_cls(const ntt_plan_s* p, int c, void* data, uint32_t batch, bool inv,
                         uint32_t split, uint32_t* work, hipStream_t s) {
  const int n = p->log_n, n1 = (int)split, n2 = n - n1;
  const int rb = row_rb_for(p, inv, split, batch);
  hipError_t e = hipSuccess;
  if (work && fused_shape_ok(p, split)) {
    FusedArgs fa;
    fa.data = data;
    fa.limbs = p->d_limbs;
    fa.cls_limbs = p->d_cls_limbs + p->cls_off[c];
    fa.L = p->L;
    fa.batch = batch;
    fa.log_n = p->log_n;
    fa.n_tr = batch * p->cls_cnt[c];
    fa.spin_limit = fused_spin_limit();
    fa.target_extra = fused_force_expire() ? 1u : 0u;
    fa.work = work + (size_t)batch * p->cls_off[c] + c;
    fa.expired = work + (size_t)batch * p->L + 3;
    return inv ? launch_fused<A, true>(n1, fa, p->device, s, rb)
               : launch_fused<A, false>(n1, fa, p->device, s, rb);
  }
  if (n1 == 0) {
    RowArgs a = row_args(p, c, data, data, nullptr, batch, n1);
    e = inv ? launch_row<A, true, false>(n2, a, s, rb) : launch_row<A, false, false>(n2, a, s, rb);
  } else if (n2 == 0) {
    ColArgs a = col_args(p, c, data, data, batch, n1);
    e = inv ? launch_col<A, true, false>(n1, a, s) : launch_col<A, false, false>(n1, a, s);
  } else if (!inv) {
    ColArgs ca = col_args(p, c, data, data, batch, n1);
    e = launch_col<A, false, true>(n1, ca, s);
    if (e == hipSuccess) {
      RowArgs ra = row_args(p, c, data, data, nullptr, batch, n1);
      e = launch_row<A, false, true>(n2, ra, s, rb);
    }
  } else {
    RowArgs ra = row_args(p, c, data, data, nullptr, batch, n1);
    e = launch_row<A, true, true>(n2, ra, s, rb);
    if (e == hipSuccess) {
      ColArgs ca = col_args(p, c, data, data, batch, n1);
      e = launch_col<A, true, true>(n1, ca, s);
    }
  }
  return e;
}

template <class A>
hipError_t pointwise_cls(const ntt_plan_s* p, int c, void* out, const void* a,
                                const void* b, uint32_t batch, hipStream_t s) {
  EltArgs ea;
  ea.dst = out;
  ea.a = a;
  ea.b = b;
  ea.limbs = p->d_limbs;
  ea.cls_limbs = p->d_cls_limbs + p->cls_off[c];
  ea.n_cls = p->cls_cnt[c];
  ea.L = p->L;
  ea.log_n = p->log_n;
  ea.total = ((uint64_t)batch * p->cls_cnt[c]) << p->log_n;  // < 2^32 (checked by the caller)
  constexpr int kVec = 16 / (int)sizeof(typename A::W);
  auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  const bool vec = (1u << p->log_n) >= (uint32_t)kVec && aligned(out) && aligned(a) && aligned(b);
  const int per = vec ? kVec : 1;
  const uint32_t blocks = (uint32_t)((ea.total / per + kEltBlock - 1) / kEltBlock);
  LaunchTimer t("pointwise", A::kName, p->log_n, false, false, ea.total, s);
  if (vec) hipLaunchKernelGGL((pointwise_kernel<A, kVec>), dim3(blocks), dim3(kEltBlock), 0, s, ea);
  else hipLaunchKernelGGL((pointwise_kernel<A, 1>), dim3(blocks), dim3(kEltBlock), 0, s, ea);
  return hipGetLastError();
}

template <class A>
hipError_t polymul_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* b,
                       void* ws, uint32_t batch, uint32_t split, hipStream_t s) {
  const int n = p->log_n, n1 = (int)split, n2 = n - n1;
  const int rb = polymul_rb_for(p, split, batch);
  hipError_t e;
  if (n1 == 0) {
    RowArgs ra = row_args(p, c, out, a, b, batch, n1);
    return launch_pm<A, false>(n2, ra, s, rb);
  }
  if (n2 == 0) {
    // Tiny N: forward both into out / ws, multiply, inverse.
    ColArgs ca = col_args(p, c, out, a, batch, n1);
    if ((e = launch_col<A, false, false>(n1, ca, s)) != hipSuccess) return e;
    ca = col_args(p, c, ws, b, batch, n1);
    if ((e = launch_col<A, false, false>(n1, ca, s)) != hipSuccess) return e;
    if ((e = pointwise_cls<A>(p, c, out, out, ws, batch, s)) != hipSuccess) return e;
    ca = col_args(p, c, out, out, batch, n1);
    return launch_col<A, true, false>(n1, ca, s);
  }
  // Column passes of a (into out) and b (into ws) in one launch.
  ColArgs ca = col_args(p, c, out, a, batch, n1);
  ca.dst2 = ws;
  ca.src2 = b;
  if ((e = launch_col<A, false, true>(n1, ca, s)) != hipSuccess) return e;
  RowArgs ra = row_args(p, c, out, out, ws, batch, n1);
  if ((e = launch_pm<A, true>(n2, ra, s, rb)) != hipSuccess) return e;
  ca = col_args(p, c, out, out, batch, n1);
  return launch_col<A, true, true>(n1, ca, s);
}

// Two-pass polymul whose operands and results live in separate buffers: limb-row
// poly * L + limb of a, b and out is at a_rows / b_rows / out_rows[that row]
// (byte addresses).  The first column launch reads a and b through the tables
// (into o and ws), the last one writes out through its table; o and ws are
// contiguous [batch][L][N] scratch.  The caller checks polymul_rows_ok.
template <class A>
hipError_t polymul_rows_cls(const ntt_plan_s* p, int c, const uint64_t* out_rows,
                            const uint64_t* a_rows, const uint64_t* b_rows, void* o, void* ws,
                            uint32_t batch, uint32_t split, hipStream_t s) {
  const int n = p->log_n, n1 = (int)split, n2 = n - n1;
  if (n1 == 0 || n2 == 0) return hipErrorInvalidValue;
  const int rb = polymul_rb_for(p, split, batch);
  hipError_t e;
  ColArgs ca = col_args(p, c, o, nullptr, batch, n1);
  ca.src_rows = a_rows;
  ca.dst2 = ws;
  ca.src2_rows = b_rows;
  if ((e = launch_col<A, false, true>(n1, ca, s)) != hipSuccess) return e;
  RowArgs ra = row_args(p, c, o, o, ws, batch, n1);
  if ((e = launch_pm<A, true>(n2, ra, s, rb)) != hipSuccess) return e;
  ca = col_args(p, c, nullptr, o, batch, n1);
  ca.dst_rows = out_rows;
  return launch_col<A, true, true>(n1, ca, s);
}

// Forward transforms of a and b in place and out = a (.) b, with polymul's
// split (n1 >= 1 or a row part of at most 2^13 words) and row radix.
template <class A>
hipError_t fwdmul_cls(const ntt_plan_s* p, int c, void* out, void* a, void* b, uint32_t batch,
                      uint32_t split, hipStream_t s) {
  const int n = p->log_n, n1 = (int)split, n2 = n - n1;
  const int rb = polymul_rb_for(p, split, batch);
  hipError_t e;
  if (n2 == 0 || n2 > 13) {
    // no paired rows for this split: two transforms and the product
    if ((e = transform_cls<A>(p, c, a, batch, false, split, nullptr, s)) != hipSuccess) return e;
    if ((e = transform_cls<A>(p, c, b, batch, false, split, nullptr, s)) != hipSuccess) return e;
    return pointwise_cls<A>(p, c, out, a, b, batch, s);
  }
  RowArgs ra = row_args(p, c, a, a, b, batch, n1);
  ra.dst2 = out;
  if (n1 == 0) return launch_fm<A, false>(n2, ra, s, rb);
  ColArgs ca = col_args(p, c, a, a, batch, n1);
  ca.dst2 = b;
  ca.src2 = b;
  if ((e = launch_col<A, false, true>(n1, ca, s)) != hipSuccess) return e;
  return launch_fm<A, true>(n2, ra, s, rb);
}

template <class A>
hipError_t mac_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* key,
                          uint32_t rows, uint32_t cols, uint32_t num_operands, hipStream_t s) {
  MacArgs m;
  m.dst = out;
  m.a = a;
  m.key = key;
  m.limbs = p->d_limbs;
  m.cls_limbs = p->d_cls_limbs + p->cls_off[c];
  m.n_cls = p->cls_cnt[c];
  m.L = p->L;
  m.log_n = p->log_n;
  m.rows = rows;
  m.cols = cols;
  m.num_operands = num_operands;
  m.groups = (num_operands + rows - 1) / rows;
  m.total = ((uint64_t)m.groups * cols * p->cls_cnt[c]) << p->log_n;  // < 2^32 (checked)
  constexpr int kVec = 16 / (int)sizeof(typename A::W);
  auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  const bool vec = (1u << p->log_n) >= (uint32_t)kVec && aligned(out) && aligned(a) && aligned(key);
  const int per = vec ? kVec : 1;
  const uint32_t blocks = (uint32_t)((m.total / per + kEltBlock - 1) / kEltBlock);
  LaunchTimer t("mac", A::kName, p->log_n, false, false, m.total, s);
  if (vec) hipLaunchKernelGGL((mac_kernel<A, kVec>), dim3(blocks), dim3(kEltBlock), 0, s, m);
  else hipLaunchKernelGGL((mac_kernel<A, 1>), dim3(blocks), dim3(kEltBlock), 0, s, m);
  return hipGetLastError();
}

template <class A, int LOGN2>
hipError_t launch_xprod_n(const XpArgs& x, uint32_t groups, hipStream_t s) {
  // Radix-8 slots (twice the threads, half the butterflies per thread) when the
  // workgroup still fits 1024 threads: the launch is latency-bound, one
  // workgroup per (group, limb), so a shorter chain per thread is what counts.
  constexpr uint32_t kN = 1u << LOGN2;
  const bool r8 = LOGN2 >= 10 && x.rows * (kN / 8) <= 1024;
  const uint32_t threads = x.rows * (kN >> (r8 ? 3 : 4));
  const size_t lds = (size_t)x.rows * (kN + kN / 16) * sizeof(typename A::V);
  LaunchTimer t(x.rot ? "cmux" : x.levels ? "xprod_dec" : "xprod", A::kName, LOGN2, false, false,
                ((uint64_t)groups * x.cols * x.n_cls) << LOGN2, s);
  const dim3 grid(groups * x.n_cls), block(threads);
  if constexpr (LOGN2 >= 10) {
    if (r8) {
      if (x.rot)
        hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpCmux, 3>), grid, block, lds, s, x);
      else if (x.levels)
        hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpDecompose, 3>), grid, block, lds, s, x);
      else
        hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpOperands, 3>), grid, block, lds, s, x);
      return hipGetLastError();
    }
  }
  if (x.rot)
    hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpCmux>), grid, block, lds, s, x);
  else if (x.levels)
    hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpDecompose>), grid, block, lds, s, x);
  else
    hipLaunchKernelGGL((xprod_kernel<A, LOGN2, kXpOperands>), grid, block, lds, s, x);
  return hipGetLastError();
}

// comps / levels / log_base: the operands are the digits of ciphertexts in `a`
// (levels = 0: the operands themselves are in `a`).
template <class A>
hipError_t xprod_cls(const ntt_plan_s* p, int c, void* out, const void* a, const void* key,
                     uint32_t rows, uint32_t cols, uint32_t num_operands, hipStream_t s,
                     uint32_t comps = 0, uint32_t levels = 0, uint32_t log_base = 0,
                     const uint32_t* rot = nullptr) {
  XpArgs x;
  x.rot = rot;
  x.comps = comps;
  x.levels = levels;
  x.log_base = log_base;
  x.dec_offset = levels ? digit_offset(levels, log_base) : 0;
  x.dst = out;
  x.a = a;
  x.key = key;
  x.limbs = p->d_limbs;
  x.cls_limbs = p->d_cls_limbs + p->cls_off[c];
  x.n_cls = p->cls_cnt[c];
  x.L = p->L;
  x.rows = rows;
  x.cols = cols;
  x.num_operands = num_operands;
  const uint32_t groups = (num_operands + rows - 1) / rows;
  switch (p->log_n) {
    case 4: return launch_xprod_n<A, 4>(x, groups, s);
    case 5: return launch_xprod_n<A, 5>(x, groups, s);
    case 6: return launch_xprod_n<A, 6>(x, groups, s);
    case 7: return launch_xprod_n<A, 7>(x, groups, s);
    case 8: return launch_xprod_n<A, 8>(x, groups, s);
    case 9: return launch_xprod_n<A, 9>(x, groups, s);
    case 10: return launch_xprod_n<A, 10>(x, groups, s);
    case 11: return launch_xprod_n<A, 11>(x, groups, s);
    case 12: return launch_xprod_n<A, 12>(x, groups, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nttk
