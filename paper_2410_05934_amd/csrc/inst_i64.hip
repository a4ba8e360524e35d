// inst_i64.hip -- kernels and launchers of the ArI64 arithmetic class.
#include "ntt_launch.hpp"

namespace nttk {
template hipError_t transform_cls<ArI64>(const ntt_plan_s*, int, void*, uint32_t, bool,
                                        uint32_t, uint32_t*, hipStream_t);
template hipError_t pointwise_cls<ArI64>(const ntt_plan_s*, int, void*, const void*, const void*,
                                         uint32_t, hipStream_t);
template hipError_t polymul_cls<ArI64>(const ntt_plan_s*, int, void*, const void*, const void*,
                                       void*, uint32_t, uint32_t, hipStream_t);
template hipError_t mac_cls<ArI64>(const ntt_plan_s*, int, void*, const void*, const void*,
                                   uint32_t, uint32_t, uint32_t, hipStream_t);
template hipError_t xprod_cls<ArI64>(const ntt_plan_s*, int, void*, const void*, const void*,
                                    uint32_t, uint32_t, uint32_t, hipStream_t, uint32_t,
                                    uint32_t, uint32_t, const uint32_t*);
template hipError_t polymul_rows_cls<ArI64>(const ntt_plan_s*, int, const uint64_t*,
                                              const uint64_t*, const uint64_t*, void*, void*,
                                              uint32_t, uint32_t, hipStream_t);
template hipError_t fwdmul_cls<ArI64>(const ntt_plan_s*, int, void*, void*, void*, uint32_t,
                                      uint32_t, hipStream_t);
}  // namespace nttk
