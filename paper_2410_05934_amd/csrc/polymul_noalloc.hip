// polymul_noalloc.hip -- the negacyclic product (Eq. (1)) for callers that
// cannot allocate device memory: code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc.
//
// A two-pass product needs a workspace of batch * L * N words (the column pass
// of b lands there, since b is read-only).  ntt_polymul takes it from the
// stream-ordered pool on every call; this entry point takes it from `scratch`,
// a file-scope device array of kScratchBytes that every GPU the library runs on
// holds until the process ends.  Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that address
// is ever handed to kernels: in host code the array's name is a host-side
// stand-in, not a device pointer.  The workspace is written in full by the
// column pass before the row pass reads it, so nothing needs clearing.  All
// calls on one GPU share the array: two calls that overlap in time on one GPU
// (different streams, or host threads without ordering) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ntt_internal.hpp"

static constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call on that device.
ntt_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nttk::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return nttk::fail(NTT_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return nttk::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return nttk::fail(NTT_EDEVICE, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NTT_OK;
}

}  // namespace

using namespace nttk;

extern "C" {

ntt_status ntt_polymul_noalloc(ntt_plan_t plan, void* out, const void* a, const void* b,
                               uint32_t batch, void* stream) {
  clear_error();
  if (!plan) return fail(NTT_EINVAL, "null plan");
  if (batch == 0) return fail(NTT_EINVAL, "batch must be >= 1");
  if (((uint64_t)batch * plan->L << plan->log_n) >= (1ull << 32))
    return fail(NTT_EINVAL, "batch * L * N must be < 2^32 words");
  if (!out || !a || !b) return fail(NTT_EINVAL, "null data");
  if (out == a || out == b) return fail(NTT_EINVAL, "out must not alias a or b");
  if (plan->flags & NTT_FLAG_VALIDATE)
    return fail(NTT_EINVAL, "plans with NTT_FLAG_VALIDATE allocate and wait for the range check; "
                            "use ntt_polymul");
  const size_t bytes = polymul_ws_bytes(plan, batch);
  if (bytes > kScratchBytes)
    return fail(NTT_EINVAL, "workspace of %zu bytes exceeds the %zu-byte scratch (batch * L * N * word "
                            "bytes for two-pass products)", bytes, kScratchBytes);
  void* ws = nullptr;
  if (bytes) {
    const ntt_status st = scratch_on_current_device(&ws);
    if (st != NTT_OK) return st;
  }
  return polymul_into(plan, out, a, b, batch, ws, static_cast<hipStream_t>(stream));
}

}  // extern "C"
