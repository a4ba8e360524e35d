// twiddles.cpp -- device-resident twiddle tables, one per (device, prime, class),
// shared by every plan that uses the prime.
//
// With psi_N = g^((q-1)/2N) (g the smallest non-residue) we have
// psi_N = psi_2N^2, and the bit-reversed table of length N,
// T_N[k] = psi_N^brv_n(k), is exactly the first N entries of T_2N.  So one table
// built for the largest length the prime admits (up to 2^16) serves every N:
// a plan for N reads the prefix k < N.  Twiddles are precomputed per modulus
// as the paper keeps them resident in constant memory (Sec. II-E); here they
// live in HBM and are read through L2.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ntt_internal.hpp"
#include "numtheory.hpp"

namespace nttk {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, uint64_t, uint32_t>, PrimeTable*> g_tables;

double centred(uint64_t w, uint64_t q) { return w > q / 2 ? -(double)(q - w) : (double)w; }
}  // namespace

uint32_t table_log_len(uint64_t q) {
  const int v = two_adic(q - 1);  // q - 1 = 2^v * odd; 2N | q - 1 => N <= 2^(v-1)
  return (uint32_t)std::min(16, v - 1);
}

ntt_status acquire_table(int device, uint64_t q, uint32_t cls, const PrimeTable** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_tuple(device, q, cls);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    it->second->refs += 1;
    *out = it->second;
    return NTT_OK;
  }
  const uint32_t lt = table_log_len(q);
  const uint32_t n = 1u << lt;
  const uint64_t g = nt_smallest_nonresidue(q);
  const uint64_t psi = nt_pow(g, (q - 1) / (2ull * n), q);
  const uint64_t psi_inv = nt_pow(psi, q - 2, q);
  std::vector<uint64_t> pw(n), pwi(n);
  pw[0] = pwi[0] = 1;
  for (uint32_t k = 1; k < n; ++k) {
    pw[k] = nt_mul(pw[k - 1], psi, q);
    pwi[k] = nt_mul(pwi[k - 1], psi_inv, q);
  }
  const size_t entry = cls == 2 ? sizeof(TwI64) : sizeof(double);
  const size_t bytes = entry * (size_t)n * 2;
  std::vector<unsigned char> host(bytes);
  if (cls == 2) {
    TwI64* f = reinterpret_cast<TwI64*>(host.data());
    TwI64* iv = f + n;
    for (uint32_t k = 0; k < n; ++k) {
      const uint64_t w = pw[brv(k, (int)lt)], wi = pwi[brv(k, (int)lt)];
      f[k] = TwI64{w, (uint64_t)(((u128)w << 64) / q)};
      iv[k] = TwI64{wi, (uint64_t)(((u128)wi << 64) / q)};
    }
  } else {
    double* f = reinterpret_cast<double*>(host.data());
    double* iv = f + n;
    for (uint32_t k = 0; k < n; ++k) {
      f[k] = centred(pw[brv(k, (int)lt)], q);
      iv[k] = centred(pwi[brv(k, (int)lt)], q);
    }
  }
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(twiddle table)");
  e = hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(e, "hipMemcpy(twiddle table)");
  }
  PrimeTable* t = new PrimeTable();
  t->device = device;
  t->q = q;
  t->cls = cls;
  t->log_len = lt;
  t->mem = mem;
  t->twf = mem;
  t->twi = static_cast<unsigned char*>(mem) + entry * n;
  t->refs = 1;
  t->bytes = bytes;
  g_tables[key] = t;
  *out = t;
  return NTT_OK;
}

void release_table(const PrimeTable* t) {
  if (!t) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tables.find(std::make_tuple(t->device, t->q, t->cls));
  if (it == g_tables.end()) return;
  PrimeTable* p = it->second;
  if (--p->refs == 0) {
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipFree(p->mem);
    if (have && cur != p->device) (void)hipSetDevice(cur);
    g_tables.erase(it);
    delete p;
  }
}

size_t resident_table_bytes() {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t b = 0;
  for (const auto& kv : g_tables) b += kv.second->bytes;
  return b;
}

}  // namespace nttk
