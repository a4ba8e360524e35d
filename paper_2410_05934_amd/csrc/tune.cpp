// tune.cpp -- the autotuner and its tuning table.
//
// The paper chooses the switching point between its two phases so that the
// number of independent chunks is closest to the SM count (Sec. V-D, the
// (I1, I2) sweep of Sec. VI-D).  That rule is for one polynomial.  Here a call
// transforms batch * L limb-rows at once, so the concurrency is
// batch * L * N1 chunks and the best split moves with the batch.  The tuner
// therefore measures: for a shape it times every admissible split on scratch
// data and records the fastest under the key (log2 N, arithmetic class,
// floor(log2(batch * L))).  With each split it also times the row-pass radices
// (16, 8 or 4 values per thread: the threads per chunk, the paper's threads per
// block) per direction and records the fastest; at the chosen split and radices
// it times column passes of 256, 128 and 64 columns per workgroup (4, 2 or 1
// waves; one thread per column), then polymul rows of both radices.  Calls
// without a forced split look the keys up (the nearest recorded row bucket
// within two powers of two), else use the defaults.  The row pass's LDS padding
// is fixed (one spare slot per 16 words): its bank conflicts are measured at
// 0.04-0.12 per access, so there is nothing for a search to win.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ntt_internal.hpp"

namespace nttk {

namespace {

struct Entry {
  uint32_t value;
  float us;
};

// key: (kind, log_n, cls, bucket); kind 0 = pass split, 1 = ragged row length,
// 2 / 3 / 4 = values per thread (log2) of forward / inverse / polymul row passes,
// 5 = columns (threads) per workgroup of the column passes
using Key = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>;

std::mutex g_mu;
std::map<Key, Entry> g_table;
bool g_env_loaded = false;

uint32_t bucket_of(uint64_t rows) {
  uint32_t b = 0;
  while (b < 24 && (2ull << b) <= rows) ++b;
  return b;
}

ntt_status load_locked(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(NTT_EINVAL, "cannot open tuning file %s", path);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  const size_t ent = text.find("\"entries\"");
  if (ent == std::string::npos) return fail(NTT_EINVAL, "tuning file %s has no entries", path);
  size_t pos = ent;
  auto field = [](const std::string& obj, const char* key, double* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = obj.find(k);
    if (at == std::string::npos) return false;
    const size_t colon = obj.find(':', at + k.size());
    if (colon == std::string::npos) return false;
    *out = std::strtod(obj.c_str() + colon + 1, nullptr);
    return true;
  };
  while ((pos = text.find('{', pos + 1)) != std::string::npos) {
    const size_t end = text.find('}', pos);
    if (end == std::string::npos) break;
    const std::string obj = text.substr(pos, end - pos + 1);
    double kind, log_n, cls, bucket, value, us = 0;
    if (field(obj, "kind", &kind) && field(obj, "log_n", &log_n) && field(obj, "cls", &cls) &&
        field(obj, "bucket", &bucket) && field(obj, "value", &value)) {
      field(obj, "us", &us);
      g_table[Key((uint32_t)kind, (uint32_t)log_n, (uint32_t)cls, (uint32_t)bucket)] =
          Entry{(uint32_t)value, (float)us};
    }
    pos = end;
  }
  return NTT_OK;
}

void ensure_env_loaded() {
  if (g_env_loaded) return;
  g_env_loaded = true;
  const char* f = std::getenv("NTT_TUNE_FILE");
  if (f && *f) (void)load_locked(f);
}

uint32_t class_of(uint64_t q, uint32_t word_bits) {
  if (word_bits == 32) return 0;
  return q < kF64LBound ? 1u : 2u;
}

__global__ void fill_words(uint64_t* p, size_t n64) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n64) p[i] = 0;
}

}  // namespace

namespace {
// The entry of `kind` for (log_n, cls) recorded at the bucket of `rows`, else at
// the nearest bucket within two powers of two whose value `ok` accepts.
template <class Ok>
uint32_t lookup(uint32_t kind, uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback, Ok ok) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_env_loaded();
  const uint32_t b = bucket_of(rows);
  for (int d = 0; d <= 2; ++d) {
    for (int sgn : {1, -1}) {
      const int bb = (int)b + sgn * d;
      if (bb < 0) continue;
      auto it = g_table.find(Key(kind, log_n, cls, (uint32_t)bb));
      if (it != g_table.end() && ok(it->second.value)) return it->second.value;
      if (d == 0) break;
    }
  }
  return fallback;
}
}  // namespace

uint32_t tuned_split_for(uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback) {
  return lookup(0u, log_n, cls, rows, fallback,
                [&](uint32_t v) { return split_valid((int)log_n, (int)v); });
}

uint32_t tuned_row_rb(uint32_t kind, uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback) {
  return lookup(kind, log_n, cls, rows, fallback, [](uint32_t v) { return v >= 2 && v <= 4; });
}

uint32_t tuned_col_block(uint32_t log_n, uint32_t cls, uint64_t rows, uint32_t fallback) {
  return lookup(5u, log_n, cls, rows, fallback,
                [](uint32_t v) { return v == 64 || v == 128 || v == 256; });
}

uint32_t tuned_ragged_row_log(uint32_t log_n, uint32_t fallback) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_env_loaded();
  auto it = g_table.find(Key(1u, log_n, 0u, 0u));
  if (it != g_table.end() && (it->second.value == 11 || it->second.value == 12))
    return it->second.value;
  return fallback;
}

}  // namespace nttk

using namespace nttk;

extern "C" {

ntt_status ntt_tune_split(uint32_t N, const uint64_t* moduli, uint32_t num_moduli,
                          uint32_t word_bits, uint32_t batch, uint32_t* best_n1, float* best_us) {
  if (!moduli || num_moduli == 0 || batch == 0) return fail(NTT_EINVAL, "bad tuning shape");
  const uint64_t words = (uint64_t)batch * num_moduli * N;
  if (words >= (1ull << 32)) return fail(NTT_EINVAL, "tuning shape too large");
  int log_n = 0;
  while ((1u << log_n) < N) ++log_n;
  void* buf = nullptr;
  const size_t bytes = words * (word_bits / 8);
  hipError_t e = hipMalloc(&buf, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(tuning scratch)");
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return hip_fail(e, "hipStreamCreate");
  }
  const size_t n64 = (bytes + 7) / 8;
  hipLaunchKernelGGL(fill_words, dim3((unsigned)((n64 + 255) / 256)), dim3(256), 0, s,
                     static_cast<uint64_t*>(buf), n64);
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const int reps = (int)std::max<uint64_t>(8, std::min<uint64_t>(40, (1ull << 24) / std::max<uint64_t>(1, words)));
  // Time one direction of one (split, radix) configuration: the fastest of
  // three timed groups of `reps` calls (configurations a few percent apart
  // must not be ranked by one noisy sample).
  auto time_dir = [&](ntt_plan_t p, bool inv, float* us) -> ntt_status {
    for (int w = 0; w < 2; ++w) (inv ? ntt_inverse : ntt_forward)(p, buf, batch, s);
    float best_ms = 1e30f;
    for (int trial = 0; trial < 3; ++trial) {
      (void)hipEventRecord(a, s);
      for (int r = 0; r < reps; ++r) (inv ? ntt_inverse : ntt_forward)(p, buf, batch, s);
      (void)hipEventRecord(b, s);
      hipError_t he = hipEventSynchronize(b);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, a, b);
      if (he != hipSuccess) return hip_fail(he, "tuning run");
      best_ms = std::min(best_ms, ms);
    }
    *us = best_ms * 1000.f / reps;
    return NTT_OK;
  };
  float best = 1e30f;
  uint32_t best_split = 0, best_rb_f = 4, best_rb_i = 4;
  ntt_status st = NTT_OK;
  bool any = false;
  for (int n1 = 0; n1 <= log_n && st == NTT_OK; ++n1) {
    if (!split_valid(log_n, n1)) continue;
    const int n2 = log_n - n1;
    float bf = 1e30f, bi = 1e30f;
    uint32_t rf = 4, ri = 4;
    for (int rb : {4, 3, 2}) {
      if (rb != 4 && !row_rb_ok(rb, n2)) continue;  // radix-16 also stands for "no row pass"
      ntt_plan_t p = nullptr;
      st = ntt_plan_create(&p, N, moduli, num_moduli, word_bits, NTT_FLAG_SPLIT(n1));
      if (st != NTT_OK) break;
      p->row_rb = rb;  // pin the radix for this measurement
      float uf = 0, ui = 0;
      st = time_dir(p, false, &uf);
      if (st == NTT_OK) st = time_dir(p, true, &ui);
      ntt_plan_destroy(p);
      if (st != NTT_OK) break;
      if (uf < bf) { bf = uf; rf = (uint32_t)rb; }
      if (ui < bi) { bi = ui; ri = (uint32_t)rb; }
    }
    if (st != NTT_OK) break;
    if (bf + bi < best) {
      best = bf + bi;
      best_split = (uint32_t)n1;
      best_rb_f = rf;
      best_rb_i = ri;
    }
    any = true;
  }
  // Column-pass workgroup size at the chosen split and radices (the default,
  // 256, unless another is faster).
  uint32_t best_cb = 0;
  float best_cb_us = 0.f;
  if (st == NTT_OK && any && best_split > 0) {
    float bc = 1e30f;
    for (uint32_t cb : {256u, 128u, 64u}) {
      ntt_plan_t p = nullptr;
      st = ntt_plan_create(&p, N, moduli, num_moduli, word_bits, NTT_FLAG_SPLIT(best_split));
      if (st != NTT_OK) break;
      p->col_block = cb;
      float uf = 0, ui = 0;
      p->row_rb = (int)best_rb_f;
      st = time_dir(p, false, &uf);
      p->row_rb = (int)best_rb_i;
      if (st == NTT_OK) st = time_dir(p, true, &ui);
      ntt_plan_destroy(p);
      if (st != NTT_OK) break;
      if (uf + ui < bc) {
        bc = uf + ui;
        best_cb = cb;
      }
    }
    best_cb_us = bc;
  }
  // Polymul rows at the chosen split: radix-16 against radix-8 (b aliases a; out
  // is a second buffer).  Skipped when that buffer cannot be had.
  uint32_t best_rb_pm = 0;
  if (st == NTT_OK && any) {
    // polymul's own split rule: its rows are at most 2^13 words
    const uint32_t pm_split = polymul_split_log((uint32_t)log_n, best_split);
    const int n2 = log_n - (int)pm_split;
    void* out = nullptr;
    if (n2 >= 10 && n2 <= 13 && hipMalloc(&out, bytes) == hipSuccess) {
      float bp = 1e30f;
      for (int rb : {4, 3}) {
        ntt_plan_t p = nullptr;
        st = ntt_plan_create(&p, N, moduli, num_moduli, word_bits,
                             NTT_FLAG_SPLIT(best_split) | (rb == 3 ? NTT_FLAG_ROW_RADIX8 : 0u));
        if (st != NTT_OK) break;
        if (rb == 4) p->row_rb = 4;
        for (int w = 0; w < 2 && st == NTT_OK; ++w) st = ntt_polymul(p, out, buf, buf, batch, s);
        float ms = 1e30f;
        hipError_t he = hipSuccess;
        for (int trial = 0; trial < 3 && st == NTT_OK && he == hipSuccess; ++trial) {
          (void)hipEventRecord(a, s);
          for (int r = 0; r < reps && st == NTT_OK; ++r) st = ntt_polymul(p, out, buf, buf, batch, s);
          (void)hipEventRecord(b, s);
          he = hipEventSynchronize(b);
          float t = 0.f;
          if (he == hipSuccess) he = hipEventElapsedTime(&t, a, b);
          ms = std::min(ms, t);
        }
        ntt_plan_destroy(p);
        if (st != NTT_OK) break;
        if (he != hipSuccess) { st = hip_fail(he, "tuning run"); break; }
        if (ms < bp) { bp = ms; best_rb_pm = (uint32_t)rb; }
      }
      (void)hipFree(out);
    } else {
      (void)hipGetLastError();
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  (void)hipFree(buf);
  if (st != NTT_OK) return st;
  if (!any) return fail(NTT_EINVAL, "no admissible split for N=%u", N);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_env_loaded();
    const uint32_t cls = class_of(moduli[0], word_bits);
    const uint32_t bk = bucket_of((uint64_t)batch * num_moduli);
    g_table[Key(0u, (uint32_t)log_n, cls, bk)] = Entry{best_split, best};
    g_table[Key(2u, (uint32_t)log_n, cls, bk)] = Entry{best_rb_f, 0.f};
    g_table[Key(3u, (uint32_t)log_n, cls, bk)] = Entry{best_rb_i, 0.f};
    if (best_rb_pm) g_table[Key(4u, (uint32_t)log_n, cls, bk)] = Entry{best_rb_pm, 0.f};
    if (best_cb) g_table[Key(5u, (uint32_t)log_n, cls, bk)] = Entry{best_cb, best_cb_us};
  }
  if (best_n1) *best_n1 = best_split;
  if (best_us) *best_us = best;
  return NTT_OK;
}

ntt_status ntt_tune_ragged(uint32_t N, const uint64_t* moduli, uint32_t num_moduli, uint32_t batch,
                           uint32_t* best_row_log, float* best_us) {
  if (!moduli || num_moduli == 0 || batch == 0) return fail(NTT_EINVAL, "bad tuning shape");
  int log_n = 0;
  while ((1u << log_n) < N) ++log_n;
  if (log_n < 13) return fail(NTT_EINVAL, "ragged row length is only tuned for N >= 2^13");
  const uint64_t words = (uint64_t)batch * num_moduli * N;
  if (words >= (1ull << 32)) return fail(NTT_EINVAL, "tuning shape too large");
  ntt_plan_t p = nullptr;
  ntt_status st = ntt_plan_create(&p, N, moduli, num_moduli, 64, 0);
  if (st != NTT_OK) return st;
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, words * 8);
  if (e != hipSuccess) {
    ntt_plan_destroy(p);
    return hip_fail(e, "hipMalloc(tuning scratch)");
  }
  hipStream_t s = nullptr;
  (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  hipLaunchKernelGGL(fill_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                     static_cast<uint64_t*>(buf), (size_t)words);
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  float best = 1e30f;
  uint32_t best_log = 12;
  for (uint32_t rl : {11u, 12u}) {
    ntt_job jobs[2] = {{p, NTT_OP_FORWARD, batch, buf}, {p, NTT_OP_INVERSE, batch, buf}};
    ntt_ragged_t rf = nullptr, ri = nullptr;
    const uint32_t fl = NTT_RAGGED_NO_GRAPH | NTT_RAGGED_IN_WORKGROUP | NTT_RAGGED_ROW_LOG(rl);
    st = ntt_ragged_create(&rf, &jobs[0], 1, fl);
    if (st == NTT_OK) st = ntt_ragged_create(&ri, &jobs[1], 1, fl);
    if (st != NTT_OK) {
      if (rf) ntt_ragged_destroy(rf);
      break;
    }
    for (int w = 0; w < 2; ++w) {
      ntt_ragged_run(rf, s);
      ntt_ragged_run(ri, s);
    }
    const int reps = 10;
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) {
      ntt_ragged_run(rf, s);
      ntt_ragged_run(ri, s);
    }
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    ntt_ragged_destroy(rf);
    ntt_ragged_destroy(ri);
    const float us = ms * 1000.f / reps;
    if (us < best) {
      best = us;
      best_log = rl;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  (void)hipFree(buf);
  ntt_plan_destroy(p);
  if (st != NTT_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_env_loaded();
    g_table[Key(1u, (uint32_t)log_n, 0u, 0u)] = Entry{best_log, best};
  }
  if (best_row_log) *best_row_log = best_log;
  if (best_us) *best_us = best;
  return NTT_OK;
}

ntt_status ntt_tune_save(const char* path) {
  if (!path) return fail(NTT_EINVAL, "null path");
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(NTT_EINVAL, "cannot write %s", path);
  std::fprintf(f, "{\n  \"version\": 1,\n  \"arch\": \"gfx950\",\n  \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : g_table) {
    std::fprintf(f, "    {\"kind\": %u, \"log_n\": %u, \"cls\": %u, \"bucket\": %u, \"value\": %u, \"us\": %.3f}%s\n",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 std::get<3>(kv.first), kv.second.value, kv.second.us,
                 ++i < g_table.size() ? "," : "");
  }
  std::fprintf(f, "  ]\n}\n");
  std::fclose(f);
  return NTT_OK;
}

ntt_status ntt_tune_load(const char* path) {
  if (!path) return fail(NTT_EINVAL, "null path");
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_loaded = true;
  return load_locked(path);
}

ntt_status ntt_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_loaded = true;
  g_table.clear();
  return NTT_OK;
}

}  // extern "C"
