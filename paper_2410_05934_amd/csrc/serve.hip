// serve.hip -- continuous batching of NTT / polymul requests on one GPU.
//
// A host thread owns the device side.  Requests wait in a FIFO; the thread
// admits the oldest request whose device bytes fit under the HBM budget
// (bytes of requests already in flight are still held), then pulls every
// other waiting request that can share its launch and also fits, up to
// max_batch polynomials, and issues them as ONE launch: gather kernel -> the
// library's batched transform/polymul -> scatter kernel, on one of n_streams
// streams.  Requests share a launch when they have the same shape (op, N, word
// width, memory kind, moduli).  With NTT_SERVER_MERGE_MODULI the moduli may
// differ as long as every modulus of both requests is in the same arithmetic
// class (the CKKS-shaped requests of a serving mix each carry their own number
// of limbs).  Such a launch runs over one virtual plan whose limbs are the
// requests' limbs laid end to end ([sum batch_i L_i][N], the gathered layout),
// with the limb constants gathered on the device from the requests' own plans.  Requests that arrive while launches run are
// admitted as memory and stream slots free up, so their work overlaps on the
// device.  Plans (and their twiddle tables) are created on first use and stay
// resident.  The batched arithmetic is the same per polynomial as alone, so a
// request's result does not depend on what it was batched with.
//
// The paper batches the TFHE CMux of all ciphertexts into one gate per key bit
// (Sec. IV-A, Tab. lut-opt) to raise utilisation and cut launches; this server
// does the same for independent requests arriving over time.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "ntt_internal.hpp"

namespace nttk {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kPollUs = 4;       // completion polling interval of the server thread
constexpr uint64_t kMaxLaunchWords = 1ull << 32;  // words per library call: batch * L * N below this
constexpr int kMaxCopies = 96;  // descriptors per gather/scatter launch (kernel-argument payload)
constexpr uint64_t kMaxMergedLimbs = 4096;  // limb-rows of a launch over requests of different moduli

// Copy n64 8-byte units; with period != 0 the source repeats every `period`
// units (dst[i] = src[i % period]: a limb table replicated per polynomial).
struct CopyDesc {
  uint64_t* dst;
  const uint64_t* src;
  uint64_t n64;  // 8-byte units
  uint64_t period;
};
struct CopyList {
  CopyDesc d[kMaxCopies];
  uint32_t n;
};

__global__ void copy_list_kernel(CopyList list) {
  const CopyDesc c = list.d[blockIdx.y];
  if (!c.period && ((reinterpret_cast<uintptr_t>(c.dst) | reinterpret_cast<uintptr_t>(c.src)) & 15u) == 0) {
    // 16-byte accesses; the odd last unit, if any, by one thread
    const uint64_t n128 = c.n64 >> 1;
    uint4* d = reinterpret_cast<uint4*>(c.dst);
    const uint4* s = reinterpret_cast<const uint4*>(c.src);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n128;
         i += (uint64_t)gridDim.x * blockDim.x)
      d[i] = s[i];
    if ((c.n64 & 1) && blockIdx.x == 0 && threadIdx.x == 0) c.dst[c.n64 - 1] = c.src[c.n64 - 1];
    return;
  }
  if (c.period) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < c.n64;
         i += (uint64_t)gridDim.x * blockDim.x)
      c.dst[i] = c.src[i % c.period];
    return;
  }
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < c.n64;
       i += (uint64_t)gridDim.x * blockDim.x)
    c.dst[i] = c.src[i];
}

hipError_t copy_many(const std::vector<CopyDesc>& v, hipStream_t s) {
  for (size_t off = 0; off < v.size(); off += kMaxCopies) {
    CopyList l;
    l.n = (uint32_t)std::min<size_t>(kMaxCopies, v.size() - off);
    uint64_t mx = 0, units = 0;
    for (uint32_t i = 0; i < l.n; ++i) {
      l.d[i] = v[off + i];
      mx = std::max(mx, l.d[i].n64);
      units += l.d[i].n64;
    }
    // blocks per descriptor: one per 512 units of the longest, at most 16384
    // blocks in all (at least 64 per descriptor); the loops stride the rest
    const uint64_t cap = std::max<uint64_t>(64, 16384 / l.n);
    const uint32_t bx = (uint32_t)std::min<uint64_t>(cap, (mx + 511) / 512);
    LaunchTimer t("server_copy", "u64", 0, false, false, units, s);
    hipLaunchKernelGGL(copy_list_kernel, dim3(std::max(1u, bx), l.n), dim3(256), 0, s, l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per-request row-table entries of a launch whose kernels address the
// requests' own buffers: limb-rows start .. start + rows - 1 of the launch are
// rows 0 .. rows - 1 of a, b and out (row_bytes apart).
constexpr uint32_t kMaxReqs = 64;  // requests per launch
struct RowTabEntry {
  uint64_t a, b, out;
  uint32_t start, rows;
};
struct RowTabList {
  RowTabEntry e[kMaxReqs];
  uint64_t row_bytes;
};

__global__ void row_table_kernel(RowTabList l, uint64_t* ta, uint64_t* tb, uint64_t* to) {
  const RowTabEntry q = l.e[blockIdx.y];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < q.rows; j += gridDim.x * blockDim.x) {
    const uint64_t off = (uint64_t)j * l.row_bytes;
    ta[q.start + j] = q.a + off;
    tb[q.start + j] = q.b + off;
    to[q.start + j] = q.out + off;
  }
}

struct Req {
  uint64_t id = 0;
  ntt_request r{};
  std::vector<uint64_t> moduli;
  int cls = -1;         // arithmetic class shared by every modulus, or -1
  uint64_t words = 0;   // batch * L * N
  uint64_t bytes = 0;   // device bytes held while in flight
  ntt_request_info info{};
  bool done = false;
};

struct Batch {
  std::vector<Req*> reqs;
  uint64_t launch_id = 0;
  int stream = 0;
  hipEvent_t ev = nullptr;
  uint64_t bytes = 0;
  double t_ready = 0;  // dry run: modelled completion time
};

using ShapeKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, std::vector<uint64_t>>;

ShapeKey shape_of(const Req* q) {
  return ShapeKey(q->r.op, q->r.N, q->r.word_bits, q->r.memory, q->moduli);
}

// Requests of different moduli share a launch when this key matches and is
// defined (cls >= 0).
using MergeKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, int>;
MergeKey merge_of(const Req* q) {
  return MergeKey(q->r.op, q->r.N, q->r.word_bits, q->r.memory, q->cls);
}

// Arithmetic class of one modulus (the plan's rule): 32-bit words, fp64 with
// 64-bit words below kF64LBound, 64-bit integer above.
int class_of(uint64_t q, uint32_t word_bits) {
  if (word_bits == 32) return 0;
  return q < kF64LBound ? 1 : 2;
}

}  // namespace
}  // namespace nttk

using namespace nttk;

struct ntt_server_s {
  uint64_t budget = 0;
  uint32_t n_streams = 1;
  uint32_t max_batch = 4096;
  uint32_t flags = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_load;
  // Per-stream staging arena, grown on demand and reused in stream order (a
  // later batch on the same stream runs after the earlier one's scatter).
  std::vector<void*> arena;
  std::vector<size_t> arena_bytes;
  std::vector<hipEvent_t> free_events;  // completion events, reused (server thread only)
  uint32_t max_reqs = kMaxReqs;
  std::atomic<uint64_t> direct_launches{0};  // set by the server thread outside the lock
  std::map<std::tuple<uint32_t, uint32_t, std::vector<uint64_t>>, ntt_plan_t> plans;

  // Moduli already checked for (N, word_bits): a submit checks each modulus of
  // a request once per server, not once per request (a check costs a few
  // microseconds; a request carries up to dozens of moduli).
  std::mutex checked_mu;
  std::set<std::tuple<uint32_t, uint32_t, uint64_t>> checked;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<Batch*> inflight;
  uint64_t inflight_bytes = 0;
  uint64_t next_id = 1;
  bool stopping = false;
  ntt_server_counters ctr{};
  std::thread th;

  uint32_t* d_iota = nullptr;  // 0, 1, ..., kMaxMergedLimbs - 1: the limb list of a merged launch

  bool serial() const { return flags & NTT_SERVER_SERIAL; }
  bool dry() const { return flags & NTT_SERVER_DRY_RUN; }
  bool merging() const { return !serial() && (flags & NTT_SERVER_MERGE_MODULI); }

  ntt_plan_t plan_for(const Req* q, ntt_status* st) {
    auto key = std::make_tuple(q->r.N, q->r.word_bits, q->moduli);
    auto it = plans.find(key);
    if (it != plans.end()) return it->second;
    ntt_plan_t p = nullptr;
    *st = ntt_plan_create(&p, q->r.N, q->moduli.data(), (uint32_t)q->moduli.size(), q->r.word_bits, 0);
    if (*st != NTT_OK) return nullptr;
    plans[key] = p;
    std::lock_guard<std::mutex> lk(mu);  // counters are read under the lock
    ctr.plans_cached = plans.size();
    return p;
  }

  // Issue one batch: requests of one shape, or (NTT_SERVER_MERGE_MODULI) of one
  // merge key.  Called by the server thread without the lock; it takes the
  // lock only to update the counters.
  ntt_status launch(Batch* b) {
    const double t = now_s();
    uint32_t polys = 0;
    for (Req* q : b->reqs) {
      q->info.t_launch = t;
      q->info.batched_with = (uint32_t)b->reqs.size();
      q->info.launch_id = b->launch_id;
      polys += q->r.batch;
    }
    if (dry()) {
      // Modelled duration: 50 us per launch plus 2 ns per word.
      uint64_t w = 0;
      for (Req* q : b->reqs) w += q->words;
      b->t_ready = t + 50e-6 + 2e-9 * (double)w;
      return NTT_OK;
    }
    hipStream_t s = streams[b->stream];
    const Req* q0 = b->reqs[0];
    ntt_status st = NTT_OK;
    ntt_plan_t plan = plan_for(q0, &st);
    if (!plan) return st;
    const uint32_t wb = q0->r.word_bits / 8;
    const bool pm = q0->r.op == NTT_REQ_POLYMUL;
    const bool host = q0->r.memory == NTT_REQ_HOST;
    const bool single = b->reqs.size() == 1 && !host;
    bool mixed = false;
    for (const Req* q : b->reqs) mixed = mixed || q->moduli != q0->moduli;
    // A launch over requests of different moduli runs one polynomial of a
    // virtual plan whose limbs are every request's limbs, polynomial by
    // polynomial, in gather order.  Its host constants are concatenated here;
    // its device constants are gathered into the arena with the operands.
    ntt_plan_s vp;
    std::vector<const ntt_plan_s*> src_plans;
    ntt_plan_t run = plan;
    uint32_t run_batch = polys;
    if (mixed) {
      if (!d_iota) return fail(NTT_ENOMEM, "server limb list missing");
      vp.device = plan->device;
      vp.N = plan->N;
      vp.log_n = plan->log_n;
      vp.word_bits = plan->word_bits;
      vp.log_n1 = plan->log_n1;
      for (const Req* q : b->reqs) {
        ntt_plan_t qp = plan_for(q, &st);
        if (!qp) return st;
        src_plans.push_back(qp);
        for (uint32_t k = 0; k < q->r.batch; ++k) {
          vp.moduli.insert(vp.moduli.end(), qp->moduli.begin(), qp->moduli.end());
          vp.psi.insert(vp.psi.end(), qp->psi.begin(), qp->psi.end());
          vp.cls.insert(vp.cls.end(), qp->cls.begin(), qp->cls.end());
          vp.h_limbs.insert(vp.h_limbs.end(), qp->h_limbs.begin(), qp->h_limbs.end());
        }
      }
      vp.L = (uint32_t)vp.moduli.size();
      const int c = q0->cls;
      vp.cls_cnt[c] = vp.L;
      vp.h_cls_limbs.resize(vp.L);
      for (uint32_t l = 0; l < vp.L; ++l) vp.h_cls_limbs[l] = l;
      vp.d_cls_limbs = d_iota;
      run = &vp;
      run_batch = 1;
    }
    hipError_t e = hipSuccess;
    // Grow this stream's arena to `need` bytes: wait for its earlier batches,
    // then reallocate (rare: the arena keeps its largest size).  The arenas
    // together never hold more than the budget: when growing this one would
    // pass it, the other streams' arenas are released first (after their
    // streams have finished with them) and regrown on demand.  need is at most
    // the batch's admitted bytes, which fit in the budget.
    auto reserve = [&](size_t need) -> hipError_t {
      const int me = b->stream;
      if (arena_bytes[me] >= need) return hipSuccess;
      hipError_t r = hipStreamSynchronize(s);
      if (r == hipSuccess && arena[me]) r = hipFree(arena[me]);
      arena[me] = nullptr;
      arena_bytes[me] = 0;
      const size_t grow = (size_t)std::min<uint64_t>(std::max(need, (size_t)64 << 20),
                                                     std::max<uint64_t>(need, budget));
      uint64_t others = 0;
      for (size_t j = 0; j < arena.size(); ++j) others += arena_bytes[j];
      for (size_t j = 0; r == hipSuccess && others + grow > budget && j < arena.size(); ++j) {
        if ((int)j == me || !arena[j]) continue;
        r = hipStreamSynchronize(streams[j]);
        if (r == hipSuccess) r = hipFree(arena[j]);
        others -= arena_bytes[j];
        arena[j] = nullptr;
        arena_bytes[j] = 0;
      }
      if (r == hipSuccess) r = hipMalloc(&arena[me], grow);
      if (r == hipSuccess) arena_bytes[me] = grow;
      uint64_t held = 0;
      for (size_t j = 0; j < arena.size(); ++j) held += arena_bytes[j];
      std::lock_guard<std::mutex> lk(mu);
      ctr.arena_bytes = held;
      ctr.max_arena_bytes = std::max(ctr.max_arena_bytes, held);
      return r;
    };
    if (single) {
      // Operands are resident: run in place on the request's own buffers; a
      // two-pass polymul takes its workspace from the stream's arena.
      const Req* q = q0;
      if (pm) {
        const size_t ws = polymul_ws_bytes(plan, q->r.batch);
        if (ws && (e = reserve(ws)) != hipSuccess) return hip_fail(e, "server staging allocation");
        st = polymul_into(plan, q->r.out, q->r.a, q->r.b, q->r.batch, ws ? arena[b->stream] : nullptr, s);
      } else {
        if (q->r.out != q->r.a)
          e = hipMemcpyAsync(q->r.out, q->r.a, q->words * wb, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          st = q->r.op == NTT_REQ_FORWARD ? ntt_forward(plan, q->r.out, q->r.batch, s)
                                           : ntt_inverse(plan, q->r.out, q->r.batch, s);
      }
    } else if (pm && !host && polymul_rows_ok(run, run_batch)) {
      // Two-pass polymul straight from and into the requests' buffers: the first
      // column launch reads every a and b through row tables, the last one
      // writes every out through one; nothing is gathered or scattered.
      // Arena layout: O | workspace | limb constants (mixed launch) | tables.
      uint64_t total = 0;
      for (const Req* q : b->reqs) total += q->words * wb;
      const uint64_t rows = (uint64_t)run_batch * run->L;
      const size_t limb_off = ((size_t)2 * total + 255) & ~(size_t)255;
      const size_t tab_off = (limb_off + (mixed ? (size_t)vp.L * sizeof(LimbDev) : 0) + 255) & ~(size_t)255;
      const size_t need = tab_off + (size_t)3 * rows * sizeof(uint64_t);
      if ((e = reserve(need)) != hipSuccess) return hip_fail(e, "server staging allocation");
      unsigned char* base = static_cast<unsigned char*>(arena[b->stream]);
      void* O = base;
      void* WS = base + total;
      uint64_t* ta = reinterpret_cast<uint64_t*>(base + tab_off);
      uint64_t* tb = ta + rows;
      uint64_t* to = tb + rows;
      RowTabList list{};
      list.row_bytes = (uint64_t)q0->r.N * wb;
      uint32_t start = 0, most = 0;
      for (size_t i = 0; i < b->reqs.size(); ++i) {
        const Req* q = b->reqs[i];
        const uint32_t qr = q->r.batch * (uint32_t)q->moduli.size();
        list.e[i] = RowTabEntry{reinterpret_cast<uint64_t>(q->r.a), reinterpret_cast<uint64_t>(q->r.b),
                                reinterpret_cast<uint64_t>(q->r.out), start, qr};
        start += qr;
        most = std::max(most, qr);
      }
      hipLaunchKernelGGL(row_table_kernel, dim3((most + 255) / 256, (uint32_t)b->reqs.size()), dim3(256),
                         0, s, list, ta, tb, to);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "server row tables");
      if (mixed) {
        unsigned char* dl = base + limb_off;
        vp.d_limbs = reinterpret_cast<LimbDev*>(dl);
        std::vector<CopyDesc> lc;
        for (size_t i = 0; i < b->reqs.size(); ++i) {
          const Req* q = b->reqs[i];
          const uint64_t unit = q->moduli.size() * sizeof(LimbDev) / 8;
          lc.push_back(CopyDesc{reinterpret_cast<uint64_t*>(dl),
                                reinterpret_cast<const uint64_t*>(src_plans[i]->d_limbs),
                                unit * q->r.batch, unit});
          dl += unit * 8 * q->r.batch;
        }
        if ((e = copy_many(lc, s)) != hipSuccess) return hip_fail(e, "server limb constants");
      }
      st = polymul_rows_into(run, to, ta, tb, run_batch, O, WS, s);
      if (st == NTT_OK) direct_launches.fetch_add(1, std::memory_order_relaxed);
    } else {
      // Gather every operand into one contiguous batch, run one launch, scatter.
      // Arena layout: A | B | O | polymul workspace (polymul), A (transforms);
      // then, for a mixed launch, the virtual plan's limb constants.
      uint64_t total = 0;
      for (const Req* q : b->reqs) total += q->words * wb;
      const size_t ws = pm ? polymul_ws_bytes(run, run_batch) : 0;
      const size_t limb_off = (((size_t)total * (pm ? 3 : 1) + ws) + 255) & ~(size_t)255;
      const size_t need = mixed ? limb_off + (size_t)vp.L * sizeof(LimbDev)
                                : (size_t)total * (pm ? 3 : 1) + ws;
      if ((e = reserve(need)) != hipSuccess) return hip_fail(e, "server staging allocation");
      void* A = arena[b->stream];
      void* B = pm ? static_cast<unsigned char*>(A) + total : nullptr;
      void* O = pm ? static_cast<unsigned char*>(A) + 2 * total : nullptr;
      void* WS = ws ? static_cast<unsigned char*>(A) + 3 * total : nullptr;
      std::vector<CopyDesc> in;
      if (mixed) {
        static_assert(sizeof(LimbDev) % 8 == 0, "limb constants copy in 8-byte units");
        unsigned char* dl = static_cast<unsigned char*>(A) + limb_off;
        vp.d_limbs = reinterpret_cast<LimbDev*>(dl);
        for (size_t i = 0; i < b->reqs.size(); ++i) {
          const Req* q = b->reqs[i];
          const uint64_t unit = q->moduli.size() * sizeof(LimbDev) / 8;
          in.push_back(CopyDesc{reinterpret_cast<uint64_t*>(dl),
                                reinterpret_cast<const uint64_t*>(src_plans[i]->d_limbs),
                                unit * q->r.batch, unit});
          dl += unit * 8 * q->r.batch;
        }
      }
      uint64_t off = 0;
      for (Req* q : b->reqs) {
        const uint64_t bytes = q->words * wb;
        unsigned char* da = static_cast<unsigned char*>(A) + off;
        if (host) {
          e = hipMemcpyAsync(da, q->r.a, bytes, hipMemcpyHostToDevice, s);
          if (e == hipSuccess && pm)
            e = hipMemcpyAsync(static_cast<unsigned char*>(B) + off, q->r.b, bytes,
                               hipMemcpyHostToDevice, s);
          if (e != hipSuccess) return hip_fail(e, "server input copy");
        } else {
          in.push_back(CopyDesc{reinterpret_cast<uint64_t*>(da), static_cast<const uint64_t*>(q->r.a), bytes / 8, 0});
          if (pm)
            in.push_back(CopyDesc{reinterpret_cast<uint64_t*>(static_cast<unsigned char*>(B) + off),
                                  static_cast<const uint64_t*>(q->r.b), bytes / 8, 0});
        }
        off += bytes;
      }
      if (!in.empty() && (e = copy_many(in, s)) != hipSuccess) return hip_fail(e, "server gather");
      void* res = pm ? O : A;
      if (pm) st = polymul_into(run, O, A, B, run_batch, WS, s);
      else st = q0->r.op == NTT_REQ_FORWARD ? ntt_forward(run, A, run_batch, s)
                                             : ntt_inverse(run, A, run_batch, s);
      if (st != NTT_OK) return st;
      std::vector<CopyDesc> outc;
      off = 0;
      for (Req* q : b->reqs) {
        const uint64_t bytes = q->words * wb;
        const unsigned char* src = static_cast<const unsigned char*>(res) + off;
        if (host) {
          e = hipMemcpyAsync(q->r.out, src, bytes, hipMemcpyDeviceToHost, s);
          if (e != hipSuccess) return hip_fail(e, "server output copy");
        } else {
          outc.push_back(CopyDesc{static_cast<uint64_t*>(q->r.out), reinterpret_cast<const uint64_t*>(src), bytes / 8, 0});
        }
        off += bytes;
      }
      if (!outc.empty() && (e = copy_many(outc, s)) != hipSuccess) return hip_fail(e, "server scatter");
    }
    if (st != NTT_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "server launch");
    if (!free_events.empty()) {
      b->ev = free_events.back();
      free_events.pop_back();
    } else {
      e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(b->ev, s);
    return e == hipSuccess ? NTT_OK : hip_fail(e, "server event");
  }

  bool batch_done(Batch* b) {
    if (dry()) return now_s() >= b->t_ready;
    return hipEventQuery(b->ev) != hipErrorNotReady;
  }

  void finish(Batch* b, int32_t status) {
    const double t = now_s();
    for (Req* q : b->reqs) {
      q->info.t_done = t;
      q->info.status = status;
      q->done = true;
      ctr.completed += 1;
    }
    inflight_bytes -= b->bytes;
    stream_load[b->stream] -= 1;
    if (b->ev) free_events.push_back(b->ev);
    delete b;
  }

  int pick_stream() {
    int best = 0;
    for (int i = 1; i < (int)stream_load.size(); ++i)
      if (stream_load[i] < stream_load[best]) best = i;
    return best;
  }

  // Form batches under the lock: reserve their bytes and stream slots.
  void admit(std::vector<Batch*>* out) {
    const uint32_t slots = serial() ? 1u : n_streams * 2u;
    while (!pending.empty() && inflight.size() < slots) {
      // Oldest request that fits in the budget.
      auto it = pending.begin();
      if (!serial()) {
        while (it != pending.end() && inflight_bytes + (*it)->bytes > budget) ++it;
      } else if (inflight_bytes + (*it)->bytes > budget) {
        it = pending.end();
      }
      if (it == pending.end()) break;
      Batch* b = new Batch();
      Req* head = *it;
      pending.erase(it);
      b->reqs.push_back(head);
      b->bytes = head->bytes;
      uint32_t polys = head->r.batch;
      uint64_t words = head->words;
      uint64_t limbs = (uint64_t)head->r.batch * head->moduli.size();
      bool mixed = false;
      if (!serial()) {
        const ShapeKey key = shape_of(head);
        const MergeKey mkey = merge_of(head);
        const bool can_merge = merging() && head->cls >= 0;
        for (auto jt = pending.begin(); jt != pending.end();) {
          Req* q = *jt;
          if (b->reqs.size() >= max_reqs) break;
          const uint64_t ql = (uint64_t)q->r.batch * q->moduli.size();
          // a launch covers fewer than 2^32 words (the library's per-call
          // limit), so a request never fails because of its batch mates
          const bool fits = polys + q->r.batch <= max_batch && words + q->words < kMaxLaunchWords &&
                            inflight_bytes + b->bytes + q->bytes <= budget;
          const bool same = fits && shape_of(q) == key;
          const bool other = fits && !same && can_merge && q->cls >= 0 && merge_of(q) == mkey;
          // a launch that mixes moduli holds at most kMaxMergedLimbs limb-rows
          const bool mate = (same || other) && (!(mixed || other) || limbs + ql <= kMaxMergedLimbs);
          if (mate) {
            b->reqs.push_back(q);
            b->bytes += q->bytes;
            polys += q->r.batch;
            words += q->words;
            limbs += ql;
            mixed = mixed || !same;
            jt = pending.erase(jt);
          } else {
            ++jt;
          }
        }
      }
      if (mixed) ctr.merged_launches += 1;
      const double t = now_s();
      for (Req* q : b->reqs) q->info.t_admit = t;
      b->stream = pick_stream();
      stream_load[b->stream] += 1;
      inflight_bytes += b->bytes;
      ctr.max_inflight_bytes = std::max(ctr.max_inflight_bytes, inflight_bytes);
      ctr.launches += 1;
      b->launch_id = ctr.launches;
      inflight.push_back(b);
      uint64_t nreq = 0;
      for (Batch* x : inflight) nreq += x->reqs.size();
      ctr.max_inflight_requests = std::max(ctr.max_inflight_requests, nreq);
      out->push_back(b);
    }
  }

  // The device work (HIP calls) runs without the lock, so submitters never
  // wait behind a launch; only the server thread touches `inflight`, the
  // streams and the plan cache.
  void loop() {
    std::vector<Batch*> done, launched, failed;
    std::vector<ntt_status> fail_st;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu);
        if (inflight.empty() && pending.empty()) {
          if (stopping) break;
          cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
          continue;
        }
      }
      done.clear();
      for (Batch* b : inflight)
        if (batch_done(b)) done.push_back(b);
      launched.clear();
      {
        std::lock_guard<std::mutex> lk(mu);
        for (Batch* b : done) {
          inflight.erase(std::find(inflight.begin(), inflight.end(), b));
          finish(b, NTT_OK);
        }
        if (!done.empty()) cv_done.notify_all();
        admit(&launched);
      }
      failed.clear();
      fail_st.clear();
      for (Batch* b : launched) {
        const ntt_status st = launch(b);
        if (st != NTT_OK) {
          failed.push_back(b);
          fail_st.push_back(st);
        }
      }
      if (!failed.empty()) {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < failed.size(); ++i) {
          inflight.erase(std::find(inflight.begin(), inflight.end(), failed[i]));
          finish(failed[i], fail_st[i]);
        }
        cv_done.notify_all();
      }
      if (done.empty() && launched.empty()) {
        std::unique_lock<std::mutex> lk(mu);
        // Poll in-flight work every few microseconds; wake early for new arrivals.
        cv_work.wait_for(lk, std::chrono::microseconds(kPollUs));
      }
    }
  }
};

extern "C" {

ntt_status ntt_server_create(ntt_server_t* out, uint64_t budget_bytes, uint32_t n_streams,
                             uint32_t max_batch, uint32_t flags) {
  if (!out || budget_bytes == 0 || n_streams == 0 || n_streams > 64)
    return fail(NTT_EINVAL, "bad server arguments");
  *out = nullptr;
  ntt_server_s* s = new (std::nothrow) ntt_server_s();
  if (!s) return fail(NTT_ENOMEM, "host allocation");
  s->budget = budget_bytes;
  s->n_streams = n_streams;
  s->max_batch = max_batch ? max_batch : 4096;
  s->flags = flags;
  s->ctr.budget_bytes = budget_bytes;
  s->stream_load.assign(n_streams, 0);
  s->arena.assign(n_streams, nullptr);
  s->arena_bytes.assign(n_streams, 0);
  if (!s->dry()) {
    hipError_t e = hipGetDevice(&s->device);
    // Staging buffers come from the device's default stream-ordered pool; keep
    // freed blocks cached there (no release to the driver at synchronisation
    // points), so a launch's staging allocation is a pool hit.
    hipMemPool_t pool = nullptr;
    if (e == hipSuccess && hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) {
      uint64_t keep = budget_bytes;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    for (uint32_t i = 0; e == hipSuccess && i < n_streams; ++i) {
      hipStream_t st = nullptr;
      e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e == hipSuccess) {
      std::vector<uint32_t> iota(kMaxMergedLimbs);
      for (uint32_t i = 0; i < kMaxMergedLimbs; ++i) iota[i] = i;
      e = hipMalloc(&s->d_iota, kMaxMergedLimbs * sizeof(uint32_t));
      if (e == hipSuccess)
        e = hipMemcpy(s->d_iota, iota.data(), kMaxMergedLimbs * sizeof(uint32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
      if (s->d_iota) (void)hipFree(s->d_iota);
      delete s;
      return hip_fail(e, "server streams");
    }
  }
  s->th = std::thread([s] {
    // The loop polls in-flight launches with short timed waits; the default
    // 50 us timer slack of a Linux thread would stretch every one of them.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    if (!s->dry()) (void)hipSetDevice(s->device);
    s->loop();
  });
  *out = s;
  return NTT_OK;
}

ntt_status ntt_server_submit(ntt_server_t s, const ntt_request* r, uint64_t* id) {
  if (!s || !r || !id) return fail(NTT_EINVAL, "null argument");
  if (r->op > NTT_REQ_INVERSE || r->batch == 0 || !r->moduli || r->num_moduli == 0 ||
      (r->memory != NTT_REQ_DEVICE && r->memory != NTT_REQ_HOST))
    return fail(NTT_EINVAL, "bad request");
  if (!s->dry() && (!r->a || !r->out || (r->op == NTT_REQ_POLYMUL && !r->b)))
    return fail(NTT_EINVAL, "null operand");
  for (uint32_t l = 0; l < r->num_moduli; ++l) {
    const auto key = std::make_tuple(r->N, r->word_bits, r->moduli[l]);
    {
      std::lock_guard<std::mutex> lk(s->checked_mu);
      if (s->checked.count(key)) continue;
    }
    const ntt_status st = ntt_check_modulus(r->N, r->moduli[l], r->word_bits);
    if (st != NTT_OK) return st;
    std::lock_guard<std::mutex> lk(s->checked_mu);
    s->checked.insert(key);
  }
  Req* q = new (std::nothrow) Req();
  if (!q) return fail(NTT_ENOMEM, "host allocation");
  q->r = *r;
  q->moduli.assign(r->moduli, r->moduli + r->num_moduli);
  q->r.moduli = nullptr;
  q->cls = class_of(q->moduli[0], r->word_bits);
  for (uint64_t m : q->moduli)
    if (class_of(m, r->word_bits) != q->cls) q->cls = -1;
  q->words = (uint64_t)r->batch * r->num_moduli * r->N;
  if (q->words >= kMaxLaunchWords) {
    delete q;
    return fail(NTT_EINVAL, "request of %llu words: batch * L * N must be below 2^32",
                (unsigned long long)((uint64_t)r->batch * r->num_moduli * r->N));
  }
  const uint64_t opnd = q->words * (r->word_bits / 8);
  // Device bytes while in flight: staging for inputs and output (+ the
  // polymul workspace when the transform has a column pass), and per limb-row
  // the constants a merged launch copies and the three row-table entries of an
  // in-place launch, plus alignment slack: a launch's arena never needs more
  // than the bytes its requests were admitted with.
  const uint64_t nbuf = r->op == NTT_REQ_POLYMUL ? 4 : 2;
  const uint64_t limb_rows = (uint64_t)r->batch * r->num_moduli;
  q->bytes = opnd * nbuf + limb_rows * (sizeof(LimbDev) + 3 * sizeof(uint64_t)) + 1024;
  std::lock_guard<std::mutex> lk(s->mu);
  q->id = s->next_id++;
  q->info.id = q->id;
  q->info.t_submit = now_s();
  q->info.bytes = q->bytes;
  s->ctr.submitted += 1;
  if (q->bytes > s->budget) {
    s->ctr.rejected += 1;
    delete q;
    return fail(NTT_ENOMEM, "request needs %llu bytes, budget is %llu",
                (unsigned long long)q->bytes, (unsigned long long)s->budget);
  }
  if (s->stopping) {
    delete q;
    return fail(NTT_EBUSY, "server is stopping");
  }
  s->reqs[q->id] = q;
  s->pending.push_back(q);
  *id = q->id;
  s->cv_work.notify_one();
  return NTT_OK;
}

ntt_status ntt_server_wait(ntt_server_t s, uint64_t id, ntt_request_info* info, int32_t timeout_ms) {
  if (!s) return fail(NTT_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(NTT_EINVAL, "unknown request %llu", (unsigned long long)id);
  Req* q = it->second;
  auto ready = [&] { return q->done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return fail(NTT_ETIMEOUT, "request %llu not done", (unsigned long long)id);
  }
  if (info) *info = q->info;
  const int32_t st = q->info.status;
  s->reqs.erase(it);
  delete q;
  return st == NTT_OK ? NTT_OK : (ntt_status)st;
}

ntt_status ntt_server_replay(ntt_server_t s, const ntt_request* reqs, const double* arrival_s,
                             uint32_t n, uint64_t* ids) {
  if (!s || !reqs || !arrival_s || !ids) return fail(NTT_EINVAL, "null argument");
  const double t0 = now_s();
  for (uint32_t i = 0; i < n; ++i) {
    const double due = t0 + arrival_s[i];
    while (now_s() < due) {
    }
    const ntt_status st = ntt_server_submit(s, &reqs[i], &ids[i]);
    if (st != NTT_OK) {
      for (uint32_t j = i; j < n; ++j) ids[j] = 0;
      return st;
    }
  }
  return NTT_OK;
}

ntt_status ntt_server_counters_get(ntt_server_t s, ntt_server_counters* c) {
  if (!s || !c) return fail(NTT_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *c = s->ctr;
  c->direct_launches = s->direct_launches.load(std::memory_order_relaxed);
  return NTT_OK;
}

ntt_status ntt_server_destroy(ntt_server_t s) {
  if (!s) return fail(NTT_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->reqs) delete kv.second;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (void* a : s->arena)
    if (a) (void)hipFree(a);
  for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
  for (auto& kv : s->plans) ntt_plan_destroy(kv.second);
  if (s->d_iota) (void)hipFree(s->d_iota);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return NTT_OK;
}

}  // extern "C"
