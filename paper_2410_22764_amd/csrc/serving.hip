// serving.hip -- continuous-batching request loop.
//
// One worker thread owns a resident set of requests on the device.  Every
// step it
//   1. admits queued requests while a state range, a descriptor slot and
//      their device buffers fit the budget (admission by HBM footprint);
//      newcomers are validated, get their initial partition {F, Q\F} and
//      append their states to the shared active list;
//   2. runs ONE refinement round (the same fused kernels as the batch path)
//      over every resident request -- requests that arrived while others were
//      on the device join at the next step, so their work overlaps;
//   3. retires every request whose round split nothing: canonical numbering
//      of its states only (segmented scan), copy-out, buffers released.
// Instances never interact: block ids are global state ids, so a request's
// result is the same alone and in any mix.
#include "serving.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "closure.h"
#include "engine.h"

namespace dfamin {

namespace {

constexpr uint32_t kSlots = 4096;               // resident requests at most
constexpr uint64_t kDefaultArenaStates = 1ull << 26;
constexpr uint32_t kDefaultAutoRounds = 8;
constexpr size_t kMaxQueue = 1u << 16;

inline uint32_t ceil_log2_u64(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// First-fit allocator of state-id ranges in [0, cap).
class RangeAlloc {
 public:
  void reset(uint64_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(uint64_t n, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length
};

// Caching device allocator with power-of-two size classes, bounded by a
// byte budget.  Blocks are reused by later requests; nothing is returned to
// HIP until the pool is destroyed (or space is needed for a larger class).
class DevicePool {
 public:
  ~DevicePool() { release_all(); }
  void set_budget(uint64_t b) { budget_ = b; }
  uint64_t used() const { return used_; }
  uint64_t budget() const { return budget_; }
  static size_t size_class(size_t bytes) {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
  }
  uint64_t live() const { return used_ - cached_; }
  void* alloc(size_t bytes) {
    const size_t c = size_class(bytes);
    auto& fl = free_[c];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      cached_ -= c;
      return p;
    }
    if (used_ + c > budget_) trim(used_ + c - budget_);
    if (used_ + c > budget_) return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    used_ += c;
    return p;
  }
  void free(void* p, size_t bytes) {
    if (!p) return;
    const size_t c = size_class(bytes);
    free_[c].push_back(p);
    cached_ += c;
  }
  void release_all() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipFree(p);
    free_.clear();
    used_ -= cached_;
    cached_ = 0;
  }

 private:
  void trim(uint64_t need) {
    for (auto& kv : free_) {
      while (!kv.second.empty() && need > 0) {
        (void)hipFree(kv.second.back());
        kv.second.pop_back();
        used_ -= kv.first;
        cached_ -= kv.first;
        need = need > kv.first ? need - kv.first : 0;
      }
    }
  }
  std::map<size_t, std::vector<void*>> free_;
  uint64_t budget_ = 0, used_ = 0, cached_ = 0;
};

// Page-locked host buffers for request inputs and outputs, reused by
// power-of-two size class and bounded by a byte cap.  Copies from and to
// page-locked memory run as asynchronous DMA at the full link rate, and
// reuse spares every request the page faults of fresh host memory.  Shared
// by the callers of submit/wait and the worker (hence the lock).
class PinnedPool {
 public:
  explicit PinnedPool(uint64_t cap) : cap_(cap) {}
  ~PinnedPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
  }
  // nullptr when the cap or the allocator says no (callers fall back to
  // pageable memory)
  void* alloc(size_t bytes, size_t* cls) {
    const size_t c = DevicePool::size_class(bytes);
    std::lock_guard<std::mutex> g(mu_);
    auto& fl = free_[c];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      *cls = c;
      return p;
    }
    // Blocks are never given back before the pool goes: unpinning (and
    // pinning again) hundreds of megabytes costs far more than the pageable
    // copy it would save, so past the cap requests use ordinary memory.
    if (total_ + c > cap_) return nullptr;
    void* p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    total_ += c;
    *cls = c;
    return p;
  }
  void free(void* p, size_t cls) {
    std::lock_guard<std::mutex> g(mu_);
    free_[cls].push_back(p);
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
  uint64_t cap_ = 0, total_ = 0;
};
constexpr uint64_t kPinnedCap = 8ull << 30;

// A host buffer of a request: page-locked from the pool when it fits, else
// ordinary memory.
struct HostStage {
  std::shared_ptr<PinnedPool> pool;
  void* pinned = nullptr;
  size_t cls = 0;
  std::vector<uint8_t> plain;
  void* data() { return pinned ? pinned : plain.data(); }
  bool make(const std::shared_ptr<PinnedPool>& pl, size_t bytes) {
    release();
    pool = pl;
    pinned = pool ? pool->alloc(bytes, &cls) : nullptr;
    if (pinned) return true;
    try {
      plain.resize(bytes);
    } catch (...) {
      return false;
    }
    return true;
  }
  void release() {
    if (pinned) pool->free(pinned, cls);
    pinned = nullptr;
    std::vector<uint8_t>().swap(plain);
  }
  ~HostStage() { release(); }
};

struct Request {
  uint64_t ticket = 0;
  uint32_t n = 0, k = 0, q0 = 0;
  dfamin_opts opts{};
  HostStage in;   // delta (4nk bytes), then the accept bitmap (ceil(n/8) bytes)
  HostStage out;  // n block ids, filled by the worker at retirement
  dfamin_result result{};
  int status = 1;  // 1 pending, else a DFAMIN_* code
  std::atomic<bool> cancelled{false};
  size_t delta_bytes() const { return 4ull * n * k; }
  size_t accept_bytes() const { return ((size_t)n + 7) / 8; }
  const void* delta() { return in.data(); }
  const void* accept() { return static_cast<char*>(in.data()) + delta_bytes(); }
};

struct Resident {
  std::shared_ptr<Request> req;
  uint32_t slot = 0;
  uint64_t off = 0;
  void* d_delta = nullptr;
  void* d_accept = nullptr;
  void* d_out = nullptr;
  void* d_sig = nullptr;
  std::vector<std::pair<void*, size_t>> closure_bufs;  // closure level storage
  size_t sz_delta = 0, sz_accept = 0, sz_out = 0, sz_sig = 0;
  std::vector<uint32_t> nonid;
  std::vector<uint64_t> rows;
  uint32_t rounds = 0;
  uint32_t levels = 0;
  bool closure = false;
  bool dead = false;
  // unary instances under AUTO refine by doubling (one closure level per
  // round); mj: the current partition is Moore's P_mj; step: this round's t
  bool dbl = false;
  uint64_t mj = 0, step = 1;
  // doubling levels computed in the round that first reads them (rows hold
  // pointers to all L level buffers; `built` of them are filled)
  bool lazy = false;
  uint32_t built = 0;
  uint32_t used = 0;  // the highest level a round that split a block read
  bool uploaded = false;  // inputs on the device (or on their way: see `up`)
  // in the resident set (joined): only then do its descriptor, states and
  // output take part in rounds and retirement; until then it only holds
  // its slot and buffers while its inputs upload
  bool joined = false;
  hipEvent_t up = nullptr;  // recorded behind the input upload
};

}  // namespace

struct Serving::Impl {
  explicit Impl(Context* c) : ctx(c) {}
  ~Impl() { shutdown(); }

  Context* ctx;
  // declared before the queue and the tickets: requests give their host
  // buffers back to it, so it must outlive them (they also hold a reference)
  std::shared_ptr<PinnedPool> pinned = std::make_shared<PinnedPool>(pinned_cap());
  static uint64_t pinned_cap() {
    // DFAMIN_SERVING_PINNED_BYTES overrides the cap (0: ordinary memory only)
    if (const char* e = std::getenv("DFAMIN_SERVING_PINNED_BYTES")) {
      char* end = nullptr;
      const unsigned long long v = std::strtoull(e, &end, 10);
      if (end != e) return v;
    }
    return kPinnedCap;
  }
  // worker-side totals (printed at shutdown with DFAMIN_TRACE)
  double t_join = 0, t_round = 0;
  uint64_t iters = 0, joined = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool started = false;
  std::thread worker;
  int init_rc = DFAMIN_OK;

  // ---- device state (worker thread only)
  hipStream_t stream = nullptr;
  // Inputs of admitted requests go to the device on their own stream while
  // the resident set's rounds run on `stream`; a request joins once the
  // event behind its upload has completed.
  hipStream_t ustream = nullptr;
  std::vector<Resident*> staged;  // admitted, inputs on their way (in admission order)
  std::vector<hipEvent_t> free_events;
  uint64_t cap = 0;  // state arena capacity
  DevicePool pool;
  RangeAlloc arena;
  std::vector<Resident*> slots;
  std::vector<InstDesc> desc;
  std::vector<uint64_t> rows_host;
  uint32_t m = 0;
  uint64_t salt = 0x9E3779B97F4A7C15ull;
  // fixed device buffers
  void *d_block = nullptr, *d_inst_of = nullptr, *d_act = nullptr, *d_act2 = nullptr;
  void *d_slot_of = nullptr, *d_nb = nullptr, *d_keep = nullptr, *d_rank = nullptr;
  void *d_status = nullptr, *d_table = nullptr, *d_desc = nullptr, *d_rows = nullptr;
  void *d_changed = nullptr, *d_last = nullptr, *d_refine = nullptr, *d_dead = nullptr;
  void *d_minF = nullptr, *d_minN = nullptr, *d_ctrl = nullptr, *d_results = nullptr;
  void *d_totals = nullptr;
  size_t rows_cap = 0;
  uint64_t table_cap = 0;
  // scratch that grows
  DevBuf s_jobs, s_off, s_flags, s_wg, s_part, s_slot, s_aux, s_fjobs;
  HostBuf h_flags, h_ctrl, h_results, h_fres;  // h_ctrl: a Ctrl, then the per-slot flags of d_last
  std::vector<char> job_stage;                 // host side of upload_jobs
  std::vector<uint32_t> join_list;             // host side of a join's job list
  struct FusedBatch {
    std::vector<Resident*> fs;
    std::vector<uint32_t> pos;   // per entry of fs: index in jobs (class order)
    std::vector<FusedJob> jobs;  // host side of the job list
    bool live = false;           // in flight on fstream
  } fb;
  std::vector<Resident*> fpend;  // small requests waiting for the next batch
  hipStream_t fstream = nullptr;
  hipEvent_t fev = nullptr;
  uint32_t* h_last() { return reinterpret_cast<uint32_t*>(static_cast<char*>(h_ctrl.p) + sizeof(Ctrl)); }

  void shutdown() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv_work.notify_all();
    if (worker.joinable()) worker.join();
    // a fused batch may still be copying outputs into requests' buffers:
    // let it finish before their waiters wake
    if (fstream) (void)hipStreamSynchronize(fstream);
    if (std::getenv("DFAMIN_TRACE"))
      std::fprintf(stderr, "[dfamin] serving: %llu iterations, %llu joined; join %.0f us, rounds %.0f us\n",
                   (unsigned long long)iters, (unsigned long long)joined, t_join, t_round);
    {
      std::lock_guard<std::mutex> g(mu);
      for (auto& r : queue) { r->status = DFAMIN_E_CANCELLED; }
      queue.clear();
      for (auto& kv : tickets)
        if (kv.second->status == 1) kv.second->status = DFAMIN_E_CANCELLED;
    }
    cv_done.notify_all();
    free_device();
  }

  // ------------------------------------------------------------ memory
  void* dmalloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 64) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  bool grow(DevBuf& b, size_t bytes) {
    if (b.cap >= bytes) return true;
    if (b.p) (void)hipFree(b.p);
    size_t want = (bytes + bytes / 4 + 4095) & ~size_t(4095);
    b.p = dmalloc(want);
    b.cap = b.p ? want : 0;
    return b.p != nullptr;
  }
  // Page-locked, coherent and mapped: kernels may write results straight
  // into it (b.dp), with no device cache holding them back.
  bool grow_host(HostBuf& b, size_t bytes) {
    if (b.cap >= bytes) return true;
    if (b.p) (void)hipHostFree(b.p);
    b.p = b.dp = nullptr;
    b.cap = 0;
    size_t want = bytes + bytes / 4 + 64;
    if (hipHostMalloc(&b.p, want, hipHostMallocCoherent) != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();
      return false;
    }
    if (hipHostGetDevicePointer(&b.dp, b.p, 0) != hipSuccess || !b.dp) {
      (void)hipHostFree(b.p);
      b.p = b.dp = nullptr;
      (void)hipGetLastError();
      return false;
    }
    b.cap = want;
    return true;
  }

  // A job list and its workgroup offsets in one upload into s_jobs; the
  // offsets follow the jobs (returned in *off).
  int upload_jobs(const std::vector<RowJob>& jobs, const std::vector<uint32_t>& joboff, uint32_t** off) {
    const size_t jb = jobs.size() * sizeof(RowJob), ob = joboff.size() * 4;
    if (!grow(s_jobs, jb + ob)) return DFAMIN_E_NOMEM;
    job_stage.resize(jb + ob);
    std::memcpy(job_stage.data(), jobs.data(), jb);
    std::memcpy(job_stage.data() + jb, joboff.data(), ob);
    if (hipMemcpyAsync(s_jobs.p, job_stage.data(), jb + ob, hipMemcpyHostToDevice, stream) != hipSuccess)
      return DFAMIN_E_DEVICE;
    *off = reinterpret_cast<uint32_t*>(static_cast<char*>(s_jobs.p) + jb);
    return DFAMIN_OK;
  }
  void free_device() {
    if (ustream) (void)hipStreamSynchronize(ustream);  // uploads still reading host staging
    if (fstream) (void)hipStreamSynchronize(fstream);  // a fused batch still running
    staged.clear();
    fpend.clear();
    fb.fs.clear();
    fb.live = false;
    for (Resident* r : slots)
      if (r) release_resident(r);
    slots.clear();
    void** ps[] = {&d_block, &d_inst_of, &d_act, &d_act2, &d_slot_of, &d_nb, &d_keep, &d_rank,
                   &d_status, &d_table, &d_desc, &d_rows, &d_changed, &d_refine, &d_dead,
                   &d_minF, &d_minN, &d_ctrl, &d_results, &d_totals};
    for (void** p : ps)
      if (*p) { (void)hipFree(*p); *p = nullptr; }
    d_last = nullptr;  // part of d_ctrl's allocation
    DevBuf* db[] = {&s_jobs, &s_off, &s_flags, &s_wg, &s_part, &s_slot, &s_aux, &s_fjobs};
    for (DevBuf* b : db)
      if (b->p) { (void)hipFree(b->p); b->p = nullptr; b->cap = 0; }
    HostBuf* hb[] = {&h_flags, &h_ctrl, &h_results, &h_fres};
    for (HostBuf* b : hb)
      if (b->p) { (void)hipHostFree(b->p); b->p = nullptr; b->cap = 0; }
    pool.release_all();
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    free_events.clear();
    if (stream) { (void)hipStreamDestroy(stream); stream = nullptr; }
    if (ustream) { (void)hipStreamDestroy(ustream); ustream = nullptr; }
    if (fstream) { (void)hipStreamDestroy(fstream); fstream = nullptr; }
    if (fev) { (void)hipEventDestroy(fev); fev = nullptr; }
  }

  int init_device() {
    if (hipSetDevice(ctx->device) != hipSuccess) return DFAMIN_E_DEVICE;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return DFAMIN_E_DEVICE;
    if (hipStreamCreateWithFlags(&ustream, hipStreamNonBlocking) != hipSuccess) return DFAMIN_E_DEVICE;
    if (hipStreamCreateWithFlags(&fstream, hipStreamNonBlocking) != hipSuccess) return DFAMIN_E_DEVICE;
    if (hipEventCreateWithFlags(&fev, hipEventDisableTiming) != hipSuccess) return DFAMIN_E_DEVICE;
    // arena sized from the budget: ~37 bytes per state of fixed buffers,
    // 16 per state of hash table, the rest for request buffers
    cap = kDefaultArenaStates;
    if (const char* e = std::getenv("DFAMIN_SERVING_STATES")) {
      const unsigned long long v = std::strtoull(e, nullptr, 10);
      if (v >= 1024 && v < (1ull << 31)) cap = v;
    }
    while (cap > (1u << 16) && cap * 64 > ctx->budget / 2) cap >>= 1;
    const uint64_t fixed = cap * 53;
    pool.set_budget(ctx->budget > fixed ? ctx->budget - fixed : 0);
    d_block = dmalloc(cap * 4); d_inst_of = dmalloc(cap * 4);
    d_act = dmalloc(cap * 4); d_act2 = dmalloc(cap * 4);
    d_slot_of = dmalloc(cap * 4); d_nb = dmalloc(cap * 4);
    d_keep = dmalloc(cap); d_rank = dmalloc(cap * 4 + 4);
    d_status = dmalloc(((size_t)scan_tiles(cap, kScanItemsSmall) + kSlots + 1) * 8);
    table_cap = 1ull << std::max<uint32_t>(9, ceil_log2_u64(2 * cap));
    d_table = dmalloc(table_cap * sizeof(Slot));
    d_desc = dmalloc(kSlots * sizeof(InstDesc));
    d_changed = dmalloc(kSlots * 4);
    d_refine = dmalloc(kSlots * 4); d_dead = dmalloc(kSlots * 4);
    d_minF = dmalloc(kSlots * 4); d_minN = dmalloc(kSlots * 4);
    // the round's control words and per-slot "still refining" flags sit
    // together, so one copy reads both back
    d_ctrl = dmalloc(sizeof(Ctrl) + kSlots * 4); d_results = dmalloc(kSlots * sizeof(ResultDev));
    d_totals = dmalloc(kSlots * 4);
    void* all[] = {d_block, d_inst_of, d_act, d_act2, d_slot_of, d_nb, d_keep, d_rank, d_status,
                   d_table, d_desc, d_changed, d_refine, d_dead, d_minF, d_minN, d_ctrl,
                   d_results, d_totals};
    for (void* p : all)
      if (!p) return DFAMIN_E_NOMEM;
    d_last = static_cast<char*>(d_ctrl) + sizeof(Ctrl);
    if (hipMemsetAsync(d_changed, 0, kSlots * 4, stream) != hipSuccess ||
        hipMemsetAsync(d_refine, 0, kSlots * 4, stream) != hipSuccess ||
        hipMemsetAsync(d_dead, 0, kSlots * 4, stream) != hipSuccess ||
        hipMemsetAsync(d_ctrl, 0, sizeof(Ctrl), stream) != hipSuccess)
      return DFAMIN_E_DEVICE;
    if (!grow_host(h_ctrl, sizeof(Ctrl) + kSlots * 4) || !grow_host(h_results, kSlots * sizeof(ResultDev)))
      return DFAMIN_E_NOMEM;
    arena.reset(cap);
    slots.assign(kSlots, nullptr);
    desc.assign(kSlots, InstDesc{});
    return stream_wait(stream) == hipSuccess ? DFAMIN_OK : DFAMIN_E_DEVICE;
  }

  void release_resident(Resident* r) {
    if (r->up) free_events.push_back(r->up);
    pool.free(r->d_delta, r->sz_delta);
    pool.free(r->d_accept, r->sz_accept);
    pool.free(r->d_out, r->sz_out);
    pool.free(r->d_sig, r->sz_sig);
    for (auto& cb : r->closure_bufs) pool.free(cb.first, cb.second);
    arena.release(r->off, r->req->n);
    slots[r->slot] = nullptr;
    desc[r->slot] = InstDesc{};
    delete r;
  }

  // Device bytes a request needs besides the fixed per-state buffers.
  static size_t footprint(const Request& q) {
    const size_t n = q.n, k = q.k;
    size_t b = DevicePool::size_class(4 * n * k) + DevicePool::size_class((n + 7) / 8) +
               DevicePool::size_class(4 * n) + DevicePool::size_class(4 * n * (k + 1));
    if (q.opts.closure != DFAMIN_CLOSURE_OFF) {
      const size_t L = floor_log2_u32(q.n);
      b += DevicePool::size_class(4 * n * k * L) + DevicePool::size_class(4 * n * (k * (L + 1) + 1));
    }
    return b;
  }

  // ------------------------------------------------------------ worker
  void finish(const std::shared_ptr<Request>& r, int status) {
    {
      std::lock_guard<std::mutex> g(mu);
      r->status = status;
    }
    cv_done.notify_all();
  }

  // (re)upload descriptors and row pointers of every resident request
  // Level passes of the coming round (step 0: each resident's first missing
  // level, step 1 the next, ...), one launch per step, queued before it.
  struct LevelTodo {
    Resident* r;
    uint32_t level, step;
  };
  std::vector<LevelTodo> todo;
  int queue_levels() {
    uint32_t S = 0;
    for (const LevelTodo& t : todo) S = std::max(S, t.step + 1);
    std::vector<RowJob> jobs;
    std::vector<uint32_t> joboff, begin(S + 1, 0), wgs(S, 0);
    for (uint32_t st = 0; st < S; ++st) {
      begin[st] = (uint32_t)jobs.size();
      uint32_t w = 0;
      for (const LevelTodo& t : todo) {
        if (t.step != st) continue;
        RowJob J;
        J.src = t.r->rows[t.level - 1];
        J.dst = t.r->rows[t.level];
        J.n = t.r->req->n;
        J.flag_idx = (uint32_t)jobs.size();
        joboff.push_back(w);
        w += (J.n + kRowTile - 1) / kRowTile;
        jobs.push_back(J);
      }
      wgs[st] = w;
      }
    begin[S] = (uint32_t)jobs.size();
    todo.clear();
    uint32_t* d_off = nullptr;
    const int urc = upload_jobs(jobs, joboff, &d_off);
    if (urc != DFAMIN_OK) return urc;
    for (uint32_t st = 0; st < S; ++st)
      if (begin[st + 1] > begin[st])  // (levels read as built are not tested: no flags)
        launch_closure_level(s_jobs.as<RowJob>() + begin[st], d_off + begin[st],
                             begin[st + 1] - begin[st], wgs[st], nullptr, nullptr, stream);
    return hipGetLastError() == hipSuccess ? DFAMIN_OK : DFAMIN_E_DEVICE;
  }

  // Level storage for a unary AUTO resident, which then refines by doubling
  // from its first round (the same schedule as the batch path).  Returns
  // false, leaving the resident plain, when the pool has no room.
  bool plan_lazy_levels(Resident* r) {
    uint32_t L = floor_log2_u32(r->req->n);
    if (r->req->opts.max_levels && r->req->opts.max_levels < L) L = r->req->opts.max_levels;
    const size_t bytes = 4ull * L * r->req->n;
    char* base = nullptr;
    if (bytes) {
      if (pool.live() + bytes > pool.budget()) return false;
      base = static_cast<char*>(pool.alloc(bytes));
      if (!base) return false;
      r->closure_bufs.emplace_back(base, bytes);
    }
    std::vector<uint64_t> rows(1 + (size_t)L);
    rows[0] = reinterpret_cast<uint64_t>(r->d_delta) + 4ull * r->nonid[0] * r->req->n;
    for (uint32_t l = 1; l <= L; ++l) rows[l] = reinterpret_cast<uint64_t>(base + 4ull * (l - 1) * r->req->n);
    r->rows = std::move(rows);
    r->lazy = true;
    r->built = 0;
    r->levels = 0;
    r->closure = true;
    r->dbl = true;
    return true;
  }

  int upload_layout() {
    rows_host.clear();
    for (uint32_t s = 0; s < kSlots; ++s) {
      Resident* r = slots[s];
      if (!r || !r->joined) continue;
      desc[s].rows_off = (uint32_t)rows_host.size();
      desc[s].kp = (uint32_t)r->rows.size();
      if (r->dbl) {  // the single closure level 2^l <= mj + 1
        uint32_t lvl = 0;
        for (uint64_t x = r->mj + 1; x >> 1; x >>= 1) ++lvl;
        if (lvl > r->rows.size() - 1) lvl = (uint32_t)r->rows.size() - 1;
        r->step = 1ull << lvl;
        desc[s].rows_off += lvl;
        desc[s].kp = 1;
        if (r->lazy && r->built < lvl) {
          for (uint32_t l = r->built + 1; l <= lvl; ++l) todo.push_back({r, l, l - r->built - 1});
          r->built = lvl;
        }
      }
      rows_host.insert(rows_host.end(), r->rows.begin(), r->rows.end());
    }
    if (!todo.empty()) {
      const int rc = queue_levels();
      if (rc != DFAMIN_OK) return rc;
    }
    if (rows_host.size() * 8 > rows_cap) {
      if (d_rows) (void)hipFree(d_rows);
      rows_cap = (rows_host.size() * 8 * 2 + 4096);
      d_rows = dmalloc(rows_cap);
      if (!d_rows) return DFAMIN_E_NOMEM;
    }
    if (!rows_host.empty() &&
        hipMemcpyAsync(d_rows, rows_host.data(), rows_host.size() * 8, hipMemcpyHostToDevice, stream) !=
            hipSuccess)
      return DFAMIN_E_DEVICE;
    // slots are taken lowest first: the occupied ones lie below slot_hi()
    const uint32_t hi = slot_hi();
    if (hi && hipMemcpyAsync(d_desc, desc.data(), hi * sizeof(InstDesc), hipMemcpyHostToDevice, stream) !=
                  hipSuccess)
      return DFAMIN_E_DEVICE;
    return DFAMIN_OK;
  }

  // One past the highest occupied slot.
  uint32_t slot_hi() const {
    uint32_t hi = 0;
    for (uint32_t s = 0; s < (uint32_t)slots.size(); ++s)
      if (slots[s]) hi = s + 1;
    return hi;
  }

  ClosureScratch scratch() {
    ClosureScratch sc;
    sc.ensure = [this](int b, size_t bytes) -> void* {
      DevBuf* bufs[4] = {&s_jobs, &s_off, &s_flags, &s_wg};
      return grow(*bufs[b], bytes) ? bufs[b]->p : nullptr;
    };
    sc.host_flags = [this](size_t bytes) -> void* { return grow_host(h_flags, bytes) ? h_flags.p : nullptr; };
    return sc;
  }

  // Closure (Algorithm 5) for the given residents, one resident at a time so
  // that each one's level storage comes from the pool in its own pieces (and
  // goes back at retire); swaps their signature buffers for ones sized to the
  // new letter count.
  int build_closures(const std::vector<Resident*>& rs) {
    for (Resident* r : rs) {
      std::vector<ClosureSpec> specs(1);
      uint32_t L = floor_log2_u32(r->req->n);
      if (r->req->opts.max_levels && r->req->opts.max_levels < L) L = r->req->opts.max_levels;
      specs[0].n = r->req->n;
      specs[0].delta = static_cast<const uint32_t*>(r->d_delta);
      specs[0].letters = r->nonid;
      specs[0].L = L;
      ClosureScratch sc = scratch();
      sc.level_storage = [this, r](size_t bytes) -> void* {
        if (pool.live() + bytes > pool.budget()) return nullptr;
        void* p = pool.alloc(bytes);
        if (p) r->closure_bufs.emplace_back(p, bytes);
        return p;
      };
      std::vector<std::vector<uint64_t>> rows;
      std::vector<uint32_t> depth;
      int rc = build_closure_levels(specs, sc, stream, rows, depth);
      if (rc != DFAMIN_OK) return rc;
      // The signature records for the new letter count come first: where
      // the budget has no room for them, the resident keeps refining on its
      // plain letters (sound: any subset of closure letters is) and its
      // level storage goes back, instead of failing every request.
      const size_t sz = (size_t)r->req->n * (rows[0].size() + 1) * 4;
      void* sig = sz <= r->sz_sig ? r->d_sig : (pool.live() + sz <= pool.budget() ? pool.alloc(sz) : nullptr);
      if (!sig) {
        for (auto& cb : r->closure_bufs) pool.free(cb.first, cb.second);
        r->closure_bufs.clear();
        continue;
      }
      if (sig != r->d_sig) {
        pool.free(r->d_sig, r->sz_sig);
        r->d_sig = sig;
        r->sz_sig = sz;
      }
      r->rows = rows[0];
      r->levels = depth[0];
      r->closure = true;
      desc[r->slot].sig = reinterpret_cast<uint64_t>(r->d_sig);
    }
    return DFAMIN_OK;
  }

  // Inputs of newly admitted requests go to the device on the upload
  // stream, each followed by its event.
  int stage(const std::vector<Resident*>& rs) {
    for (Resident* r : rs) {
      if (free_events.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return DFAMIN_E_DEVICE;
        free_events.push_back(e);
      }
      r->up = free_events.back();
      free_events.pop_back();
      if (hipMemcpyAsync(r->d_delta, r->req->delta(), r->sz_delta, hipMemcpyHostToDevice, ustream) !=
              hipSuccess ||
          hipMemcpyAsync(r->d_accept, r->req->accept(), r->req->accept_bytes(), hipMemcpyHostToDevice,
                         ustream) != hipSuccess ||
          hipEventRecord(r->up, ustream) != hipSuccess)
        return DFAMIN_E_DEVICE;
      r->uploaded = true;
      staged.push_back(r);
    }
    return DFAMIN_OK;
  }

  // A request of up to kFusedMaxStates states (closure OFF or AUTO) is
  // minimized whole by one workgroup of the fused kernel as it joins: no
  // rounds of the resident set, and it is done when its inputs and output
  // have crossed.  The kernel hands back an instance that needs closure
  // letters; those join the resident set as any other request.
  static bool fusable(const Request& q) {
    return q.n <= kFusedMaxStates && q.k <= kFusedMaxLetters &&
           (q.opts.closure == DFAMIN_CLOSURE_AUTO || q.opts.closure == DFAMIN_CLOSURE_OFF) &&
           q.opts.method == DFAMIN_METHOD_SIGNATURE;
  }
  // Small requests run as batches of the fused kernel on a stream of their
  // own (fstream), one batch at a time, beside the resident set's rounds:
  // fpend collects them, launch_fused_batch issues a batch (kernels, their
  // outputs' copies back, an event), collect_fused publishes it once the
  // event has completed.  The batch's results land in h_fres (mapped host
  // memory) and its job list in s_fjobs, both held by the batch in flight.
  int launch_fused_batch() {
    fb.fs.swap(fpend);
    fpend.clear();
    const size_t F = fb.fs.size();
    std::vector<FusedJob>& jobs = fb.jobs;
    jobs.assign(F, FusedJob{});
    fb.pos.assign(F, 0);
    uint32_t at = 0, start[4] = {0, 0, 0, 0};
    for (int cls = 2; cls >= 0; --cls) {
      start[cls] = at;
      for (size_t w = 0; w < F; ++w) {
        Resident* r = fb.fs[w];
        const Request& q = *r->req;
        if (fused_class(q.n) != cls) continue;
        FusedJob& J = jobs[at];
        J.delta = reinterpret_cast<uint64_t>(r->d_delta);
        J.accept = reinterpret_cast<uint64_t>(r->d_accept);
        J.out = reinterpret_cast<uint64_t>(r->d_out);
        J.n = q.n;
        J.k = q.k;
        J.q0 = q.q0;
        J.closure = q.opts.closure;
        uint32_t L = floor_log2_u32(q.n);
        if (q.opts.max_levels && q.opts.max_levels < L) L = q.opts.max_levels;
        J.levels = L;
        J.auto_rounds = q.opts.auto_rounds ? q.opts.auto_rounds : kDefaultAutoRounds;
        J.max_rounds = q.opts.max_rounds ? q.opts.max_rounds : q.n + 1u;
        fb.pos[w] = at++;
      }
    }
    start[3] = at;
    if ((F > 1 && !grow(s_fjobs, F * sizeof(FusedJob))) || !grow_host(h_fres, F * sizeof(FusedRes)))
      return DFAMIN_E_NOMEM;
    for (Resident* r : fb.fs) {
      if (r->uploaded) continue;
      if (hipMemcpyAsync(r->d_delta, r->req->delta(), r->sz_delta, hipMemcpyHostToDevice, fstream) !=
              hipSuccess ||
          hipMemcpyAsync(r->d_accept, r->req->accept(), r->req->accept_bytes(), hipMemcpyHostToDevice,
                         fstream) != hipSuccess)
        return DFAMIN_E_DEVICE;
      r->uploaded = true;
    }
    // one job travels as a kernel argument
    FusedRes* res = static_cast<FusedRes*>(h_fres.dp);
    if (F == 1) {
      launch_fused(nullptr, res, 1, fused_class(jobs[0].n), fstream, &jobs[0]);
    } else {
      if (hipMemcpyAsync(s_fjobs.p, jobs.data(), F * sizeof(FusedJob), hipMemcpyHostToDevice, fstream) !=
          hipSuccess)
        return DFAMIN_E_DEVICE;
      for (int cls = 2; cls >= 0; --cls) {
        const uint32_t b = start[cls], e = cls == 0 ? start[3] : start[cls - 1];
        launch_fused(s_fjobs.as<FusedJob>() + b, res + b, e - b, cls, fstream);
      }
    }
    if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
    // every output comes back with the results (a bad or handed-back one is
    // simply not published)
    for (Resident* r : fb.fs) {
      if (!r->req->out.make(pinned, 4ull * r->req->n)) return DFAMIN_E_NOMEM;
      if (hipMemcpyAsync(r->req->out.data(), r->d_out, 4ull * r->req->n, hipMemcpyDeviceToHost, fstream) !=
          hipSuccess)
        return DFAMIN_E_DEVICE;
    }
    if (hipEventRecord(fev, fstream) != hipSuccess) return DFAMIN_E_DEVICE;
    fb.live = true;
    return DFAMIN_OK;
  }

  // Publish the batch in flight (its event has completed); requests the
  // kernel handed back go to handed_back, to join the resident set.
  int collect_fused(std::vector<Resident*>& handed_back) {
    const FusedRes* fr = h_fres.as<FusedRes>();
    for (size_t w = 0; w < fb.fs.size(); ++w) {
      Resident* r = fb.fs[w];
      const FusedRes& f = fr[fb.pos[w]];
      if (f.status == kFusedHandOff) {
        handed_back.push_back(r);
        continue;
      }
      auto req = r->req;
      int st = DFAMIN_OK;
      if (f.status == kFusedOk) {
        dfamin_result& o = req->result;
        o.num_blocks = f.num_blocks;
        o.initial_block = f.initial_block;
        o.refine_rounds = f.refine_rounds;
        o.rounds_executed = f.refine_rounds + 1;
        o.closure_levels = f.doubling ? f.levels_used : 0;
        o.closure_letters = f.doubling ? f.levels_used + 1 : 0;
        o.status = DFAMIN_OK;
      } else {
        st = f.status == kFusedBad ? DFAMIN_E_BAD_DFA : DFAMIN_E_INTERNAL;
      }
      req->in.release();
      if (st != DFAMIN_OK) req->out.release();
      const bool cancelled = req->cancelled;
      release_resident(r);
      finish(req, cancelled && st == DFAMIN_OK ? DFAMIN_E_CANCELLED : st);
    }
    fb.fs.clear();
    fb.live = false;
    return DFAMIN_OK;
  }

  // Bring newly admitted requests into the resident set.
  int join(std::vector<Resident*>& js) {
    // upload inputs
    for (Resident* r : js) {
      if (r->uploaded) continue;
      if (hipMemcpyAsync(r->d_delta, r->req->delta(), r->sz_delta, hipMemcpyHostToDevice, stream) !=
              hipSuccess ||
          hipMemcpyAsync(r->d_accept, r->req->accept(), r->req->accept_bytes(), hipMemcpyHostToDevice,
                         stream) != hipSuccess)
        return DFAMIN_E_DEVICE;
    }
    // validation and identity letters: one row job per (request, letter)
    std::vector<RowJob> jobs;
    std::vector<uint32_t> joboff;
    uint32_t wgs = 0;
    for (Resident* r : js)
      for (uint32_t a = 0; a < r->req->k; ++a) {
        RowJob J;
        J.src = reinterpret_cast<uint64_t>(r->d_delta) + 4ull * a * r->req->n;
        J.dst = 0;
        J.n = r->req->n;
        J.flag_idx = (uint32_t)jobs.size();
        joboff.push_back(wgs);
        wgs += (J.n + kLongTile - 1) / kLongTile;
        jobs.push_back(J);
      }
    if (!grow(s_wg, (size_t)wgs * 4) || !grow_host(h_flags, jobs.size() * 4)) return DFAMIN_E_NOMEM;
    uint32_t* d_off = nullptr;
    const int urc = upload_jobs(jobs, joboff, &d_off);
    if (urc != DFAMIN_OK) return urc;
    // the per-row flags go straight to the mapped host buffer
    launch_row_check(s_jobs.as<RowJob>(), d_off, (uint32_t)jobs.size(), wgs, s_wg.as<uint32_t>(),
                     static_cast<uint32_t*>(h_flags.dp), stream);
    if (hipGetLastError() != hipSuccess || stream_wait(stream) != hipSuccess) return DFAMIN_E_DEVICE;
    for (Resident* r : js) r->req->in.release();  // the inputs are on the device now
    const uint32_t* f = h_flags.as<uint32_t>();
    std::vector<Resident*> ok, need_closure;
    size_t j = 0;
    for (Resident* r : js) {
      bool bad = false;
      r->nonid.clear();
      for (uint32_t a = 0; a < r->req->k; ++a, ++j) {
        if (f[j] & kFlagBad) bad = true;
        if (f[j] & kFlagNonId) r->nonid.push_back(a);
      }
      if (bad) {
        auto req = r->req;
        release_resident(r);
        finish(req, DFAMIN_E_BAD_DFA);
        continue;
      }
      r->rows.clear();
      for (uint32_t a : r->nonid)
        r->rows.push_back(reinterpret_cast<uint64_t>(r->d_delta) + 4ull * a * r->req->n);
      InstDesc& D = desc[r->slot];
      D = InstDesc{};
      D.state_off = (uint32_t)r->off;
      D.n = r->req->n;
      D.k = r->req->k;
      D.q0 = r->req->q0;
      D.accept = reinterpret_cast<uint64_t>(r->d_accept);
      D.out = reinterpret_cast<uint64_t>(r->d_out);
      D.sig = reinterpret_cast<uint64_t>(r->d_sig);
      r->joined = true;  // its descriptor is set: layout and rounds include it from here
      ok.push_back(r);
      if (r->req->opts.closure == DFAMIN_CLOSURE_ON) need_closure.push_back(r);
      if (r->req->opts.closure == DFAMIN_CLOSURE_AUTO && r->nonid.size() == 1) (void)plan_lazy_levels(r);
    }
    js = ok;
    if (js.empty()) return DFAMIN_OK;
    if (!need_closure.empty()) {
      int rc = build_closures(need_closure);
      if (rc != DFAMIN_OK) return rc;
    }
    // first round of each newcomer groups on exact keys from accept bits
    for (Resident* r : js) {
      desc[r->slot].ebits = (r->rows.size() + 1 <= 31) ? 1u : 0u;
      desc[r->slot].dsrc = 1u;
    }
    int rc = upload_layout();
    if (rc != DFAMIN_OK) return rc;
    // reset per-slot counters and build the initial partition
    const size_t nj = js.size();
    std::vector<uint32_t>& jl = join_list;  // slot ids, workgroup offsets, act offsets
    jl.resize(3 * nj);
    uint32_t iw = 0, am = m;
    for (size_t j = 0; j < nj; ++j) {
      jl[j] = js[j]->slot;
      jl[nj + j] = iw;
      jl[2 * nj + j] = am;
      iw += (js[j]->req->n + kRowTile - 1) / kRowTile;
      am += js[j]->req->n;
    }
    if (!grow(s_slot, nj * 4 * 3) || !grow(s_part, (size_t)iw * 8)) return DFAMIN_E_NOMEM;
    uint32_t* d_sl = s_slot.as<uint32_t>();
    if (hipMemcpyAsync(d_sl, jl.data(), nj * 4 * 3, hipMemcpyHostToDevice, stream) != hipSuccess)
      return DFAMIN_E_DEVICE;
    launch_init_minmax_slots(static_cast<InstDesc*>(d_desc), d_sl, d_sl + nj, (uint32_t)nj, iw,
                             s_part.as<unsigned long long>(), static_cast<uint32_t*>(d_minF),
                             static_cast<uint32_t*>(d_minN), stream);
    launch_init_join(static_cast<InstDesc*>(d_desc), d_sl, d_sl + nj, (uint32_t)nj, iw, d_sl + 2 * nj,
                     static_cast<uint32_t*>(d_minF), static_cast<uint32_t*>(d_minN),
                     static_cast<uint32_t*>(d_inst_of), static_cast<uint32_t*>(d_block),
                     static_cast<uint32_t*>(d_act), static_cast<uint32_t*>(d_changed),
                     static_cast<uint32_t*>(d_refine), static_cast<uint32_t*>(d_dead), stream);
    if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
    // no wait: the copies' host sources are members that live until the
    // next join, and everything after this runs behind it on the stream
    m = am;
    return DFAMIN_OK;
  }

  // Canonical numbering and copy-out for retiring residents.
  int retire(const std::vector<Resident*>& rs) {
    std::vector<Resident*> live;
    for (Resident* r : rs)
      if (!r->dead) live.push_back(r);
    if (!live.empty()) {
      const size_t nj = live.size();
      std::vector<uint32_t> jl(3 * nj);  // slot ids, scan tile offsets, workgroup offsets
      uint32_t tiles = 0, wgs = 0;
      uint64_t states = 0;
      for (Resident* r : live) states += r->req->n;
      const int items = scan_items_for(states);
      for (size_t j = 0; j < nj; ++j) {
        jl[j] = live[j]->slot;
        jl[nj + j] = tiles;
        jl[2 * nj + j] = wgs;
        tiles += scan_tiles(live[j]->req->n, items);
        wgs += (live[j]->req->n + kRowTile - 1) / kRowTile;
      }
      if (!grow(s_aux, nj * 4 * 3)) return DFAMIN_E_NOMEM;
      uint32_t* d_sl = s_aux.as<uint32_t>();
      if (hipMemcpyAsync(d_sl, jl.data(), nj * 4 * 3, hipMemcpyHostToDevice, stream) != hipSuccess)
        return DFAMIN_E_DEVICE;
      launch_prep_scan(static_cast<unsigned long long*>(d_status), tiles, static_cast<Ctrl*>(d_ctrl), stream);
      launch_scan_jobs(static_cast<InstDesc*>(d_desc), d_sl, d_sl + nj, (uint32_t)nj, tiles,
                       static_cast<uint32_t*>(d_block), static_cast<uint32_t*>(d_rank),
                       static_cast<uint32_t*>(d_totals), static_cast<Ctrl*>(d_ctrl),
                       static_cast<unsigned long long*>(d_status), items, stream);
      launch_emit_jobs(static_cast<InstDesc*>(d_desc), d_sl, d_sl + 2 * nj, (uint32_t)nj, wgs,
                       static_cast<uint32_t*>(d_block), static_cast<uint32_t*>(d_rank), stream);
      launch_results_jobs(static_cast<InstDesc*>(d_desc), d_sl, (uint32_t)nj,
                          static_cast<uint32_t*>(d_totals), static_cast<uint32_t*>(d_refine),
                          static_cast<ResultDev*>(d_results), stream);
      if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
      for (Resident* r : live) {
        if (!r->req->out.make(pinned, 4ull * r->req->n)) return DFAMIN_E_NOMEM;
        if (hipMemcpyAsync(r->req->out.data(), r->d_out, 4ull * r->req->n, hipMemcpyDeviceToHost, stream) !=
            hipSuccess)
          return DFAMIN_E_DEVICE;
      }
      if (hipMemcpyAsync(h_results.p, d_results, nj * sizeof(ResultDev), hipMemcpyDeviceToHost, stream) !=
              hipSuccess ||
          hipMemcpyAsync(h_ctrl.p, d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream) != hipSuccess ||
          stream_wait(stream) != hipSuccess)
        return DFAMIN_E_DEVICE;
      if (h_ctrl.as<Ctrl>()->fault) return DFAMIN_E_INTERNAL;
      const ResultDev* res = h_results.as<ResultDev>();
      for (size_t w = 0; w < nj; ++w) {
        Resident* r = live[w];
        dfamin_result& o = r->req->result;
        o.num_blocks = res[w].num_blocks;
        o.initial_block = res[w].initial_block;
        o.refine_rounds = res[w].refine_rounds;
        o.rounds_executed = res[w].refine_rounds + 1;
        o.closure_levels = !r->closure ? 0 : (r->lazy ? r->used : r->levels);
        o.closure_letters = !r->closure ? 0 : (r->lazy ? r->used + 1 : (uint32_t)r->rows.size());
        o.status = DFAMIN_OK;
      }
    }
    for (Resident* r : rs) {
      auto req = r->req;
      const bool dead = r->dead;
      release_resident(r);
      finish(req, dead ? DFAMIN_E_CANCELLED : DFAMIN_OK);
    }
    return DFAMIN_OK;
  }

  // One refinement round over every resident request.
  int round() {
    // cancellations take effect in this round's compaction
    bool dirty = false;
    for (uint32_t s = 0; s < kSlots; ++s) {
      Resident* r = slots[s];
      if (r && r->joined && !r->dead && r->req->cancelled) {
        r->dead = true;
        const uint32_t one = 1;
        if (hipMemcpyAsync(static_cast<uint32_t*>(d_dead) + s, &one, 4, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            stream_wait(stream) != hipSuccess)
          return DFAMIN_E_DEVICE;
        dirty = true;
      }
    }
    (void)dirty;
    if (m > 0) {
      int retries = 0;
      while (true) {
        const uint32_t tbits = std::max<uint32_t>(9, ceil_log2_u64(2ull * m));
        const uint64_t tsize = 1ull << tbits;
        if (tsize > table_cap) return DFAMIN_E_INTERNAL;
        const int citems = scan_items_for(m);
        const uint32_t ntiles = scan_tiles(m, citems);
        uint32_t* act = static_cast<uint32_t*>(d_act);
        uint32_t* nxt = static_cast<uint32_t*>(d_act2);
        launch_clear_table(static_cast<Slot*>(d_table), tsize, static_cast<Ctrl*>(d_ctrl), stream);
        launch_signature(true, act, m, static_cast<uint32_t*>(d_inst_of), static_cast<InstDesc*>(d_desc),
                         static_cast<uint64_t*>(d_rows), static_cast<uint32_t*>(d_block), nullptr, 4,
                         static_cast<Slot*>(d_table), tbits, static_cast<uint32_t*>(d_slot_of), salt,
                         static_cast<Ctrl*>(d_ctrl), kSigDefaultVariant, stream,
                         2 /* hash-mode groups claim their slot by CAS first */);
        launch_resolve(true, act, m, static_cast<uint32_t*>(d_inst_of), static_cast<InstDesc*>(d_desc),
                       static_cast<Slot*>(d_table), static_cast<uint32_t*>(d_slot_of),
                       static_cast<uint32_t*>(d_block), static_cast<uint32_t*>(d_nb),
                       static_cast<uint8_t*>(d_keep), static_cast<uint32_t*>(d_changed),
                       static_cast<Ctrl*>(d_ctrl), static_cast<unsigned long long*>(d_status), ntiles, stream);
        launch_compact(true, act, m, static_cast<uint32_t*>(d_inst_of), static_cast<uint32_t*>(d_nb),
                       static_cast<uint8_t*>(d_keep), static_cast<uint32_t*>(d_changed),
                       static_cast<uint32_t*>(d_dead), static_cast<uint32_t*>(d_block), nxt,
                       static_cast<Ctrl*>(d_ctrl), static_cast<unsigned long long*>(d_status), citems, stream);
        launch_round_end(kSlots, static_cast<uint32_t*>(d_changed), static_cast<uint32_t*>(d_refine),
                         static_cast<uint32_t*>(d_last), static_cast<Ctrl*>(d_ctrl), stream);
        if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
        if (hipMemcpyAsync(h_ctrl.p, d_ctrl, sizeof(Ctrl) + 4ull * slot_hi(), hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            stream_wait(stream) != hipSuccess)
          return DFAMIN_E_DEVICE;
        const Ctrl c = *h_ctrl.as<Ctrl>();
        if (c.fault) return DFAMIN_E_INTERNAL;
        if (c.collision) {
          if (++retries > 8) return DFAMIN_E_INTERNAL;
          salt = mix64(salt + 0x9E3779B97F4A7C15ull);
          continue;
        }
        std::swap(d_act, d_act2);
        m = c.m_next;
        break;
      }
    } else {
      std::memset(h_last(), 0, kSlots * 4);
    }
    // who is done, who needs the closure, whose next round hashes
    const uint32_t* last = h_last();
    std::vector<Resident*> done, auto_closure;
    bool desc_dirty = false;
    for (uint32_t s = 0; s < kSlots; ++s) {
      Resident* r = slots[s];
      if (!r || !r->joined) continue;  // admitted, inputs still uploading
      r->rounds += 1;
      if (!last[s] || r->dead) {
        done.push_back(r);
        continue;
      }
      if (r->dbl) r->used = std::max<uint32_t>(r->used, (uint32_t)__builtin_ctzll(r->step));
      r->mj += r->dbl ? r->step : 1;
      if (r->dbl) desc_dirty = true;  // next level
      if (desc[s].dsrc) {  // accept bits only describe the first round's partition
        desc[s].ebits = 0;
        desc[s].dsrc = 0;
        desc_dirty = true;
      }
      const uint32_t ar = r->req->opts.auto_rounds ? r->req->opts.auto_rounds : kDefaultAutoRounds;
      if (r->req->opts.closure == DFAMIN_CLOSURE_AUTO && !r->closure && r->rounds == ar)
        auto_closure.push_back(r);
    }
    if (!auto_closure.empty()) {
      int rc = build_closures(auto_closure);
      if (rc != DFAMIN_OK) return rc;
      // (one that kept its plain letters for want of room refines plainly)
      for (Resident* r : auto_closure) r->dbl = r->closure && r->nonid.size() == 1;
      desc_dirty = true;
    }
    if (desc_dirty) {
      int rc = upload_layout();
      if (rc != DFAMIN_OK) return rc;
    }
    if (!done.empty()) return retire(done);
    return DFAMIN_OK;
  }

  // a slot held (joined or still uploading)
  bool any_resident() const {
    for (Resident* r : slots)
      if (r) return true;
    return false;
  }
  bool any_joined() const {
    for (Resident* r : slots)
      if (r && r->joined) return true;
    return false;
  }

  void fail_all(int rc) {
    if (ustream) (void)hipStreamSynchronize(ustream);  // uploads still reading host staging
    if (fstream) (void)hipStreamSynchronize(fstream);  // a fused batch still running
    staged.clear();
    fpend.clear();
    fb.fs.clear();
    fb.live = false;
    std::vector<std::shared_ptr<Request>> rs;
    {
      std::lock_guard<std::mutex> g(mu);
      for (auto& r : queue) rs.push_back(r);
      queue.clear();
    }
    for (Resident* r : slots)
      if (r) rs.push_back(r->req);
    for (Resident* r : slots)
      if (r) release_resident(r);
    for (auto& r : rs) finish(r, rc);
  }

  void run() {
    init_rc = init_device();
    if (init_rc != DFAMIN_OK) {
      fail_all(init_rc);
      std::unique_lock<std::mutex> lk(mu);
      while (!stop) {
        for (auto& r : queue) r->status = init_rc;
        queue.clear();
        cv_done.notify_all();
        cv_work.wait(lk);
      }
      return;
    }
    std::vector<Resident*> admitted;
    while (true) {
      std::vector<Resident*> joining;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !queue.empty() || any_resident() || !staged.empty(); });
        if (stop) break;
        // admission by footprint, first come first served
        while (!queue.empty()) {
          std::shared_ptr<Request> q = queue.front();
          if (q->cancelled) {
            queue.pop_front();
            q->status = DFAMIN_E_CANCELLED;
            cv_done.notify_all();
            continue;
          }
          uint32_t slot = kSlots;
          for (uint32_t s = 0; s < kSlots; ++s)
            if (!slots[s]) { slot = s; break; }
          uint64_t off = 0;
          const size_t fp = footprint(*q);
          const bool fits = slot < kSlots && pool.live() + fp <= pool.budget() && arena.alloc(q->n, &off);
          if (!fits) {
            if (!any_resident() && admitted.empty() && staged.empty()) {
              // can never fit: reject instead of waiting forever
              queue.pop_front();
              q->status = DFAMIN_E_NOMEM;
              cv_done.notify_all();
              continue;
            }
            break;
          }
          Resident* r = new Resident;
          r->req = q;
          r->slot = slot;
          r->off = off;
          r->sz_delta = 4ull * q->n * q->k;
          r->sz_accept = (q->n + 7) / 8;
          r->sz_out = 4ull * q->n;
          r->sz_sig = 4ull * q->n * (q->k + 1);
          r->d_delta = pool.alloc(r->sz_delta);
          r->d_accept = pool.alloc(r->sz_accept);
          r->d_out = pool.alloc(r->sz_out);
          r->d_sig = pool.alloc(r->sz_sig);
          slots[slot] = r;
          if (!r->d_delta || !r->d_accept || !r->d_out || !r->d_sig) {
            release_resident(r);
            if (!any_resident() && admitted.empty() && staged.empty()) {
              queue.pop_front();
              q->status = DFAMIN_E_NOMEM;
              cv_done.notify_all();
              continue;
            }
            break;
          }
          queue.pop_front();
          admitted.push_back(r);
        }
      }
      int rc = stage(admitted);
      admitted.clear();
      // requests whose inputs are on the device join, in admission order;
      // with nothing else to run, wait for the oldest upload
      if (rc == DFAMIN_OK && !staged.empty()) {
        if (!any_joined() && hipEventSynchronize(staged.front()->up) != hipSuccess) rc = DFAMIN_E_DEVICE;
        size_t take = 0;
        while (rc == DFAMIN_OK && take < staged.size()) {
          const hipError_t e = hipEventQuery(staged[take]->up);
          if (e == hipErrorNotReady) break;
          if (e != hipSuccess) rc = DFAMIN_E_DEVICE;
          ++take;
        }
        if (rc == DFAMIN_OK) {
          joining.assign(staged.begin(), staged.begin() + take);
          staged.erase(staged.begin(), staged.begin() + take);
        }
      }
      const auto t0 = std::chrono::steady_clock::now();
      if (!joining.empty()) {
        std::vector<Resident*> rest;
        for (Resident* r : joining) (fusable(*r->req) ? fpend : rest).push_back(r);
        joining.swap(rest);
      }
      if (rc == DFAMIN_OK && fb.live) {
        // with nothing else to run, wait for the batch in flight
        const bool idle = !any_joined() && joining.empty() && staged.empty();
        const hipError_t e = idle ? hipEventSynchronize(fev) : hipEventQuery(fev);
        if (e == hipSuccess) rc = collect_fused(joining);
        else if (e != hipErrorNotReady) rc = DFAMIN_E_DEVICE;
      }
      if (rc == DFAMIN_OK && !fb.live && !fpend.empty()) rc = launch_fused_batch();
      if (rc == DFAMIN_OK && !joining.empty()) rc = join(joining);
      const auto t1 = std::chrono::steady_clock::now();
      if (rc == DFAMIN_OK && any_joined()) rc = round();
      const auto t2 = std::chrono::steady_clock::now();
      t_join += std::chrono::duration<double, std::micro>(t1 - t0).count();
      t_round += std::chrono::duration<double, std::micro>(t2 - t1).count();
      iters += 1;
      joined += joining.size();
      if (rc != DFAMIN_OK) {
        fail_all(rc);
        m = 0;
        arena.reset(cap);
        if (rc == DFAMIN_E_DEVICE) {
          ctx->device_lost = true;
          std::unique_lock<std::mutex> lk(mu);
          while (!stop) {
            for (auto& r : queue) r->status = rc;
            queue.clear();
            cv_done.notify_all();
            cv_work.wait(lk);
          }
          return;
        }
      }
    }
  }
};

Serving::Serving(Context* ctx) : impl_(new Impl(ctx)) {}

Serving::~Serving() { delete impl_; }

int Serving::submit(const dfamin_dfa& dfa, const dfamin_opts& opts, uint64_t* ticket) {
  auto r = std::make_shared<Request>();
  r->n = dfa.n;
  r->k = dfa.k;
  r->q0 = dfa.q0;
  r->opts = opts;
  if (!r->in.make(impl_->pinned, r->delta_bytes() + r->accept_bytes())) return DFAMIN_E_NOMEM;
  std::memcpy(r->in.data(), dfa.delta, r->delta_bytes());
  std::memcpy(static_cast<char*>(r->in.data()) + r->delta_bytes(), dfa.accept, r->accept_bytes());
  {
    std::lock_guard<std::mutex> g(impl_->mu);
    if (impl_->stop) return DFAMIN_E_CANCELLED;
    if (impl_->queue.size() >= kMaxQueue) return DFAMIN_E_BUSY;
    r->ticket = impl_->next_ticket++;
    impl_->tickets[r->ticket] = r;
    impl_->queue.push_back(r);
    if (!impl_->started) {
      impl_->started = true;
      impl_->worker = std::thread([this] { impl_->run(); });
    }
  }
  impl_->cv_work.notify_all();
  *ticket = r->ticket;
  return DFAMIN_OK;
}

int Serving::wait(uint64_t ticket, int64_t timeout_us, uint32_t* out, dfamin_result* result) {
  std::unique_lock<std::mutex> lk(impl_->mu);
  auto it = impl_->tickets.find(ticket);
  if (it == impl_->tickets.end()) return DFAMIN_E_INVAL;
  std::shared_ptr<Request> r = it->second;
  auto done = [&] { return r->status != 1; };
  if (timeout_us < 0) {
    impl_->cv_done.wait(lk, done);
  } else if (!impl_->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    return DFAMIN_E_TIMEOUT;
  }
  const int st = r->status;
  impl_->tickets.erase(it);
  lk.unlock();  // the request is ours now: copy out without holding the lock
  if (st == DFAMIN_OK) {
    std::memcpy(out, r->out.data(), 4ull * r->n);
    if (result) *result = r->result;
  } else if (result) {
    std::memset(result, 0, sizeof(*result));
    result->status = st;
  }
  r->out.release();
  return st;
}

int Serving::cancel(uint64_t ticket) {
  {
    std::lock_guard<std::mutex> g(impl_->mu);
    auto it = impl_->tickets.find(ticket);
    if (it == impl_->tickets.end()) return DFAMIN_E_INVAL;
    it->second->cancelled = true;
  }
  impl_->cv_work.notify_all();
  return DFAMIN_OK;
}

}  // namespace dfamin
