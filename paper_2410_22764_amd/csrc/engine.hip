// engine.hip -- host driver of one minimization call (single or batched).
//
// Order of work (each step cites the paper passage it implements):
//   1. validate delta and find identity letters (one pass over delta);
//   2. signature letters: the non-identity letters of Sigma, or the levels of
//      Sigma^T (Section 3.4, Algorithm 5) when the closure is on; an identity
//      letter or a level equal to the previous one adds a component already
//      in every signature, so dropping it leaves every round's partition as
//      it is;
//   3. initial partition {F, Q\F} (Algorithm 4 initialisation);
//   4. rounds until no instance splits a block (Algorithm 4 loop);
//   5. canonical numbering by least member and emission.
#include "engine.h"

#include "closure.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>

namespace dfamin {

namespace {

inline uint32_t floor_log2_u64(uint64_t x) {
  uint32_t l = 0;
  while (x >> 1) { x >>= 1; ++l; }
  return l;
}

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

constexpr uint32_t kDefaultAutoRounds = 8;
constexpr uint64_t kClearAheadSlots = 1ull << 22;  // 32 MiB: a few microseconds to clear
constexpr uint32_t kQueueRounds = 8;               // queued signature rounds per graph (even)

}  // namespace

// ------------------------------------------------------------------ Profiler
Profiler::~Profiler() {
  for (auto& p : pending_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : free_events_) (void)hipEventDestroy(e);
}

void Profiler::set_enabled(bool on) {
  on_ = on;
  const char* t = std::getenv("DFAMIN_TRACE");
  trace_ = t && *t && *t != '0';
  if (on) stats_.clear();
}

int Profiler::stat_index(const char* name) {
  for (size_t i = 0; i < stats_.size(); ++i)
    if (!std::strncmp(stats_[i].name, name, sizeof(stats_[i].name))) return (int)i;
  dfamin_kernel_stat st{};
  std::strncpy(st.name, name, sizeof(st.name) - 1);
  stats_.push_back(st);
  return (int)stats_.size() - 1;
}

hipEvent_t Profiler::get_event() {
  if (!free_events_.empty()) {
    hipEvent_t e = free_events_.back();
    free_events_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(hipStream_t s, const char* name, double alg_bytes) {
  if (!on_) return;
  cur_.stat = stat_index(name);
  cur_.bytes = alg_bytes;
  stats_[cur_.stat].alg_bytes += alg_bytes;
  stats_[cur_.stat].launches += 1;
  cur_.a = get_event();
  cur_.b = get_event();
  if (cur_.a) (void)hipEventRecord(cur_.a, s);
}

void Profiler::end(hipStream_t s) {
  if (!on_) return;
  if (cur_.b) (void)hipEventRecord(cur_.b, s);
  pending_.push_back(cur_);
}

void Profiler::collect() {
  for (auto& p : pending_) {
    float ms = 0.f;
    if (p.a && p.b && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) stats_[p.stat].total_ms += ms;
    if (trace_)
      std::fprintf(stderr, "[dfamin] %-14s %9.1f us %8.1f GB/s\n", stats_[p.stat].name, 1e3 * ms,
                   ms > 0 ? p.bytes / (ms * 1e-3) / 1e9 : 0.0);
    if (p.a) free_events_.push_back(p.a);
    if (p.b) free_events_.push_back(p.b);
  }
  pending_.clear();
}

int Profiler::copy_stats(dfamin_kernel_stat* out, int cap) const {
  int n = (int)stats_.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = stats_[i];
  return n;
}

#define TRY(x)                    \
  do {                            \
    int _rc = (x);                \
    if (_rc != DFAMIN_OK) return _rc; \
  } while (0)
#define HIP(x) TRY(check_hip(x))

// ------------------------------------------------------------------ Engine
Engine::~Engine() {
  if (fused_stream_) {
    (void)hipStreamSynchronize(fused_stream_);
    (void)hipStreamDestroy(fused_stream_);
  }
  if (fused_ready_) (void)hipEventDestroy(fused_ready_);
  if (fused_done_) (void)hipEventDestroy(fused_done_);
  if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
  if (queue_exec_) (void)hipGraphExecDestroy(queue_exec_);
  if (ev_rb_) (void)hipEventDestroy(ev_rb_);
  DevBuf* bufs[] = {&d_desc_, &d_rows_, &d_jobs_, &d_joboff_, &d_flags_, &d_inst_off_, &d_minF_,
                    &d_minN_, &d_inst_of_, &d_block_, &d_act_, &d_act2_, &d_slot_of_, &d_nb_,
                    &d_keep_, &d_rank_, &d_sig_, &d_table_, &d_status_, &d_changed_, &d_rb_,
                    &d_results_, &d_wgflags_, &d_part_, &d_dense_,
                    &d_djobs_, &d_visit_, &d_bfs_rows_, &d_min_delta_, &d_min_acc_,
                    &d_lvl_, &d_lvl_wg_, &d_lvl_flags_, &d_qdbl_, &d_fjobs_, &d_notify_, &d_lbl_, &d_gcount_, &d_dtab_};
  // device buffers of the fixed-region mode belong to the region
  if (!fixed()) {
    for (DevBuf* b : bufs)
      if (b->p) (void)hipFree(b->p);
    for (DevBuf& b : closure_bufs_)
      if (b.p) (void)hipFree(b.p);
  }
  HostBuf* hb[] = {&h_ctrl_, &h_flags_, &h_results_, &h_counts_, &h_jobs_, &h_rb_, &h_qdbl_,
                   &stage_[0].buf, &stage_[1].buf, &h_fjobs_, &h_fres_};
  for (HostBuf* b : hb)
    if (b->p) (void)hipHostFree(b->p);
}

uint64_t Engine::device_bytes() const {
  const DevBuf* bufs[] = {&d_desc_, &d_rows_, &d_jobs_, &d_joboff_, &d_flags_, &d_inst_off_, &d_minF_,
                          &d_minN_, &d_inst_of_, &d_block_, &d_act_, &d_act2_, &d_slot_of_, &d_nb_,
                          &d_keep_, &d_rank_, &d_sig_, &d_table_, &d_status_, &d_changed_, &d_rb_,
                          &d_results_, &d_wgflags_, &d_part_, &d_dense_,
                          &d_djobs_, &d_visit_, &d_bfs_rows_, &d_min_delta_, &d_min_acc_,
                          &d_lvl_, &d_lvl_wg_, &d_lvl_flags_, &d_qdbl_, &d_fjobs_, &d_notify_, &d_lbl_, &d_gcount_, &d_dtab_};
  uint64_t t = 0;
  for (const DevBuf* b : bufs) t += b->cap;
  for (const DevBuf& b : closure_bufs_) t += b.cap;
  return t;
}

int Engine::check_hip(hipError_t e) {
  if (e == hipSuccess) return DFAMIN_OK;
  if (e == hipErrorOutOfMemory) return DFAMIN_E_NOMEM;
  ctx_->device_lost = true;
  return DFAMIN_E_DEVICE;
}

int Engine::ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return DFAMIN_OK;
  if (fixed()) {
    // carved from the region; what the buffer held before stays unused
    // until the next call restarts the carving
    const size_t at = (fixed_off_ + 255) & ~size_t(255);
    if (at > fixed_cap_ || bytes > fixed_cap_ - at) return DFAMIN_E_NOMEM;
    b.p = fixed_base_ + at;
    b.cap = bytes;
    fixed_off_ = at + bytes;
    return DFAMIN_OK;
  }
  size_t want = bytes + bytes / 8;  // head-room for the next, slightly larger call
  want = (want + 4095) & ~size_t(4095);
  if (b.p) {
    (void)hipFree(b.p);
    ctx_->used -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  if (ctx_->used + want > ctx_->budget) {
    want = (bytes + 4095) & ~size_t(4095);
    if (ctx_->used + want > ctx_->budget) return DFAMIN_E_NOMEM;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? DFAMIN_E_NOMEM : check_hip(e);
  }
  b.cap = want;
  ctx_->used += want;
  return DFAMIN_OK;
}

int Engine::ensure_host(HostBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return DFAMIN_OK;
  if (fixed() && b.p) return DFAMIN_E_NOMEM;  // sized once at set-up
  if (b.p) (void)hipHostFree(b.p);
  b.p = b.dp = nullptr;
  b.cap = 0;
  size_t want = (bytes + bytes / 8 + 64 + 15) & ~size_t(15);
  // coherent: the copy kernels read and write it directly, uncached on the
  // device side, so no device cache can hold a stale copy between calls
  if (hipHostMalloc(&b.p, want, hipHostMallocCoherent) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return DFAMIN_E_NOMEM;
  }
  if (hipHostGetDevicePointer(&b.dp, b.p, 0) != hipSuccess || !b.dp) {
    (void)hipHostFree(b.p);
    b.p = b.dp = nullptr;
    return check_hip(hipErrorInvalidValue);
  }
  b.cap = want;
  return DFAMIN_OK;
}

int Engine::set_fixed_region(void* base, size_t cap, size_t host_bytes) {
  if (!base || fixed() || device_bytes() != 0) return DFAMIN_E_INTERNAL;
  HostBuf* hb[] = {&h_ctrl_, &h_flags_, &h_results_, &h_counts_, &h_jobs_, &h_rb_, &h_qdbl_,
                   &stage_[0].buf, &stage_[1].buf, &h_fjobs_, &h_fres_};
  for (HostBuf* b : hb) TRY(ensure_host(*b, host_bytes));
  if (!ev_rb_) HIP(hipEventCreateWithFlags(&ev_rb_, hipEventDisableTiming));
  fixed_base_ = static_cast<char*>(base);
  fixed_cap_ = cap;
  fixed_off_ = 0;
  return DFAMIN_OK;
}

void Engine::reset_fixed_region() {
  DevBuf* bufs[] = {&d_desc_, &d_rows_, &d_jobs_, &d_joboff_, &d_flags_, &d_inst_off_, &d_minF_,
                    &d_minN_, &d_inst_of_, &d_block_, &d_act_, &d_act2_, &d_slot_of_, &d_nb_,
                    &d_keep_, &d_rank_, &d_sig_, &d_table_, &d_status_, &d_changed_, &d_rb_,
                    &d_results_, &d_wgflags_, &d_part_, &d_dense_,
                    &d_djobs_, &d_visit_, &d_bfs_rows_, &d_min_delta_, &d_min_acc_,
                    &d_lvl_, &d_lvl_wg_, &d_lvl_flags_, &d_qdbl_, &d_ctrl_, &d_refine_, &d_counts_,
                    &d_fjobs_, &d_notify_, &d_lbl_, &d_gcount_, &d_dtab_};
  for (DevBuf* b : bufs) *b = DevBuf{};
  closure_bufs_.clear();
  fixed_off_ = 0;
}

uint64_t Engine::closure_cap() const {
  if (fixed()) return fixed_cap_ > fixed_off_ ? (fixed_cap_ - fixed_off_) / 3 : 0;
  return ctx_->budget > ctx_->used ? (ctx_->budget - ctx_->used) / 2 : 0;
}

int Engine::upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return DFAMIN_OK;
  TRY(flush_segs(s));  // queued copies first, in the order they were asked for
  Stage& st = stage_[stage_cur_];
  size_t at = (st.off + 15) & ~size_t(15);
  if (at + bytes > st.buf.cap) {
    // every copy staged so far has run once the stream has drained; the
    // arena then grows to twice what this phase has asked for
    HIP(stream_wait(s));
    stage_idle();
    // (a fixed-region engine reuses its arena from the start, never grows it)
    if (!fixed() || st.buf.cap < bytes)
      TRY(ensure_host(st.buf, std::max<size_t>(2 * (at + bytes), size_t(64) << 10)));
    at = 0;
  }
  std::memcpy(st.buf.as<char>() + at, src, bytes);
  st.off = at + bytes;
  launch_copy_bytes(dst, static_cast<const char*>(st.buf.dp) + at, bytes, s);
  return check_hip(hipGetLastError());
}

int Engine::stage_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return DFAMIN_OK;
  Stage& st = stage_[stage_cur_];
  size_t at = (st.off + 15) & ~size_t(15);
  if (at + bytes > st.buf.cap) {
    // the queued copies read the arena: issue them before it is reused
    TRY(flush_segs(s));
    HIP(stream_wait(s));
    stage_idle();
    if (!fixed() || st.buf.cap < bytes)
      TRY(ensure_host(st.buf, std::max<size_t>(2 * (at + bytes), size_t(64) << 10)));
    at = 0;
  }
  std::memcpy(st.buf.as<char>() + at, src, bytes);
  st.off = at + bytes;
  if (segs_.n == kMemSegs) TRY(flush_segs(s));
  segs_.seg[segs_.n++] = MemSeg{dst, static_cast<const char*>(st.buf.dp) + at, bytes, 0, 0};
  return DFAMIN_OK;
}

int Engine::queue_fill(void* dst, uint32_t byte, size_t bytes, hipStream_t s) {
  if (!bytes) return DFAMIN_OK;
  if (segs_.n == kMemSegs) TRY(flush_segs(s));
  segs_.seg[segs_.n++] = MemSeg{dst, nullptr, bytes, byte & 0xffu, 0};
  return DFAMIN_OK;
}

int Engine::flush_segs(hipStream_t s) {
  if (!segs_.n) return DFAMIN_OK;
  launch_mem_segs(segs_, s);
  segs_.n = 0;
  return check_hip(hipGetLastError());
}

int Engine::readback(HostBuf& h, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return DFAMIN_OK;
  if (h.cap < bytes || !h.dp) return DFAMIN_E_INTERNAL;
  launch_copy_bytes(h.dp, src, bytes, s);
  return check_hip(hipGetLastError());
}

// Rebuild descriptors, row pointers and signature-record offsets from the
// per-instance row lists and upload them (queued: left in the copy queue for
// the caller's flush_segs).
int Engine::upload_layout(hipStream_t s, bool queued) {
  const size_t I = in_.size();
  rows_.clear();
  uint64_t sig_words = 0;
  row_base_.assign(I, 0);
  for (size_t i = 0; i < I; ++i) {
    desc_[i].rows_off = (uint32_t)rows_.size();
    row_base_[i] = desc_[i].rows_off;
    desc_[i].kp = (uint32_t)inst_rows_[i].size();
    rows_.insert(rows_.end(), inst_rows_[i].begin(), inst_rows_[i].end());
    desc_[i].sig = sig_words;  // word offset for now, made absolute below
    sig_words += (uint64_t)desc_[i].n * (desc_[i].kp + 1);
  }
  TRY(ensure(d_sig_, sig_words * 4));
  for (size_t i = 0; i < I; ++i) desc_[i].sig = reinterpret_cast<uint64_t>(d_sig_.p) + 4 * desc_[i].sig;
  TRY(ensure(d_desc_, I * sizeof(InstDesc)));
  TRY(ensure(d_rows_, std::max<size_t>(rows_.size(), 1) * 8));
  TRY(stage_copy(d_desc_.p, desc_.data(), I * sizeof(InstDesc), s));
  if (!rows_.empty()) TRY(stage_copy(d_rows_.p, rows_.data(), rows_.size() * 8, s));
  return queued ? DFAMIN_OK : flush_segs(s);
}

// Partial transitive closure (Algorithm 5) for the listed instances.  Level
// storage comes from this call's list of level buffers, at most half of the
// context's remaining budget: a closure cut short by that cap keeps the levels
// it has (any subset of closure letters is sound).
int Engine::build_closure(const std::vector<uint32_t>& which, const dfamin_opts& opts,
                          hipStream_t s) {
  std::vector<ClosureSpec> specs(which.size());
  for (size_t w = 0; w < which.size(); ++w) {
    const uint32_t i = which[w];
    uint32_t l = floor_log2_u32(in_[i].n);
    if (opts.max_levels && opts.max_levels < l) l = opts.max_levels;
    specs[w].n = in_[i].n;
    specs[w].delta = in_[i].delta;
    specs[w].letters = nonid_[i];
    specs[w].L = l;
  }
  const uint64_t cap = closure_cap();
  uint64_t taken = 0;
  ClosureScratch scratch;
  DevBuf* bufs[4] = {&d_jobs_, &d_joboff_, &d_flags_, &d_wgflags_};
  scratch.ensure = [&](int b, size_t bytes) -> void* {
    return ensure(*bufs[b], bytes) == DFAMIN_OK ? bufs[b]->p : nullptr;
  };
  scratch.host_flags = [&](size_t bytes) -> void* {
    return ensure_host(h_flags_, bytes) == DFAMIN_OK ? h_flags_.p : nullptr;
  };
  scratch.upload = [&](void* d, const void* h, size_t bytes) { return upload(d, h, bytes, s) == DFAMIN_OK; };
  scratch.flags_to_host = [&](const void* d, size_t bytes) {
    return readback(h_flags_, d, bytes, s) == DFAMIN_OK;
  };
  scratch.level_storage = [&](size_t bytes) -> void* {
    if (taken + bytes > cap) return nullptr;
    if (closure_cursor_ == closure_bufs_.size()) closure_bufs_.emplace_back();
    DevBuf& b = closure_bufs_[closure_cursor_];
    if (ensure(b, bytes) != DFAMIN_OK) return nullptr;
    ++closure_cursor_;
    taken += bytes;
    return b.p;
  };
  std::vector<std::vector<uint64_t>> rows;
  std::vector<uint32_t> depth;
  if (ctx_->prof.enabled()) {
    double bytes = 0;
    for (auto& sp : specs) bytes += 12.0 * sp.letters.size() * sp.L * sp.n;
    ctx_->prof.begin(s, "closure", bytes);
  }
  const int rc = build_closure_levels(specs, scratch, s, rows, depth);
  if (ctx_->prof.enabled()) {
    ctx_->prof.end(s);
    ctx_->prof.collect();
  }
  if (rc != DFAMIN_OK) return rc;
  for (size_t w = 0; w < which.size(); ++w) {
    inst_rows_[which[w]] = rows[w];
    levels_[which[w]] = depth[w];
    has_closure_[which[w]] = 1;
  }
  return DFAMIN_OK;
}

// Level storage for the unary instances in `which` that refine by doubling
// (one non-identity letter a).  A doubling round from P_j reads the single
// level 2^l <= j+1, and j at least doubles from one round to the next, so
// each level is computed (one pointer-jumping pass, Algorithm 5) in the round
// that first reads it rather than all up front between host checks.  No
// level is tested for equality with its predecessor or for the identity:
// with t <= j+1 the letter a^t gives P_{j+t} whatever it is.  Rows 0..L point
// at delta_a and the L level buffers; the other instances of `which` go to
// `rest` (all of them if the storage does not fit under the closure cap).
int Engine::lazy_levels(const std::vector<uint32_t>& which, const dfamin_opts& opts,
                        std::vector<uint32_t>& rest, std::vector<uint8_t>& lazy) {
  std::vector<uint32_t> uni;
  for (uint32_t i : which) (nonid_[i].size() == 1 ? uni : rest).push_back(i);
  if (uni.empty()) return DFAMIN_OK;
  auto levels_of = [&](uint32_t i) {
    uint32_t l = floor_log2_u32(in_[i].n);
    if (opts.max_levels && opts.max_levels < l) l = opts.max_levels;
    return l;
  };
  uint64_t words = 0;
  for (uint32_t i : uni) words += (uint64_t)levels_of(i) * in_[i].n;
  const uint64_t cap = closure_cap();
  char* base = nullptr;
  if (words) {
    if (words * 4 > cap) {
      rest.insert(rest.end(), uni.begin(), uni.end());
      return DFAMIN_OK;
    }
    if (closure_cursor_ == closure_bufs_.size()) closure_bufs_.emplace_back();
    DevBuf& b = closure_bufs_[closure_cursor_];
    if (ensure(b, words * 4) != DFAMIN_OK) {
      rest.insert(rest.end(), uni.begin(), uni.end());
      return DFAMIN_OK;
    }
    ++closure_cursor_;
    base = static_cast<char*>(b.p);
  }
  uint64_t off = 0;
  for (uint32_t i : uni) {
    const uint32_t L = levels_of(i), a = nonid_[i][0];
    std::vector<uint64_t> r(1 + (size_t)L);
    r[0] = reinterpret_cast<uint64_t>(in_[i].delta) + 4ull * a * in_[i].n;
    for (uint32_t l = 1; l <= L; ++l) {
      r[l] = reinterpret_cast<uint64_t>(base + 4 * off);
      off += in_[i].n;
    }
    inst_rows_[i] = std::move(r);
    levels_[i] = 0;
    has_closure_[i] = 1;
    lazy[i] = 1;
  }
  return DFAMIN_OK;
}

// Queues the level passes of one round: step 0 holds each instance's first
// missing level, step 1 the next one, and so on (one launch per step).
int Engine::queue_levels(const std::vector<LevelTodo>& todo, hipStream_t s) {
  const size_t J = todo.size();
  uint32_t S = 0;
  for (const LevelTodo& t : todo) S = std::max(S, t.step + 1);
  const size_t bytes = J * (sizeof(RowJob) + 4);
  // assembled here, then staged by upload(): two calls in one round (with
  // the round's kernels queued in between) never share host memory
  lvl_host_.resize(bytes);
  TRY(ensure(d_lvl_, bytes));
  RowJob* hj = reinterpret_cast<RowJob*>(lvl_host_.data());
  uint32_t* ho = reinterpret_cast<uint32_t*>(hj + J);
  std::vector<uint32_t> begin(S + 1, 0), wgs(S, 0);
  uint32_t c = 0;
  double alg = 0;
  for (uint32_t st = 0; st < S; ++st) {
    begin[st] = c;
    uint32_t w = 0;
    for (const LevelTodo& t : todo) {
      if (t.step != st) continue;
      const std::vector<uint64_t>& r = inst_rows_[t.inst];
      RowJob R;
      R.src = r[t.level - 1];
      R.dst = r[t.level];
      R.n = in_[t.inst].n;
      R.flag_idx = c;
      hj[c] = R;
      ho[c] = w;
      w += (R.n + kRowTile - 1) / kRowTile;
      alg += 12.0 * R.n;
      ++c;
    }
    wgs[st] = w;
  }
  begin[S] = c;
  TRY(upload(d_lvl_.p, lvl_host_.data(), bytes, s));
  RowJob* dj = d_lvl_.as<RowJob>();
  uint32_t* dof = reinterpret_cast<uint32_t*>(dj + J);
  Profiler& prof = ctx_->prof;
  prof.begin(s, "closure", alg);
  for (uint32_t st = 0; st < S; ++st)
    if (begin[st + 1] > begin[st])
      // (a level read by a doubling round is not tested for being equal to
      // its predecessor or the identity: no flags)
      launch_closure_level(dj + begin[st], dof + begin[st], begin[st + 1] - begin[st], wgs[st], nullptr,
                           nullptr, s);
  prof.end(s);
  HIP(hipGetLastError());
  return DFAMIN_OK;
}

// Queued signature rounds.  Once every instance still refining groups by
// hash (which lasts: block counts only grow) and needs no closure change and
// no count scan, a round needs no decision of the host.  The kernels then
// take the live active count and the salt from the control block, the grids
// and the table are sized for the current m (which never grows), a one-thread
// step ends each round (a new salt after a hash collision, else the next
// count, and stop once nothing split), and every kernel of a later round
// returns at once after stop.  Rounds go to the stream in captured graphs of
// kQueueRounds (or directly), and the host reads the control block after 1,
// 2, 4 ... of them.  `executed`: the refining rounds run (the one that found
// nothing to split included).
int Engine::queued_rounds(uint64_t m, uint32_t tbits, int variant, int items, uint64_t salt, uint32_t* cur,
                          uint32_t* nxt, uint64_t max_left, bool use_graph, const QueueDbl* dq, hipStream_t s,
                          uint64_t& executed) {
  const size_t I = in_.size();
  const bool batch = I > 1;
  const uint64_t tsize = 1ull << tbits;
  const uint32_t ntiles = scan_tiles(m, items);
  launch_queue_start(d_ctrl_.as<Ctrl>(), (uint32_t)m, salt, s);
  HIP(hipGetLastError());
  auto queue = [&](uint32_t* a, uint32_t* b) {
    if (dq) {
      launch_queue_plan(*dq, d_desc_.as<InstDesc>(), d_ctrl_.as<Ctrl>(), s);
      launch_queue_levels(*dq, d_rows_.as<uint64_t>(), d_ctrl_.as<Ctrl>(), s);
    }
    launch_clear_table(d_table_.as<Slot>(), tsize, d_ctrl_.as<Ctrl>(), s, 1);
    launch_signature(batch, a, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                     d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), d_dense_.p, 4, d_table_.as<Slot>(), tbits,
                     d_slot_of_.as<uint32_t>(), salt, d_ctrl_.as<Ctrl>(), variant, s, 1 | (int)cas_bits_);
    launch_resolve(batch, a, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                   d_table_.as<Slot>(), d_slot_of_.as<uint32_t>(), d_block_.as<uint32_t>(), d_nb_.as<uint32_t>(),
                   d_keep_.as<uint8_t>(), d_changed_.as<uint32_t>(), d_ctrl_.as<Ctrl>(),
                   d_status_.as<unsigned long long>(), ntiles, s, 1);
    launch_compact(batch, a, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_nb_.as<uint32_t>(),
                   d_keep_.as<uint8_t>(), d_changed_.as<uint32_t>(), nullptr, d_block_.as<uint32_t>(), b,
                   d_ctrl_.as<Ctrl>(), d_status_.as<unsigned long long>(), items, s, 1);
    launch_round_end((uint32_t)I, d_changed_.as<uint32_t>(), d_refine_.as<uint32_t>(),
                     dq ? const_cast<uint32_t*>(dq->last) : nullptr, d_ctrl_.as<Ctrl>(), s, nullptr, 0, 1);
    if (dq) launch_queue_advance(*dq, d_ctrl_.as<Ctrl>(), s);
    launch_round_step(d_ctrl_.as<Ctrl>(), s);
  };
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    const std::array<uint64_t, kQueueKeyWords> key{
        m, tbits, (uint64_t)variant, (uint64_t)items, I,
        reinterpret_cast<uint64_t>(cur), reinterpret_cast<uint64_t>(nxt), reinterpret_cast<uint64_t>(d_inst_of_.p),
        reinterpret_cast<uint64_t>(d_desc_.p), reinterpret_cast<uint64_t>(d_rows_.p),
        reinterpret_cast<uint64_t>(d_block_.p), reinterpret_cast<uint64_t>(d_table_.p),
        reinterpret_cast<uint64_t>(d_slot_of_.p), reinterpret_cast<uint64_t>(d_nb_.p),
        reinterpret_cast<uint64_t>(d_keep_.p), reinterpret_cast<uint64_t>(d_changed_.p),
        reinterpret_cast<uint64_t>(d_refine_.p), reinterpret_cast<uint64_t>(d_ctrl_.p),
        reinterpret_cast<uint64_t>(d_status_.p), reinterpret_cast<uint64_t>(d_dense_.p),
        reinterpret_cast<uint64_t>(s), 1u | cas_bits_, dq ? reinterpret_cast<uint64_t>(dq->mj) : 0,
        dq ? ((uint64_t)dq->count << 32 | dq->wgs) : 0};
    if (queue_exec_ && queue_key_ == key) {
      exec = queue_exec_;
    } else {
      if (queue_exec_) (void)hipGraphExecDestroy(queue_exec_);
      queue_exec_ = nullptr;
      hipGraph_t g = nullptr;
      HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      for (uint32_t r = 0; r < kQueueRounds; ++r) queue(r & 1 ? nxt : cur, r & 1 ? cur : nxt);
      const hipError_t ce = hipStreamEndCapture(s, &g);
      if (ce != hipSuccess || !g) return check_hip(ce != hipSuccess ? ce : hipErrorUnknown);
      const hipError_t ie = hipGraphInstantiate(&queue_exec_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP(ie);
      queue_key_ = key;
      exec = queue_exec_;
    }
  }
  uint32_t per_check = 1;
  while (true) {
    for (uint32_t b = 0; b < per_check; ++b) {
      if (exec) {
        HIP(hipGraphLaunch(exec, s));
      } else {
        for (uint32_t r = 0; r < kQueueRounds; ++r) queue(r & 1 ? nxt : cur, r & 1 ? cur : nxt);
      }
    }
    HIP(hipGetLastError());
    TRY(readback(h_rb_, d_rb_.p, sizeof(Ctrl), s));
    HIP(stream_wait(s));
    stage_idle();
    const Ctrl c = *h_rb_.as<Ctrl>();
    if (c.fault) return DFAMIN_E_INTERNAL;
    executed = c.iterations;
    if (c.stop) return DFAMIN_OK;
    if (executed > max_left) return DFAMIN_E_INTERNAL;
    per_check = std::min<uint32_t>(per_check * 2, 8);
  }
}

// Signature rounds (Algorithm 4, Section 3.3) over the active states until no
// instance splits a block.
int Engine::signature_rounds(const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s) {
  const size_t I = in_.size();
  const bool batch = I > 1;
  const uint64_t N = N_;
  Profiler& prof = ctx_->prof;
  const uint32_t auto_rounds = opts.auto_rounds ? opts.auto_rounds : kDefaultAutoRounds;
  bool any_auto = false;
  for (auto& x : in_) any_auto |= (x.closure == DFAMIN_CLOSURE_AUTO);
  uint64_t m = N;
  // upper bound on each instance's block count before the next round
  std::vector<uint64_t> ub(I, 2);
  uint32_t* cur = d_act_.as<uint32_t>();
  uint32_t* nxt = d_act2_.as<uint32_t>();
  uint64_t salt = 0x5DEECE66Dull;
  int retries = 0;
  uint64_t rounds = 0;
  int dense_width = 4;
  // Algorithmic bytes per active state of the signature kernel, averaged
  // over instances weighted by n: act [+ inst_of] + own key + per letter the
  // delta' entry and the gathered key + the signature record (hash mode) +
  // slot id + one slot update.  Keys are an accept bit (1 byte read), a
  // dense number (dense_width bytes) or a block id (4 bytes).
  auto sig_bytes = [&]() {
    double w = 0;
    for (size_t i = 0; i < I; ++i) {
      const InstDesc& D = desc_[i];
      const double key = D.ebits ? (D.dsrc ? 1.0 : (double)dense_width) : 4.0;
      const double rec = D.ebits ? 0.0 : 4.0 * (D.kp + 1);
      w += (double)D.n * (4.0 + (batch ? 4.0 : 0.0) + key + D.kp * (4.0 + key) + rec + 4.0 + 8.0);
    }
    return N ? w / (double)N : 0.0;
  };
  // Per instance: still refining (every round so far split a block), and
  // the length j of the Moore partition P_j it holds (P_j: states agree on
  // all words of length <= j).  Unary instances that get the closure under
  // AUTO refine by doubling: from P_j, the one letter a^t with t <= j+1
  // gives exactly P_{j+t}, and a round that splits nothing proves P_j
  // stable (P_j >= P_{j+1} >= P_{j+t} = P_j).  t is the largest closure
  // level 2^l <= j+1, so each round gathers one successor instead of one
  // per level.
  std::vector<uint8_t> active(I, 1), dbl(I, 0);
  std::vector<uint64_t> mj(I, 0), step(I, 1);
  // Doubling instances with lazily built levels: levels computed so far
  // (possibly one ahead of the rounds) and the highest level a round read.
  // On every way out the rows are cut to the levels read, all of them built,
  // which is what later readers of the closure rows (the reachability
  // search) may follow and what the results report.
  std::vector<uint8_t> lazy = lazy_;  // planned by run() before the layout went up
  lazy.resize(I, 0);
  for (size_t i = 0; i < I; ++i) dbl[i] = lazy[i];
  std::vector<uint32_t> built(I, 0), used(I, 0);
  std::vector<LevelTodo> todo;
  uint64_t spec_clear = 0;  // table slots cleared ahead for the coming round
  bool prev_all_hash = false;  // the last round grouped every instance by hash

  struct TrimLazy {
    Engine* e;
    const std::vector<uint8_t>& lazy;
    const std::vector<uint32_t>& used;
    ~TrimLazy() {
      for (size_t i = 0; i < lazy.size(); ++i)
        if (lazy[i]) {
          e->inst_rows_[i].resize((size_t)used[i] + 1);
          e->levels_[i] = used[i];
        }
    }
  } trim_lazy{this, lazy, used};
  // Exact block counts (and instance-relative ranks in d_rank_) of the
  // instances scanned at the end of the previous round; cnt_ok marks them.
  std::vector<uint64_t> cnt(I, 0);
  std::vector<uint8_t> cnt_ok(I, 0);
  // an instance whose next signature could fit 31 bits is counted exactly
  // at the end of a round (B <= min(n, B^(kp+1)) after it)
  auto would_scan = [&](uint32_t i) {
    const uint64_t B = cnt_ok[i] ? std::max<uint64_t>(cnt[i], 1) : ub[i];
    const uint64_t kp1 = desc_[i].kp + 1ull;
    const uint32_t bits = std::max<uint32_t>(1, ceil_log2_u64(B));
    const uint64_t nb = (kp1 * bits >= 40) ? in_[i].n : std::min<uint64_t>(in_[i].n, 1ull << (kp1 * bits));
    return kp1 * std::max<uint32_t>(1, ceil_log2_u64(nb)) <= 31;
  };
  std::vector<uint32_t> exact, scan;
  std::vector<uint32_t> alist(I);  // instances still refining, in order
  // After a round (not redone): per-instance bounds, j, the closure levels
  // read, and which instances still refine (rc: refine counters).
  auto settle = [&](const uint32_t* rc) {
    for (uint32_t i : alist) {
      // a round maps each block to at most B^(kp+1) signatures
      const uint64_t kp1 = desc_[i].kp + 1ull;
      const uint32_t bits = std::max<uint32_t>(1, ceil_log2_u64(ub[i]));
      ub[i] = (kp1 * bits >= 40) ? in_[i].n : std::min<uint64_t>(in_[i].n, 1ull << (kp1 * bits));
      if (cnt_ok[i]) ub[i] = std::max<uint64_t>(cnt[i], 1);
      mj[i] += dbl[i] ? step[i] : 1;
      active[i] = rc[i] == rounds;
      // closure levels reported: the highest one a splitting round read
      if (dbl[i] && active[i]) used[i] = std::max<uint32_t>(used[i], floor_log2_u64(step[i]));
      // every block a singleton: stable, whatever the other instances do
      // (it plans no further level and reads none)
      if (cnt_ok[i] && cnt[i] >= in_[i].n) active[i] = 0;
    }
    alist.erase(std::remove_if(alist.begin(), alist.end(), [&](uint32_t i) { return !active[i]; }), alist.end());
  };
  // the dense numbers of the coming round were written by the first round's labels
  bool dense_from_labels = false;
  // key bits of a count table cleared behind the last round's copy (0: none)
  uint32_t dtab_ready = 0;
  all_single_ = false;
  // slot labels (launch_compact) for one instance, unless rounds are queued
  // (their resolve steps compare ids) or a testing knob turns them off; and
  // whether block[] holds such labels from the last round
  const bool slots_ok = !batch && !slots_off_ && !(opts.flags & DFAMIN_FLAG_QUEUE);
  bool slot_prev = false;
  TRY(ensure(d_gcount_, 2 * kGroupCounters * 4));
  uint32_t* const gcount = d_gcount_.as<uint32_t>();
  for (size_t i = 0; i < I; ++i) alist[i] = (uint32_t)i;
  TRY(ensure(d_djobs_, 4 * I * 4 + 64));
  TRY(ensure_host(h_jobs_, 4 * I * 4 + 64));
  uint32_t* hj = h_jobs_.as<uint32_t>();
  uint32_t* dj = d_djobs_.as<uint32_t>();
  // job lists already on the device (uploaded again only when they change)
  std::vector<uint32_t> up_dense, up_scan;
  auto upload_if_changed = [&](std::vector<uint32_t>& last, const uint32_t* h, uint32_t* d, size_t words) {
    if (last.size() == words && std::equal(last.begin(), last.end(), h)) return DFAMIN_OK;
    last.assign(h, h + words);
    return upload(d, h, words * 4, s);
  };
  // host-side time per phase of the round loop (printed with DFAMIN_TRACE)
  const bool trace = std::getenv("DFAMIN_TRACE") != nullptr;
  double t_plan = 0, t_issue = 0, t_wait = 0, t_post = 0, t_closure = 0, t_desc = 0;
  uint32_t n_dirty = 0;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto us = [](auto a, auto b) { return std::chrono::duration<double, std::micro>(b - a).count(); };
  auto tp0 = now();
  while (m > 0) {
    tp0 = now();
    if (any_auto && rounds == auto_rounds) {
      // other instances still refining after auto_rounds rounds get the closure
      std::vector<uint32_t> which;
      for (uint32_t i : alist)
        if (in_[i].closure == DFAMIN_CLOSURE_AUTO && !has_closure_[i]) which.push_back(i);
      if (!which.empty()) {
        std::vector<uint32_t> rest;
        TRY(lazy_levels(which, opts, rest, lazy));
        if (!rest.empty()) TRY(build_closure(rest, opts, s));
        if (trace)
          std::fprintf(stderr, "[dfamin] closure planned for %zu instances (%zu built up front): %.0f us\n",
                       which.size(), rest.size(), us(tp0, now()));
        TRY(upload_layout(s));
        for (uint32_t i : which) dbl[i] = nonid_[i].size() == 1;
      }
      if (trace) t_closure += us(tp0, now());
    }
    if (rounds >= max_rounds) return DFAMIN_E_INTERNAL;
    bool dirty = false;
    // doubling instances: this round's single closure level
    for (uint32_t i : alist) {
      if (!dbl[i]) continue;
      const uint32_t nrows = (uint32_t)inst_rows_[i].size();
      uint32_t lvl = (uint32_t)floor_log2_u64(mj[i] + 1);
      if (lvl > nrows - 1) lvl = nrows - 1;
      step[i] = 1ull << lvl;
      if (lazy[i] && built[i] < lvl) {
        for (uint32_t l = built[i] + 1; l <= lvl; ++l) todo.push_back({i, l, l - built[i] - 1});
        built[i] = lvl;
      }
      if (desc_[i].rows_off != row_base_[i] + lvl || desc_[i].kp != 1) {
        desc_[i].rows_off = row_base_[i] + lvl;
        desc_[i].kp = 1;
        dirty = true;
      }
    }
    if (!todo.empty()) {
      TRY(queue_levels(todo, s));
      todo.clear();
    }
    // Key mode per instance (see InstDesc): exact keys while
    // (kp+1) * ceil(log2 B) fits in 31 bits, B = blocks before this round
    // (exact, from the scan at the end of the previous round).  Round 1
    // takes its keys from the accept bits.
    exact.clear();
    uint32_t eb_max = 0;
    bool any_hash = false;
    for (uint32_t i : alist) {
      const uint64_t kp1 = desc_[i].kp + 1ull;
      uint32_t eb = 0, ds = 0;
      if (rounds == 0) {
        if (kp1 <= 31) { eb = 1; ds = 1; }
      } else if (cnt_ok[i]) {
        const uint32_t bits = std::max<uint32_t>(1, ceil_log2_u64(std::max<uint64_t>(cnt[i], 1)));
        if (kp1 * bits <= 31) {
          eb = bits;
          exact.push_back(i);
          eb_max = std::max(eb_max, eb);
        }
      }
      if (eb == 0) any_hash = true;
      if (desc_[i].ebits != eb || desc_[i].dsrc != ds) {
        desc_[i].ebits = eb;
        desc_[i].dsrc = ds;
        dirty = true;
      }
    }
    if (!exact.empty()) {
      // dense numbers from the ranks of the previous scan (or the first
      // round's label numbers, one byte each)
      dense_width = eb_max <= 8 ? 1 : (eb_max <= 16 ? 2 : 4);
      const uint32_t ne = (uint32_t)exact.size();
      uint32_t wgs = 0;
      double es = 0;
      for (uint32_t j = 0; j < ne; ++j) {
        hj[j] = exact[j];
        hj[ne + j] = wgs;
        wgs += (in_[exact[j]].n + kRowTile - 1) / kRowTile;
        es += in_[exact[j]].n;
      }
      TRY(ensure(d_dense_, N * 4));
      if (!dense_from_labels) {
        TRY(upload_if_changed(up_dense, hj, dj, 2 * ne));
        prof.begin(s, "dense", (8.0 + dense_width) * es);
        launch_dense_jobs(d_desc_.as<InstDesc>(), dj, dj + ne, ne, wgs, d_block_.as<uint32_t>(),
                          d_rank_.as<uint32_t>(), d_dense_.p, dense_width, s);
        prof.end(s);
      }
    }
    if (dirty) {
      const auto td = now();
      TRY(upload(d_desc_.p, desc_.data(), I * sizeof(InstDesc), s));
      if (trace) {
        t_desc += us(td, now());
        ++n_dirty;
      }
    }
    // The first round by labels (launch_label): every instance has at most
    // kMaxLabelLetters signature letters.  Every state stays active; in the
    // rare batch where an instance did not split, a compaction then drops
    // that instance's states.
    const bool label_round = rounds == 0 && labels_planned_ && !alist.empty();
    if (label_round) {
      // planned by run_path, which then left out the initial partition
      for (uint32_t i : alist)
        if (desc_[i].kp + 1 > label_bits_) return DFAMIN_E_INTERNAL;
      TRY(ensure(d_dense_, N * 4));
      // (lmin set to all ones by run_path)
      const uint32_t nl = label_bits_ <= 8 ? 256u : 512u, lw = label_bits_ <= 8 ? 1u : 2u;
      uint32_t* lmin = d_lbl_.as<uint32_t>();
      void* rank = lmin + I * nl;
      const int litems = scan_items_for(m);
      const uint32_t ltiles = scan_tiles(m, litems);
      double lb = 0;
      // own bit, kp row entries and bitmap bytes, the label written and read,
      // the dense byte, the id and the list entry [instance map]
      for (size_t i = 0; i < I; ++i)
        lb += (double)in_[i].n * (0.125 + 5.0 * desc_[i].kp + 2.0 * lw + 1.0 + 8.0 + (batch ? 4.0 : 0.0));
      prof.begin(s, "label", lb);
      // one-byte labels become the dense numbers in place; two-byte ones
      // are kept in the (here unused) new-id array
      launch_label(d_desc_.as<InstDesc>(), d_inst_off_.as<uint32_t>(), (uint32_t)I, init_wgs_,
                   d_rows_.as<uint64_t>(), label_bits_, lmin, rank, lw == 1 ? d_dense_.p : d_nb_.p,
                   d_dense_.as<uint8_t>(), d_counts_.as<uint32_t>(), d_changed_.as<uint32_t>(), d_ctrl_.as<Ctrl>(),
                   d_block_.as<uint32_t>(), 1u, (uint32_t)m, d_act_.as<uint32_t>(),
                   batch ? d_inst_of_.as<uint32_t>() : nullptr, s);
      prof.end(s);
      launch_round_end((uint32_t)I, d_changed_.as<uint32_t>(), d_refine_.as<uint32_t>(), nullptr,
                       d_ctrl_.as<Ctrl>(), s);
      HIP(hipGetLastError());
      // control block, refine counters and every instance's label count
      TRY(readback(h_rb_, d_rb_.p, sizeof(Ctrl) + 8 * I, s));
      // One instance's next round may group in a count table of at most
      // (kp+1)^2 key bits: it is cleared behind the copy, while the host
      // waits and plans (wasted only if this round was the last).
      dtab_ready = 0;
      const bool lover = !prof.enabled();
      if (lover) {
        if (!ev_rb_) HIP(hipEventCreateWithFlags(&ev_rb_, hipEventDisableTiming));
        HIP(hipEventRecord(ev_rb_, s));
        const uint32_t bits = (desc_[0].kp + 1u) * (desc_[0].kp + 1u);
        if (!batch && slots_ok && !direct_off_ && !fixed() && bits <= kDirectMaxBits && bits >= 1 &&
            (1ull << bits) <= 8ull * m) {
          TRY(ensure(d_dtab_, 4ull << bits));
          launch_clear_table(d_dtab_.as<Slot>(), 1ull << (bits - 1), d_ctrl_.as<Ctrl>(), s, 0, gcount);
          HIP(hipGetLastError());
          dtab_ready = bits;
        }
      }
      HIP(lover ? event_wait(ev_rb_) : stream_wait(s));
      stage_flip();
      prof.collect();
      const Ctrl c = *h_rb_.as<Ctrl>();
      const uint32_t* h_refine = reinterpret_cast<const uint32_t*>(h_rb_.as<char>() + sizeof(Ctrl));
      if (c.fault) return DFAMIN_E_INTERNAL;
      for (size_t i = 0; i < I; ++i) {
        cnt[i] = h_refine[I + i];
        cnt_ok[i] = 1;
      }
      if (trace) t_issue += us(tp0, now());
      ++rounds;
      const size_t before = alist.size();
      settle(h_refine);
      dense_from_labels = true;
      if (I == 1) all_single_ = cnt[0] >= in_[0].n;
      if (!c.any_changed || alist.empty()) break;
      if (alist.size() < before) {
        // Some instance split nothing (or only into single states): its
        // states leave the list, kept by a compaction whose per-instance
        // flags are the instances still refining.
        std::vector<uint32_t>& live = live_;
        live.assign(I, 0);
        for (uint32_t i : alist) live[i] = 1;
        TRY(stage_copy(d_changed_.p, live.data(), I * 4, s));
        TRY(queue_fill(d_keep_.p, 1, m, s));
        TRY(flush_segs(s));
        launch_prep_scan(d_status_.as<unsigned long long>(), ltiles, d_ctrl_.as<Ctrl>(), s);
        prof.begin(s, "compact", (double)m * (4 + 4 + 4 + 1 + 4));
        launch_compact(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_block_.as<uint32_t>(),
                       d_keep_.as<uint8_t>(), d_changed_.as<uint32_t>(), nullptr, d_block_.as<uint32_t>(), nxt,
                       d_ctrl_.as<Ctrl>(), d_status_.as<unsigned long long>(), litems, s);
        prof.end(s);
        TRY(queue_fill(d_changed_.p, 0, I * 4, s));
        TRY(flush_segs(s));
        HIP(hipGetLastError());
        TRY(readback(h_rb_, d_rb_.p, sizeof(Ctrl), s));
        HIP(stream_wait(s));
        stage_flip();
        prof.collect();
        const Ctrl c2 = *h_rb_.as<Ctrl>();
        if (c2.fault) return DFAMIN_E_INTERNAL;
        std::swap(cur, nxt);
        m = c2.m_next;
      }
      continue;
    }
    // Table: twice the number of groups this round can form, at most m.  An
    // exact-key instance forms at most 2^((kp+1) * ebits) groups.
    uint64_t groups = 0;
    for (uint32_t i : alist) {
      if (groups >= m) break;
      const uint64_t width = (desc_[i].kp + 1ull) * desc_[i].ebits;
      groups += (desc_[i].ebits && width < 32) ? std::min<uint64_t>(in_[i].n, 1ull << width) : in_[i].n;
    }
    groups = std::min<uint64_t>(groups, m);
    const uint32_t tbits = std::max<uint32_t>(9, ceil_log2_u64(2 * groups));
    // Table insertion order (table_insert).  A hash-mode group is mostly
    // new to the table: a CAS on the home slot claims it without a read
    // first (C1's third round: 2.05 -> 1.85 ms).  Exact keys do the same
    // unless few global groups take inserts from many workgroups: each
    // workgroup tile (at most 1,024 states) inserts at most one local group
    // per global group, and above 64 inserts per global group on average the
    // read first lets most joins skip the atomic on a hot slot (C1's first
    // round, 32 groups: 0.38 ms, against 0.62 ms with the CAS; batch_mixed's
    // first round, about 2M groups over 4,096 instances: 1.01 ms with the
    // CAS, against 1.23 ms).
    {
      uint64_t ex_groups = 0, ex_inserts = 0;
      for (uint32_t i : alist) {
        if (!desc_[i].ebits) continue;
        const uint64_t width = (desc_[i].kp + 1ull) * desc_[i].ebits;
        const uint64_t gi = width < 32 ? std::min<uint64_t>(in_[i].n, 1ull << width) : in_[i].n;
        ex_groups += gi;
        ex_inserts += ((in_[i].n + 1023ull) / 1024ull) * std::min<uint64_t>(1024, gi);
      }
      cas_bits_ = 2u | (ex_inserts <= 64 * ex_groups ? 4u : 0u);
      if (cas_forced_ >= 0) cas_bits_ = (uint32_t)cas_forced_;
    }
    const uint64_t tsize = 1ull << tbits;
    TRY(ensure(d_table_, tsize * sizeof(Slot)));
    const int citems = scan_items_for(m);
    const uint32_t ntiles = scan_tiles(m, citems);
    const double md = (double)m;
    const double inst_b = batch ? 4.0 : 0.0;

    const auto tp1 = now();
    t_plan += us(tp0, tp1);
    if (trace && rounds == 0)
      std::fprintf(stderr, "[dfamin] round 1 planned in %.0f us (descriptors %.0f us)\n", us(tp0, tp1), t_desc);
    // Signature tile: forced, cached for this size class, or tuned now by
    // running every variant once on a freshly cleared table (the last run's
    // table and slot ids are as valid as any other's).
    Tuner& tu = ctx_->tuner;
    const uint32_t tkey = (batch ? 1u : 0u) | (any_hash ? 2u : 0u) | ((uint32_t)dense_width << 2) |
                          (ceil_log2_u64(m) << 8);
    int variant = kSigDefaultVariant;
    bool tuned_now = false;
    const auto tuned = tu.best.find(tkey);
    // Queued rounds (queued_rounds): every instance still refining grouped by
    // hash in this round and the last, none refines by doubling or still
    // waits for its AUTO closure, and none needs a count scan.
    const bool all_hash = rounds > 0 && exact.empty();
    const bool queue_allowed = !prof.enabled() && (opts.flags & DFAMIN_FLAG_QUEUE);
    bool queue_ok = all_hash && prev_all_hash && queue_allowed;
    for (uint32_t i : alist) {
      if (!queue_ok) break;
      if (dbl[i] || would_scan(i) ||
          (in_[i].closure == DFAMIN_CLOSURE_AUTO && !has_closure_[i] && rounds < auto_rounds))
        queue_ok = false;
    }
    prev_all_hash = all_hash;
    // ... or every instance still refining doubles, with levels built as
    // read: the device then plans the levels too, and every round groups by
    // hash (always exact; for one gathered letter about as fast as exact
    // keys with their count scans)
    bool queue_dbl = !queue_ok && queue_allowed && rounds > 0 && !alist.empty();
    for (uint32_t i : alist) {
      if (!queue_dbl) break;
      if (!dbl[i] || !lazy[i]) queue_dbl = false;
    }
    QueueDbl dq{};
    if (queue_dbl) {
      const uint32_t T = (uint32_t)alist.size();
      const size_t bytes = 8ull * T + 36ull * T;
      TRY(ensure(d_qdbl_, bytes + 4ull * I));  // then one changed flag per instance
      TRY(ensure_host(h_qdbl_, bytes));
      uint64_t* hmj = h_qdbl_.as<uint64_t>();
      uint32_t* h32 = reinterpret_cast<uint32_t*>(hmj + T);
      uint32_t* f[9];
      for (int a = 0; a < 9; ++a) f[a] = h32 + (size_t)a * T;  // list built lmax rbase need lv used n wgoff
      uint32_t wgs = 0;
      for (uint32_t t = 0; t < T; ++t) {
        const uint32_t i = alist[t];
        hmj[t] = mj[i];
        f[0][t] = i;
        f[1][t] = built[i];
        f[2][t] = (uint32_t)inst_rows_[i].size() - 1;
        f[3][t] = row_base_[i];
        f[4][t] = 0;
        f[5][t] = 0;
        f[6][t] = used[i];
        f[7][t] = in_[i].n;
        f[8][t] = wgs;
        wgs += (in_[i].n + kRowTile - 1) / kRowTile;
        desc_[i].ebits = 0;  // hash keys from here on
        desc_[i].dsrc = 0;
      }
      TRY(upload(d_qdbl_.p, h_qdbl_.p, bytes, s));
      TRY(upload(d_desc_.p, desc_.data(), I * sizeof(InstDesc), s));
      uint64_t* dmj = d_qdbl_.as<uint64_t>();
      uint32_t* d32 = reinterpret_cast<uint32_t*>(dmj + T);
      dq.mj = dmj;
      dq.list = d32;
      dq.built = d32 + T;
      dq.lmax = d32 + 2 * T;
      dq.rbase = d32 + 3 * T;
      dq.need = d32 + 4 * T;
      dq.lv = d32 + 5 * T;
      dq.used = d32 + 6 * T;
      dq.n = d32 + 7 * T;
      dq.wgoff = d32 + 8 * T;
      dq.last = d32 + 9 * T;
      dq.count = T;
      dq.wgs = wgs;
    }
    if (queue_ok || queue_dbl) {
      if (tu.forced >= 0) variant = tu.forced;
      else if (tuned != tu.best.end()) variant = tuned->second;
      const bool use_graph = !(opts.flags & DFAMIN_FLAG_NO_GRAPH) && s != nullptr;
      // hash keys for every instance: at most m groups
      const uint32_t qtbits = queue_dbl ? std::max<uint32_t>(9, ceil_log2_u64(2 * m)) : tbits;
      TRY(ensure(d_table_, (1ull << qtbits) * sizeof(Slot)));
      uint64_t executed = 0;
      TRY(queued_rounds(m, qtbits, variant, citems, salt, cur, nxt, max_rounds - rounds, use_graph,
                        queue_dbl ? &dq : nullptr, s, executed));
      if (queue_dbl) {
        // levels built and read on the device
        const uint32_t T = dq.count;
        TRY(readback(h_qdbl_, d_qdbl_.p, 8ull * T + 36ull * T, s));
        HIP(stream_wait(s));
        const uint32_t* h32 = reinterpret_cast<const uint32_t*>(h_qdbl_.as<uint64_t>() + T);
        for (uint32_t t = 0; t < T; ++t) {
          const uint32_t i = h32[t];
          built[i] = std::max(built[i], h32[T + t]);
          used[i] = std::max(used[i], h32[6 * T + t]);
        }
      }
      rounds += executed;
      all_single_ = false;
      if (rounds > max_rounds) return DFAMIN_E_INTERNAL;
      if (trace) std::fprintf(stderr, "[dfamin] %llu queued rounds from m=%llu\n", (unsigned long long)executed,
                              (unsigned long long)m);
      break;
    }
    // Slot labels (launch_compact): one instance in an exact-key round whose
    // block count is known, followed by a hash round with no count scan
    // (which reads labels as well as ids and then restores least-member
    // ids).  The resolve step and its random read of a slot per state are
    // left out.  Where the key space is small enough (at most
    // 2^kDirectMaxBits keys, at most 8 per active state) the groups form in
    // a direct count table instead of the hash table.
    const uint32_t i0 = alist.empty() ? 0u : alist[0];
    const bool slot_cand = slots_ok && !slot_prev && alist.size() == 1 && desc_[i0].ebits && cnt_ok[i0] &&
                           cnt[i0] + m >= in_[i0].n && !would_scan(i0);
    const uint32_t dwidth = (desc_[i0].kp + 1u) * desc_[i0].ebits;
    // (not in the fixed region, whose size is set for the hash table)
    const bool direct =
        slot_cand && !fixed() && !direct_off_ && dwidth <= kDirectMaxBits && (1ull << dwidth) <= 8ull * m;
    if (tu.forced >= 0) {
      variant = tu.forced;
    } else if (direct) {
      if (tuned != tu.best.end()) variant = tuned->second;
    } else if (m >= kTuneMinStates) {
      auto it = tuned;
      if (it != tu.best.end()) {
        variant = it->second;
      } else {
        if (!tu.have_events) {
          for (hipEvent_t& e : tu.ev) HIP(hipEventCreate(&e));
          tu.have_events = true;
        }
        for (int v = 0; v < kSigVariants; ++v) {
          launch_clear_table(d_table_.as<Slot>(), tsize, d_ctrl_.as<Ctrl>(), s, 0, gcount);
          HIP(hipEventRecord(tu.ev[2 * v], s));
          launch_signature(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                           d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), d_dense_.p, dense_width,
                           d_table_.as<Slot>(), tbits, d_slot_of_.as<uint32_t>(), salt, d_ctrl_.as<Ctrl>(),
                           v, s, (int)cas_bits_, nullptr, gcount);
          HIP(hipEventRecord(tu.ev[2 * v + 1], s));
        }
        HIP(hipGetLastError());
        HIP(hipEventSynchronize(tu.ev[2 * kSigVariants - 1]));
        float best_ms = 0;
        for (int v = 0; v < kSigVariants; ++v) {
          float ms = 0;
          HIP(hipEventElapsedTime(&ms, tu.ev[2 * v], tu.ev[2 * v + 1]));
          if (v == 0 || ms < best_ms) { best_ms = ms; variant = v; }
        }
        tu.best[tkey] = variant;
        tuned_now = true;
        if (std::getenv("DFAMIN_TRACE"))
          std::fprintf(stderr, "[dfamin] tuned class 0x%x (m=%llu): variant %d, %.3f ms\n", tkey,
                       (unsigned long long)m, variant, best_ms);
      }
    }
    const bool cleared = spec_clear >= tsize;  // by the previous round's tail
    if (direct) {
      // (the group counters are cleared with the count table: a hash table
      // cleared ahead would no longer come with cleared counters)
      spec_clear = 0;
      if (dwidth > dtab_ready) {  // else cleared behind the last round's copy
        TRY(ensure(d_dtab_, 4ull << dwidth));
        prof.begin(s, "clear_table", 4.0 * (double)(1ull << dwidth));
        launch_clear_table(d_dtab_.as<Slot>(), 1ull << (dwidth - 1), d_ctrl_.as<Ctrl>(), s, 0, gcount);
        prof.end(s);
      }
      prof.begin(s, "signature", md * sig_bytes());
      launch_signature(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                       d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), d_dense_.p, dense_width,
                       d_table_.as<Slot>(), tbits, d_slot_of_.as<uint32_t>(), salt, d_ctrl_.as<Ctrl>(),
                       variant, s, (int)cas_bits_, nullptr, gcount, d_dtab_.as<uint32_t>());
      prof.end(s);
    } else if (!tuned_now) {
      spec_clear = 0;
      if (!cleared) {
        prof.begin(s, "clear_table", 8.0 * (double)tsize);
        launch_clear_table(d_table_.as<Slot>(), tsize, d_ctrl_.as<Ctrl>(), s, 0, gcount);
        prof.end(s);
      }
      prof.begin(s, "signature", md * sig_bytes());
      launch_signature(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                       d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), d_dense_.p, dense_width,
                       d_table_.as<Slot>(), tbits, d_slot_of_.as<uint32_t>(), salt, d_ctrl_.as<Ctrl>(),
                       variant, s, (int)cas_bits_, d_notify_.as<uint8_t>(), gcount);
      prof.end(s);
    } else {
      spec_clear = 0;
    }
    dtab_ready = 0;  // the count table cleared ahead serves this round only
    // (through the hash table, lone claimers must be marked: no tuning run)
    const bool slot_round = slot_cand && (direct || (!tuned_now && tbits <= 31));
    if (slot_round) {
      // blocks among the active states: every state off the list is a
      // singleton block of its own
      const uint64_t before = cnt[i0] - (in_[i0].n - m);
      launch_prep_scan(d_status_.as<unsigned long long>(), ntiles, d_ctrl_.as<Ctrl>(), s);
      prof.begin(s, "compact", md * (4 + 4 + 1 + 4 + 4));
      launch_compact(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), nullptr, nullptr,
                     d_changed_.as<uint32_t>(), nullptr, d_block_.as<uint32_t>(), nxt, d_ctrl_.as<Ctrl>(),
                     d_status_.as<unsigned long long>(), citems, s, 0, d_slot_of_.as<uint32_t>(),
                     d_notify_.as<uint8_t>(), gcount, (uint32_t)before, direct ? d_dtab_.as<uint32_t>() : nullptr);
      prof.end(s);
    } else {
      prof.begin(s, "resolve", md * (4 + inst_b + 4 + 8 + 4 + 4 + 1));
      launch_resolve(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                     d_table_.as<Slot>(), d_slot_of_.as<uint32_t>(),
                     d_block_.as<uint32_t>(), d_nb_.as<uint32_t>(), d_keep_.as<uint8_t>(),
                     d_changed_.as<uint32_t>(), d_ctrl_.as<Ctrl>(),
                     d_status_.as<unsigned long long>(), ntiles, s, 0,
                     tuned_now ? nullptr : d_notify_.as<uint8_t>(), slot_prev ? gcount : nullptr);
      prof.end(s);
      prof.begin(s, "compact", md * (4 + inst_b + 4 + 1 + 4));
      launch_compact(batch, cur, (uint32_t)m, d_inst_of_.as<uint32_t>(), d_nb_.as<uint32_t>(),
                     d_keep_.as<uint8_t>(), d_changed_.as<uint32_t>(), nullptr, d_block_.as<uint32_t>(),
                     nxt, d_ctrl_.as<Ctrl>(), d_status_.as<unsigned long long>(), citems, s);
      prof.end(s);
    }
    // Exact block counts for the next round, queued before the one sync of
    // the round: instances that were refining before this round and whose
    // next signature could fit 31 bits, B <= min(n, B^(kp+1)) after it.
    scan.clear();
    for (uint32_t i : alist)
      if (would_scan(i)) scan.push_back((uint32_t)i);
    const uint32_t ns = (uint32_t)scan.size();
    uint32_t* hs = hj + 2 * I;
    uint32_t* ds = dj + 2 * I;
    uint32_t stiles = 0;
    double sstates = 0;
    int sitems = kScanItemsSmall;
    if (ns) {
      for (uint32_t j = 0; j < ns; ++j) sstates += in_[scan[j]].n;
      sitems = scan_items_for((uint64_t)sstates);
      for (uint32_t j = 0; j < ns; ++j) {
        hs[j] = scan[j];
        hs[ns + j] = stiles;
        stiles += scan_tiles(in_[scan[j]].n, sitems);
      }
      TRY(ensure(d_status_, ((size_t)stiles + 1) * 8));
    }
    // round counters; also clears the scan status for the count scan
    launch_round_end((uint32_t)I, d_changed_.as<uint32_t>(), d_refine_.as<uint32_t>(), nullptr,
                     d_ctrl_.as<Ctrl>(), s, ns ? d_status_.as<unsigned long long>() : nullptr, stiles);
    if (ns) {
      TRY(upload_if_changed(up_scan, hs, ds, 2 * ns));
      prof.begin(s, "scan_jobs", 8.0 * sstates);
      launch_scan_jobs(d_desc_.as<InstDesc>(), ds, ds + ns, ns, stiles, d_block_.as<uint32_t>(),
                       d_rank_.as<uint32_t>(), d_counts_.as<uint32_t>(), d_ctrl_.as<Ctrl>(),
                       d_status_.as<unsigned long long>(), sitems, s);
      prof.end(s);
    }
    HIP(hipGetLastError());
    // one copy: control block, refine counters, and the counts just scanned
    TRY(readback(h_rb_, d_rb_.p, sizeof(Ctrl) + 4 * I + 4 * (size_t)ns, s));
    // Work of the next round that needs none of this round's results is
    // queued behind the copy and runs while the host waits and plans: the
    // next level of each doubling instance (j grows by this round's step; if
    // the round is redone, the level is just ready early) and a cleared table
    // of this round's size, which the next round uses when its own table is
    // no larger (table sizes mostly shrink with m).  Only small tables are
    // cleared ahead: after the last round the clear is wasted, and a large
    // one would then delay the final numbering.  The host waits for the copy
    // alone; with profiling on it waits for everything, so that every timed
    // launch has finished when the times are collected.
    const bool overlap = !prof.enabled();
    if (overlap) {
      if (!ev_rb_) HIP(hipEventCreateWithFlags(&ev_rb_, hipEventDisableTiming));
      HIP(hipEventRecord(ev_rb_, s));
      for (uint32_t i : alist) {
        if (!dbl[i] || !lazy[i]) continue;
        const uint32_t nrows = (uint32_t)inst_rows_[i].size();
        uint32_t lvl = (uint32_t)floor_log2_u64(mj[i] + step[i] + 1);
        if (lvl > nrows - 1) lvl = nrows - 1;
        for (uint32_t l = built[i] + 1; l <= lvl; ++l) todo.push_back({i, l, l - built[i] - 1});
        if (built[i] < lvl) built[i] = lvl;
      }
      if (!todo.empty()) {
        TRY(queue_levels(todo, s));
        todo.clear();
      }
      if (slot_round) {
        // a hash round follows if this one split: its table (at most twice
        // this round's active states) is cleared now, while the host plans
        const uint64_t next = 1ull << std::max<uint32_t>(9, ceil_log2_u64(2 * m));
        TRY(ensure(d_table_, next * sizeof(Slot)));
        launch_clear_table(d_table_.as<Slot>(), next, d_ctrl_.as<Ctrl>(), s, 0, gcount);
        HIP(hipGetLastError());
        spec_clear = next;
      } else if (tsize <= kClearAheadSlots) {
        launch_clear_table(d_table_.as<Slot>(), tsize, d_ctrl_.as<Ctrl>(), s, 0, gcount);
        HIP(hipGetLastError());
        spec_clear = tsize;
      }
    }
    const auto tp2 = now();
    t_issue += us(tp1, tp2);
    HIP(overlap ? event_wait(ev_rb_) : stream_wait(s));
    stage_flip();  // every upload of the previous round has run
    const auto tp3 = now();
    t_wait += us(tp2, tp3);
    prof.collect();
    const Ctrl c = *h_rb_.as<Ctrl>();
    const uint32_t* h_refine = reinterpret_cast<const uint32_t*>(h_rb_.as<char>() + sizeof(Ctrl));
    const uint32_t* h_cnt = h_refine + I;
    if (c.fault) return DFAMIN_E_INTERNAL;
    std::fill(cnt_ok.begin(), cnt_ok.end(), 0);
    for (uint32_t j = 0; j < ns; ++j) {
      cnt[scan[j]] = h_cnt[j];
      cnt_ok[scan[j]] = 1;
    }
    if (prof.enabled() && std::getenv("DFAMIN_TRACE"))
      std::fprintf(stderr,
                   "[dfamin] round %llu: m=%llu table=2^%u next=%u changed=%u collision=%u exact=%zu slot=%d "
                   "direct=%d\n",
                   (unsigned long long)rounds + 1, (unsigned long long)m, tbits, c.m_next, c.any_changed,
                   c.collision, exact.size(), (int)slot_round, (int)direct);
    if (c.collision) {
      // the partition is unchanged, so the counts just taken still hold
      if (++retries > (int)kMaxSaltRetries) return DFAMIN_E_INTERNAL;
      salt = mix64(salt + 0x9E3779B97F4A7C15ull);
      continue;
    }
    ++rounds;
    retries = 0;  // the bound is on redoing one round
    settle(h_refine);
    dense_from_labels = false;
    slot_prev = slot_round;
    // one instance, and this round split blocks and kept no state (every
    // block is a singleton), or counted n blocks
    if (I == 1) all_single_ = (c.any_changed && c.m_next == 0) || (cnt_ok[0] && cnt[0] >= in_[0].n);
    // (a slot round that kept every state may have left its list in place)
    if (!(slot_round && c.m_next == m)) std::swap(cur, nxt);
    m = c.m_next;
    t_post += us(tp3, now());
    if (!c.any_changed) break;
  }
  if (trace)
    std::fprintf(stderr,
                 "[dfamin] host us over %llu rounds: plan %.0f (closure %.0f, descriptors %.0f in %u rounds) "
                 "issue %.0f wait %.0f post %.0f\n",
                 (unsigned long long)rounds, t_plan, t_closure, t_desc, n_dirty, t_issue, t_wait, t_post);

  return DFAMIN_OK;
}

// Leader-election rounds (Algorithm 2, Section 3.2) over all states.  Rounds
// are queued ahead of the host -- each one returns at once after a round that
// split nothing (ctrl->stop) -- and, unless DFAMIN_FLAG_NO_GRAPH is set or
// kernels are being profiled, replayed from a captured HIP graph of
// kGraphRounds rounds (kernels only).  With closure AUTO, auto_rounds rounds
// run on Sigma first; instances that split a block in every one of them then
// get the closure letters (the paper's transPR is closure ON with this method).
int Engine::leader_rounds(const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s) {
  const size_t I = in_.size();
  const bool batch = I > 1;
  const uint32_t N = (uint32_t)N_;
  Profiler& prof = ctx_->prof;
  uint32_t* nl[2] = {d_nb_.as<uint32_t>(), d_slot_of_.as<uint32_t>()};
  uint8_t* differs = d_keep_.as<uint8_t>();
  HIP(hipMemsetAsync(nl[0], 0xff, (size_t)N * 4, s));
  HIP(hipMemsetAsync(nl[1], 0xff, (size_t)N * 4, s));
  uint64_t queued = 0;  // rounds queued so far: round r uses nl[r & 1]
  // the kernels' algorithmic bytes per state and round (no early exit)
  double kbar = 0;
  for (size_t i = 0; i < I; ++i) kbar += (double)desc_[i].n * desc_[i].kp;
  kbar = N ? kbar / N : 0.0;
  auto queue_direct = [&](uint64_t count) {
    for (uint64_t c = 0; c < count; ++c, ++queued) {
      prof.begin(s, "leader_round", (double)N * (4.0 + 16.0 * kbar + 1.0 + 9.0 + (batch ? 4.0 : 0.0)));
      launch_naive_round(batch, N, (uint32_t)I, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                         d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), nl[queued & 1], nl[(queued + 1) & 1],
                         differs, d_changed_.as<uint32_t>(), d_refine_.as<uint32_t>(), d_ctrl_.as<Ctrl>(), s);
      prof.end(s);
    }
  };
  auto read_ctrl = [&](Ctrl& c) -> int {
    HIP(hipGetLastError());
    TRY(readback(h_rb_, d_rb_.p, sizeof(Ctrl) + 4 * I, s));
    HIP(stream_wait(s));
    stage_idle();
    prof.collect();
    c = *h_rb_.as<Ctrl>();
    if (c.fault) return DFAMIN_E_INTERNAL;
    if (c.iterations > max_rounds) return DFAMIN_E_INTERNAL;
    return DFAMIN_OK;
  };
  Ctrl c{};
  bool any_auto = false;
  for (auto& x : in_) any_auto |= (x.closure == DFAMIN_CLOSURE_AUTO);
  if (any_auto) {
    const uint32_t auto_rounds = opts.auto_rounds ? opts.auto_rounds : kDefaultAutoRounds;
    queue_direct(auto_rounds);
    TRY(read_ctrl(c));
    if (!c.stop) {
      const uint32_t* rc = reinterpret_cast<const uint32_t*>(h_rb_.as<char>() + sizeof(Ctrl));
      std::vector<uint32_t> which;
      for (size_t i = 0; i < I; ++i)
        if (in_[i].closure == DFAMIN_CLOSURE_AUTO && rc[i] == c.iterations) which.push_back((uint32_t)i);
      if (!which.empty()) {
        TRY(build_closure(which, opts, s));
        TRY(upload_layout(s));
      }
    }
  }
  const bool graphs = !(opts.flags & DFAMIN_FLAG_NO_GRAPH) && !prof.enabled() && s != nullptr;
  hipGraphExec_t exec = nullptr;
  if (graphs && !c.stop) {
    // capture kGraphRounds rounds starting at this parity, or reuse the
    // graph of an earlier call with the same pointers and sizes
    const GraphKey key{N, (uint32_t)I, (uint32_t)(queued & 1), d_inst_of_.p, d_desc_.p, d_rows_.p, d_block_.p,
                       nl[0], nl[1], differs, d_changed_.p, d_refine_.p, d_ctrl_.p, s};
    if (graph_exec_ && graph_key_ == key) {
      exec = graph_exec_;
    } else {
      if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
      graph_exec_ = nullptr;
      hipGraph_t g = nullptr;
      HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      const uint64_t q0 = queued;
      for (uint32_t r = 0; r < kGraphRounds; ++r)
        launch_naive_round(batch, N, (uint32_t)I, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                           d_rows_.as<uint64_t>(), d_block_.as<uint32_t>(), nl[(q0 + r) & 1],
                           nl[(q0 + r + 1) & 1], differs, d_changed_.as<uint32_t>(), d_refine_.as<uint32_t>(),
                           d_ctrl_.as<Ctrl>(), s);
      const hipError_t ce = hipStreamEndCapture(s, &g);
      if (ce != hipSuccess || !g) return check_hip(ce != hipSuccess ? ce : hipErrorUnknown);
      const hipError_t ie = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP(ie);
      graph_key_ = key;
      exec = graph_exec_;
    }
  }
  // queue batches of rounds; the host checks less and less often
  uint32_t per_check = 1;
  while (!c.stop) {
    for (uint32_t b = 0; b < per_check; ++b) {
      if (exec) {
        HIP(hipGraphLaunch(exec, s));
        queued += kGraphRounds;
      } else {
        queue_direct(kGraphRounds);
      }
    }
    TRY(read_ctrl(c));
    per_check = std::min<uint32_t>(per_check * 2, 64);
  }
  return DFAMIN_OK;
}

int Engine::minimal_dfa(const dfamin_opts& opts, hipStream_t s, uint32_t nb, uint32_t initial_block,
                        MinimalInfo& info, const uint32_t** min_delta, const uint8_t** min_acc) {
  if (in_.size() != 1) return DFAMIN_E_INVAL;
  const InstInput& x = in_[0];
  const uint32_t n = x.n, k = x.k;
  Profiler& prof = ctx_->prof;
  const size_t words = ((size_t)n + 31) / 32;
  TRY(ensure(d_visit_, words * 4));
  TRY(ensure(d_min_delta_, (size_t)k * n * 4));
  TRY(ensure(d_min_acc_, ((size_t)n + 7) / 8));
  TRY(ensure_host(h_jobs_, 64));
  uint32_t* visited = d_visit_.as<uint32_t>();
  uint32_t* frontier = d_act_.as<uint32_t>();
  uint32_t* next = d_act2_.as<uint32_t>();
  uint32_t* counter = d_counts_.as<uint32_t>();
  // start: visited = {q0}, frontier = [q0]
  uint32_t* hj = h_jobs_.as<uint32_t>();
  hj[0] = 1u << (x.q0 & 31u);
  hj[1] = x.q0;
  HIP(hipMemsetAsync(visited, 0, words * 4, s));
  HIP(hipMemcpyAsync(visited + (x.q0 >> 5), &hj[0], 4, hipMemcpyHostToDevice, s));
  HIP(hipMemcpyAsync(frontier, &hj[1], 4, hipMemcpyHostToDevice, s));
  // the rows followed: the non-identity letters, then their closure levels
  std::vector<uint64_t> rows = inst_rows_[0];
  bool closure_used = has_closure_[0] != 0;
  auto upload_rows = [&]() -> int {
    TRY(ensure(d_bfs_rows_, std::max<size_t>(rows.size(), 1) * 8));
    if (!rows.empty())
      HIP(hipMemcpyAsync(d_bfs_rows_.p, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, s));
    return DFAMIN_OK;
  };
  TRY(upload_rows());
  uint32_t fcount = 1, reached = 1, levels = 0;
  while (fcount) {
    if (levels == kBfsLevelsBeforeClosure && !closure_used && !nonid_[0].empty()) {
      // a long path: closure letters (words over Sigma) shorten it
      TRY(build_closure({0u}, opts, s));
      rows = inst_rows_[0];
      closure_used = true;
      TRY(upload_rows());
    }
    HIP(hipMemsetAsync(counter, 0, 4, s));
    prof.begin(s, "bfs_level", 4.0 * fcount * (1.0 + 3.0 * rows.size()));
    launch_bfs_level(d_bfs_rows_.as<uint64_t>(), (uint32_t)rows.size(), frontier, fcount, visited, next,
                     counter, s);
    prof.end(s);
    HIP(hipGetLastError());
    HIP(hipMemcpyAsync(&hj[2], counter, 4, hipMemcpyDeviceToHost, s));
    HIP(stream_wait(s));
    prof.collect();
    fcount = hj[2];
    reached += fcount;
    ++levels;
    std::swap(frontier, next);
  }
  // quotient of the reachable classes
  uint32_t* sel = d_nb_.as<uint32_t>();
  uint32_t* rid = d_rank_.as<uint32_t>();
  uint32_t* rep = d_slot_of_.as<uint32_t>();
  HIP(hipMemsetAsync(sel, 0xff, (size_t)nb * 4, s));
  TRY(ensure(d_status_, ((size_t)scan_tiles(nb, scan_items_for(nb)) + 1) * 8));
  prof.begin(s, "quotient", (double)n * 12.0 + (double)nb * (16.0 + 8.0 * k));
  launch_quotient(n, k, nb, x.delta, x.accept, d_block_.as<uint32_t>(), x.out, visited, sel, rid, rep,
                  d_min_delta_.as<uint32_t>(), d_keep_.as<uint8_t>(), d_min_acc_.as<uint8_t>(),
                  d_ctrl_.as<Ctrl>(), d_status_.as<unsigned long long>(), s);
  prof.end(s);
  HIP(hipGetLastError());
  HIP(hipMemcpyAsync(&hj[3], rid + nb, 4, hipMemcpyDeviceToHost, s));
  HIP(hipMemcpyAsync(&hj[4], rid + initial_block, 4, hipMemcpyDeviceToHost, s));
  HIP(hipMemcpyAsync(h_ctrl_.p, d_ctrl_.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP(stream_wait(s));
  prof.collect();
  if (h_ctrl_.as<Ctrl>()->fault) return DFAMIN_E_INTERNAL;
  info.n = hj[3];
  info.q0 = hj[4];
  info.reachable = reached;
  info.bfs_levels = levels;
  *min_delta = d_min_delta_.as<uint32_t>();
  *min_acc = d_min_acc_.as<uint8_t>();
  return DFAMIN_OK;
}

// ---------------------------------------------------------- fused kernels
uint32_t Engine::fused_limit(const dfamin_opts& opts) const {
  // the round engine's testing knobs (hash width, table insertion order)
  // and queued rounds concern its own rounds: those calls keep to it
  if (no_fused || opts.method != DFAMIN_METHOD_SIGNATURE || (opts.flags & DFAMIN_FLAG_QUEUE)) return 0;
  if (std::getenv("DFAMIN_HASH_BITS") || std::getenv("DFAMIN_CAS_FIRST")) return 0;
  uint32_t lim = kFusedMaxStates;
  if (const char* e = std::getenv("DFAMIN_FUSED_MAX_STATES")) {  // testing: 0 turns the fused path off
    const long v = std::atol(e);
    lim = v <= 0 ? 0u : (uint32_t)std::min<long>(v, (long)kFusedMaxStates);
  }
  return lim;
}

int Engine::fused_issue(const std::vector<InstInput>& in, const std::vector<uint32_t>& which,
                        const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s) {
  const size_t F = which.size();
  if (F > 1) TRY(ensure(d_fjobs_, F * sizeof(FusedJob)));
  TRY(ensure_host(h_fjobs_, F * sizeof(FusedJob)));
  TRY(ensure_host(h_fres_, F * sizeof(FusedRes)));
  // jobs grouped by size class, largest class first
  FusedJob* hj = h_fjobs_.as<FusedJob>();
  fused_pos_.assign(F, 0);
  uint32_t at = 0, start[4] = {0, 0, 0, 0};
  double bytes = 0;
  for (int cls = 2; cls >= 0; --cls) {
    start[cls] = at;
    for (size_t w = 0; w < F; ++w) {
      const InstInput& x = in[which[w]];
      if (fused_class(x.n) != cls) continue;
      FusedJob& J = hj[at];
      J.delta = reinterpret_cast<uint64_t>(x.delta);
      J.accept = reinterpret_cast<uint64_t>(x.accept);
      J.out = reinterpret_cast<uint64_t>(x.out);
      J.n = x.n;
      J.k = x.k;
      J.q0 = x.q0;
      J.closure = x.closure;
      uint32_t L = floor_log2_u32(x.n);
      if (opts.max_levels && opts.max_levels < L) L = opts.max_levels;
      J.levels = L;
      J.auto_rounds = opts.auto_rounds ? opts.auto_rounds : kDefaultAutoRounds;
      J.max_rounds = (uint32_t)std::min<uint64_t>(max_rounds, 0xFFFFFFFFull);
      J.pad = 0;
      fused_pos_[w] = at++;
      // transitions read once for validation, accept bits, the output write
      bytes += 4.0 * x.n * x.k + x.n / 8.0 + 4.0 * x.n;
    }
  }
  start[3] = at;
  // The kernels write their results straight into the mapped page-locked
  // buffer the host reads after its wait; one job travels as a kernel
  // argument, so a single small instance costs one launch and no copies.
  FusedRes* res = static_cast<FusedRes*>(h_fres_.dp);
  if (F > 1) launch_copy_bytes(d_fjobs_.p, h_fjobs_.dp, F * sizeof(FusedJob), s);
  Profiler& prof = ctx_->prof;
  prof.begin(s, "fused", bytes);
  if (F == 1) {
    launch_fused(nullptr, res, 1, fused_class(hj[0].n), s, &hj[0]);
  } else {
    for (int cls = 2; cls >= 0; --cls) {
      const uint32_t b = start[cls], e = cls == 0 ? start[3] : start[cls - 1];
      launch_fused(d_fjobs_.as<FusedJob>() + b, res + b, e - b, cls, s);
    }
  }
  prof.end(s);
  return check_hip(hipGetLastError());
}

int Engine::fused_collect(const std::vector<InstInput>& in, const std::vector<uint32_t>& which,
                          std::vector<InstOutcome>& res, std::vector<uint32_t>& handoff) {
  (void)in;
  const FusedRes* r = h_fres_.as<FusedRes>();
  int rc = DFAMIN_OK;
  for (size_t w = 0; w < which.size(); ++w) {
    const FusedRes& f = r[fused_pos_[w]];
    InstOutcome& o = res[which[w]];
    switch (f.status) {
      case kFusedOk:
        o.num_blocks = f.num_blocks;
        o.initial_block = f.initial_block;
        o.refine_rounds = f.refine_rounds;
        o.rounds_executed = f.refine_rounds + 1;
        // a doubling instance reports the levels its rounds read, as the
        // round engine does
        o.closure_levels = f.doubling ? f.levels_used : 0;
        o.closure_letters = f.doubling ? f.levels_used + 1 : 0;
        o.status = DFAMIN_OK;
        break;
      case kFusedHandOff:
        handoff.push_back(which[w]);
        break;
      case kFusedBad:
        o.status = DFAMIN_E_BAD_DFA;
        if (rc == DFAMIN_OK) rc = DFAMIN_E_BAD_DFA;
        break;
      default:
        rc = DFAMIN_E_INTERNAL;
        break;
    }
  }
  return rc;
}

// Small instances are minimized whole by the fused kernels (one workgroup
// each, every round in LDS), the others by the round engine.  A single
// small instance is validated inside its kernel; a batch is validated as a
// whole first, so that a bad instance leaves every output untouched.  The
// fused kernels go to the stream ahead of the round engine's work; an
// instance they hand back (it needs closure letters) then runs through the
// round engine as well.
int Engine::run_all(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
                    std::vector<InstOutcome>& res) {
  const size_t I = in.size();
  const uint32_t lim = fused_limit(opts);
  std::vector<uint32_t> small, big;
  uint32_t nmax = 0;
  uint64_t N = 0;
  for (size_t i = 0; i < I; ++i) {
    nmax = std::max(nmax, in[i].n);
    N += in[i].n;
    const bool ok = in[i].n <= lim && in[i].k <= kFusedMaxLetters &&
                    (in[i].closure == DFAMIN_CLOSURE_AUTO || in[i].closure == DFAMIN_CLOSURE_OFF);
    (ok ? small : big).push_back((uint32_t)i);
  }
  if (small.empty() || N >= kMaxStates) return run_path(in, opts, s, res);
  const uint64_t max_rounds = opts.max_rounds ? opts.max_rounds : (uint64_t)nmax + 1;
  res.assign(I, InstOutcome{});
  std::vector<uint32_t> handoff;
  // (the letter lists are members that keep their capacity from call to
  // call: a batch of thousands of instances then allocates none of them)
  auto subset = [&](const std::vector<uint32_t>& idx, std::vector<InstInput>& sub,
                    std::vector<std::vector<uint32_t>>& sub_nonid, const std::vector<std::vector<uint32_t>>& all) {
    sub.clear();
    if (sub_nonid.size() < idx.size()) sub_nonid.resize(idx.size());
    for (size_t t = 0; t < idx.size(); ++t) {
      sub.push_back(in[idx[t]]);
      sub_nonid[t].assign(all[idx[t]].begin(), all[idx[t]].end());
    }
  };
  auto run_subset = [&](const std::vector<uint32_t>& idx, const std::vector<std::vector<uint32_t>>& all) {
    std::vector<InstInput> sub;
    subset(idx, sub, sub_nonid_, all);
    std::vector<InstOutcome> sub_res;
    const int rc = run_path(sub, opts, s, sub_res, &sub_nonid_);
    if (rc == DFAMIN_OK)
      for (size_t t = 0; t < idx.size(); ++t) res[idx[t]] = sub_res[t];
    return rc;
  };
  if (I == 1) {
    stage_idle();
    TRY(fused_issue(in, small, opts, max_rounds, s));
    HIP(stream_wait(s));
    ctx_->prof.collect();
    TRY(fused_collect(in, small, res, handoff));
    if (handoff.empty()) return DFAMIN_OK;
    return run_path(in, opts, s, res);
  }
  const bool trace = std::getenv("DFAMIN_TRACE") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  auto us_since = [&](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - a).count();
  };
  in_ = in;
  stage_idle();
  stage_cur_ = 0;
  TRY(validate(s, res));
  const double t_valid = us_since(t0);
  // this call's letter lists, kept apart from nonid_, which the subsets' runs
  // overwrite (the swap hands nonid_ the previous call's lists to reuse)
  vnonid_.swap(nonid_);
  const std::vector<std::vector<uint32_t>>& nonid_all = vnonid_;
  // With larger instances in the call, the fused kernels run on their own
  // stream beside the round engine's rounds (whose host syncs leave the GPU
  // idle now and then), after this call's validation.
  hipStream_t fs = s;
  // (with kernel timing on, everything stays on one stream: the profiler
  // collects a launch's events after that stream's waits)
  if (!big.empty() && !fixed() && !ctx_->prof.enabled()) {
    if (!fused_stream_) {
      HIP(hipStreamCreateWithFlags(&fused_stream_, hipStreamNonBlocking));
      HIP(hipEventCreateWithFlags(&fused_ready_, hipEventDisableTiming));
      HIP(hipEventCreateWithFlags(&fused_done_, hipEventDisableTiming));
    }
    HIP(hipEventRecord(fused_ready_, s));
    HIP(hipStreamWaitEvent(fused_stream_, fused_ready_, 0));
    fs = fused_stream_;
  }
  const double t_pre = us_since(t0);
  int frc = fused_issue(in, small, opts, max_rounds, fs);
  if (frc == DFAMIN_OK && fs != s) frc = check_hip(hipEventRecord(fused_done_, fs));
  const double t_fused = us_since(t0);
  if (frc == DFAMIN_OK && !big.empty()) frc = run_subset(big, nonid_all);
  if (trace)
    std::fprintf(stderr, "[dfamin] batch of %zu (%zu fused): host us to validation %.0f, to fused issue %.0f, "
                 "fused issued %.0f, round engine done %.0f\n", I, small.size(), t_valid, t_pre, t_fused,
                 us_since(t0));
  if (frc != DFAMIN_OK) {
    if (fs != s && !ctx_->device_lost) (void)hipStreamSynchronize(fs);  // nothing of the call left queued
    return frc;
  }
  HIP(stream_wait(s));
  if (fs != s) HIP(hipEventSynchronize(fused_done_));
  ctx_->prof.collect();
  TRY(fused_collect(in, small, res, handoff));
  if (!handoff.empty()) TRY(run_subset(handoff, nonid_all));
  return DFAMIN_OK;
}

int Engine::run(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
                std::vector<InstOutcome>& res) {
  if (fixed()) reset_fixed_region();
  const int rc = run_all(in, opts, s, res);
  // A call that stops early may leave work queued behind its last wait (the
  // next round's level passes and table clear): let it finish before the
  // buffers are handed to another call.
  if (rc != DFAMIN_OK && !ctx_->device_lost) (void)hipStreamSynchronize(s);
  return rc;
}

// Validation (Section 2: every transition target < n) and the non-identity
// letters of every instance of in_: one row job per (instance, letter).
int Engine::validate(hipStream_t s, std::vector<InstOutcome>& res) {
  const size_t I = in_.size();
  Profiler& prof = ctx_->prof;
  const bool trace = std::getenv("DFAMIN_TRACE") != nullptr;
  const auto v0 = std::chrono::steady_clock::now();
  auto us_since = [&](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - a).count();
  };
  double t_jobs = 0, t_issue = 0, t_wait = 0;
  // (the job vectors are members, so a call of the same shape allocates nothing)
  size_t njobs = 0;
  for (auto& x : in_) njobs += x.k;
  std::vector<RowJob>& jobs = vjobs_;
  std::vector<uint32_t>& joboff = vjoboff_;
  jobs.resize(njobs);
  joboff.resize(njobs);
  uint32_t wgs = 0;
  {
    size_t j = 0;
    for (size_t i = 0; i < I; ++i)
      for (uint32_t a = 0; a < in_[i].k; ++a, ++j) {
        RowJob& J = jobs[j];
        J.src = reinterpret_cast<uint64_t>(in_[i].delta) + 4ull * a * in_[i].n;
        J.dst = 0;
        J.n = in_[i].n;
        J.flag_idx = (uint32_t)j;
        joboff[j] = wgs;
        wgs += (J.n + kLongTile - 1) / kLongTile;
      }
  }
  TRY(ensure(d_jobs_, jobs.size() * sizeof(RowJob)));
  TRY(ensure(d_joboff_, joboff.size() * 4));
  TRY(ensure(d_flags_, jobs.size() * 4));
  TRY(ensure(d_wgflags_, (size_t)wgs * 4));
  TRY(ensure_host(h_flags_, jobs.size() * 4));
  t_jobs = us_since(v0);
  TRY(stage_copy(d_jobs_.p, jobs.data(), jobs.size() * sizeof(RowJob), s));
  TRY(stage_copy(d_joboff_.p, joboff.data(), joboff.size() * 4, s));
  TRY(queue_fill(d_flags_.p, 0, jobs.size() * 4, s));
  TRY(flush_segs(s));
  {
    double bytes = 0;
    for (auto& x : in_) bytes += 4.0 * x.n * x.k;
    prof.begin(s, "validate", bytes);
    launch_row_check(d_jobs_.as<RowJob>(), d_joboff_.as<uint32_t>(), (uint32_t)jobs.size(), wgs,
                     d_wgflags_.as<uint32_t>(), d_flags_.as<uint32_t>(), s);
    prof.end(s);
    HIP(hipGetLastError());
  }
  TRY(readback(h_flags_, d_flags_.p, jobs.size() * 4, s));
  t_issue = us_since(v0);
  HIP(stream_wait(s));
  t_wait = us_since(v0);
  stage_idle();
  prof.collect();
  bool any_bad = false;
  if (nonid_.size() < I) nonid_.resize(I);  // (longer lists are left as they are)
  {
    // jobs are ordered (instance, letter): job j of instance i is letter j - first(i)
    const uint32_t* f = h_flags_.as<uint32_t>();
    size_t j = 0;
    for (size_t i = 0; i < I; ++i) {
      std::vector<uint32_t>& letters = nonid_[i];
      letters.clear();
      for (uint32_t a = 0; a < in_[i].k; ++a, ++j) {
        const uint32_t fl = f[j];
        if (fl & kFlagBad) {
          res[i].status = DFAMIN_E_BAD_DFA;
          any_bad = true;
        }
        if (fl & kFlagNonId) letters.push_back(a);
      }
    }
  }
  if (trace)
    std::fprintf(stderr, "[dfamin] validation of %zu rows: host us jobs %.0f, issued %.0f, waited %.0f, done %.0f\n",
                 jobs.size(), t_jobs, t_issue, t_wait, us_since(v0));
  return any_bad ? DFAMIN_E_BAD_DFA : DFAMIN_OK;
}

int Engine::run_path(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
                     std::vector<InstOutcome>& res, const std::vector<std::vector<uint32_t>>* nonid) {
  in_ = in;
  const size_t I = in_.size();
  res.assign(I, InstOutcome{});
  if (I == 0) return DFAMIN_OK;
  const bool batch = I > 1;
  uint64_t N = 0;
  uint32_t nmax = 0;
  for (auto& x : in_) { N += x.n; nmax = std::max(nmax, x.n); }
  if (N >= kMaxStates) return DFAMIN_E_INVAL;  // state ids are 31-bit in hash slots
  N_ = N;
  closure_cursor_ = 0;
  // the previous call ended with its stream drained (run() drains on errors)
  stage_idle();
  stage_cur_ = 0;
  Profiler& prof = ctx_->prof;
  // host time per phase of the call (printed with DFAMIN_TRACE)
  const bool trace = std::getenv("DFAMIN_TRACE") != nullptr;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto us = [](auto a, auto b) { return std::chrono::duration<double, std::micro>(b - a).count(); };
  const auto t_start = now();

  // ---- 1. validation + identity letters (unless the call has done it)
  if (nonid) {
    // element by element: the lists keep their capacity (nonid_ may stay
    // longer than this call's instances)
    if (nonid_.size() < I) nonid_.resize(I);
    for (size_t i = 0; i < I; ++i) nonid_[i].assign((*nonid)[i].begin(), (*nonid)[i].end());
  } else {
    TRY(validate(s, res));
  }
  const auto t_valid = now();

  // ---- 2. descriptors and signature letters
  desc_.assign(I, InstDesc{});
  inst_rows_.resize(I);
  for (auto& r : inst_rows_) r.clear();
  levels_.assign(I, 0);
  has_closure_.assign(I, 0);
  {
    uint64_t off = 0;
    for (size_t i = 0; i < I; ++i) {
      InstDesc& D = desc_[i];
      D.state_off = (uint32_t)off;
      D.n = in_[i].n;
      D.k = in_[i].k;
      D.q0 = in_[i].q0;
      D.accept = reinterpret_cast<uint64_t>(in_[i].accept);
      D.out = reinterpret_cast<uint64_t>(in_[i].out);
      off += in_[i].n;
      for (uint32_t a : nonid_[i])
        inst_rows_[i].push_back(reinterpret_cast<uint64_t>(in_[i].delta) + 4ull * a * in_[i].n);
    }
  }
  const auto t_desc = now();
  {
    std::vector<uint32_t> on;
    for (size_t i = 0; i < I; ++i)
      if (in_[i].closure == DFAMIN_CLOSURE_ON) on.push_back((uint32_t)i);
    if (!on.empty()) TRY(build_closure(on, opts, s));
  }
  const auto t_closure = now();

  // ---- 3. buffers sized for N
  TRY(ensure(d_block_, N * 4));
  TRY(ensure(d_act_, N * 4));
  TRY(ensure(d_act2_, N * 4));
  TRY(ensure(d_slot_of_, N * 4));
  TRY(ensure(d_nb_, N * 4));
  TRY(ensure(d_keep_, N));
  TRY(ensure(d_notify_, N));
  TRY(ensure(d_rank_, (N + 1) * 4));
  const uint64_t max_tiles = scan_tiles(N, kScanItemsSmall) + 1;
  TRY(ensure(d_status_, max_tiles * 8));
  TRY(ensure(d_changed_, I * 4));
  // control block, per-instance refine counters and block counts share one
  // allocation so that a round's results come back in one copy
  TRY(ensure(d_rb_, sizeof(Ctrl) + 8 * I));
  d_ctrl_.p = d_rb_.p;
  d_ctrl_.cap = sizeof(Ctrl);
  d_refine_.p = static_cast<char*>(d_rb_.p) + sizeof(Ctrl);
  d_refine_.cap = 4 * I;
  d_counts_.p = static_cast<char*>(d_rb_.p) + sizeof(Ctrl) + 4 * I;
  d_counts_.cap = 4 * I;
  TRY(ensure_host(h_rb_, sizeof(Ctrl) + 8 * I));
  TRY(ensure(d_minF_, I * 4));
  TRY(ensure(d_minN_, I * 4));
  TRY(ensure(d_results_, I * sizeof(ResultDev)));
  TRY(ensure(d_inst_off_, I * 4));
  if (batch) TRY(ensure(d_inst_of_, N * 4));
  TRY(ensure_host(h_ctrl_, sizeof(Ctrl)));
  TRY(ensure_host(h_results_, I * sizeof(ResultDev)));
  TRY(ensure_host(h_counts_, I * 4));
  // One-letter AUTO instances refine by doubling from the first signature
  // round (their levels are built as the rounds read them); planning their
  // level storage here lets the layout go up once.  Those whose storage does
  // not fit stay plain until the AUTO closure is decided.
  lazy_.assign(I, 0);
  if (opts.method == DFAMIN_METHOD_SIGNATURE) {
    std::vector<uint32_t> uni, rest;
    for (size_t i = 0; i < I; ++i)
      if (in_[i].closure == DFAMIN_CLOSURE_AUTO && nonid_[i].size() == 1) uni.push_back((uint32_t)i);
    if (!uni.empty()) TRY(lazy_levels(uni, opts, rest, lazy_));
  }
  const auto t_bufs = now();
  // testing: force the table insertion order of every signature round
  // (DFAMIN_CAS_FIRST=b: bit 0 hash-mode states, bit 1 exact-key states)
  cas_forced_ = -1;
  if (const char* e = std::getenv("DFAMIN_CAS_FIRST")) cas_forced_ = (std::atoi(e) & 3) << 1;
  // testing: bit 0, the first round groups through the table as later
  // rounds do; bit 1, no slot labels; bit 2, no direct count tables
  {
    const char* e = std::getenv("DFAMIN_NO_LABELS");
    const int v = e ? std::atoi(e) : 0;
    label_off_ = (v & 1) != 0;
    slots_off_ = (v & 2) != 0;
    direct_off_ = (v & 4) != 0;
  }
  // The initial partition {F, Q\F} is not needed when the first round goes
  // by labels (every instance with at most kMaxLabelLetters signature
  // letters in that round; one-letter AUTO instances read one level), whose
  // kernels write every block id, the active list and the instance map.
  labels_planned_ = opts.method == DFAMIN_METHOD_SIGNATURE && !label_off_;
  label_bits_ = 1;
  for (size_t i = 0; i < I && labels_planned_; ++i) {
    const uint32_t kp0 = lazy_[i] ? 1u : (uint32_t)inst_rows_[i].size();
    if (kp0 > kMaxLabelLetters) labels_planned_ = false;
    label_bits_ = std::max(label_bits_, kp0 + 1);
  }
  // the first round's key mode (accept bits), so that no descriptor changes
  // for it unless a doubling instance reads one level
  for (size_t i = 0; i < I; ++i) {
    const uint32_t kp0 = lazy_[i] ? 1u : (uint32_t)inst_rows_[i].size();
    desc_[i].ebits = desc_[i].dsrc = kp0 + 1 <= 31 ? 1u : 0u;
  }
  // Descriptors, row pointers, init job offsets and the cleared per-call
  // state go out in one launch.
  TRY(upload_layout(s, true));
  const auto t_layout = now();
  // workgroup offsets of the per-instance init jobs
  std::vector<uint32_t> inst_off(I);
  uint32_t init_wgs = 0;
  for (size_t i = 0; i < I; ++i) {
    inst_off[i] = init_wgs;
    init_wgs += (in_[i].n + kRowTile - 1) / kRowTile;
  }
  init_wgs_ = init_wgs;
  TRY(stage_copy(d_inst_off_.p, inst_off.data(), I * 4, s));
  TRY(ensure(d_part_, (size_t)init_wgs * 8));
  TRY(queue_fill(d_changed_.p, 0, I * 4, s));
  // joiners' marks of lone slot claimers (each round's resolve step returns
  // the ones it reads to 0)
  TRY(queue_fill(d_notify_.p, 0, N, s));
  TRY(queue_fill(d_refine_.p, 0, I * 4, s));
  TRY(queue_fill(d_ctrl_.p, 0, sizeof(Ctrl), s));
  if (labels_planned_) {
    // the first round's least member per label: all ones (none yet); then
    // the labels' numbers, one or two bytes each
    const size_t nl = label_bits_ <= 8 ? 256 : 512;
    TRY(ensure(d_lbl_, I * nl * (label_bits_ <= 8 ? 5 : 6)));
    TRY(queue_fill(d_lbl_.p, 0xff, I * nl * 4, s));
  }
  TRY(flush_segs(s));
  if (const char* e = std::getenv("DFAMIN_HASH_BITS")) {
    // testing: weak signature hashes (see Ctrl::hash_mask)
    const int bits = std::atoi(e);
    if (bits >= 1 && bits < 64) {
      const uint64_t mask = (1ull << bits) - 1ull;
      launch_store_u64(&d_ctrl_.as<Ctrl>()->hash_mask, mask, s);
    }
  }

  // ---- 4. initial partition {F, Q\F} (unless the first round goes by labels)
  if (!labels_planned_) {
    prof.begin(s, "init_minmax", (double)N / 8.0);
    launch_init_minmax(d_desc_.as<InstDesc>(), d_inst_off_.as<uint32_t>(), (uint32_t)I, init_wgs,
                       d_part_.as<unsigned long long>(), d_minF_.as<uint32_t>(), d_minN_.as<uint32_t>(), s);
    prof.end(s);
    prof.begin(s, "init_block", (8.125 + (batch ? 4.0 : 0.0)) * (double)N);
    launch_init_block(d_desc_.as<InstDesc>(), d_inst_off_.as<uint32_t>(), (uint32_t)I, init_wgs,
                      d_minF_.as<uint32_t>(), d_minN_.as<uint32_t>(),
                      batch ? d_inst_of_.as<uint32_t>() : nullptr, d_block_.as<uint32_t>(),
                      d_act_.as<uint32_t>(), s);
    prof.end(s);
    HIP(hipGetLastError());
  }

  // ---- 5. rounds
  const auto t_setup = now();
  all_single_ = false;
  {
    const uint64_t max_rounds = opts.max_rounds ? opts.max_rounds : (uint64_t)nmax + 1;
    TRY(opts.method == DFAMIN_METHOD_LEADER ? leader_rounds(opts, max_rounds, s)
                                            : signature_rounds(opts, max_rounds, s));
  }

  // ---- 6. canonical numbering and emission
  const auto t_rounds = now();
  if (opts.method == DFAMIN_METHOD_SIGNATURE && !batch && all_single_) {
    // every block a singleton: each state is its own least member
    prof.begin(s, "emit", 4.0 * (double)N);
    launch_identity_out(d_desc_.as<InstDesc>(), (uint32_t)N, d_refine_.as<uint32_t>(),
                        d_results_.as<ResultDev>(), s);
    prof.end(s);
  } else {
    const int fitems = scan_items_for(N);
    const uint32_t ntilesN = scan_tiles(N, fitems);
    launch_prep_scan(d_status_.as<unsigned long long>(), ntilesN, d_ctrl_.as<Ctrl>(), s);
    prof.begin(s, "scan_reps", 8.0 * (double)N);
    launch_scan_reps(d_block_.as<uint32_t>(), (uint32_t)N, d_rank_.as<uint32_t>(), d_ctrl_.as<Ctrl>(),
                     d_status_.as<unsigned long long>(), fitems, s);
    prof.end(s);
    prof.begin(s, "emit", (12.0 + (batch ? 4.0 : 0.0)) * (double)N);
    launch_emit(batch, (uint32_t)N, d_inst_of_.as<uint32_t>(), d_desc_.as<InstDesc>(),
                d_block_.as<uint32_t>(), d_rank_.as<uint32_t>(), s);
    prof.end(s);
    launch_results((uint32_t)I, d_desc_.as<InstDesc>(), d_rank_.as<uint32_t>(),
                   d_refine_.as<uint32_t>(), d_results_.as<ResultDev>(), s);
  }
  HIP(hipGetLastError());
  TRY(readback(h_results_, d_results_.p, I * sizeof(ResultDev), s));
  TRY(readback(h_ctrl_, d_ctrl_.p, sizeof(Ctrl), s));
  HIP(stream_wait(s));
  prof.collect();
  if (h_ctrl_.as<Ctrl>()->fault) return DFAMIN_E_INTERNAL;
  if (trace)
    std::fprintf(stderr,
                 "[dfamin] call of %zu instances, host us: validation %.0f, "
                 "setup %.0f (descriptors %.0f, closure %.0f, buffers %.0f, layout %.0f, init %.0f), "
                 "rounds %.0f, numbering %.0f\n",
                 I, us(t_start, t_valid),
                 us(t_valid, t_setup), us(t_valid, t_desc), us(t_desc, t_closure), us(t_closure, t_bufs),
                 us(t_bufs, t_layout), us(t_layout, t_setup), us(t_setup, t_rounds), us(t_rounds, now()));
  const ResultDev* r = h_results_.as<ResultDev>();
  for (size_t i = 0; i < I; ++i) {
    res[i].num_blocks = r[i].num_blocks;
    res[i].initial_block = r[i].initial_block;
    res[i].refine_rounds = r[i].refine_rounds;
    res[i].rounds_executed = r[i].refine_rounds + 1;
    res[i].closure_levels = has_closure_[i] ? levels_[i] : 0;
    res[i].closure_letters = has_closure_[i] ? (uint32_t)inst_rows_[i].size() : 0;
    res[i].status = DFAMIN_OK;
  }
  return DFAMIN_OK;
}

}  // namespace dfamin
