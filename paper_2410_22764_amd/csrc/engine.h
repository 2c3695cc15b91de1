// engine.h -- host-side driver of the refinement kernels (one context).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <array>
#include <map>
#include <vector>

#include "../../include/dfamin.h"
#include "internal.h"

namespace dfamin {

// A device buffer that only grows; its bytes count against the context budget.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Host staging buffer in pinned memory (grow-only).  dp is the same memory
// as the device addresses it (set for the engine's buffers, which are
// page-locked with hipHostMallocCoherent so that kernels may read and write
// them directly).
struct HostBuf {
  void* p = nullptr;
  void* dp = nullptr;
  size_t cap = 0;
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Per-kernel HIP-event timing.
class Profiler {
 public:
  ~Profiler();
  void set_enabled(bool on);
  bool enabled() const { return on_; }
  // Turn timing on or off without clearing the stats; returns the old state.
  bool swap_enabled(bool on) {
    const bool was = on_;
    on_ = on;
    return was;
  }
  // Record a start event for kernel `name`; `alg_bytes` is what it must move.
  void begin(hipStream_t s, const char* name, double alg_bytes);
  void end(hipStream_t s);
  // Accumulate every finished pair (call after a stream synchronisation).
  void collect();
  int copy_stats(dfamin_kernel_stat* out, int cap) const;

 private:
  struct Pending {
    int stat;
    hipEvent_t a, b;
    double bytes;
  };
  int stat_index(const char* name);
  hipEvent_t get_event();
  bool on_ = false;
  bool trace_ = false;  // DFAMIN_TRACE set: print every timed launch to stderr
  std::vector<dfamin_kernel_stat> stats_;
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> free_events_;
  Pending cur_{};
};

struct InstInput {
  uint32_t n, k, q0;
  uint32_t closure;      // DFAMIN_CLOSURE_*
  const uint32_t* delta; // device, letter-major
  const uint8_t* accept; // device bitmap
  uint32_t* out;         // device, n entries
};

struct MinimalInfo {
  uint32_t n = 0, q0 = 0, reachable = 0, bfs_levels = 0;
};

struct InstOutcome {
  uint32_t num_blocks = 0, initial_block = 0, refine_rounds = 0, rounds_executed = 0;
  uint32_t closure_levels = 0, closure_letters = 0;
  int32_t status = 0;
};

class Context;

// Runs the whole path for a set of instances that live in device memory.
class Engine {
 public:
  explicit Engine(Context* ctx) : ctx_(ctx) {}
  ~Engine();
  // On an error return, the stream has been drained: no work of the call is
  // left queued on the context's buffers (a later call may use another stream).
  int run(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
          std::vector<InstOutcome>& res);
  uint64_t device_bytes() const;
  // Fixed-region mode, for callers that cannot allocate.  Every device
  // buffer of a call is carved from [base, base + cap), which the engine
  // does not own; carving restarts at every call.  The host buffers are
  // page-locked here once with host_bytes each and never grow: a call that
  // would need more fails with DFAMIN_E_NOMEM, as does one whose device
  // buffers do not fit in the region.  Call once, at set-up.
  int set_fixed_region(void* base, size_t cap, size_t host_bytes);
  bool fixed() const { return fixed_base_ != nullptr; }

 private:
  // Instances of `in` in small_ ones minimized whole by the fused kernels
  // and the others by the round engine (run_path).
  int run_all(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
              std::vector<InstOutcome>& res);
  // nonid: the non-identity letters of each instance when the call has
  // already validated them (validation is then skipped), else nullptr.
  int run_path(const std::vector<InstInput>& in, const dfamin_opts& opts, hipStream_t s,
               std::vector<InstOutcome>& res, const std::vector<std::vector<uint32_t>>* nonid = nullptr);
  // Validation of every instance of in_ (entries < n) and its non-identity
  // letters (nonid_); DFAMIN_E_BAD_DFA marks res[i].status of bad ones.
  int validate(hipStream_t s, std::vector<InstOutcome>& res);
  // Largest instance the fused kernels take under these options (0: none).
  uint32_t fused_limit(const dfamin_opts& opts) const;
  // Queues the fused kernels for the instances `which` of `in`; they write
  // their results into h_fres_ (mapped, read after the stream has drained).
  int fused_issue(const std::vector<InstInput>& in, const std::vector<uint32_t>& which,
                  const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s);
  // Results of fused_issue's instances: res entries of the finished ones,
  // the handed-back ones in handoff; DFAMIN_E_BAD_DFA / _E_INTERNAL.
  int fused_collect(const std::vector<InstInput>& in, const std::vector<uint32_t>& which,
                    std::vector<InstOutcome>& res, std::vector<uint32_t>& handoff);
  int ensure(DevBuf& b, size_t bytes);
  int ensure_host(HostBuf& b, size_t bytes);
  // Closure level storage a call may still take: half of the context's
  // remaining budget, or a third of what is left of the fixed region (the
  // signature records of the levels need about as much again).
  uint64_t closure_cap() const;
  void reset_fixed_region();
  int build_closure(const std::vector<uint32_t>& which, const dfamin_opts& opts, hipStream_t s);
  // Closure levels of unary doubling instances, computed round by round.
  struct LevelTodo {
    uint32_t inst, level, step;
  };
  int lazy_levels(const std::vector<uint32_t>& which, const dfamin_opts& opts,
                  std::vector<uint32_t>& rest, std::vector<uint8_t>& lazy);
  int queue_levels(const std::vector<LevelTodo>& todo, hipStream_t s);
  // Host-to-device uploads of a call go through two page-locked arenas: the
  // bytes are staged at the arena's next free offset and a copy kernel moves
  // them in stream order.  An arena's space is reused only after a host wait
  // that every copy out of it precedes: stage_flip() after a signature
  // round's readback event (the arena used before the previous flip is free
  // then), stage_idle() after the stream has drained; an arena that runs out
  // drains the stream and grows.
  int upload(void* dst, const void* src, size_t bytes, hipStream_t s);
  // Copies staged like upload() and byte fills, queued and then issued as
  // one launch by flush_segs() (which a full queue calls by itself).
  int stage_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
  int queue_fill(void* dst, uint32_t byte, size_t bytes, hipStream_t s);
  int flush_segs(hipStream_t s);
  void stage_flip() {
    stage_cur_ ^= 1;
    stage_[stage_cur_].off = 0;
  }
  void stage_idle() { stage_[0].off = stage_[1].off = 0; }
  // device -> engine host buffer (page-locked, mapped) by a copy kernel
  int readback(HostBuf& h, const void* src, size_t bytes, hipStream_t s);
  int signature_rounds(const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s);
 public:
  // After run() on one instance: the states reachable from q0 (breadth
  // first; closure rows join as extra edges after 64 levels) and the
  // quotient of their classes.  nb / initial_block: run()'s num_blocks and
  // out[q0].  On return *min_delta (k*m entries, letter-major) and *min_acc
  // (ceil(m/8) bytes) point into device buffers owned by the engine.
  int minimal_dfa(const dfamin_opts& opts, hipStream_t s, uint32_t nb, uint32_t initial_block,
                  MinimalInfo& info, const uint32_t** min_delta, const uint8_t** min_acc);
 private:
  int leader_rounds(const dfamin_opts& opts, uint64_t max_rounds, hipStream_t s);
  int upload_layout(hipStream_t s, bool queued = false);
  int check_hip(hipError_t e);

  Context* ctx_;
  // host-side layout
  std::vector<InstInput> in_;
  std::vector<InstDesc> desc_;
  std::vector<uint64_t> rows_;                   // signature row pointers
  std::vector<std::vector<uint64_t>> inst_rows_;  // per instance
  std::vector<std::vector<uint32_t>> nonid_;      // per instance: non-identity letters
  std::vector<uint32_t> levels_;                  // closure levels built per instance
  std::vector<uint8_t> has_closure_;
  std::vector<uint32_t> row_base_;                // first row of each instance in rows_
  uint64_t N_ = 0;
  std::vector<DevBuf> closure_bufs_;  // closure level storage, reused across calls
  size_t closure_cursor_ = 0;
  // device buffers
  DevBuf d_desc_, d_rows_, d_jobs_, d_joboff_, d_flags_, d_inst_off_, d_minF_, d_minN_;
  DevBuf d_inst_of_, d_block_, d_act_, d_act2_, d_slot_of_, d_nb_, d_keep_, d_rank_;
  DevBuf d_sig_, d_table_, d_status_, d_changed_, d_refine_, d_results_, d_ctrl_;
  DevBuf d_wgflags_, d_part_, d_dense_, d_counts_, d_djobs_;
  DevBuf d_notify_;  // one byte per state: a joiner marked this lone slot claimer
  DevBuf d_lbl_;     // first round by labels: least member and number per (instance, label)
  DevBuf d_gcount_;  // group counters of a signature round
  DevBuf d_dtab_;    // direct count table of an exact-key round
  DevBuf d_visit_, d_bfs_rows_, d_min_delta_, d_min_acc_;
  DevBuf d_lvl_, d_lvl_wg_, d_lvl_flags_;  // level jobs of lazily built closure levels
  DevBuf d_rb_;  // owns d_ctrl_, d_refine_ and d_counts_ (views into it, reset every run)
  HostBuf h_ctrl_, h_flags_, h_results_, h_counts_, h_jobs_, h_rb_;
  struct Stage {
    HostBuf buf;
    size_t off = 0;
  };
  Stage stage_[2];
  MemSegs segs_{};  // queued copies and fills (stage_copy, queue_fill)
  uint32_t stage_cur_ = 0;
  std::vector<char> lvl_host_;  // level jobs being assembled
  std::vector<RowJob> vjobs_;    // validation jobs of a call
  std::vector<uint32_t> vjoboff_;
  std::vector<uint8_t> lazy_;    // per instance: levels built as the doubling rounds read them
  uint32_t cas_bits_ = 2;        // signature gmode bits 1-2 (table insertion order) of the round
  int cas_forced_ = -1;          // testing override of cas_bits_
  bool label_off_ = false;       // testing: the first round groups through the table
  bool slots_off_ = false;       // testing: no slot labels
  bool direct_off_ = false;      // testing: slot labels through the hash table only
  bool labels_planned_ = false;  // this call's first signature round goes by labels
  uint32_t label_bits_ = 1;      // bits of its widest label (kp + 1)
  std::vector<uint32_t> live_;   // per instance: still refining (after the first round)
  // a batched call's letter lists, and those of the subset passed to run_path
  std::vector<std::vector<uint32_t>> vnonid_, sub_nonid_;
  uint32_t init_wgs_ = 0;        // kRowTile-state jobs over all instances (d_inst_off_)
  bool all_single_ = false;      // single instance: the rounds ended with every block a singleton
  // captured leader-election rounds, reused while pointers and sizes match
  struct GraphKey {
    uint32_t n, ninst, parity;
    const void *inst_of, *desc, *rows, *block, *nl0, *nl1, *differs, *changed, *refine, *ctrl;
    hipStream_t stream;
    bool operator==(const GraphKey& o) const {
      return n == o.n && ninst == o.ninst && parity == o.parity && inst_of == o.inst_of && desc == o.desc &&
             rows == o.rows && block == o.block && nl0 == o.nl0 && nl1 == o.nl1 && differs == o.differs &&
             changed == o.changed && refine == o.refine && ctrl == o.ctrl && stream == o.stream;
    }
  };
  GraphKey graph_key_{};
  hipGraphExec_t graph_exec_ = nullptr;
  hipEvent_t ev_rb_ = nullptr;  // a signature round's readback, waited for by itself
  // captured queued signature rounds, reused while every pointer and size in
  // the key matches
  static constexpr int kQueueKeyWords = 24;
  std::array<uint64_t, kQueueKeyWords> queue_key_{};
  hipGraphExec_t queue_exec_ = nullptr;
  int queued_rounds(uint64_t m, uint32_t tbits, int variant, int items, uint64_t salt, uint32_t* cur,
                    uint32_t* nxt, uint64_t max_left, bool use_graph, const QueueDbl* dq, hipStream_t s,
                    uint64_t& executed);
  DevBuf d_qdbl_;   // per-instance doubling state of queued rounds
  HostBuf h_qdbl_;
  // fused kernels: jobs in class order, their results, and where each sits
  DevBuf d_fjobs_;
  HostBuf h_fjobs_, h_fres_;
  std::vector<uint32_t> fused_pos_;  // per entry of `which`: index in the job array
  // A batch's fused kernels run on their own stream beside the round
  // engine's work (created at the first batch; not in fixed-region mode,
  // which creates nothing after set-up): fused_ready_ on the caller's
  // stream after validation, fused_done_ behind the results' copy.
  hipStream_t fused_stream_ = nullptr;
  hipEvent_t fused_ready_ = nullptr, fused_done_ = nullptr;
 public:
  // Set by callers that read the round engine's buffers after run() (the
  // minimal DFA): every instance then goes through the round engine.
  bool no_fused = false;
 private:
  // fixed-region mode (set_fixed_region)
  char* fixed_base_ = nullptr;
  size_t fixed_cap_ = 0, fixed_off_ = 0;
};

// Signature-tile autotuner state of a context: a forced variant, or the
// fastest variant measured per size class.
struct Tuner {
  int forced = -1;
  std::map<uint32_t, int> best;
  hipEvent_t ev[2 * kSigVariants] = {};
  bool have_events = false;
};

// The object behind dfamin_ctx.
class Serving;
class Context {
 public:
  int device = 0;
  uint64_t budget = 0;
  uint64_t used = 0;
  hipStream_t stream = nullptr;  // internal stream for host-input calls
  Profiler prof;
  Tuner tuner;
  Engine engine{this};
  // the engine of dfamin_minimize_device_noalloc: its device buffers live in
  // the library's static scratch array of this device (fixed-region mode)
  Engine fixed_engine{this};
  // staging for host-input calls
  DevBuf in_delta, in_accept, in_out;
  HostBuf h_in, h_out;
  Serving* serving = nullptr;
  bool device_lost = false;
};

}  // namespace dfamin
