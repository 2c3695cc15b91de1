// internal.h -- device data layout and kernel launchers of libdfamin.
//
// Layout (all in HBM of one device):
//   * Instances are laid side by side in one global state space: instance i
//     owns global state ids [state_off, state_off + n).  Block ids are global
//     state ids too: the id of a block is its least member state.  Two
//     instances therefore never share a block id, which keeps every
//     instance's signatures apart when many are refined by one launch.
//   * delta stays in the caller's letter-major layout (Section 2,
//     "Representation"); each signature letter is a pointer to one row of n
//     local successor ids (an input row, or a closure level).
//   * act[] lists the global ids of the states still in non-singleton blocks
//     of instances still refining, in increasing order within each instance.
//     A singleton block can never split again, so its states leave the list.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <stdint.h>

namespace dfamin {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
// Scan / compaction tiles: 8 items per thread (2,048 per tile) for small
// launches, 32 (8,192 per tile) from 2^20 elements on, where the per-tile
// cost of the look-back dominates.  Callers size tile counts and status
// arrays with the same choice.
constexpr int kScanItemsSmall = 8;
constexpr int kScanItemsLarge = 32;
inline int scan_items_for(uint64_t elems) { return elems >= (1ull << 20) ? kScanItemsLarge : kScanItemsSmall; }
inline uint32_t scan_tile(int items) { return (uint32_t)kBlock * (uint32_t)items; }
inline uint32_t scan_tiles(uint64_t elems, int items) {
  return (uint32_t)((elems + scan_tile(items) - 1) / scan_tile(items));
}
// Signature kernel variants: 1, 2 or 4 states per thread (256, 512 or 1024
// states per workgroup, an LDS table of twice as many slots).  The variant is
// picked per size class by the engine's autotuner.
constexpr int kSigVariants = 3;
constexpr int kSigDefaultVariant = 1;
constexpr uint64_t kTuneMinStates = 1ull << 18;  // smaller rounds use the default
constexpr uint32_t kGraphRounds = 16;  // leader-election rounds per captured graph
constexpr uint32_t kBfsLevelsBeforeClosure = 64;  // BFS levels before closure rows join
constexpr uint64_t kMaxStates = 0x7FFFFF00ull;  // states per call: ids are 31-bit in hash slots
constexpr int kRowTile = kBlock * 4;  // row elements per workgroup in row jobs
constexpr int kLongTile = kBlock * 16;  // row elements per workgroup of validation

// Per-instance descriptor (device copy).  64 bytes.
//
// Key mode of the current round.  With B blocks before the round, a state's
// signature (own block, successor blocks) in dense block numbers 0..B-1 is
// an exact integer of (kp+1)*ceil(log2 B) bits.  When that fits in 31 bits
// (ebits > 0) the round groups on that exact key: no hashing shortcut, so no
// signature records and no verification.  Otherwise (ebits == 0) it groups
// on a 64-bit hash and verifies full signatures.  Dense numbers come from
// the accept bitmap while the partition is still {F, Q\F} (dsrc == 1) or
// from the dense[] array (dsrc == 0).
struct InstDesc {
  uint32_t state_off;   // first global state id
  uint32_t n;           // states
  uint32_t kp;          // signature letters in use (rows)
  uint32_t rows_off;    // index of the first row pointer in rows[]
  uint64_t sig;         // device address of the signature records: n * (kp + 1) words
  uint64_t accept;      // device address of the accept bitmap
  uint64_t out;         // device address of the output (n uint32)
  uint32_t q0;
  uint32_t k;           // original alphabet size
  uint32_t ebits;       // bits per key component in exact mode, 0 = hash mode
  uint32_t dsrc;        // exact mode: 1 = accept bit, 0 = dense[] array
  uint64_t pad;
};

// Global hash-table slot: one 64-bit word, 0 = empty.
//   bits 63..32  fragment of the signature hash (never 0)
//   bit  31      shared: at least two active states carry this hash
//   bits 30..0   least (global) state id carrying this hash: the new block id
// The home position comes from the low hash bits, the fragment from the high
// ones.  A slot is claimed, joined and lowered with 64-bit CAS only.
typedef unsigned long long Slot;
constexpr uint32_t kSlotShared = 0x80000000u;
constexpr uint32_t kSlotIndexMask = 0x7fffffffu;
// slot_of[j] bit 31 (tables of at most 2^31 slots): state j claimed an empty
// slot with no other state of its tile in its group.  Unless a later joiner
// marked it in the round's notify bytes, it is then alone in its group, and
// the resolve step needs no read of the slot.
constexpr uint32_t kSlotClaimedAlone = 0x80000000u;
// Group counters of a signature round (gcount, 2 * kGroupCounters words,
// zeroed by the table clear before the round): workgroup w adds to word
// w % kGroupCounters the slots it claimed (groups formed) and, at offset
// kGroupCounters, the slots that became shared through it (claimed by a
// tile group of two or more, or joined for the first time).  Spreading
// the sums over many words keeps any one word from taking an atomic from
// every workgroup.
constexpr uint32_t kGroupCounters = 64;
// Slot labels: after an exact-key round whose groups are counted, a state
// of a shared group may carry kSlotLabel | (its group's slot) as its block
// label instead of the least member (a state id, below 2^31): the labels
// tell the same partition.  A state alone in its group carries its own id,
// which is its least member.
constexpr uint32_t kSlotLabel = 0x80000000u;
// Direct count tables (launch_signature's dtab) of at most 2^kDirectMaxBits
// words: 128 MB, which the memory-side cache can hold.
constexpr uint32_t kDirectMaxBits = 25;

// Control block shared by the round kernels and read by the host.  The flags
// only go from 0 to 1 within a kernel (plain stores of one value); the tile
// counter and m_next are updated with device atomics and the tile counter
// lives on its own 128-byte line.
struct Ctrl {
  uint32_t any_changed;   // some block split this round
  uint32_t collision;     // two different signatures shared a hash this round
  uint32_t m_next;        // active states for the next round
  uint32_t fault;         // a bounded device wait or probe ran out (never expected)
  uint32_t stop;          // queued rounds: nothing left to split, later rounds do nothing
  uint32_t iterations;    // queued rounds run (leader rounds: the one that found stability included)
  uint32_t m_cur;         // queued signature rounds: active states of the coming round
  uint32_t retries;       // queued signature rounds: times the coming round was redone (hash collision)
  uint64_t salt;          // queued signature rounds: hash salt of the coming round
  uint64_t hash_mask;     // testing: nonzero keeps only these bits of a signature hash
  uint32_t prev_shared;   // shared groups of the last round that ended with slot labels
  uint32_t pad0[19];
  uint32_t tile_counter;  // dynamic tile ids for the look-back scans
  uint32_t pad1[31];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl layout");

// Bounds on device-side waiting and probing: hitting one sets Ctrl::fault,
// the kernel finishes, and the host reports DFAMIN_E_INTERNAL.
constexpr uint32_t kMaxSpin = 1u << 22;

// Host-side wait for a stream.  Round loops wait for a few microseconds of
// queued work many times per call; a blocking wait's wake-up costs tens of
// microseconds each time, so short waits poll the stream and only waits
// beyond 2 ms fall back to the blocking call.
inline hipError_t stream_wait(hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000))
      return hipStreamSynchronize(s);
  }
}

// The same wait for one event (work queued behind it keeps running).
inline hipError_t event_wait(hipEvent_t ev) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000))
      return hipEventSynchronize(ev);
  }
}

// One row of n entries handled by a row job (validation, closure level).
struct RowJob {
  uint64_t src;        // device address of a uint32[n] row
  uint64_t dst;        // destination row (closure level) or 0
  uint32_t n;
  uint32_t flag_idx;   // which flag word this job reports into
};

// Per-instance results written on the device.
struct ResultDev {
  uint32_t num_blocks;
  uint32_t initial_block;
  uint32_t refine_rounds;
  uint32_t pad;
};

// Whole minimization of small instances, one workgroup each (fused.hip).
// Instances of up to kFusedMaxStates states and kFusedMaxLetters letters,
// closure OFF or AUTO, signature rounds.
struct FusedJob {
  uint64_t delta, accept, out;  // device addresses (letter-major rows, bitmap, n outputs)
  uint32_t n, k, q0, closure;
  uint32_t levels;       // highest closure level a doubling round may read (floor(log2 n) or max_levels)
  uint32_t auto_rounds;  // AUTO: rounds after which an instance with >= 2 non-identity letters
                         // that is still splitting is handed back to the round engine
  uint32_t max_rounds;   // round cap
  uint32_t pad;
};
struct FusedRes {
  int32_t status;  // kFused*
  uint32_t num_blocks, initial_block, refine_rounds;
  uint32_t levels_used;  // doubling: the highest closure level a round read
  uint32_t doubling;     // 1: refined by doubling (one non-identity letter, AUTO)
  uint32_t pad[2];
};
constexpr int32_t kFusedOk = 0;
constexpr int32_t kFusedBad = 1;       // some entry >= n; the output is not written
constexpr int32_t kFusedHandOff = 2;   // needs closure letters: run it through the round engine
constexpr int32_t kFusedRoundCap = 3;  // max_rounds reached
constexpr int32_t kFusedFault = 4;     // a bounded probe ran out (never expected)
constexpr uint32_t kFusedMaxStates = 16384;
constexpr uint32_t kFusedMaxLetters = 32;
// size class of a fused instance: 0 up to 2,048 states (256 threads),
// 1 up to 8,192 (512 threads), 2 up to 16,384 (1,024 threads, 160 KB of LDS)
inline int fused_class(uint32_t n) { return n <= 2048 ? 0 : (n <= 8192 ? 1 : 2); }
// one (nullable): a single job passed by value (jobs is then ignored and
// njobs taken as 1).  res may be mapped page-locked host memory.
void launch_fused(const FusedJob* jobs, FusedRes* res, uint32_t njobs, int cls, hipStream_t s,
                  const FusedJob* one = nullptr);

// Row-check flag bits.
constexpr uint32_t kFlagBad = 1u;      // entry >= n
constexpr uint32_t kFlagNonId = 2u;    // entry != its own index
constexpr uint32_t kFlagDiffers = 4u;  // closure level differs from the previous level

// Kernel launchers (kernels.hip).  All are asynchronous on `s`.
// Jobs: a list of work units each covering `len` elements; job_wg_off[j] is
// the first workgroup of job j (exclusive prefix over ceil(len/tile)).
// Row checks write one flag word per workgroup (wg_flags) and then OR them
// into one word per job (flags); no contended atomics.
void launch_row_check(const RowJob* jobs, const uint32_t* job_wg_off, uint32_t njobs,
                      uint32_t total_wgs, uint32_t* wg_flags, uint32_t* flags, hipStream_t s);
// (flags null: no flags are computed, and wg_flags is not used)
void launch_closure_level(const RowJob* jobs, const uint32_t* job_wg_off, uint32_t njobs,
                          uint32_t total_wgs, uint32_t* wg_flags, uint32_t* flags, hipStream_t s);
// Least accepting / non-accepting state per instance: per-workgroup partial
// minima over the instance's states, reduced per instance.
void launch_init_minmax(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst,
                        uint32_t total_wgs, unsigned long long* wg_part, uint32_t* minF,
                        uint32_t* minN, hipStream_t s);
void launch_init_block(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst,
                       uint32_t total_wgs, const uint32_t* minF, const uint32_t* minN,
                       uint32_t* inst_of, uint32_t* block, uint32_t* act, hipStream_t s);
// gmode (clear_table, signature, resolve, compact, round_end): a queued
// round whose kernels return at once when ctrl->stop is set and otherwise
// take the active count (m) and the salt from ctrl->m_cur and ctrl->salt; m
// is then an upper bound that only sizes the grid.
// gcount (nullable): the group counters, zeroed with the table.
void launch_clear_table(Slot* table, uint64_t tsize, Ctrl* ctrl, hipStream_t s, int gmode = 0,
                        uint32_t* gcount = nullptr);
// dense / dense_width: dense block numbers (exact-key rounds that read them),
// stored dense_width (1, 2 or 4) bytes per state.  gmode bit 0 as above;
// bits 1 and 2: hash-mode / exact-key states insert their group with a CAS
// on the home slot before reading it (table_insert).
// notify (nullable): one byte per global state, all 0 before the round; the
// resolve step of the round returns them to 0.
// gcount (nullable): the round's group counters.
// dtab (nullable; exact keys of one instance): a direct count table of
// 2^((kp+1)*ebits) words, all 0 before the round, takes the place of the
// hash table: each local group adds its size to the word its key indexes,
// the key is the slot id, and a lone claimer is known by its word's count.
void launch_signature(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                      const InstDesc* desc, const uint64_t* rows, const uint32_t* block,
                      const void* dense, int dense_width, Slot* table, uint32_t tbits,
                      uint32_t* slot_of, uint64_t salt, Ctrl* ctrl, int variant, hipStream_t s,
                      int gmode = 0, uint8_t* notify = nullptr, uint32_t* gcount = nullptr,
                      uint32_t* dtab = nullptr);
// dense[g] = rank[block[g]] - rank[state_off]: the block's number among the
// instance's blocks in order of least member, dense_width bytes wide (every
// number must fit).
void launch_dense(bool batch, uint32_t N, const uint32_t* inst_of, const InstDesc* desc,
                  const uint32_t* block, const uint32_t* rank, void* dense, int dense_width,
                  hipStream_t s);
// counts[i] = number of blocks of instance i (from rank).
void launch_block_counts(uint32_t ninst, const InstDesc* desc, const uint32_t* rank,
                         uint32_t* counts, hipStream_t s);
// notify must be what the round's launch_signature was given (both null, or
// the same bytes): only then are the slot ids it wrote free of the
// claimed-alone bit, or is that bit read as such.
// count_gcount (nullable, one instance only): the round follows one that
// left slot labels, so a state's old label is no least member; the
// instance split iff this round formed more groups (from these counters)
// than that round left shared (ctrl->prev_shared).
void launch_resolve(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                    const InstDesc* desc, const Slot* table,
                    const uint32_t* slot_of, const uint32_t* block, uint32_t* nb, uint8_t* keep,
                    uint32_t* changed_inst, Ctrl* ctrl, unsigned long long* scan_status,
                    uint32_t ntiles, hipStream_t s, int gmode = 0, uint8_t* notify = nullptr,
                    const uint32_t* count_gcount = nullptr);
// dead (nullable): instances whose states leave the active list (cancelled).
// Slot labels (slot_of non-null; one instance, an exact-key round with
// lone claimers marked in notify and groups counted in gcount; takes the
// place of the resolve step, whose scan status clearing launch_prep_scan
// does): the instance split iff the round formed more groups than
// prev_count, the blocks its active states were in before the round.  If
// so, a state of a shared group (not a lone claimer, or one a joiner
// marked) gets kSlotLabel | slot and stays active, a state alone gets its
// own id; changed_inst[0] and ctrl->prev_shared (the shared groups) are
// set.  If not, no block id changes and no state stays.  The notify bytes
// read are returned to 0.  With dtab (the round's direct count table) a
// lone claimer's group is shared iff its word counts two or more, and no
// notify byte is read; where at most one in 64 states formed a group alone,
// every state stays active under its label instead (prev_shared is then
// every group formed), and act_next is not written: m_next = m, and the
// caller keeps act as the list of the next round.
void launch_compact(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                    const uint32_t* nb, const uint8_t* keep, uint32_t* changed_inst,
                    const uint32_t* dead, uint32_t* block, uint32_t* act_next, Ctrl* ctrl,
                    unsigned long long* scan_status, int items, hipStream_t s, int gmode = 0,
                    const uint32_t* slot_of = nullptr, uint8_t* notify = nullptr,
                    const uint32_t* gcount = nullptr, uint32_t prev_count = 0,
                    const uint32_t* dtab = nullptr);
// last (nullable) receives this round's per-instance changed flags.
void launch_round_end(uint32_t ninst, uint32_t* changed_inst, uint32_t* refine_cnt, uint32_t* last,
                      Ctrl* ctrl, hipStream_t s, unsigned long long* clear_status = nullptr,
                      uint32_t clear_tiles = 0, int gmode = 0);
// Queued signature rounds: start (stop, iterations and retries cleared,
// m_cur and salt set) and the one-thread step that ends each round: after a
// hash collision a new salt (the round is redone; too many set fault and
// stop), else iterations + 1, m_cur = m_next, and stop once a round split
// nothing or left no active state.
void launch_queue_start(Ctrl* ctrl, uint32_t m, uint64_t salt, hipStream_t s);
// *p = v, in stream order
void launch_store_u64(uint64_t* p, uint64_t v, hipStream_t s);
// Copies `bytes` from src to dst as a kernel on the stream (16-byte units
// where both addresses and the size allow, else 4-byte or 1-byte units).  Either side may be page-locked host memory
// mapped into the device's address space; stores reach memory before the
// kernel ends, so a host wait on a later event sees them.  Between two
// kernels such a copy costs a few microseconds, where a copy-engine transfer
// of 32 KB or more adds about 15 us of hand-off in each direction.
void launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
// Small copies and fills batched into one launch (launch_mem_segs): src
// non-null copies `bytes` from src (device memory, or page-locked host memory
// mapped for the device) to dst, src null sets `bytes` bytes of dst to fill.
// For host-to-device staging only: a copy to host memory needs
// launch_copy_bytes, which makes its stores visible to the host.
constexpr uint32_t kMemSegs = 8;
struct MemSeg {
  void* dst;
  const void* src;
  uint64_t bytes;
  uint32_t fill, pad;
};
struct MemSegs {
  MemSeg seg[kMemSegs];
  uint32_t n;
};
void launch_mem_segs(const MemSegs& q, hipStream_t s);
// Queued rounds of instances refining by doubling (one closure level per
// round, 2^l <= j+1): per listed instance t (instance list[t]) the device
// keeps j (mj), the levels built and the highest level read.  Before a
// round, plan points the descriptor at this round's level (and notes a
// level to build: at most one, since j at least doubles) and levels builds
// it (dst = src o src, Algorithm 5) over the instance's states; after a
// round that was not redone, advance adds 2^l to j and, if the instance
// split a block in it, raises its highest level read (used).  All return at
// once when ctrl->stop is set.
struct QueueDbl {
  uint64_t* mj;
  uint32_t *list, *built, *lmax, *rbase, *need, *lv, *used, *n, *wgoff;
  uint32_t* last;  // per instance (all of the call): split a block in this round
  uint32_t count, wgs;
};
void launch_queue_plan(const QueueDbl& q, InstDesc* desc, const Ctrl* ctrl, hipStream_t s);
void launch_queue_levels(const QueueDbl& q, const uint64_t* rows, const Ctrl* ctrl, hipStream_t s);
void launch_queue_advance(const QueueDbl& q, const Ctrl* ctrl, hipStream_t s);
void launch_round_step(Ctrl* ctrl, hipStream_t s);
constexpr uint32_t kMaxSaltRetries = 8;
// One round of leader-based refinement (Algorithm 2, Section 3.2) over all
// N states: elect (states that differ from their leader in a successor
// block; the least of them becomes new_leader[leader]), move (they join the
// new leader's block; resets next_leader for the following round), then
// launch_round_end and a one-thread check that sets ctrl->stop when no
// block split.  Every kernel returns at once when ctrl->stop is set, so
// rounds can be queued (or replayed from a graph) ahead of the host.
void launch_naive_round(bool batch, uint32_t N, uint32_t ninst, const uint32_t* inst_of,
                        const InstDesc* desc, const uint64_t* rows, uint32_t* block, uint32_t* new_leader,
                        uint32_t* next_leader, uint8_t* differs, uint32_t* changed_inst, uint32_t* refine_cnt,
                        Ctrl* ctrl, hipStream_t s);
// Instances joining a running set: like launch_init_block, with instance
// ids slot[j] for job j and their states appended to act at act_off[j];
// zero_a/b/c[slot[j]] (per-slot counters) are set to 0.
void launch_init_join(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                      uint32_t njobs, uint32_t total_wgs, const uint32_t* act_off,
                      const uint32_t* minF, const uint32_t* minN, uint32_t* inst_of,
                      uint32_t* block, uint32_t* act, uint32_t* zero_a, uint32_t* zero_b, uint32_t* zero_c,
                      hipStream_t s);
void launch_init_minmax_slots(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                              uint32_t njobs, uint32_t total_wgs, unsigned long long* wg_part,
                              uint32_t* minF, uint32_t* minN, hipStream_t s);
// Per-instance (segmented) canonical numbering for the instances slot[j]:
// rank[g] = representatives before g within its instance; totals[j] = the
// instance's block count; then out[q] = rank[block[g]] and per-instance
// results.  job_tile_off: scan tiles (kScanTile states) per job, prefix.
void launch_scan_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_tile_off,
                      uint32_t njobs, uint32_t total_tiles, const uint32_t* block, uint32_t* rank,
                      uint32_t* totals, Ctrl* ctrl, unsigned long long* scan_status, int items,
                      hipStream_t s);
void launch_emit_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                      uint32_t njobs, uint32_t total_wgs, const uint32_t* block, const uint32_t* rank,
                      hipStream_t s);
// dense[g] = rank[block[g]] (instance-relative ranks from launch_scan_jobs)
// for the states of the listed instances, dense_width bytes wide;
// job_wg_off: kRowTile-state workgroups per job, prefix.
void launch_dense_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                       uint32_t njobs, uint32_t total_wgs, const uint32_t* block, const uint32_t* rank,
                       void* dense, int dense_width, hipStream_t s);
// The first signature round from {F, Q\F} by labels (instances of at most
// kMaxLabelLetters signature letters): the label of q is its accept bit and
// those of its successors, an exact key of label_bits <= kMaxLabelLetters+1
// bits.  NL = 256 labels per instance for label_bits <= 8, else 512; labels
// and their numbers are then one byte, else two.  Per instance (jobs of
// kRowTile states, job_wg_off as for the init jobs): lmin (NL words per
// instance, all ones before the call) receives each label's least member,
// rank (NL per instance) the labels' numbers in order, counts[i] the number
// of labels present, changed_inst[i] = 1 where that exceeds the number of
// blocks of {F, Q\F}.  label (one per state, scratch) holds the labels;
// then block[g] = the least-member id, dense[g] = the label's number in one
// byte (every instance whose next round groups on exact keys has at most 32
// blocks; dense may be label itself when labels are one byte), act[g] = g
// and inst_of[g] = i (nullable): the initial partition need not be
// computed first.  The round flags of ctrl are cleared, and with set_m
// m_next is set to m (every state stays active).
constexpr uint32_t kMaxLabelLetters = 8;
void launch_label(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst, uint32_t total_wgs,
                  const uint64_t* rows, uint32_t label_bits, uint32_t* lmin, void* rank, void* label,
                  uint8_t* dense, uint32_t* counts, uint32_t* changed_inst, Ctrl* ctrl, uint32_t* block,
                  uint32_t set_m, uint32_t m, uint32_t* act, uint32_t* inst_of, hipStream_t s);
// One instance whose blocks are all singletons: out[q] = q and its results
// (n blocks, initial block q0).
void launch_identity_out(const InstDesc* desc, uint32_t n, const uint32_t* refine_cnt, ResultDev* res,
                         hipStream_t s);
void launch_results_jobs(const InstDesc* desc, const uint32_t* slot, uint32_t njobs,
                         const uint32_t* totals, const uint32_t* refine_cnt, ResultDev* res,
                         hipStream_t s);
// One BFS level: frontier states follow every row; newly visited successors
// are appended to next (next_count is the append counter).
void launch_bfs_level(const uint64_t* rows, uint32_t nrows, const uint32_t* frontier, uint32_t fcount,
                      uint32_t* visited, uint32_t* next, uint32_t* next_count, hipStream_t s);
// The quotient of the reachable classes (single instance, state ids 0..n-1):
// cls = canonical class per state (nb classes), visited = reachability
// bitmap, block = least-member ids.  Writes rid[c] (dense number of kept
// class c, rid[nb] = their count m), min_delta (letter-major, m per letter),
// min_acc8 (one byte per state) and min_acc (LSB-first bitmap).  sel must
// hold all ones for the nb classes.
void launch_quotient(uint32_t n, uint32_t k, uint32_t nb, const uint32_t* delta, const uint8_t* accept,
                     const uint32_t* block, const uint32_t* cls, const uint32_t* visited, uint32_t* sel,
                     uint32_t* rid, uint32_t* rep, uint32_t* min_delta, uint8_t* min_acc8, uint8_t* min_acc,
                     Ctrl* ctrl, unsigned long long* scan_status, hipStream_t s);
void launch_prep_scan(unsigned long long* scan_status, uint32_t ntiles, Ctrl* ctrl, hipStream_t s);
void launch_scan_reps(const uint32_t* block, uint32_t N, uint32_t* rank, Ctrl* ctrl,
                      unsigned long long* scan_status, int items, hipStream_t s);
void launch_emit(bool batch, uint32_t N, const uint32_t* inst_of, const InstDesc* desc,
                 const uint32_t* block, const uint32_t* rank, hipStream_t s);
void launch_results(uint32_t ninst, const InstDesc* desc, const uint32_t* rank,
                    const uint32_t* refine_cnt, ResultDev* res, hipStream_t s);

}  // namespace dfamin
