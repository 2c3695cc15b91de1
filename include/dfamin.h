/*
 * dfamin.h -- C-ABI of libdfamin: massively parallel DFA minimization on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Martens & Wijs, "An Evaluation of Massively Parallel Algorithms
 * for DFA Minimization" (GandALF 2024).  Signature-based partition
 * refinement (Section 3.3, Algorithm 4: every round each state gathers the
 * block ids of its successors; states with equal signatures form the new
 * blocks; stop when the block count no longer grows), optionally on the
 * automaton extended by the partial transitive closure of Section 3.4
 * (Algorithm 5: letters a^(2^i), built by pointer jumping), which leaves the
 * classes unchanged and cuts the number of rounds on deep inputs.
 *
 * Problem statement (Section 2, Preliminaries): a complete DFA
 * (Q, Sigma, delta, F, q0) goes in; out comes the language-equivalence class
 * of EVERY state (unreachable states are not removed; the paper treats that
 * as separate pre-processing).
 *
 * Conventions shared by every call:
 *   - States are 0..n-1, letters 0..k-1.
 *   - delta is letter-major, as in Section 2 "Representation":
 *     delta[(size_t)a*n + q] = delta(q, a), uint32, every entry < n.
 *   - accept is a bitmap of ceil(n/8) bytes, LSB first:
 *     q is accepting iff (accept[q >> 3] >> (q & 7)) & 1.
 *   - Output: out[q] = canonical block id of q.  Blocks are numbered
 *     0,1,2,... in increasing order of their least member state, so out[0]
 *     is always 0 and the first state not in block 0 opens block 1.
 *   - All arithmetic is exact integer arithmetic; results are
 *     deterministic (independent of atomic ordering and hash salts).
 *   - Every call returns an int status: DFAMIN_OK (0) or a negative
 *     DFAMIN_E_* code.  No exception crosses the ABI.
 *   - Ownership: the caller owns every buffer it passes.  No call retains a
 *     caller pointer after it returns, except dfamin_submit, which copies
 *     its inputs before returning.
 *   - Threading: one context must not be used by two threads at once,
 *     except dfamin_submit / dfamin_wait / dfamin_cancel, which are
 *     thread-safe.
 */
#ifndef DFAMIN_H
#define DFAMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DFAMIN_OK            0
#define DFAMIN_E_INVAL      -1  /* null pointer, n == 0, k == 0, q0 >= n, size overflow, bad option */
#define DFAMIN_E_BAD_DFA    -2  /* some delta entry >= n (checked on the device); outputs untouched */
#define DFAMIN_E_NOMEM      -3  /* the context's HBM budget or a device allocation was exceeded */
#define DFAMIN_E_DEVICE     -4  /* a HIP runtime error; the context should be destroyed */
#define DFAMIN_E_TIMEOUT    -5  /* dfamin_wait: the request is not done yet */
#define DFAMIN_E_CANCELLED  -6  /* the request was cancelled */
#define DFAMIN_E_BUSY       -7  /* the serving queue is full */
#define DFAMIN_E_INTERNAL   -8  /* round cap exceeded or repeated hash collisions (never a wrong result) */

/* ---- types ------------------------------------------------------------- */
typedef struct dfamin_ctx dfamin_ctx;  /* opaque */

/* A complete DFA (Section 2).  For dfamin_minimize / _batch / _submit the
 * pointers are host pointers; for the *_device calls they are device
 * pointers (HIP device memory of the context's device). */
typedef struct {
  uint32_t n;             /* number of states, 1 <= n < 2^31 - 256 (state ids are 31-bit; the
                             states of one batched call also sum below that) */
  uint32_t k;             /* number of letters, >= 1 */
  const uint32_t *delta;  /* k*n entries, letter-major, each < n */
  const uint8_t *accept;  /* ceil(n/8) bytes, LSB first */
  uint32_t q0;            /* initial state < n; reported (out[q0]), not used by refinement */
} dfamin_dfa;

/* Closure policy (Section 3.4).  AUTO is 0, so a NULL or zeroed options
 * struct selects it. */
#define DFAMIN_CLOSURE_AUTO  0u  /* refine on Sigma; an instance with one non-identity letter refines by
                                    doubling from the first round (one closure level per round, each
                                    built when first read); any other instance gets Sigma^T built if
                                    it is still refining after auto_rounds rounds */
#define DFAMIN_CLOSURE_OFF   1u  /* refine on Sigma only */
#define DFAMIN_CLOSURE_ON    2u  /* build Sigma^T before the first round */

/* Refinement method. */
#define DFAMIN_METHOD_SIGNATURE 0u  /* signature rounds (Section 3.3, Algorithm 4): each round groups
                                       equal (own block, successor blocks) signatures */
#define DFAMIN_METHOD_LEADER    1u  /* leader-based rounds (Section 3.2, Algorithm 2, naivePR): each round
                                       splits off the states that differ from their block's leader; with
                                       closure ON this is the paper's transPR (Algorithm 5) */

/* Flags. */
#define DFAMIN_FLAG_NO_GRAPH 1u     /* leader rounds and queued signature rounds: launch kernels directly
                                       instead of replaying a captured HIP graph of rounds (same results) */
#define DFAMIN_FLAG_QUEUE 2u        /* signature rounds: once every instance still refining groups by hash
                                       (or refines by doubling, whose levels the device then plans), queue
                                       the remaining rounds on the device, replayed from a captured HIP
                                       graph on a non-null stream, and check for the end after 8, 24, 56 ...
                                       rounds.  Same partition and round counts; not the default, because
                                       on the benchmark workloads rounds planned by the host (with the next
                                       round's independent work overlapped) measure as fast or faster */

typedef struct {
  uint32_t closure;      /* DFAMIN_CLOSURE_*; 0 (a zeroed struct, or opts == NULL) means AUTO */
  uint32_t max_levels;   /* closure levels 0..L with L = min(floor(log2 n), max_levels); 0 = no cap */
  uint32_t auto_rounds;  /* AUTO: plain rounds before the closure is built; 0 = default (8) */
  uint32_t max_rounds;   /* give up with DFAMIN_E_INTERNAL after this many rounds; 0 = n + 1 */
  uint32_t method;       /* DFAMIN_METHOD_*; 0 = signature rounds.  The serving entry points
                            (dfamin_submit) accept DFAMIN_METHOD_SIGNATURE only */
  uint32_t flags;        /* DFAMIN_FLAG_* bits; 0 = none */
} dfamin_opts;

typedef struct {
  uint32_t num_blocks;       /* number of classes over all n states (|Q / ~|) */
  uint32_t initial_block;    /* out[q0] */
  uint32_t refine_rounds;    /* rounds that split at least one block */
  uint32_t rounds_executed;  /* refine_rounds + 1 (the last round finds no split) */
  uint32_t closure_levels;   /* closure levels built (L, or fewer when a letter reaches a repeated
                                or identity level); for a one-letter instance refining by doubling
                                under AUTO, the highest level read by a round that split a block
                                (each level is built when first read); 0 if no closure was built */
  uint32_t closure_letters;  /* letters of Sigma^T kept for refinement (identity letters and
                                repeated levels are dropped: they cannot split a block), else 0 */
  int32_t status;            /* per-instance status (batch): DFAMIN_OK or DFAMIN_E_BAD_DFA */
  uint32_t reserved;
} dfamin_result;

/* Per-kernel timing gathered while profiling is on (dfamin_set_profiling). */
typedef struct {
  char name[32];
  uint64_t launches;
  double total_ms;        /* sum of HIP-event durations of the launches */
  double alg_bytes;       /* algorithmic bytes those launches must move: the bytes per
                             processed element stated beside each kernel in the
                             library source, times the elements processed */
} dfamin_kernel_stat;

/* ---- context ----------------------------------------------------------- */
/* Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device memory the context may hold (0 = 90% of the device's free memory).
 * Returns DFAMIN_E_DEVICE if the device cannot be used. */
int dfamin_create(int hip_device, uint64_t hbm_budget_bytes, dfamin_ctx **out);

/* Destroy a context; stops its serving loop (pending requests are
 * cancelled) and frees its device memory.  NULL is ignored. */
void dfamin_destroy(dfamin_ctx *ctx);

/* ---- minimization ------------------------------------------------------ */
/* Minimize one DFA held in host memory; out: host buffer of n uint32.
 * On DFAMIN_E_BAD_DFA / _INVAL `out` is not written. */
int dfamin_minimize(dfamin_ctx *ctx, const dfamin_dfa *host_dfa, const dfamin_opts *opts,
                    uint32_t *out, dfamin_result *result);

/* Minimize one DFA whose delta / accept already live in device memory;
 * dev_out: device buffer of n uint32.  Work is issued on `hip_stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * null stream) and the call returns when it has completed. */
int dfamin_minimize_device(dfamin_ctx *ctx, const dfamin_dfa *dev_dfa, const dfamin_opts *opts,
                           uint32_t *dev_out, dfamin_result *result, void *hip_stream);

/* Size of the static device array behind dfamin_minimize_device_noalloc. */
#define DFAMIN_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate: code around HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as dfamin_minimize_device, but the call allocates nothing: no
 * hipMalloc / hipFree, no page-locked host memory, no events, no graphs.
 * Every device buffer of the call (block ids, active lists, hash table,
 * signature records, closure levels, scan status, control block) is carved
 * from one static device array of DFAMIN_NOALLOC_SCRATCH_BYTES bytes, which
 * the library holds on each device it runs on until the process ends; the
 * host-side staging it uses was set up by dfamin_create.  The caller still
 * passes delta, accept and dev_out in device memory.
 *   - Size limit: n * (66 + 16 * (k + 1)) + 2^20 must not exceed
 *     DFAMIN_NOALLOC_SCRATCH_BYTES (about 579,000 states at k = 2);
 *     larger inputs return DFAMIN_E_NOMEM before any work and leave
 *     dev_out untouched.
 *   - opts: method SIGNATURE only, and no DFAMIN_FLAG_QUEUE (both would
 *     instantiate HIP graphs): DFAMIN_E_INVAL otherwise.
 *   - Kernel timing (dfamin_set_profiling) is suspended for the call.
 *   - The array is shared by every context and every call on a device and
 *     keeps the last call's contents (each call clears what it needs).
 *     Calls that overlap on one device race: the caller must serialize
 *     them, across contexts and threads.
 * Returns when the work has completed, like dfamin_minimize_device. */
int dfamin_minimize_device_noalloc(dfamin_ctx *ctx, const dfamin_dfa *dev_dfa, const dfamin_opts *opts,
                                   uint32_t *dev_out, dfamin_result *result, void *hip_stream);

/* Minimize `count` independent DFAs (host memory) together: all instances
 * are refined by the same kernel launches, one fused round at a time
 * (block ids are global state ids, so instances never mix), and each
 * instance leaves the round loop when it stops refining.  outs[i] is a
 * host buffer of dfas[i].n uint32 (local state ids, canonical local block
 * ids); results[i] is filled for every instance.  If any instance has a
 * delta entry >= n, nothing is minimized, results[i].status marks the bad
 * instances and DFAMIN_E_BAD_DFA is returned. */
int dfamin_minimize_batch(dfamin_ctx *ctx, uint32_t count, const dfamin_dfa *dfas,
                          const dfamin_opts *opts, uint32_t *const *outs,
                          dfamin_result *results);

/* As dfamin_minimize_batch, with every delta / accept / outs[i] in device
 * memory (dfas and outs themselves are host arrays of device pointers). */
int dfamin_minimize_batch_device(dfamin_ctx *ctx, uint32_t count, const dfamin_dfa *dev_dfas,
                                 const dfamin_opts *opts, uint32_t *const *dev_outs,
                                 dfamin_result *results, void *hip_stream);

/* ---- the minimal DFA of the reachable part ------------------------------ */
/* Section 2: the minimal DFA is the quotient, by the equivalence, of the
 * states reachable from q0.  dfamin_minimize partitions ALL n states; this
 * call also finds the states reachable from q0 (breadth first on the GPU)
 * and emits the quotient automaton of their classes. */
typedef struct {
  uint32_t n;           /* states of the minimal DFA (classes holding a reachable state) */
  uint32_t q0;          /* its initial state */
  uint32_t num_blocks;  /* classes over all input states (as dfamin_result.num_blocks) */
  uint32_t reachable;   /* input states reachable from q0 */
  uint32_t bfs_levels;  /* breadth-first levels run; after 64 levels the closure letters join
                           as extra edges (words over Sigma: same reachable set, fewer levels) */
  uint32_t refine_rounds;  /* as dfamin_result */
  uint32_t reserved[2];
} dfamin_minimal;

/* Minimize one DFA held in host memory and emit its minimal DFA.  States of
 * the result are numbered by the least input state of their class; letter a
 * from state s leads to min_delta[a * info->n + s] (letter-major); s accepts
 * iff bit s of min_accept (LSB first) is set.  Caller-owned host buffers:
 * min_delta with room for k*n entries, min_accept for ceil(n/8) bytes,
 * `out` (may be NULL) for the n canonical class ids of dfamin_minimize.
 * Errors as dfamin_minimize; buffers are not written on error. */
int dfamin_minimal_dfa(dfamin_ctx *ctx, const dfamin_dfa *host_dfa, const dfamin_opts *opts,
                       uint32_t *min_delta, uint8_t *min_accept, uint32_t *out, dfamin_minimal *info);

/* ---- serving (continuous batching) -------------------------------------- */
/* Queue a request.  The DFA (host memory) is copied before the call returns.
 * A background loop admits queued requests while their device footprint
 * fits the context's budget, refines every resident request with one fused
 * round per step (newcomers join at the next step) and retires each request
 * as soon as it stops refining.  *ticket identifies the request. */
int dfamin_submit(dfamin_ctx *ctx, const dfamin_dfa *host_dfa, const dfamin_opts *opts,
                  uint64_t *ticket);

/* Wait up to timeout_us microseconds (< 0 = forever) for a request; on
 * success copies the n block ids into `out` (host) and fills `result`, and
 * the ticket is released.  DFAMIN_E_TIMEOUT leaves the ticket valid. */
int dfamin_wait(dfamin_ctx *ctx, uint64_t ticket, int64_t timeout_us, uint32_t *out,
                dfamin_result *result);

/* Cancel a request that has not completed; a later dfamin_wait on it
 * returns DFAMIN_E_CANCELLED.  Returns DFAMIN_E_INVAL for unknown tickets. */
int dfamin_cancel(dfamin_ctx *ctx, uint64_t ticket);

/* ---- diagnostics -------------------------------------------------------- */
/* Static string naming a status code. */
const char *dfamin_status_str(int status);

/* Turn per-kernel HIP-event timing on (1) or off (0); turning it on resets
 * the counters. */
int dfamin_set_profiling(dfamin_ctx *ctx, int on);

/* Copy up to `cap` kernel statistics into `stats`; returns the number of
 * entries available (may exceed cap), or a negative status. */
int dfamin_get_kernel_stats(dfamin_ctx *ctx, dfamin_kernel_stat *stats, int cap);

/* ---- tuning ------------------------------------------------------------- */
/* Signature-kernel tile: variant 0, 1 or 2 processes 256, 512 or 1024 states
 * per workgroup (1, 2 or 4 per thread, with an LDS pre-grouping table of
 * twice as many slots).  With variant = -1 (the default) the context tunes
 * itself: the first round of each size class (log2 of the active states,
 * key mode, dense width; classes of at least 2^18 states) runs every
 * variant once, timed with HIP events, and later rounds of that class use
 * the fastest.  0..2 force one variant (results never depend on it).
 * Returns DFAMIN_E_INVAL for a null ctx or another value; clears the cache. */
int dfamin_set_tuning(dfamin_ctx *ctx, int variant);

#ifdef __cplusplus
}
#endif
#endif /* DFAMIN_H */
