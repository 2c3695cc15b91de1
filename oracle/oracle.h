/*
 * oracle.h -- CPU reference implementations for DFA minimization.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library (libdfamin) may
 * include, link or call this code; only tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  The two share no source.
 *
 * Conventions (all functions):
 *   - States are 0..n-1 and letters 0..k-1 (the paper's Preliminaries,
 *     "Representation"; its closed intervals are read as 0..|Q|-1, 0..|Sigma|-1).
 *   - delta is letter-major: delta[(size_t)a*n + q] = delta(q, a)  (same
 *     paragraph: |Sigma| arrays of length |Q|).
 *   - accept is a bitmap of ceil(n/8) bytes, LSB first:
 *     q in F  iff  (accept[q >> 3] >> (q & 7)) & 1.
 *   - Every partition that leaves this library is in canonical form: blocks
 *     numbered 0,1,2,... in increasing order of their least member state.
 *   - Return value: 0 on success, -1 on bad arguments (delta entry >= n,
 *     n == 0, null pointer), -2 on allocation failure.
 *
 * All arithmetic is integer; no floating point anywhere.
 */
#ifndef DFAMIN_ORACLE_H
#define DFAMIN_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Relabel an arbitrary labelling (labels < n) into canonical block ids:
 * out[q] = number of distinct labels whose least member is < the least
 * member of q's label.  Returns the number of blocks. */
uint32_t oracle_canonicalize(uint32_t n, const uint32_t *labels, uint32_t *out);

/* Hopcroft's O(k n log n) partition refinement (Hopcroft 1971, the
 * reference cited in the paper's introduction).  Computes Myhill-Nerode
 * equivalence over ALL n states (no reachability pruning, as in the
 * paper's Preliminaries). */
int oracle_hopcroft(uint32_t n, uint32_t k, const uint32_t *delta,
                    const uint8_t *accept, uint32_t *out, uint32_t *num_blocks);

/* Moore-style signature refinement with the round semantics of the paper's
 * sorting algorithm (Section 3.3, Algorithm 4): start from {F, Q\F}; each
 * round gives every state the signature (block[q], block[delta(q,0)], ...,
 * block[delta(q,k-1)]), sorts states by it lexicographically and numbers
 * the runs of equal signatures; stop when the block count is unchanged.
 * refine_rounds = rounds that increased the count.  Fails with -3 if more
 * than max_rounds rounds would run (0 = no cap). */
int oracle_moore(uint32_t n, uint32_t k, const uint32_t *delta,
                 const uint8_t *accept, uint32_t max_rounds, uint32_t *out,
                 uint32_t *num_blocks, uint32_t *refine_rounds);

/* The partition after exactly `rounds` rounds of the refinement above (or
 * the stable partition if it is reached earlier); rounds == 0 gives
 * {F, Q\F}.  refine_rounds counts the rounds among them that refined. */
int oracle_moore_partial(uint32_t n, uint32_t k, const uint32_t *delta,
                         const uint8_t *accept, uint32_t rounds, uint32_t *out,
                         uint32_t *num_blocks, uint32_t *refine_rounds);

/* Moore refinement started from a given partition `init` (any labels < n)
 * instead of {F, Q\F}.  The own-block component still comes first in the
 * signature, so every round refines the previous one.  Used to check that
 * restarting from an intermediate partition reaches the same result. */
int oracle_moore_from(uint32_t n, uint32_t k, const uint32_t *delta,
                      const uint32_t *init, uint32_t max_rounds, uint32_t *out,
                      uint32_t *num_blocks, uint32_t *refine_rounds);

/* Algorithm 2 (naivePR, Section 3.2): leader-based refinement.  Blocks are
 * named by a leader state; every iteration, the states that differ from
 * their leader in some successor block elect a new leader (here: the least
 * of them) and move to its block.  *iterations = while-loop iterations,
 * the final one (that finds the partition stable) included.  Fails with -3
 * if more than max_iter iterations would run (0 = no cap). */
int oracle_naive(uint32_t n, uint32_t k, const uint32_t *delta,
                 const uint8_t *accept, uint32_t max_iter, uint32_t *out,
                 uint32_t *num_blocks, uint32_t *iterations);

/* Partial transitive closure of the paper's Algorithm 5 (Section 3.4):
 * rows[(a*(L+1) + i)*n + q] = delta^T(q, a^(2^i)) for a < k, 0 <= i <= L,
 * where level 0 is delta itself and level i applies level i-1 twice.
 * rows must hold k*(L+1)*n entries. */
int oracle_closure(uint32_t n, uint32_t k, const uint32_t *delta, uint32_t L,
                   uint32_t *rows);

/* floor(log2 n) for n >= 1 (the level count of the closure alphabet). */
uint32_t oracle_floor_log2(uint32_t n);

/* Brute force 1: the sequential reading of the paper's pair-graph
 * algorithm (Section 3.1): mark pairs that differ on acceptance, then
 * repeatedly mark (p,q) when some letter leads to a marked pair; unmarked
 * pairs are equivalent.  O(n^2) memory: for small n only. */
int oracle_pair_marking(uint32_t n, uint32_t k, const uint32_t *delta,
                        const uint8_t *accept, uint32_t *out,
                        uint32_t *num_blocks);

/* Brute force 2: the definition of language equivalence (Preliminaries):
 * p ~ q iff delta*(p,w) in F <=> delta*(q,w) in F for every word w with
 * |w| <= max(n-1, 0), enumerated explicitly.  For tiny n*k only; fails with
 * -3 if k^(n-1) words exceed 2^22. */
int oracle_word_equivalence(uint32_t n, uint32_t k, const uint32_t *delta,
                            const uint8_t *accept, uint32_t *out,
                            uint32_t *num_blocks);

/* Breadth-first reachability from q0; mark[q] = 1 iff q is reachable.
 * Returns the number of reachable states. */
uint32_t oracle_reachable(uint32_t n, uint32_t k, const uint32_t *delta,
                          uint32_t q0, uint8_t *mark);

/* The minimal DFA in the textbook sense (Section 2): the quotient by the
 * equivalence of the states reachable from q0.  States: the classes that
 * contain a reachable state, numbered by least member.  min_delta:
 * letter-major, (*min_n) entries per letter (capacity k*n); min_accept:
 * LSB-first bitmap (capacity ceil(n/8)).  *num_reachable (may be NULL):
 * input states reachable from q0. */
int oracle_minimal_dfa(uint32_t n, uint32_t k, const uint32_t *delta,
                       const uint8_t *accept, uint32_t q0, uint32_t *min_n,
                       uint32_t *min_delta, uint8_t *min_accept, uint32_t *min_q0,
                       uint32_t *num_reachable);

/* Exhaustive cross-check over EVERY complete DFA with n states, k letters
 * and every accepting set: Hopcroft vs pair marking vs Moore (and word
 * enumeration when n <= 4).  Returns the number of DFAs checked; writes the
 * number of disagreements to *mismatches. */
uint64_t oracle_exhaustive_check(uint32_t n, uint32_t k, uint64_t *mismatches);

#ifdef __cplusplus
}
#endif
#endif
