/*
 * oracle.c -- plain, sequential CPU reference for DFA minimization.
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the product library; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source with the GPU path.
 *
 * What is computed (paper, Preliminaries): for a complete DFA
 * (Q, Sigma, delta, F, q0), the partition of ALL states into classes of the
 * language equivalence p ~ q  iff  for every word w, delta*(p,w) in F <=>
 * delta*(q,w) in F.  Unreachable states are kept (the paper treats their
 * removal as a separate pre-processing step).  The coarsest such partition
 * is unique, so every algorithm below must return the same canonical
 * labelling.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

#define ACC(acc, q) (((acc)[(q) >> 3] >> ((q) & 7)) & 1u)

static int check_args(uint32_t n, uint32_t k, const uint32_t *delta,
                      const uint8_t *accept, const uint32_t *out) {
  if (n == 0 || k == 0 || !delta || !accept || !out) return -1;
  size_t nk = (size_t)n * k;
  for (size_t i = 0; i < nk; ++i)
    if (delta[i] >= n) return -1;
  return 0;
}

uint32_t oracle_floor_log2(uint32_t n) {
  uint32_t L = 0;
  while ((n >> 1) >= 1) { n >>= 1; ++L; }
  return L;
}

/* Canonical numbering: scan states in increasing order; a label seen for
 * the first time opens the next block id.  The first state that carries a
 * label is that label's least member, so ids increase with least members. */
uint32_t oracle_canonicalize(uint32_t n, const uint32_t *labels, uint32_t *out) {
  uint32_t *map = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  if (!map) return 0;
  for (uint32_t i = 0; i < n; ++i) map[i] = UINT32_MAX;
  uint32_t next = 0;
  for (uint32_t q = 0; q < n; ++q) {
    uint32_t l = labels[q];
    if (map[l] == UINT32_MAX) map[l] = next++;
    out[q] = map[l];
  }
  free(map);
  return next;
}

/* ------------------------------------------------------------------------ */
/* Hopcroft (1971).  Refinable partition: the states of each block occupy a
 * contiguous range of `elems`; marking a state swaps it into the marked
 * prefix of its block.  Splitters are (block, letter) pairs; after a split
 * of Y into Y and Z, a pair (Y,b) already waiting gets (Z,b) added,
 * otherwise only the smaller of Y and Z is added ("process the smaller
 * half"). */
int oracle_hopcroft(uint32_t n, uint32_t k, const uint32_t *delta,
                    const uint8_t *accept, uint32_t *out, uint32_t *num_blocks) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  size_t nk = (size_t)n * k;
  uint32_t *pred_off = (uint32_t *)calloc((size_t)k * (n + 1), sizeof(uint32_t));
  uint32_t *pred = (uint32_t *)malloc(sizeof(uint32_t) * nk);
  uint32_t *elems = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *loc = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *blk = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *first = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *end = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *mid = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint8_t *inW = (uint8_t *)calloc(nk, 1);
  uint32_t *wstack = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (nk + k));
  uint32_t *X = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *touched = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!pred_off || !pred || !elems || !loc || !blk || !first || !end || !mid ||
      !inW || !wstack || !X || !touched) {
    rc = -2;
    goto done;
  }

  /* Predecessor lists per letter, as CSR: pred_a(p) = {q : delta(q,a) = p}. */
  for (uint32_t a = 0; a < k; ++a) {
    uint32_t *off = pred_off + (size_t)a * (n + 1);
    const uint32_t *row = delta + (size_t)a * n;
    for (uint32_t q = 0; q < n; ++q) off[row[q] + 1]++;
    for (uint32_t p = 0; p < n; ++p) off[p + 1] += off[p];
    uint32_t *fill = X; /* reuse as cursor */
    for (uint32_t p = 0; p < n; ++p) fill[p] = off[p];
    for (uint32_t q = 0; q < n; ++q) pred[(size_t)a * n + fill[row[q]]++] = q;
  }

  /* Initial partition {F, Q\F} (only non-empty blocks). */
  uint32_t nF = 0;
  for (uint32_t q = 0; q < n; ++q) nF += ACC(accept, q);
  uint32_t nb = 0;
  {
    uint32_t pf = 0, pn = nF;
    for (uint32_t q = 0; q < n; ++q) {
      uint32_t pos = ACC(accept, q) ? pf++ : pn++;
      elems[pos] = q;
      loc[q] = pos;
    }
    if (nF > 0) { first[nb] = 0; end[nb] = nF; mid[nb] = 0; ++nb; }
    if (nF < n) { first[nb] = nF; end[nb] = n; mid[nb] = nF; ++nb; }
    for (uint32_t b = 0; b < nb; ++b)
      for (uint32_t i = first[b]; i < end[b]; ++i) blk[elems[i]] = b;
  }

  size_t wtop = 0;
  if (nb == 2) {
    uint32_t small = (end[0] - first[0] <= end[1] - first[1]) ? 0 : 1;
    for (uint32_t a = 0; a < k; ++a) {
      wstack[2 * wtop] = small; wstack[2 * wtop + 1] = a; ++wtop;
      inW[(size_t)small * k + a] = 1;
    }
  }

  while (wtop > 0) {
    --wtop;
    uint32_t C = wstack[2 * wtop], a = wstack[2 * wtop + 1];
    inW[(size_t)C * k + a] = 0;
    /* X = pred_a(C), collected before any state moves. */
    uint32_t nx = 0;
    const uint32_t *off = pred_off + (size_t)a * (n + 1);
    const uint32_t *pl = pred + (size_t)a * n;
    for (uint32_t i = first[C]; i < end[C]; ++i) {
      uint32_t p = elems[i];
      for (uint32_t j = off[p]; j < off[p + 1]; ++j) X[nx++] = pl[j];
    }
    /* Mark: move each state of X into the marked prefix of its block. */
    uint32_t nt = 0;
    for (uint32_t i = 0; i < nx; ++i) {
      uint32_t q = X[i], Y = blk[q];
      if (mid[Y] == first[Y]) touched[nt++] = Y;
      uint32_t pos = loc[q], m = mid[Y];
      uint32_t other = elems[m];
      elems[m] = q; loc[q] = m;
      elems[pos] = other; loc[other] = pos;
      mid[Y] = m + 1;
    }
    /* Split every touched block that is only partly marked. */
    for (uint32_t t = 0; t < nt; ++t) {
      uint32_t Y = touched[t];
      if (mid[Y] == end[Y]) { mid[Y] = first[Y]; continue; }
      uint32_t Z = nb++;
      first[Z] = first[Y]; end[Z] = mid[Y]; mid[Z] = first[Z];
      first[Y] = mid[Y]; mid[Y] = first[Y];
      for (uint32_t i = first[Z]; i < end[Z]; ++i) blk[elems[i]] = Z;
      uint32_t szY = end[Y] - first[Y], szZ = end[Z] - first[Z];
      for (uint32_t b = 0; b < k; ++b) {
        uint32_t add;
        if (inW[(size_t)Y * k + b]) add = Z;
        else add = (szZ <= szY) ? Z : Y;
        if (!inW[(size_t)add * k + b]) {
          inW[(size_t)add * k + b] = 1;
          wstack[2 * wtop] = add; wstack[2 * wtop + 1] = b; ++wtop;
        }
      }
    }
  }

  {
    uint32_t c = oracle_canonicalize(n, blk, out);
    if (num_blocks) *num_blocks = c;
  }
  rc = 0;
done:
  free(pred_off); free(pred); free(elems); free(loc); free(blk);
  free(first); free(end); free(mid); free(inW); free(wstack); free(X);
  free(touched);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Moore / sortPR round semantics.  One round, exactly as Algorithm 4 of the
 * paper reads when run sequentially: build every signature from the
 * partition of the previous round, sort the states by (own block, then the
 * successor blocks in letter order), put a 1 wherever two neighbours in the
 * sorted order differ, prefix-sum those flags into new block numbers, and
 * write them back.  Stop as soon as the block count does not grow. */

typedef struct {
  uint32_t k1;          /* k + 1 words per signature */
  const uint32_t *sig;  /* sig[q*k1 + 0] = block[q], then successor blocks */
} sig_ctx;

static int sig_cmp(const sig_ctx *c, uint32_t p, uint32_t q) {
  const uint32_t *sp = c->sig + (size_t)p * c->k1;
  const uint32_t *sq = c->sig + (size_t)q * c->k1;
  for (uint32_t i = 0; i < c->k1; ++i) {
    if (sp[i] < sq[i]) return -1;
    if (sp[i] > sq[i]) return 1;
  }
  return 0;
}

/* Stable bottom-up merge sort of the index array by signature. */
static void sort_by_sig(const sig_ctx *c, uint32_t *idx, uint32_t *tmp, uint32_t n) {
  for (uint32_t w = 1; w < n; w *= 2) {
    for (uint32_t lo = 0; lo < n; lo += 2 * w) {
      uint32_t m = lo + w < n ? lo + w : n;
      uint32_t hi = lo + 2 * w < n ? lo + 2 * w : n;
      uint32_t i = lo, j = m, o = lo;
      while (i < m && j < hi) tmp[o++] = (sig_cmp(c, idx[j], idx[i]) < 0) ? idx[j++] : idx[i++];
      while (i < m) tmp[o++] = idx[i++];
      while (j < hi) tmp[o++] = idx[j++];
    }
    memcpy(idx, tmp, sizeof(uint32_t) * n);
  }
}

static int moore_core(uint32_t n, uint32_t k, const uint32_t *delta,
                      uint32_t *block, uint32_t max_rounds, int stop_at_cap,
                      uint32_t *out, uint32_t *num_blocks,
                      uint32_t *refine_rounds) {
  uint32_t k1 = k + 1;
  uint32_t *sig = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * k1);
  uint32_t *state = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!sig || !state || !tmp) { free(sig); free(state); free(tmp); return -2; }

  /* Count of the starting partition. */
  uint32_t count = oracle_canonicalize(n, block, tmp);
  memcpy(block, tmp, sizeof(uint32_t) * n);
  uint32_t refining = 0, rounds = 0;
  sig_ctx c = {k1, sig};
  for (;;) {
    if (max_rounds && rounds >= max_rounds) {
      if (stop_at_cap) break;
      free(sig); free(state); free(tmp);
      return -3;
    }
    ++rounds;
    for (uint32_t q = 0; q < n; ++q) {
      sig[(size_t)q * k1] = block[q];
      for (uint32_t a = 0; a < k; ++a)
        sig[(size_t)q * k1 + 1 + a] = block[delta[(size_t)a * n + q]];
    }
    for (uint32_t q = 0; q < n; ++q) state[q] = q;
    sort_by_sig(&c, state, tmp, n);
    /* adjacent difference + inclusive scan -> new block of state[i] */
    uint32_t nbk = 0;
    tmp[state[0]] = 0;
    for (uint32_t i = 1; i < n; ++i) {
      if (sig_cmp(&c, state[i], state[i - 1]) != 0) ++nbk;
      tmp[state[i]] = nbk;
    }
    uint32_t newcount = nbk + 1;
    memcpy(block, tmp, sizeof(uint32_t) * n);
    if (newcount == count) break;
    ++refining;
    count = newcount;
  }
  uint32_t cb = oracle_canonicalize(n, block, out);
  if (num_blocks) *num_blocks = cb;
  if (refine_rounds) *refine_rounds = refining;
  free(sig); free(state); free(tmp);
  return 0;
}

int oracle_moore(uint32_t n, uint32_t k, const uint32_t *delta,
                 const uint8_t *accept, uint32_t max_rounds, uint32_t *out,
                 uint32_t *num_blocks, uint32_t *refine_rounds) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  uint32_t *block = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!block) return -2;
  /* {F, Q\F}; labels must stay below n, so a lone state is labelled 0 */
  for (uint32_t q = 0; q < n; ++q) block[q] = (ACC(accept, q) || n == 1) ? 0u : 1u;
  rc = moore_core(n, k, delta, block, max_rounds, 0, out, num_blocks, refine_rounds);
  free(block);
  return rc;
}

int oracle_moore_partial(uint32_t n, uint32_t k, const uint32_t *delta,
                         const uint8_t *accept, uint32_t rounds, uint32_t *out,
                         uint32_t *num_blocks, uint32_t *refine_rounds) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  uint32_t *block = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!block) return -2;
  for (uint32_t q = 0; q < n; ++q) block[q] = (ACC(accept, q) || n == 1) ? 0u : 1u;
  if (rounds == 0) {
    uint32_t c = oracle_canonicalize(n, block, out);
    if (num_blocks) *num_blocks = c;
    if (refine_rounds) *refine_rounds = 0;
    free(block);
    return 0;
  }
  rc = moore_core(n, k, delta, block, rounds, 1, out, num_blocks, refine_rounds);
  free(block);
  return rc;
}

int oracle_moore_from(uint32_t n, uint32_t k, const uint32_t *delta,
                      const uint32_t *init, uint32_t max_rounds, uint32_t *out,
                      uint32_t *num_blocks, uint32_t *refine_rounds) {
  if (n == 0 || k == 0 || !delta || !init || !out) return -1;
  for (size_t i = 0; i < (size_t)n * k; ++i)
    if (delta[i] >= n) return -1;
  uint32_t *block = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!block) return -2;
  for (uint32_t q = 0; q < n; ++q) {
    if (init[q] >= n) { free(block); return -1; }
    block[q] = init[q];
  }
  int rc = moore_core(n, k, delta, block, max_rounds, 0, out, num_blocks, refine_rounds);
  free(block);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (naivePR, Section 3.2): blocks are named by a leader state.
 * Every iteration, each state q that differs from its leader L = block[q]
 * in some successor block (block[delta(q,a)] != block[delta(L,a)]) takes
 * part in electing new_leader[L]; then every such state moves to block
 * new_leader[L].  The paper elects by concurrent writes (any writer may
 * win); here the least candidate wins, which keeps every leader the least
 * member of its block and makes the iteration count reproducible.  Both
 * phases read the partition of the start of the iteration (the synchronous
 * parallel step the algorithm is written for).  *iterations counts the
 * while-loop iterations including the last, which finds the partition
 * stable.  The initial leaders are the least accepting and the least
 * non-accepting state. */
int oracle_naive(uint32_t n, uint32_t k, const uint32_t *delta,
                 const uint8_t *accept, uint32_t max_iter, uint32_t *out,
                 uint32_t *num_blocks, uint32_t *iterations) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  uint32_t *block = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *new_leader = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint8_t *differs = (uint8_t *)malloc(n);
  if (!block || !new_leader || !differs) {
    free(block); free(new_leader); free(differs);
    return -2;
  }
  uint32_t qf = n, qn = n;
  for (uint32_t q = 0; q < n; ++q) {
    if (ACC(accept, q)) { if (qf == n) qf = q; }
    else if (qn == n) qn = q;
  }
  for (uint32_t q = 0; q < n; ++q) {
    block[q] = ACC(accept, q) ? qf : qn;
    new_leader[q] = UINT32_MAX;
  }
  uint32_t iter = 0;
  int stable = 0;
  while (!stable) {
    if (max_iter && iter >= max_iter) {
      free(block); free(new_leader); free(differs);
      return -3;
    }
    ++iter;
    stable = 1;
    /* phase 1: compare with the leader, elect the new leader */
    for (uint32_t q = 0; q < n; ++q) {
      const uint32_t L = block[q];
      differs[q] = 0;
      for (uint32_t a = 0; a < k; ++a)
        if (block[delta[(size_t)a * n + q]] != block[delta[(size_t)a * n + L]]) differs[q] = 1;
      if (differs[q] && q < new_leader[L]) new_leader[L] = q;
    }
    /* phase 2: split the differing states from their leader */
    for (uint32_t q = 0; q < n; ++q) {
      if (!differs[q]) continue;
      block[q] = new_leader[block[q]];
      stable = 0;
    }
    for (uint32_t q = 0; q < n; ++q) new_leader[q] = UINT32_MAX;
  }
  const uint32_t c = oracle_canonicalize(n, block, out);
  if (num_blocks) *num_blocks = c;
  if (iterations) *iterations = iter;
  free(block); free(new_leader); free(differs);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 5, closure part: level 0 is delta; level i is level i-1
 * applied twice (pointer jumping). */
int oracle_closure(uint32_t n, uint32_t k, const uint32_t *delta, uint32_t L,
                   uint32_t *rows) {
  if (n == 0 || k == 0 || !delta || !rows) return -1;
  for (size_t i = 0; i < (size_t)n * k; ++i)
    if (delta[i] >= n) return -1;
  for (uint32_t a = 0; a < k; ++a) {
    uint32_t *lvl0 = rows + ((size_t)a * (L + 1)) * n;
    memcpy(lvl0, delta + (size_t)a * n, sizeof(uint32_t) * n);
    for (uint32_t i = 1; i <= L; ++i) {
      const uint32_t *prev = rows + ((size_t)a * (L + 1) + i - 1) * n;
      uint32_t *cur = rows + ((size_t)a * (L + 1) + i) * n;
      for (uint32_t q = 0; q < n; ++q) cur[q] = prev[prev[q]];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Pair marking (table filling). */
int oracle_pair_marking(uint32_t n, uint32_t k, const uint32_t *delta,
                        const uint8_t *accept, uint32_t *out,
                        uint32_t *num_blocks) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  uint8_t *mark = (uint8_t *)calloc((size_t)n * n, 1);
  uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!mark || !lab) { free(mark); free(lab); return -2; }
  for (uint32_t p = 0; p < n; ++p)
    for (uint32_t q = 0; q < n; ++q)
      mark[(size_t)p * n + q] = ACC(accept, p) != ACC(accept, q);
  int changed = 1;
  while (changed) {
    changed = 0;
    for (uint32_t p = 0; p < n; ++p)
      for (uint32_t q = p + 1; q < n; ++q) {
        if (mark[(size_t)p * n + q]) continue;
        for (uint32_t a = 0; a < k; ++a) {
          uint32_t pp = delta[(size_t)a * n + p], qq = delta[(size_t)a * n + q];
          if (mark[(size_t)pp * n + qq]) {
            mark[(size_t)p * n + q] = mark[(size_t)q * n + p] = 1;
            changed = 1;
            break;
          }
        }
      }
  }
  /* label = least state not marked apart from q */
  for (uint32_t q = 0; q < n; ++q) {
    uint32_t l = q;
    for (uint32_t p = 0; p < q; ++p)
      if (!mark[(size_t)p * n + q]) { l = p; break; }
    lab[q] = l;
  }
  uint32_t c = oracle_canonicalize(n, lab, out);
  if (num_blocks) *num_blocks = c;
  free(mark); free(lab);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Literal language equivalence on all words of length <= n-1. */
int oracle_word_equivalence(uint32_t n, uint32_t k, const uint32_t *delta,
                            const uint8_t *accept, uint32_t *out,
                            uint32_t *num_blocks) {
  int rc = check_args(n, k, delta, accept, out);
  if (rc) return rc;
  uint32_t maxlen = n > 1 ? n - 1 : 0;
  /* number of words sum_{l<=maxlen} k^l */
  uint64_t words = 0, pw = 1;
  for (uint32_t l = 0; l <= maxlen; ++l) {
    words += pw;
    if (words > (1u << 22)) return -3;
    pw *= k;
  }
  /* resp[q * words + w] = acceptance of state q after word w */
  uint8_t *resp = (uint8_t *)malloc((size_t)n * words);
  uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *digits = (uint32_t *)malloc(sizeof(uint32_t) * (maxlen + 1));
  if (!resp || !lab || !digits) { free(resp); free(lab); free(digits); return -2; }
  uint64_t w = 0;
  for (uint32_t l = 0; l <= maxlen; ++l) {
    uint64_t cnt = 1;
    for (uint32_t i = 0; i < l; ++i) cnt *= k;
    for (uint64_t x = 0; x < cnt; ++x, ++w) {
      uint64_t y = x;
      for (uint32_t i = 0; i < l; ++i) { digits[i] = (uint32_t)(y % k); y /= k; }
      for (uint32_t q = 0; q < n; ++q) {
        uint32_t s = q;
        for (uint32_t i = 0; i < l; ++i) s = delta[(size_t)digits[i] * n + s];
        resp[(size_t)q * words + w] = (uint8_t)ACC(accept, s);
      }
    }
  }
  for (uint32_t q = 0; q < n; ++q) {
    uint32_t l = q;
    for (uint32_t p = 0; p < q; ++p)
      if (memcmp(resp + (size_t)p * words, resp + (size_t)q * words, words) == 0) { l = p; break; }
    lab[q] = l;
  }
  uint32_t c = oracle_canonicalize(n, lab, out);
  if (num_blocks) *num_blocks = c;
  free(resp); free(lab); free(digits);
  return 0;
}

/* ------------------------------------------------------------------------ */
uint32_t oracle_reachable(uint32_t n, uint32_t k, const uint32_t *delta,
                          uint32_t q0, uint8_t *mark) {
  if (n == 0 || q0 >= n || !delta || !mark) return 0;
  uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!queue) return 0;
  memset(mark, 0, n);
  uint32_t head = 0, tail = 0;
  mark[q0] = 1;
  queue[tail++] = q0;
  while (head < tail) {
    uint32_t q = queue[head++];
    for (uint32_t a = 0; a < k; ++a) {
      uint32_t s = delta[(size_t)a * n + q];
      if (s < n && !mark[s]) { mark[s] = 1; queue[tail++] = s; }
    }
  }
  free(queue);
  return tail;
}

/* ------------------------------------------------------------------------ */
/* The minimal DFA in the textbook sense (Section 2): the quotient by the
 * equivalence of the states reachable from q0.  Its states are the classes
 * that contain a reachable state, numbered by least member; from class c
 * (least member r) letter a leads to the class of delta(r, a) -- the same
 * class for every member, since the equivalence is a congruence; c is
 * accepting iff r is; the initial state is the class of q0.  min_delta holds
 * (*min_n) entries per letter, letter-major (capacity k*n); min_accept is an
 * LSB-first bitmap (capacity ceil(n/8) bytes). */
int oracle_minimal_dfa(uint32_t n, uint32_t k, const uint32_t *delta,
                       const uint8_t *accept, uint32_t q0, uint32_t *min_n,
                       uint32_t *min_delta, uint8_t *min_accept, uint32_t *min_q0,
                       uint32_t *num_reachable) {
  if (n == 0 || k == 0 || !delta || !accept || !min_n || !min_delta || !min_accept || !min_q0 || q0 >= n)
    return -1;
  uint32_t *cls = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint8_t *reach = (uint8_t *)malloc(n);
  uint32_t *rep = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *rid = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!cls || !reach || !rep || !rid) {
    free(cls); free(reach); free(rep); free(rid);
    return -2;
  }
  uint32_t nb = 0;
  int rc = oracle_hopcroft(n, k, delta, accept, cls, &nb);
  if (rc) { free(cls); free(reach); free(rep); free(rid); return rc; }
  const uint32_t nr = oracle_reachable(n, k, delta, q0, reach);
  for (uint32_t c = 0; c < nb; ++c) { rep[c] = UINT32_MAX; rid[c] = UINT32_MAX; }
  for (uint32_t q = 0; q < n; ++q)
    if (rep[cls[q]] == UINT32_MAX) rep[cls[q]] = q;      /* least member */
  for (uint32_t q = 0; q < n; ++q)
    if (reach[q]) rid[cls[q]] = 1;                        /* class is kept */
  uint32_t m = 0;
  for (uint32_t c = 0; c < nb; ++c)
    if (rid[c] != UINT32_MAX) rid[c] = m++;
  memset(min_accept, 0, (m + 7) / 8);
  for (uint32_t c = 0; c < nb; ++c) {
    if (rid[c] == UINT32_MAX) continue;
    const uint32_t r = rep[c];
    for (uint32_t a = 0; a < k; ++a)
      min_delta[(size_t)a * m + rid[c]] = rid[cls[delta[(size_t)a * n + r]]];
    if (ACC(accept, r)) min_accept[rid[c] >> 3] |= (uint8_t)(1u << (rid[c] & 7));
  }
  *min_n = m;
  *min_q0 = rid[cls[q0]];
  if (num_reachable) *num_reachable = nr;
  free(cls); free(reach); free(rep); free(rid);
  return 0;
}

