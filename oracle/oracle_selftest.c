/*
 * oracle_selftest.c -- exhaustive cross-check of the oracle's independent
 * algorithms over every small complete DFA.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * For given n and k, every transition function in [0,n)^(n*k) is combined
 * with every accepting set in 2^Q.  Hopcroft, pair marking and Moore must
 * return the same canonical partition; for n <= 4 the literal word
 * enumeration is checked as well.  Any disagreement means one of them has
 * a bug (a dropped split, a wrong index, a transposed operand, ...).
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

uint64_t oracle_exhaustive_check(uint32_t n, uint32_t k, uint64_t *mismatches) {
  if (n == 0 || k == 0 || n > 6 || (size_t)n * k > 12) {
    if (mismatches) *mismatches = 0;
    return 0;
  }
  uint32_t nk = n * k;
  uint32_t delta[12];
  uint8_t acc[1];
  uint32_t o1[8], o2[8], o3[8], o4[8], o5[8];
  uint64_t checked = 0, bad = 0;
  memset(delta, 0, sizeof(delta));
  for (;;) {
    for (uint32_t fm = 0; fm < (1u << n); ++fm) {
      acc[0] = (uint8_t)fm;
      uint32_t c1 = 0, c2 = 0, c3 = 0, c4 = 0, r = 0;
      int e1 = oracle_hopcroft(n, k, delta, acc, o1, &c1);
      int e2 = oracle_pair_marking(n, k, delta, acc, o2, &c2);
      int e3 = oracle_moore(n, k, delta, acc, 0, o3, &c3, &r);
      int ok = !e1 && !e2 && !e3 && c1 == c2 && c2 == c3 &&
               !memcmp(o1, o2, n * sizeof(uint32_t)) &&
               !memcmp(o2, o3, n * sizeof(uint32_t));
      /* Moore refines at most n-2 times for n >= 2, never for n = 1. */
      if (r > (n >= 2 ? n - 2 : 0)) ok = 0;
      /* Algorithm 2 reaches the same partition; each of its iterations
       * but the last adds at least one block, so it runs at most n. */
      uint32_t c5 = 0, it5 = 0;
      int e5 = oracle_naive(n, k, delta, acc, 0, o5, &c5, &it5);
      ok = ok && !e5 && c5 == c1 && !memcmp(o1, o5, n * sizeof(uint32_t)) && it5 >= 1 && it5 <= n;
      if (n <= 4) {
        int e4 = oracle_word_equivalence(n, k, delta, acc, o4, &c4);
        ok = ok && !e4 && c4 == c1 && !memcmp(o1, o4, n * sizeof(uint32_t));
      }
      bad += !ok;
      ++checked;
    }
    /* next transition function (odometer over nk digits in base n) */
    uint32_t i = 0;
    while (i < nk) {
      if (++delta[i] < n) break;
      delta[i] = 0;
      ++i;
    }
    if (i == nk) break;
  }
  if (mismatches) *mismatches = bad;
  return checked;
}
