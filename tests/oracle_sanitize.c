/*
 * Driver for the sanitizer build of the C oracle (tests only): linked with
 * oracle/oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer, it
 * runs every exported entry point on small random pairs (empty sequences
 * included, several alphabets and gap costs, all three modes, one and
 * several threads) and checks relations that hold for any correct oracle:
 *   - a band wide enough to hold the whole matrix gives the full score;
 *   - explicit diagonal limits covering the matrix give the full score;
 *   - the batch drivers agree with the pair functions, for 1 and 3 threads;
 *   - a traceback's alignment, rescored from its columns, equals its score,
 *     and that score equals the score-only optimum;
 *   - local >= semi-global >= global for the same pair.
 * Prints "ok" and exits 0, or names the first failing case and exits 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_align_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n, const int8_t *subst,
                          int32_t asz, int64_t alpha, int64_t beta, int32_t mode);
int64_t oracle_banded_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n, const int8_t *subst,
                           int32_t asz, int64_t alpha, int64_t beta, int32_t mode, int64_t w);
int64_t oracle_diag_band_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n, const int8_t *subst,
                              int32_t asz, int64_t alpha, int64_t beta, int32_t mode, int64_t lo, int64_t hi);
void oracle_align_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                        const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                        int64_t alpha, int64_t beta, int32_t mode, int32_t nthreads, int64_t *out);
void oracle_banded_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                         const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                         int64_t alpha, int64_t beta, int32_t mode, const int64_t *band_w,
                         int32_t nthreads, int64_t *out);
int64_t oracle_alignment_score(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n, const int8_t *subst,
                               int32_t asz, int64_t alpha, int64_t beta, int32_t mode, const uint8_t *ops,
                               int64_t n_ops, const int32_t *span);
int64_t oracle_traceback_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n, const int8_t *subst,
                              int32_t asz, int64_t alpha, int64_t beta, int32_t mode, uint8_t *ops_out,
                              int32_t *span_out);
void oracle_traceback_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                            const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                            int64_t alpha, int64_t beta, int32_t mode, int32_t nthreads, uint8_t *ops,
                            int32_t *span, int64_t *out);
void oracle_alignment_score_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                  const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                                  int64_t alpha, int64_t beta, int32_t mode, int32_t nthreads,
                                  const uint8_t *ops, const int32_t *span, int64_t *out);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(uint32_t bound) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)((rng_state >> 33) % bound);
}

#define FAIL(...)                  \
  do {                             \
    printf(__VA_ARGS__);           \
    printf("\n");                  \
    return 1;                      \
  } while (0)

int main(void) {
  enum { kPairs = 160, kMaxLen = 48 };
  for (int trial = 0; trial < 12; ++trial) {
    const int asz = (int)(2 + rnd(19));
    int8_t *subst = (int8_t *)malloc((size_t)(asz * asz));
    for (int i = 0; i < asz * asz; ++i) subst[i] = (int8_t)((int)rnd(9) - 5);
    for (int i = 0; i < asz; ++i) subst[i * asz + i] = (int8_t)(1 + rnd(5));
    const int64_t beta = rnd(4), alpha = beta + rnd(6);
    /* CSR batch; lengths 0..kMaxLen, B sometimes a copy of A */
    int64_t offs_a[kPairs + 1], offs_b[kPairs + 1];
    offs_a[0] = offs_b[0] = 0;
    uint8_t *sa = (uint8_t *)malloc(kPairs * kMaxLen + 1), *sb = (uint8_t *)malloc(kPairs * kMaxLen + 1);
    for (int p = 0; p < kPairs; ++p) {
      const int64_t m = rnd(kMaxLen + 1), n = rnd(4) == 0 ? m : rnd(kMaxLen + 1);
      for (int64_t k = 0; k < m; ++k) sa[offs_a[p] + k] = (uint8_t)rnd((uint32_t)asz);
      for (int64_t k = 0; k < n; ++k)
        sb[offs_b[p] + k] = (n == m && rnd(3)) ? sa[offs_a[p] + k] : (uint8_t)rnd((uint32_t)asz);
      offs_a[p + 1] = offs_a[p] + m;
      offs_b[p + 1] = offs_b[p] + n;
    }
    int64_t full[3][kPairs];
    for (int mode = 0; mode < 3; ++mode) {
      int64_t out1[kPairs], out3[kPairs], band_out[kPairs], wide[kPairs], tb_out[kPairs], rescored[kPairs];
      oracle_align_batch(sa, offs_a, sb, offs_b, kPairs, subst, asz, alpha, beta, mode, 1, out1);
      oracle_align_batch(sa, offs_a, sb, offs_b, kPairs, subst, asz, alpha, beta, mode, 3, out3);
      for (int p = 0; p < kPairs; ++p) wide[p] = 2 * kMaxLen + 2;
      oracle_banded_batch(sa, offs_a, sb, offs_b, kPairs, subst, asz, alpha, beta, mode, wide, 3, band_out);
      uint8_t *ops = (uint8_t *)malloc((size_t)(offs_a[kPairs] + offs_b[kPairs] + 1));
      int32_t *span = (int32_t *)malloc(sizeof(int32_t) * 5 * kPairs);
      oracle_traceback_batch(sa, offs_a, sb, offs_b, kPairs, subst, asz, alpha, beta, mode, 3, ops, span,
                             tb_out);
      oracle_alignment_score_batch(sa, offs_a, sb, offs_b, kPairs, subst, asz, alpha, beta, mode, 3, ops, span,
                                   rescored);
      for (int p = 0; p < kPairs; ++p) {
        const uint8_t *q = sa + offs_a[p], *s = sb + offs_b[p];
        const int64_t m = offs_a[p + 1] - offs_a[p], n = offs_b[p + 1] - offs_b[p];
        const int64_t v = oracle_align_pair(q, m, s, n, subst, asz, alpha, beta, mode);
        full[mode][p] = v;
        if (out1[p] != v || out3[p] != v) FAIL("batch/pair differ: trial %d mode %d pair %d", trial, mode, p);
        if (band_out[p] != v) FAIL("wide band differs: trial %d mode %d pair %d", trial, mode, p);
        if (oracle_banded_pair(q, m, s, n, subst, asz, alpha, beta, mode, m + n + 1) != v)
          FAIL("wide banded pair differs: trial %d mode %d pair %d", trial, mode, p);
        if (oracle_diag_band_pair(q, m, s, n, subst, asz, alpha, beta, mode, -m, n) != v)
          FAIL("full diagonal range differs: trial %d mode %d pair %d", trial, mode, p);
        if (tb_out[p] != v || rescored[p] != v)
          FAIL("traceback score %lld rescored %lld optimum %lld: trial %d mode %d pair %d", (long long)tb_out[p],
               (long long)rescored[p], (long long)v, trial, mode, p);
        uint8_t one_ops[2 * kMaxLen + 1];
        int32_t one_span[5];
        const int64_t tv = oracle_traceback_pair(q, m, s, n, subst, asz, alpha, beta, mode, one_ops, one_span);
        if (tv != v || oracle_alignment_score(q, m, s, n, subst, asz, alpha, beta, mode, one_ops, one_span[0],
                                              one_span + 1) != v)
          FAIL("pair traceback differs: trial %d mode %d pair %d", trial, mode, p);
      }
      free(ops);
      free(span);
    }
    for (int p = 0; p < kPairs; ++p)
      if (!(full[2][p] >= full[1][p] && full[1][p] >= full[0][p]))
        FAIL("mode order violated: trial %d pair %d: %lld %lld %lld", trial, p, (long long)full[0][p],
             (long long)full[1][p], (long long)full[2][p]);
    free(sa);
    free(sb);
    free(subst);
  }
  printf("ok\n");
  return 0;
}
