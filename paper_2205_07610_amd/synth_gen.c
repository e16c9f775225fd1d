/* Seeded residue and mutation generator for large synthetic batches.
 *
 * Input generation only: no alignment arithmetic.  Every sequence draws from
 * its own counter-based stream, x_k = splitmix64(key + k * 0x9E3779B97F4A7C15)
 * with key = splitmix64(seed ^ (index * 0xD1B54A32D192ED03)), so the output
 * does not depend on the number of threads.
 *
 * Mutation model, per source residue in order (the same law as the Python
 * generator): with probability p_sub it is replaced by a uniformly different
 * residue; with p_ins, L ~ Geometric(1/2) random residues are inserted before
 * it; with p_del, it and the next L - 1 residues (not past the sequence's
 * end) are deleted.  Events at deleted positions still insert; deletions
 * overlap as a union.
 */
#include <pthread.h>
#include <stdint.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t key, ctr;
} stream_t;

static inline stream_t stream_for(uint64_t seed, int64_t index) {
  stream_t s;
  s.key = mix64(seed ^ ((uint64_t)index * 0xD1B54A32D192ED03ULL));
  s.ctr = 0;
  return s;
}
static inline uint64_t next64(stream_t *s) {
  s->ctr += 0x9E3779B97F4A7C15ULL;
  return mix64(s->key + s->ctr);
}
static inline double next_unit(stream_t *s) { return (double)(next64(s) >> 11) * (1.0 / 9007199254740992.0); }
static inline uint32_t next_below(stream_t *s, uint32_t k) {
  return (uint32_t)(((next64(s) >> 32) * (uint64_t)k) >> 32);
}
static inline int64_t next_geometric_half(stream_t *s) {
  uint64_t r = next64(s);
  while (r == 0) r = next64(s);
  return 1 + __builtin_ctzll(r);
}

typedef struct {
  int64_t lo, hi;
  uint64_t seed;
  const int64_t *offs;
  uint8_t *out;
  int asz;
  /* mutation */
  const int64_t *src_offs;
  const uint8_t *src;
  const double *p_sub, *p_ins, *p_del;
  const int64_t *dst_offs;
  uint8_t *dst;
  int64_t *dst_lens;
} job_t;

static void *residues_job(void *arg) {
  job_t *j = (job_t *)arg;
  for (int64_t p = j->lo; p < j->hi; ++p) {
    stream_t s = stream_for(j->seed, p);
    uint8_t *o = j->out + j->offs[p];
    const int64_t n = j->offs[p + 1] - j->offs[p];
    if (j->asz == 4) {
      int64_t i = 0;
      while (i < n) {
        uint64_t r = next64(&s);
        for (int b = 0; b < 32 && i < n; ++b, ++i, r >>= 2) o[i] = (uint8_t)(r & 3u);
      }
    } else {
      for (int64_t i = 0; i < n; ++i) o[i] = (uint8_t)next_below(&s, (uint32_t)j->asz);
    }
  }
  return 0;
}

static void *mutate_job(void *arg) {
  job_t *j = (job_t *)arg;
  for (int64_t p = j->lo; p < j->hi; ++p) {
    stream_t s = stream_for(j->seed, p);
    const uint8_t *a = j->src + j->src_offs[p];
    const int64_t m = j->src_offs[p + 1] - j->src_offs[p];
    const double ps = j->p_sub[p], pi = ps + j->p_ins[p], pd = pi + j->p_del[p];
    uint8_t *o = j->dst ? j->dst + j->dst_offs[p] : 0;
    int64_t k = 0, skip_until = 0;
    for (int64_t i = 0; i < m; ++i) {
      const double u = next_unit(&s);
      uint8_t c = a[i];
      if (u < ps) {
        c = (uint8_t)((c + 1 + next_below(&s, (uint32_t)(j->asz - 1))) % j->asz);
      } else if (u < pi) {
        const int64_t L = next_geometric_half(&s);
        for (int64_t t = 0; t < L; ++t, ++k) {
          const uint8_t r = (uint8_t)next_below(&s, (uint32_t)j->asz);
          if (o) o[k] = r;
        }
      } else if (u < pd) {
        const int64_t end = i + next_geometric_half(&s);
        if (end > skip_until) skip_until = end < m ? end : m;
      }
      if (i >= skip_until) {
        if (o) o[k] = c;
        ++k;
      }
    }
    if (j->dst_lens) j->dst_lens[p] = k;
  }
  return 0;
}

static void run_jobs(job_t *base, int64_t n, int nthreads, void *(*fn)(void *)) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  job_t jobs[256];
  const int64_t chunk = (n + nthreads - 1) / nthreads;
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = *base;
    jobs[t].lo = (int64_t)t * chunk;
    jobs[t].hi = jobs[t].lo + chunk < n ? jobs[t].lo + chunk : n;
    if (jobs[t].lo >= jobs[t].hi) break;
    if (pthread_create(&th[t], 0, fn, &jobs[t]) != 0) {
      fn(&jobs[t]);
      continue;
    }
    started = t + 1;
  }
  for (int t = 0; t < started; ++t) pthread_join(th[t], 0);
}

/* Uniform residues 0..asz-1 for every sequence of a CSR batch. */
void synth_residues(uint64_t seed, int64_t n_seq, const int64_t *offs, int asz, uint8_t *out, int nthreads) {
  job_t j;
  memset(&j, 0, sizeof(j));
  j.seed = seed;
  j.offs = offs;
  j.out = out;
  j.asz = asz;
  run_jobs(&j, n_seq, nthreads, residues_job);
}

/* Mutated copies: with dst == NULL only dst_lens is written (first pass);
 * the second pass, with dst_offs the prefix sums of those lengths, writes
 * the residues.  Both passes draw the same streams. */
void synth_mutate(uint64_t seed, int64_t n_seq, const int64_t *src_offs, const uint8_t *src, const double *p_sub,
                  const double *p_ins, const double *p_del, int asz, const int64_t *dst_offs, uint8_t *dst,
                  int64_t *dst_lens, int nthreads) {
  job_t j;
  memset(&j, 0, sizeof(j));
  j.seed = seed;
  j.asz = asz;
  j.src_offs = src_offs;
  j.src = src;
  j.p_sub = p_sub;
  j.p_ins = p_ins;
  j.p_del = p_del;
  j.dst_offs = dst_offs;
  j.dst = dst;
  j.dst_lens = dst_lens;
  run_jobs(&j, n_seq, nthreads, mutate_job);
}
