/*
 * datagen.c -- seeded synthetic column generator.
 *
 * Input generation only: this file holds no predicate evaluation, counting,
 * compaction or any other arithmetic of the selectivity method.  Both the
 * oracle side and the device side read the arrays it writes.
 *
 * Randomness is counter based: element i of stream s under seed S is the
 * (i+1)-th output of a SplitMix64 sequence (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) whose state
 * starts at mix(S + (s+1) * gamma).  Any element can be computed on its
 * own, so the output does not depend on the number of threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function (variant 13 of Stafford's mixers). */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t dg_rand(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t state = mix64(seed + (stream + 1) * GAMMA);
  return mix64(state + (i + 1) * GAMMA);
}

/* uniform double in [0, 1) from the top 53 bits */
static double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

static void store(int width, void* out, uint64_t i, int64_t v) {
  switch (width) {
    case 1: ((int8_t*)out)[i] = (int8_t)v; break;
    case 2: ((int16_t*)out)[i] = (int16_t)v; break;
    case 4: ((int32_t*)out)[i] = (int32_t)v; break;
    default: ((int64_t*)out)[i] = v; break;
  }
}

/* ---- a tiny parallel-for over [0, n) in chunks aligned to 32 rows ------- */

typedef struct job {
  void (*fn)(const struct job*, uint64_t, uint64_t);
  uint64_t lo, hi;
  int width;
  uint64_t seed, stream;
  int64_t a, b;
  double x, y;
  const double* cdf;
  uint64_t ncodes;
  void* out;
  uint64_t* counter;
} job;

static void* run_job(void* p) {
  job* j = (job*)p;
  j->fn(j, j->lo, j->hi);
  return NULL;
}

static void parallel(job proto, uint64_t n, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  uint64_t nwords = (n + 31) / 32;
  if ((uint64_t)nthreads > nwords) nthreads = nwords > 0 ? (int)nwords : 1;
  job* jobs = (job*)calloc((size_t)nthreads, sizeof(job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  uint64_t* counts = (uint64_t*)calloc((size_t)nthreads, sizeof(uint64_t));
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = proto;
    uint64_t wlo = nwords * (uint64_t)t / (uint64_t)nthreads;
    uint64_t whi = nwords * (uint64_t)(t + 1) / (uint64_t)nthreads;
    jobs[t].lo = wlo * 32;
    jobs[t].hi = whi * 32 < n ? whi * 32 : n;
    jobs[t].counter = &counts[t];
  }
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, run_job, &jobs[t]);
  run_job(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
  if (proto.counter) {
    uint64_t s = 0;
    for (int t = 0; t < nthreads; t++) s += counts[t];
    *proto.counter = s;
  }
  free(jobs);
  free(th);
  free(counts);
}

/* ---- uniform integers in [a, b] by the multiply-high range map ---------- */

static void uniform_fn(const job* j, uint64_t lo, uint64_t hi) {
  uint64_t range = (uint64_t)(j->b - j->a) + 1;  /* 0 means the full 2^64 */
  for (uint64_t i = lo; i < hi; i++) {
    uint64_t r = dg_rand(j->seed, j->stream, i);
    uint64_t off = range ? (uint64_t)(((unsigned __int128)r * range) >> 64) : r;
    store(j->width, j->out, i, (int64_t)((uint64_t)j->a + off));
  }
}

void dg_uniform(int width, uint64_t seed, uint64_t stream, int64_t a, int64_t b,
                void* out, uint64_t n, int nthreads) {
  job p;
  memset(&p, 0, sizeof p);
  p.fn = uniform_fn;
  p.width = width;
  p.seed = seed;
  p.stream = stream;
  p.a = a;
  p.b = b;
  p.out = out;
  parallel(p, n, nthreads);
}

/* ---- Zipf(s) over ranks 1..C, stored as code = rank - 1 ----------------- */

/* cdf[k] = P(rank <= k+1), k = 0..C-1 (cdf[C-1] forced to 1). */
void dg_zipf_cdf(double s, uint64_t C, double* cdf) {
  double z = 0.0;
  for (uint64_t k = 1; k <= C; k++) z += pow((double)k, -s);
  double acc = 0.0;
  for (uint64_t k = 1; k <= C; k++) {
    acc += pow((double)k, -s) / z;
    cdf[k - 1] = acc;
  }
  cdf[C - 1] = 1.0;
}

static void zipf_fn(const job* j, uint64_t lo, uint64_t hi) {
  for (uint64_t i = lo; i < hi; i++) {
    double u = u01(dg_rand(j->seed, j->stream, i));
    uint64_t l = 0, h = j->ncodes - 1; /* first k with u < cdf[k] */
    while (l < h) {
      uint64_t m = (l + h) / 2;
      if (u < j->cdf[m]) h = m; else l = m + 1;
    }
    store(j->width, j->out, i, (int64_t)l);
  }
}

void dg_zipf(int width, uint64_t seed, uint64_t stream, const double* cdf, uint64_t ncodes,
             void* out, uint64_t n, int nthreads) {
  job p;
  memset(&p, 0, sizeof p);
  p.fn = zipf_fn;
  p.width = width;
  p.seed = seed;
  p.stream = stream;
  p.cdf = cdf;
  p.ncodes = ncodes;
  p.out = out;
  parallel(p, n, nthreads);
}

/* ---- log-normal(mu, sigma) rounded to int64, by Box-Muller -------------- */

static void lognormal_fn(const job* j, uint64_t lo, uint64_t hi) {
  const double two_pi = 6.283185307179586476925286766559;
  for (uint64_t i = lo; i < hi; i++) {
    double u1 = 1.0 - u01(dg_rand(j->seed, j->stream, 2 * i));  /* (0, 1] */
    double u2 = u01(dg_rand(j->seed, j->stream, 2 * i + 1));
    double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    store(8, j->out, i, (int64_t)llround(exp(j->x + j->y * z)));
  }
}

void dg_lognormal_i64(uint64_t seed, uint64_t stream, double mu, double sigma, int64_t* out,
                      uint64_t n, int nthreads) {
  job p;
  memset(&p, 0, sizeof p);
  p.fn = lognormal_fn;
  p.seed = seed;
  p.stream = stream;
  p.x = mu;
  p.y = sigma;
  p.out = out;
  parallel(p, n, nthreads);
}

/* ---- validity: each row NULL with probability rate (Bernoulli) ---------- */

static void validity_fn(const job* j, uint64_t lo, uint64_t hi) {
  /* threshold on the top 53 bits: NULL iff r>>11 < rate * 2^53 */
  uint64_t thr = (uint64_t)(j->x * 9007199254740992.0);
  uint32_t* words = (uint32_t*)j->out;
  uint64_t nulls = 0;
  for (uint64_t w = lo / 32; w * 32 < hi; w++) {
    uint32_t v = 0;
    for (uint64_t b = 0; b < 32; b++) {
      uint64_t i = w * 32 + b;
      if (i >= hi) break;
      int null = (dg_rand(j->seed, j->stream, i) >> 11) < thr;
      if (null) nulls++; else v |= 1u << b;
    }
    words[w] = v;
  }
  *j->counter = nulls;
}

/* Writes ceil(n/32) words; returns the number of NULL rows. */
uint64_t dg_validity(uint64_t seed, uint64_t stream, double rate, uint32_t* words, uint64_t n,
                     int nthreads) {
  uint64_t nulls = 0;
  job p;
  memset(&p, 0, sizeof p);
  p.fn = validity_fn;
  p.seed = seed;
  p.stream = stream;
  p.x = rate;
  p.out = words;
  p.counter = &nulls;
  parallel(p, n, nthreads);
  return nulls;
}

/* Overwrite the data slot of every NULL row with `v` (used to plant values
 * that would satisfy a predicate if NULLs were not handled). */
void dg_fill_nulls(int width, void* data, const uint32_t* valid, uint64_t n, int64_t v) {
  for (uint64_t i = 0; i < n; i++)
    if (((valid[i / 32] >> (i % 32)) & 1u) == 0) store(width, data, i, v);
}

/* out[i] = (i >> shift) + base */
void dg_iota(int width, void* out, uint64_t n, uint32_t shift, int64_t base) {
  for (uint64_t i = 0; i < n; i++) store(width, out, i, (int64_t)(i >> shift) + base);
}

/* bit c of words (nbits bits) set iff dg_rand(seed, stream, c) % mod == 0 */
void dg_code_bitmap(uint64_t seed, uint64_t stream, uint64_t mod, uint32_t* words, uint64_t nbits) {
  memset(words, 0, (size_t)((nbits + 31) / 32) * 4);
  for (uint64_t c = 0; c < nbits; c++)
    if (dg_rand(seed, stream, c) % mod == 0) words[c / 32] |= 1u << (c % 32);
}

/* FNV-1a 64 over a byte range (data checksums). */
uint64_t dg_fnv1a(const void* p, uint64_t nbytes) {
  const uint8_t* b = (const uint8_t*)p;
  uint64_t h = 0xcbf29ce484222325ULL;
  for (uint64_t i = 0; i < nbytes; i++) {
    h ^= b[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}
