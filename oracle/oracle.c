/*
 * oracle.c -- the CPU reference for the exact-selectivity path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (libsel and its Python
 * binding) may include, link, load or call this file; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * What it computes, from the thesis (Shin 2018, arXiv:1806.08384):
 *  - Ch.3 sec.3.1: the selectivity of a pushed-down selection sigma(R) is
 *    the answer of SELECT COUNT(*) FROM R WHERE <R's predicates>, i.e. the
 *    exact number of rows of R that satisfy the selection.  oc_count is that
 *    definition written out: one plain loop over the rows, one recursive
 *    walk of the predicate TREE per row (not a postfix program, so the
 *    product's compiler and interpreter are checked as well).
 *  - Algorithm 1 (function Execute): the count is compared with maxSize and
 *    a count above it aborts the push-down; otherwise the selection is
 *    materialised.  oc_pushdown returns that outcome and the materialised
 *    sigma(R) as its ascending row ids.
 *  - Ch.3 sec.3.3 / Algorithm 1 push selections down on the relations that
 *    are not probed; oc_keybitmap represents such a pushed-down dimension
 *    as the set of its qualifying keys, and oc_star_count counts the fact
 *    rows whose foreign keys all fall in those sets.
 * The thesis does not discuss NULLs; the predicates are SQL WHERE clauses,
 * so SQL's three-valued logic applies: comparisons on NULL are UNKNOWN,
 * AND is the minimum and OR the maximum under FALSE < UNKNOWN < TRUE, NOT
 * swaps TRUE and FALSE, and a row counts only if its predicate is TRUE.
 *
 * Pins (tests, CPU): Kleene truth tables; SQLite on small random tables;
 * closed forms on constructed columns; invariants such as
 * count(p) + count(NOT p) + count(p IS UNKNOWN) = N.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* truth values, ordered so that AND = min and OR = max */
enum { OC_F = 0, OC_U = 1, OC_T = 2 };

enum {
  OC_CMP = 1,      /* col <cmp> v1                              */
  OC_BETWEEN = 2,  /* v1 <= col <= v2                           */
  OC_IN = 3,       /* col in i64pool[off .. off+cnt)            */
  OC_CODESET = 4,  /* 0 <= col < cnt and bit col of u32pool[off..] */
  OC_ISNULL = 5,
  OC_NOTNULL = 6,
  OC_AND = 7,      /* children[off .. off+nchild)               */
  OC_OR = 8,
  OC_NOT = 9,      /* children[off]                             */
  OC_ISUNKNOWN = 10,
  OC_TRUE = 11,
  OC_FALSE = 12
};

enum { CMP_EQ = 1, CMP_NE = 2, CMP_LT = 3, CMP_LE = 4, CMP_GT = 5, CMP_GE = 6 };

typedef struct oc_node {
  int32_t kind, col, cmp, nchild;
  int64_t v1, v2;
  int64_t off, cnt;
} oc_node;

typedef struct oc_expr {
  const oc_node* nodes;
  int32_t root;
  int32_t pad;
  const int32_t* children;
  const int64_t* i64pool;
  const uint32_t* u32pool;
} oc_expr;

typedef struct oc_col {
  int32_t width;            /* bytes per value: 1, 2, 4 or 8 (signed) */
  int32_t pad;
  const void* data;
  const uint32_t* valid;    /* NULL = no NULLs; bit i%32 of word i/32 */
} oc_col;

static int is_null(const oc_col* c, uint64_t row) {
  if (!c->valid) return 0;
  return ((c->valid[row / 32] >> (row % 32)) & 1u) == 0;
}

static int64_t value(const oc_col* c, uint64_t row) {
  switch (c->width) {
    case 1: return ((const int8_t*)c->data)[row];
    case 2: return ((const int16_t*)c->data)[row];
    case 4: return ((const int32_t*)c->data)[row];
    default: return ((const int64_t*)c->data)[row];
  }
}

static int from_bool(int b) { return b ? OC_T : OC_F; }

static int eval(const oc_expr* e, const oc_col* cols, int32_t id, uint64_t row) {
  const oc_node* n = &e->nodes[id];
  switch (n->kind) {
    case OC_TRUE: return OC_T;
    case OC_FALSE: return OC_F;
    case OC_ISNULL: return from_bool(is_null(&cols[n->col], row));
    case OC_NOTNULL: return from_bool(!is_null(&cols[n->col], row));
    case OC_CMP: {
      const oc_col* c = &cols[n->col];
      if (is_null(c, row)) return OC_U;
      int64_t x = value(c, row);
      switch (n->cmp) {
        case CMP_EQ: return from_bool(x == n->v1);
        case CMP_NE: return from_bool(x != n->v1);
        case CMP_LT: return from_bool(x < n->v1);
        case CMP_LE: return from_bool(x <= n->v1);
        case CMP_GT: return from_bool(x > n->v1);
        default: return from_bool(x >= n->v1);
      }
    }
    case OC_BETWEEN: {
      const oc_col* c = &cols[n->col];
      if (is_null(c, row)) return OC_U;
      int64_t x = value(c, row);
      return from_bool(n->v1 <= x && x <= n->v2);
    }
    case OC_IN: {
      const oc_col* c = &cols[n->col];
      if (is_null(c, row)) return OC_U;
      int64_t x = value(c, row);
      for (int64_t k = 0; k < n->cnt; k++)
        if (e->i64pool[n->off + k] == x) return OC_T;
      return OC_F;
    }
    case OC_CODESET: {
      const oc_col* c = &cols[n->col];
      if (is_null(c, row)) return OC_U;
      int64_t x = value(c, row);
      if (x < 0 || x >= n->cnt) return OC_F;
      uint32_t w = e->u32pool[n->off + x / 32];
      return from_bool((w >> (x % 32)) & 1u);
    }
    case OC_AND: {
      int r = OC_T;
      for (int32_t k = 0; k < n->nchild; k++) {
        int v = eval(e, cols, e->children[n->off + k], row);
        if (v < r) r = v;
      }
      return r;
    }
    case OC_OR: {
      int r = OC_F;
      for (int32_t k = 0; k < n->nchild; k++) {
        int v = eval(e, cols, e->children[n->off + k], row);
        if (v > r) r = v;
      }
      return r;
    }
    case OC_NOT: {
      int v = eval(e, cols, e->children[n->off], row);
      return v == OC_T ? OC_F : (v == OC_F ? OC_T : OC_U);
    }
    case OC_ISUNKNOWN:
      return from_bool(eval(e, cols, e->children[n->off], row) == OC_U);
  }
  abort();
}

/* Truth value of the predicate on one row (0 = FALSE, 1 = UNKNOWN, 2 = TRUE). */
int oc_eval_row(const oc_expr* e, const oc_col* cols, uint64_t row) {
  return eval(e, cols, e->root, row);
}

/* Truth values of all rows into out[0..nrows). */
void oc_eval_all(const oc_expr* e, const oc_col* cols, uint64_t nrows, uint8_t* out) {
  for (uint64_t i = 0; i < nrows; i++) out[i] = (uint8_t)eval(e, cols, e->root, i);
}

/* ---- COUNT(*) ... WHERE p: the count query of Ch.3 sec.3.1 ---------------- */

typedef struct count_job {
  const oc_expr* e;
  const oc_col* cols;
  uint64_t lo, hi, count;
} count_job;

static void* count_range(void* arg) {
  count_job* j = (count_job*)arg;
  uint64_t c = 0;
  for (uint64_t i = j->lo; i < j->hi; i++)
    if (eval(j->e, j->cols, j->e->root, i) == OC_T) c++;
  j->count = c;
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

/* Number of rows whose predicate is TRUE.  nthreads <= 0: one per online
 * core; rows are split into contiguous ranges and the counts summed. */
uint64_t oc_count(const oc_expr* e, const oc_col* cols, uint64_t nrows, int nthreads) {
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > nrows) nt = nrows > 0 ? (int)nrows : 1;
  count_job* jobs = (count_job*)calloc((size_t)nt, sizeof(count_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; t++) {
    jobs[t].e = e;
    jobs[t].cols = cols;
    jobs[t].lo = nrows * (uint64_t)t / (uint64_t)nt;
    jobs[t].hi = nrows * (uint64_t)(t + 1) / (uint64_t)nt;
  }
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, count_range, &jobs[t]);
  count_range(&jobs[0]);
  uint64_t total = jobs[0].count;
  for (int t = 1; t < nt; t++) {
    pthread_join(th[t], NULL);
    total += jobs[t].count;
  }
  free(jobs);
  free(th);
  return total;
}

/* ---- Execute(node, isSPD, maxSize) of Algorithm 1 ------------------------- */

/* Ascending ids of the TRUE rows; writes at most cap of them, returns the
 * total number of TRUE rows. */
uint64_t oc_rowids(const oc_expr* e, const oc_col* cols, uint64_t nrows,
                   uint32_t* out, uint64_t cap) {
  uint64_t c = 0;
  for (uint64_t i = 0; i < nrows; i++) {
    if (eval(e, cols, e->root, i) == OC_T) {
      if (c < cap) out[c] = (uint32_t)i;
      c++;
    }
  }
  return c;
}

/* The same ids with the rows split into contiguous ranges over nthreads
 * threads (<= 0: one per online core): each range is counted, the counts give
 * each range its first output position, and each range then writes its ids
 * there.  Ranges are in row order, so the concatenation is ascending and
 * equal to oc_rowids' list.  Writes at most cap ids; returns the total. */
typedef struct rowid_job {
  const oc_expr* e;
  const oc_col* cols;
  uint64_t lo, hi, count, first;
  uint32_t* out;
  uint64_t cap;
} rowid_job;

static void* rowid_count_range(void* arg) {
  rowid_job* j = (rowid_job*)arg;
  uint64_t c = 0;
  for (uint64_t i = j->lo; i < j->hi; i++)
    if (eval(j->e, j->cols, j->e->root, i) == OC_T) c++;
  j->count = c;
  return NULL;
}

static void* rowid_write_range(void* arg) {
  rowid_job* j = (rowid_job*)arg;
  uint64_t pos = j->first;
  for (uint64_t i = j->lo; i < j->hi; i++) {
    if (eval(j->e, j->cols, j->e->root, i) == OC_T) {
      if (pos < j->cap) j->out[pos] = (uint32_t)i;
      pos++;
    }
  }
  return NULL;
}

uint64_t oc_rowids_mt(const oc_expr* e, const oc_col* cols, uint64_t nrows,
                      uint32_t* out, uint64_t cap, int nthreads) {
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > nrows) nt = nrows > 0 ? (int)nrows : 1;
  rowid_job* jobs = (rowid_job*)calloc((size_t)nt, sizeof(rowid_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; t++) {
    jobs[t].e = e;
    jobs[t].cols = cols;
    jobs[t].lo = nrows * (uint64_t)t / (uint64_t)nt;
    jobs[t].hi = nrows * (uint64_t)(t + 1) / (uint64_t)nt;
    jobs[t].out = out;
    jobs[t].cap = cap;
  }
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, rowid_count_range, &jobs[t]);
  rowid_count_range(&jobs[0]);
  for (int t = 1; t < nt; t++) pthread_join(th[t], NULL);
  uint64_t total = 0;
  for (int t = 0; t < nt; t++) {
    jobs[t].first = total;
    total += jobs[t].count;
  }
  if (out != NULL && cap > 0) {
    for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, rowid_write_range, &jobs[t]);
    rowid_write_range(&jobs[0]);
    for (int t = 1; t < nt; t++) pthread_join(th[t], NULL);
  }
  free(jobs);
  free(th);
  return total;
}

/* Algorithm 1: count first; a count above max_rows aborts (status 1, nothing
 * written); a count above the caller's capacity is status 2 (nothing
 * written); otherwise the ascending ids are written (status 0). */
int oc_pushdown(const oc_expr* e, const oc_col* cols, uint64_t nrows,
                uint64_t max_rows, uint32_t* out, uint64_t cap, uint64_t* count) {
  uint64_t c = oc_count(e, cols, nrows, 1);
  *count = c;
  if (c > max_rows) return 1;
  if (c > cap) return 2;
  oc_rowids(e, cols, nrows, out, cap);
  return 0;
}

/* A pushed-down dimension as a key bitmap: bit (key - key_min) is set for
 * every qualifying row.  e == NULL means every row qualifies.  Returns 0, or
 * -6 if a qualifying key lies outside [key_min, key_min + nbits). */
int oc_keybitmap(const oc_expr* e, const oc_col* cols, uint64_t nrows, int32_t key_col,
                 int64_t key_min, uint32_t* bitmap, uint64_t nbits, uint64_t* count) {
  memset(bitmap, 0, (size_t)((nbits + 31) / 32) * sizeof(uint32_t));
  uint64_t c = 0;
  int status = 0;
  for (uint64_t i = 0; i < nrows; i++) {
    if (e && eval(e, cols, e->root, i) != OC_T) continue;
    c++;
    int64_t k = value(&cols[key_col], i);
    if (k < key_min || (uint64_t)(k - key_min) >= nbits) {
      status = -6;
      continue;
    }
    uint64_t b = (uint64_t)(k - key_min);
    bitmap[b / 32] |= 1u << (b % 32);
  }
  *count = c;
  return status;
}

/* ---- star semi-join count ------------------------------------------------- */

typedef struct star_job {
  const oc_expr* e;
  const oc_col* cols;
  int32_t nfk;
  const int32_t* fk_cols;
  const uint32_t* const* bitmaps;
  const uint64_t* nbits;
  uint64_t lo, hi, count;
} star_job;

static int star_row(const star_job* j, uint64_t i) {
  for (int32_t d = 0; d < j->nfk; d++) {
    const oc_col* c = &j->cols[j->fk_cols[d]];
    if (is_null(c, i)) return 0;
    int64_t k = value(c, i);
    if (k < 0 || (uint64_t)k >= j->nbits[d]) return 0;
    if (((j->bitmaps[d][k / 32] >> (k % 32)) & 1u) == 0) return 0;
  }
  if (j->e && eval(j->e, j->cols, j->e->root, i) != OC_T) return 0;
  return 1;
}

static void* star_range(void* arg) {
  star_job* j = (star_job*)arg;
  uint64_t c = 0;
  for (uint64_t i = j->lo; i < j->hi; i++) c += (uint64_t)star_row(j, i);
  j->count = c;
  return NULL;
}

/* Fact rows whose every foreign key hits a set bit of its dimension bitmap
 * (and, if e != NULL, whose own predicate is TRUE). */
uint64_t oc_star_count(const oc_expr* e, const oc_col* cols, uint64_t nrows, int32_t nfk,
                       const int32_t* fk_cols, const uint32_t* const* bitmaps,
                       const uint64_t* nbits, int nthreads) {
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > nrows) nt = nrows > 0 ? (int)nrows : 1;
  star_job* jobs = (star_job*)calloc((size_t)nt, sizeof(star_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; t++) {
    star_job j = {e, cols, nfk, fk_cols, bitmaps, nbits,
                  nrows * (uint64_t)t / (uint64_t)nt,
                  nrows * (uint64_t)(t + 1) / (uint64_t)nt, 0};
    jobs[t] = j;
  }
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, star_range, &jobs[t]);
  star_range(&jobs[0]);
  uint64_t total = jobs[0].count;
  for (int t = 1; t < nt; t++) {
    pthread_join(th[t], NULL);
    total += jobs[t].count;
  }
  free(jobs);
  free(th);
  return total;
}
