/*
 * sel.h -- C ABI of libsel, exact selectivity by a COUNT scan (gfx950).
 *
 * The method (Shin 2018, "Novel Selectivity Estimation Strategy for Modern
 * DBMS", Ch.3 sec.3.1 "Selectivity Computation") replaces a cardinality
 * estimate of a pushed-down selection sigma(R) by the exact answer of
 * SELECT COUNT(*) FROM R WHERE <R's predicates>, run on the in-memory GPU
 * executor while the query is still being optimised.  If the count is at
 * most a limit (Algorithm 1, function Execute: the count is compared with
 * maxSize and an exception aborts the push-down when it is larger), sigma(R)
 * is materialised at once while R's columns are resident (Ch.3 sec.3.3
 * "Materialization").  This header exposes exactly that path:
 *
 *   sel_count               exact COUNT(*) of rows whose predicate is TRUE
 *   sel_pushdown_rowids     count, limit check, then ascending row ids
 *   sel_pushdown_keybitmap  count + dimension-key bitmap (push-down on a
 *                           non-probe relation, Ch.3 sec.3.3 / Algorithm 1)
 *   sel_star_count          exact fact-table count of a star semi-join over
 *                           such key bitmaps
 *
 * Conventions
 *  - Every function returns sel_status; nothing throws across the ABI.
 *    Negative = error (nothing was computed or written unless stated),
 *    positive = a non-error outcome (SEL_OVER_LIMIT, SEL_E_CAPACITY), for
 *    which *out_count is still valid.
 *  - Column data, validity bitmaps and every output buffer named d_* are
 *    DEVICE pointers owned by the caller (BORROWED: the caller keeps them
 *    alive while a table / program / call uses them).  Pointers named h_* or
 *    out_* without the d_ prefix are host pointers.
 *  - Column data must be 16-byte aligned; validity bitmaps 4-byte aligned.
 *    Kernels may read (never write, never use) the bytes after a column's
 *    last element up to the next 4-byte boundary, which lie in that
 *    element's 16-byte-aligned block and so in the same memory page.
 *  - Synchronous calls return after results are on the host.  *_async
 *    calls only enqueue work on the context's stream.
 *  - A context is used by one host thread at a time.  Tables and programs
 *    made from a context are destroyed before it.
 *  - Rows are numbered 0..nrows-1; nrows < 2^32 (row ids are uint32).
 *
 * Truth values follow SQL three-valued (Kleene) logic: a comparison on a
 * NULL value is UNKNOWN, AND = min and OR = max over FALSE < UNKNOWN < TRUE,
 * NOT swaps TRUE and FALSE, and WHERE keeps only TRUE rows.
 */
#ifndef SEL_H
#define SEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sel_status {
  SEL_OK = 0,
  SEL_OVER_LIMIT = 1,  /* count > max_rows: nothing materialised (Algorithm 1:
                          Execute throws, EvaluateAndPushDown reverts) */
  SEL_E_CAPACITY = 2,  /* count > caller's output capacity: nothing written */
  SEL_E_INVALID = -1,  /* bad handle, argument or program; found before any
                          device work was enqueued */
  SEL_E_TYPE = -2,     /* operation not valid for the column's type */
  SEL_E_NOMEM = -3,    /* device or host allocation failed */
  SEL_E_DEVICE = -4,   /* HIP runtime error; sel_last_error() has its text */
  SEL_E_BUSY = -5,     /* admission refused (server memory budget) */
  SEL_E_RANGE = -6     /* a qualifying key fell outside the key-bitmap range */
} sel_status;

/* Column element types.  Values are signed and compared after sign extension
 * to int64.  TEXT columns are dictionary codes (int32 in [0, dict_card)),
 * DECIMAL(p,2) columns are int64 scaled by 100 and DATE columns are int32
 * day numbers: the thesis' TPC-H predicates on INTEGER, TEXT, DECIMAL(15,2)
 * and DATE attributes (Ch.5 sec.5.2) all become integer tests. */
typedef enum sel_type { SEL_I8 = 1, SEL_I16 = 2, SEL_I32 = 3, SEL_I64 = 4 } sel_type;

typedef struct sel_column {
  int32_t type;            /* sel_type */
  uint32_t dict_card;      /* > 0: dictionary-coded, codes in [0, dict_card) */
  const void* data;        /* device, nrows elements, 16-byte aligned, BORROWED */
  const uint32_t* valid;   /* device, ceil(nrows/32) words; bit (i%32) of word
                              i/32 is 1 iff row i is not NULL.  NULL pointer =
                              the column has no NULLs.  BORROWED. */
} sel_column;

/* Predicate program: postfix (reverse Polish) code.  Leaves push one truth
 * value, NOT / IS_UNKNOWN pop one and push one, AND / OR pop two and push
 * one; the program must leave exactly one value.  These are the selection
 * predicates of the count query of Ch.3 sec.3.1 (conjunctions of =, <, >,
 * BETWEEN and OR-groups) plus IN-lists, pre-resolved LIKE (a set of
 * dictionary codes) and NULL tests. */
typedef enum sel_op {
  SEL_OP_EQ = 1,          /* col = a                                         */
  SEL_OP_NE = 2,          /* col <> a                                        */
  SEL_OP_LT = 3,          /* col < a                                         */
  SEL_OP_LE = 4,          /* col <= a                                        */
  SEL_OP_GT = 5,          /* col > a                                         */
  SEL_OP_GE = 6,          /* col >= a                                        */
  SEL_OP_BETWEEN = 7,     /* a <= col <= b (a > b: FALSE for non-NULL rows)  */
  SEL_OP_IN = 8,          /* col IN (list): aux = pool byte offset (8-aligned)
                             of b int64 values, b >= 1, any order, duplicates
                             allowed                                         */
  SEL_OP_CODESET = 9,     /* 0 <= col < b and bit col of the set: aux = pool
                             byte offset (4-aligned) of ceil(b/32) uint32
                             words, bit c = word c/32 bit c%32; b <= 2^24.
                             A LIKE pattern on a dictionary column resolved
                             to the codes it matches.                        */
  SEL_OP_IS_NULL = 10,    /* never UNKNOWN                                   */
  SEL_OP_IS_NOT_NULL = 11,/* never UNKNOWN                                   */
  SEL_OP_AND = 16,
  SEL_OP_OR = 17,
  SEL_OP_NOT = 18,
  SEL_OP_IS_UNKNOWN = 19, /* (p) IS UNKNOWN: TRUE iff p is UNKNOWN           */
  SEL_OP_TRUE = 20,
  SEL_OP_FALSE = 21
} sel_op;

typedef struct sel_instr {   /* 24 bytes */
  uint16_t op;               /* sel_op */
  uint16_t col;              /* column index for leaves, else 0 */
  uint32_t aux;              /* pool byte offset for IN / CODESET */
  int64_t a;
  int64_t b;
} sel_instr;

#define SEL_MAX_INSTRS 64         /* postfix length                       */
#define SEL_MAX_DEPTH 8           /* evaluation stack after operand reordering */
#define SEL_MAX_POOL_BYTES 65536  /* constant pool                         */
#define SEL_MAX_COLUMNS 64

typedef struct sel_ctx sel_ctx;
typedef struct sel_table sel_table;
typedef struct sel_program sel_program;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (for instance torch.cuda.current_stream().cuda_stream) on which every call
 * enqueues its work, so the calls are ordered after earlier work on that
 * stream that produced their inputs.  NULL is the device's null stream (the
 * handle torch reports for its default stream); SEL_STREAM_OWN makes the
 * context create a non-blocking stream of its own, and the caller then
 * synchronises its inputs before each call.
 * Errors: SEL_E_INVALID (bad device / out NULL), SEL_E_DEVICE, SEL_E_NOMEM. */
#define SEL_STREAM_OWN ((void*)(intptr_t)-1)
sel_status sel_ctx_create(int device, void* hip_stream, sel_ctx** out);
void sel_ctx_destroy(sel_ctx* ctx);

/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the same context.  ctx may be NULL (errors of sel_ctx_create). */
const char* sel_last_error(const sel_ctx* ctx);

/* Number of compute units of the context's device (for launch sizing). */
uint32_t sel_ctx_num_cus(const sel_ctx* ctx);

/* ---- tables ----------------------------------------------------------- */

/* Describe a resident columnar table of `nrows` rows and `ncols` columns.
 * The descriptor array is copied; the device buffers it names are borrowed.
 * Errors: SEL_E_INVALID (nrows >= 2^32, ncols 0 or > SEL_MAX_COLUMNS,
 * unknown type, NULL data with nrows > 0, misaligned data). */
sel_status sel_table_create(sel_ctx* ctx, uint64_t nrows, uint32_t ncols,
                            const sel_column* cols, sel_table** out);
void sel_table_destroy(sel_table* t);  /* never frees borrowed buffers */
uint64_t sel_table_nrows(const sel_table* t);

/* ---- predicate programs ------------------------------------------------ */

/* Validate postfix `code[0..n)` against `table` and compile it to the device
 * form: comparisons become closed integer ranges clamped to the column type,
 * IN-lists are sorted and deduplicated and dense ones become bitmaps,
 * operands of AND/OR may be reordered to bound the stack depth (Kleene AND
 * and OR are commutative, so the truth value of every row is unchanged).
 * `pool` (host, `pool_bytes` bytes) holds IN values and code bitmaps; it is
 * copied.  The program owns a device copy and is bound to `table`.
 * Errors: SEL_E_INVALID (unknown op, column index out of range, stack
 * underflow / overflow, final depth != 1, pool offset out of bounds or
 * misaligned, n == 0 or n > SEL_MAX_INSTRS, IN with b < 1),
 * SEL_E_TYPE (CODESET on a column that is not dictionary-coded),
 * SEL_E_NOMEM / SEL_E_DEVICE. */
sel_status sel_program_compile(sel_ctx* ctx, const sel_table* table,
                               const sel_instr* code, uint32_t n,
                               const void* pool, uint32_t pool_bytes,
                               sel_program** out);
void sel_program_destroy(sel_program* p);

/* Validate and lower a program for a table described by `cols` without any
 * device work (usable on a machine without a GPU; column data pointers may
 * be NULL -- only type, dict_card and whether `valid` is NULL matter).  On
 * success `text` receives a listing of the lowered program, one device
 * instruction per line; on failure `err` receives the reason.  Either buffer
 * may be NULL.  Returns the status sel_program_compile would return. */
sel_status sel_program_check(uint64_t nrows, uint32_t ncols, const sel_column* cols,
                             const sel_instr* code, uint32_t n, const void* pool,
                             uint32_t pool_bytes, char* text, size_t text_len, char* err,
                             size_t err_len);

/* Listing of a compiled program (as sel_program_check prints it); owned by
 * the program. */
const char* sel_program_listing(const sel_program* p);

/* Bytes per row the scan of this program reads from device memory: the
 * element size of every column whose values it tests plus 1/8 for every
 * column whose validity bitmap it reads (the algorithmic traffic). */
double sel_program_bytes_per_row(const sel_program* p);

/* ---- the count query (Ch.3 sec.3.1) ------------------------------------ */

/* Exact number of rows of `table` for which `prog` is TRUE.
 * Errors: SEL_E_INVALID (NULL handle, program bound to another table),
 * SEL_E_DEVICE. */
sel_status sel_count(sel_ctx* ctx, const sel_table* table,
                     const sel_program* prog, uint64_t* out_count);

/* Same count, enqueued only: the result is written to *d_count (device,
 * 8 bytes) when the context's stream reaches it. */
sel_status sel_count_async(sel_ctx* ctx, const sel_table* table,
                           const sel_program* prog, uint64_t* d_count);

/* ---- push-down with materialisation (Algorithm 1, Ch.3 sec.3.3) --------- */

/* floor(nrows * ratio), the product taken in double precision, for ratio in
 * [0, 1]: Algorithm 1's maxSize = R.size * PUSH_DOWN_MAX_SELECTIVITY.  For an
 * integer count c, c > nrows*ratio iff c > floor(nrows*ratio).  ratio
 * outside [0,1] (or NaN) is clamped: <= 0 gives 0, >= 1 gives nrows. */
uint64_t sel_max_rows(uint64_t nrows, double ratio);

/* Count the qualifying rows; if count > max_rows return SEL_OVER_LIMIT and
 * write nothing (the thesis throws and reverts the push-down).  If count >
 * cap return SEL_E_CAPACITY and write nothing.  Otherwise write the count
 * qualifying row ids in ascending order to d_out[0..count) (device, caller
 * owned) and return SEL_OK.  *out_count is set for every status >= 0.
 * max_rows = UINT64_MAX disables the limit. */
sel_status sel_pushdown_rowids(sel_ctx* ctx, const sel_table* table,
                               const sel_program* prog, uint64_t max_rows,
                               uint32_t* d_out, uint64_t cap,
                               uint64_t* out_count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc after start-up):
 * the same push-down, with the same arguments, statuses and results as
 * sel_pushdown_rowids, whose kernels it shares, but its workspace (packed
 * mask words, tile counts and offsets, chunk sums and offsets, tile lane
 * maps: about N/8 + 16*N/2048 bytes plus 16 KB) is a fixed 64 MiB array
 * that the library holds on each device it runs on until the process ends.
 * The call allocates nothing and creates no timing events (its kernels are
 * not counted by sel_ctx_read_timing).  A table whose workspace would
 * exceed 64 MiB (more than about 505 M rows) gives SEL_E_INVALID with the
 * sizes in sel_last_error, before any launch.  Every call on one device
 * shares that device's array: calls that overlap on one device (several
 * contexts or host threads) race and must be serialised by the caller.
 * Nothing in the array needs clearing: each call writes every word it reads
 * before reading it. */
sel_status sel_pushdown_rowids_noalloc(sel_ctx* ctx, const sel_table* table,
                                       const sel_program* prog, uint64_t max_rows,
                                       uint32_t* d_out, uint64_t cap,
                                       uint64_t* out_count);

/* Push the selection down on a dimension relation: zero d_bitmap[0 ..
 * ceil(nbits/32)) and set bit (key - key_min) for every row whose predicate
 * is TRUE, where key is column `key_col` (an int32 or int64 column without
 * NULLs).  *out_count = number of qualifying rows.  A qualifying key outside
 * [key_min, key_min + nbits) gives SEL_E_RANGE (bitmap contents then
 * unspecified).  prog may be NULL (every row qualifies).  Keys are expected
 * unique (a primary key); duplicates set the same bit. */
sel_status sel_pushdown_keybitmap(sel_ctx* ctx, const sel_table* dim,
                                  uint32_t key_col, int64_t key_min,
                                  const sel_program* prog, uint32_t* d_bitmap,
                                  uint64_t nbits, uint64_t* out_count);

/* Exact star semi-join count: the number of fact rows i such that for every
 * d < nfk, 0 <= fk_d[i] < nbits[d] and bit fk_d[i] of d_bitmaps[d] is set,
 * and (fact_pred == NULL or fact_pred is TRUE on row i).  fk columns are
 * int32 or int64 columns of `fact`; a NULL foreign key never matches.  With
 * unique dimension keys this equals the cardinality of the FK-PK star join
 * of the fact table with the pushed-down dimensions.  nfk in 1..8.
 * d_bitmaps is a host array of nfk device pointers; nbits a host array. */
sel_status sel_star_count(sel_ctx* ctx, const sel_table* fact,
                          const sel_program* fact_pred, uint32_t nfk,
                          const uint32_t* fk_cols,
                          const uint32_t* const* d_bitmaps,
                          const uint64_t* nbits, uint64_t* out_count);

/* Projected columns of a materialised sigma(R) (Ch.3 sec.3.3: the pushed-down
 * selection is stored with the columns the query needs, while R is resident;
 * Algorithm 1's CoalesceNodes fuses the selection with that projection).
 * For k in [0, count): d_out[c][k] = column cols[c] of `table` at row
 * d_ids[k] (values of the column's width, sign as stored), and, when
 * d_valid_out is not NULL and d_valid_out[c] is not NULL, bit k % 32 of
 * word k / 32 of d_valid_out[c] = that row's validity (1 = not NULL; every
 * word up to ceil(count/32) is written whole, bits past count are 0).  The
 * ids are typically sel_pushdown_rowids' output (ascending, any order
 * works).  ncols in 1..16; cols, d_out and d_valid_out are host arrays of
 * ncols entries; d_ids and the outputs are device memory, caller owned.
 * Errors: SEL_E_INVALID for bad arguments (before any launch) or, after
 * the launch, for ids >= the table's rows (their outputs are 0 and NULL). */
sel_status sel_gather(sel_ctx* ctx, const sel_table* table, const uint32_t* d_ids, uint64_t count,
                      uint32_t ncols, const uint32_t* cols, void* const* d_out,
                      uint32_t* const* d_valid_out);

/* ---- the push-down decision over a query's relations (Algorithm 1) ------ */

/* One scanned relation R of a query: its table, the selection extracted for
 * it (NULL: the query has no predicate on R), and a caller-owned device
 * buffer for the ascending row ids of sigma(R) should it be pushed down. */
typedef struct sel_spd_relation {
  const sel_table* table;
  const sel_program* pred;     /* bound to table, or NULL */
  uint32_t* d_out;             /* device, caller owned; may be NULL if cap == 0 */
  uint64_t cap;                /* capacity of d_out in row ids */
} sel_spd_relation;

typedef enum sel_spd_decision {
  SEL_SPD_PUSHED = 0,     /* count <= maxSize: sigma(R) materialised in d_out */
  SEL_SPD_REVERTED = 1,   /* count > maxSize (or > cap): push-down reverted   */
  SEL_SPD_PROBE = 2,      /* the largest relation: kept for the probe side    */
  SEL_SPD_SMALL = 3,      /* size <= min_table_size: never evaluated          */
  SEL_SPD_NO_PRED = 4     /* queued, but no selection to push down            */
} sel_spd_decision;

typedef struct sel_spd_result {
  int32_t decision;       /* sel_spd_decision                                  */
  int32_t status;         /* sel_pushdown_rowids' status for an evaluated R    */
                          /* (SEL_OK, SEL_OVER_LIMIT or SEL_E_CAPACITY), else 0 */
  uint32_t order;         /* position in the evaluation order, or UINT32_MAX   */
  uint32_t pad;
  uint64_t count;         /* exact |sigma(R)| of an evaluated R, else 0        */
  uint64_t max_rows;      /* maxSize = sel_max_rows(R.size, max_selectivity)   */
} sel_spd_result;

/* EvaluateAndPushDown of Algorithm 1 (Ch.4 sec.4.2) over n relations:
 * relations larger than min_table_size (PUSH_DOWN_MIN_TABLE_SIZE, strict >)
 * enter a queue ordered by size, largest first (equal sizes: lower index
 * first); the first, the relation to be probed, is removed; each other
 * queued relation with a selection is then, in queue order, counted exactly
 * and either pushed down (ids written to d_out) or reverted, by
 * sel_pushdown_rowids with max_rows = maxSize = floor(R.size *
 * max_selectivity) (PUSH_DOWN_MAX_SELECTIVITY).  A count above cap reverts
 * too (status SEL_E_CAPACITY, nothing written).  out (host, n) gets one
 * result per relation, in input order.  Errors: SEL_E_INVALID (n == 0,
 * NULL arrays or tables, a program bound to another table, NaN ratio; checked
 * before any launch), or the first error of a push-down (device or memory),
 * which ends the loop with the results so far filled in. */
sel_status sel_select_pushdown(sel_ctx* ctx, uint32_t n, const sel_spd_relation* rels,
                               uint64_t min_table_size, double max_selectivity,
                               sel_spd_result* out);

/* ---- batching (Algorithm 1 counts every candidate relation) ------------- */

/* Exact counts of n (table, program) pairs in ONE batched launch sequence
 * (n in 1..1024; progs[i] must be bound to tables[i]; tables may repeat and
 * may differ in size).  Tiles of every table form one index space; a wave
 * takes a tile and evaluates every program of one pass over that tile's
 * table on it.  A table's programs are packed into as few passes as the
 * per-wave evaluation state allows, and each pass reads the columns its
 * programs use from HBM once: a table is read once per pass, not once per
 * program.  Programs in conjunctive form (every one without IS UNKNOWN
 * whose clauses and columns fit) are counted by one lookup per column and
 * row into per-column tables of program bits (up to 32 programs a pass);
 * the rest by leaf-major evaluation.  out_counts (host, n)
 * receives count i for pair i; each equals what sel_count returns for it.
 * Algorithm 1 computes one count per candidate relation in its loop over
 * the relation queue; a batch computes all of them at once.
 * Errors: SEL_E_INVALID (n out of range, NULL entries, program bound to
 * another table), SEL_E_NOMEM, SEL_E_DEVICE. */
sel_status sel_count_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                           const sel_program* const* progs, uint64_t* out_counts);

/* A batch captured once in a HIP graph (the persistent kernel + the copy of
 * the counts to pinned host memory) and replayed by sel_batch_run.  The
 * batch owns its device descriptors, accumulators and stream; it reads the
 * tables and programs, which must outlive it.  Same argument rules and
 * errors as sel_count_batch. */
typedef struct sel_batch sel_batch;
sel_status sel_batch_create(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                            const sel_program* const* progs, sel_batch** out);

/* Replace program i by another program bound to the same table.  Only the
 * device descriptor is rewritten (in stream order); the graph is not
 * captured again.  Errors: SEL_E_INVALID. */
sel_status sel_batch_set_program(sel_batch* b, uint32_t i, const sel_program* prog);

/* Replay the graph after all work already enqueued on the context's stream,
 * wait for it, and write the n counts to out_counts (host). */
sel_status sel_batch_run(sel_batch* b, uint64_t* out_counts);
void sel_batch_destroy(sel_batch* b);

/* The same star semi-join as a program over the fact table (bitmap-probe
 * leaves ANDed with the optional fact predicate), usable wherever a program
 * is: sel_count of it equals sel_star_count, and it can join batches and
 * served requests.  The bitmaps are BORROWED: they must stay valid and
 * unchanged while the program is used.  Same argument rules and errors as
 * sel_star_count. */
sel_status sel_program_star(sel_ctx* ctx, const sel_table* fact, const sel_program* fact_pred,
                            uint32_t nfk, const uint32_t* fk_cols,
                            const uint32_t* const* d_bitmaps, const uint64_t* nbits,
                            sel_program** out);

/* ---- conjunct counts: the estimate that exact counting replaces --------- */

/* Exact counts of the top-level AND factors (conjuncts) of a selection and
 * of the whole selection, in one batched launch: the figures behind the
 * worked example of Ch.1 sec.1.1, where the product of per-predicate
 * selectivities (the attribute-value independence assumption of
 * statistics-based estimators) gives 0.0015 while the selection's true
 * selectivity is 0.167.  *nfactors = number of factors (1 if the root is
 * not an AND), in the order the compiled program evaluates them (the
 * compiler may reorder operands); factor_counts (host, cap entries) receives
 * their counts and *count the selection's count.  Errors: SEL_E_INVALID;
 * SEL_E_CAPACITY (positive) when *nfactors > cap, with nothing counted. */
sel_status sel_factor_counts(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                             uint32_t cap, uint64_t* factor_counts, uint32_t* nfactors,
                             uint64_t* count);

/* The independence estimate of a conjunction's count: nrows * prod over
 * the n factors of (counts[k] / nrows), in double; 0 when nrows is 0. */
double sel_independence_estimate(uint64_t nrows, uint32_t n, const uint64_t* counts);

/* ---- join sizes from exact selection counts (Ch.1 sec.1.1) -------------- */

/* The size of R join S on attribute A by the simplified formula of Ch.1
 * sec.1.1: |R| |S| / max(V(R,A), V(S,A)), with V the number of distinct
 * values of A; 0 when both distinct counts are 0. */
double sel_join_size(double r_rows, double s_rows, double v_r, double v_s);

/* A left-deep plan over a star: the fact table's selection (fact_rows rows)
 * joined with its dimensions in `order` (a permutation of 0..ndims-1).
 * Dimension d has dim_rows[d] distinct keys, all referenced by the fact
 * table's foreign key (so V of the key is dim_rows[d] on both sides), and
 * sel_rows[d] rows (and keys) after its own selection -- the exact counts
 * this library computes.  Each join is sized by sel_join_size; inter (host,
 * ndims, may be NULL) receives the size after each join, and the return
 * value is their sum (the plan's intermediate rows), or -1 for bad input
 * (ndims 0 or > 64, NULL arrays, an order that is not a permutation). */
double sel_star_plan_cost(double fact_rows, uint32_t ndims, const double* dim_rows,
                          const double* sel_rows, const uint32_t* order, double* inter);

/* The left-deep order of least sel_star_plan_cost: the dimensions by
 * ascending retained fraction sel_rows[d] / dim_rows[d] (equal fractions in
 * index order), written to order (host, ndims); *cost receives its cost.
 * SEL_E_INVALID for bad input. */
sel_status sel_star_plan_order(double fact_rows, uint32_t ndims, const double* dim_rows,
                               const double* sel_rows, uint32_t* order, double* cost);

/* ---- serving: continuous batching of estimate requests ------------------ */

/* A server keeps the tables resident (they are the caller's) and answers
 * requests as they arrive.  A request is a set of count queries (one exact
 * count per (table, program), Ch.3 sec.3.1) and optionally one push-down
 * with materialisation (Algorithm 1's Execute: count, limit check, ascending
 * row ids).  Count queries are served by cooperative scans: each table with
 * pending programs is cut into rounds_per_cycle chunks (fewer if a chunk
 * would exceed chunk_rows rows), and a round is one batched launch over the
 * current chunk of every such table for every program attached to it, so
 * every table completes a cycle in the same number of rounds.  A program
 * attaches at the next round and is done after one revolution over its
 * table, so requests arriving while others are on the GPU share their
 * scans.  A request is admitted (FIFO) when its
 * device footprint (accumulators, program code, and for a push-down the
 * result mask, tile counts and its id capacity) fits the budget beside the
 * admitted ones; push-downs run on their own stream, overlapping the rounds.
 * Identical programs (the same sel_program) attached by different requests
 * are evaluated once per chunk and their chunk count is handed to each.
 * Counts are exact: a request's results do not depend on what else runs. */
typedef struct sel_server sel_server;

typedef struct sel_server_config {
  uint64_t hbm_budget_bytes;   /* device bytes admitted requests may hold (0 = 1 GiB) */
  uint64_t chunk_rows;         /* most rows per cooperative-scan chunk (0 = no cap) */
  uint32_t max_programs;       /* programs in flight (<= 4096; 0 = 4096) */
  uint32_t rounds_in_flight;   /* rounds queued on the device (1..4; 0 = 1) */
  uint32_t rounds_per_cycle;   /* chunks per table (0 = 3) */
  uint32_t pad;
} sel_server_config;

typedef struct sel_request {
  uint32_t nprog;                      /* count queries (may be 0 with a push-down) */
  const sel_table* const* tables;      /* nprog entries */
  const sel_program* const* progs;     /* progs[i] bound to tables[i] */
  const sel_table* pd_table;           /* push-down, or NULL for none */
  const sel_program* pd_prog;
  uint64_t pd_max_rows;                /* Algorithm 1's maxSize */
  uint32_t* pd_out;                    /* device, caller-owned, pd_cap ids */
  uint64_t pd_cap;
} sel_request;

typedef struct sel_result {
  sel_status status;                   /* the push-down's status (SEL_OK without one) */
  int32_t pad;
  uint64_t pd_count;                   /* the push-down's count */
  double latency_ms;                   /* submit -> completion */
} sel_result;

typedef struct sel_server_stats {
  uint64_t submitted, completed, rejected;
  uint64_t rounds;                     /* batched launches */
  uint64_t round_programs;             /* programs summed over rounds */
  uint64_t shared_rounds;              /* table scans serving programs of >= 2 requests */
  uint32_t max_admitted;               /* most requests admitted at once */
  uint32_t pad;
  double p50_ms, p99_ms, mean_ms, max_ms;  /* request latency, submit -> completion */
  double elapsed_s;                    /* first submit -> last completion */
  uint64_t round_groups;               /* distinct programs summed over rounds */
  double round_gpu_ms;                 /* device time of the rounds, summed */
  double round_host_ms;                /* host time planning and launching them */
  double round_bytes;                  /* bytes the rounds read, summed: per table
                                          and round, the chunk's rows times the
                                          element sizes of the columns its
                                          programs test (+1/8 per validity bitmap) */
} sel_server_stats;

/* Start a server (two worker threads, its own streams and a push-down
 * context) on ctx's device.  cfg may be NULL for defaults. */
sel_status sel_server_create(sel_ctx* ctx, const sel_server_config* cfg, sel_server** out);

/* Queue a request; *ticket names it.  The arrays are copied; tables,
 * programs and pd_out must stay valid until the request completes.  The
 * request's device work runs on the server's streams after whatever was
 * enqueued on the context's stream before this call (an event recorded at
 * submission), so inputs produced there need no host synchronisation.
 * Errors: SEL_E_INVALID (bad entries, or a program with more than 64 leaf
 * and validity words to batch), SEL_E_BUSY (the request alone needs
 * more than the budget: it is rejected, never queued), SEL_E_DEVICE (a
 * worker failed). */
sel_status sel_server_submit(sel_server* s, const sel_request* req, uint64_t* ticket);

/* *done = 1 once the request completed. */
sel_status sel_server_poll(sel_server* s, uint64_t ticket, int* done);

/* Block until the request completes; counts (host, nprog) and *res (either
 * may be NULL) receive its results; the ticket is then released. */
sel_status sel_server_wait(sel_server* s, uint64_t ticket, uint64_t* counts, sel_result* res);

/* Counters and latency percentiles of completed requests (reset != 0
 * clears them). */
sel_status sel_server_get_stats(sel_server* s, sel_server_stats* out, int reset);

/* Finish in-flight work and stop.  Requests still queued are dropped. */
void sel_server_destroy(sel_server* s);

/* ---- launch configuration and timing ------------------------------------ */

typedef struct sel_launch {
  uint32_t block;          /* threads per workgroup: 64, 128 or 256 (scans)   */
  uint32_t grid;           /* workgroups; 0 = library default                  */
  uint32_t cached;         /* scans: 1 = column loads through the caches,
                              0 = nontemporal loads (the default)             */
  uint32_t tiles_per_step; /* scans: consecutive 2048-row tiles a wave takes
                              per step, 1, 2 or 4 (0 = 1)                     */
  uint32_t stage_words;    /* scans: most LDS words of the program's bitmaps
                              and IN lists copied to LDS first (0 = all that
                              fit 32 KB; 1 = none)                            */
  uint32_t rows_per_lane;  /* lookup-table batch kernel: rows per lane per
                              segment, 4 or 8 (0 = 8; four-dword passes
                              always take 4)                                  */
} sel_launch;

/* Override (or with NULL, restore) the launch configuration used by the
 * scan kernels of this context.  Errors: SEL_E_INVALID for an unsupported
 * block size, tiles_per_step or rows_per_lane. */
sel_status sel_ctx_set_launch(sel_ctx* ctx, const sel_launch* launch);

/* ---- autotuning (offline: launches real kernels; not for the latency path) */

/* Time the count scan (with_mask = 0) or the count + mask scan
 * (with_mask != 0) of `prog` on `table`, `reps` times each (0 = 5): first
 * every launch shape (workgroups of 64/128/256 threads, 4..32 resident
 * waves per CU), then, with the fastest shape, cached against nontemporal
 * loads, then 1, 2 or 4 tiles per step, then the LDS staging limit (all,
 * 2048 words, none) -- one knob at a time, each kept at its fastest
 * (median).  The result is recorded for this program class (bytes per row,
 * length) and table size on the context; later calls with no fixed
 * configuration use it.  *best / *best_ms (either may be NULL) receive it. */
sel_status sel_autotune(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                        int with_mask, uint32_t reps, sel_launch* best, double* best_ms);

/* Same for the batched count of these n pairs (see sel_count_batch): the
 * leaf-major kernel's workgroups of 64 to 768 threads whose LDS fits the
 * batch's plan, then the lookup-table kernel's rows per lane (4 or 8). */
sel_status sel_autotune_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                              const sel_program* const* progs, uint32_t reps,
                              sel_launch* best, double* best_ms);

/* Save / load the context's tuned configurations as text ("key block grid
 * cached tiles_per_step stage_words rows_per_lane" lines, or the older
 * "key block grid" ones;
 * grids are rescaled if the file was written on a device with another
 * number of CUs).  sel_ctx_create loads the file named by the environment
 * variable SEL_TUNE_CACHE, if set. */
sel_status sel_tune_save(const sel_ctx* ctx, const char* path);
sel_status sel_tune_load(sel_ctx* ctx, const char* path);
uint32_t sel_tune_entries(const sel_ctx* ctx);

/* Kernel timing: when enabled, the library brackets each scan-kernel launch
 * with HIP events on the context's stream and accumulates the elapsed time
 * per kernel kind.  Reading the totals synchronises the stream. */
typedef enum sel_kernel_kind {
  SEL_K_COUNT = 0,       /* fused evaluate + count                      */
  SEL_K_MASK = 1,        /* evaluate + count + packed result mask,
                            tile lane maps and tile counts              */
  SEL_K_SCAN = 2,        /* exclusive scan of tile counts               */
  SEL_K_COMPACT = 3,     /* mask -> ascending row ids                   */
  SEL_K_KEYBITMAP = 4,   /* dimension key bitmap build                  */
  SEL_K_STAR = 5,        /* star semi-join probe count                  */
  SEL_K_BATCH = 6,       /* persistent batched count                    */
  SEL_K_GATHER = 7,      /* projected columns by row id                 */
  SEL_K_NKINDS = 8
} sel_kernel_kind;

typedef struct sel_timing {
  double ms[SEL_K_NKINDS];         /* summed kernel time                  */
  uint64_t launches[SEL_K_NKINDS]; /* number of timed launches            */
} sel_timing;

sel_status sel_ctx_enable_timing(sel_ctx* ctx, int enable);
sel_status sel_ctx_read_timing(sel_ctx* ctx, sel_timing* out, int reset);

#ifdef __cplusplus
}
#endif
#endif /* SEL_H */
