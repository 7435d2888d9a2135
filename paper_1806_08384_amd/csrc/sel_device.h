// sel_device.h -- device form of a compiled predicate program and the
// launch interface between the host runtime (api.cpp, compile.cpp) and the
// HIP kernels (kernels.hip).
#pragma once

#include <stdint.h>

namespace sel {

// Row <-> lane mapping of one wave tile (2048 rows).  Lane L owns rows
//   tile_base + 256*j + 4*L + i      (j = 0..7 "steps", i = 0..3)
// and keeps its 32 truth bits in one 32-bit word, bit b = 4*j + i.  Four
// consecutive rows per lane per step keep every column's loads wide and
// coalesced for all element widths (int8: 4 B, int16: 8 B, int32: 16 B,
// int64: 2 x 16 B per lane per step) while every column maps rows to the
// same (lane, bit), so truth words of different columns combine bitwise.
constexpr int kWave = 64;
constexpr int kRowsPerStep = 4;
constexpr int kSteps = 8;
constexpr int kTileRows = kWave * kRowsPerStep * kSteps;  // 2048
constexpr int kMaxDepth = 8;

// Bytes of the fixed device workspace of the push-down that allocates
// nothing (mask words, tile counts and offsets, chunk sums and offsets,
// tile lane maps): 64 MiB, enough for tables of about 505 M rows.
constexpr unsigned long long kNoAllocScratchBytes = 64ull << 20;

enum DevType : uint32_t { T_I8 = 1, T_I16 = 2, T_I32 = 3, T_I64 = 4 };

// Device opcodes (the lowered program).
enum DevOp : uint32_t {
  D_RANGE = 1,     // lo <= x <= lo + span (unsigned span), x in column type
  D_BITMAP = 2,    // 0 <= x - lo < nbits and bit (x - lo) of aux
  D_INLIST = 3,    // x in aux[0..n) (sorted, distinct int64)
  D_NN_TRUE = 4,   // TRUE on non-NULL rows, UNKNOWN on NULL rows
  D_NN_FALSE = 5,  // FALSE on non-NULL rows, UNKNOWN on NULL rows
  D_ISNULL = 6,
  D_NOTNULL = 7,
  D_AND = 16,
  D_OR = 17,
  D_NOT = 18,
  D_ISUNK = 19,
  D_TRUE = 20,
  D_FALSE = 21
};

enum DevFlags : uint32_t {
  F_GUARD_AND = 1,  // leaf is the right operand of the next AND: rows whose
                    // left operand is FALSE need not be evaluated
  F_GUARD_OR = 2,   // ... of the next OR: rows whose left operand is TRUE
  F_HASHED = 4      // D_INLIST: two cuckoo tables follow the sorted list;
                    // bits 8..12 hold their log2 size, bits 16..18 the
                    // multiplier pair
};

// IN lists of up to kInHashMax values also get two cuckoo tables of
// 2^b >= 2n slots each: value x lives in slot in_hash(x, c1, b) of the
// first or in_hash(x, c2, b) of the second, and empty slots hold a list
// value.  The hash folds the two 32-bit halves, multiplies by an odd
// constant and keeps the top b bits.
constexpr uint32_t kInHashMax = 1024;
constexpr uint32_t kInHashPairs = 8;
constexpr uint32_t kInHashMul[kInHashPairs][2] = {
    {0x9E3779B1u, 0x85EBCA77u}, {0xC2B2AE3Du, 0x27D4EB2Fu}, {0x165667B1u, 0xD3A2646Du},
    {0xFD7046C5u, 0xB55A4F09u}, {0x2545F491u, 0x9E6C63D1u}, {0x5851F42Du, 0x4C957F2Du},
    {0x7FEB352Du, 0x846CA68Bu}, {0xE6546B65u, 0x1B873593u}};
constexpr uint32_t in_hash(int64_t x, uint32_t c, uint32_t b) {
  const uint64_t u = (uint64_t)x;
  return (((uint32_t)u ^ (uint32_t)(u >> 32)) * c) >> (32 - b);
}
constexpr uint32_t in_hash_bits(uint32_t flags) { return (flags >> 8) & 31u; }
constexpr uint32_t in_hash_pair(uint32_t flags) { return (flags >> 16) & 7u; }

struct DevInstr {          // 64 bytes, read with scalar loads
  uint32_t op;
  uint32_t type;           // DevType of the column (leaves)
  uint32_t flags;          // DevFlags
  uint32_t n;              // D_INLIST: list length
  const void* data;        // column values
  const uint32_t* valid;   // validity words or nullptr
  int64_t lo;              // D_RANGE lower bound / D_BITMAP base
  uint64_t span;           // D_RANGE: hi - lo (unsigned) / D_BITMAP: nbits
  const void* aux;         // D_BITMAP words / D_INLIST values
  uint32_t slot;           // batched evaluation: LDS slot of the leaf's word
  uint32_t lds_word;       // batched D_BITMAP: offset of its staged copy in
                           // LDS (n = index of a zero bit past it), or kNoLds
};
static_assert(sizeof(DevInstr) == 64, "DevInstr layout");

// Per-launch completion slot: an accumulator and a ticket that the last
// workgroup resets, so that no memset is needed between launches.
struct DevSlot {
  unsigned long long acc;    // running count
  unsigned long long acc2;   // second counter (out-of-range keys)
  unsigned int ticket;
  unsigned int pad[3];
};

enum ScanMode : int { M_COUNT = 0, M_MASK = 1, M_KEYBITMAP = 2 };

struct BatchBitmap;

struct ScanArgs {
  const DevInstr* prog;
  uint32_t nins;
  uint32_t nstage;             // bitmaps the workgroups copy to LDS first
  uint32_t cached;             // 1: column loads through the caches (0: nontemporal)
  uint32_t tiles_per_step;     // consecutive tiles a wave takes per step (0: 1)
  uint64_t nrows;
  uint64_t ntiles;
  DevSlot* slot;
  unsigned long long* out;     // out[0] = count, out[1] = out-of-range keys
  // M_MASK: per tile, the result words that hold a TRUE row, packed at the
  // front of the tile's 64-word slot in lane order (the rest of the slot is
  // not written); the lanes they belong to; and the tile's TRUE rows
  uint32_t* mask;
  uint64_t* tile_lanes;
  uint32_t* tile_counts;
  // M_KEYBITMAP
  const void* key_data;
  uint32_t key_type;
  uint32_t stage_words;        // LDS words of the staged bitmaps
  int64_t key_min;
  uint64_t nbits;
  uint32_t* bitmap;
  const BatchBitmap* stage;    // nstage entries (src, words, mask, offset)
};

// Single-program scans stage the program's IN lists (or their cuckoo
// tables) and small bitmaps (in program order, up to this many words: 48 KB
// per workgroup, three of which fit a CU, so that two 2048-slot cuckoo
// tables or a 200 k-key dimension's bitmap beside two smaller ones fit) in
// LDS; lookups into them skip the memory system.
constexpr uint32_t kScanStageWords = 12288;

struct CompactArgs {
  const uint32_t* mask;        // packed nonzero result words (see ScanArgs)
  const uint64_t* tile_lanes;  // the lanes they belong to
  const uint32_t* offsets;     // exclusive prefix of tile counts within a chunk
  const uint32_t* chunk_offs;  // exclusive prefix of chunk (1024 tiles) totals
  uint64_t ntiles;
  uint32_t* out;
  uint64_t cap;
  // the count the mask pass published; the compaction writes nothing when
  // it is 0 or above `limit` (Algorithm 1's maxSize, or the capacity)
  const unsigned long long* total;
  uint64_t limit;
};

// Projected columns of a materialised sigma(R): value k of each output
// column is the source column's value at row ids[k] (and bit k of its
// validity words that row's validity); at most kMaxGatherCols columns per
// launch, all passed by value.
constexpr uint32_t kMaxGatherCols = 16;
struct GatherCol {             // 40 bytes
  const void* src;
  const uint32_t* valid;       // nullptr: the column has no NULLs
  void* out;
  uint32_t* out_valid;         // nullptr: no validity wanted
  uint32_t width;              // bytes per value: 1, 2, 4 or 8
  uint32_t pad;
};
struct GatherArgs {
  const uint32_t* ids;
  uint64_t count;
  uint64_t nrows;
  DevSlot* slot;
  unsigned long long* out;     // out[1]: ids >= nrows
  uint32_t ncols, pad;
  GatherCol cols[kMaxGatherCols];
};

// Batched count (many programs over several tables in one launch),
// evaluated leaf-major.  Tiles of all entries form one flat index space.  For
// its tile a wave loads each column the entry's programs read once, runs
// every leaf test on that column while the values sit in registers, and
// parks each leaf's truth word (and each nullable column's validity word) in
// an LDS slot of its own; then each program's combinators run over the
// slots.  A column is thus read from HBM once per entry, however many
// programs and leaves use it.
constexpr uint32_t kBatchSlots = 40;      // LDS slots per wave (256 B each) that
                                          // passes are packed to
constexpr uint32_t kBatchMaxSlots = 64;   // one program alone: at most 32 leaves
                                          // and 32 validity words (its pass then
                                          // runs in 512-thread workgroups)
constexpr uint32_t kNoSlot = 0xFFFu;
// Batched leaves reuse DevInstr::flags for their guard: kNoGuard (test every
// row) or kAccGuard (below).
constexpr uint32_t kNoGuard = 0xFFFFFFFFu;
// When a pass starts on a workgroup it builds, in LDS, a lookup table for
// each narrow column with several leaves (entry x - lo holds one bit per
// leaf), and stages the bitmaps of other leaves (code sets, IN lists).  The
// batch kernel runs one workgroup per CU whose waves share one set of
// tables: 768 threads (twelve waves, three per SIMD) when every pass fits
// kBatchSlots slots, else 512 threads.  Each pass lays out the LDS for
// itself: at most 4 KB of per-program counters, its tables and bitmaps, and
// its slots for every wave; the tables get what the slots leave of 160 KB
// (7168 words with 64 slots in 8 waves, 9216 with 40 in 12, 27648 with 16).
constexpr uint32_t kBatchBlock = 768;
constexpr uint32_t kLdsPerCu = 160u * 1024u;
// Bytes per lookup-table entry (LDS or device memory): the narrowest of 1,
// 2 and 4 that holds one bit per table leaf (at most 32).
inline constexpr uint32_t tab_entry_bytes(uint32_t m) { return m <= 8 ? 1u : m <= 16 ? 2u : 4u; }
constexpr uint32_t kNoLds = 0xFFFFFFFFu;
// Entry tile ranges are padded to a multiple of this, so that the waves of
// one workgroup (1, 2, 3, 4, 6, 8 or 12) always work on the same entry.
constexpr uint32_t kBatchTileAlign = 24;

// Combinator op of a batched program: op | p_slot << 8 | v_slot << 20.
//   D_RANGE    leaf with predicate word in p_slot (any value test)
//   D_NN_TRUE .. D_NOTNULL   null tests on the validity word in v_slot
//   D_TRUE, D_FALSE, D_AND, D_OR, D_NOT, D_ISUNK as in programs
//   B_AND_LEAF, B_OR_LEAF    a value-test leaf fused with the AND / OR that
//                            consumes it: top = top AND/OR leaf
// v_slot == kNoSlot: the column has no NULLs (validity all ones).
constexpr uint32_t B_AND_LEAF = 24;
constexpr uint32_t B_OR_LEAF = 25;
//   B_ACC        push the program's accumulator: its TRUE word in p_slot
//                (v_slot is kNoSlot; FALSE is taken as NOT TRUE, which the
//                AND at the program's root never lets reach its TRUE word)
//   B_AND_ACC    top = top AND accumulator
constexpr uint32_t B_ACC = 26;
constexpr uint32_t B_AND_ACC = 27;

// The slot field of a batched leaf: bits 0..11 its slot, bits 24..30 the
// slot of its column's validity word or kAccNoValid (no NULLs); the leaf
// stores its TRUE word (test AND validity) there.  With kAccTarget set the
// leaf is a direct factor of one program's conjunction, and bits 0..11 name
// that program's accumulator, into which its TRUE word is ANDed.
// With kAccOr set as well, the leaf belongs to an OR factor of narrow tests
// and its TRUE word is ORed into that factor's word instead.
constexpr uint32_t kAccTarget = 0x80000000u;
constexpr uint32_t kAccOr = 0x00800000u;
constexpr uint32_t kAccNoValid = 0x7Fu;
// Its flags field kAccGuard: lookups are needed only on rows the
// accumulator still holds TRUE.
constexpr uint32_t kAccGuard = 0xFFFFFFFEu;
// Accumulator reset list entries: slot | kInitTrue (reset to ~0) or slot
// (reset to 0), once per tile before the first column.
constexpr uint32_t kInitTrue = 0x80000000u;
inline constexpr uint32_t batch_op(uint32_t op, uint32_t p, uint32_t v) {
  return op | (p << 8) | (v << 20);
}

struct BatchTable {            // 80 bytes: one pass over a table or a chunk
  uint64_t nrows;              // rows of the whole table
  uint64_t tile_begin;         // first flat tile index of this entry
  uint64_t row_begin;          // first row of the entry (a multiple of kTileRows)
  uint64_t ntiles;             // tiles of the entry (its flat range is padded
                               // to a multiple of kBatchTileAlign)
  uint32_t prog_begin;         // into the BatchProg array
  uint32_t prog_count;
  uint32_t col_begin;          // into the BatchCol array
  uint32_t col_count;
  uint32_t bm_begin;           // into the BatchBitmap array
  uint32_t bm_count;
  uint32_t ntab;               // columns with a lookup table
  uint32_t init_begin;         // accumulator reset list, in the ops array
  uint32_t init_count;
  uint32_t bm_words;           // LDS layout of this pass: words of its tables
  uint32_t slot_words;         // and staged bitmaps; each wave's slots (slots * 64)
  uint32_t pad;
};

struct BatchBitmap {           // 24 bytes: a bitmap staged in LDS (batch or scan)
  const uint32_t* src;
  uint32_t words;              // words copied; a zero word follows them
  uint32_t last_mask;          // bits of the last word below nbits
  uint32_t lds_word;           // offset in the workgroup's bitmap area
  uint32_t pad;
};

struct BatchCol {              // 64 bytes: a column one entry reads
  const void* data;
  const uint32_t* valid;       // nullptr: no NULLs
  uint32_t type;               // DevType
  uint32_t vslot;              // slot of the validity word, or kNoSlot
  uint32_t leaf_begin;         // its leaf tests: DevInstr array, slot field set
  uint32_t leaf_count;
  // Lookup table (narrow columns): its first tab_count leaves are bits
  // 0 .. tab_count-1 of entry min(x - tab_lo, tab_n); entry tab_n is zero.
  // Entries are tab_entry_bytes(tab_count) wide.  The table is built in
  // device memory at gtab; one that fits LDS is copied to LDS word offset
  // tab_word when a workgroup starts the pass and read there.
  // tab_word == kNoLds and gtab == nullptr: no table.
  uint32_t tab_word;
  uint32_t tab_count;
  int32_t tab_lo;
  uint32_t tab_n;
  const uint32_t* gtab;
  uint32_t tab_guarded;        // every table leaf has a guard: rows outside
                               // all guards read entry tab_n
  uint32_t pad;
};

// A lookup table in device memory, built by k_tables before the batch
// launch: entry i (i < n) holds bit k = leaf k's test of value lo + i, for
// the m leaves at `leaves`; entry n is zero.  Entries are
// tab_entry_bytes(m) wide.
struct TableBuild {            // 48 bytes
  uint32_t* dst;
  const DevInstr* leaves;
  int64_t lo;
  uint64_t n;
  uint64_t entry_begin;        // first entry of this table in the launch's flat range
  uint32_t m;
  uint32_t pad;
};

struct BatchProg {             // 16 bytes
  const uint32_t* ops;         // batch_op words, postfix
  uint32_t nops;               // | kTwoValued: no NOT and no IS UNKNOWN (TRUE words suffice);
                               // | kAndList (see below)
  uint32_t acc_index;          // accumulator line this program adds into
};

constexpr uint32_t kTwoValued = 0x80000000u;
// | kAndList: the program is a conjunction of TRUE words (its accumulator,
// OR words, leaves) and evaluates to none but TRUE words; its ops array
// then holds the LDS word offsets (slot * 64) of the words to AND.
constexpr uint32_t kAndList = 0x40000000u;
constexpr int kBatchMaxProgs = 1024;
constexpr int kBatchAccStride = 16;   // u64 per accumulator: one 128-byte line each

struct BatchArgs {
  const BatchTable* tables;
  const BatchCol* cols;
  const DevInstr* leaves;
  const BatchProg* progs;
  const BatchBitmap* bms;
  const uint32_t* ops;         // combinator words and accumulator reset lists
  uint32_t ntables;
  uint32_t nprogs;
  uint64_t total_tiles;        // a multiple of kBatchTileAlign
  unsigned long long* acc;     // accumulator lines (kBatchAccStride u64 each)
  // After the launch, the last workgroup moves accumulator done[k] to out[k]
  // and zeroes it (k < ndone); done == nullptr means lines 0 .. ndone-1.
  // Lines not listed keep accumulating across launches.
  const uint32_t* done;
  uint32_t ndone;
  uint32_t acc_words;          // LDS counters: min(nprogs, kBatchMaxProgs)
  unsigned long long* out;
  DevSlot* slot;
};

// ---- batched count over per-column lookup tables of program bits ---------
// A pass holds up to 32 programs whose predicates are conjunctions of
// clauses (ORs of possibly negated leaf tests and null tests): the CNF of
// the program once NOTs are pushed down to the leaves (exact in three-valued
// logic; a row counts when every clause is TRUE).  A row's accumulator is D
// dwords (D = 1, 2 or 4); dword d holds the programs pos_d .. pos_d + G_d - 1
// of the pass, in words of b_d bits (b_d = 32, 16, 8 or 4; G_d <= b_d):
//   word 0 (NA):  bit g set when a clause of program pos_d + g whose
//                 literals all test one column is FALSE or UNKNOWN;
//   word k >= 1:  bit g set when that program's k-th clause spanning
//                 several columns has a TRUE literal (bits of absent
//                 clauses start at 1).
// Every word is combined by OR over the pass's columns, so a column
// contributes one D-dword entry per row: the bits its value (or NULL) sets.
// Program pos_d + g counts the row when bit g of ~NA & word1 & word2 ... is
// set (folded within the dword), and each row's program bits T are added
// into per-lane carry-save bit-plane counters, read out every few dozen
// tiles.
enum LutKind : uint32_t {
  LK_DIRECT = 0,   // entry min(max(x, lo-1), lo+n) - lo + 1; n+2 NULL, n+3 zero
  LK_RANK = 1,     // entry #{k : x >= bound[k]} (n bounds); n+1 NULL, n+2 zero
  LK_VALID = 2     // entry 0 non-NULL, entry 1 NULL (the column's data is not read)
};

// One bit a column sets: for a FAIL atom when none of its literals is TRUE
// (a single-column clause), for a SAT atom when one is (that column's
// literals of a multi-column clause).
enum LutAtomKind : uint32_t { LA_FAIL = 0, LA_SAT = 1 };
struct LutAtom {             // 16 bytes
  uint32_t lit_begin;        // literals: DevInstr with flags = kLitNeg or 0
  uint32_t lit_count;
  uint32_t kind;             // LutAtomKind
  uint32_t bit;              // bit index in the entry's D dwords (dword = bit / 32)
};
constexpr uint32_t kLitNeg = 1;   // DevInstr::flags of a negated literal

struct LutCol {              // 64 bytes
  const void* data;          // values (nullptr for LK_VALID)
  const uint32_t* valid;     // validity words, nullptr: no NULLs
  uint32_t type;             // DevType
  uint32_t kind;             // LutKind
  int64_t lo;                // LK_DIRECT: value of entry 1
  uint32_t n;                // LK_DIRECT: window size; LK_RANK: bounds
  uint32_t lds_word;         // table at this LDS word offset, or kNoLds (device memory)
  const uint32_t* gtab;      // the table in device memory (built by k_luts)
  uint32_t first;            // LK_RANK: first bound
  uint32_t atom_count;       // atoms of the column (table build)
  uint32_t atom_begin;
  uint32_t guard;            // device table: rows no program still needs read the zero entry
};

struct LutPass {             // 112 bytes: one pass over a table or a chunk of it
  uint64_t nrows;            // rows of the whole table
  uint64_t tile_begin;       // first flat tile index (ranges padded to kLutTileAlign)
  uint64_t row_begin;        // first row (a multiple of kTileRows)
  uint64_t ntiles;
  uint32_t col_begin, col_count;
  uint32_t prog_begin, prog_count;   // programs own bits 0 .. prog_count-1
  uint32_t bits;             // bits of T per row in the counters: 8, 16 or 32
  uint32_t dwords;           // D
  uint32_t lds_words;        // LDS words of the pass's staged tables
  uint32_t pmask;            // bits of T that are programs
  uint32_t init[4];          // accumulator start value per dword
  uint32_t fold[4];          // per dword: b_d | G_d << 8 | pos_d << 16 (G_d = 0: unused)
  uint32_t ndata;            // columns with data (the first ones); validity-only ones follow
  uint32_t slot_col[2];      // byte k: the data column (index in the pass) loaded into
                             // register slot k, kSlotHigh set on the second slot of an
                             // int64 column; kNoSlotCol for an unused slot
  uint32_t pad;
};
static_assert(sizeof(LutPass) == 112, "LutPass layout");

// Table build: entry e of column `col` (e < nentries) at dst + e * dwords.
struct LutBuild {            // 40 bytes
  uint32_t* dst;
  uint64_t entry_begin;      // in the launch's flat entry range
  uint32_t col;              // into the LutCol array
  uint32_t nentries;
  uint32_t dwords;
  uint32_t reps;             // LK_RANK: first representative value (int64 array)
  uint32_t pad[2];
};

constexpr uint32_t kLutTileAlign = 48;   // waves of a workgroup: 1, 2, 3, 4, 6, 8, 12 or 16
constexpr uint32_t kLutSlots = 8;        // register slots of two vectors per segment (8 rows per lane)
constexpr uint32_t kNoSlotCol = 0xFF;
constexpr uint32_t kSlotColMask = 0x1F;
constexpr uint32_t kSlotHigh = 0x20;

constexpr uint32_t kLutFlushTiles = 48;  // tiles between reads of the bit-plane counters

struct LutArgs {
  const LutPass* passes;
  const LutCol* cols;
  const LutAtom* atoms;
  const DevInstr* lits;
  const int64_t* bounds;     // LK_RANK bounds (int64, ascending per column)
  const int64_t* reps;       // LK_RANK representative values, one per rank
  const uint32_t* acc_index; // per program of the launch: its accumulator line
  const LutBuild* builds;
  uint32_t npasses;
  uint32_t nprogs;
  uint32_t nbuilds;
  uint32_t acc_words;        // LDS counters: min(nprogs, kBatchMaxProgs)
  uint64_t nentries;         // table entries k_luts writes
  uint64_t total_tiles;      // a multiple of kLutTileAlign
  unsigned long long* acc;   // accumulator lines (kBatchAccStride u64 each)
  const uint32_t* done;      // as BatchArgs
  uint32_t ndone;
  uint32_t pad;
  unsigned long long* out;
  DevSlot* slot;
};

}  // namespace sel

// Launchers implemented in kernels.hip (return hipError_t as int).
extern "C++" {
// Address on `device` (which must be current) of the fixed workspace of
// sel_pushdown_rowids_noalloc, looked up once per device.
int sel_noalloc_scratch(int device, void** ptr);
int sel_launch_scan(int mode, const sel::ScanArgs& a, uint32_t grid, uint32_t block, void* stream);
int sel_launch_scan_tiles(const uint32_t* counts, uint32_t* offsets, uint32_t* chunk_sums,
                          uint32_t* chunk_offs, uint64_t n, void* stream);
int sel_launch_compact(const sel::CompactArgs& a, uint32_t grid, uint32_t block, void* stream);
int sel_launch_gather(const sel::GatherArgs& a, uint32_t grid, uint32_t block, void* stream);
int sel_launch_fill(uint32_t* p, uint64_t nwords, uint32_t value, void* stream);
int sel_launch_tables(const sel::TableBuild* d_builds, uint32_t nbuilds, uint64_t nentries,
                      void* stream);
int sel_scan_occupancy(int mode, uint32_t block, int* blocks_per_cu);
int sel_launch_batch(const sel::BatchArgs& a, uint32_t grid, uint32_t block, uint32_t lds_bytes,
                     void* stream);
int sel_batch_occupancy(uint32_t block, uint32_t lds_bytes, int* blocks_per_cu);
// Table builds, then the lookup-table batch kernel over the passes with
// `dwords` accumulator dwords per row (block at most sel_lbatch_block(dwords),
// the kernel's own workgroup: one per CU, whose LDS it takes).
int sel_launch_luts(const sel::LutArgs& a, void* stream);
uint32_t sel_lbatch_block(uint32_t dwords);
// `rows`: rows per lane per segment, 4 or 8 (four-dword passes take 4).
int sel_launch_lbatch(const sel::LutArgs& a, uint32_t dwords, uint32_t rows, uint32_t grid, uint32_t block,
                      uint32_t lds_bytes, void* stream);
int sel_lbatch_occupancy(uint32_t dwords, uint32_t rows, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu);
}
