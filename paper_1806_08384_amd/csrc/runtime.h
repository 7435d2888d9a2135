// runtime.h -- host runtime objects of libsel (contexts, tables, programs)
// and the helpers the C-ABI translation units share.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sel.h"
#include "sel_device.h"
#include "sel_internal.h"

using sel::DevInstr;
using sel::DevSlot;

namespace selrt {

struct EventPair {
  hipEvent_t a, b;
};

// First-fit allocator over one device buffer, for compiled programs: a
// compile then costs one async copy instead of a hipMalloc.  Blocks are
// reused in stream order (all work of a context runs on its one stream), so
// a kernel still reading a freed program finishes before the next copy into
// that block.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  void init(char* base, size_t size) {
    base_ = base;
    free_.clear();
    free_[0] = size;
  }
  char* alloc(size_t n) {
    n = (n + kAlign - 1) & ~(kAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, left = it->second - n;
        free_.erase(it);
        if (left) free_[off + n] = left;
        used_[off] = n;
        return base_ + off;
      }
    }
    return nullptr;
  }
  bool owns(const void* p) const { return base_ && used_.count((size_t)((const char*)p - base_)); }
  void release(void* p) {
    auto u = used_.find((size_t)((char*)p - base_));
    if (u == used_.end()) return;
    size_t off = u->first, n = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  char* base_ = nullptr;
  std::map<size_t, size_t> free_;  // offset -> bytes
  std::map<size_t, size_t> used_;
};

constexpr size_t kArenaBytes = 8u << 20;
// Resident waves per CU of an untuned scan launch.
constexpr int kScanWavesPerCu = 12;
constexpr size_t kStageBytes = 1u << 20;
}  // namespace selrt

struct sel_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint32_t num_cus = 0;
  std::string err;

  DevSlot* slot = nullptr;                 // device
  unsigned long long* dout = nullptr;      // device, 2 values
  unsigned long long* hout = nullptr;      // pinned host, 2 values
  char* hstage = nullptr;                  // pinned host staging (kStageBytes)
  hipEvent_t stage_free = nullptr;         // recorded after each copy out of hstage
  DevInstr* dstar = nullptr;               // device, star-count program (128)
  sel::BatchBitmap* dstage = nullptr;      // device, its staged bitmaps (kMaxStage)
  DevInstr* dtrue = nullptr;               // device, the program TRUE
  void* arena_mem = nullptr;               // device, programs
  void* batch_mem = nullptr;               // device, sel_count_batch workspace
  size_t batch_bytes = 0;
  unsigned long long* hbatch = nullptr;    // pinned host, kBatchMaxProgs counts
  selrt::Arena arena;
  void* scratch = nullptr;                 // device, grow-only
  void* fixed_scratch = nullptr;           // device, the library's fixed
                                           // workspace on this device
  size_t scratch_bytes = 0;

  sel_launch launch{256, 0, 0, 1, 0, 0};
  bool launch_fixed = false;
  std::map<uint64_t, sel_launch> tune;     // autotuned launch shapes by class
  int occ[3] = {0, 0, 0};                  // blocks per CU per scan mode at 256 threads

  bool timing = false;
  std::vector<selrt::EventPair> free_events;
  std::vector<std::pair<int, selrt::EventPair>> pending;
  double ms[SEL_K_NKINDS] = {};
  uint64_t launches[SEL_K_NKINDS] = {};
};

struct sel_table {
  sel_ctx* ctx;
  uint64_t nrows;
  std::vector<sel_column> cols;
};

struct sel_program {
  sel_ctx* ctx;
  const sel_table* table;
  void* dev = nullptr;              // code then blob: in the context's arena,
  bool own_alloc = false;           // or its own hipMalloc if the arena is full
  DevInstr* dcode = nullptr;
  std::vector<DevInstr> host_code;  // with device pointers (for star programs)
  std::vector<DevInstr> factor_code;  // the conjuncts as written (range tests of a
                                      // column not merged), same device constants
  std::vector<uint8_t> host_blob;   // host copy of the constants (IN lists, bitmaps)
  uintptr_t blob_dev = 0;           // their device address
  const sel::BatchBitmap* dstage = nullptr;   // bitmaps a scan stages in LDS
  uint32_t nstage = 0, stage_words = 0;
  std::vector<uint32_t> stage_end;  // per staged bitmap: the LDS words up to its end
  uint32_t nins = 0;
  uint32_t tune_class = 0;          // bytes-per-row and length bucket
  int depth = 0;
  double bytes_per_row = 0.0;
  std::string text;
  // the batched count's conjunctive form of the program (for the lookup-
  // table kernel), made on first use and kept: a program does not change
  // after its compile.  Null when the program has none.
  mutable std::once_flag lut_once;
  mutable std::shared_ptr<const void> lut_form;
};

namespace selrt {

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
    dev_ = dev;
  }
  ~DeviceGuard() {
    if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1, dev_ = 0;
};

sel_status set_err(sel_ctx* ctx, sel_status st, const std::string& msg);
sel_status hip_err(sel_ctx* ctx, hipError_t e, const char* where);
uint32_t dev_type(int32_t t);
uint32_t type_bytes(uint32_t dt);
sel_status ensure_scratch(sel_ctx* ctx, size_t bytes);
sel_status stage_copy(sel_ctx* ctx, void* dst, const void* src, size_t n);
sel_status read_out(sel_ctx* ctx, uint64_t* v0, uint64_t* v1);
EventPair take_events(sel_ctx* ctx);
uint64_t ntiles_of(uint64_t nrows);

// Launch-shape classes for the tuner: a class of programs (bytes per row,
// length) and a size bucket of the table (log2 of its tile count).
uint32_t tune_class_of(double bytes_per_row, uint32_t nins);
uint64_t tune_key(int kind, uint32_t cls, uint64_t ntiles);
enum TuneKind { TK_COUNT = 0, TK_MASK = 1, TK_KEYBITMAP = 2, TK_BATCH = 3 };
inline uint32_t batch_class(uint32_t nprogs) {
  uint32_t c = 0;
  while ((1u << c) < nprogs) ++c;
  return c;
}
// The launch configuration a context uses when the caller fixed none.
constexpr sel_launch kDefaultLaunch{256, 0, 0, 1, 0, 0};
void scan_shape(sel_ctx* ctx, int mode, uint32_t cls, uint64_t ntiles, sel_launch& cfg, uint32_t& grid,
                uint32_t& block);
sel_status run_scan(sel_ctx* ctx, int mode, uint32_t cls, sel::ScanArgs& a, int kind,
                    bool timed = true, const std::vector<uint32_t>* stage_end = nullptr);

// Byte layout of the row-id path's workspace for a table of ntiles tiles:
// the packed mask words, tile counts, tile offsets, chunk sums, chunk
// offsets and tile lane maps, in that order.
struct RowidScratch {
  size_t mask, counts, chunk, lanes;
  explicit RowidScratch(uint64_t ntiles)
      : mask((size_t)ntiles * sel::kWave * 4),
        counts(((size_t)ntiles * 4 + 255) & ~size_t(255)),
        chunk(2048 * 4),
        lanes(((size_t)ntiles * 8 + 255) & ~size_t(255)) {}
  size_t total() const { return mask + 2 * counts + 2 * chunk + lanes; }
};
// The push-down of sel_pushdown_rowids with its workspace at `sp` (at least
// RowidScratch(ntiles).total() bytes of device memory); arguments checked.
sel_status pushdown_rowids_with(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                                uint64_t max_rows, uint32_t* d_out, uint64_t cap,
                                uint64_t* out_count, char* sp, bool timed);

// Descriptors of the batched count over per-column lookup tables of program
// bits (k_luts, k_lbatch): passes of up to 32 programs in conjunctive form.
struct LutPlan {
  std::vector<sel::LutPass> passes;
  std::vector<sel::LutCol> cols;       // gtab holds a word offset until written
  std::vector<sel::LutAtom> atoms;
  std::vector<DevInstr> lits;
  std::vector<int64_t> bounds, reps;
  std::vector<uint32_t> acc_index;     // per program: its accumulator line
  std::vector<sel::LutBuild> builds;   // dst holds a word offset until written
  uint64_t gtab_words = 0;             // tables in device memory, in words
  uint64_t nentries = 0;
  uint64_t total_tiles = 0;
  uint32_t max_lds_words = 0;
  void clear();
  bool empty() const { return passes.empty(); }
  // Passes over rows [row_begin, row_end) of t for the programs it can
  // express; returns the indices (into prg) of the others.
  std::vector<uint32_t> add(const sel_table* t, uint64_t row_begin, uint64_t row_end,
                            const sel_program* const* prg, const uint32_t* acc, uint32_t n);
  size_t bytes() const;
  void write(uint8_t* host, char* dev, uint32_t* gtab_dev, sel::LutArgs& a) const;
  uint32_t acc_words() const {
    return ((uint32_t)std::min<size_t>(acc_index.size(), (size_t)sel::kBatchMaxProgs) + 3u) & ~3u;
  }
  uint32_t lds_bytes() const { return 4u * (acc_words() + max_lds_words); }
};

// Descriptors of one leaf-major batched launch (k_batch).  add() appends
// passes over rows [row_begin, row_end) of a table for a list of programs;
// a pass holds as many programs as fit kBatchSlots LDS slots (deduplicated
// leaf words plus validity words; a single larger program gets a pass of its
// own), so each pass reads its columns once.
struct BatchPlan {
  // programs in conjunctive form go to the lookup-table kernel, the others
  // to the leaf-major one; both add into the same accumulator lines
  LutPlan lut;
  bool allow_lut = false;                // set by the caller before add()
  mutable sel::LutArgs largs{};          // as written
  uint32_t num_cus = 256;
  uint32_t lut_block = 0, lut_grid = 0;  // 0: the defaults
  mutable uint32_t lut_rows = 8;         // rows per lane per segment (four-dword passes: 4)
  std::vector<sel::BatchTable> entries;
  std::vector<sel::BatchCol> cols;
  std::vector<DevInstr> leaves;
  std::vector<sel::BatchProg> progs;   // ops holds an index into `ops` until written
  std::vector<uint32_t> ops;
  std::vector<sel::BatchBitmap> bms;
  std::vector<uint64_t> col_gtab;        // per column: word offset of its device table, or ~0
  std::vector<sel::TableBuild> builds;   // dst / leaves hold offsets until written
  uint64_t gtab_words = 0;               // device-memory tables of k_batch, in words
  uint64_t table_entries = 0;            // entries k_tables writes
  uint64_t total_tiles = 0;
  uint32_t max_slots = 0;
  void clear();
  // acc[k]: accumulator line of progs[k].  Programs of an empty range add
  // nothing (their lines stay zero).
  void add(const sel_table* t, uint64_t row_begin, uint64_t row_end,
           const sel_program* const* progs, const uint32_t* acc, uint32_t n);
  size_t bytes() const;
  // Device-memory tables of both kernels, in words.
  uint64_t gtab_total() const { return gtab_words + lut.gtab_words; }
  // Image of the descriptors for device address `dev` into `host` (bytes()
  // long), with the device tables at gtab_dev (gtab_total() words); sets
  // the descriptor pointers and counts of `a` (and of largs) and the device
  // address of the table builds.
  void write(uint8_t* host, char* dev, uint32_t* gtab_dev, sel::BatchArgs& a,
             const sel::TableBuild** d_builds) const;
  // Enqueue the table builds (if any) and the batch kernels: the lookup-table
  // kernel (its own launch shape) first, then k_batch (grid x block); the
  // last of them moves the finished accumulator lines out.
  int launch(const sel::BatchArgs& a, const sel::TableBuild* d_builds, uint32_t grid,
             uint32_t block, void* stream) const;
  // Launch shape of the lookup-table kernel for passes of `dwords` dwords.
  void lut_shape(uint32_t dwords, uint32_t& grid, uint32_t& block) const;
  uint32_t acc_words() const {
    return (uint32_t)std::min<size_t>(progs.size(), (size_t)sel::kBatchMaxProgs);
  }
  // Dynamic LDS of the batch kernel: the largest pass layout (counters,
  // tables and bitmaps, every wave's slots).
  uint32_t lds_bytes(uint32_t block) const {
    uint32_t m = 0;
    for (const sel::BatchTable& e : entries)
      m = std::max(m, 4u * (acc_words() + e.bm_words + e.slot_words * (block / 64)));
    return m;
  }
  // Workgroup size: kBatchBlock when its LDS fits a CU, else 512 (a pass
  // with more than kBatchSlots slots).
  uint32_t default_block() const { return lds_bytes(sel::kBatchBlock) <= sel::kLdsPerCu ? sel::kBatchBlock : 512u; }
};

// The postfix ranges [begin, end) of a program's top-level AND factors,
// left to right as the program evaluates them (the whole program if its root
// is not an AND).
std::vector<std::pair<size_t, size_t>> and_factors(const std::vector<sel::DevInstr>& code);
// LDS slots a program needs in a pass of its own (distinct leaves plus
// validity words); batching requires at most kBatchMaxSlots.
uint32_t batch_slots_alone(const sel_program* p);
// The bitmaps of a program that a single-program scan stages in LDS: in
// program order, distinct, windows inside int32 for narrow columns, at most
// kScanStageWords words with one zero word after each.  Returns the words.
constexpr uint32_t kMaxStage = 64;
uint32_t plan_scan_stage(const std::vector<DevInstr>& code, std::vector<sel::BatchBitmap>& out);
inline void set_stage(sel::ScanArgs& a, const sel_program* p) {
  a.stage = p ? p->dstage : nullptr;
  a.nstage = p ? p->nstage : 0;
  a.stage_words = p ? p->stage_words : 0;
}
// Keep only the staged bitmaps that end within `limit` LDS words (a prefix:
// they are placed in order); 0 keeps them all.
inline void limit_stage(sel::ScanArgs& a, const std::vector<uint32_t>& stage_end, uint32_t limit) {
  if (limit == 0) return;
  uint32_t k = 0;
  while (k < a.nstage && k < stage_end.size() && stage_end[k] <= limit) ++k;
  a.nstage = k;
  a.stage_words = k ? stage_end[k - 1] : 0;
}

sel_status plan_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                      const sel_program* const* progs, BatchPlan& bp);

// Brackets one kernel launch with events when timing is on.
struct TimedLaunch {
  sel_ctx* ctx;
  int kind;
  EventPair ev{};
  bool on;
  // timed = false: never (the calls that must not create events)
  TimedLaunch(sel_ctx* c, int k, bool timed = true);
  void done();
};

}  // namespace selrt

#define HIP_TRY(ctx, call, where)                                   \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return selrt::hip_err(ctx, e_, where);    \
  } while (0)
