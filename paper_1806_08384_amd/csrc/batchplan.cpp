// batchplan.cpp -- descriptors of a leaf-major batched launch.
//
// Algorithm 1 asks for one exact count per candidate relation; a query's
// candidates are predicates over the same few tables, so their leaf tests
// overlap in the columns they read.  The plan regroups the leaves of all
// programs of a table by column: k_batch then reads each column once per
// pass and tile, tests every leaf on it from registers, and runs each
// program's combinators over the resulting truth words held in LDS slots.
#include <algorithm>
#include <cstdio>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>

#include "runtime.h"

using namespace sel;

namespace selrt {

namespace {

// Leaves that test the same column with the same operation share one slot.
using LeafKey = std::tuple<uint32_t, const void*, int64_t, uint64_t, const void*, uint32_t>;

LeafKey key_of(const DevInstr& I) { return LeafKey{I.op, I.data, I.lo, I.span, I.aux, I.n}; }

bool is_value_test(uint32_t op) { return op == D_RANGE || op == D_BITMAP || op == D_INLIST; }
bool is_null_test(uint32_t op) { return op >= D_NN_TRUE && op <= D_NOTNULL; }

struct PassCol {
  const void* data = nullptr;
  const uint32_t* valid = nullptr;
  uint32_t type = 0;
  uint32_t vslot = kNoSlot;
  std::vector<DevInstr> leaves;
  uint32_t tab_word = kNoLds, tab_count = 0, tab_n = 0;
  int32_t tab_lo = 0;
  bool gtab = false;                 // table in device memory instead of LDS
  bool tab_guarded = false;          // ... read only where a leaf's guard holds
};

// A device-memory table pays when it stays in L2 (4 MB per XCD): past this
// size, random lookups into it miss and each costs an HBM burst, while
// separate (guarded) bitmaps of the same leaves are 8 to 32 times smaller.
constexpr uint64_t kMaxDeviceTableBytes = 2ull << 20;
// A table read only where guards hold may be larger: few rows reach it.
constexpr uint64_t kMaxGuardedDeviceTableBytes = 32ull << 20;

// A program split at its top-level conjunction: the instruction ranges
// [begin, end) of its AND factors (postfix subtrees are contiguous) and the
// stack depth each needs.  One factor if the root is not an AND.
struct Factors {
  std::vector<std::pair<size_t, size_t>> ranges;
  std::vector<int> depth;
  bool ok = false;
};

Factors split_and(const std::vector<DevInstr>& code) {
  struct Node { uint32_t op; size_t begin, end; int a, b, depth; };
  std::vector<Node> nodes;
  std::vector<int> st;
  Factors F;
  for (size_t k = 0; k < code.size(); ++k) {
    const uint32_t op = code[k].op;
    if (op == D_AND || op == D_OR) {
      if (st.size() < 2) return F;
      const int b = st.back(); st.pop_back();
      const int a = st.back(); st.pop_back();
      nodes.push_back(Node{op, nodes[a].begin, k + 1, a, b,
                           std::max(nodes[a].depth, 1 + nodes[b].depth)});
    } else if (op == D_NOT || op == D_ISUNK) {
      if (st.empty()) return F;
      const int a = st.back(); st.pop_back();
      nodes.push_back(Node{op, nodes[a].begin, k + 1, a, -1, nodes[a].depth});
    } else {
      nodes.push_back(Node{op, k, k + 1, -1, -1, 1});
    }
    st.push_back((int)nodes.size() - 1);
  }
  if (st.size() != 1) return F;
  std::vector<int> todo{st.back()};
  while (!todo.empty()) {
    const Node n = nodes[todo.back()];
    todo.pop_back();
    if (n.op == D_AND) {
      todo.push_back(n.b);
      todo.push_back(n.a);
    } else {
      F.ranges.push_back({n.begin, n.end});
      F.depth.push_back(n.depth);
    }
  }
  F.ok = true;
  return F;
}

void type_range(uint32_t t, int64_t& lo, int64_t& hi) {
  switch (t) {
    case T_I8: lo = INT8_MIN; hi = INT8_MAX; break;
    case T_I16: lo = INT16_MIN; hi = INT16_MAX; break;
    case T_I32: lo = INT32_MIN; hi = INT32_MAX; break;
    default: lo = INT64_MIN; hi = INT64_MAX; break;
  }
}

// Values [lo, hi] a table leaf can be TRUE on (within the column's type).
bool leaf_window(const DevInstr& L, int64_t& lo, int64_t& hi) {
  int64_t tmin, tmax;
  type_range(L.type, tmin, tmax);
  if (L.op == D_RANGE) {
    lo = L.lo;
    hi = (int64_t)((uint64_t)L.lo + L.span);
  } else if (L.op == D_BITMAP && L.span > 0) {
    lo = L.lo;
    if (L.lo > tmax) return false;
    hi = L.span - 1 > (uint64_t)(tmax - L.lo) ? tmax : L.lo + (int64_t)(L.span - 1);
  } else {
    return false;
  }
  lo = std::max(lo, tmin);
  hi = std::min(hi, tmax);
  return lo <= hi;
}

// One pass under construction.
struct Pass {
  std::vector<PassCol> cols;
  std::map<LeafKey, uint32_t> leaf_slot;
  std::map<const uint32_t*, uint32_t> valid_slot;
  std::vector<std::pair<std::vector<uint32_t>, uint32_t>> progs;  // (ops, acc line)
  uint32_t slots = 0;
  std::vector<uint32_t> inits;   // accumulator slots to reset per tile (| kInitTrue: to ~0)
  std::vector<BatchBitmap> bms;             // staged in LDS
  std::map<const void*, uint32_t> bm_at;    // source -> its BatchBitmap
  uint32_t bm_words = 0;
  uint32_t bm_budget = 0;                   // LDS words for tables and bitmaps

  // Lookup tables and staged bitmaps, within the LDS words the pass's slots
  // leave (bm_budget): first a
  // table for each narrow column whose value-test leaves (bitmaps and
  // ranges, at most 32) cost more per row than a lookup, most leaves first;
  // then the bitmaps of the remaining leaves.  Table leaves move to the
  // front of their column.
  void finalize() {
    // the LDS the pass's slots leave for its tables and bitmaps: every wave
    // of a 768-thread workgroup, or of a 512-thread one past kBatchSlots
    const int64_t waves = slots > kBatchSlots ? 512 / kWave : kBatchBlock / kWave;
    const int64_t left = (int64_t)kLdsPerCu - 4 * (int64_t)kBatchMaxProgs - (int64_t)slots * 256 * waves;
    bm_budget = left > 0 ? (uint32_t)(left / 4) : 0u;
    std::vector<PassCol*> order;
    for (PassCol& c : cols) order.push_back(&c);
    std::stable_sort(order.begin(), order.end(),
                     [](const PassCol* a, const PassCol* b) { return a->leaves.size() > b->leaves.size(); });
    // two rounds: LDS tables within the budget, then device-memory tables
    // for the columns left (one lookup served from L2 instead of one per
    // leaf: for dimension bitmaps too large for LDS)
    for (int round = 0; round < 2; ++round)
    for (PassCol* c : order) {
      if (c->type == T_I64 || c->tab_word != kNoLds || c->gtab) continue;
      std::vector<DevInstr> tab, rest;
      int64_t lo = INT64_MAX, hi = INT64_MIN;
      for (const DevInstr& L : c->leaves) {
        int64_t a, b;
        if (tab.size() < 32 && (L.op == D_RANGE || L.op == D_BITMAP)) {
          if (leaf_window(L, a, b)) {
            lo = std::min(lo, a);
            hi = std::max(hi, b);
          }
          tab.push_back(L);
        } else {
          rest.push_back(L);
        }
      }
      // per row: a table costs a lookup and a 32 x 32 bit transpose (about
      // 13 vector ops for all its leaves); a direct range test about 3, a
      // bitmap lookup about 7 per leaf
      uint32_t direct = 0;
      for (const DevInstr& L : tab) direct += L.op == D_RANGE ? 3u : 7u;
      if (direct <= 13) continue;
      if (lo > hi) { lo = 0; hi = 0; }   // every leaf empty: one all-zero entry
      const uint64_t n = (uint64_t)(hi - lo) + 1;
      // a device table whose every leaf is guarded is read only on rows some
      // leaf needs; the other rows all read its zero entry
      bool guarded = true;
      for (const DevInstr& L : tab) guarded &= L.flags != kNoGuard;
      const uint64_t bytes = (n + 1) * tab_entry_bytes((uint32_t)tab.size());
      if (round == 0) {
        if ((bytes + 3) / 4 > bm_budget - bm_words) continue;
        c->tab_word = bm_words;
        bm_words += (uint32_t)((bytes + 3) / 4);
      } else {
        if (bytes > (guarded ? kMaxGuardedDeviceTableBytes : kMaxDeviceTableBytes)) continue;
        c->gtab = true;
        c->tab_guarded = guarded;
      }
      c->tab_count = (uint32_t)tab.size();
      c->tab_lo = (int32_t)lo;
      c->tab_n = (uint32_t)n;
      c->leaves = tab;
      c->leaves.insert(c->leaves.end(), rest.begin(), rest.end());
    }
    for (PassCol& c : cols) {
      const size_t first = c.tab_word != kNoLds || c.gtab ? c.tab_count : 0;
      for (size_t k = first; k < c.leaves.size(); ++k) stage(c.leaves[k]);
    }
  }

  // Stage a bitmap leaf in LDS if it fits the budget and (for narrow
  // columns) its window [lo, lo + nbits) lies inside int32.
  void stage(DevInstr& L) {
    L.lds_word = kNoLds;
    const uint64_t nbits = L.span;
    if (L.op != D_BITMAP || nbits == 0) return;
    if (L.type != T_I64 &&
        (L.lo < INT32_MIN || L.lo > INT32_MAX || nbits - 1 > (uint64_t)(INT32_MAX - L.lo)))
      return;
    const uint64_t words = (nbits + 31) / 32;
    auto it = bm_at.find(L.aux);
    if (it == bm_at.end() || bms[it->second].words != words) {
      if (bm_words + words + 1 > bm_budget) return;
      BatchBitmap b{};
      b.src = (const uint32_t*)L.aux;
      b.words = (uint32_t)words;
      b.last_mask = nbits % 32 ? (1u << (nbits % 32)) - 1u : ~0u;
      b.lds_word = bm_words;
      bm_words += (uint32_t)words + 1;
      bms.push_back(b);
      it = bm_at.insert_or_assign(L.aux, (uint32_t)bms.size() - 1).first;
    }
    L.lds_word = bms[it->second].lds_word;
    L.n = (uint32_t)words * 32;   // index of a zero bit past the copy
  }

  // A program's plan in this pass: its direct factors (single value-test
  // leaves on narrow columns, applied straight to the program's accumulator
  // word), its OR factors over such leaves only (each ORed into one word of
  // its own), and the other factors in the order they are emitted.
  struct Split {
    std::vector<size_t> direct;
    std::vector<std::pair<size_t, size_t>> ors;
    std::vector<std::pair<size_t, size_t>> rest;
  };
  static bool narrow_test(const DevInstr& I) { return is_value_test(I.op) && I.type != T_I64; }
  // [b, e) is an OR of at least two narrow value tests (postfix: tests and
  // ORs only)
  static bool or_of_tests(const std::vector<DevInstr>& code, size_t b, size_t e) {
    if (e - b < 3) return false;
    for (size_t k = b; k < e; ++k)
      if (!narrow_test(code[k]) && code[k].op != D_OR) return false;
    return true;
  }
  static Split split(const sel_program* p) {
    Split S;
    const std::vector<DevInstr>& code = p->host_code;
    Factors F = split_and(code);
    if (!F.ok) {
      S.rest.push_back({0, code.size()});
      return S;
    }
    std::vector<std::pair<int, std::pair<size_t, size_t>>> rest;
    for (size_t k = 0; k < F.ranges.size(); ++k) {
      const auto r = F.ranges[k];
      const DevInstr& I = code[r.first];
      if (r.second == r.first + 1 && narrow_test(I)) S.direct.push_back(r.first);
      else if (or_of_tests(code, r.first, r.second)) S.ors.push_back(r);
      else rest.push_back({F.depth[k], r});
    }
    // deepest factor first: the chain then needs no more stack than the
    // program did
    std::stable_sort(rest.begin(), rest.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& r : rest) S.rest.push_back(r.second);
    return S;
  }
  // slots a program would add to this pass
  uint32_t new_slots(const sel_program* p) const {
    const Split S = split(p);
    std::vector<LeafKey> nl;
    std::vector<const uint32_t*> nv;
    for (const auto& r : S.rest)
      for (size_t k = r.first; k < r.second; ++k) {
        const DevInstr& I = p->host_code[k];
        if (!is_value_test(I.op)) continue;
        const LeafKey key = key_of(I);
        if (!leaf_slot.count(key) && std::find(nl.begin(), nl.end(), key) == nl.end()) nl.push_back(key);
      }
    for (const DevInstr& I : p->host_code)
      if ((is_value_test(I.op) || is_null_test(I.op)) && I.valid && !valid_slot.count(I.valid) &&
          std::find(nv.begin(), nv.end(), I.valid) == nv.end())
        nv.push_back(I.valid);
    const uint32_t acc = (S.direct.empty() ? 0u : 1u) + (uint32_t)S.ors.size();
    return (uint32_t)(nl.size() + nv.size()) + acc;
  }
  uint32_t vslot_of(const DevInstr& I) {
    if (!I.valid) return kNoSlot;
    auto it = valid_slot.find(I.valid);
    if (it != valid_slot.end()) return it->second;
    const uint32_t s = slots++;
    valid_slot[I.valid] = s;
    // the validity word is loaded with the column holding it (a column that
    // only null tests read joins the list with no leaves)
    PassCol* home = nullptr;
    for (PassCol& c : cols)
      if (c.valid == I.valid || (c.data == I.data && c.data != nullptr)) { home = &c; break; }
    if (!home) {
      cols.push_back(PassCol{});
      home = &cols.back();
      home->data = I.data;
      home->type = I.type;
    }
    home->valid = I.valid;
    home->vslot = s;
    return s;
  }
  PassCol& home_of(const DevInstr& I) {
    for (PassCol& c : cols)
      if (c.data == I.data) return c;
    cols.push_back(PassCol{});
    cols.back().data = I.data;
    cols.back().type = I.type;
    return cols.back();
  }
  // ops of instructions [b, e) of a program, leaves shared across programs
  void emit(const std::vector<DevInstr>& code, size_t b, size_t e, std::vector<uint32_t>& ops) {
    for (size_t pc = b; pc < e; ++pc) {
      const DevInstr& I = code[pc];
      const uint32_t op = I.op;
      if (is_value_test(op)) {
        const LeafKey k = key_of(I);
        auto it = leaf_slot.find(k);
        uint32_t sl;
        const uint32_t vs = vslot_of(I);
        if (it != leaf_slot.end()) {
          sl = it->second;
        } else {
          sl = slots++;
          leaf_slot[k] = sl;
          DevInstr L = I;
          L.flags = kNoGuard;
          L.slot = ((vs == kNoSlot ? kAccNoValid : vs) << 24) | sl;
          L.lds_word = kNoLds;
          home_of(I).leaves.push_back(L);
        }
        ops.push_back(batch_op(D_RANGE, sl, vs));
      } else if (is_null_test(op)) {
        ops.push_back(batch_op(op, 0, vslot_of(I)));
      } else {
        ops.push_back(batch_op(op, 0, 0));
      }
    }
  }
  void add(const sel_program* p, uint32_t acc) {
    const std::vector<DevInstr>& code = p->host_code;
    const Split S = split(p);
    std::vector<uint32_t> ops;
    ops.reserve(code.size() + 2);
    for (size_t k = 0; k < S.rest.size(); ++k) {
      emit(code, S.rest[k].first, S.rest[k].second, ops);
      if (k > 0) ops.push_back(batch_op(D_AND, 0, 0));
    }
    if (!S.direct.empty()) {
      // the program's accumulator: the TRUE word of the conjunction of its
      // direct factors (reset to ~0 per tile).  The count needs only TRUE
      // rows, and the root is an AND, so FALSE and UNKNOWN rows of the
      // accumulator need no word of their own.  Each direct factor ANDs its
      // TRUE word into it when its column is evaluated, and a direct bitmap
      // factor skips lookups on rows that are no longer TRUE.
      const uint32_t ts = slots++;
      inits.push_back(ts | kInitTrue);
      for (size_t pc : S.direct) {
        const DevInstr& I = code[pc];
        const uint32_t vs = vslot_of(I);
        DevInstr L = I;
        L.flags = I.op == D_BITMAP ? kAccGuard : kNoGuard;
        L.slot = kAccTarget | ((vs == kNoSlot ? kAccNoValid : vs) << 24) | ts;
        L.lds_word = kNoLds;
        home_of(I).leaves.push_back(L);
      }
      ops.push_back(batch_op(B_ACC, ts, kNoSlot));
      if (!S.rest.empty()) ops.push_back(batch_op(D_AND, 0, 0));
    }
    // an OR factor of narrow tests: its TRUE word (reset to 0 per tile) is
    // the OR of its leaves' TRUE words, ORed in as their columns are
    // evaluated; it then enters the AND chain like a leaf.  As with the
    // accumulator, only its TRUE rows matter under the root AND.
    for (size_t k = 0; k < S.ors.size(); ++k) {
      const uint32_t os = slots++;
      inits.push_back(os);
      for (size_t pc = S.ors[k].first; pc < S.ors[k].second; ++pc) {
        const DevInstr& I = code[pc];
        if (!is_value_test(I.op)) continue;
        const uint32_t vs = vslot_of(I);
        DevInstr L = I;
        L.flags = kNoGuard;
        L.slot = kAccTarget | kAccOr | ((vs == kNoSlot ? kAccNoValid : vs) << 24) | os;
        L.lds_word = kNoLds;
        home_of(I).leaves.push_back(L);
      }
      ops.push_back(batch_op(D_RANGE, os, kNoSlot));
      if (!S.rest.empty() || !S.direct.empty() || k > 0) ops.push_back(batch_op(D_AND, 0, 0));
    }
    // a value-test leaf (or the accumulator) that is the right operand of
    // the AND / OR right after it combines with the top of the stack directly
    std::vector<uint32_t> fused;
    fused.reserve(ops.size());
    for (size_t k = 0; k < ops.size(); ++k) {
      const uint32_t op = ops[k] & 0xFFu, next = k + 1 < ops.size() ? ops[k + 1] & 0xFFu : 0u;
      if (op == D_RANGE && (next == D_AND || next == D_OR)) {
        fused.push_back((ops[k] & ~0xFFu) | (next == D_AND ? B_AND_LEAF : B_OR_LEAF));
        ++k;
      } else if (op == B_ACC && next == D_AND) {
        fused.push_back((ops[k] & ~0xFFu) | B_AND_ACC);
        ++k;
      } else {
        fused.push_back(ops[k]);
      }
    }
    progs.emplace_back(std::move(fused), acc);
  }
};

}  // namespace

uint32_t batch_slots_alone(const sel_program* p) { return Pass{}.new_slots(p); }

std::vector<std::pair<size_t, size_t>> and_factors(const std::vector<DevInstr>& code) {
  Factors F = split_and(code);
  if (!F.ok) return {{0, code.size()}};
  return F.ranges;
}

void BatchPlan::clear() {
  lut.clear();
  largs = LutArgs{};
  entries.clear();
  cols.clear();
  leaves.clear();
  progs.clear();
  ops.clear();
  bms.clear();
  col_gtab.clear();
  builds.clear();
  gtab_words = 0;
  table_entries = 0;
  total_tiles = 0;
  max_slots = 0;
}

namespace {
// SEL_TRACE_PLAN=1 prints every pass a batch plan makes to stderr.
bool trace_plan() {
  static const bool on = [] {
    const char* v = std::getenv("SEL_TRACE_PLAN");
    return v && std::atoi(v) != 0;
  }();
  return on;
}
}  // namespace

void BatchPlan::add(const sel_table* t, uint64_t row_begin, uint64_t row_end,
                    const sel_program* const* prg_all, const uint32_t* acc_all, uint32_t n_all) {
  if (row_end <= row_begin || n_all == 0) return;
  // The lookup-table kernel takes the programs it can express when the
  // caller allows it: one lookup per column and row serves every program of
  // a pass.  The rest (IS UNKNOWN, too many clauses or columns, a value
  // window whose table would not stay in cache and too many bounds to rank)
  // go to the leaf-major kernel.  The environment variable SEL_BATCH_KERNEL
  // forces either kernel ("lut": every expressible program, "leaf": none).
  std::vector<const sel_program*> prg_v;
  std::vector<uint32_t> acc_v;
  const char* mode = std::getenv("SEL_BATCH_KERNEL");
  const bool force_lut = mode && std::strcmp(mode, "lut") == 0;
  if ((mode && std::strcmp(mode, "leaf") == 0) || (!force_lut && !allow_lut)) {
    prg_v.assign(prg_all, prg_all + n_all);
    acc_v.assign(acc_all, acc_all + n_all);
  } else {
    const size_t first_pass = lut.passes.size();
    const std::vector<uint32_t> rej = lut.add(t, row_begin, row_end, prg_all, acc_all, n_all);
    if (trace_plan())
      for (size_t k = first_pass; k < lut.passes.size(); ++k) {
        const LutPass& e = lut.passes[k];
        uint32_t ldsc = 0;
        for (uint32_t c = 0; c < e.col_count; ++c) ldsc += lut.cols[e.col_begin + c].lds_word != kNoLds;
        std::fprintf(stderr,
                     "sel plan: lut pass rows %llu+%llu programs %u columns %u (data %u, in LDS %u) "
                     "dwords %u LDS words %u\n",
                     (unsigned long long)e.row_begin, (unsigned long long)(row_end - row_begin), e.prog_count,
                     e.col_count, e.ndata, ldsc, e.dwords, e.lds_words);
      }
    for (uint32_t i : rej) {
      prg_v.push_back(prg_all[i]);
      acc_v.push_back(acc_all[i]);
    }
  }
  const sel_program* const* prg = prg_v.data();
  const uint32_t* acc = acc_v.data();
  const uint32_t n = (uint32_t)prg_v.size();
  if (n == 0) return;
  const uint64_t tiles = (row_end - row_begin + kTileRows - 1) / kTileRows;
  auto flush = [&](Pass& ps) {
    if (ps.progs.empty()) return;
    ps.finalize();
    BatchTable e{};
    e.nrows = t->nrows;
    e.tile_begin = total_tiles;
    e.row_begin = row_begin;
    e.prog_begin = (uint32_t)progs.size();
    e.prog_count = (uint32_t)ps.progs.size();
    e.col_begin = (uint32_t)cols.size();
    e.col_count = (uint32_t)ps.cols.size();
    e.ntiles = tiles;
    e.init_begin = (uint32_t)ops.size();
    e.init_count = (uint32_t)ps.inits.size();
    e.bm_words = ps.bm_words;
    e.slot_words = ps.slots * (uint32_t)kWave;
    ops.insert(ops.end(), ps.inits.begin(), ps.inits.end());
    e.bm_begin = (uint32_t)bms.size();
    e.bm_count = (uint32_t)ps.bms.size();
    bms.insert(bms.end(), ps.bms.begin(), ps.bms.end());
    for (PassCol& c : ps.cols) {
      BatchCol bc{};
      bc.data = c.data;
      bc.valid = c.valid;
      bc.type = c.type;
      bc.vslot = c.vslot;
      bc.leaf_begin = (uint32_t)leaves.size();
      bc.leaf_count = (uint32_t)c.leaves.size();
      bc.tab_word = c.tab_word;
      bc.tab_count = c.tab_count;
      bc.tab_lo = c.tab_lo;
      bc.tab_n = c.tab_n;
      bc.tab_guarded = c.tab_guarded ? 1u : 0u;
      col_gtab.push_back(~0ull);
      // every lookup table is built once per launch in device memory by
      // k_tables; an LDS table is then copied into each workgroup's LDS
      if (c.gtab || c.tab_word != kNoLds) {
        TableBuild tbd{};
        tbd.dst = (uint32_t*)(uintptr_t)gtab_words;          // offset until written
        tbd.leaves = (const DevInstr*)(uintptr_t)bc.leaf_begin;  // index until written
        tbd.lo = c.tab_lo;
        tbd.n = c.tab_n;
        tbd.entry_begin = table_entries;
        tbd.m = c.tab_count;
        builds.push_back(tbd);
        col_gtab.back() = gtab_words;
        table_entries += (uint64_t)c.tab_n + 1;
        const uint64_t bytes = ((uint64_t)c.tab_n + 1) * tab_entry_bytes(c.tab_count);
        gtab_words += ((bytes + 255) & ~255ull) / 4;   // 256-byte aligned tables
      }
      e.ntab += c.tab_word != kNoLds ? 1u : 0u;
      leaves.insert(leaves.end(), c.leaves.begin(), c.leaves.end());
      cols.push_back(bc);
    }
    for (auto& pr : ps.progs) {
      BatchProg bp{};
      bp.ops = (const uint32_t*)(uintptr_t)ops.size();
      bp.nops = (uint32_t)pr.first.size();
      bool two = true;   // TRUE words suffice: no NOT, no IS UNKNOWN
      for (uint32_t w : pr.first) {
        const uint32_t op = w & 0xFFu;
        if (op == D_NOT || op == D_ISUNK) two = false;
      }
      if (two) bp.nops |= kTwoValued;
      // a conjunction of TRUE words (a first word, then words ANDed in):
      // store the words' LDS offsets so the kernel needs no decoding
      bool and_list = two && !pr.first.empty();
      for (size_t k = 0; k < pr.first.size() && and_list; ++k) {
        const uint32_t op = pr.first[k] & 0xFFu;
        and_list = k == 0 ? (op == B_ACC || op == D_RANGE) : (op == B_AND_LEAF || op == B_AND_ACC);
      }
      if (and_list) {
        bp.nops = (uint32_t)pr.first.size() | kAndList;
        for (uint32_t w : pr.first) ops.push_back(((w >> 8) & 0xFFFu) * (uint32_t)kWave);
      } else {
        ops.insert(ops.end(), pr.first.begin(), pr.first.end());
      }
      bp.acc_index = pr.second;
      progs.push_back(bp);
    }
    entries.push_back(e);
    max_slots = std::max(max_slots, ps.slots);
    total_tiles += (tiles + kBatchTileAlign - 1) / kBatchTileAlign * kBatchTileAlign;
  };
  // Pack programs that read the same wide columns into the same passes, so
  // that a pass which needs no wide column does not read one: order them by
  // their column sets, widest columns first.
  std::vector<std::vector<std::pair<uint32_t, uintptr_t>>> key(n);
  for (uint32_t i = 0; i < n; ++i) {
    for (const DevInstr& I : prg[i]->host_code) {
      if (!is_value_test(I.op)) continue;
      const std::pair<uint32_t, uintptr_t> c{8u - type_bytes(I.type), (uintptr_t)I.data};
      if (std::find(key[i].begin(), key[i].end(), c) == key[i].end()) key[i].push_back(c);
    }
    std::sort(key[i].begin(), key[i].end());
  }
  std::vector<uint32_t> order(n);
  for (uint32_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return key[x] < key[y]; });
  Pass ps;
  const size_t first_entry = entries.size();
  for (uint32_t i : order) {
    // callers admit only programs that fit a pass of their own
    if (!ps.progs.empty() && ps.slots + ps.new_slots(prg[i]) > kBatchSlots) {
      flush(ps);
      ps = Pass{};
    }
    ps.add(prg[i], acc[i]);
  }
  flush(ps);
  if (trace_plan())
    for (size_t k = first_entry; k < entries.size(); ++k)
      std::fprintf(stderr, "sel plan: leaf pass rows %llu+%llu programs %u columns %u tables %u slots %u\n",
                   (unsigned long long)entries[k].row_begin, (unsigned long long)(row_end - row_begin),
                   entries[k].prog_count, entries[k].col_count, entries[k].ntab, entries[k].slot_words / kWave);
}

namespace {
size_t up(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

namespace {
size_t leaf_bytes(const BatchPlan& p) {
  size_t o = up(p.entries.size() * sizeof(BatchTable));
  o = up(o + p.cols.size() * sizeof(BatchCol));
  o = up(o + p.leaves.size() * sizeof(DevInstr));
  o = up(o + p.progs.size() * sizeof(BatchProg));
  o = up(o + p.ops.size() * sizeof(uint32_t));
  o = up(o + p.bms.size() * sizeof(BatchBitmap));
  return up(o + p.builds.size() * sizeof(TableBuild));
}
}  // namespace

size_t BatchPlan::bytes() const { return leaf_bytes(*this) + (lut.empty() ? 0 : lut.bytes()); }

void BatchPlan::write(uint8_t* host, char* dev, uint32_t* gtab_dev, BatchArgs& a,
                      const TableBuild** d_builds) const {
  const size_t o_cols = up(entries.size() * sizeof(BatchTable));
  const size_t o_leaves = up(o_cols + cols.size() * sizeof(BatchCol));
  const size_t o_progs = up(o_leaves + leaves.size() * sizeof(DevInstr));
  const size_t o_ops = up(o_progs + progs.size() * sizeof(BatchProg));
  const size_t o_bms = up(o_ops + ops.size() * sizeof(uint32_t));
  const size_t o_builds = up(o_bms + bms.size() * sizeof(BatchBitmap));
  std::memset(host, 0, leaf_bytes(*this));
  if (!lut.empty()) {
    const size_t lo = leaf_bytes(*this);
    lut.write(host + lo, dev + lo, gtab_dev + gtab_words, largs);
  }
  if (!entries.empty()) std::memcpy(host, entries.data(), entries.size() * sizeof(BatchTable));
  BatchCol* hc = (BatchCol*)(host + o_cols);
  for (size_t k = 0; k < cols.size(); ++k) {
    hc[k] = cols[k];
    hc[k].gtab = col_gtab[k] == ~0ull ? nullptr : gtab_dev + col_gtab[k];
  }
  TableBuild* hb = (TableBuild*)(host + o_builds);
  for (size_t k = 0; k < builds.size(); ++k) {
    hb[k] = builds[k];
    hb[k].dst = gtab_dev + (uintptr_t)builds[k].dst;
    hb[k].leaves = (const DevInstr*)(dev + o_leaves) + (uintptr_t)builds[k].leaves;
  }
  if (d_builds) *d_builds = (const TableBuild*)(dev + o_builds);
  if (!leaves.empty()) std::memcpy(host + o_leaves, leaves.data(), leaves.size() * sizeof(DevInstr));
  BatchProg* hp = (BatchProg*)(host + o_progs);
  for (size_t k = 0; k < progs.size(); ++k) {
    hp[k] = progs[k];
    hp[k].ops = (const uint32_t*)(dev + o_ops + sizeof(uint32_t) * (uintptr_t)progs[k].ops);
  }
  if (!ops.empty()) std::memcpy(host + o_ops, ops.data(), ops.size() * sizeof(uint32_t));
  if (!bms.empty()) std::memcpy(host + o_bms, bms.data(), bms.size() * sizeof(BatchBitmap));
  a.tables = (const BatchTable*)dev;
  a.cols = (const BatchCol*)(dev + o_cols);
  a.leaves = (const DevInstr*)(dev + o_leaves);
  a.progs = (const BatchProg*)(dev + o_progs);
  a.bms = (const BatchBitmap*)(dev + o_bms);
  a.ops = (const uint32_t*)(dev + o_ops);
  a.ntables = (uint32_t)entries.size();
  a.nprogs = (uint32_t)progs.size();
  a.total_tiles = total_tiles;
  a.acc_words = acc_words();
}

void BatchPlan::lut_shape(uint32_t dwords, uint32_t& grid, uint32_t& block) const {
  block = sel_lbatch_block(dwords);
  // an override applies when its waves divide the tile padding of a pass
  if (lut_block && lut_block < block && lut_block % kWave == 0 && kLutTileAlign % (lut_block / kWave) == 0)
    block = lut_block;
  uint64_t g = lut_grid;
  if (g == 0) {
    int occ = 1;
    if (sel_lbatch_occupancy(dwords, lut_rows, block, lut.lds_bytes(), &occ) != 0 || occ < 1) occ = 1;
    g = (uint64_t)occ * num_cus;
  }
  const uint64_t need = std::max<uint64_t>(1, lut.total_tiles / (block / kWave));
  grid = (uint32_t)std::min(g, need);
}

int BatchPlan::launch(const BatchArgs& a, const TableBuild* d_builds, uint32_t grid, uint32_t block,
                      void* stream) const {
  const bool leaf = !entries.empty() || lut.empty();
  if (!lut.empty()) {
    LutArgs la = largs;
    la.acc = a.acc;
    la.out = a.out;
    la.slot = a.slot;
    la.done = a.done;
    // the last launch moves the finished lines out: k_batch if it runs
    int e = sel_launch_luts(la, stream);
    if (e) return e;
    // one launch per accumulator width present; each takes its own passes
    bool present[5] = {false, false, false, false, false};
    for (const LutPass& p : lut.passes) present[p.dwords] = true;
    const uint32_t last = present[4] ? 4u : present[2] ? 2u : 1u;
    for (uint32_t d : {1u, 2u, 4u}) {
      if (!present[d]) continue;
      la.ndone = !leaf && d == last ? a.ndone : 0u;
      uint32_t lg, lb;
      lut_shape(d, lg, lb);
      e = sel_launch_lbatch(la, d, lut_rows, lg, lb, lut.lds_bytes(), stream);
      if (e) return e;
    }
  }
  if (!leaf) return 0;
  if (!builds.empty()) {
    const int e = sel_launch_tables(d_builds, (uint32_t)builds.size(), table_entries, stream);
    if (e) return e;
  }
  return sel_launch_batch(a, grid, block, lds_bytes(block), stream);
}

uint32_t plan_scan_stage(const std::vector<DevInstr>& code, std::vector<BatchBitmap>& out) {
  out.clear();
  uint32_t words = 0;
  // IN lists first, at even word offsets for their int64 values: the two
  // cuckoo tables of a hashed list (two reads per row), else the sorted
  // list (log2(n) reads per row)
  for (const DevInstr& I : code) {
    if (I.op != D_INLIST || I.n == 0 || out.size() == kMaxStage) continue;
    const bool hashed = (I.flags & F_HASHED) != 0;
    const uint32_t* src = (const uint32_t*)I.aux + (hashed ? 2 * I.n : 0);
    bool seen = false;
    for (const BatchBitmap& b : out) seen |= b.src == src;
    if (seen) continue;
    const uint32_t w = hashed ? 4u << in_hash_bits(I.flags) : 2 * I.n;
    const uint32_t at = (words + 1) & ~1u;
    if (at + w + 1 > kScanStageWords) continue;
    BatchBitmap b{};
    b.src = src;
    b.words = w;
    b.last_mask = ~0u;
    b.lds_word = at;
    out.push_back(b);
    words = at + w + 1;
  }
  for (const DevInstr& I : code) {
    if (I.op != D_BITMAP || I.span == 0 || out.size() == kMaxStage) continue;
    if (I.type != T_I64 &&
        (I.lo < INT32_MIN || I.lo > INT32_MAX || I.span - 1 > (uint64_t)(INT32_MAX - I.lo)))
      continue;
    bool seen = false;
    for (const BatchBitmap& b : out) seen |= b.src == (const uint32_t*)I.aux;
    if (seen) continue;
    const uint64_t w = (I.span + 31) / 32;
    if (words + w + 1 > kScanStageWords) continue;
    BatchBitmap b{};
    b.src = (const uint32_t*)I.aux;
    b.words = (uint32_t)w;
    b.last_mask = I.span % 32 ? (1u << (I.span % 32)) - 1u : ~0u;
    b.lds_word = words;
    out.push_back(b);
    words += (uint32_t)w + 1;
  }
  return words;
}

}  // namespace selrt
