// lutplan.cpp -- descriptors of the batched count over per-column lookup
// tables of program bits (k_luts builds the tables, k_lbatch counts).
//
// Algorithm 1 asks for one exact count per candidate relation, and a query's
// candidates are predicates over the same few columns.  Each program is put
// in conjunctive form: NOTs are pushed down to the leaves (De Morgan and
// double negation hold in three-valued logic), then ORs are distributed
// over ANDs, giving clauses of possibly negated leaf tests.  A row counts
// when every clause has a TRUE literal.  For each column of a pass, one
// table maps the column's value (or NULL) to the bits it sets for every
// program at once: a clause whose literals all test that column sets its
// program's failure bit when none is TRUE, and a clause spanning several
// columns has a word bit of its own that each column sets when one of its
// literals there is TRUE.  Programs with IS UNKNOWN, or whose conjunctive
// form is too large, stay with the leaf-major kernel.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>

#include "runtime.h"

using namespace sel;

namespace selrt {

namespace {

constexpr size_t kMaxClauses = 24;        // clauses of one program
constexpr size_t kMaxClauseLits = 16;     // literals of one clause
constexpr uint32_t kMaxPassProgs = 32;    // program bits of a pass
constexpr uint32_t kMaxPassCols = 16;
constexpr uint32_t kMaxRankBounds = 32;
// device-memory tables up to 2 MB (a 512 K-value window at one dword): a
// larger one misses the L2 on most lookups, where a bitmap leaf of the
// leaf-major kernel (one bit per value) would not
constexpr uint64_t kMaxTableBytes = 2ull << 20;
// LDS of the kernel's workgroup: 160 KB less the per-program counters
constexpr uint32_t kLutLdsWords = (kLdsPerCu - 4u * (uint32_t)kBatchMaxProgs) / 4u;

struct Lit {
  DevInstr ins;
  bool neg;
};
using Clause = std::vector<Lit>;

bool is_value(uint32_t op) { return op == D_RANGE || op == D_BITMAP || op == D_INLIST; }

struct Node {
  uint32_t op;
  int a, b;
  DevInstr ins;
};

// Conjunctive form of the subtree at `at` (negated if neg); false if it has
// IS UNKNOWN or outgrows the limits.  No clauses: TRUE; an empty clause:
// FALSE.
bool cnf(const std::vector<Node>& t, int at, bool neg, std::vector<Clause>& out) {
  const Node& n = t[at];
  switch (n.op) {
    case D_NOT:
      return cnf(t, n.a, !neg, out);
    case D_ISUNK:
      return false;
    case D_TRUE:
    case D_FALSE:
      out.clear();
      if ((n.op == D_TRUE) == neg) out.push_back(Clause{});
      return true;
    case D_AND:
    case D_OR: {
      std::vector<Clause> A, B;
      if (!cnf(t, n.a, neg, A) || !cnf(t, n.b, neg, B)) return false;
      if ((n.op == D_AND) != neg) {   // a conjunction: both clause lists
        out = std::move(A);
        out.insert(out.end(), B.begin(), B.end());
      } else {                        // a disjunction: clause by clause
        if (A.size() * B.size() > kMaxClauses) return false;
        out.clear();
        for (const Clause& x : A)
          for (const Clause& y : B) {
            Clause c = x;
            c.insert(c.end(), y.begin(), y.end());
            out.push_back(std::move(c));
          }
      }
      if (out.size() > kMaxClauses) return false;
      for (const Clause& c : out)
        if (c.size() > kMaxClauseLits) return false;
      return true;
    }
    default:
      out.assign(1, Clause{Lit{n.ins, neg}});
      return true;
  }
}

// The column a literal reads: its data for a value test; for a null test
// the data of a value test in the same clause with the same validity, else
// the validity words alone (tagged so they never equal a data pointer).
uintptr_t lit_col(const Lit& L, const Clause& c) {
  if (is_value(L.ins.op)) return (uintptr_t)L.ins.data;
  for (const Lit& o : c)
    if (is_value(o.ins.op) && o.ins.valid == L.ins.valid) return (uintptr_t)o.ins.data;
  return (uintptr_t)L.ins.valid | 1u;
}

uint32_t bits_for(uint32_t nprogs) { return nprogs <= 8 ? 8u : nprogs <= 16 ? 16u : 32u; }

// Width of the words of a dword whose programs need up to W words (the
// failure word and one per multi-column clause): 32 / width words fit.
uint32_t word_bits(uint32_t W) { return W <= 1 ? 32u : W == 2 ? 16u : W <= 4 ? 8u : W <= 8 ? 4u : 0u; }

// Dwords of a pass: programs taken in order of their word counts, each
// dword holding as many as its word width allows.
struct DwordGroup {
  uint32_t W = 1, count = 0;
};
std::vector<DwordGroup> pack_dwords(std::vector<uint32_t> Ws) {
  std::stable_sort(Ws.begin(), Ws.end());
  std::vector<DwordGroup> g;
  for (uint32_t W : Ws) {
    if (!g.empty()) {
      const uint32_t w2 = std::max(g.back().W, W);
      if (g.back().count + 1 <= word_bits(w2)) {
        g.back().W = w2;
        ++g.back().count;
        continue;
      }
    }
    g.push_back(DwordGroup{W, 1});
  }
  return g;
}
uint32_t dwords_for(const std::vector<uint32_t>& Ws) {
  const size_t d = pack_dwords(Ws).size();
  return d <= 1 ? 1u : d == 2 ? 2u : d <= 4 ? 4u : 0u;
}

struct Form {
  std::vector<Clause> clauses;
  std::vector<std::vector<uintptr_t>> cols;   // per clause: its columns (distinct)
  std::map<uintptr_t, uint32_t> slots;        // per column: register slots of its data
  uint32_t ncross = 0;                        // clauses over several columns
  bool always_false = false;
  const sel_program* prog = nullptr;
};

bool make_form(const sel_program* p, Form& f) {
  const std::vector<DevInstr>& code = p->host_code;
  std::vector<Node> t;
  std::vector<int> st;
  for (const DevInstr& I : code) {
    Node n{I.op, -1, -1, I};
    if (I.op == D_AND || I.op == D_OR) {
      if (st.size() < 2) return false;
      n.b = st.back();
      st.pop_back();
      n.a = st.back();
      st.pop_back();
    } else if (I.op == D_NOT || I.op == D_ISUNK) {
      if (st.empty()) return false;
      n.a = st.back();
      st.pop_back();
    }
    t.push_back(n);
    st.push_back((int)t.size() - 1);
  }
  if (st.size() != 1) return false;
  if (!cnf(t, st.back(), false, f.clauses)) return false;
  f.prog = p;
  for (const Clause& c : f.clauses)
    if (c.empty()) f.always_false = true;
  if (f.always_false) f.clauses.clear();
  for (const Clause& c : f.clauses) {
    std::vector<uintptr_t> cs;
    for (const Lit& L : c) {
      const uintptr_t k = lit_col(L, c);
      if (std::find(cs.begin(), cs.end(), k) == cs.end()) cs.push_back(k);
      if (is_value(L.ins.op)) f.slots[k] = L.ins.type == T_I64 ? 2u : 1u;
      else f.slots.emplace(k, 0u);
    }
    if (cs.size() > 1) ++f.ncross;
    f.cols.push_back(std::move(cs));
  }
  return word_bits(f.ncross + 1) != 0;
}

// The program's form, made once and shared by every plan that takes the
// program (plans are built on several threads: the caller's and a server's).
const Form* form_of(const sel_program* p) {
  std::call_once(p->lut_once, [p] {
    auto f = std::make_shared<Form>();
    if (make_form(p, *f)) p->lut_form = std::move(f);
  });
  return static_cast<const Form*>(p->lut_form.get());
}

// A program of one plan: its form and its place in the caller's list.
struct FormRef {
  const Form* f;
  uint32_t acc;
};

void type_range(uint32_t ty, int64_t& lo, int64_t& hi) {
  switch (ty) {
    case T_I8: lo = INT8_MIN; hi = INT8_MAX; break;
    case T_I16: lo = INT16_MIN; hi = INT16_MAX; break;
    case T_I32: lo = INT32_MIN; hi = INT32_MAX; break;
    default: lo = INT64_MIN; hi = INT64_MAX; break;
  }
}

// The values of a sorted IN list, from the program's host copy of its
// constants (none if the copy is missing).
bool inlist_values(const sel_program* p, const DevInstr& I, std::vector<int64_t>& v) {
  if (!p || p->host_blob.empty()) return false;
  const uintptr_t off = (uintptr_t)I.aux - p->blob_dev;
  if ((uintptr_t)I.aux < p->blob_dev || off + 8ull * I.n > p->host_blob.size()) return false;
  v.resize(I.n);
  std::memcpy(v.data(), p->host_blob.data() + off, 8ull * I.n);
  return true;
}

struct ColAtom {
  std::vector<Lit> lits;
  uint32_t kind, bit;
};

struct PassCol {
  uintptr_t key = 0;
  const void* data = nullptr;
  const uint32_t* valid = nullptr;
  uint32_t type = 0;
  bool valid_only = true;
  std::vector<ColAtom> atoms;
  std::vector<const sel_program*> owners;   // program of each value-test literal (IN values)
  // placement
  uint32_t kind = LK_VALID;
  int64_t lo = 0;
  uint64_t n = 0;
  std::vector<int64_t> bounds, reps;
  uint64_t entries = 0;
  bool lds = false;
};

}  // namespace

void LutPlan::clear() {
  passes.clear();
  cols.clear();
  atoms.clear();
  lits.clear();
  bounds.clear();
  reps.clear();
  acc_index.clear();
  builds.clear();
  gtab_words = 0;
  nentries = 0;
  total_tiles = 0;
  max_lds_words = 0;
}

namespace {

// Window, kind and table size of a pass column; false if it has no form
// the kernel takes.
bool place_col(PassCol& c, uint32_t dwords) {
  if (c.valid_only) {
    c.kind = LK_VALID;
    c.entries = 2;
    return true;
  }
  int64_t tmin, tmax;
  type_range(c.type, tmin, tmax);
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  bool rankable = true;
  std::vector<int64_t> b;
  size_t li = 0;
  for (const ColAtom& A : c.atoms)
    for (const Lit& L : A.lits) {
      if (!is_value(L.ins.op)) continue;
      const sel_program* owner = c.owners[li++];
      int64_t a, z;
      if (L.ins.op == D_RANGE) {
        a = L.ins.lo;
        z = (int64_t)((uint64_t)L.ins.lo + L.ins.span);
        if (a > tmin) b.push_back(a);
        if (z < tmax) b.push_back(z + 1);
      } else if (L.ins.op == D_BITMAP) {
        if (L.ins.span == 0) continue;
        a = L.ins.lo;
        z = L.ins.span - 1 > (uint64_t)tmax - (uint64_t)a ? tmax : (int64_t)((uint64_t)a + L.ins.span - 1);
        rankable = false;
      } else {   // D_INLIST: [min, max] of the sorted list
        a = L.ins.lo;
        z = (int64_t)((uint64_t)L.ins.lo + L.ins.span);
        std::vector<int64_t> v;
        if (!inlist_values(owner, L.ins, v)) {
          rankable = false;
        } else {
          for (int64_t x : v) {
            if (x > tmin) b.push_back(x);
            if (x < tmax) b.push_back(x + 1);
          }
        }
      }
      a = std::max(a, tmin);
      z = std::min(z, tmax);
      if (a > z) continue;
      lo = std::min(lo, a);
      hi = std::max(hi, z);
    }
  if (lo > hi) {   // no value can make a value test TRUE
    lo = 0;
    hi = 0;
  }
  const uint64_t n = (uint64_t)hi - (uint64_t)lo + 1;   // 0: all of int64
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end()), b.end());
  const bool direct_ok = n != 0 && n <= (1ull << 30) && (n + 4) * 4ull * dwords <= kMaxTableBytes &&
                         (c.type != T_I64 || hi < INT64_MAX);
  rankable = rankable && b.size() <= kMaxRankBounds;
  if (!direct_ok && !rankable) return false;
  // a window that would not fit LDS costs a device-memory lookup per row;
  // a few bounds cost two compares each instead
  const bool small = direct_ok && (n + 4) * dwords <= kLutLdsWords / 2;
  if (direct_ok && (small || !rankable || b.size() > 8)) {
    c.kind = LK_DIRECT;
    c.lo = lo;
    c.n = n;
    c.entries = n + 4;
  } else {
    c.kind = LK_RANK;
    c.bounds = b;
    c.reps.clear();
    c.reps.push_back(b.empty() ? std::max<int64_t>(0, tmin) : b[0] - 1);
    for (int64_t x : b) c.reps.push_back(x);
    c.n = b.size();
    c.entries = b.size() + 3;
  }
  return true;
}

}  // namespace

std::vector<uint32_t> LutPlan::add(const sel_table* t, uint64_t row_begin, uint64_t row_end,
                                   const sel_program* const* prg, const uint32_t* acc, uint32_t n) {
  std::vector<uint32_t> rejected;
  if (row_end <= row_begin || n == 0) return rejected;
  const uint64_t tiles = (row_end - row_begin + kTileRows - 1) / kTileRows;
  std::vector<FormRef> forms;
  forms.reserve(n);
  for (uint32_t i = 0; i < n; ++i) {
    const Form* f = form_of(prg[i]);
    if (!f) {
      rejected.push_back(i);
      continue;
    }
    forms.push_back(FormRef{f, i});
  }
  // programs that read the same columns share passes: order by column set
  std::vector<std::vector<uintptr_t>> key(forms.size());
  for (size_t i = 0; i < forms.size(); ++i) {
    for (const auto& cs : forms[i].f->cols)
      for (uintptr_t k : cs)
        if (std::find(key[i].begin(), key[i].end(), k) == key[i].end()) key[i].push_back(k);
    std::sort(key[i].begin(), key[i].end());
  }
  std::map<uintptr_t, uint32_t> slots;
  for (const FormRef& r : forms)
    for (const auto& kv : r.f->slots) slots[kv.first] = std::max(slots[kv.first], kv.second);
  auto slots_of = [&](const std::set<uintptr_t>& cs) {
    uint32_t n = 0;
    for (uintptr_t k : cs) n += slots[k];
    return n;
  };
  std::vector<size_t> order(forms.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });

  // a pass's programs, then its columns, bits and tables
  auto emit = [&](std::vector<const FormRef*> ps) -> bool {
    // programs by word count: the pass's dwords take them in this order
    std::stable_sort(ps.begin(), ps.end(),
                     [](const FormRef* x, const FormRef* y) { return x->f->ncross < y->f->ncross; });
    const uint32_t P = (uint32_t)ps.size();
    std::vector<uint32_t> Ws;
    for (const FormRef* r : ps) Ws.push_back(1 + r->f->ncross);
    const std::vector<DwordGroup> groups = pack_dwords(Ws);
    const uint32_t B = bits_for(P), D = dwords_for(Ws);
    if (D == 0) return false;
    // program j: its dword, slot and the dword's word width
    std::vector<uint32_t> pd(P), pg(P), pb(P);
    {
      uint32_t j = 0;
      for (uint32_t d = 0; d < groups.size(); ++d)
        for (uint32_t g = 0; g < groups[d].count; ++g, ++j) {
          pd[j] = d;
          pg[j] = g;
          pb[j] = word_bits(groups[d].W);
        }
    }
    std::vector<PassCol> pc;
    auto col_of = [&](uintptr_t k, const Lit& L) -> PassCol& {
      for (PassCol& c : pc)
        if (c.key == k) return c;
      pc.push_back(PassCol{});
      PassCol& c = pc.back();
      c.key = k;
      c.type = L.ins.type;
      return c;
    };
    for (uint32_t j = 0; j < P; ++j) {
      const Form& f = *ps[j]->f;
      uint32_t cross = 0;
      for (size_t ci = 0; ci < f.clauses.size(); ++ci) {
        const Clause& cl = f.clauses[ci];
        const bool local = f.cols[ci].size() == 1;
        const uint32_t bit = 32 * pd[j] + (local ? 0u : (++cross) * pb[j]) + pg[j];
        for (uintptr_t k : f.cols[ci]) {
          ColAtom A;
          A.kind = local ? LA_FAIL : LA_SAT;
          A.bit = bit;
          for (const Lit& L : cl)
            if (lit_col(L, cl) == k) A.lits.push_back(L);
          PassCol& c = col_of(k, A.lits.front());
          for (const Lit& L : A.lits) {
            if (L.ins.valid) c.valid = L.ins.valid;
            if (is_value(L.ins.op)) {
              c.data = L.ins.data;
              c.type = L.ins.type;
              c.valid_only = false;
              c.owners.push_back(f.prog);
            }
          }
          c.atoms.push_back(std::move(A));
        }
      }
    }
    if (pc.size() > kMaxPassCols) return false;
    for (PassCol& c : pc)
      if (!place_col(c, D)) return false;
    // LDS for the smallest tables first; validity-only columns are read from
    // device memory with scalar loads.  Columns with data come first, tables
    // in device memory (guarded) after those in LDS.
    std::vector<PassCol*> order_c;
    for (PassCol& c : pc) order_c.push_back(&c);
    std::stable_sort(order_c.begin(), order_c.end(),
                     [](const PassCol* a, const PassCol* b) { return a->entries < b->entries; });
    uint32_t lds_words = 0;
    for (PassCol* c : order_c) {
      if (c->kind == LK_VALID) continue;
      const uint64_t words = (c->entries * D + 3) & ~3ull;
      if (lds_words + words <= kLutLdsWords) {
        c->lds = true;
        lds_words += (uint32_t)words;
      }
    }
    std::stable_sort(order_c.begin(), order_c.end(), [](const PassCol* a, const PassCol* b) {
      const int ra = a->kind == LK_VALID ? 2 : a->lds ? 0 : 1;
      const int rb = b->kind == LK_VALID ? 2 : b->lds ? 0 : 1;
      return ra < rb;
    });
    LutPass e{};
    e.nrows = t->nrows;
    e.tile_begin = total_tiles;
    e.row_begin = row_begin;
    e.ntiles = tiles;
    e.col_begin = (uint32_t)cols.size();
    e.col_count = (uint32_t)pc.size();
    e.prog_begin = (uint32_t)acc_index.size();
    e.prog_count = P;
    e.bits = B;
    e.dwords = D;
    e.pmask = P == 32 ? ~0u : (1u << P) - 1u;
    // accumulator start: failure bits clear (set for a program that is
    // always FALSE and for unused slots), clause bits clear where the
    // program has that clause and set elsewhere; per dword the fold: word
    // width, programs, first program
    for (uint32_t d = 0; d < 4; ++d) {
      e.init[d] = ~0u;
      e.fold[d] = 32u;   // no programs
    }
    {
      uint32_t j = 0;
      for (uint32_t d = 0; d < groups.size(); ++d) {
        const uint32_t b = word_bits(groups[d].W);
        e.fold[d] = b | (groups[d].count << 8) | (j << 16);
        uint32_t init = ~0u;
        for (uint32_t g = 0; g < groups[d].count; ++g, ++j) {
          if (!ps[j]->f->always_false) init &= ~(1u << g);
          for (uint32_t k = 1; k <= ps[j]->f->ncross; ++k) init &= ~(1u << (k * b + g));
        }
        e.init[d] = init;
      }
    }
    // register slots: int64 columns first (two each, aligned), then the
    // narrower ones
    e.slot_col[0] = e.slot_col[1] = ~0u;
    {
      uint32_t k = 0;
      for (int wide = 1; wide >= 0; --wide)
        for (uint32_t ci = 0; ci < order_c.size(); ++ci) {
          const PassCol* c = order_c[ci];
          if (c->kind == LK_VALID || (c->type == T_I64) != (wide == 1)) continue;
          const uint32_t need = c->type == T_I64 ? 2u : 1u;
          if (k + need > kLutSlots) return false;
          for (uint32_t h = 0; h < need; ++h, ++k) {
            e.slot_col[k / 4] &= ~(0xFFu << (8 * (k % 4)));
            e.slot_col[k / 4] |= (ci | (h ? kSlotHigh : 0u)) << (8 * (k % 4));
          }
        }
    }
    uint32_t lw = 0;
    for (PassCol* c : order_c) {
      LutCol lc{};
      lc.data = c->kind == LK_VALID ? nullptr : c->data;
      lc.valid = c->valid;
      lc.type = c->type;
      lc.kind = c->kind;
      lc.lo = c->lo;
      lc.n = (uint32_t)c->n;
      lc.first = (uint32_t)bounds.size();
      lc.atom_begin = (uint32_t)atoms.size();
      lc.atom_count = (uint32_t)c->atoms.size();
      lc.lds_word = kNoLds;
      if (c->lds) {
        lc.lds_word = lw;
        lw += (uint32_t)((c->entries * D + 3) & ~3ull);
      }
      lc.guard = c->lds || c->kind == LK_VALID ? 0u : 1u;
      for (const ColAtom& A : c->atoms) {
        LutAtom la{};
        la.lit_begin = (uint32_t)lits.size();
        la.lit_count = (uint32_t)A.lits.size();
        la.kind = A.kind;
        la.bit = A.bit;
        for (const Lit& L : A.lits) {
          DevInstr I = L.ins;
          I.flags = L.neg ? kLitNeg : 0u;
          lits.push_back(I);
        }
        atoms.push_back(la);
      }
      LutBuild b{};
      b.dst = (uint32_t*)(uintptr_t)gtab_words;   // offset until written
      b.entry_begin = nentries;
      b.col = (uint32_t)cols.size();
      b.nentries = (uint32_t)c->entries;
      b.dwords = D;
      b.reps = (uint32_t)reps.size();
      builds.push_back(b);
      lc.gtab = (const uint32_t*)(uintptr_t)gtab_words;
      nentries += c->entries;
      gtab_words += ((c->entries * D * 4 + 255) & ~255ull) / 4;
      bounds.insert(bounds.end(), c->bounds.begin(), c->bounds.end());
      // whole blocks of eight for the kernel's block loads
      while (bounds.size() % 8) bounds.push_back(INT64_MAX);
      reps.insert(reps.end(), c->reps.begin(), c->reps.end());
      if (c->kind != LK_VALID) ++e.ndata;
      cols.push_back(lc);
    }
    e.lds_words = lw;
    max_lds_words = std::max(max_lds_words, lw);
    for (const FormRef* r : ps) acc_index.push_back(acc[r->acc]);
    passes.push_back(e);
    total_tiles += (tiles + kLutTileAlign - 1) / kLutTileAlign * kLutTileAlign;
    return true;
  };
  // greedy packing; a pass that cannot be placed sends its programs back
  std::vector<const FormRef*> cur;
  std::set<uintptr_t> cur_cols;
  auto flush = [&]() {
    if (cur.empty()) return;
    // emit checks everything before it appends anything
    if (!emit(cur))
      for (const FormRef* r : cur) rejected.push_back(r->acc);
    cur.clear();
    cur_cols.clear();
  };
  for (size_t oi : order) {
    const FormRef& r = forms[oi];
    const Form& f = *r.f;
    std::set<uintptr_t> cs = cur_cols;
    for (const auto& c : f.cols) cs.insert(c.begin(), c.end());
    const uint32_t P = (uint32_t)cur.size() + 1;
    std::vector<uint32_t> Ws;
    for (const FormRef* g : cur) Ws.push_back(1 + g->f->ncross);
    Ws.push_back(1 + f.ncross);
    if (!cur.empty() && (P > kMaxPassProgs || dwords_for(Ws) == 0 || cs.size() > kMaxPassCols ||
                         slots_of(cs) > kLutSlots)) {
      flush();
      cs.clear();
      for (const auto& c : f.cols) cs.insert(c.begin(), c.end());
    }
    cur.push_back(&r);
    cur_cols = cs;
  }
  flush();
  std::sort(rejected.begin(), rejected.end());
  return rejected;
}

namespace {
size_t up(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

size_t LutPlan::bytes() const {
  size_t o = up(passes.size() * sizeof(LutPass));
  o = up(o + cols.size() * sizeof(LutCol));
  o = up(o + atoms.size() * sizeof(LutAtom));
  o = up(o + lits.size() * sizeof(DevInstr));
  o = up(o + bounds.size() * sizeof(int64_t));
  o = up(o + reps.size() * sizeof(int64_t));
  o = up(o + acc_index.size() * sizeof(uint32_t));
  return up(o + builds.size() * sizeof(LutBuild));
}

void LutPlan::write(uint8_t* host, char* dev, uint32_t* gtab_dev, LutArgs& a) const {
  const size_t o_cols = up(passes.size() * sizeof(LutPass));
  const size_t o_atoms = up(o_cols + cols.size() * sizeof(LutCol));
  const size_t o_lits = up(o_atoms + atoms.size() * sizeof(LutAtom));
  const size_t o_bounds = up(o_lits + lits.size() * sizeof(DevInstr));
  const size_t o_reps = up(o_bounds + bounds.size() * sizeof(int64_t));
  const size_t o_acc = up(o_reps + reps.size() * sizeof(int64_t));
  const size_t o_builds = up(o_acc + acc_index.size() * sizeof(uint32_t));
  std::memset(host, 0, bytes());
  if (!passes.empty()) std::memcpy(host, passes.data(), passes.size() * sizeof(LutPass));
  LutCol* hc = (LutCol*)(host + o_cols);
  for (size_t k = 0; k < cols.size(); ++k) {
    hc[k] = cols[k];
    hc[k].gtab = gtab_dev + (uintptr_t)cols[k].gtab;
  }
  if (!atoms.empty()) std::memcpy(host + o_atoms, atoms.data(), atoms.size() * sizeof(LutAtom));
  if (!lits.empty()) std::memcpy(host + o_lits, lits.data(), lits.size() * sizeof(DevInstr));
  if (!bounds.empty()) std::memcpy(host + o_bounds, bounds.data(), bounds.size() * sizeof(int64_t));
  if (!reps.empty()) std::memcpy(host + o_reps, reps.data(), reps.size() * sizeof(int64_t));
  if (!acc_index.empty()) std::memcpy(host + o_acc, acc_index.data(), acc_index.size() * sizeof(uint32_t));
  LutBuild* hb = (LutBuild*)(host + o_builds);
  for (size_t k = 0; k < builds.size(); ++k) {
    hb[k] = builds[k];
    hb[k].dst = gtab_dev + (uintptr_t)builds[k].dst;
  }
  a.passes = (const LutPass*)dev;
  a.cols = (const LutCol*)(dev + o_cols);
  a.atoms = (const LutAtom*)(dev + o_atoms);
  a.lits = (const DevInstr*)(dev + o_lits);
  a.bounds = (const int64_t*)(dev + o_bounds);
  a.reps = (const int64_t*)(dev + o_reps);
  a.acc_index = (const uint32_t*)(dev + o_acc);
  a.builds = (const LutBuild*)(dev + o_builds);
  a.npasses = (uint32_t)passes.size();
  a.nprogs = (uint32_t)acc_index.size();
  a.nbuilds = (uint32_t)builds.size();
  a.acc_words = acc_words();
  a.nentries = nentries;
  a.total_tiles = total_tiles;
}

}  // namespace selrt
