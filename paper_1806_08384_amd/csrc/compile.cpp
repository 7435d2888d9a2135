// compile.cpp -- predicate program compiler: postfix sel_instr -> device
// program (sel_device.h).  Pure host C++ with no HIP calls, so it also runs
// (through sel_program_check) on machines without a GPU.
//
// What it does, per leaf, for a column of type [tmin, tmax]:
//   col = a           -> RANGE [a, a]            (a outside the type: FALSE)
//   col <> a          -> NOT RANGE [a, a]        (keeps NULL rows UNKNOWN)
//   col < a, <= a     -> RANGE [tmin, a-1 | a]   clamped; empty -> FALSE
//   col > a, >= a     -> RANGE [a+1 | a, tmax]   clamped
//   a <= col <= b     -> RANGE [a, b] clamped    (a > b -> FALSE)
//   col IN (list)     -> values outside the type dropped, sorted, deduped;
//                        1 value or a run -> RANGE; span <= 65536 -> BITMAP
//                        over [min, max]; otherwise a sorted list
//   CODESET(nbits)    -> BITMAP over [0, nbits); no code set -> FALSE
//   IS [NOT] NULL     -> constant when the column has no NULLs
// where "FALSE"/"TRUE" of a comparison mean FALSE/TRUE on non-NULL rows and
// UNKNOWN on NULL rows (SQL three-valued logic), and become plain constants
// only on columns without NULLs.  A RANGE covering the whole type needs no
// column data at all.  Then AND/OR operands are ordered so the subtree that
// needs the deeper stack runs first (Sethi-Ullman); Kleene AND and OR are
// commutative, so no row's truth value changes.  Finally a leaf that is the
// right operand of AND (OR) is flagged so the kernel may skip its lookups
// on rows whose left operand is already FALSE (TRUE).
#include <algorithm>
#include <functional>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/sel.h"
#include "sel_device.h"
#include "sel_internal.h"

namespace sel {

namespace {

constexpr uint64_t kMaxBitmapSpanForIn = 65536;

struct Node {
  enum Kind { LEAF, AND, OR, NOT, ISUNK, TRUE_, FALSE_ } kind = LEAF;
  DevInstr ins{};
  std::vector<uint8_t> aux;  // bitmap words or sorted int64 list
  int a = -1, b = -1;        // children
  int need = 1;              // stack depth needed (Sethi-Ullman)
  uint32_t col = 0;
};

void type_range(uint32_t ty, int64_t& lo, int64_t& hi) {
  switch (ty) {
    case T_I8: lo = INT8_MIN; hi = INT8_MAX; break;
    case T_I16: lo = INT16_MIN; hi = INT16_MAX; break;
    case T_I32: lo = INT32_MIN; hi = INT32_MAX; break;
    default: lo = INT64_MIN; hi = INT64_MAX; break;
  }
}

const char* type_name(uint32_t ty) {
  switch (ty) {
    case T_I8: return "i8";
    case T_I16: return "i16";
    case T_I32: return "i32";
    default: return "i64";
  }
}

// Two cuckoo tables of 2^b slots (b the least with 2^b >= 2 n, at least
// 4) for the sorted distinct values v: each value in slot
// in_hash(x, c1, b) of the first table or in_hash(x, c2, b) of the second,
// empty slots holding v[0].  Multiplier pairs are tried in order; false if
// insertion cycles under all of them.
bool cuckoo_tables(const std::vector<int64_t>& v, std::vector<int64_t>& tabs, uint32_t& b, uint32_t& pair) {
  b = 4;
  while ((1ull << b) < 2 * v.size()) ++b;
  const size_t m = size_t(1) << b;
  for (pair = 0; pair < kInHashPairs; ++pair) {
    const uint32_t c[2] = {kInHashMul[pair][0], kInHashMul[pair][1]};
    std::vector<int64_t> t(2 * m);
    std::vector<char> used(2 * m, 0);
    bool ok = true;
    for (int64_t x : v) {
      int64_t cur = x;
      int side = 0;
      bool placed = false;
      for (int kick = 0; kick < 64 && !placed; ++kick) {
        const size_t slot = side * m + in_hash(cur, c[side], b);
        if (!used[slot]) {
          used[slot] = 1;
          t[slot] = cur;
          placed = true;
        } else {
          std::swap(cur, t[slot]);   // evict the occupant to its other table
          side ^= 1;
        }
      }
      if (!placed) {
        ok = false;
        break;
      }
    }
    if (!ok) continue;
    for (size_t k = 0; k < 2 * m; ++k)
      if (!used[k]) t[k] = v[0];
    tabs.swap(t);
    return true;
  }
  return false;
}

struct Builder {
  const ColInfo* cols;
  uint32_t ncols;
  std::vector<Node> nodes;
  std::string* err;
  bool merged = false;

  int add(Node n) {
    nodes.push_back(std::move(n));
    return (int)nodes.size() - 1;
  }

  int constant(bool v) {
    Node n;
    n.kind = v ? Node::TRUE_ : Node::FALSE_;
    return add(n);
  }

  // TRUE (FALSE) on every non-NULL row, UNKNOWN on NULL rows.
  int nonnull_const(uint32_t col, bool v) {
    if (!cols[col].nullable) return constant(v);
    Node n;
    n.ins.op = v ? D_NN_TRUE : D_NN_FALSE;
    n.ins.type = cols[col].type;
    n.ins.valid = cols[col].valid;
    n.col = col;
    return add(n);
  }

  int range(uint32_t col, int64_t lo, int64_t hi) {
    int64_t tmin, tmax;
    type_range(cols[col].type, tmin, tmax);
    if (lo > hi || hi < tmin || lo > tmax) return nonnull_const(col, false);
    lo = std::max(lo, tmin);
    hi = std::min(hi, tmax);
    if (lo == tmin && hi == tmax) return nonnull_const(col, true);
    Node n;
    n.ins.op = D_RANGE;
    n.ins.type = cols[col].type;
    n.ins.data = cols[col].data;
    n.ins.valid = cols[col].valid;
    n.ins.lo = lo;
    n.ins.span = (uint64_t)hi - (uint64_t)lo;
    n.col = col;
    return add(n);
  }

  int bitmap(uint32_t col, int64_t base, const std::vector<uint32_t>& words, uint64_t nbits) {
    Node n;
    n.ins.op = D_BITMAP;
    n.ins.type = cols[col].type;
    n.ins.data = cols[col].data;
    n.ins.valid = cols[col].valid;
    n.ins.lo = base;
    n.ins.span = nbits;
    n.aux.resize(words.size() * 4);
    if (!words.empty()) std::memcpy(n.aux.data(), words.data(), n.aux.size());
    n.col = col;
    return add(n);
  }

  int unary(Node::Kind k, int child) {
    Node n;
    n.kind = k;
    n.a = child;
    return add(n);
  }

  int in_list(uint32_t col, const int64_t* vals, uint64_t count) {
    int64_t tmin, tmax;
    type_range(cols[col].type, tmin, tmax);
    std::vector<int64_t> v;
    for (uint64_t k = 0; k < count; ++k)
      if (vals[k] >= tmin && vals[k] <= tmax) v.push_back(vals[k]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if (v.empty()) return nonnull_const(col, false);
    const int64_t mn = v.front(), mx = v.back();
    const uint64_t span = (uint64_t)mx - (uint64_t)mn + 1;  // 0 if all of int64
    if (span != 0 && span == v.size()) return range(col, mn, mx);
    if (span != 0 && span <= kMaxBitmapSpanForIn) {
      std::vector<uint32_t> words((span + 31) / 32, 0u);
      for (int64_t x : v) {
        const uint64_t d = (uint64_t)x - (uint64_t)mn;
        words[d / 32] |= 1u << (d % 32);
      }
      return bitmap(col, mn, words, span);
    }
    Node n;
    n.ins.op = D_INLIST;
    n.ins.type = cols[col].type;
    n.ins.data = cols[col].data;
    n.ins.valid = cols[col].valid;
    n.ins.n = (uint32_t)v.size();
    n.ins.lo = mn;   // the list's window [lo, lo + span]
    n.ins.span = (uint64_t)mx - (uint64_t)mn;
    n.aux.resize(v.size() * 8);
    std::memcpy(n.aux.data(), v.data(), n.aux.size());
    // short lists: two cuckoo tables after the sorted list, for the scans
    std::vector<int64_t> tabs;
    uint32_t b = 0, pair = 0;
    if (v.size() <= kInHashMax && cuckoo_tables(v, tabs, b, pair)) {
      n.ins.flags |= F_HASHED | (b << 8) | (pair << 16);
      const size_t at = n.aux.size();
      n.aux.resize(at + tabs.size() * 8);
      std::memcpy(n.aux.data() + at, tabs.data(), tabs.size() * 8);
    }
    n.col = col;
    return add(n);
  }
};

// Range tests of one column under the same conjunction become one test of
// the intersection of their ranges (an empty one: FALSE on every non-NULL
// row).  Exact in three-valued logic: on a NULL row every such test, the
// merged one too, is UNKNOWN.  A column is then read once per tile instead
// of once per test.  Returns the node that replaces `id`.
void and_operands(const std::vector<Node>& nodes, int id, std::vector<int>& ops) {
  if (nodes[id].kind == Node::AND) {
    and_operands(nodes, nodes[id].a, ops);
    and_operands(nodes, nodes[id].b, ops);
  } else {
    ops.push_back(id);
  }
}

int merge_and_ranges(Builder& B, int id) {
  const Node::Kind kind = B.nodes[id].kind;
  if (kind == Node::NOT || kind == Node::ISUNK) {
    const int a = merge_and_ranges(B, B.nodes[id].a);
    B.nodes[id].a = a;
    return id;
  }
  if (kind == Node::OR) {
    const int a = merge_and_ranges(B, B.nodes[id].a);
    const int b = merge_and_ranges(B, B.nodes[id].b);
    B.nodes[id].a = a;
    B.nodes[id].b = b;
    return id;
  }
  if (kind != Node::AND) return id;
  std::vector<int> ops;
  and_operands(B.nodes, id, ops);
  for (int& o : ops) o = merge_and_ranges(B, o);
  bool merged = false;
  for (size_t i = 0; i < ops.size(); ++i) {
    if (ops[i] < 0) continue;
    const Node& first = B.nodes[ops[i]];
    if (first.kind != Node::LEAF || first.ins.op != D_RANGE) continue;
    int64_t lo = first.ins.lo;
    int64_t hi = (int64_t)((uint64_t)first.ins.lo + first.ins.span);
    bool any = false;
    for (size_t j = i + 1; j < ops.size(); ++j) {
      if (ops[j] < 0) continue;
      const Node& o = B.nodes[ops[j]];
      if (o.kind != Node::LEAF || o.ins.op != D_RANGE || o.col != first.col) continue;
      lo = std::max(lo, o.ins.lo);
      hi = std::min(hi, (int64_t)((uint64_t)o.ins.lo + o.ins.span));
      ops[j] = -1;
      any = true;
    }
    if (!any) continue;
    merged = true;
    B.merged = true;
    const uint32_t col = B.nodes[ops[i]].col;
    if (lo > hi) {
      ops[i] = B.nonnull_const(col, false);
    } else {   // a new leaf: the tree's nodes are left as they are
      Node c = B.nodes[ops[i]];
      c.ins.lo = lo;
      c.ins.span = (uint64_t)hi - (uint64_t)lo;
      ops[i] = B.add(c);
    }
  }
  if (!merged) {
    // the operands may have changed below: rebuild the chain as it was
    // shaped only if something merged at this level
    int k = 0;
    std::function<int(int)> relink = [&](int n) -> int {
      if (B.nodes[n].kind == Node::AND) {
        const int a = relink(B.nodes[n].a);
        const int b = relink(B.nodes[n].b);
        B.nodes[n].a = a;
        B.nodes[n].b = b;
        return n;
      }
      return ops[k++];
    };
    return relink(id);
  }
  // the remaining operands, in their order, as a chain of ANDs
  int acc = -1;
  for (int o : ops) {
    if (o < 0) continue;
    if (acc < 0) {
      acc = o;
      continue;
    }
    Node nd;
    nd.kind = Node::AND;
    nd.a = acc;
    nd.b = o;
    acc = B.add(nd);
  }
  return acc;
}

int fail(std::string* err, sel_status st, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  *err = buf;
  return st;
}

int compute_need(std::vector<Node>& nodes, int id) {
  Node& n = nodes[id];
  switch (n.kind) {
    case Node::AND:
    case Node::OR: {
      int l = compute_need(nodes, n.a), r = compute_need(nodes, n.b);
      if (r > l) { std::swap(nodes[id].a, nodes[id].b); std::swap(l, r); }
      nodes[id].need = l == r ? l + 1 : l;
      return nodes[id].need;
    }
    case Node::NOT:
    case Node::ISUNK:
      nodes[id].need = compute_need(nodes, n.a);
      return nodes[id].need;
    default:
      nodes[id].need = 1;
      return 1;
  }
}

void emit(std::vector<Node>& nodes, int id, Lowered& out, uint32_t guard) {
  Node& n = nodes[id];
  switch (n.kind) {
    case Node::LEAF: {
      DevInstr ins = n.ins;
      // the guard of this position, beside what the leaf itself carries
      // (a hashed IN list's table geometry)
      ins.flags = ((ins.op == D_RANGE || ins.op == D_BITMAP || ins.op == D_INLIST) ? guard : 0u) |
                  (n.ins.flags & ~(uint32_t)(F_GUARD_AND | F_GUARD_OR));
      if (!n.aux.empty()) {
        size_t off = (out.blob.size() + 7) & ~size_t(7);
        out.blob.resize(off + n.aux.size());
        std::memcpy(out.blob.data() + off, n.aux.data(), n.aux.size());
        ins.aux = (const void*)(uintptr_t)off;
        out.aux_is_offset.push_back(1);
      } else {
        out.aux_is_offset.push_back(0);
      }
      out.code.push_back(ins);
      if (std::find(out.columns.begin(), out.columns.end(), n.col) == out.columns.end() &&
          (ins.op == D_RANGE || ins.op == D_BITMAP || ins.op == D_INLIST))
        out.columns.push_back(n.col);
      if (ins.valid &&
          std::find(out.valid_columns.begin(), out.valid_columns.end(), n.col) == out.valid_columns.end())
        out.valid_columns.push_back(n.col);
      return;
    }
    case Node::TRUE_:
    case Node::FALSE_: {
      DevInstr ins{};
      ins.op = n.kind == Node::TRUE_ ? D_TRUE : D_FALSE;
      out.code.push_back(ins);
      out.aux_is_offset.push_back(0);
      return;
    }
    case Node::NOT:
    case Node::ISUNK: {
      emit(nodes, n.a, out, 0);
      DevInstr ins{};
      ins.op = n.kind == Node::NOT ? D_NOT : D_ISUNK;
      out.code.push_back(ins);
      out.aux_is_offset.push_back(0);
      return;
    }
    case Node::AND:
    case Node::OR: {
      emit(nodes, n.a, out, 0);
      emit(nodes, n.b, out, n.kind == Node::AND ? F_GUARD_AND : F_GUARD_OR);
      DevInstr ins{};
      ins.op = n.kind == Node::AND ? D_AND : D_OR;
      out.code.push_back(ins);
      out.aux_is_offset.push_back(0);
      return;
    }
  }
}

}  // namespace

std::string listing(const Lowered& L) {
  std::string s;
  char buf[256];
  for (size_t k = 0; k < L.code.size(); ++k) {
    const DevInstr& I = L.code[k];
    const char* g = (I.flags & F_GUARD_AND) ? " guard_and" : (I.flags & F_GUARD_OR) ? " guard_or" : "";
    switch (I.op) {
      case D_RANGE:
        std::snprintf(buf, sizeof buf, "RANGE %s lo=%lld hi=%lld%s%s\n", type_name(I.type),
                      (long long)I.lo, (long long)((uint64_t)I.lo + I.span), I.valid ? " nullable" : "", g);
        break;
      case D_BITMAP:
        std::snprintf(buf, sizeof buf, "BITMAP %s base=%lld nbits=%llu%s%s\n", type_name(I.type),
                      (long long)I.lo, (unsigned long long)I.span, I.valid ? " nullable" : "", g);
        break;
      case D_INLIST:
        std::snprintf(buf, sizeof buf, "INLIST %s n=%u%s%s%s\n", type_name(I.type), I.n,
                      (I.flags & F_HASHED) ? " hashed" : "", I.valid ? " nullable" : "", g);
        break;
      case D_NN_TRUE: std::snprintf(buf, sizeof buf, "NONNULL_TRUE\n"); break;
      case D_NN_FALSE: std::snprintf(buf, sizeof buf, "NONNULL_FALSE\n"); break;
      case D_ISNULL: std::snprintf(buf, sizeof buf, "ISNULL\n"); break;
      case D_NOTNULL: std::snprintf(buf, sizeof buf, "NOTNULL\n"); break;
      case D_AND: std::snprintf(buf, sizeof buf, "AND\n"); break;
      case D_OR: std::snprintf(buf, sizeof buf, "OR\n"); break;
      case D_NOT: std::snprintf(buf, sizeof buf, "NOT\n"); break;
      case D_ISUNK: std::snprintf(buf, sizeof buf, "ISUNKNOWN\n"); break;
      case D_TRUE: std::snprintf(buf, sizeof buf, "TRUE\n"); break;
      default: std::snprintf(buf, sizeof buf, "FALSE\n"); break;
    }
    s += buf;
  }
  return s;
}

size_t aux_bytes(const DevInstr& I) {
  if (I.op == D_BITMAP) return (size_t)((I.span + 31) / 32) * 4;
  if (I.op == D_INLIST)
    return (size_t)I.n * 8 + ((I.flags & F_HASHED) ? (size_t(16) << in_hash_bits(I.flags)) : 0);
  return 0;
}

int lower_program(const ColInfo* cols, uint32_t ncols, const sel_instr* code, uint32_t n,
                  const uint8_t* pool, uint32_t pool_bytes, Lowered& out, std::string& err,
                  bool merge_ranges) {
  out = Lowered{};
  if (code == nullptr || n == 0 || n > SEL_MAX_INSTRS)
    return fail(&err, SEL_E_INVALID, "program length %u invalid (1..64)", n);
  if (pool_bytes > SEL_MAX_POOL_BYTES)
    return fail(&err, SEL_E_INVALID, "pool of %u bytes exceeds 65536", pool_bytes);
  if (pool_bytes > 0 && pool == nullptr) return fail(&err, SEL_E_INVALID, "pool is NULL (%u bytes)", pool_bytes);
  Builder B{cols, ncols, {}, &err};
  std::vector<int> stack;
  for (uint32_t pc = 0; pc < n; ++pc) {
    const sel_instr& I = code[pc];
    const uint32_t op = I.op;
    const bool leaf = op >= SEL_OP_EQ && op <= SEL_OP_IS_NOT_NULL;
    if (leaf && I.col >= ncols)
      return fail(&err, SEL_E_INVALID, "instruction %u: column %u out of range", pc, (unsigned)I.col);
    int id = -1;
    switch (op) {
      case SEL_OP_EQ: id = B.range(I.col, I.a, I.a); break;
      case SEL_OP_NE: id = B.unary(Node::NOT, B.range(I.col, I.a, I.a)); break;
      case SEL_OP_LT:
        id = I.a == INT64_MIN ? B.nonnull_const(I.col, false) : B.range(I.col, INT64_MIN, I.a - 1);
        break;
      case SEL_OP_LE: id = B.range(I.col, INT64_MIN, I.a); break;
      case SEL_OP_GT:
        id = I.a == INT64_MAX ? B.nonnull_const(I.col, false) : B.range(I.col, I.a + 1, INT64_MAX);
        break;
      case SEL_OP_GE: id = B.range(I.col, I.a, INT64_MAX); break;
      case SEL_OP_BETWEEN: id = B.range(I.col, I.a, I.b); break;
      case SEL_OP_IN: {
        if (I.b < 1 || I.b > (int64_t)(SEL_MAX_POOL_BYTES / 8))
          return fail(&err, SEL_E_INVALID, "instruction %u: IN list length %lld invalid", pc, (long long)I.b);
        if (I.aux % 8 != 0 || (uint64_t)I.aux + 8ull * (uint64_t)I.b > pool_bytes)
          return fail(&err, SEL_E_INVALID, "instruction %u: IN list at pool offset %u out of bounds or misaligned", pc, (unsigned)I.aux);
        std::vector<int64_t> vals((size_t)I.b);
        std::memcpy(vals.data(), pool + I.aux, vals.size() * 8);
        id = B.in_list(I.col, vals.data(), vals.size());
        break;
      }
      case SEL_OP_CODESET: {
        if (cols[I.col].dict_card == 0)
          return fail(&err, SEL_E_TYPE, "instruction %u: CODESET on column %u that is not dictionary-coded", pc, (unsigned)I.col);
        if (I.b < 0 || I.b > (int64_t)(1u << 24))
          return fail(&err, SEL_E_INVALID, "instruction %u: CODESET nbits %lld invalid", pc, (long long)I.b);
        const uint64_t nbits = (uint64_t)I.b, nwords = (nbits + 31) / 32;
        if (I.aux % 4 != 0 || (uint64_t)I.aux + 4 * nwords > pool_bytes)
          return fail(&err, SEL_E_INVALID, "instruction %u: code set at pool offset %u out of bounds or misaligned", pc, (unsigned)I.aux);
        std::vector<uint32_t> words(nwords);
        if (nwords) std::memcpy(words.data(), pool + I.aux, nwords * 4);
        if (nbits % 32) words.back() &= (1u << (nbits % 32)) - 1u;
        bool any = false;
        for (uint32_t w : words) any |= w != 0;
        id = any ? B.bitmap(I.col, 0, words, nbits) : B.nonnull_const(I.col, false);
        break;
      }
      case SEL_OP_IS_NULL:
      case SEL_OP_IS_NOT_NULL: {
        const bool isnull = op == SEL_OP_IS_NULL;
        if (!cols[I.col].nullable) {
          id = B.constant(!isnull);
        } else {
          Node nd;
          nd.ins.op = isnull ? D_ISNULL : D_NOTNULL;
          nd.ins.type = cols[I.col].type;
          nd.ins.valid = cols[I.col].valid;
          nd.col = I.col;
          id = B.add(nd);
        }
        break;
      }
      case SEL_OP_TRUE: id = B.constant(true); break;
      case SEL_OP_FALSE: id = B.constant(false); break;
      case SEL_OP_NOT:
      case SEL_OP_IS_UNKNOWN: {
        if (stack.empty()) return fail(&err, SEL_E_INVALID, "instruction %u: stack underflow", pc);
        const int x = stack.back();
        stack.pop_back();
        id = B.unary(op == SEL_OP_NOT ? Node::NOT : Node::ISUNK, x);
        break;
      }
      case SEL_OP_AND:
      case SEL_OP_OR: {
        if (stack.size() < 2) return fail(&err, SEL_E_INVALID, "instruction %u: stack underflow", pc);
        Node nd;
        nd.kind = op == SEL_OP_AND ? Node::AND : Node::OR;
        nd.b = stack.back();
        stack.pop_back();
        nd.a = stack.back();
        stack.pop_back();
        id = B.add(nd);
        break;
      }
      default:
        return fail(&err, SEL_E_INVALID, "instruction %u: unknown op %u", pc, (unsigned)op);
    }
    stack.push_back(id);
  }
  if (stack.size() != 1)
    return fail(&err, SEL_E_INVALID, "program leaves %u values on the stack (must be 1)", (unsigned)stack.size());
  const int root = merge_ranges ? merge_and_ranges(B, stack[0]) : stack[0];
  out.merged = B.merged;
  out.depth = compute_need(B.nodes, root);
  if (out.depth > SEL_MAX_DEPTH)
    return fail(&err, SEL_E_INVALID, "program needs a stack of depth %d (max 8)", out.depth);
  emit(B.nodes, root, out, 0);
  out.text = listing(out);
  return SEL_OK;
}

}  // namespace sel
