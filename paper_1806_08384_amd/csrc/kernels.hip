// kernels.hip -- gfx950 kernels of the exact-selectivity path.
//
//  k_scan<M_COUNT>      fused predicate evaluation + COUNT(*)   (Ch.3 sec.3.1)
//  k_scan<M_MASK>       same, also writing the per-row result mask and the
//                       per-tile TRUE counts that materialisation needs
//                       (Algorithm 1: count first, then materialise)
//  k_scan<M_KEYBITMAP>  same, setting bit (key - key_min) for every TRUE
//                       row of a pushed-down dimension (Ch.3 sec.3.3)
//  k_chunk_scan,        exclusive scan of the per-tile counts (two levels)
//  k_chunk_offsets
//  k_compact            mask -> ascending row ids (wave prefix by DPP,
//                       ballot + mbcnt; no LDS memory)
//  k_batch              many programs over several tables in one launch,
//                       one count per program
//
// Evaluation is bit-sliced: each lane owns 32 rows of a 2048-row wave tile
// (sel_device.h) and every truth value of SQL's three-valued logic is a pair
// of 32-bit words (t, f): bit set in t = TRUE, in f = FALSE, in neither =
// UNKNOWN.  Kleene AND is (t1 & t2, f1 | f2), OR is (t1 | t2, f1 & f2), NOT
// swaps the words.  The postfix program is wave-uniform, so its dispatch is
// scalar; only the leaf tests touch per-row data.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "sel_device.h"

using namespace sel;

typedef int32_t v2i __attribute__((ext_vector_type(2)));
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Pointers read from memory are generic to the compiler; casting them to
// the global (1) or constant (4) address space gives global_load / s_load
// instead of flat loads.
#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4)))
typedef const CONSTANT DevInstr* CInstr;

namespace {

template <class T>
__device__ __forceinline__ const GLOBAL T* gptr(const void* p) {
  return (const GLOBAL T*)p;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Bitmaps of the program staged in the workgroup's LDS: a leaf whose bitmap
// address is listed reads the copy (followed by a zero word) instead.
struct StageView {
  const CONSTANT BatchBitmap* list;
  uint32_t n;
  const uint32_t* lds;
};

// ---------------------------------------------------------------- loads --
// Raw storage of one lane's 32 rows of a column in a full tile.  All loads
// of a column are issued before any is used, so each lane keeps 32 rows of
// loads in flight; they are nontemporal (streamed once, not re-read).
// int64 columns are loaded in two halves of four steps (16 rows per lane),
// so one half's loads (8 x 16 B per lane) are in flight at a time.
template <int TY> struct Raw;
template <> struct Raw<T_I8> { uint32_t w[kSteps]; };
template <> struct Raw<T_I16> { v2i w[kSteps]; };
template <> struct Raw<T_I32> { v4i w[kSteps]; };
template <> struct Raw<T_I64> { v4i w[kSteps]; };

// A streamed load: nontemporal (NT, the default) or through the caches as
// usual; which one is faster is left to the tuner.
template <bool NT, class T>
__device__ __forceinline__ T ldg(const GLOBAL T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <int TY, bool NT = true>
__device__ __forceinline__ void load_full(Raw<TY>& r, const void* data, uint64_t tb, uint32_t lane) {
  if constexpr (TY == T_I8) {
    const GLOBAL uint32_t* p = gptr<uint32_t>((const int8_t*)data + tb) + lane;
#pragma unroll
    for (int j = 0; j < kSteps; ++j) r.w[j] = ldg<NT>(p + 64 * j);
  } else if constexpr (TY == T_I16) {
    const GLOBAL v2i* p = gptr<v2i>((const int16_t*)data + tb) + lane;
#pragma unroll
    for (int j = 0; j < kSteps; ++j) r.w[j] = ldg<NT>(p + 64 * j);
  } else if constexpr (TY == T_I32) {
    const GLOBAL v4i* p = gptr<v4i>((const int32_t*)data + tb) + lane;
#pragma unroll
    for (int j = 0; j < kSteps; ++j) r.w[j] = ldg<NT>(p + 64 * j);
  }
}

// one half (steps 4h .. 4h+3) of an int64 column
template <bool NT = true>
__device__ __forceinline__ void load_half64(Raw<T_I64>& r, const void* data, uint64_t tb,
                                            uint32_t lane, int h) {
  const GLOBAL v4i* p = gptr<v4i>((const int64_t*)data + tb) + 2 * lane + 128 * 4 * h;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    r.w[2 * j] = ldg<NT>(p + 128 * j);
    r.w[2 * j + 1] = ldg<NT>(p + 128 * j + 1);
  }
}

// value of row bit b (= 4*j + i) from the raw registers; b is a constant
// after unrolling.  Narrow types are sign-extended to int32.
template <int TY>
__device__ __forceinline__ auto get(const Raw<TY>& r, int b) {
  const int j = b >> 2, i = b & 3;
  if constexpr (TY == T_I8) {
    return (int32_t)(int8_t)(r.w[j] >> (8 * i));
  } else if constexpr (TY == T_I16) {
    return (int32_t)(int16_t)((uint32_t)r.w[j][i >> 1] >> (16 * (i & 1)));
  } else if constexpr (TY == T_I32) {
    return (int32_t)r.w[j][i];
  } else {  // b indexes the loaded half: 0..15
    const v4i& q = r.w[2 * j + (i >> 1)];
    const int k = 2 * (i & 1);
    return (int64_t)(((uint64_t)(uint32_t)q[k + 1] << 32) | (uint32_t)q[k]);
  }
}

template <int TY>
__device__ __forceinline__ auto load_elem(const void* data, uint64_t row) {
  if constexpr (TY == T_I8) return (int32_t)gptr<int8_t>(data)[row];
  else if constexpr (TY == T_I16) return (int32_t)gptr<int16_t>(data)[row];
  else if constexpr (TY == T_I32) return (int32_t)gptr<int32_t>(data)[row];
  else return (int64_t)gptr<int64_t>(data)[row];
}

__device__ __forceinline__ uint64_t row_of(uint64_t tb, uint32_t lane, int b) {
  return tb + 256u * (uint32_t)(b >> 2) + 4u * lane + (uint32_t)(b & 3);
}

// Predicate bits of one lane's 32 rows: bit b = pred(value of row b).  The
// word is built highest row first as P = 2P + bit, one add-with-carry per
// row after the compare.
template <int TY, bool FULL, bool NT = true, class Pred>
__device__ __forceinline__ uint32_t pred_bits(const void* data, uint64_t tb, uint32_t lane,
                                              uint64_t nrows, Pred pred) {
  uint32_t P = 0;
  if constexpr (FULL && TY == T_I64) {
#pragma unroll
    for (int h = 1; h >= 0; --h) {
      Raw<TY> r;
      load_half64<NT>(r, data, tb, lane, h);
#pragma unroll
      for (int b = 15; b >= 0; --b) P = (P << 1) + (uint32_t)pred(get<TY>(r, b), 16 * h + b);
    }
  } else if constexpr (FULL) {
    Raw<TY> r;
    load_full<TY, NT>(r, data, tb, lane);
#pragma unroll
    for (int b = 31; b >= 0; --b) P = (P << 1) + (uint32_t)pred(get<TY>(r, b), b);
  } else {
    // the one partial tile of a table: element loads, kept rolled
#pragma unroll 1
    for (int b = 31; b >= 0; --b) {
      const uint64_t row = row_of(tb, lane, b);
      uint32_t bit = 0;
      if (row < nrows) bit = (uint32_t)pred(load_elem<TY>(data, row), b);
      P = (P << 1) + bit;
    }
  }
  return P;
}

// Validity bits of the lane's rows (all ones for a column without NULLs).
template <bool FULL>
__device__ __forceinline__ uint32_t valid_bits(const uint32_t* valid, uint64_t tb, uint32_t lane,
                                               uint64_t nrows) {
  if (valid == nullptr) return ~0u;
  const GLOBAL uint32_t* vw = gptr<uint32_t>(valid) + tb / 32 + (lane >> 3);
  const uint32_t sh = 4 * (lane & 7);
  uint32_t V = 0;
#pragma unroll
  for (int j = 0; j < kSteps; ++j) {
    if (FULL || tb + 256u * j + 4u * lane < nrows)
      V |= ((vw[8 * j] >> sh) & 0xFu) << (4 * j);
  }
  return V;
}

__device__ __forceinline__ uint32_t inrange_bits(uint64_t tb, uint32_t lane, uint64_t nrows) {
  uint32_t m = 0;
#pragma unroll 1
  for (int b = 0; b < 32; ++b) m |= (uint32_t)(row_of(tb, lane, b) < nrows) << b;
  return m;
}

// Values of rows 8q .. 8q + 7 of the lane (steps 2q, 2q + 1), as int64:
// wide loads on a full tile as for a range test, element loads (0 past the
// table) on the partial one.
template <int TY, bool FULL, bool NT>
__device__ __forceinline__ void load8(const void* data, uint64_t tb, uint32_t lane, uint64_t nrows, int q,
                                      int64_t (&x)[8]) {
  if constexpr (FULL) {
#pragma unroll
    for (int js = 0; js < 2; ++js) {
      const int j = 2 * q + js;
      if constexpr (TY == T_I8) {
        const uint32_t w = ldg<NT>(gptr<uint32_t>((const int8_t*)data + tb) + lane + 64 * j);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * js + i] = (int64_t)(int8_t)(w >> (8 * i));
      } else if constexpr (TY == T_I16) {
        const v2i w = ldg<NT>(gptr<v2i>((const int16_t*)data + tb) + lane + 64 * j);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * js + i] = (int64_t)(int16_t)((uint32_t)w[i >> 1] >> (16 * (i & 1)));
      } else if constexpr (TY == T_I32) {
        const v4i w = ldg<NT>(gptr<v4i>((const int32_t*)data + tb) + lane + 64 * j);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * js + i] = (int64_t)w[i];
      } else {
        const GLOBAL v4i* p = gptr<v4i>((const int64_t*)data + tb) + 2 * lane + 128 * j;
        const v4i w0 = ldg<NT>(p), w1 = ldg<NT>(p + 1);
        x[4 * js + 0] = (int64_t)(((uint64_t)(uint32_t)w0[1] << 32) | (uint32_t)w0[0]);
        x[4 * js + 1] = (int64_t)(((uint64_t)(uint32_t)w0[3] << 32) | (uint32_t)w0[2]);
        x[4 * js + 2] = (int64_t)(((uint64_t)(uint32_t)w1[1] << 32) | (uint32_t)w1[0]);
        x[4 * js + 3] = (int64_t)(((uint64_t)(uint32_t)w1[3] << 32) | (uint32_t)w1[2]);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t row = row_of(tb, lane, 8 * q + k);
      x[k] = row < nrows ? (int64_t)load_elem<TY>(data, row) : 0;
    }
  }
}

// IN-list test of a lane's 32 rows against a sorted list of n values (in
// LDS or device memory): wide loads of the column as for a range test, then
// a branch-free lower bound that moves the eight rows of two steps one
// search step at a time, so that their list reads are in flight together.
template <int TY, bool FULL, bool NT = true, class List>
__device__ __forceinline__ uint32_t inlist_bits(const void* data, uint64_t tb, uint32_t lane,
                                                uint64_t nrows, List list, uint32_t n, uint32_t need) {
  uint32_t P = 0;
#pragma unroll 1
  for (int q = 3; q >= 0; --q) {   // bits 8q .. 8q + 7: steps 2q, 2q + 1
    int64_t x[8];
    load8<TY, FULL, NT>(data, tb, lane, nrows, q, x);
    uint32_t base[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) base[k] = 0;
    for (uint32_t len = n; len > 1;) {
      const uint32_t half = len >> 1;
#pragma unroll
      for (int k = 0; k < 8; ++k) base[k] = list[base[k] + half] <= x[k] ? base[k] + half : base[k];
      len -= half;
    }
#pragma unroll
    for (int k = 7; k >= 0; --k)
      P = (P << 1) + (uint32_t)(((need >> (8 * q + k)) & 1u) && list[base[k]] == x[k]);
  }
  return P;
}

// The same test through the list's two cuckoo tables of 2^b slots each (T
// then T + 2^b, in LDS or device memory): a value is in the list if and
// only if it sits in its slot of either table, so two reads per row answer
// it (empty slots hold a list value, which can only match a member).
template <int TY, bool FULL, bool NT = true, class Tab>
__device__ __forceinline__ uint32_t inhash_bits(const void* data, uint64_t tb, uint32_t lane, uint64_t nrows,
                                                Tab T, uint32_t b, uint32_t c1, uint32_t c2, uint32_t need) {
  const uint32_t m = 1u << b;
  uint32_t P = 0;
#pragma unroll 1
  for (int q = 3; q >= 0; --q) {
    int64_t x[8];
    load8<TY, FULL, NT>(data, tb, lane, nrows, q, x);
#pragma unroll
    for (int k = 7; k >= 0; --k) {
      const bool hit = T[in_hash(x[k], c1, b)] == x[k] || T[m + in_hash(x[k], c2, b)] == x[k];
      P = (P << 1) + (uint32_t)(((need >> (8 * q + k)) & 1u) && hit);
    }
  }
  return P;
}

// ---------------------------------------------------------------- leaves --
// SCAN: called by the scan kernels, whose leaves carry DevFlags (a batch's
// copies of the leaves reuse the flags word for their own guard marks, and
// read an IN list through its sorted values only).
template <int TY, bool FULL, bool NT = true, bool SCAN = true>
__device__ __forceinline__ uint32_t leaf_pred(uint32_t op, CInstr I, uint64_t tb, uint32_t lane,
                                              uint64_t nrows, uint32_t need, const StageView& sv) {
  const void* data = I->data;
  const int64_t lo = I->lo;
  const uint64_t span = I->span;
  if (op == D_INLIST) {
    const uint32_t f = I->flags;
    if (SCAN && (f & F_HASHED)) {
      // the cuckoo tables after the sorted list: their LDS copy if staged
      const uint32_t b = in_hash_bits(f), c1 = kInHashMul[in_hash_pair(f)][0], c2 = kInHashMul[in_hash_pair(f)][1];
      const uint32_t* tabs = (const uint32_t*)I->aux + 2 * I->n;
      for (uint32_t k = 0; k < sv.n; ++k)
        if (sv.list[k].src == tabs)
          return inhash_bits<TY, FULL, NT>(data, tb, lane, nrows, (const int64_t*)(sv.lds + sv.list[k].lds_word),
                                           b, c1, c2, need);
      return inhash_bits<TY, FULL, NT>(data, tb, lane, nrows, gptr<int64_t>(tabs), b, c1, c2, need);
    }
    // the list's LDS copy if the scan staged it
    for (uint32_t k = 0; k < sv.n; ++k)
      if (sv.list[k].src == (const uint32_t*)I->aux)
        return inlist_bits<TY, FULL, NT>(data, tb, lane, nrows, (const int64_t*)(sv.lds + sv.list[k].lds_word),
                                     I->n, need);
    return inlist_bits<TY, FULL, NT>(data, tb, lane, nrows, gptr<int64_t>(I->aux), I->n, need);
  }
  if (op == D_BITMAP && sv.n) {
    uint32_t off = kNoLds, z = 0;
    for (uint32_t k = 0; k < sv.n; ++k) {
      if (sv.list[k].src == (const uint32_t*)I->aux) {
        off = sv.list[k].lds_word;
        z = sv.list[k].words * 32;
        break;
      }
    }
    if (off != kNoLds) {
      // an offset outside the window, or a row the guard skips, reads the
      // zero bit z after the copy; for narrow columns the window lies inside
      // int32 (the host stages only such bitmaps)
      const uint32_t* bm = sv.lds + off;
      if constexpr (TY == T_I64) {
        return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int64_t x, int b) -> uint32_t {
          const uint64_t d = (uint64_t)x - (uint64_t)lo;
          const uint32_t k = ((need >> b) & 1u) && d < z ? (uint32_t)d : z;
          return (bm[k >> 5] >> (k & 31)) & 1u;
        });
      } else {
        const uint32_t lo32 = (uint32_t)lo;
        return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int32_t x, int b) -> uint32_t {
          const uint32_t d = (uint32_t)x - lo32;
          const uint32_t k = ((need >> b) & 1u) && d < z ? d : z;
          return (bm[k >> 5] >> (k & 31)) & 1u;
        });
      }
    }
  }
  if (op == D_RANGE) {
    if constexpr (TY == T_I64) {
      return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int64_t x, int) {
        return (uint64_t)x - (uint64_t)lo <= span;
      });
    } else {
      const uint32_t lo32 = (uint32_t)lo, span32 = (uint32_t)span;
      return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int32_t x, int) {
        return (uint32_t)x - lo32 <= span32;
      });
    }
  } else if (op == D_BITMAP) {
    // rows that need no test (guard) or fall outside [lo, lo + nbits) read
    // word 0 and are masked: no branch, so all 32 lookups issue together
    const GLOBAL uint32_t* bits = gptr<uint32_t>(I->aux);
    if constexpr (TY == T_I64) {
      return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int64_t x, int b) -> uint32_t {
        const uint64_t d = (uint64_t)x - (uint64_t)lo;
        const bool ok = d < span && ((need >> b) & 1u);
        const uint32_t k = ok ? (uint32_t)d : 0u;  // nbits <= 2^32
        return ok & ((bits[k >> 5] >> (k & 31)) & 1u);
      });
    } else {
      // x - lo in 64 bits: a negative key must not alias a bit when nbits
      // exceeds 2^31
      return pred_bits<TY, FULL, NT>(data, tb, lane, nrows, [=](int32_t x, int b) -> uint32_t {
        const uint64_t d = (uint64_t)((int64_t)x - lo);
        const bool ok = d < span && ((need >> b) & 1u);
        const uint32_t k = ok ? (uint32_t)d : 0u;
        return ok & ((bits[k >> 5] >> (k & 31)) & 1u);
      });
    }
  } else {  // D_INLIST, handled above
    return 0u;
  }
}

template <bool FULL, bool NT = true>
__device__ __forceinline__ void eval_leaf(uint32_t op, CInstr I, uint64_t tb, uint32_t lane,
                                          uint64_t nrows, uint32_t tos_t, uint32_t tos_f,
                                          uint32_t& t, uint32_t& f, const StageView& sv) {
  const uint32_t* valid = I->valid;
  const uint32_t V = valid_bits<FULL>(valid, tb, lane, nrows);
  if (op >= D_NN_TRUE) {
    switch (op) {
      case D_NN_TRUE: t = V; f = 0; return;
      case D_NN_FALSE: t = 0; f = V; return;
      case D_ISNULL: t = ~V; f = V; return;
      default: t = V; f = ~V; return;  // D_NOTNULL
    }
  }
  const uint32_t flags = I->flags;
  uint32_t need = ~0u;
  if (flags & F_GUARD_AND) need = ~tos_f;
  else if (flags & F_GUARD_OR) need = ~tos_t;
  uint32_t P;
  switch (I->type) {
    case T_I8: P = leaf_pred<T_I8, FULL, NT>(op, I, tb, lane, nrows, need, sv); break;
    case T_I16: P = leaf_pred<T_I16, FULL, NT>(op, I, tb, lane, nrows, need, sv); break;
    case T_I32: P = leaf_pred<T_I32, FULL, NT>(op, I, tb, lane, nrows, need, sv); break;
    default: P = leaf_pred<T_I64, FULL, NT>(op, I, tb, lane, nrows, need, sv); break;
  }
  t = P & V;
  f = ~P & V;
}

// ---------------------------------------------------------- interpreter --
// The stack below the top is held in registers; its index is uniform, so
// the unrolled selects below compile to scalar branches / v_cndmask and no
// private memory is used.
__device__ __forceinline__ void spill(uint32_t (&st)[kMaxDepth], uint32_t (&sf)[kMaxDepth],
                                      int idx, uint32_t t, uint32_t f) {
#pragma unroll
  for (int k = 0; k < kMaxDepth; ++k)
    if (k == idx) { st[k] = t; sf[k] = f; }
}
__device__ __forceinline__ void fill(const uint32_t (&st)[kMaxDepth], const uint32_t (&sf)[kMaxDepth],
                                     int idx, uint32_t& t, uint32_t& f) {
  t = 0; f = 0;
#pragma unroll
  for (int k = 0; k < kMaxDepth; ++k)
    if (k == idx) { t = st[k]; f = sf[k]; }
}

// TRUE bits of the lane's 32 rows of the tile starting at row tb.
template <bool FULL, bool NT = true>
__device__ __forceinline__ uint32_t eval_tile(CInstr prog, uint32_t nins, uint64_t tb,
                                              uint32_t lane, uint64_t nrows, const StageView& sv) {
  uint32_t st[kMaxDepth], sf[kMaxDepth];
  uint32_t tt = 0, tf = 0;
  int d = 0;  // values on the stack; the top is (tt, tf)
  for (uint32_t pc = 0; pc < nins; ++pc) {
    CInstr I = prog + pc;
    const uint32_t op = I->op;
    if (op < D_AND || op == D_TRUE || op == D_FALSE) {
      uint32_t t, f;
      if (op == D_TRUE) { t = ~0u; f = 0; }
      else if (op == D_FALSE) { t = 0; f = ~0u; }
      else eval_leaf<FULL, NT>(op, I, tb, lane, nrows, tt, tf, t, f, sv);
      spill(st, sf, d - 1, tt, tf);
      tt = t; tf = f;
      ++d;
    } else if (op == D_NOT) {
      const uint32_t x = tt; tt = tf; tf = x;
    } else if (op == D_ISUNK) {
      const uint32_t k = tt | tf; tt = ~k; tf = k;
    } else {
      uint32_t at, af;
      fill(st, sf, d - 2, at, af);
      if (op == D_AND) { tt &= at; tf |= af; }
      else { tt |= at; tf &= af; }
      --d;
    }
  }
  return tt;
}

// ------------------------------------------------------------ reductions --
// Wait until this thread's earlier memory operations, atomics included,
// have completed.  The end-of-launch ticket hand-offs below need no more:
// what one workgroup passes to the last one travels only through
// device-scope atomics, which are coherent by themselves, so the cache
// write-back and invalidation of a device-scope fence (issued by every
// workgroup, tens of microseconds at the end of a short scan) are not
// needed.  Plain stores (results, masks) are read after the launch.
__device__ __forceinline__ void atomics_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Sum over the 64 lanes: DPP within quads and 16-lane rows, then the four
// row sums by readlane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);  // row_ror:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// Block sum, one device atomic per workgroup, and the last workgroup (by
// ticket) publishes the total and resets the slot for the next launch.
__device__ void finish(DevSlot* slot, unsigned long long* out, uint32_t c0, uint32_t c1, bool two) {
  __shared__ unsigned long long red0[16], red1[16];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t s0 = wave_sum(c0);
  const uint32_t s1 = two ? wave_sum(c1) : 0u;
  if (lane == 0) { red0[wave] = s0; red1[wave] = s1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b0 = 0, b1 = 0;
    for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) { b0 += red0[w]; b1 += red1[w]; }
    if (b0) atomicAdd(&slot->acc, b0);
    if (b1) atomicAdd(&slot->acc2, b1);
    atomics_done();
    const unsigned int ticket = atomicAdd(&slot->ticket, 1u);
    if (ticket == gridDim.x - 1) {
      out[0] = atomicAdd(&slot->acc, 0ull);
      if (two) out[1] = atomicAdd(&slot->acc2, 0ull);
      atomicExch(&slot->acc, 0ull);
      atomicExch(&slot->acc2, 0ull);
      atomics_done();
      atomicExch(&slot->ticket, 0u);
    }
  }
}

template <int MODE, bool NT>
__global__ void __launch_bounds__(256) k_scan(const DevInstr* __restrict__ prog_, ScanArgs a) {
  CInstr prog = (CInstr)prog_;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t W = (uint64_t)gridDim.x * nw;
  extern __shared__ __align__(16) uint32_t sbm[];
  const StageView sv{(const CONSTANT BatchBitmap*)a.stage, a.nstage, sbm};
  if (a.nstage) {
    // the program's small bitmaps, each followed by a zero word
    for (uint32_t k = 0; k < a.nstage; ++k) {
      const CONSTANT BatchBitmap* B = sv.list + k;
      const uint32_t n = B->words, last = B->last_mask;
      const GLOBAL uint32_t* src = gptr<uint32_t>(B->src);
      uint32_t* dst = sbm + B->lds_word;
      for (uint32_t i = threadIdx.x; i <= n; i += blockDim.x) {
        uint32_t w = 0;
        if (i < n) w = i + 1 == n ? src[i] & last : src[i];
        dst[i] = w;
      }
    }
    __syncthreads();
  }
  uint32_t cnt = 0, oor = 0;
  // M_MASK: result words of the last 8 tiles, written together with
  // nontemporal stores (fewer, fuller store bursts interleaved with the
  // loads).  Only words holding a TRUE row are written, packed at the front
  // of their tile's slot: at low selectivity most words are zero, and the
  // writes, not their bytes' share of the traffic, slow the scan.
  uint32_t pend[8];
  uint64_t pidx[8];
  int np = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) { pend[k] = 0; pidx[k] = 0; }
  // each wave takes runs of tps consecutive tiles, W runs apart
  const uint64_t tps = a.tiles_per_step ? a.tiles_per_step : 1;
  const uint64_t wid = uni64((uint64_t)blockIdx.x * nw + (threadIdx.x >> 6));
  for (uint64_t step = wid * tps; step < a.ntiles; step += W * tps)
  for (uint64_t tile = step; tile < step + tps && tile < a.ntiles; ++tile) {
    const uint64_t tb = tile * kTileRows;
    uint32_t T;
    if (tb + kTileRows <= a.nrows) {
      T = eval_tile<true, NT>(prog, a.nins, tb, lane, a.nrows, sv);
    } else {
      T = eval_tile<false, NT>(prog, a.nins, tb, lane, a.nrows, sv) & inrange_bits(tb, lane, a.nrows);
    }
    cnt += __builtin_popcount(T);
    if constexpr (MODE == M_MASK) {
      // lanes with a TRUE row; a lane's word goes to the rank of its lane
      // among them
      const uint64_t nz = __ballot(T != 0u);
      const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(nz >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)nz, 0u));
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k == np) { pend[k] = T; pidx[k] = tile * kWave + pos; }
      ++np;
      if (np == 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (pend[k]) __builtin_nontemporal_store(pend[k], &a.mask[pidx[k]]);
        np = 0;
      }
      const uint32_t tc = wave_sum(__builtin_popcount(T));
      if (lane == 0) {
        a.tile_counts[tile] = tc;
        a.tile_lanes[tile] = nz;
      }
    } else if constexpr (MODE == M_KEYBITMAP) {
      uint32_t m = T;
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1;
        const uint64_t row = row_of(tb, lane, b);
        const int64_t key = a.key_type == T_I64 ? ((const int64_t*)a.key_data)[row]
                                                : (int64_t)((const int32_t*)a.key_data)[row];
        const uint64_t d = (uint64_t)key - (uint64_t)a.key_min;
        if (d < a.nbits) atomicOr(&a.bitmap[d >> 5], 1u << (d & 31));
        else ++oor;
      }
    }
  }
  if constexpr (MODE == M_MASK) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < np && pend[k]) __builtin_nontemporal_store(pend[k], &a.mask[pidx[k]]);
  }
  finish(a.slot, a.out, cnt, oor, MODE == M_KEYBITMAP);
}

// Exclusive scan of the tile counts in two levels.  k_chunk_scan: one
// workgroup of 1024 threads per chunk of 1024 tiles writes each tile's
// offset within its chunk and the chunk's total.  k_chunk_offsets: one
// workgroup scans the chunk totals (at most 2048 for 2^32 rows).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += y;
  }
  return x;
}

// exclusive prefix of v over the (up to 1024) threads of the block
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v) {
  __shared__ uint32_t wsum[16];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v, lane);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t w = lane < nw ? wsum[lane] : 0u;
    const uint32_t wi = wave_incl_scan(w, lane);
    if (lane < nw) wsum[lane] = wi - w;
  }
  __syncthreads();
  return wsum[wave] + inc - v;
}

__global__ void __launch_bounds__(1024) k_chunk_scan(const uint32_t* __restrict__ counts,
                                                     uint32_t* __restrict__ offsets,
                                                     uint32_t* __restrict__ chunk_sums, uint64_t n) {
  __shared__ uint32_t tot;
  const uint64_t i = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
  const uint32_t v = i < n ? counts[i] : 0u;
  const uint32_t ex = block_excl_scan(v);
  if (i < n) offsets[i] = ex;
  if (threadIdx.x == 1023) tot = ex + v;
  __syncthreads();
  if (threadIdx.x == 0) chunk_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_chunk_offsets(const uint32_t* __restrict__ chunk_sums,
                                                        uint32_t* __restrict__ chunk_offs,
                                                        uint64_t nchunks) {
  // two chunks per thread: up to 2048 chunks
  const uint64_t i0 = 2 * (uint64_t)threadIdx.x, i1 = i0 + 1;
  const uint32_t a = i0 < nchunks ? chunk_sums[i0] : 0u;
  const uint32_t b = i1 < nchunks ? chunk_sums[i1] : 0u;
  const uint32_t ex = block_excl_scan(a + b);
  if (i0 < nchunks) chunk_offs[i0] = ex;
  if (i1 < nchunks) chunk_offs[i1] = ex + a;
}

// Row ids of TRUE rows in ascending order: rows are ordered (step j, lane,
// i), so a row's rank is the tile offset + TRUE rows of earlier steps +
// TRUE rows of this step in lower lanes (ballot per bit plane, mbcnt) +
// TRUE rows earlier in the lane's own nibble.  Each wave takes kCompactTiles
// consecutive tiles and issues all their loads before using any.
constexpr int kCompactTiles = 4;

// Inclusive sum over the 64 lanes: DPP shifts within each 16-lane row, then
// the row totals by readlane.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x, uint32_t lane, uint32_t& total) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
  const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
  total = r0 + r1 + r2 + r3;
  const uint32_t row = lane >> 4;
  return x + (row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r0 + r1 : r0 + r1 + r2);
}

// A row's rank in the tile is: TRUE rows of earlier steps + TRUE rows of this
// step in lower lanes + TRUE rows before it in the lane's own nibble.  The
// per-lane counts of the 8 steps are packed two to a word (16-bit fields; a
// step holds at most 256 TRUE rows) and prefix-summed over the lanes four
// words at a time.
__device__ __forceinline__ void compact_tile(uint32_t w, uint64_t base, uint64_t tile,
                                             uint32_t lane, uint32_t* __restrict__ out,
                                             uint64_t cap) {
  const uint64_t tb = tile * kTileRows;
  uint32_t excl[4], tot[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = __builtin_popcount((w >> (8 * q)) & 0xFu);
    const uint32_t hi = __builtin_popcount((w >> (8 * q + 4)) & 0xFu);
    const uint32_t packed = lo | (hi << 16);
    excl[q] = wave_incl_sum(packed, lane, tot[q]) - packed;
  }
  if (__ballot(__builtin_popcount(w) > 2u) == 0ull) {
    // sparse tile (at most two TRUE rows per lane): each lane walks its own
    // set bits.  Field j of the packed words becomes the rank of step j's
    // first TRUE row of this lane: TRUE rows of earlier steps (uniform)
    // plus those of step j in lower lanes (at most 2048 < 2^16, so the two
    // fields of a word stay apart)
    uint32_t first[4];
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t t0 = tot[q] & 0xFFFFu, t1 = tot[q] >> 16;
      first[q] = excl[q] + (run | ((run + t0) << 16));
      run += t0 + t1;
    }
    uint32_t prev = ~0u;   // step of the lane's first TRUE row
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      if (w != 0u) {
        const uint32_t b = __builtin_ctz(w);
        const uint32_t j = b >> 2;
        const uint32_t q = j >> 1;
        const uint32_t word = q & 2u ? (q & 1u ? first[3] : first[2]) : (q & 1u ? first[1] : first[0]);
        // plus one if the lane's first TRUE row is earlier in this nibble
        const uint64_t p = base + ((word >> (16u * (j & 1u))) & 0xFFFFu) + (j == prev ? 1u : 0u);
        if (p < cap) out[p] = (uint32_t)(tb + 256u * j + 4u * lane + (b & 3u));
        prev = j;
        w &= w - 1u;
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < kSteps; ++j) {
    const uint32_t nib = (w >> (4 * j)) & 0xFu;
    const uint32_t sh = 16 * (j & 1);
    const uint32_t below = (excl[j >> 1] >> sh) & 0xFFFFu;
    const uint32_t total = (tot[j >> 1] >> sh) & 0xFFFFu;
    if (nib) {
      const uint64_t pos = base + below;
      const uint32_t id = (uint32_t)(tb + 256u * j + 4u * lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if ((nib >> i) & 1u) {
          const uint64_t p = pos + __builtin_popcount(nib & ((1u << i) - 1u));
          if (p < cap) out[p] = id + i;
        }
      }
    }
    base += total;
  }
}

__global__ void __launch_bounds__(256) k_compact(CompactArgs a) {
  // the limit check of Algorithm 1 on the device: an empty or over-limit
  // selection writes no id, so the host learns the outcome with one wait
  const uint64_t total = *a.total;
  if (total == 0 || total > a.limit) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t step = (uint64_t)gridDim.x * nw * kCompactTiles;
  for (uint64_t t0 = uni64(((uint64_t)blockIdx.x * nw + (threadIdx.x >> 6)) * kCompactTiles);
       t0 < a.ntiles; t0 += step) {
    uint32_t raw[kCompactTiles];
    uint32_t off[kCompactTiles], coff[kCompactTiles];
    uint64_t nz[kCompactTiles];
#pragma unroll
    for (int k = 0; k < kCompactTiles; ++k) {
      const uint64_t tile = t0 + k;
      const bool in = tile < a.ntiles;
      // the lanes whose word the mask pass wrote; and the tile's packed
      // words read whole, one per lane (coalesced, and not waiting for the
      // lane map: the words past the packed ones are not used)
      nz[k] = in ? uni64(a.tile_lanes[tile]) : 0ull;
      raw[k] = in ? a.mask[tile * kWave + lane] : 0u;
      off[k] = in ? a.offsets[tile] : 0u;
      coff[k] = in ? a.chunk_offs[tile >> 10] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kCompactTiles; ++k) {
      if (nz[k] == 0ull) continue;  // no TRUE row in the tile
      // a set lane's word is packed at its rank among the set lanes
      const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(nz[k] >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)nz[k], 0u));
      const uint32_t mine = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(pos << 2), (int)raw[k]);
      const uint32_t w = (nz[k] >> lane) & 1u ? mine : 0u;
      compact_tile(w, (uint64_t)uni(coff[k]) + uni(off[k]), t0 + k, lane, a.out, a.cap);
    }
  }
}

// ---------------------------------------------------- projected columns --
// Materialised sigma(R) with its projected columns (Ch.3 sec.3.3): each wave
// takes kGatherUnroll x 64 consecutive outputs, loads all their row ids
// first (coalesced; ascending ids make neighbouring lanes read neighbouring
// rows), then per column issues every gather before any store; the validity
// bits of each 64 outputs are one ballot, written as two words.  An id past
// the table's rows gives 0 and NULL and is counted.
constexpr int kGatherUnroll = 4;

template <class T>
__device__ __forceinline__ void gather_col(const GatherCol& C, uint64_t base, uint32_t lane,
                                           const uint32_t (&row)[kGatherUnroll],
                                           const bool (&in)[kGatherUnroll],
                                           const bool (&ok)[kGatherUnroll]) {
  const GLOBAL T* src = gptr<T>(C.src);
  T v[kGatherUnroll];
#pragma unroll
  for (int j = 0; j < kGatherUnroll; ++j) v[j] = ok[j] ? src[row[j]] : (T)0;
#pragma unroll
  for (int j = 0; j < kGatherUnroll; ++j)
    if (in[j]) ((T*)C.out)[base + 64 * j + lane] = v[j];
}

__global__ void __launch_bounds__(256) k_gather(GatherArgs a) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kGatherUnroll;
  uint32_t bad = 0;
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u)) * kGatherUnroll;
       base < a.count; base += stride) {
    uint32_t row[kGatherUnroll];
    bool in[kGatherUnroll], ok[kGatherUnroll];
#pragma unroll
    for (int j = 0; j < kGatherUnroll; ++j) {
      const uint64_t k = base + 64 * j + lane;
      in[j] = k < a.count;
      row[j] = in[j] ? __builtin_nontemporal_load(gptr<uint32_t>(a.ids) + k) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kGatherUnroll; ++j) {
      ok[j] = in[j] && row[j] < a.nrows;
      bad += (in[j] && !ok[j]) ? 1u : 0u;
    }
    for (uint32_t c = 0; c < a.ncols; ++c) {
      const GatherCol& C = a.cols[c];
      switch (C.width) {
        case 1: gather_col<uint8_t>(C, base, lane, row, in, ok); break;
        case 2: gather_col<uint16_t>(C, base, lane, row, in, ok); break;
        case 4: gather_col<uint32_t>(C, base, lane, row, in, ok); break;
        default: gather_col<uint64_t>(C, base, lane, row, in, ok); break;
      }
      if (C.out_valid) {
        uint32_t vw[kGatherUnroll];
#pragma unroll
        for (int j = 0; j < kGatherUnroll; ++j)
          vw[j] = ok[j] && C.valid != nullptr ? gptr<uint32_t>(C.valid)[row[j] >> 5] : ~0u;
#pragma unroll
        for (int j = 0; j < kGatherUnroll; ++j) {
          const bool v = ok[j] && ((vw[j] >> (row[j] & 31)) & 1u);
          const uint64_t m = __ballot(v);
          const uint64_t w = (base + 64 * j) >> 5;
          if (lane == 0 && in[j]) C.out_valid[w] = (uint32_t)m;
          if (lane == 32 && in[j]) C.out_valid[w + 1] = (uint32_t)(m >> 32);
        }
      }
    }
  }
  finish(a.slot, a.out, 0u, bad, true);
}

// --------------------------------------------------------- batched count --
// Column values of one pipeline segment: a full tile of a narrow column or
// half a tile of an int64 column, 128 B per lane at most.  Narrow types use
// the leading components of each step's vector.
struct Seg { v4i w[kSteps]; };

template <int TY>
__device__ __forceinline__ auto seg_get(const Seg& r, int b) {
  const int j = b >> 2, i = b & 3;
  if constexpr (TY == T_I8) {
    return (int32_t)(int8_t)((uint32_t)r.w[j][0] >> (8 * i));
  } else if constexpr (TY == T_I16) {
    return (int32_t)(int16_t)((uint32_t)r.w[j][i >> 1] >> (16 * (i & 1)));
  } else if constexpr (TY == T_I32) {
    return (int32_t)r.w[j][i];
  } else {  // b indexes the loaded half: 0..15
    const v4i& q = r.w[2 * j + (i >> 1)];
    const int k = 2 * (i & 1);
    return (int64_t)(((uint64_t)(uint32_t)q[k + 1] << 32) | (uint32_t)q[k]);
  }
}

// Issue the loads of a segment (and, with a column's first segment, of its
// validity word); nothing waits for them here.
__device__ __forceinline__ void seg_issue(Seg& r, uint32_t& V, const CONSTANT BatchCol* C, int h,
                                          uint64_t tb, uint32_t lane) {
  const void* data = C->data;
  switch (C->type) {
    case T_I8: {
      const GLOBAL uint32_t* p = gptr<uint32_t>((const int8_t*)data + tb) + lane;
#pragma unroll
      for (int j = 0; j < kSteps; ++j) r.w[j][0] = (int32_t)__builtin_nontemporal_load(p + 64 * j);
      break;
    }
    case T_I16: {
      const GLOBAL v2i* p = gptr<v2i>((const int16_t*)data + tb) + lane;
#pragma unroll
      for (int j = 0; j < kSteps; ++j) {
        const v2i x = __builtin_nontemporal_load(p + 64 * j);
        r.w[j][0] = x[0];
        r.w[j][1] = x[1];
      }
      break;
    }
    case T_I32: {
      const GLOBAL v4i* p = gptr<v4i>((const int32_t*)data + tb) + lane;
#pragma unroll
      for (int j = 0; j < kSteps; ++j) r.w[j] = __builtin_nontemporal_load(p + 64 * j);
      break;
    }
    default: {  // int64: h = 0 loads steps 4..7 (bits 16..31), h = 1 steps 0..3
      const GLOBAL v4i* p = gptr<v4i>((const int64_t*)data + tb) + 2 * lane + 128 * 4 * (1 - h);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r.w[2 * j] = __builtin_nontemporal_load(p + 128 * j);
        r.w[2 * j + 1] = __builtin_nontemporal_load(p + 128 * j + 1);
      }
      break;
    }
  }
  if (h == 0 && C->vslot != kNoSlot) V = valid_bits<true>(C->valid, tb, lane, tb + kTileRows);
}

// Rows a direct factor of a conjunction still needs tested: those its
// program's accumulator still holds TRUE.
__device__ __forceinline__ uint32_t acc_need(uint32_t sl, const uint32_t* wl, uint32_t lane) {
  return wl[(sl & 0xFFFu) * kWave + lane];
}

// Validity word of a leaf's column (all ones without NULLs).
__device__ __forceinline__ uint32_t leaf_valid(uint32_t sl, const uint32_t* wl, uint32_t lane) {
  const uint32_t vs = (sl >> 24) & 0x7Fu;
  return vs == kAccNoValid ? ~0u : wl[vs * kWave + lane];
}

// Stores a leaf's TRUE word (its test on non-NULL rows): into its slot, or
// for a direct factor of a conjunction ANDed into its program's accumulator,
// or for a leaf of an OR factor of narrow tests ORed into that factor's word.
__device__ __forceinline__ void put_leaf(uint32_t* wl, uint32_t lane, uint32_t sl, uint32_t P) {
  const uint32_t T = P & leaf_valid(sl, wl, lane);
  uint32_t* w = wl + (sl & 0xFFFu) * kWave + lane;
  if (!(sl & kAccTarget)) *w = T;
  else if (sl & kAccOr) *w |= T;
  else *w &= T;
}

// Resets the accumulators of an entry's programs for a new tile.
__device__ __forceinline__ void reset_acc(const CONSTANT BatchTable* E, const CONSTANT uint32_t* ops,
                                          uint32_t* wl, uint32_t lane) {
  const uint32_t ib = E->init_begin, in = E->init_count;
  for (uint32_t k = 0; k < in; ++k) {
    const uint32_t w = ops[ib + k];
    wl[(w & 0xFFFu) * kWave + lane] = (w & kInitTrue) ? ~0u : 0u;
  }
}

// Value tests of one leaf on a segment: bits [0, nb) of the result, highest
// row first.  A bitmap leaf in global memory that is a direct factor of a
// conjunction looks up only rows its program's accumulator does not hold
// FALSE; the others read word 0 and test FALSE.  `gshift` places the
// segment's rows in the guard word (16 for the upper half of an int64
// column).
template <int TY>
__device__ __forceinline__ uint32_t seg_leaf(const Seg& r, uint32_t op, CInstr I,
                                             const uint32_t* bmlds, const uint32_t* wl,
                                             uint32_t lane, int gshift) {
  constexpr int nb = TY == T_I64 ? 16 : 32;
  const int64_t lo = I->lo;
  const uint64_t span = I->span;
  uint32_t P = 0;
  if (op == D_BITMAP && I->lds_word != kNoLds) {
    // staged copy: an offset past the window is clamped to the zero bit z
    // that follows the copied words, so no test or select is needed.  For
    // narrow columns the window lies inside int32 (the host stages only
    // such bitmaps), so 32-bit differences are exact.
    const uint32_t* bm = bmlds + I->lds_word;
    const uint32_t z = I->n;
    if constexpr (TY == T_I64) {
#pragma unroll
      for (int b = nb - 1; b >= 0; --b) {
        const uint64_t d = (uint64_t)seg_get<TY>(r, b) - (uint64_t)lo;
        const uint32_t k = d < z ? (uint32_t)d : z;
        P = (P << 1) + ((bm[k >> 5] >> (k & 31)) & 1u);
      }
    } else {
      // eight rows at a time: their LDS reads are all issued before the
      // first bit is taken, so one wait covers eight round trips
      const uint32_t lo32 = (uint32_t)lo;
#pragma unroll
      for (int g = nb - 8; g >= 0; g -= 8) {
        uint32_t k[8], w[8];
#pragma unroll
        for (int q = 7; q >= 0; --q) {
          const uint32_t d = (uint32_t)seg_get<TY>(r, g + q) - lo32;
          k[q] = d < z ? d : z;
        }
#pragma unroll
        for (int q = 7; q >= 0; --q) w[q] = bm[k[q] >> 5];
#pragma unroll
        for (int q = 7; q >= 0; --q) P = (P << 1) + ((w[q] >> (k[q] & 31)) & 1u);
      }
    }
  } else if (op == D_RANGE) {
    if constexpr (TY == T_I64) {
      // one-sided ranges (x >= lo, x <= hi) need one compare per row
      if ((uint64_t)lo + span == (uint64_t)INT64_MAX) {
#pragma unroll
        for (int b = nb - 1; b >= 0; --b) P = (P << 1) + (uint32_t)(seg_get<TY>(r, b) >= lo);
      } else if (lo == INT64_MIN) {
        const int64_t hi = (int64_t)((uint64_t)lo + span);
#pragma unroll
        for (int b = nb - 1; b >= 0; --b) P = (P << 1) + (uint32_t)(seg_get<TY>(r, b) <= hi);
      } else {
#pragma unroll
        for (int b = nb - 1; b >= 0; --b)
          P = (P << 1) + (uint32_t)((uint64_t)seg_get<TY>(r, b) - (uint64_t)lo <= span);
      }
    } else {
      const uint32_t lo32 = (uint32_t)lo, span32 = (uint32_t)span;
#pragma unroll
      for (int b = nb - 1; b >= 0; --b)
        P = (P << 1) + (uint32_t)((uint32_t)seg_get<TY>(r, b) - lo32 <= span32);
    }
  } else {  // D_BITMAP in global memory
    const GLOBAL uint32_t* bits = gptr<uint32_t>(I->aux);
    uint32_t need = ~0u;
    if (I->flags == kAccGuard) need = acc_need(I->slot, wl, lane) >> gshift;
#pragma unroll
    for (int b = nb - 1; b >= 0; --b) {
      uint64_t d;
      if constexpr (TY == T_I64) d = (uint64_t)seg_get<TY>(r, b) - (uint64_t)lo;
      else d = (uint64_t)((int64_t)seg_get<TY>(r, b) - lo);
      const bool ok = d < span && ((need >> b) & 1u);
      const uint32_t k = ok ? (uint32_t)d : 0u;
      P = (P << 1) + (ok & ((bits[k >> 5] >> (k & 31)) & 1u));
    }
  }
  return P;
}

// In-register transpose of a 32 x 32 bit matrix: on return a[c] bit r is
// what a[r] bit c was.  Each stage swaps, in every 2s x 2s block, the s x s
// block above the diagonal with the one below it.
// Only words 0 .. NOUT-1 of the result are wanted: later stages mix words
// within blocks of S, so a stage updates only the words below
// ceil(NOUT / S) * S.
template <int S, int NOUT>
__device__ __forceinline__ void transpose_stage(uint32_t (&a)[32], uint32_t m) {
  constexpr int R = (NOUT + S - 1) / S * S;
#pragma unroll
  for (int g = 0; g < 32; g += 2 * S) {
#pragma unroll
    for (int k = g; k < g + S; ++k) {
      if (k >= R) continue;
      const uint32_t t = ((a[k] >> S) ^ a[k + S]) & m;
      if (k + S < R) a[k + S] ^= t;
      a[k] ^= t << S;
    }
  }
}

template <int NOUT>
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
  transpose_stage<16, NOUT>(a, 0x0000FFFFu);
  transpose_stage<8, NOUT>(a, 0x00FF00FFu);
  transpose_stage<4, NOUT>(a, 0x0F0F0F0Fu);
  transpose_stage<2, NOUT>(a, 0x33333333u);
  transpose_stage<1, NOUT>(a, 0x55555555u);
}

// The table leaves of a narrow column on one segment: one lookup per row
// (entries of E: one bit per leaf, NOUT >= the leaf count) serves them all;
// transposed, word i holds leaf i's truth bits.
template <class E, int NOUT, int TY>
__device__ __forceinline__ void tab_leaves(const Seg& r, const CONSTANT BatchCol* C, CInstr tl,
                                           const uint32_t* bmlds, uint32_t* wl, uint32_t lane) {
  const uint32_t L32 = (uint32_t)C->tab_lo, n = C->tab_n, m = C->tab_count;
  uint32_t T[32];
  if (C->tab_word != kNoLds) {
    const E* tab = (const E*)(bmlds + C->tab_word);
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      const uint32_t d = (uint32_t)seg_get<TY>(r, b) - L32;
      T[b] = tab[d < n ? d : n];
    }
  } else {
    // 32-bit byte offsets from the table's uniform base (device tables
    // are at most 32 MB)
    const GLOBAL char* tab = gptr<char>(C->gtab);
    if (C->tab_guarded) {
      // rows no table leaf needs (the complement of the union of the
      // leaves' guards) read the zero entry n: with g all ones on such a
      // row, min(d | g, n) is n, and on the others it is min(d, n)
      uint32_t need = 0;
      for (uint32_t i = 0; i < m; ++i) need |= acc_need(tl[i].slot, wl, lane);
      const uint32_t skip = ~need;
#pragma unroll
      for (int b = 0; b < 32; ++b) {
        const uint32_t d = (uint32_t)seg_get<TY>(r, b) - L32;
        const uint32_t g = (uint32_t)((int32_t)(skip << (31 - b)) >> 31);
        const uint32_t k = min(d | g, n);
        T[b] = *(const GLOBAL E*)(tab + k * (uint32_t)sizeof(E));
      }
    } else {
#pragma unroll
      for (int b = 0; b < 32; ++b) {
        const uint32_t d = (uint32_t)seg_get<TY>(r, b) - L32;
        const uint32_t k = min(d, n);
        T[b] = *(const GLOBAL E*)(tab + k * (uint32_t)sizeof(E));
      }
    }
  }
  // row b's entry holds leaf i in bit i; transposed, T[i] holds leaf i's
  // word (bit b = row b)
  transpose32<NOUT>(T);
#pragma unroll
  for (int i = 0; i < NOUT; ++i)
    if ((uint32_t)i < m) put_leaf(wl, lane, tl[i].slot, T[i]);
}

// A sparse IN-list leaf of the batched kernel: rows one at a time (its
// registers are spent on the column pipeline), loop kept rolled.
template <int TY>
__device__ __noinline__ uint32_t inlist_rows(CInstr I, uint64_t tb, uint32_t lane, uint64_t nrows) {
  const GLOBAL int64_t* list = gptr<int64_t>(I->aux);
  const uint32_t n = I->n;
  return pred_bits<TY, false>(I->data, tb, lane, nrows, [=](auto x, int) -> uint32_t {
    const int64_t xx = (int64_t)x;
    uint32_t base = 0, len = n;
    while (len > 1) {
      const uint32_t half = len >> 1;
      base = list[base + half] <= xx ? base + half : base;
      len -= half;
    }
    return list[base] == xx ? 1u : 0u;
  });
}

// Every leaf of one segment; truth words go to the wave's slots.  An int64
// column's upper half (h = 0) writes bits 16..31, its lower half completes
// them.  Sparse value lists take the element path once, with the last
// segment of their column.
template <int TY>
__device__ __forceinline__ void seg_leaves(const Seg& r, const CONSTANT BatchCol* C, int h,
                                           CInstr leaves, uint64_t tb, uint32_t lane,
                                           uint32_t* wl, const uint32_t* bmlds) {
  const uint32_t lb = C->leaf_begin, ln = C->leaf_count;
  const uint32_t tw = TY != T_I64 ? C->tab_word : kNoLds;
  const bool tabled = TY != T_I64 && (tw != kNoLds || C->gtab != nullptr);
  // leaves outside the table first: the values die once the table is read
  for (uint32_t k = tabled ? C->tab_count : 0u; k < ln; ++k) {
    CInstr I = leaves + lb + k;
    const uint32_t op = I->op;
    if (op == D_INLIST) {
      if (TY != T_I64 || h == 1) put_leaf(wl, lane, I->slot, inlist_rows<TY>(I, tb, lane, tb + kTileRows));
      continue;
    }
    const uint32_t P = seg_leaf<TY>(r, op, I, bmlds, wl, lane, TY == T_I64 && h == 0 ? 16 : 0);
    if constexpr (TY != T_I64) {
      put_leaf(wl, lane, I->slot, P);
    } else {  // int64 leaves always have a slot of their own
      const uint32_t sl = I->slot;
      uint32_t* w = wl + (sl & 0xFFFu) * kWave + lane;
      if (h == 0) *w = P;
      else *w = ((*w << 16) | P) & leaf_valid(sl, wl, lane);
    }
  }
  if constexpr (TY != T_I64) {
    if (tw != kNoLds || C->gtab != nullptr) {
      const uint32_t m = C->tab_count;
      if (m <= 8) tab_leaves<uint8_t, 8, TY>(r, C, leaves + lb, bmlds, wl, lane);
      else if (m <= 16) tab_leaves<uint16_t, 16, TY>(r, C, leaves + lb, bmlds, wl, lane);
      else tab_leaves<uint32_t, 32, TY>(r, C, leaves + lb, bmlds, wl, lane);
    }
  }
}

// All leaf tests of an entry on a full tile, as a software pipeline over
// the segments of the columns that have leaves: the loads of the next
// segment are in flight while the leaves of the current one run.
__device__ __forceinline__ void entry_leaves_full(const CONSTANT BatchTable* E,
                                                  const CONSTANT BatchCol* cols, CInstr leaves,
                                                  uint64_t tb, uint32_t lane, uint32_t* wl,
                                                  const uint32_t* bmlds, const CONSTANT uint32_t* ops) {
  const uint32_t cb = E->col_begin, cn = E->col_count;
  reset_acc(E, ops, wl, lane);
  // columns that only null tests read: validity alone
  for (uint32_t c = 0; c < cn; ++c) {
    const CONSTANT BatchCol* C = cols + cb + c;
    if (!C->leaf_count && C->vslot != kNoSlot)
      wl[C->vslot * kWave + lane] = valid_bits<true>(C->valid, tb, lane, tb + kTileRows);
  }
  uint32_t c = 0;
  while (c < cn && !cols[cb + c].leaf_count) ++c;
  if (c == cn) return;
  Seg cur;
  uint32_t curV = ~0u;
  int h = 0;
  seg_issue(cur, curV, cols + cb + c, h, tb, lane);
  for (;;) {
    const CONSTANT BatchCol* C = cols + cb + c;
    const uint32_t ty = C->type;
    uint32_t nc = c;
    int nh = 0;
    if (ty == T_I64 && h == 0) {
      nh = 1;
    } else {
      ++nc;
      while (nc < cn && !cols[cb + nc].leaf_count) ++nc;
    }
    const bool more = nc < cn;
    Seg nxt;
    uint32_t nxtV = ~0u;
    if (more) seg_issue(nxt, nxtV, cols + cb + nc, nh, tb, lane);
    if (h == 0 && C->vslot != kNoSlot) wl[C->vslot * kWave + lane] = curV;
    switch (ty) {
      case T_I8: seg_leaves<T_I8>(cur, C, h, leaves, tb, lane, wl, bmlds); break;
      case T_I16: seg_leaves<T_I16>(cur, C, h, leaves, tb, lane, wl, bmlds); break;
      case T_I32: seg_leaves<T_I32>(cur, C, h, leaves, tb, lane, wl, bmlds); break;
      default: seg_leaves<T_I64>(cur, C, h, leaves, tb, lane, wl, bmlds); break;
    }
    if (!more) break;
    cur = nxt;
    curV = nxtV;
    c = nc;
    h = nh;
  }
}

// All leaf tests of an entry on the partial last tile of its table.
__device__ __forceinline__ void entry_leaves_partial(const CONSTANT BatchTable* E,
                                                     const CONSTANT BatchCol* cols, CInstr leaves,
                                                     uint64_t tb, uint32_t lane, uint64_t nrows,
                                                     uint32_t* wl, const CONSTANT uint32_t* ops) {
  const uint32_t cb = E->col_begin, cn = E->col_count;
  reset_acc(E, ops, wl, lane);
  for (uint32_t c = 0; c < cn; ++c) {
    const CONSTANT BatchCol* C = cols + cb + c;
    const uint32_t lb = C->leaf_begin, ln = C->leaf_count;
    // validity first: direct factors read it when they are stored
    const uint32_t vs = C->vslot;
    if (vs != kNoSlot) wl[vs * kWave + lane] = valid_bits<false>(C->valid, tb, lane, nrows);
    for (uint32_t k = 0; k < ln; ++k) {
      CInstr I = leaves + lb + k;
      uint32_t P;
      switch (C->type) {
        case T_I8: P = leaf_pred<T_I8, false, true, false>(I->op, I, tb, lane, nrows, ~0u, StageView{}); break;
        case T_I16: P = leaf_pred<T_I16, false, true, false>(I->op, I, tb, lane, nrows, ~0u, StageView{}); break;
        case T_I32: P = leaf_pred<T_I32, false, true, false>(I->op, I, tb, lane, nrows, ~0u, StageView{}); break;
        default: P = leaf_pred<T_I64, false, true, false>(I->op, I, tb, lane, nrows, ~0u, StageView{}); break;
      }
      put_leaf(wl, lane, I->slot, P);
    }
  }
}

// TRUE bits of the lane's rows for one batched program: its postfix
// combinators over the leaf and validity words in the wave's slots.
__device__ __forceinline__ uint32_t run_ops(const CONSTANT uint32_t* ops, uint32_t nops,
                                            const uint32_t* wl, uint32_t lane) {
  uint32_t st[kMaxDepth], sf[kMaxDepth];
  uint32_t tt = 0, tf = 0;
  int d = 0;
  for (uint32_t pc = 0; pc < nops; ++pc) {
    const uint32_t w = ops[pc];
    const uint32_t op = w & 0xFFu;
    if (op == B_AND_LEAF || op == B_OR_LEAF) {
      const uint32_t vs = w >> 20;
      const uint32_t V = vs == kNoSlot ? ~0u : wl[vs * kWave + lane];
      const uint32_t P = wl[((w >> 8) & 0xFFFu) * kWave + lane];
      if (op == B_AND_LEAF) { tt &= P & V; tf |= ~P & V; }
      else { tt |= P & V; tf &= ~P & V; }
    } else if (op == B_ACC || op == B_AND_ACC) {
      const uint32_t fs = w >> 20;
      const uint32_t T = wl[((w >> 8) & 0xFFFu) * kWave + lane];
      const uint32_t F = fs == kNoSlot ? ~T : wl[fs * kWave + lane];
      if (op == B_AND_ACC) {
        tt &= T; tf |= F;
      } else {
        if (d > 0) {
          st[uni(d - 1)] = tt;
          sf[uni(d - 1)] = tf;
        }
        tt = T; tf = F;
        ++d;
      }
    } else if (op < D_AND || op == D_TRUE || op == D_FALSE) {
      uint32_t t, f;
      const uint32_t vs = w >> 20;
      const uint32_t V = (vs == kNoSlot || op >= D_TRUE) ? ~0u : wl[vs * kWave + lane];
      switch (op) {
        case D_RANGE: {
          const uint32_t P = wl[((w >> 8) & 0xFFFu) * kWave + lane];
          t = P & V; f = ~P & V;
          break;
        }
        case D_NN_TRUE: t = V; f = 0; break;
        case D_NN_FALSE: t = 0; f = V; break;
        case D_ISNULL: t = ~V; f = V; break;
        case D_NOTNULL: t = V; f = ~V; break;
        case D_TRUE: t = ~0u; f = 0; break;
        default: t = 0; f = ~0u; break;  // D_FALSE
      }
      if (d > 0) {
        st[uni(d - 1)] = tt;
        sf[uni(d - 1)] = tf;
      }
      tt = t; tf = f;
      ++d;
    } else if (op == D_NOT) {
      const uint32_t x = tt; tt = tf; tf = x;
    } else if (op == D_ISUNK) {
      const uint32_t k = tt | tf; tt = ~k; tf = k;
    } else {
      const uint32_t at = st[uni(d - 2)], af = sf[uni(d - 2)];
      if (op == D_AND) { tt &= at; tf |= af; }
      else { tt |= at; tf &= af; }
      --d;
    }
  }
  return tt;
}

// The same for a program with no NOT and no IS UNKNOWN: the TRUE word of an
// AND or OR is the AND or OR of its operands' TRUE words, so the TRUE words
// of leaves (NULL rows cleared) and null tests are all it needs, one word
// per stack entry.
__device__ __forceinline__ uint32_t run_ops2(const CONSTANT uint32_t* ops, uint32_t nops,
                                             const uint32_t* wl, uint32_t lane) {
  uint32_t st[kMaxDepth];
  uint32_t tt = 0;
  int d = 0;
  for (uint32_t pc = 0; pc < nops; ++pc) {
    const uint32_t w = ops[pc];
    const uint32_t op = w & 0xFFu;
    if (op >= B_AND_LEAF) {   // fused leaves and the accumulator
      const uint32_t P = wl[((w >> 8) & 0xFFFu) * kWave + lane];
      if (op == B_AND_LEAF || op == B_AND_ACC) {
        tt &= P;
      } else if (op == B_OR_LEAF) {
        tt |= P;
      } else {  // B_ACC
        if (d > 0) st[uni(d - 1)] = tt;
        tt = P;
        ++d;
      }
    } else if (op < D_AND || op == D_TRUE || op == D_FALSE) {
      uint32_t t;
      if (op == D_RANGE) {
        t = wl[((w >> 8) & 0xFFFu) * kWave + lane];
      } else {
        const uint32_t vs = w >> 20;
        const uint32_t V = (vs == kNoSlot || op >= D_TRUE) ? ~0u : wl[vs * kWave + lane];
        t = (op == D_NN_TRUE || op == D_NOTNULL) ? V : op == D_ISNULL ? ~V : op == D_TRUE ? ~0u : 0u;
      }
      if (d > 0) st[uni(d - 1)] = tt;
      tt = t;
      ++d;
    } else if (op == D_NOT) {
      tt = ~tt;
    } else if (op == D_ISUNK) {
      tt = 0;
    } else {
      const uint32_t at = st[uni(d - 2)];
      if (op == D_AND) tt &= at;
      else tt |= at;
      --d;
    }
  }
  return tt;
}

// Per workgroup, per-program counts accumulate in LDS; at the end each
// workgroup adds them to per-program accumulator lines (128 bytes each, so
// atomics on different programs do not contend), and the last workgroup by
// ticket moves the finished lines out and zeroes them.  Entries may be
// chunks of tables (row_begin), and lines not finished by this launch keep
// accumulating: a cooperative scan adds one chunk per launch.
__global__ void __launch_bounds__(768) k_batch(BatchArgs a) {
  // LDS: per-program counters, tables and staged bitmaps, each wave's slots
  extern __shared__ __align__(16) uint32_t dyn[];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t nacc = a.acc_words;   // min(nprogs, kBatchMaxProgs)
  uint32_t* acc = dyn;
  uint32_t* bmlds = dyn + nacc;
  uint32_t* wl = bmlds;   // this wave's slots, placed by each pass's layout
  for (uint32_t p = threadIdx.x; p < nacc; p += blockDim.x) acc[p] = 0;
  __syncthreads();
  const CONSTANT BatchTable* tables = (const CONSTANT BatchTable*)a.tables;
  const CONSTANT BatchCol* cols = (const CONSTANT BatchCol*)a.cols;
  CInstr leaves = (CInstr)a.leaves;
  const CONSTANT BatchProg* progs = (const CONSTANT BatchProg*)a.progs;
  const CONSTANT BatchBitmap* bms = (const CONSTANT BatchBitmap*)a.bms;
  // the workgroup takes groups of nw consecutive tiles; entry ranges are
  // padded to multiples of kBatchTileAlign, so a group never straddles two
  // entries and the loop below (with its barriers) is uniform over the
  // workgroup
  const uint64_t ngroups = a.total_tiles / nw;
  uint32_t staged = 0xFFFFFFFFu;
  for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const uint64_t flat = g * nw + wave;
    // entry holding this tile: last e with tile_begin <= flat (uniform search)
    uint32_t lo = 0, hi = a.ntables;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tables[mid].tile_begin <= flat) lo = mid; else hi = mid;
    }
    lo = uni(lo);
    const CONSTANT BatchTable* E = tables + lo;
    if (lo != staged) {
      // a new pass: its own LDS layout (tables, bitmaps, slots), so every
      // wave must be done with the previous one's first
      __syncthreads();
      wl = bmlds + E->bm_words + wave * E->slot_words;
      if (E->bm_count || E->ntab) {
        // lookup tables: copies of the ones k_tables built in device memory
        for (uint32_t c = 0; c < E->col_count; ++c) {
          const CONSTANT BatchCol* C = cols + E->col_begin + c;
          if (C->tab_word == kNoLds) continue;
          const uint32_t words = ((C->tab_n + 1) * tab_entry_bytes(C->tab_count) + 3) / 4;
          const GLOBAL uint32_t* src = gptr<uint32_t>(C->gtab);
          uint32_t* dst = bmlds + C->tab_word;
          for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
        }
        for (uint32_t k = 0; k < E->bm_count; ++k) {
          const CONSTANT BatchBitmap* B = bms + E->bm_begin + k;
          const uint32_t n = B->words, last = B->last_mask;
          const GLOBAL uint32_t* src = gptr<uint32_t>(B->src);
          uint32_t* dst = bmlds + B->lds_word;
          for (uint32_t i = threadIdx.x; i <= n; i += blockDim.x) {
            uint32_t w = 0;
            if (i < n) w = i + 1 == n ? src[i] & last : src[i];
            dst[i] = w;
          }
        }
        __syncthreads();
      }
      staged = lo;
    }
    const uint64_t local = flat - E->tile_begin;
    if (local >= E->ntiles) continue;   // padding
    const uint64_t nrows = E->nrows;
    const uint64_t tb = E->row_begin + local * kTileRows;
    const uint32_t pb = E->prog_begin, pn = E->prog_count;
    const bool full = tb + kTileRows <= nrows;
    uint32_t inr = ~0u;
    if (full) {
      entry_leaves_full(E, cols, leaves, tb, lane, wl, bmlds, (const CONSTANT uint32_t*)a.ops);
    } else {
      entry_leaves_partial(E, cols, leaves, tb, lane, nrows, wl, (const CONSTANT uint32_t*)a.ops);
      inr = inrange_bits(tb, lane, nrows);
    }
    // programs in pairs: both popcounts (at most 2048 per wave each) share
    // one wave reduction, 16 bits apart
    for (uint32_t k = 0; k < pn; k += 2) {
      uint32_t T[2] = {0u, 0u};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (k + q >= pn) break;
        const CONSTANT BatchProg* P = progs + pb + k + q;
        const uint32_t nops = P->nops;
        const CONSTANT uint32_t* ops = (const CONSTANT uint32_t*)P->ops;
        uint32_t t;
        if (nops & kAndList) {   // a conjunction of TRUE words at these offsets
          const uint32_t n = nops & ~kAndList;
          t = wl[ops[0] + lane];
          for (uint32_t j = 1; j < n; ++j) t &= wl[ops[j] + lane];
        } else if (nops & kTwoValued) {
          t = run_ops2(ops, nops & ~kTwoValued, wl, lane);
        } else {
          t = run_ops(ops, nops, wl, lane);
        }
        T[q] = t & inr;
      }
      const uint32_t c2 = wave_sum(__builtin_popcount(T[0]) | (__builtin_popcount(T[1]) << 16));
      if (lane == 0 && c2) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const uint32_t c = q ? c2 >> 16 : c2 & 0xFFFFu;
          if (!c) continue;
          if (pb + k + q < nacc) {
            atomicAdd(&acc[pb + k + q], c);
          } else {  // beyond the LDS table: straight to the accumulator line
            atomicAdd(&a.acc[(uint64_t)progs[pb + k + q].acc_index * kBatchAccStride], (unsigned long long)c);
          }
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < nacc; p += blockDim.x)
    if (acc[p]) atomicAdd(&a.acc[(uint64_t)progs[p].acc_index * kBatchAccStride], (unsigned long long)acc[p]);
  atomics_done();
  __syncthreads();
  __shared__ bool last;
  if (threadIdx.x == 0) {
    const unsigned int ticket = atomicAdd(&a.slot->ticket, 1u);
    last = ticket == gridDim.x - 1;
  }
  __syncthreads();
  if (last) {
    for (uint32_t k = threadIdx.x; k < a.ndone; k += blockDim.x) {
      const uint64_t line = a.done ? a.done[k] : k;
      a.out[k] = atomicExch(&a.acc[line * kBatchAccStride], 0ull);
    }
    atomics_done();
    __syncthreads();
    if (threadIdx.x == 0) atomicExch(&a.slot->ticket, 0u);
  }
}

// Device-memory lookup tables of a batch (one thread per entry; the bitmap
// words of neighbouring entries are shared, so the reads coalesce).
__global__ void __launch_bounds__(256) k_tables(const TableBuild* __restrict__ tb, uint32_t nb,
                                                uint64_t nentries) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nentries; e += stride) {
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tb[mid].entry_begin <= e) lo = mid; else hi = mid;
    }
    const TableBuild& B = tb[lo];
    const uint64_t i = e - B.entry_begin;
    uint32_t w = 0;
    if (i < B.n) {
      const int64_t x = B.lo + (int64_t)i;
      for (uint32_t k = 0; k < B.m; ++k) {
        const DevInstr& I = B.leaves[k];
        const uint64_t d = (uint64_t)x - (uint64_t)I.lo;
        uint32_t bit;
        if (I.op == D_RANGE) {
          bit = d <= I.span;
        } else {  // D_BITMAP
          const uint32_t* bits = (const uint32_t*)I.aux;
          bit = d < I.span ? (bits[d >> 5] >> (d & 31)) & 1u : 0u;
        }
        w |= bit << k;
      }
    }
    const uint32_t eb = tab_entry_bytes(B.m);
    if (eb == 1) ((uint8_t*)B.dst)[i] = (uint8_t)w;
    else if (eb == 2) ((uint16_t*)B.dst)[i] = (uint16_t)w;
    else B.dst[i] = w;
  }
}

// ------------------------------------------ batched count, column tables --
// A program of a pass owns one bit of each word of a row's accumulator (its
// single-column clauses that failed, and one word per clause spanning
// columns); a column ORs into it the entry of its value in its lookup table,
// so one lookup serves every program of the pass on that column.

// Truth of a literal (a leaf test, possibly negated) on a row: `nonnull`
// says whether the row's value is present, `inwin` whether x lies in the
// window of the column's value tests (outside it every value test is FALSE).
__device__ __forceinline__ bool lit_true(const DevInstr& L, bool nonnull, bool inwin, int64_t x) {
  const bool neg = (L.flags & kLitNeg) != 0u;
  switch (L.op) {
    case D_NN_TRUE: return nonnull && !neg;
    case D_NN_FALSE: return nonnull && neg;
    case D_ISNULL: return nonnull ? neg : !neg;
    case D_NOTNULL: return nonnull ? !neg : neg;
    default: break;
  }
  if (!nonnull) return false;   // a value test on NULL is UNKNOWN, negated or not
  bool v = false;
  if (inwin) {
    const uint64_t d = (uint64_t)x - (uint64_t)L.lo;
    if (L.op == D_RANGE) {
      v = d <= L.span;
    } else if (L.op == D_BITMAP) {
      v = d < L.span && ((((const uint32_t*)L.aux)[d >> 5] >> (d & 31)) & 1u);
    } else {  // D_INLIST: lower bound in the sorted list
      const int64_t* list = (const int64_t*)L.aux;
      uint32_t base = 0, len = L.n;
      while (len > 1) {
        const uint32_t half = len >> 1;
        base = list[base + half] <= x ? base + half : base;
        len -= half;
      }
      v = list[base] == x;
    }
  }
  return v != neg;
}

// The bits the atoms [ab, ab + an) set for one row (dwords w0 .. w3).
__device__ __forceinline__ void atoms_eval(const LutAtom* atoms, const DevInstr* lits, uint32_t ab,
                                           uint32_t an, bool nonnull, bool inwin, int64_t x,
                                           uint32_t& w0, uint32_t& w1, uint32_t& w2, uint32_t& w3) {
  for (uint32_t k = 0; k < an; ++k) {
    const LutAtom A = atoms[ab + k];
    bool any = false;
    for (uint32_t l = 0; l < A.lit_count && !any; ++l) any = lit_true(lits[A.lit_begin + l], nonnull, inwin, x);
    if (any != (A.kind == LA_SAT)) continue;
    const uint32_t m = 1u << (A.bit & 31);
    switch (A.bit >> 5) {
      case 0: w0 |= m; break;
      case 1: w1 |= m; break;
      case 2: w2 |= m; break;
      default: w3 |= m; break;
    }
  }
}

// Lookup tables of a launch, in device memory (one thread per entry).
__global__ void __launch_bounds__(256) k_luts(LutArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.nentries; e += stride) {
    uint32_t lo = 0, hi = a.nbuilds;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (a.builds[mid].entry_begin <= e) lo = mid; else hi = mid;
    }
    const LutBuild& B = a.builds[lo];
    const LutCol& C = a.cols[B.col];
    const uint32_t i = (uint32_t)(e - B.entry_begin);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    bool zero = false, nonnull = true, inwin = true;
    int64_t x = 0;
    if (C.kind == LK_DIRECT) {
      // 0: below the window, 1..n: values lo.., n+1: above, n+2: NULL, n+3: zero
      if (i == 0 || i == C.n + 1) inwin = false;
      else if (i == C.n + 2) nonnull = false;
      else if (i == C.n + 3) zero = true;
      else x = C.lo + (int64_t)(i - 1);
    } else if (C.kind == LK_RANK) {
      // 0..n: by rank, n+1: NULL, n+2: zero
      if (i == C.n + 1) nonnull = false;
      else if (i == C.n + 2) zero = true;
      else x = a.reps[B.reps + i];
    } else {  // LK_VALID: 0 non-NULL, 1 NULL
      nonnull = i == 0;
      inwin = false;
    }
    if (!zero) atoms_eval(a.atoms, a.lits, C.atom_begin, C.atom_count, nonnull, inwin, x, w0, w1, w2, w3);
    uint32_t* dst = B.dst + (uint64_t)i * B.dwords;
    dst[0] = w0;
    if (B.dwords > 1) dst[1] = w1;
    if (B.dwords > 2) {
      dst[2] = w2;
      dst[3] = w3;
    }
  }
}

// Values of one lane's rows of one column in a segment: 4 S rows (S steps
// of the tile's row mapping) held from vector w[0]: step s of a narrow
// column in w[s] (its leading components); of an int64 column, rows 0 and 1
// of step s in w[s] and rows 2 and 3 in w[S + s] (the next slot).
template <int TY, int S>
__device__ __forceinline__ auto lget(const v4i* w, int s, int i) {
  if constexpr (TY == T_I8) {
    return (int32_t)(int8_t)((uint32_t)w[s][0] >> (8 * i));
  } else if constexpr (TY == T_I16) {
    return (int32_t)(int16_t)((uint32_t)w[s][i >> 1] >> (16 * (i & 1)));
  } else if constexpr (TY == T_I32) {
    return (int32_t)w[s][i];
  } else {
    const v4i& q = w[S * (i >> 1) + s];   // rows 2, 3 in the next slot
    const int k = 2 * (i & 1);
    return (int64_t)(((uint64_t)(uint32_t)q[k + 1] << 32) | (uint32_t)q[k]);
  }
}

// Buffer resource over rows [tb, min(tb + 2048, nrows)) of a column of
// `width`-byte values: 32-bit offsets from the tile's start, and a read past
// the table's last row returns zero without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* data, uint64_t tb, uint64_t nrows,
                                                            uint32_t width) {
  const uint64_t rows = nrows - tb < (uint64_t)kTileRows ? nrows - tb : (uint64_t)kTileRows;
  return __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)data + tb * width), (short)0,
                                           (int)(rows * width), 0x00020000);
}

constexpr int kNt = 2;   // buffer-load cache policy: nontemporal (streamed once)

// One register slot's loads for steps j0 .. j0 + S - 1: one 16-byte load
// per step at the lane's first row, whatever the column's width, so that
// every slot has the same shape and no slot's registers depend on a branch
// (a branch would make the compiler wait for loads in flight).  A column
// narrower than 4 bytes reads its neighbours' rows too (the same cache
// lines); an int64 column takes two slots, the second one 16 bytes further.
// The resource bounds the reads: past the table, or for an unused slot (no
// bytes), they return zero without touching memory.
template <int S>
__device__ __forceinline__ void slot_issue(v4i* w, __amdgpu_buffer_rsrc_t rs, uint32_t width, int j0,
                                           uint32_t lane) {
#pragma unroll
  for (int s = 0; s < S; ++s)
    w[s] = (v4i)__builtin_amdgcn_raw_buffer_load_b128(rs, (int)(width * (4u * lane + 256u * (uint32_t)(j0 + s))), 0,
                                                      kNt);
}

// Validity of the segment's rows: bit 4 s + i = row (step j0 + s, i) is not
// NULL (0 past nrows).
template <int R>
__device__ __forceinline__ uint32_t lseg_valid(const uint32_t* valid, uint64_t tb, int j0, uint32_t lane,
                                               uint64_t nrows, bool full) {
  constexpr int S = R / 4;
  const GLOBAL uint32_t* vw = gptr<uint32_t>(valid) + tb / 32 + (lane >> 3) + 8 * j0;
  const uint32_t sh = 4 * (lane & 7);
  uint32_t V = 0;
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (full || tb + 256u * (uint32_t)(j0 + s) + 4u * lane < nrows) V |= ((vw[8 * s] >> sh) & 0xFu) << (4 * s);
  return V;
}



template <int D>
__device__ __forceinline__ void ent_or(const uint32_t* tab, uint32_t idx, uint32_t (&acc)[D]) {
  if constexpr (D == 1) {
    acc[0] |= tab[idx];
  } else if constexpr (D == 2) {
    const v2u e = ((const v2u*)tab)[idx];
    acc[0] |= e[0];
    acc[1] |= e[1];
  } else {
    const v4u e = ((const v4u*)tab)[idx];
#pragma unroll
    for (int d = 0; d < 4; ++d) acc[d] |= e[d];
  }
}

#define LDS_PTR(T) __attribute__((address_space(3))) T*

// The entry at LDS byte address e ORed into the accumulators.
template <int D>
__device__ __forceinline__ void ent_or_lds(LDS_PTR(const char) e, uint32_t (&acc)[D]) {
  if constexpr (D == 1) {
    acc[0] |= *(LDS_PTR(const uint32_t))e;
  } else if constexpr (D == 2) {
    const v2u x = *(LDS_PTR(const v2u))e;
    acc[0] |= x[0];
    acc[1] |= x[1];
  } else {
    const v4u x = *(LDS_PTR(const v4u))e;
#pragma unroll
    for (int d = 0; d < 4; ++d) acc[d] |= x[d];
  }
}

// Entry idx of a device-memory table through a buffer resource: a 32-bit
// offset per lane instead of a 64-bit address, and an offset past the
// table reads zero.
template <int D>
__device__ __forceinline__ void gent_or(__amdgpu_buffer_rsrc_t tab, uint32_t idx, uint32_t (&acc)[D]) {
  if constexpr (D == 1) {
    acc[0] |= __builtin_amdgcn_raw_buffer_load_b32(tab, (int)(idx * 4u), 0, 0);
  } else if constexpr (D == 2) {
    const v2u e = __builtin_amdgcn_raw_buffer_load_b64(tab, (int)(idx * 8u), 0, 0);
    acc[0] |= e[0];
    acc[1] |= e[1];
  } else {
    const v4u e = __builtin_amdgcn_raw_buffer_load_b128(tab, (int)(idx * 16u), 0, 0);
#pragma unroll
    for (int d = 0; d < 4; ++d) acc[d] |= e[d];
  }
}

// Buffer resource of a device table of `entries` D-dword entries (gfx9
// raw buffer: stride 0, bounds checked against the byte size).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const uint32_t* tab, uint32_t entries, uint32_t dwords) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)tab, (short)0, (int)(entries * dwords * 4u), 0x00020000);
}

// A register slot's column as its lookups need it, decoded once per tile.
struct SlotD {
  uint32_t info;          // kSd* flags, type in bits 0..3, kind in bits 4..5
  uint32_t n;             // DIRECT: window size; RANK: bounds
  int64_t lo;             // DIRECT: value of entry 1
  uint32_t tab;           // table: LDS word offset, or kNoLds
  uint32_t first;         // RANK: first bound
  const uint32_t* gtab;   // table in device memory
  const char* data;       // the slot's bytes of the tile's first row
  const uint32_t* valid;  // validity word of the tile's first row
  uint32_t bytes, vbytes; // readable bytes from there (0: none)
};
constexpr uint32_t kSdNullable = 1u << 8, kSdGuard = 1u << 10, kSdData = 1u << 11;

__device__ __forceinline__ SlotD slot_decode(const CONSTANT LutPass* P, const CONSTANT LutCol* cb, int k,
                                             uint64_t tb, uint64_t rows) {
  SlotD d{};
  const uint32_t code = (P->slot_col[k / 4] >> (8 * (k % 4))) & 0xFFu;
  if (code == kNoSlotCol) {
    d.info = T_I32;
    d.data = (const char*)P;
    d.valid = (const uint32_t*)P;
  } else {
    const CONSTANT LutCol* C = cb + (code & kSlotColMask);
    const uint32_t ty = C->type;
    const uint32_t width = ty == T_I8 ? 1u : ty == T_I16 ? 2u : ty == T_I32 ? 4u : 8u;
    const uint32_t half = code & kSlotHigh ? 16u : 0u;
    d.info = ty | (C->kind << 4) | (C->valid ? kSdNullable : 0u) | (C->guard ? kSdGuard : 0u) |
             (half ? 0u : kSdData);
    d.n = C->n;
    d.lo = C->lo;
    d.tab = C->lds_word;
    d.first = C->first;
    d.gtab = C->gtab;
    d.data = (const char*)C->data + tb * width + half;
    // whole dwords: a raw buffer load zeroes a dword that crosses the
    // bound, and the bytes up to the next 4-byte boundary share the last
    // element's 16-byte-aligned block (the same memory page)
    const uint32_t span = ((uint32_t)(rows * width) + 3u) & ~3u;
    // made scalar: the compiler turns this into a saturating subtract that
    // only the vector unit has, and a buffer resource built from a vector
    // register is wrapped in a readfirstlane loop at every load
    d.bytes = uni(span > half ? span - half : 0u);
    const bool hv = !half && C->valid;
    d.valid = hv ? C->valid + tb / 32 : (const uint32_t*)P;
    d.vbytes = hv ? (uint32_t)(((rows + 31) / 32) * 4) : 0u;
  }
  return d;
}

// Table indices of an item's rows to entries, ORed into the accumulators of
// segment rows OFF .. OFF + NR - 1: from LDS, or from device memory where a
// guarded table is read only on rows some program of the pass can still
// count (the others read the zero entry).
template <int D, int R, int NR, int OFF>
__device__ __forceinline__ void lookup_or(const SlotD& sd, const uint32_t* lds, uint32_t (&idx)[NR],
                                          uint32_t zero, const CONSTANT LutPass* P, uint32_t (&acc)[R][D]) {
  if (sd.tab != kNoLds) {
    const uint32_t* tab = lds + sd.tab;
#pragma unroll
    for (int r = 0; r < NR; ++r) ent_or<D>(tab, idx[r], acc[OFF + r]);
  } else {
    const __amdgpu_buffer_rsrc_t tab = table_rsrc(sd.gtab, zero + 1, D);
    if (sd.info & kSdGuard) {
      // a row some program can still count: a failure bit (word 0 of a
      // dword) still clear
      uint32_t am[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const uint32_t g = (P->fold[d] >> 8) & 0xFFu;
        am[d] = g >= 32 ? ~0u : (1u << g) - 1u;
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        uint32_t alive = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) alive |= ~acc[OFF + r][d] & am[d];
        idx[r] = alive ? idx[r] : zero;
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) gent_or<D>(tab, idx[r], acc[OFF + r]);
  }
}

// One column on one segment: every row's entry ORed into its accumulator.
// V holds the validity of the segment's R rows.
template <int D, int R, int TY, int NR, int OFF>
__device__ __forceinline__ void lut_col(const v4i* seg, const SlotD& sd, const LutArgs& a, uint32_t V,
                                        const uint32_t* lds, const CONSTANT LutPass* P, uint32_t (&acc)[R][D]) {
  constexpr int S = NR / 4;
  const uint32_t kind = (sd.info >> 4) & 3u, n = sd.n;
  const bool nullable = (sd.info & kSdNullable) != 0;
  uint32_t idx[NR];
  if (kind == LK_DIRECT) {
    const int64_t lo = sd.lo;
    if constexpr (TY != T_I64) {
      if (sd.tab != kNoLds && !nullable) {
        // clamped value straight to the entry's LDS byte address: the
        // table's address less (lo - 1) entries, plus the value's entries
        constexpr int64_t tmin = TY == T_I8 ? INT8_MIN : TY == T_I16 ? INT16_MIN : INT32_MIN;
        constexpr int64_t tmax = TY == T_I8 ? INT8_MAX : TY == T_I16 ? INT16_MAX : INT32_MAX;
        const int32_t cl = (int32_t)(lo - 1 < tmin ? tmin : lo - 1);
        const int32_t ch = (int32_t)(lo + (int64_t)n > tmax ? tmax : lo + (int64_t)n);
        // byte offsets within LDS, through an LDS-space pointer (32-bit)
        const LDS_PTR(const char) l3 = (LDS_PTR(const char))lds;
        const uint32_t abase = sd.tab * 4u - (uint32_t)(lo - 1) * (4u * D);
        int32_t chv = ch;   // in a vector register once: one scalar operand per VALU op
        asm volatile("v_mov_b32 %0, %1" : "=v"(chv) : "s"(ch));
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int32_t x = lget<TY, S>(seg, s, i);
            int32_t m;
            asm("v_med3_i32 %0, %1, %2, %3" : "=v"(m) : "v"(x), "s"(cl), "v"(chv));
            ent_or_lds<D>(l3 + (abase + (uint32_t)m * (4u * D)), acc[OFF + 4 * s + i]);
          }
        return;
      }
      // clamp to [lo - 1, lo + n] (inside the type), then offset: entry 0
      // below the window, n + 1 above it
      constexpr int64_t tmin = TY == T_I8 ? INT8_MIN : TY == T_I16 ? INT16_MIN : INT32_MIN;
      constexpr int64_t tmax = TY == T_I8 ? INT8_MAX : TY == T_I16 ? INT16_MAX : INT32_MAX;
      const int32_t cl = (int32_t)(lo - 1 < tmin ? tmin : lo - 1);
      const int32_t ch = (int32_t)(lo + (int64_t)n > tmax ? tmax : lo + (int64_t)n);
      const uint32_t base = (uint32_t)(lo - 1);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int32_t x = lget<TY, S>(seg, s, i);
          idx[4 * s + i] = (uint32_t)min(max(x, cl), ch) - base;
        }
    } else {
      const int64_t cl = lo == INT64_MIN ? lo : lo - 1;
      const int64_t ch = lo + (int64_t)n;   // the planned window ends below INT64_MAX
      const uint64_t base = (uint64_t)lo - 1u;
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t x = lget<TY, S>(seg, s, i);
          const int64_t m = x < cl ? cl : x > ch ? ch : x;
          idx[4 * s + i] = (uint32_t)((uint64_t)m - base);
        }
    }
    if (nullable) {
#pragma unroll
      for (int r = 0; r < NR; ++r) idx[r] = (V >> (OFF + r)) & 1u ? idx[r] : n + 2;
    }
    lookup_or<D, R, NR, OFF>(sd, lds, idx, n + 3, P, acc);
  } else {  // LK_RANK: the number of bounds at or below the value
    // bounds in blocks of eight (the list is padded to whole blocks), one
    // scalar load per block
    const CONSTANT int64_t* b = (const CONSTANT int64_t*)a.bounds + sd.first;
#pragma unroll
    for (int r = 0; r < NR; ++r) idx[r] = 0;
    for (uint32_t k0 = 0; k0 < n; k0 += 8) {
      int64_t bb[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) bb[j] = b[k0 + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (k0 + j >= n) break;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if constexpr (TY != T_I64) idx[4 * s + i] += lget<TY, S>(seg, s, i) >= (int32_t)bb[j] ? 1u : 0u;
            else idx[4 * s + i] += lget<TY, S>(seg, s, i) >= bb[j] ? 1u : 0u;
          }
      }
    }
    if (nullable) {
#pragma unroll
      for (int r = 0; r < NR; ++r) idx[r] = (V >> (OFF + r)) & 1u ? idx[r] : n + 1;
    }
    lookup_or<D, R, NR, OFF>(sd, lds, idx, n + 2, P, acc);
  }
}

// Per-lane carry-save counters of T bits: planes of weight 1, 2, 4, 8 and
// a vertical counter of weight 16 * 2^k (at most 2047 per bit position
// between reads).
constexpr int kHsLevels = 7;
struct Hs {
  uint32_t ones, twos, fours, eights;
  uint32_t h[kHsLevels];
};

__device__ __forceinline__ void csa(uint32_t& carry, uint32_t& sum, uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t u = a ^ b;
  carry = (a & b) | (u & c);
  sum = u ^ c;
}

__device__ __forceinline__ void hs_sixteens(Hs& s, uint32_t c) {
#pragma unroll
  for (int k = 0; k < kHsLevels; ++k) {
    const uint32_t t = s.h[k] & c;
    s.h[k] ^= c;
    c = t;
  }
}

// Add NW words (NW = 1, 2, 4 or a multiple of 8), each bit position counting 0 or 1.
template <int NW>
__device__ __forceinline__ void hs_add(Hs& s, const uint32_t* w) {
  if constexpr (NW == 1) {
    const uint32_t t = s.ones & w[0];
    s.ones ^= w[0];
    const uint32_t f = s.twos & t;
    s.twos ^= t;
    const uint32_t e = s.fours & f;
    s.fours ^= f;
    const uint32_t c = s.eights & e;
    s.eights ^= e;
    hs_sixteens(s, c);
  } else if constexpr (NW > 8) {
    static_assert(NW % 8 == 0, "blocks of eight words");
#pragma unroll
    for (int k = 0; k < NW; k += 8) hs_add<8>(s, w + k);
  } else if constexpr (NW == 8) {
    uint32_t ta, tb, fa, fb, e;
    csa(ta, s.ones, s.ones, w[0], w[1]);
    csa(tb, s.ones, s.ones, w[2], w[3]);
    csa(fa, s.twos, s.twos, ta, tb);
    csa(ta, s.ones, s.ones, w[4], w[5]);
    csa(tb, s.ones, s.ones, w[6], w[7]);
    csa(fb, s.twos, s.twos, ta, tb);
    csa(e, s.fours, s.fours, fa, fb);
    const uint32_t c = s.eights & e;
    s.eights ^= e;
    hs_sixteens(s, c);
  } else if constexpr (NW == 4) {
    uint32_t ta, tb, f;
    csa(ta, s.ones, s.ones, w[0], w[1]);
    csa(tb, s.ones, s.ones, w[2], w[3]);
    csa(f, s.twos, s.twos, ta, tb);
    const uint32_t e = s.fours & f;
    s.fours ^= f;
    const uint32_t c = s.eights & e;
    s.eights ^= e;
    hs_sixteens(s, c);
  } else {
    static_assert(NW == 2, "one, two, four or a multiple of eight words");
    uint32_t t;
    csa(t, s.ones, s.ones, w[0], w[1]);
    const uint32_t f = s.twos & t;
    s.twos ^= t;
    const uint32_t e = s.fours & f;
    s.fours ^= f;
    const uint32_t c = s.eights & e;
    s.eights ^= e;
    hs_sixteens(s, c);
  }
}

// Rows' accumulators to their T words (bit p: program p counts the row),
// packed 32 / B rows to a word, into the counters.  Within dword d, word 0
// is inverted and the b_d-bit words are ANDed together by folding.
template <int D, int R>
__device__ __forceinline__ void lut_count(uint32_t (&acc)[R][D], const CONSTANT LutPass* P, uint32_t inr,
                                          Hs& hs) {
  const uint32_t B = P->bits;
  uint32_t nm[D], gm[D], ps[D], bw[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const uint32_t f = P->fold[d];
    bw[d] = f & 0xFFu;
    const uint32_t g = (f >> 8) & 0xFFu;
    ps[d] = f >> 16;
    nm[d] = bw[d] >= 32 ? ~0u : (1u << bw[d]) - 1u;
    gm[d] = g >= 32 ? ~0u : (1u << g) - 1u;
  }
  uint32_t T[R];
#pragma unroll
  for (int r = 0; r < R; ++r) T[r] = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    // the dword's width, a uniform branch around all rows
    if (bw[d] >= 32) {
#pragma unroll
      for (int r = 0; r < R; ++r) T[r] |= ((acc[r][d] ^ nm[d]) & gm[d]) << ps[d];
    } else if (bw[d] == 16) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t t = acc[r][d] ^ nm[d];
        T[r] |= ((t & (t >> 16)) & gm[d]) << ps[d];
      }
    } else if (bw[d] == 8) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t t = acc[r][d] ^ nm[d];
        t &= t >> 16;
        T[r] |= ((t & (t >> 8)) & gm[d]) << ps[d];
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t t = acc[r][d] ^ nm[d];
        t &= t >> 16;
        t &= t >> 8;
        T[r] |= ((t & (t >> 4)) & gm[d]) << ps[d];
      }
    }
  }
  if (inr != ~0u) {
#pragma unroll
    for (int r = 0; r < R; ++r) T[r] = (inr >> r) & 1u ? T[r] : 0u;
  }
  if (B == 32) {
    hs_add<R>(hs, T);
  } else if (B == 16) {
    uint32_t w[R / 2];
#pragma unroll
    for (int k = 0; k < R / 2; ++k) w[k] = T[2 * k] | (T[2 * k + 1] << 16);
    hs_add<R / 2>(hs, w);
  } else {
    uint32_t w[R / 4];
#pragma unroll
    for (int k = 0; k < R / 4; ++k)
      w[k] = T[4 * k] | (T[4 * k + 1] << 8) | (T[4 * k + 2] << 16) | (T[4 * k + 3] << 24);
    hs_add<R / 4>(hs, w);
  }
}

// Reads the counters out (wave-wide bit counts per position), adds each
// program's count to its LDS counter or accumulator line, and clears them.
// Program p's rows are counted at bit positions p, p + B, ... of the words.
__device__ __forceinline__ void hs_flush(Hs& s, const CONSTANT LutPass* P, unsigned long long* gacc,
                         const uint32_t* acc_index, uint32_t* accl, uint32_t nacc, uint32_t lane) {
  uint32_t planes[4 + kHsLevels] = {s.ones, s.twos, s.fours, s.eights};
#pragma unroll
  for (int k = 0; k < kHsLevels; ++k) planes[4 + k] = s.h[k];
  uint32_t used = 0;   // planes with a bit set in some lane
#pragma unroll
  for (int k = 0; k < 4 + kHsLevels; ++k) used |= (__ballot(planes[k] != 0u) != 0ull ? 1u : 0u) << k;
  const uint32_t B = P->bits, pb = P->prog_begin, pn = P->prog_count;
  for (uint32_t p = 0; p < pn; ++p) {
    uint32_t c = 0;
    for (uint32_t q = p; q < 32; q += B) {
#pragma unroll
      for (int k = 0; k < 4 + kHsLevels; ++k)
        if ((used >> k) & 1u) c += (uint32_t)__popcll(__ballot((planes[k] >> q) & 1u)) << k;
    }
    if (lane == 0 && c) {
      if (pb + p < nacc) atomicAdd(&accl[pb + p], c);
      else atomicAdd(&gacc[(uint64_t)acc_index[pb + p] * kBatchAccStride], (unsigned long long)c);
    }
  }
  s = Hs{};
}

// Start of a segment: accumulators to the pass's initial value, the rows in
// range (partial tile), and the columns that only null tests read (no
// data), which come last in the pass.
template <int D, int R>
__device__ __forceinline__ void lut_start(const CONSTANT LutPass* P, const CONSTANT LutCol* cols,
                                          uint64_t tb, bool full, int seg, uint32_t lane,
                                          uint32_t (&acc)[R][D], uint32_t& inr) {
  constexpr int S = R / 4;
  const uint64_t nrows = P->nrows;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const uint32_t v = P->init[d];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][d] = v;
  }
  inr = ~0u;
  if (!full) {
    inr = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      inr |= (uint32_t)(tb + 256u * (uint32_t)(seg * S + (r >> 2)) + 4u * lane + (uint32_t)(r & 3) < nrows) << r;
  }
  const uint32_t cb = P->col_begin, cn = P->col_count;
  for (uint32_t c = P->ndata; c < cn; ++c) {
    const CONSTANT LutCol* C = cols + cb + c;
    const uint32_t V = lseg_valid<R>(C->valid, tb, seg * S, lane, nrows, full);
    const CONSTANT uint32_t* e = (const CONSTANT uint32_t*)C->gtab;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint32_t e0 = e[d], e1 = e[D + d];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r][d] |= (V >> r) & 1u ? e0 : e1;
    }
  }
}

// Calls f(integral_constant<int, k>) for k = 0 .. N-1, unrolled whatever
// the size of f's body (slot indexes must stay compile-time constants for
// the slots to live in registers).
template <class F, int... K>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// Every column of a pass on one tile, in segments of R = 4 S rows per lane
// (S steps): the loads of all the segment's data columns and of their
// validity words are issued together, unconditionally, into register slots
// of S vectors (an int64 column takes two slots), so that a wave keeps
// every column of its segment in flight; other waves hide the latency while
// it waits.  Rows past the table read zeros or neighbouring values and are
// not counted.
template <int D, int R>
__device__ __forceinline__ void lut_tile(const CONSTANT LutPass* P, const CONSTANT LutCol* cols,
                                         const LutArgs& a, uint64_t tb, uint32_t lane,
                                         const uint32_t* lds, Hs& hs) {
  static_assert(R == 4 || R == 8, "segments of one or two steps");
  constexpr int S = R / 4, NSEG = kSteps / S;
  const bool full = tb + kTileRows <= P->nrows;
  const uint64_t nrows = P->nrows;
  const uint64_t rows = nrows - tb < (uint64_t)kTileRows ? nrows - tb : (uint64_t)kTileRows;
  const CONSTANT LutCol* cb = cols + P->col_begin;
  uint32_t acc[R][D];
  uint32_t inr;
  v4i buf[S * kLutSlots];
  uint32_t vr[kLutSlots][S];
  // decoded once per tile (what does not fit in scalar registers moves to
  // lanes of vector registers, cheaper than reloading it per segment)
  SlotD sd[kLutSlots];
  static_for<kLutSlots>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    sd[k] = slot_decode(P, cb, k, tb, rows);
  });
  for (int seg = 0; seg < NSEG; ++seg) {
    const int j0 = seg * S;
    static_for<kLutSlots>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t ty = sd[k].info & 15u;
      const uint32_t width = ty == T_I8 ? 1u : ty == T_I16 ? 2u : ty == T_I32 ? 4u : 8u;
      slot_issue<S>(buf + S * k,
                    __builtin_amdgcn_make_buffer_rsrc((void*)sd[k].data, (short)0, (int)sd[k].bytes, 0x00020000),
                    width, j0, lane);
      const __amdgpu_buffer_rsrc_t vrs =
          __builtin_amdgcn_make_buffer_rsrc((void*)sd[k].valid, (short)0, (int)sd[k].vbytes, 0x00020000);
#pragma unroll
      for (int st = 0; st < S; ++st)
        vr[k][st] = __builtin_amdgcn_raw_buffer_load_b32(vrs, (int)(4u * ((lane >> 3) + 8u * (uint32_t)(j0 + st))), 0, 0);
    });
    lut_start<D, R>(P, cols, tb, full, seg, lane, acc, inr);
    static_for<kLutSlots>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const SlotD& d = sd[k];
      if (!(d.info & kSdData)) return;
      uint32_t V = 0xFFu;
      if (d.info & kSdNullable) {
        V = 0;
#pragma unroll
        for (int st = 0; st < S; ++st) V |= ((vr[k][st] >> (4 * (lane & 7))) & 0xFu) << (4 * st);
      }
      switch (d.info & 15u) {
        case T_I8: lut_col<D, R, T_I8, R, 0>(buf + S * k, d, a, V, lds, P, acc); break;
        case T_I16: lut_col<D, R, T_I16, R, 0>(buf + S * k, d, a, V, lds, P, acc); break;
        case T_I32: lut_col<D, R, T_I32, R, 0>(buf + S * k, d, a, V, lds, P, acc); break;
        default:
          if constexpr (k + 1 < (int)kLutSlots) lut_col<D, R, T_I64, R, 0>(buf + S * k, d, a, V, lds, P, acc);
          break;
      }
    });
    lut_count<D, R>(acc, P, inr, hs);
  }
}

// Per workgroup, per-program counts accumulate in LDS and go to the
// accumulator lines at the end, as in k_batch; the last workgroup by ticket
// moves the finished lines out.  The workgroup takes groups of nw tiles
// (pass ranges are padded to kLutTileAlign), and copies a pass's LDS tables
// from device memory when it moves to that pass.
// Workgroup of the lookup-table kernel (one per CU, whose LDS it takes):
// twelve waves, three per SIMD (168 vector registers each); with four
// accumulator dwords the segments hold four rows per lane instead of eight,
// which fits 128 registers and so sixteen waves, four per SIMD.
template <int D>
constexpr uint32_t lbatch_threads() { return D == 4 ? 1024u : 768u; }

template <int D, int R>
__global__ void __launch_bounds__(lbatch_threads<D>()) k_lbatch(LutArgs a) {
  extern __shared__ __align__(16) uint32_t dyn[];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t nacc = a.acc_words;
  uint32_t* accl = dyn;
  uint32_t* lds = dyn + nacc;
  for (uint32_t p = threadIdx.x; p < nacc; p += blockDim.x) accl[p] = 0;
  __syncthreads();
  const CONSTANT LutPass* passes = (const CONSTANT LutPass*)a.passes;
  const CONSTANT LutCol* cols = (const CONSTANT LutCol*)a.cols;
  const uint64_t ngroups = a.total_tiles / nw;
  uint32_t staged = 0xFFFFFFFFu;
  const CONSTANT LutPass* P = nullptr;
  Hs hs{};
  uint32_t since = 0;
  for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const uint64_t flat = g * nw + wave;
    uint32_t lo = 0, hi = a.npasses;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (passes[mid].tile_begin <= flat) lo = mid; else hi = mid;
    }
    lo = uni(lo);
    if (passes[lo].dwords != (uint32_t)D) continue;   // another launch's pass
    if (lo != staged) {
      if (P) {
        hs_flush(hs, P, a.acc, a.acc_index, accl, nacc, lane);
        since = 0;
      }
      P = passes + lo;
      __syncthreads();
      for (uint32_t c = 0; c < P->col_count; ++c) {
        const CONSTANT LutCol* C = cols + P->col_begin + c;
        if (C->lds_word == kNoLds) continue;
        const uint32_t entries = C->kind == LK_DIRECT ? C->n + 4 : C->n + 3;
        const uint32_t words = entries * P->dwords;
        const GLOBAL uint32_t* src = gptr<uint32_t>(C->gtab);
        uint32_t* dst = lds + C->lds_word;
        for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
      }
      __syncthreads();
      staged = lo;
    }
    const uint64_t local = flat - P->tile_begin;
    if (local >= P->ntiles) continue;   // padding
    // the wave's tile start is wave-uniform: say so, so that the buffer
    // resources built from it stay in scalar registers
    const uint64_t tb = uni64(P->row_begin + local * kTileRows);
    lut_tile<D, R>(P, cols, a, tb, lane, lds, hs);
    if (++since == kLutFlushTiles) {
      hs_flush(hs, P, a.acc, a.acc_index, accl, nacc, lane);
      since = 0;
    }
  }
  if (P) hs_flush(hs, P, a.acc, a.acc_index, accl, nacc, lane);
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < nacc && p < a.nprogs; p += blockDim.x)
    if (accl[p]) atomicAdd(&a.acc[(uint64_t)a.acc_index[p] * kBatchAccStride], (unsigned long long)accl[p]);
  atomics_done();
  __syncthreads();
  __shared__ bool last;
  if (threadIdx.x == 0) {
    const unsigned int ticket = atomicAdd(&a.slot->ticket, 1u);
    last = ticket == gridDim.x - 1;
  }
  __syncthreads();
  if (last) {
    for (uint32_t k = threadIdx.x; k < a.ndone; k += blockDim.x) {
      const uint64_t line = a.done ? a.done[k] : k;
      a.out[k] = atomicExch(&a.acc[line * kBatchAccStride], 0ull);
    }
    atomics_done();
    __syncthreads();
    if (threadIdx.x == 0) atomicExch(&a.slot->ticket, 0u);
  }
}

__global__ void k_fill(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace

// Workspace of sel_pushdown_rowids_noalloc: a fixed array in each device's
// copy of the code object, for callers that cannot allocate device memory.
// In host code `scratch` names a host-side stand-in, not a device address;
// kernels receive the address that sel_noalloc_scratch looked up for the
// current device.
static __device__ __align__(256) uint8_t scratch[sel::kNoAllocScratchBytes];

int sel_noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> address of its array
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (p == nullptr) return (int)hipErrorInvalidSymbol;
    it = addr.emplace(device, p).first;
  }
  *ptr = it->second;
  return 0;
}

int sel_launch_scan(int mode, const ScanArgs& a, uint32_t grid, uint32_t block, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const uint32_t lds = a.nstage ? 4u * a.stage_words : 0u;
  const bool nt = !a.cached;
  switch (mode) {
    case M_COUNT:
      if (nt) hipLaunchKernelGGL((k_scan<M_COUNT, true>), dim3(grid), dim3(block), lds, s, a.prog, a);
      else hipLaunchKernelGGL((k_scan<M_COUNT, false>), dim3(grid), dim3(block), lds, s, a.prog, a);
      break;
    case M_MASK:
      if (nt) hipLaunchKernelGGL((k_scan<M_MASK, true>), dim3(grid), dim3(block), lds, s, a.prog, a);
      else hipLaunchKernelGGL((k_scan<M_MASK, false>), dim3(grid), dim3(block), lds, s, a.prog, a);
      break;
    default: hipLaunchKernelGGL((k_scan<M_KEYBITMAP, true>), dim3(grid), dim3(block), lds, s, a.prog, a); break;
  }
  return (int)hipGetLastError();
}

int sel_launch_scan_tiles(const uint32_t* counts, uint32_t* offsets, uint32_t* chunk_sums,
                          uint32_t* chunk_offs, uint64_t n, void* stream) {
  const uint64_t nchunks = (n + 1023) / 1024;
  if (nchunks == 0) return 0;
  if (nchunks > 2048) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chunk_scan, dim3((uint32_t)nchunks), dim3(1024), 0, (hipStream_t)stream,
                     counts, offsets, chunk_sums, n);
  hipLaunchKernelGGL(k_chunk_offsets, dim3(1), dim3(1024), 0, (hipStream_t)stream, chunk_sums,
                     chunk_offs, nchunks);
  return (int)hipGetLastError();
}

int sel_launch_compact(const CompactArgs& a, uint32_t grid, uint32_t block, void* stream) {
  hipLaunchKernelGGL(k_compact, dim3(grid), dim3(block), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int sel_launch_gather(const GatherArgs& a, uint32_t grid, uint32_t block, void* stream) {
  hipLaunchKernelGGL(k_gather, dim3(grid), dim3(block), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int sel_launch_tables(const TableBuild* d_builds, uint32_t nbuilds, uint64_t nentries, void* stream) {
  if (nbuilds == 0 || nentries == 0) return 0;
  uint64_t blocks = (nentries + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_tables, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, d_builds,
                     nbuilds, nentries);
  return (int)hipGetLastError();
}

int sel_launch_fill(uint32_t* p, uint64_t nwords, uint32_t value, void* stream) {
  if (nwords == 0) return 0;
  uint64_t blocks = (nwords + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, p, nwords, value);
  return (int)hipGetLastError();
}

int sel_scan_occupancy(int mode, uint32_t block, int* blocks_per_cu) {
  hipError_t e;
  switch (mode) {
    case M_COUNT: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_scan<M_COUNT, true>, block, 0); break;
    case M_MASK: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_scan<M_MASK, true>, block, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_scan<M_KEYBITMAP, true>, block, 0); break;
  }
  return (int)e;
}

int sel_launch_batch(const BatchArgs& a, uint32_t grid, uint32_t block, uint32_t lds_bytes,
                     void* stream) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), lds_bytes, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int sel_batch_occupancy(uint32_t block, uint32_t lds_bytes, int* blocks_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch, block, lds_bytes);
}

int sel_launch_luts(const LutArgs& a, void* stream) {
  if (a.nbuilds == 0 || a.nentries == 0) return 0;
  uint64_t blocks = (a.nentries + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_luts, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

// The lookup-table kernel for passes of `dwords` accumulator dwords per row,
// with `rows` rows per lane per segment (the larger choice, or half of it).
namespace {
const void* lbatch_kernel(uint32_t dwords, uint32_t rows) {
  switch (dwords) {
    case 1: return rows == 4 ? (const void*)k_lbatch<1, 4> : (const void*)k_lbatch<1, 8>;
    case 2: return rows == 4 ? (const void*)k_lbatch<2, 4> : (const void*)k_lbatch<2, 8>;
    default: return (const void*)k_lbatch<4, 4>;   // four rows per lane: sixteen waves fit
  }
}
}  // namespace

int sel_launch_lbatch(const LutArgs& a, uint32_t dwords, uint32_t rows, uint32_t grid, uint32_t block,
                      uint32_t lds_bytes, void* stream) {
  if (block == 0 || block > sel_lbatch_block(dwords) || block % kWave) return (int)hipErrorInvalidValue;
  LutArgs args = a;
  void* kargs[] = {&args};
  return (int)hipLaunchKernel(lbatch_kernel(dwords, rows), dim3(grid), dim3(block), kargs, lds_bytes,
                              (hipStream_t)stream);
}

uint32_t sel_lbatch_block(uint32_t dwords) {
  return dwords == 1 ? lbatch_threads<1>() : dwords == 2 ? lbatch_threads<2>() : lbatch_threads<4>();
}

int sel_lbatch_occupancy(uint32_t dwords, uint32_t rows, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, lbatch_kernel(dwords, rows), block,
                                                           lds_bytes);
}
