// Random-program fuzz of the host-side program compiler (compile.cpp), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Programs are random postfix sequences: every
// opcode (and invalid ones), literals at and past each column type's
// limits, pool offsets inside, at the end of and past the pool (aligned and
// not), IN and CODESET lengths up to past their limits, sequences longer
// than SEL_MAX_INSTRS and nestings deeper than SEL_MAX_DEPTH.  The compiler
// must return a status for each without touching memory it does not own;
// an accepted program must satisfy the limits the kernels rely on (at most
// two device instructions per input instruction, since <> becomes NOT of a
// RANGE; a stack of depth 1..SEL_MAX_DEPTH; constant references inside the
// uploaded blob).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "sel.h"
#include "sel_device.h"
#include "sel_internal.h"

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next() {
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t below(uint64_t n) { return n ? next() % n : 0; }

int64_t literal(uint32_t ty) {
  static const int64_t edges[] = {0, 1, -1, 127, 128, -128, -129, 32767, 32768, -32768, -32769,
                                  2147483647ll, 2147483648ll, -2147483648ll, -2147483649ll,
                                  std::numeric_limits<int64_t>::max(),
                                  std::numeric_limits<int64_t>::min()};
  switch (below(3)) {
    case 0: return edges[below(sizeof edges / sizeof edges[0])];
    case 1: return (int64_t)below(100) - 50;
    default: return (int64_t)next();
  }
  (void)ty;
}

uint32_t pool_offset(uint32_t pool_bytes) {
  switch (below(5)) {
    case 0: return 0;
    case 1: return (uint32_t)(below(pool_bytes + 1) & ~7u);
    case 2: return (uint32_t)below(pool_bytes + 64);          // any alignment, maybe past the end
    case 3: return pool_bytes;                                 // exactly the end
    default: return (uint32_t)next();                          // anywhere
  }
}

}  // namespace

int main(int argc, char** argv) {
  const long iters = argc > 1 ? std::atol(argv[1]) : 200000;
  long accepted = 0, rejected = 0, hashed_lists = 0;
  std::vector<uint8_t> pool;
  for (long it = 0; it < iters; ++it) {
    // a table of 1..6 columns of random types, some nullable, some coded
    const uint32_t ncols = 1 + (uint32_t)below(6);
    std::vector<sel::ColInfo> cols(ncols);
    static int64_t dummy_data[4];
    static uint32_t dummy_valid[4];
    for (auto& c : cols) {
      c.type = 1 + (uint32_t)below(4);
      c.dict_card = below(3) == 0 ? (uint32_t)below(5000) : 0;
      c.nullable = below(2) == 0;
      c.data = dummy_data;
      c.valid = c.nullable ? dummy_valid : nullptr;
    }
    // a pool of random bytes
    const uint32_t pool_bytes = below(4) == 0 ? 0 : (uint32_t)below(4096);
    pool.resize(pool_bytes);
    for (auto& b : pool) b = (uint8_t)next();
    // a random postfix sequence; half of them well formed (valid columns,
    // pool references in bounds, the stack reduced to one value)
    const bool tidy = below(2) == 0;
    const uint32_t n = below(10) == 0 ? (uint32_t)below(80) : 1 + (uint32_t)below(24);
    std::vector<sel_instr> code(n);
    int depth = 0;
    for (auto& in : code) {
      std::memset(&in, 0, sizeof in);
      uint32_t op;
      const uint32_t left = n - (uint32_t)(&in - code.data());   // this one included
      if (!tidy && below(20) == 0) {
        op = (uint32_t)below(40);                            // any value, valid or not
      } else if (tidy && depth >= 2 && (uint32_t)(depth - 1) >= left) {
        op = below(2) ? SEL_OP_AND : SEL_OP_OR;              // reduce before the end
      } else if (depth >= 2 && below(2) == 0) {
        op = below(2) ? SEL_OP_AND : SEL_OP_OR;
      } else if (depth >= 1 && below(6) == 0) {
        op = below(2) ? SEL_OP_NOT : SEL_OP_IS_UNKNOWN;
      } else {
        op = 1 + (uint32_t)below(11);                        // a leaf
        if (below(30) == 0) op = below(2) ? SEL_OP_TRUE : SEL_OP_FALSE;
      }
      in.op = (uint16_t)op;
      in.col = (uint16_t)(!tidy && below(15) == 0 ? below(70) : below(ncols));
      const uint32_t ty = in.col < ncols ? cols[in.col].type : 3;
      in.a = literal(ty);
      in.b = literal(ty);
      if (op == SEL_OP_IN) {
        if (tidy && pool_bytes >= 8) {
          const uint32_t k = 1 + (uint32_t)below(pool_bytes / 8);
          in.b = k;
          in.aux = 8 * (uint32_t)below(pool_bytes / 8 - k + 1);
        } else {
          in.aux = pool_offset(pool_bytes);
          in.b = below(8) == 0 ? (int64_t)next() : (int64_t)below(pool_bytes / 8 + 3);
        }
      } else if (op == SEL_OP_CODESET) {
        if (tidy && pool_bytes >= 4) {
          const uint32_t words = 1 + (uint32_t)below(pool_bytes / 4);
          in.b = 32 * (int64_t)words - (int64_t)below(32);
          in.aux = 4 * (uint32_t)below(pool_bytes / 4 - words + 1);
        } else {
          in.aux = pool_offset(pool_bytes);
          in.b = below(8) == 0 ? (int64_t)next() : (int64_t)below(pool_bytes * 8 + 64);
        }
      }
      if (op >= SEL_OP_EQ && op <= SEL_OP_IS_NOT_NULL) ++depth;
      else if (op == SEL_OP_TRUE || op == SEL_OP_FALSE) ++depth;
      else if (op == SEL_OP_AND || op == SEL_OP_OR) --depth;
    }
    sel::Lowered L;
    std::string err;
    const int st = sel::lower_program(cols.data(), ncols, code.data(), n,
                                      pool_bytes ? pool.data() : nullptr, pool_bytes, L, err);
    if (st == SEL_OK) {
      ++accepted;
      if (L.code.empty() || L.code.size() > 2 * SEL_MAX_INSTRS || L.depth < 1 || L.depth > SEL_MAX_DEPTH) {
        std::fprintf(stderr, "accepted program breaks a limit: %zu instructions, depth %d\n",
                     L.code.size(), L.depth);
        return 1;
      }
      for (size_t k = 0; k < L.aux_is_offset.size(); ++k)
        if (L.aux_is_offset[k] && (uintptr_t)L.code[k].aux >= L.blob.size()) {
          std::fprintf(stderr, "aux offset %zu past the blob (%zu bytes)\n",
                       (size_t)(uintptr_t)L.code[k].aux, L.blob.size());
          return 1;
        }
      // a hashed IN list's cuckoo tables answer membership exactly as its
      // sorted list does: on every member, its neighbours and random values
      for (size_t k = 0; k < L.code.size(); ++k) {
        const sel::DevInstr& I = L.code[k];
        if (I.op != sel::D_INLIST || !(I.flags & sel::F_HASHED)) continue;
        const uint32_t b = sel::in_hash_bits(I.flags), pr = sel::in_hash_pair(I.flags);
        const size_t m = size_t(1) << b, off = (size_t)(uintptr_t)I.aux;
        if (off + 8 * (I.n + 2 * m) > L.blob.size()) {
          std::fprintf(stderr, "hashed IN list past the blob\n");
          return 1;
        }
        std::vector<int64_t> v(I.n), t(2 * m);
        std::memcpy(v.data(), L.blob.data() + off, 8 * v.size());
        std::memcpy(t.data(), L.blob.data() + off + 8 * v.size(), 8 * t.size());
        auto hit = [&](int64_t x) {
          return t[sel::in_hash(x, sel::kInHashMul[pr][0], b)] == x ||
                 t[m + sel::in_hash(x, sel::kInHashMul[pr][1], b)] == x;
        };
        std::vector<int64_t> probes;
        for (int64_t x : v) {
          probes.push_back(x);
          probes.push_back((int64_t)((uint64_t)x + 1));
          probes.push_back((int64_t)((uint64_t)x - 1));
        }
        for (int r = 0; r < 64; ++r) probes.push_back((int64_t)next());
        for (int64_t x : probes)
          if (hit(x) != std::binary_search(v.begin(), v.end(), x)) {
            std::fprintf(stderr, "cuckoo tables disagree with the list on %lld\n", (long long)x);
            return 1;
          }
        ++hashed_lists;
      }
    } else {
      ++rejected;
      if (st != SEL_E_INVALID && st != SEL_E_TYPE) {
        std::fprintf(stderr, "unexpected status %d: %s\n", st, err.c_str());
        return 1;
      }
    }
  }
  std::printf("fuzz: %ld programs, %ld accepted, %ld rejected, %ld hashed IN lists checked\n", iters, accepted,
              rejected, hashed_lists);
  return accepted > 0 && rejected > 0 && hashed_lists > 0 ? 0 : 1;
}
