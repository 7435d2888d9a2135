// sel_internal.h -- host-side structures shared by the runtime (api.cpp)
// and the program compiler (compile.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "sel_device.h"

namespace sel {

struct ColInfo {
  uint32_t type;        // DevType
  uint32_t dict_card;
  bool nullable;
  const void* data;
  const uint32_t* valid;
};

// A lowered program before upload: DevInstr::aux of instructions whose
// aux_is_offset is 1 holds a byte offset into blob (8-byte aligned).
struct Lowered {
  std::vector<DevInstr> code;
  std::vector<uint8_t> blob;
  std::vector<int> aux_is_offset;
  std::vector<uint32_t> columns;        // columns whose data is read
  std::vector<uint32_t> valid_columns;  // columns whose validity is read
  int depth = 0;
  std::string text;                     // one line per instruction
  bool merged = false;                  // range tests of a column were merged
};

// merge_ranges: range tests of one column under one conjunction become one
// test (the code the kernels run); without it the program keeps the
// conjuncts as written (the factors an independence estimate counts).
int lower_program(const ColInfo* cols, uint32_t ncols, const struct sel_instr* code, uint32_t n,
                  const uint8_t* pool, uint32_t pool_bytes, Lowered& out, std::string& err,
                  bool merge_ranges = true);
// Bytes of a leaf's constants in the blob (bitmap words, IN list and its
// cuckoo tables), 0 for a leaf without any.
size_t aux_bytes(const DevInstr& I);
std::string listing(const Lowered& L);

}  // namespace sel
