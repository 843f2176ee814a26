// User-defined point kernels (Section 5.1): an arithmetic expression over up
// to three input images, parsed once on the host into a postfix program that
// the generic kernels interpret per pixel.  Host-only.
#pragma once
#include <string>
#include <vector>

#include "hvx_desc.h"

namespace hvx {

struct ExprProg {
  std::vector<int16_t> code;   // X_* | (argument << 8)
  std::vector<double> consts;  // literal values, by index
  int max_input = -1;          // highest input index named (a = 0)
  bool needs_float = false;    // uses sqrt or a non-integer literal
  bool int_literals_ok = true; // every literal is an integer that fits 32 bits
  bool has_offsets = false;    // reads a[dx, dy] (a local kernel)
  int rx = 0, ry = 0;          // largest |dx|, |dy| read
};

// Parse `src`.  Returns an empty string on success, else what is wrong.
std::string parse_expr(const char* src, ExprProg* out);

}  // namespace hvx
