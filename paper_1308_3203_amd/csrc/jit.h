// jit.h -- per-program kernels generated from bytecode and compiled at load
// time (hipRTC); see jit.cpp.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace rc {

// The launch shape a per-program kernel is compiled for: the NDRange, the
// number of arrays and the LDS layout of the interval log (the per-cell
// table's first cell key and size, the log's capacity in entries).  The
// kernel folds them as constants; a program whose shape or tuning changes
// needs another kernel.
// arrays: per array the descriptor fields that the program and the shape
// fix (kind, size, logged, offset, cellbase, own_stride, own_lo, own_span,
// nosync; JIT_ARRAY_WORDS words each).
constexpr uint32_t JIT_ARRAY_WORDS = 9;
struct JitShape {
  uint32_t W = 0, G = 0, n_arrays = 0, tab_base = 0, tab_cells = 0, lds_log_cap = 0;
  uint32_t nospill = 0;   // every interval's LDS-logged accesses fit the LDS log
  uint32_t nofault = 0;   // the program is proven never to fault under this shape
  uint64_t log_mask = ~0ull;   // intervals whose local-array accesses are logged
  uint32_t log_high = 1;
  std::vector<uint32_t> arrays;
  bool operator==(const JitShape& o) const {
    return W == o.W && G == o.G && n_arrays == o.n_arrays && tab_base == o.tab_base && tab_cells == o.tab_cells &&
           lds_log_cap == o.lds_log_cap && nospill == o.nospill && nofault == o.nofault && log_mask == o.log_mask &&
           log_high == o.log_high && arrays == o.arrays;
  }
};

// HIP source of the kernel `rc_jit_kernel` for one program: `code` is the
// bytecode (4 words per instruction), `threads` the workgroup size it is
// launched with (64 << width class), `shape` the launch shape it is
// specialised for.
// array_kind[a] is array a's AK_* kind (fixed by the program text).
std::string jit_source(const std::vector<uint32_t>& code, uint32_t nregs, uint32_t threads,
                       const std::vector<uint32_t>& array_kind, const JitShape& shape);

// Per instruction, whether a load or store keeps its group step when a
// program that cannot fault runs with elided steps: kept where an access
// since the group's last synchronisation conflicts with it (see jit.cpp).
// number_global: statements on arrays logged to the global log keep their
// step too (their entries are numbered by it).
std::vector<uint8_t> group_steps(const std::vector<uint32_t>& code, const JitShape& shape, bool number_global);

// Compile for gfx950; false with the compiler's log on failure.
bool jit_compile(const std::string& src, std::vector<char>* code_object, std::string* log);

}  // namespace rc
