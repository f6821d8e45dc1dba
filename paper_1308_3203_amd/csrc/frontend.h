// frontend.h -- parse, validate and compile kernel-language text to bytecode.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace rc {

struct CompiledArray {
  std::string name;
  uint32_t size = 0;
  bool global = false;
  bool written = false;   // some store targets it: its accesses can pair
};

struct Compiled {
  std::string name;
  std::vector<CompiledArray> arrays;   // global arrays first, then local arrays
  std::vector<std::string> scalars;
  std::vector<std::string> vars;
  std::vector<uint32_t> code;          // 4 words per instruction
  uint32_t n_global = 0, n_local = 0, nregs = 0, n_stmts = 0;
  // static bounds for one work-item (both branches of every if counted)
  uint64_t dyn_instr = 0;              // instructions executed
  uint64_t dyn_logged_mem = 0;         // loads/stores on written arrays
  uint64_t dyn_logged_local = 0;       // ... of which on written local arrays
  uint64_t dyn_mem = 0;                // all loads/stores
  uint64_t dyn_stores = 0;             // store statements
  std::vector<uint64_t> dyn_mem_array; // loads/stores per array
  uint64_t max_intervals = 1;          // 1 + barriers executed
  uint64_t dyn_iters = 0;              // loop iterations started
  // largest interval (accesses per work-item between two barriers) on
  // written local arrays / on all written arrays
  double interval_logged_local = 0, interval_logged_all = 0;
  // triage features 0..103: statement mix, affine index analysis, barrier
  // structure (independent of the launch shape and the bindings)
  float feat[104] = {};
};

// Returns true on success; on failure `err` holds "line:col: message" and
// `is_limit` tells a limit violation from a syntax or name error.
bool compile_program(const char* src, size_t len, Compiled* out, std::string* err, bool* is_limit);

}  // namespace rc
