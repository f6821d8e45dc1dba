// jit.h -- per-program kernels generated from bytecode and compiled at load
// time (hipRTC); see jit.cpp.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace rc {

// HIP source of the kernel `rc_jit_kernel` for one program: `code` is the
// bytecode (4 words per instruction), `threads` the workgroup size it is
// launched with (64 << width class).
// array_kind[a] is array a's AK_* kind (fixed by the program text).
std::string jit_source(const std::vector<uint32_t>& code, uint32_t nregs, uint32_t threads,
                       const std::vector<uint32_t>& array_kind);

// Compile for gfx950; false with the compiler's log on failure.
bool jit_compile(const std::string& src, std::vector<char>* code_object, std::string* log);

}  // namespace rc
