// Sanitizer driver for the library's host-side C++ (the front end and the
// static proofs), built with -fsanitize=address,undefined by
// tests/test_sanitizers.py.  Each argument is a case file as for the oracle
// driver ("G W lo hi seed0 n_seeds", then the program text).  For each it
// prints "<case> <instructions> <registers> <never_faults> <owned flags>"
// or "<case> compile-error".
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "../../paper_1308_3203_amd/csrc/frontend.h"
#include "../../paper_1308_3203_amd/csrc/ownership.h"

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    std::ifstream f(argv[a], std::ios::binary);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string all = ss.str();
    const size_t nl = all.find('\n');
    unsigned G = 0, W = 0;
    if (nl == std::string::npos || std::sscanf(all.c_str(), "%u %u", &G, &W) != 2) {
      std::fprintf(stderr, "bad header in %s\n", argv[a]);
      return 2;
    }
    const std::string src = all.substr(nl + 1);
    rc::Compiled c;
    std::string err;
    bool is_limit = false;
    if (!rc::compile_program(src.data(), src.size(), &c, &err, &is_limit)) {
      std::printf("%s compile-error\n", argv[a]);
      continue;
    }
    const rc::Ownership o = rc::prove_ownership(c, G, W);
    std::string flags;
    for (const auto& x : o.arrays) flags += x.owned ? 'o' : (x.race_free ? 'r' : '-');
    std::printf("%s %zu %u %d %s\n", argv[a], c.code.size() / 4, c.nregs, o.never_faults ? 1 : 0, flags.c_str());
  }
  return 0;
}
