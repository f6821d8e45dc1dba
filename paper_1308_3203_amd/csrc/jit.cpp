// jit.cpp -- per-program kernels.  A program's bytecode is translated into
// straight-line HIP source (one block per instruction, labels and gotos for
// the jumps), calling the same Item runtime the interpreter calls, and
// compiled with hipRTC for gfx950.  Private variables become registers of
// the generated code instead of LDS words, and the instruction dispatch
// disappears; the semantics (masks, step numbering, faults, logs) are the
// interpreter's, instruction for instruction.
#include "jit.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "rc_internal.h"

namespace rc {

#include "_gen_jit_headers.inc"   // kJitHeaderNames, kJitHeaders, kJitHeaderCount

namespace {

std::string operand(bool imm, uint32_t w) {
  char buf[64];
  if (imm) snprintf(buf, sizeof buf, "(int32_t)0x%08xu", w);
  else if (w < MAX_REGS) snprintf(buf, sizeof buf, "R%u", w);
  else snprintf(buf, sizeof buf, "it.special(%uu)", w);
  return buf;
}

// The memory statements that keep their group step when the kernel elides
// the others (RC_JIT_ELIDE: the program cannot fault and its intervals fit
// the LDS log).  A step is kept where an access since the group's last
// synchronisation conflicts with the statement's: a load of an array stored
// to, or a store to an array loaded (stores of one cell are ordered by their
// version words).  Barriers and branch votes synchronise the group, and so
// does a kept step; the statements of a loop body also follow the body's
// own end.  Arrays whose accesses never take the step (read-only or owned)
// cannot conflict; with number_global, statements on an array logged to the
// global log keep the step, which numbers its entries.  A kept step on a
// logged local array synchronises only in the intervals whose local
// accesses are logged (in the others the runtime skips it, every local
// array being race-free there).  Unless every interval is logged, such a
// step therefore settles only what a skipped step cannot break: the local
// arrays (race-free whenever it is skipped) and, with number_global, the
// arrays logged globally (each of their statements keeps its own step).
// A global array logged in LDS (one group), or logged globally on the
// interpreter's elided path, stays pending across it.
}  // namespace

std::vector<uint8_t> group_steps(const std::vector<uint32_t>& code, const JitShape& shape, bool number_global) {
  const uint32_t n = (uint32_t)(code.size() / 4), na = shape.n_arrays;
  std::vector<uint8_t> keep(n, 0);
  auto field = [&](uint32_t a, uint32_t f) { return shape.arrays[a * JIT_ARRAY_WORDS + f]; };
  const bool every_interval_logged = shape.log_mask == ~0ull && shape.log_high != 0u;
  auto may_be_quiet = [&](uint32_t a) {
    return !every_interval_logged && field(a, 0) == AK_LOCAL && field(a, 2) != LOG_NONE;
  };
  std::map<uint32_t, std::vector<uint8_t>> back;   // first body instruction -> accesses at the body's end
  for (bool changed = true; changed;) {
    changed = false;
    std::vector<uint8_t> S(na, 0);   // per array: bit 0 loaded, bit 1 stored since the last synchronisation
    for (uint32_t i = 0; i < n; ++i) {
      const auto b = back.find(i);
      if (b != back.end())
        for (uint32_t a = 0; a < na; ++a) S[a] |= b->second[a];
      const uint32_t h = code[4 * i], op = h & 63u, wc = code[4 * i + 3];
      if (op == OP_LOAD || op == OP_STORE) {
        if (wc >= na || (wc + 1) * JIT_ARRAY_WORDS > shape.arrays.size()) {
          keep[i] = 1;
          std::fill(S.begin(), S.end(), 0);
          continue;
        }
        if (field(wc, 8)) continue;   // nosync
        const uint8_t bit = op == OP_LOAD ? 1 : 2, other = op == OP_LOAD ? 2 : 1;
        if (((number_global && field(wc, 2) == LOG_GLOBAL) || (S[wc] & other)) && !keep[i]) {
          keep[i] = 1;
          changed = true;
        }
        if (keep[i]) {
          if (!may_be_quiet(wc)) {
            std::fill(S.begin(), S.end(), 0);
          } else {
            for (uint32_t a = 0; a < na; ++a)
              if (field(a, 0) == AK_LOCAL || (number_global && field(a, 2) == LOG_GLOBAL)) S[a] = 0;
          }
        }
        S[wc] |= bit;
      } else if (op == OP_IF || op == OP_BARRIER) {
        std::fill(S.begin(), S.end(), 0);
      } else if (op == OP_ENDFOR) {
        std::vector<uint8_t>& e = back[wc];
        if (e.empty()) e.assign(na, 0);
        for (uint32_t a = 0; a < na; ++a) {
          if ((e[a] | S[a]) != e[a]) {
            e[a] |= S[a];
            changed = true;
          }
        }
      }
    }
  }
  return keep;
}

std::string jit_source(const std::vector<uint32_t>& code, uint32_t nregs, uint32_t threads,
                       const std::vector<uint32_t>& array_kind, const JitShape& shape) {
  const uint32_t n = (uint32_t)(code.size() / 4);
  std::set<uint32_t> targets;
  std::set<uint32_t> slots;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t h = code[4 * i], op = h & 63u;
    if (op == OP_IF) targets.insert(code[4 * i + 2]);
    if (op == OP_ELSE || op == OP_FOR || op == OP_ENDFOR) targets.insert(code[4 * i + 3]);
    if (op == OP_FOR || op == OP_ENDFOR) slots.insert((h >> 8) & 63u);
  }
  std::string s;
  char buf[512];
  // the launch shape, folded by the runtime (item_rt.h checks every item's
  // descriptor against it)
  snprintf(buf, sizeof buf,
           "#define RC_JIT_W %uu\n#define RC_JIT_G %uu\n#define RC_JIT_NA %uu\n#define RC_JIT_TB %uu\n"
           "#define RC_JIT_TC %uu\n#define RC_JIT_LC %uu\n",
           shape.W, shape.G, shape.n_arrays, shape.tab_base, shape.tab_cells, shape.lds_log_cap);
  s += buf;
  if (shape.nospill) s += "#define RC_JIT_NOSPILL 1\n";
  if (shape.nofault) s += "#define RC_JIT_NOFAULT 1\n";
  snprintf(buf, sizeof buf, "#define RC_JIT_LOGMASK 0x%016llxull\n#define RC_JIT_LOGHIGH %uu\n",
           (unsigned long long)shape.log_mask, shape.log_high);
  s += buf;
  const bool elide = shape.nofault && shape.nospill;
  if (elide) s += "#define RC_JIT_ELIDE 1\n";
  const std::vector<uint8_t> keep = elide ? group_steps(code, shape, true) : std::vector<uint8_t>(n, 1);
  // the arrays' descriptor fields the shape fixes
  s += "#define RC_JIT_ARRAYS 1\n#ifndef __HIPCC_RTC__\n#include <hip/hip_runtime.h>\n#endif\n"
       "#include \"rc_internal.h\"\n\nnamespace rc {\n\n"
       "__device__ __forceinline__ void jit_array(uint32_t a, ArrayDesc& A) {\n  switch (a) {\n";
  for (uint32_t a = 0; a < shape.n_arrays && (a + 1) * JIT_ARRAY_WORDS <= shape.arrays.size(); ++a) {
    const uint32_t* f = &shape.arrays[a * JIT_ARRAY_WORDS];
    snprintf(buf, sizeof buf,
             "    case %uu: A.kind = %uu; A.size = %uu; A.logged = %uu; A.offset = %uu; A.cellbase = %uu;\n"
             "      A.own_stride = %d; A.own_lo = %d; A.own_span = %uu; A.nosync = %uu; break;\n",
             a, f[0], f[1], f[2], f[3], f[4], (int32_t)f[5], (int32_t)f[6], f[7], f[8]);
    s += buf;
  }
  s += "    default: break;\n  }\n}\n\n}  // namespace rc\n\n";
  s += "#include \"item_rt.h\"\n\nnamespace {\n\n__device__ __forceinline__ void jit_item(rc::Item& it) {\n";
  s += "  using namespace rc;\n";
  for (uint32_t r = 0; r < nregs; ++r) {
    snprintf(buf, sizeof buf, "  int32_t R%u = 0;\n", r);
    s += buf;
  }
  for (uint32_t sl : slots) {
    snprintf(buf, sizeof buf, "  uint32_t LC%u = 0u;\n", sl);
    s += buf;
  }
  s += "  uint32_t mbits = it.real ? 1u : 0u, ebits = 0u, eany = 0u;\n";
  s += "  (void)ebits; (void)eany;\n";
  uint32_t depth = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t h = code[4 * i], wa = code[4 * i + 1], wb = code[4 * i + 2], wc = code[4 * i + 3];
    const uint32_t op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u, spc = h >> 20;
    const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
    if (targets.count(i)) {
      snprintf(buf, sizeof buf, "L%u:;\n", i);
      s += buf;
    }
    snprintf(buf, sizeof buf, "  it.stmt(%uu);\n", spc);
    s += buf;
    char act[64];
    snprintf(act, sizeof act, "((mbits >> %uu) & 1u)", depth);
    switch (op) {
      case OP_BIN:
        snprintf(buf, sizeof buf,
                 "  { const int32_t x = %s, y = %s; bool dz = false; const int32_t r = alu_bin(%uu, x, y, dz);\n"
                 "    if (%s) { R%u = r; if (dz) it.raise(%uu, F_DIV); } }\n",
                 operand(fa, wa).c_str(), operand(fb, wb).c_str(), sub, act, dst, spc);
        s += buf;
        break;
      case OP_UN: {
        const char* e = sub == U_MOV ? "x" : sub == U_NEG ? "(int32_t)(0u - (uint32_t)x)"
                        : sub == U_BNOT ? "~x" : "(int32_t)(x == 0)";
        snprintf(buf, sizeof buf, "  { const int32_t x = %s; const int32_t r = %s; if (%s) R%u = r; }\n",
                 operand(fa, wa).c_str(), e, act, dst);
        s += buf;
        break;
      }
      case OP_LOAD:
      case OP_STORE: {
        const std::string val = op == OP_STORE ? operand(fb, wb) : std::string("0");
        const int kind = wc < array_kind.size() ? (int)array_kind[wc] : -1;
        snprintf(buf, sizeof buf,
                 "  { int32_t v = 0; if (it.mem<%d, %s>(%uu, %uu, %s, %s, %s, %uu, v)) { it.faulted = true; goto Ldone; }",
                 kind, keep[i] ? "true" : "false", op, wc, operand(fa, wa).c_str(), val.c_str(), act, spc);
        s += buf;
        if (op == OP_LOAD) {
          snprintf(buf, sizeof buf, " if (%s) R%u = v;", act, dst);
          s += buf;
        }
        s += " }\n";
        break;
      }
      case OP_IF: {
        const uint32_t d1 = depth + 1;
        snprintf(buf, sizeof buf,
                 "  { const int32_t c = %s; const bool a = %s; const bool t = a && c != 0, e = a && c == 0;\n"
                 "    mbits = (mbits & ~(1u << %uu)) | ((uint32_t)t << %uu);\n"
                 "    ebits = (ebits & ~(1u << %uu)) | ((uint32_t)e << %uu);\n"
                 "    const uint32_t any = it.group_red(t, e, false);\n"
                 "    if (any & 4u) { it.faulted = true; goto Ldone; }\n"
                 "    eany = (eany & ~(1u << %uu)) | (((any >> 1) & 1u) << %uu);\n"
                 "    if (!(any & 1u)) goto L%u; }\n",
                 operand(fa, wa).c_str(), act, d1, d1, d1, d1, d1, d1, wb);
        s += buf;
        depth = d1;
        break;
      }
      case OP_ELSE:
        snprintf(buf, sizeof buf,
                 "  mbits = (mbits & ~(1u << %uu)) | (((ebits >> %uu) & 1u) << %uu);\n"
                 "  if (!((eany >> %uu) & 1u)) goto L%u;\n",
                 depth, depth, depth, depth, wc);
        s += buf;
        break;
      case OP_ENDIF:
        --depth;
        break;
      case OP_FOR: {
        const int32_t lo = (int32_t)wa, hi = (int32_t)wb;
        snprintf(buf, sizeof buf, "  if (%s) R%u = (int32_t)0x%08xu;\n", act, dst, (uint32_t)lo);
        s += buf;
        if ((int64_t)hi - (int64_t)lo <= 0) snprintf(buf, sizeof buf, "  goto L%u;\n", wc);
        else if (shape.nofault) snprintf(buf, sizeof buf, "  LC%u = 0u;\n", sub);
        else snprintf(buf, sizeof buf, "  if (it.iter_start(%uu)) { it.faulted = true; goto Ldone; }\n  LC%u = 0u;\n", spc, sub);
        s += buf;
        break;
      }
      case OP_ENDFOR: {
        const int32_t lo = (int32_t)wa, hi = (int32_t)wb;
        const uint32_t iters = (uint32_t)((int64_t)hi - (int64_t)lo);
        // (a program proven not to fault never reaches the iteration limit)
        if (shape.nofault)
          snprintf(buf, sizeof buf,
                   "  LC%u += 1u; if (%s) R%u = (int32_t)(0x%08xu + LC%u); if (LC%u < %uu) goto L%u;\n", sub, act,
                   dst, (uint32_t)lo, sub, sub, iters, wc);
        else
          snprintf(buf, sizeof buf,
                   "  LC%u += 1u; if (%s) R%u = (int32_t)(0x%08xu + LC%u);\n"
                   "  if (LC%u < %uu) { if (it.iter_start(%uu)) { it.faulted = true; goto Ldone; } goto L%u; }\n",
                   sub, act, dst, (uint32_t)lo, sub, sub, iters, spc, wc);
        s += buf;
        break;
      }
      case OP_BARRIER:
        snprintf(buf, sizeof buf, "  if (it.barrier(%s, %uu)) { it.faulted = true; goto Ldone; }\n", act, spc);
        s += buf;
        break;
      case OP_ASSERT:
      case OP_ASSUME:
        snprintf(buf, sizeof buf, "  { const int32_t c = %s; if (%s && c == 0) it.raise(%uu, %s); }\n",
                 operand(fa, wa).c_str(), act, spc, op == OP_ASSERT ? "F_ASSERT" : "F_ASSUME");
        s += buf;
        break;
      default:  // OP_END
        s += "  if (it.end()) it.faulted = true;\n  goto Ldone;\n";
        break;
    }
  }
  s += "Ldone:;\n}\n\n}  // namespace\n\n";
  snprintf(buf, sizeof buf,
           "extern \"C\" __global__ __launch_bounds__(%u) void rc_jit_kernel(rc::PassParams PP) {\n"
           "  rc::run_items(PP, [](rc::Item& it) { jit_item(it); });\n}\n",
           threads);
  s += buf;
  return s;
}

bool jit_compile(const std::string& src, std::vector<char>* code_object, std::string* log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "rc_jit.hip", kJitHeaderCount, kJitHeaders, kJitHeaderNames) !=
      HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return false;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  log->assign(ls, '\0');
  if (ls) hiprtcGetProgramLog(prog, &(*log)[0]);
  bool ok = r == HIPRTC_SUCCESS;
  if (ok) {
    size_t cs = 0;
    ok = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
    if (ok) {
      code_object->resize(cs);
      ok = hiprtcGetCode(prog, code_object->data()) == HIPRTC_SUCCESS;
    }
  }
  hiprtcDestroyProgram(&prog);
  return ok;
}

}  // namespace rc
