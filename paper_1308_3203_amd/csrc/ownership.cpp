// ownership.cpp -- the owned-array proof of ownership.h: an abstract
// interpretation of the bytecode over affine forms.
#include "ownership.h"

#include <algorithm>
#include <map>
#include <unordered_map>
#include <utility>

#include "rc_internal.h"

namespace rc {

namespace {

typedef __int128 i128;
constexpr int64_t I32_MIN = -(int64_t(1) << 31), I32_MAX = (int64_t(1) << 31) - 1;
constexpr int64_t COEF_MAX = int64_t(1) << 34;   // larger coefficients: unknown
constexpr uint64_t VISIT_MAX = 20000000;         // instructions interpreted before giving up

bool fits(i128 v) { return v <= COEF_MAX && v >= -COEF_MAX; }

// c0 + cg * gid + cl * lid + sum(coef * loop counter), or unknown (top)
struct Form {
  bool top = true;
  int64_t c0 = 0, cg = 0, cl = 0;
  std::vector<std::pair<uint32_t, int64_t>> lc;   // (loop, coefficient), by loop, no zero coefficients

  bool operator==(const Form& o) const {
    if (top || o.top) return top == o.top;
    return c0 == o.c0 && cg == o.cg && cl == o.cl && lc == o.lc;
  }
};

Form unknown() { return Form(); }
Form konst(int64_t v) {
  Form f;
  f.top = false;
  f.c0 = v;
  return f;
}

struct Range {
  int64_t lo, hi;
};

class Prover {
 public:
  Prover(const Compiled& c, uint32_t G, uint32_t W) : c_(c), G_(G), W_(W) {}

  std::vector<OwnedArray> run() {
    const uint32_t na = (uint32_t)c_.arrays.size();
    std::vector<uint8_t> owned(na, 1);
    std::vector<OwnedArray> out(na);
    for (OwnedArray& o : out) o.owned = 1;
    if ((uint64_t)G_ * W_ <= 1) return out;     // one work-item: no pair exists
    std::vector<Form> env(MAX_REGS, konst(0));   // private variables start at 0
    block(0, (uint32_t)(c_.code.size() / 4), env);
    if (visits_ > VISIT_MAX) return std::vector<OwnedArray>(na);   // gave up: nothing is owned
    // per array: one stride, offsets within a range shorter than it
    std::vector<int64_t> stride(na, 0), olo(na, I32_MAX), ohi(na, I32_MIN);
    for (const auto& acc : access_) {
      const uint32_t a = acc.first.second;
      const Form& f = acc.second;
      if (!owned[a]) continue;
      if (f.top) { owned[a] = 0; continue; }
      int64_t S;
      if (W_ == 1) {
        S = f.cg;
      } else {
        S = f.cl;
        if (G_ > 1 && f.cg != S * (int64_t)W_) { owned[a] = 0; continue; }
      }
      if (S == 0 || (stride[a] != 0 && stride[a] != S)) { owned[a] = 0; continue; }
      stride[a] = S;
      Form off = f;
      off.cg = 0;
      off.cl = 0;
      const Range r = range(off);
      olo[a] = std::min(olo[a], r.lo);
      ohi[a] = std::max(ohi[a], r.hi);
      const int64_t span = S < 0 ? -S : S;
      if (ohi[a] - olo[a] >= span) owned[a] = 0;
    }
    for (uint32_t a = 0; a < na; ++a) {
      out[a].owned = owned[a];
      if (owned[a] && stride[a] != 0) {
        out[a].stride = stride[a];
        out[a].lo = olo[a];
        out[a].hi = ohi[a];
      }
    }
    return out;
  }

 private:
  const Compiled& c_;
  const uint32_t G_, W_;
  std::map<uint32_t, Range> loops_;                           // loop (its FOR index) -> counter range
  std::map<std::pair<uint32_t, uint32_t>, Form> access_;      // (instruction, array) -> index form
  uint64_t visits_ = 0;

  uint32_t word(uint32_t i, int k) const { return c_.code[4 * i + k]; }

  // the values a form takes over gid in [0, G), lid in [0, W) and the loop ranges
  // (saturated to +-2^62; coefficients are at most 2^34 and symbols int32)
  Range range(const Form& f) const {
    i128 lo = f.c0, hi = f.c0;
    auto add = [&](int64_t coef, int64_t a0, int64_t a1) {
      const i128 a = (i128)coef * a0, b = (i128)coef * a1;
      lo += std::min(a, b);
      hi += std::max(a, b);
    };
    add(f.cg, 0, (int64_t)G_ - 1);
    add(f.cl, 0, (int64_t)W_ - 1);
    for (const auto& t : f.lc) {
      const Range lr = loops_.at(t.first);
      add(t.second, lr.lo, lr.hi);
    }
    const i128 cap = (i128)1 << 62;
    return Range{(int64_t)std::max(lo, -cap), (int64_t)std::min(hi, cap)};
  }

  // drop symbols with a single value, bound the coefficients, and require
  // the value to stay inside int32 for every value of the symbols
  Form norm(Form f) const {
    if (f.top) return f;
    if (G_ == 1) f.cg = 0;
    if (W_ == 1) f.cl = 0;
    std::vector<std::pair<uint32_t, int64_t>> lc;
    for (const auto& t : f.lc) {
      const Range lr = loops_.at(t.first);
      if (lr.lo == lr.hi) {
        const i128 c0 = (i128)f.c0 + (i128)t.second * lr.lo;
        if (!fits(c0)) return unknown();
        f.c0 = (int64_t)c0;
      } else if (t.second != 0) {
        lc.push_back(t);
      }
    }
    f.lc = lc;
    const Range r = range(f);
    if (r.lo < I32_MIN || r.hi > I32_MAX) return unknown();
    return f;
  }

  // x + sy * y (sy = +-1) and k * x: exact in 128 bits, unknown when a
  // coefficient leaves +-2^34 (operands are normalised forms)
  static Form combine(const Form& x, const Form& y, int64_t sy) {
    if (x.top || y.top) return unknown();
    const i128 c0 = (i128)x.c0 + (i128)sy * y.c0, cg = (i128)x.cg + (i128)sy * y.cg,
               cl = (i128)x.cl + (i128)sy * y.cl;
    if (!fits(c0) || !fits(cg) || !fits(cl)) return unknown();
    Form r;
    r.top = false;
    r.c0 = (int64_t)c0;
    r.cg = (int64_t)cg;
    r.cl = (int64_t)cl;
    std::map<uint32_t, i128> m;
    for (const auto& t : x.lc) m[t.first] += t.second;
    for (const auto& t : y.lc) m[t.first] += (i128)sy * t.second;
    for (const auto& t : m) {
      if (!fits(t.second)) return unknown();
      if (t.second != 0) r.lc.emplace_back(t.first, (int64_t)t.second);
    }
    return r;
  }

  static bool is_const(const Form& f) { return !f.top && f.cg == 0 && f.cl == 0 && f.lc.empty(); }

  static Form scale(const Form& x, int64_t k) {
    if (x.top || !fits(k)) return unknown();
    const i128 c0 = (i128)x.c0 * k, cg = (i128)x.cg * k, cl = (i128)x.cl * k;
    if (!fits(c0) || !fits(cg) || !fits(cl)) return unknown();
    Form r;
    r.top = false;
    r.c0 = (int64_t)c0;
    r.cg = (int64_t)cg;
    r.cl = (int64_t)cl;
    for (const auto& t : x.lc) {
      const i128 v = (i128)t.second * k;
      if (!fits(v)) return unknown();
      if (v != 0) r.lc.emplace_back(t.first, (int64_t)v);
    }
    return r;
  }

  Form operand(bool imm, uint32_t w, const std::vector<Form>& env) const {
    if (imm) return konst((int32_t)w);
    if (w < MAX_REGS) return env[w];
    Form f;
    f.top = false;
    switch (w) {
      case SEL_LID: f.cl = 1; break;
      case SEL_GID: f.cg = 1; break;
      case SEL_TID: f.cg = W_; f.cl = 1; break;
      case SEL_WGSIZE: f.c0 = W_; break;
      case SEL_NGROUPS: f.c0 = G_; break;
      case SEL_NTHREADS: f.c0 = (int64_t)G_ * W_; break;
      default: return unknown();   // scalar parameters
    }
    return norm(f);
  }

  Form binary(uint32_t op, const Form& x, const Form& y) const {
    switch (op) {
      case B_ADD: return norm(combine(x, y, 1));
      case B_SUB: return norm(combine(x, y, -1));
      case B_MUL:
        if (is_const(y)) return norm(scale(x, y.c0));
        if (is_const(x)) return norm(scale(y, x.c0));
        return unknown();
      case B_SHL:
        if (is_const(y)) {
          const int64_t k = ((y.c0 % 32) + 32) % 32;   // the count is taken mod 32
          return norm(scale(x, int64_t(1) << k));
        }
        return unknown();
      default:
        return unknown();
    }
  }

  static void join(std::vector<Form>& a, const std::vector<Form>& b) {
    for (size_t r = 0; r < a.size(); ++r)
      if (!(a[r] == b[r])) a[r] = unknown();
  }

  // instructions [i, end) of one structured block
  void block(uint32_t i, uint32_t end, std::vector<Form>& env) {
    while (i < end) {
      if (++visits_ > VISIT_MAX) return;
      const uint32_t h = word(i, 0), op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u;
      const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
      switch (op) {
        case OP_BIN:
          env[dst] = binary(sub, operand(fa, word(i, 1), env), operand(fb, word(i, 2), env));
          ++i;
          break;
        case OP_UN: {
          const Form x = operand(fa, word(i, 1), env);
          env[dst] = sub == U_MOV ? x : sub == U_NEG ? norm(scale(x, -1)) : unknown();
          ++i;
          break;
        }
        case OP_LOAD:
          access_[{i, word(i, 3)}] = operand(fa, word(i, 1), env);
          env[dst] = unknown();
          ++i;
          break;
        case OP_STORE:
          access_[{i, word(i, 3)}] = operand(fa, word(i, 1), env);
          ++i;
          break;
        case OP_IF: {
          const uint32_t at_else = word(i, 2), at_endif = word(at_else, 3);
          std::vector<Form> other = env;
          block(i + 1, at_else, env);
          block(at_else + 1, at_endif, other);
          join(env, other);
          i = at_endif + 1;
          break;
        }
        case OP_FOR: {
          const int64_t lo = (int32_t)word(i, 1), hi = (int32_t)word(i, 2);
          const uint32_t after = word(i, 3);   // the instruction after ENDFOR
          if (hi - lo <= 0) {                  // the body never runs
            env[dst] = konst(lo);
            i = after;
            break;
          }
          loops_[i] = Range{lo, hi - 1};
          Form counter;
          counter.top = false;
          counter.lc.emplace_back(i, 1);
          counter = norm(counter);
          // the state at the top of the body: the entry state joined with
          // the state after each iteration, the counter reset by ENDFOR
          std::vector<Form> head = env;
          head[dst] = counter;
          std::vector<Form> body;
          for (;;) {
            body = head;
            block(i + 1, after - 1, body);   // also records the accesses of this pass
            std::vector<Form> next = head;
            join(next, body);
            next[dst] = counter;
            if (next == head) break;
            head = next;
          }
          // after the last iteration ENDFOR leaves the counter at hi
          env = body;
          env[dst] = konst(hi);
          i = after;
          break;
        }
        case OP_END:
          return;
        default:   // barrier, assert, assume
          ++i;
          break;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Second proof, by enumeration: when no index and no branch depends on a
// loaded value or a scalar parameter, every work-item's accesses are the
// same for every input.  Each work-item's register values are then computed
// on the host (its own path through the program: its registers do not depend
// on other work-items), and the cells each touches are compared.  A faulting
// statement stops a group; the enumeration keeps going past it, which only
// adds accesses, so an array it finds unshared is unshared.
// ---------------------------------------------------------------------------
constexpr uint64_t ENUM_STEPS_MAX = 5000000;   // instructions interpreted on the host (~0.3 s)
constexpr uint64_t ENUM_CELLS_MAX = 1ull << 26;  // owner words kept on the host (4 B each)

struct Val {
  bool known;
  int32_t v;
};

// the language's int32 operators (wrapping; division by zero is a fault)
bool host_alu(uint32_t op, int32_t x, int32_t y, int32_t* r) {
  const uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
  switch (op) {
    case B_ADD: *r = (int32_t)(ux + uy); return true;
    case B_SUB: *r = (int32_t)(ux - uy); return true;
    case B_MUL: *r = (int32_t)(ux * uy); return true;
    case B_DIV:
      if (y == 0) return false;
      *r = y == -1 ? (int32_t)(0u - ux) : x / y;
      return true;
    case B_REM:
      if (y == 0) return false;
      *r = y == -1 ? 0 : x % y;
      return true;
    case B_MOD: {
      if (y == 0) return false;
      if (y == -1 || y == 1) { *r = 0; return true; }
      int32_t m = x % y;
      if (m < 0) m = (int32_t)((uint32_t)m + (y < 0 ? 0u - uy : uy));
      *r = m;
      return true;
    }
    case B_AND: *r = x & y; return true;
    case B_OR: *r = x | y; return true;
    case B_XOR: *r = x ^ y; return true;
    case B_SHL: *r = (int32_t)(ux << (uy & 31u)); return true;
    case B_SHR: *r = x >> (int32_t)(uy & 31u); return true;
    case B_LT: *r = x < y; return true;
    case B_LE: *r = x <= y; return true;
    case B_GT: *r = x > y; return true;
    case B_GE: *r = x >= y; return true;
    case B_EQ: *r = x == y; return true;
    case B_NE: *r = x != y; return true;
    case B_LAND: *r = (x != 0) & (y != 0); return true;
    case B_LOR: *r = (x != 0) | (y != 0); return true;
    case B_MIN: *r = x < y ? x : y; return true;
    default: *r = x > y ? x : y; return true;   // B_MAX
  }
}

class Enumerator {
 public:
  Enumerator(const Compiled& c, uint32_t G, uint32_t W, std::vector<uint8_t> cand)
      : c_(c), G_(G), W_(W), cand_(std::move(cand)), cand0_(cand_) {}

  // Set by run(): no statement of any work-item can fault (every access in
  // bounds, no division by a zero or unknown divisor, every assert and
  // assume holds), whatever the inputs.
  bool never_faults = false;
  // Set by run(): the candidate local arrays that are race-free within every
  // interval (see OwnedArray), in a program that cannot fault, and the
  // intervals with a conflict on some local array (see Ownership).
  std::vector<uint8_t> race_free;
  uint64_t racy_mask = ~0ull;
  bool racy_high = true;

  // owned[a] for the candidate arrays (others 0); all 0 when the program's
  // accesses depend on its inputs or the enumeration is too long
  std::vector<uint8_t> run() {
    const uint32_t na = (uint32_t)c_.arrays.size();
    std::vector<uint8_t> none(na, 0);
    if ((double)G_ * W_ * (double)c_.dyn_instr > (double)ENUM_STEPS_MAX) return none;
    uint64_t cells = 0;
    for (uint32_t a = 0; a < na; ++a)
      if (cand_[a]) cells += c_.arrays[a].size;
    if (cells > ENUM_CELLS_MAX) return none;
    faults_ = false;
    owner_.assign(na, std::vector<int32_t>());
    for (uint32_t a = 0; a < na; ++a)
      if (cand_[a]) owner_[a].assign(c_.arrays[a].size, -1);
    rf_.assign(na, 0);
    track_.assign(na, 0);
    for (uint32_t a = 0; a < na; ++a) track_[a] = rf_[a] = cand_[a] && !c_.arrays[a].global;
    mask_ = 0;
    high_ = false;
    cells_.assign(na, std::unordered_map<uint64_t, CellUse>());
    for (uint32_t g = 0; g < G_; ++g) {
      for (uint32_t a = 0; a < na; ++a) {   // each group has its own local arrays
        if (cand_[a] && !c_.arrays[a].global) std::fill(owner_[a].begin(), owner_[a].end(), -1);
        cells_[a].clear();
      }
      for (uint32_t l = 0; l < W_; ++l) {
        bar_.clear();
        if (!item(g, l)) return none;
        // a barrier some work-items of the group pass and others skip is a
        // divergence fault: every work-item must pass the same barriers
        if (l == 0) bar0_ = bar_;
        else if (bar_ != bar0_) faults_ = true;
        bool any = !faults_;   // the fault question needs every work-item
        for (uint32_t a = 0; a < na; ++a) any = any || cand_[a];
        if (!any) return none;
      }
    }
    never_faults = !faults_;
    race_free.assign(na, 0);
    for (uint32_t a = 0; a < na; ++a) race_free[a] = never_faults && rf_[a] && !cand_[a];
    bool tracked = true;   // every local written array that is not owned was followed to the end
    for (uint32_t a = 0; a < na; ++a)
      if (!c_.arrays[a].global && cand0_[a] && !track_[a]) tracked = false;
    if (never_faults && tracked) {
      racy_mask = mask_;
      racy_high = high_;
    }
    return cand_;
  }

 private:
  const Compiled& c_;
  const uint32_t G_, W_;
  std::vector<uint8_t> cand_, cand0_;   // candidates left; the initial ones
  std::vector<std::vector<int32_t>> owner_;   // per candidate array: touching work-item, or -1
  uint64_t steps_ = 0;
  bool faults_ = false;                       // some statement may fault
  std::vector<uint32_t> bar_, bar0_;          // barriers passed: this work-item, the group's first
  // race-freeness per interval (local candidates): per (interval, cell) of
  // the current group, its writer and reader (-1 none, -2 several)
  struct CellUse {
    int32_t writer = -1, reader = -1;
  };
  std::vector<uint8_t> rf_, track_;   // race-free so far; still followed
  std::vector<std::unordered_map<uint64_t, CellUse>> cells_;
  uint64_t mask_ = 0;                 // intervals with a conflict (< 64), and any later one
  bool high_ = false;
  void racy(size_t k) {
    if (k < 64) mask_ |= 1ull << k;
    else high_ = true;
  }

  uint32_t word(uint32_t i, int k) const { return c_.code[4 * i + k]; }

  Val operand(bool imm, uint32_t w, const Val* regs, uint32_t g, uint32_t l) const {
    if (imm) return Val{true, (int32_t)w};
    if (w < MAX_REGS) return regs[w];
    switch (w) {
      case SEL_LID: return Val{true, (int32_t)l};
      case SEL_GID: return Val{true, (int32_t)g};
      case SEL_TID: return Val{true, (int32_t)(g * W_ + l)};
      case SEL_WGSIZE: return Val{true, (int32_t)W_};
      case SEL_NGROUPS: return Val{true, (int32_t)G_};
      case SEL_NTHREADS: return Val{true, (int32_t)(G_ * W_)};
      default: return Val{false, 0};   // scalar parameters differ between inputs
    }
  }

  void touch(uint32_t a, Val idx, int64_t t, bool write) {
    if (!idx.known || idx.v < 0 || (uint32_t)idx.v >= c_.arrays[a].size) faults_ = true;
    if (!cand_[a] && !track_[a]) return;
    if (!idx.known) {
      cand_[a] = 0;
      rf_[a] = 0;
      track_[a] = 0;
      return;
    }
    if (idx.v < 0 || (uint32_t)idx.v >= c_.arrays[a].size) return;   // faults: no access
    if (track_[a]) {
      CellUse& u = cells_[a][((uint64_t)bar_.size() << 32) | (uint32_t)idx.v];
      const int32_t me = (int32_t)t;
      bool conflict;
      if (write) {   // two writers, or another work-item read it
        conflict = (u.writer != -1 && u.writer != me) || (u.reader != -1 && u.reader != me);
        u.writer = me;
      } else {       // another work-item wrote it
        conflict = u.writer != -1 && u.writer != me;
        u.reader = u.reader == -1 || u.reader == me ? me : -2;
      }
      if (conflict) {
        rf_[a] = 0;
        racy(bar_.size());
      }
    }
    if (!cand_[a]) return;
    int32_t& o = owner_[a][(uint32_t)idx.v];
    if (o == -1) o = (int32_t)t;   // work-item ids are below 2^26
    else if (o != (int32_t)t) cand_[a] = 0;
  }

  // one work-item's path; false: the path depends on the inputs, or too long
  bool item(uint32_t g, uint32_t l) {
    Val regs[MAX_REGS];
    for (Val& r : regs) r = Val{true, 0};
    uint32_t lc[MAX_NEST + 1] = {};
    const int64_t t = (int64_t)g * W_ + l;
    const uint32_t n = (uint32_t)(c_.code.size() / 4);
    uint32_t pc = 0;
    while (pc < n) {
      if (++steps_ > ENUM_STEPS_MAX) return false;
      const uint32_t h = word(pc, 0), op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u;
      const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
      switch (op) {
        case OP_BIN: {
          const Val x = operand(fa, word(pc, 1), regs, g, l), y = operand(fb, word(pc, 2), regs, g, l);
          int32_t r = 0;
          const bool div = sub == B_DIV || sub == B_REM || sub == B_MOD;
          if (div && (!y.known || y.v == 0)) faults_ = true;
          regs[dst] = x.known && y.known && host_alu(sub, x.v, y.v, &r) ? Val{true, r} : Val{false, 0};
          ++pc;
          break;
        }
        case OP_UN: {
          const Val x = operand(fa, word(pc, 1), regs, g, l);
          if (!x.known) regs[dst] = x;
          else if (sub == U_MOV) regs[dst] = x;
          else if (sub == U_NEG) regs[dst] = Val{true, (int32_t)(0u - (uint32_t)x.v)};
          else if (sub == U_BNOT) regs[dst] = Val{true, ~x.v};
          else regs[dst] = Val{true, x.v == 0 ? 1 : 0};
          ++pc;
          break;
        }
        case OP_LOAD:
          touch(word(pc, 3), operand(fa, word(pc, 1), regs, g, l), t, false);
          regs[dst] = Val{false, 0};
          ++pc;
          break;
        case OP_STORE:
          touch(word(pc, 3), operand(fa, word(pc, 1), regs, g, l), t, true);
          ++pc;
          break;
        case OP_IF: {
          const Val cnd = operand(fa, word(pc, 1), regs, g, l);
          if (!cnd.known) return false;   // a data-dependent path
          pc = cnd.v != 0 ? pc + 1 : word(pc, 2) + 1;
          break;
        }
        case OP_ELSE:   // end of the taken then-branch
          pc = word(pc, 3) + 1;
          break;
        case OP_FOR: {
          const int32_t lo = (int32_t)word(pc, 1), hi = (int32_t)word(pc, 2);
          regs[dst] = Val{true, lo};
          if ((int64_t)hi - (int64_t)lo <= 0) {
            pc = word(pc, 3);
          } else {
            lc[sub] = 0;
            ++pc;
          }
          break;
        }
        case OP_ENDFOR: {
          const int32_t lo = (int32_t)word(pc, 1), hi = (int32_t)word(pc, 2);
          const uint32_t iters = (uint32_t)((int64_t)hi - (int64_t)lo);
          lc[sub] += 1;
          regs[dst] = Val{true, (int32_t)((uint32_t)lo + lc[sub])};
          pc = lc[sub] < iters ? word(pc, 3) : pc + 1;
          break;
        }
        case OP_ASSERT:
        case OP_ASSUME: {
          const Val cnd = operand(fa, word(pc, 1), regs, g, l);
          if (!cnd.known || cnd.v == 0) faults_ = true;
          ++pc;
          break;
        }
        case OP_BARRIER:
          bar_.push_back(pc);
          ++pc;
          break;
        case OP_END:
          return true;
        default:   // endif
          ++pc;
          break;
      }
    }
    return true;
  }
};

// ---------------------------------------------------------------------------
// Third proof, by value ranges, of "no statement can fault" only: every
// register holds an interval of int32 values (private variables start at
// 0; loaded values and scalar parameters are any int32), the two branches
// of an if are joined by their hull, and a loop's entry state is iterated
// to a fixed point (registers still changing after a few passes become any
// int32).  No statement can fault when every index's interval lies inside
// its array, no divisor's interval holds 0, every assert and assume
// condition's interval excludes 0, and no barrier is inside an if (loop
// bounds are constants, so every work-item of a group then passes the same
// barriers).  Unlike the enumeration it needs no input-independent
// accesses: an index (e) mod size(A) is in bounds whatever e is.
// ---------------------------------------------------------------------------
struct Iv {
  int64_t lo, hi;
  bool operator==(const Iv& o) const { return lo == o.lo && hi == o.hi; }
};

class RangeProver {
 public:
  RangeProver(const Compiled& c, uint32_t G, uint32_t W) : c_(c), G_(G), W_(W) {}

  bool run() {
    std::vector<Iv> env(MAX_REGS, Iv{0, 0});
    ok_ = true;
    block(0, (uint32_t)(c_.code.size() / 4), env, 0);
    return ok_ && visits_ <= VISIT_MAX;
  }

 private:
  const Compiled& c_;
  const uint32_t G_, W_;
  bool ok_ = true;
  uint64_t visits_ = 0;
  static constexpr int WIDEN_AFTER = 8;

  uint32_t word(uint32_t i, int k) const { return c_.code[4 * i + k]; }
  static Iv full() { return Iv{I32_MIN, I32_MAX}; }
  static Iv konst(int64_t v) { return Iv{v, v}; }
  // a result outside int32 wraps: any int32
  static Iv clamp(i128 lo, i128 hi) {
    if (lo < I32_MIN || hi > I32_MAX) return full();
    return Iv{(int64_t)lo, (int64_t)hi};
  }
  static int64_t mag(const Iv& y) { return std::max(y.lo < 0 ? -y.lo : y.lo, y.hi < 0 ? -y.hi : y.hi); }
  static bool has_zero(const Iv& y) { return y.lo <= 0 && y.hi >= 0; }
  static int64_t ones_above(int64_t v) {   // 2^k - 1 >= v
    int64_t m = 0;
    while (m < v) m = m * 2 + 1;
    return m;
  }

  Iv operand(bool imm, uint32_t w, const std::vector<Iv>& env) const {
    if (imm) return konst((int32_t)w);
    if (w < MAX_REGS) return env[w];
    switch (w) {
      case SEL_LID: return Iv{0, (int64_t)W_ - 1};
      case SEL_GID: return Iv{0, (int64_t)G_ - 1};
      case SEL_TID: return Iv{0, (int64_t)G_ * W_ - 1};
      case SEL_WGSIZE: return konst(W_);
      case SEL_NGROUPS: return konst(G_);
      case SEL_NTHREADS: return konst((int64_t)G_ * W_);
      default: return full();   // scalar parameters
    }
  }

  Iv binary(uint32_t op, const Iv& x, const Iv& y) {
    switch (op) {
      case B_ADD: return clamp((i128)x.lo + y.lo, (i128)x.hi + y.hi);
      case B_SUB: return clamp((i128)x.lo - y.hi, (i128)x.hi - y.lo);
      case B_MUL: {
        const i128 p[4] = {(i128)x.lo * y.lo, (i128)x.lo * y.hi, (i128)x.hi * y.lo, (i128)x.hi * y.hi};
        return clamp(*std::min_element(p, p + 4), *std::max_element(p, p + 4));
      }
      case B_DIV: {   // |x / y| <= |x| for |y| >= 1 (INT_MIN / -1 = INT_MIN stays inside)
        if (has_zero(y)) { ok_ = false; return full(); }
        const int64_t m = mag(x);
        return Iv{std::max(-m, I32_MIN), std::min(m, I32_MAX)};
      }
      case B_REM: {   // sign of x, |r| < |y|, |r| <= |x|
        if (has_zero(y)) { ok_ = false; return full(); }
        const int64_t m = mag(y) - 1;
        return Iv{x.lo >= 0 ? 0 : std::max(x.lo, -m), x.hi <= 0 ? 0 : std::min(x.hi, m)};
      }
      case B_MOD: {   // in [0, |y|)
        if (has_zero(y)) { ok_ = false; return full(); }
        const int64_t m = mag(y) - 1;
        return Iv{0, x.lo >= 0 ? std::min(x.hi, m) : m};
      }
      case B_AND:
        if (x.lo >= 0 && y.lo >= 0) return Iv{0, std::min(x.hi, y.hi)};
        if (x.lo >= 0) return Iv{0, x.hi};
        if (y.lo >= 0) return Iv{0, y.hi};
        return full();
      case B_OR:
      case B_XOR:
        if (x.lo >= 0 && y.lo >= 0) return Iv{0, ones_above(std::max(x.hi, y.hi))};
        return full();
      case B_SHL:
        if (y.lo == y.hi) {
          const int k = (int)(((y.lo % 32) + 32) % 32);
          return clamp((i128)x.lo << k, (i128)x.hi << k);
        }
        return full();
      case B_SHR:
        if (y.lo == y.hi) {
          const int k = (int)(((y.lo % 32) + 32) % 32);
          return Iv{x.lo >> k, x.hi >> k};
        }
        if (x.lo >= 0) return Iv{0, x.hi};
        if (x.hi < 0) return Iv{x.lo, -1};
        return x;
      case B_MIN: return Iv{std::min(x.lo, y.lo), std::min(x.hi, y.hi)};
      case B_MAX: return Iv{std::max(x.lo, y.lo), std::max(x.hi, y.hi)};
      default: return Iv{0, 1};   // comparisons and logical operators
    }
  }

  void check_index(uint32_t a, const Iv& idx) {
    if (a >= c_.arrays.size() || idx.lo < 0 || idx.hi >= (int64_t)c_.arrays[a].size) ok_ = false;
  }

  static void hull(std::vector<Iv>& a, const std::vector<Iv>& b) {
    for (size_t r = 0; r < a.size(); ++r) a[r] = Iv{std::min(a[r].lo, b[r].lo), std::max(a[r].hi, b[r].hi)};
  }

  // instructions [i, end) of one structured block, `ifs` ifs deep
  void block(uint32_t i, uint32_t end, std::vector<Iv>& env, uint32_t ifs) {
    while (i < end && ok_) {
      if (++visits_ > VISIT_MAX) { ok_ = false; return; }
      const uint32_t h = word(i, 0), op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u;
      const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
      switch (op) {
        case OP_BIN:
          env[dst] = binary(sub, operand(fa, word(i, 1), env), operand(fb, word(i, 2), env));
          ++i;
          break;
        case OP_UN: {
          const Iv x = operand(fa, word(i, 1), env);
          if (sub == U_MOV) env[dst] = x;
          else if (sub == U_NEG) env[dst] = clamp(-(i128)x.hi, -(i128)x.lo);
          else if (sub == U_BNOT) env[dst] = Iv{-x.hi - 1, -x.lo - 1};
          else env[dst] = Iv{0, 1};
          ++i;
          break;
        }
        case OP_LOAD:
          check_index(word(i, 3), operand(fa, word(i, 1), env));
          env[dst] = full();
          ++i;
          break;
        case OP_STORE:
          check_index(word(i, 3), operand(fa, word(i, 1), env));
          ++i;
          break;
        case OP_IF: {
          const uint32_t at_else = word(i, 2), at_endif = word(at_else, 3);
          std::vector<Iv> other = env;
          block(i + 1, at_else, env, ifs + 1);
          block(at_else + 1, at_endif, other, ifs + 1);
          hull(env, other);
          i = at_endif + 1;
          break;
        }
        case OP_FOR: {
          const int64_t lo = (int32_t)word(i, 1), hi = (int32_t)word(i, 2);
          const uint32_t after = word(i, 3);
          if (hi - lo <= 0) {
            env[dst] = konst(lo);
            i = after;
            break;
          }
          std::vector<Iv> head = env, body;
          head[dst] = Iv{lo, hi - 1};
          for (int pass = 0;; ++pass) {
            body = head;
            block(i + 1, after - 1, body, ifs);
            if (!ok_) return;
            std::vector<Iv> next = head;
            hull(next, body);
            next[dst] = Iv{lo, hi - 1};
            if (next == head) break;
            if (pass >= WIDEN_AFTER)
              for (size_t r = 0; r < next.size(); ++r)
                if (!(next[r] == head[r])) next[r] = full();
            head = next;
          }
          env = body;
          env[dst] = konst(hi);
          i = after;
          break;
        }
        case OP_BARRIER:
          if (ifs > 0) ok_ = false;   // reached by part of a group: a divergence fault
          ++i;
          break;
        case OP_ASSERT:
        case OP_ASSUME: {
          const Iv cnd = operand(fa, word(i, 1), env);
          if (has_zero(cnd)) ok_ = false;
          ++i;
          break;
        }
        case OP_END:
          return;
        default:   // else, endif
          ++i;
          break;
      }
    }
  }
};

}  // namespace

Ownership prove_ownership(const Compiled& c, uint32_t G, uint32_t W) {
  Prover p(c, G, W);
  Ownership out;
  out.arrays = p.run();
  // the enumeration settles written arrays the affine proof left open, and
  // whether any statement can fault
  std::vector<uint8_t> cand(out.arrays.size(), 0);
  for (size_t a = 0; a < out.arrays.size(); ++a) cand[a] = !out.arrays[a].owned && c.arrays[a].written;
  Enumerator e(c, G, W, cand);
  const std::vector<uint8_t> owned = e.run();
  for (size_t a = 0; a < out.arrays.size(); ++a) {
    if (owned[a]) out.arrays[a].owned = 1;   // owned, kept in the plain layout
    if (a < e.race_free.size() && e.race_free[a]) out.arrays[a].race_free = 1;
  }
  out.local_log_mask = e.racy_mask;
  out.local_log_high = e.racy_high;
  // the value ranges can prove "no fault" where the enumeration gives up
  // (indices that depend on the inputs)
  out.never_faults = e.never_faults || RangeProver(c, G, W).run();
  return out;
}

}  // namespace rc
