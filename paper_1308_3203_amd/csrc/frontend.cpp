// frontend.cpp -- the kernel language (paper Section 3: expressions e,
// booleans b, commands Comm, kernel tuple K(Args)) in its structured surface
// form: tokenizer, Pratt expression parser, validation of names and limits,
// static bounds, and lowering to the fixed-width bytecode run by the HIP
// interpreter.
#include "frontend.h"

#include <cctype>
#include <algorithm>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <unordered_map>

#include "rc_internal.h"

namespace rc {
namespace {

struct CompileError {
  int line, col;
  std::string msg;
  bool limit;
};

// ---------------------------------------------------------------------------
// tokens
// ---------------------------------------------------------------------------
enum TokKind { T_END, T_NUM, T_NAME, T_SYM };

struct Token {
  TokKind kind;
  std::string text;
  uint64_t num = 0;
  int line = 0, col = 0;
};

std::vector<Token> tokenize(const char* s, size_t n) {
  static const char* syms[] = {":=", "..", "<<", ">>", "<=", ">=", "==", "!=", "&&", "||",
                               "[", "]", "(", ")", "{", "}", ";", ",", "+", "-", "*", "/",
                               "%", "&", "|", "^", "~", "!", "<", ">"};
  std::vector<Token> out;
  size_t i = 0;
  int line = 1, col = 1;
  auto adv = [&](size_t k) {
    for (size_t j = 0; j < k && i < n; ++j, ++i) {
      if (s[i] == '\n') { ++line; col = 1; } else { ++col; }
    }
  };
  while (true) {
    while (i < n) {
      if (isspace((unsigned char)s[i])) { adv(1); continue; }
      if (i + 1 < n && s[i] == '/' && s[i + 1] == '/') {
        while (i < n && s[i] != '\n') adv(1);
        continue;
      }
      if (i + 1 < n && s[i] == '/' && s[i + 1] == '*') {
        int l0 = line, c0 = col;
        adv(2);
        while (i + 1 < n && !(s[i] == '*' && s[i + 1] == '/')) adv(1);
        if (i + 1 >= n) throw CompileError{l0, c0, "unterminated comment", false};
        adv(2);
        continue;
      }
      break;
    }
    Token t;
    t.line = line; t.col = col;
    if (i >= n) { t.kind = T_END; t.text = "end of input"; out.push_back(t); return out; }
    char c = s[i];
    if (isdigit((unsigned char)c)) {
      uint64_t v = 0;
      int base = 10;
      if (c == '0' && i + 1 < n && (s[i + 1] == 'x' || s[i + 1] == 'X')) { base = 16; adv(2); }
      size_t start = i;
      while (i < n && isxdigit((unsigned char)s[i]) && (base == 16 || isdigit((unsigned char)s[i]))) {
        int d = isdigit((unsigned char)s[i]) ? s[i] - '0' : 10 + (tolower((unsigned char)s[i]) - 'a');
        v = v * (uint64_t)base + (uint64_t)d;
        if (v > 0xFFFFFFFFull) throw CompileError{t.line, t.col, "integer literal out of range", false};
        adv(1);
      }
      if (i == start || (i < n && (isalnum((unsigned char)s[i]) || s[i] == '_')))
        throw CompileError{t.line, t.col, "malformed integer literal", false};
      t.kind = T_NUM; t.num = v; t.text = std::to_string(v);
      out.push_back(t);
      continue;
    }
    if (isalpha((unsigned char)c) || c == '_') {
      size_t start = i;
      while (i < n && (isalnum((unsigned char)s[i]) || s[i] == '_')) adv(1);
      t.kind = T_NAME; t.text.assign(s + start, i - start);
      if (t.text.size() > 63) throw CompileError{t.line, t.col, "name longer than 63 characters", false};
      out.push_back(t);
      continue;
    }
    bool found = false;
    for (const char* sym : syms) {
      size_t L = strlen(sym);
      if (i + L <= n && memcmp(s + i, sym, L) == 0) {
        t.kind = T_SYM; t.text = sym; adv(L); found = true;
        break;
      }
    }
    if (!found) throw CompileError{t.line, t.col, std::string("unexpected character '") + c + "'", false};
    out.push_back(t);
  }
}

// ---------------------------------------------------------------------------
// syntax tree
// ---------------------------------------------------------------------------
struct Node {           // expression
  enum Kind { NUM, VAR, SCALAR, SPECIAL, UNARY, BINARY } kind;
  int32_t value = 0;    // NUM value, VAR/SCALAR index, SPECIAL selector
  uint32_t op = 0;
  std::unique_ptr<Node> l, r;
};
using NodeP = std::unique_ptr<Node>;

struct Statement {
  enum Kind { ASSIGN, LOAD, STORE, BARRIER, ASSUME, ASSERT, IF, FOR } kind;
  uint32_t pc = 0;
  int var = -1, arr = -1;
  NodeP e1, e2;
  std::vector<Statement> then_body, else_body;
  int64_t lo = 0, hi = 0;
  uint32_t slot = 0;    // loop nesting slot
  int line = 0, col = 0;
};

bool is_reserved(const std::string& s) {
  static const char* kw[] = {"kernel", "global", "local", "int", "barrier", "assume", "assert",
                             "if", "else", "for", "in", "tid", "lid", "gid", "wgsize", "ngroups",
                             "nthreads", "size", "min", "max", "mod"};
  for (const char* k : kw) if (s == k) return true;
  return false;
}

class Parser {
 public:
  Parser(std::vector<Token> toks, Compiled* out) : t_(std::move(toks)), out_(out) {}

  void parse_kernel(std::vector<Statement>* body) {
    keyword("kernel");
    const Token& nm = cur();
    if (nm.kind != T_NAME || is_reserved(nm.text)) fail(nm, "expected the kernel name");
    out_->name = nm.text;
    ++p_;
    sym("(");
    if (!at_sym(")")) {
      while (true) {
        parse_param();
        if (at_sym(",")) { ++p_; continue; }
        break;
      }
    }
    sym(")");
    sym("{");
    while (at_name("local") || at_name("int")) parse_decl();
    while (!at_sym("}")) {
      if (cur().kind == T_END) fail(cur(), "expected '}'");
      body->push_back(parse_stmt(0, 0));
    }
    sym("}");
    if (cur().kind != T_END) fail(cur(), "trailing input after the kernel");
    if (out_->n_stmts > MAX_STMTS) throw CompileError{1, 1, "more than 4096 statements", true};
  }

 private:
  std::vector<Token> t_;
  size_t p_ = 0;
  Compiled* out_;
  std::unordered_map<std::string, int> arrays_, scalars_, vars_;
  std::vector<int> loop_vars_;

  const Token& cur() const { return t_[p_]; }
  [[noreturn]] void fail(const Token& t, const std::string& msg, bool limit = false) {
    throw CompileError{t.line, t.col, msg, limit};
  }
  bool at_sym(const char* s) const { return cur().kind == T_SYM && cur().text == s; }
  bool at_name(const char* s) const { return cur().kind == T_NAME && cur().text == s; }
  void sym(const char* s) {
    if (!at_sym(s)) fail(cur(), std::string("expected '") + s + "', found '" + cur().text + "'");
    ++p_;
  }
  void keyword(const char* s) {
    if (!at_name(s)) fail(cur(), std::string("expected '") + s + "', found '" + cur().text + "'");
    ++p_;
  }
  bool taken(const std::string& s) const {
    return is_reserved(s) || arrays_.count(s) || scalars_.count(s) || vars_.count(s);
  }
  std::string fresh_name(const char* what) {
    const Token& t = cur();
    if (t.kind != T_NAME) fail(t, std::string("expected ") + what + " name");
    if (taken(t.text)) fail(t, "name '" + t.text + "' is reserved or already declared");
    ++p_;
    return t.text;
  }
  int64_t int_literal() {
    bool neg = false;
    if (at_sym("-")) { neg = true; ++p_; }
    if (cur().kind != T_NUM) fail(cur(), "expected an integer literal");
    int64_t v = (int64_t)cur().num;
    ++p_;
    return neg ? -v : v;
  }
  uint32_t array_size() {
    sym("[");
    const Token& at = cur();
    int64_t v = int_literal();
    if (v < 1 || v > (1 << 24)) fail(at, "array size must be in [1, 2^24]", true);
    sym("]");
    return (uint32_t)v;
  }

  void parse_param() {
    if (at_name("global")) {
      ++p_;
      keyword("int");
      const Token& at = cur();
      std::string nm = fresh_name("array");
      if (out_->n_global >= MAX_GLOBAL_ARRAYS) fail(at, "more than 8 global arrays", true);
      CompiledArray a;
      a.name = nm; a.global = true; a.size = array_size();
      arrays_[nm] = (int)out_->arrays.size();
      out_->arrays.push_back(a);
      out_->n_global++;
    } else if (at_name("int")) {
      ++p_;
      const Token& at = cur();
      std::string nm = fresh_name("scalar");
      if (out_->scalars.size() >= MAX_SCALARS) fail(at, "more than 16 scalar parameters", true);
      scalars_[nm] = (int)out_->scalars.size();
      out_->scalars.push_back(nm);
    } else {
      fail(cur(), "expected a parameter: 'global int NAME[N]' or 'int NAME'");
    }
  }

  void parse_decl() {
    if (at_name("local")) {
      ++p_;
      keyword("int");
      const Token& at = cur();
      std::string nm = fresh_name("array");
      if (out_->n_local >= MAX_LOCAL_ARRAYS) fail(at, "more than 8 local arrays", true);
      CompiledArray a;
      a.name = nm; a.global = false; a.size = array_size();
      arrays_[nm] = (int)out_->arrays.size();
      out_->arrays.push_back(a);
      out_->n_local++;
      sym(";");
      return;
    }
    keyword("int");
    while (true) {
      const Token& at = cur();
      std::string nm = fresh_name("variable");
      if (out_->vars.size() >= MAX_VARS) fail(at, "more than 32 private variables", true);
      vars_[nm] = (int)out_->vars.size();
      out_->vars.push_back(nm);
      if (at_sym(",")) { ++p_; continue; }
      break;
    }
    sym(";");
  }

  // Pratt parser; binding power grows with precedence
  static int infix_power(const Token& t, uint32_t* op) {
    struct E { const char* s; int bp; uint32_t op; };
    static const E table[] = {
        {"||", 1, B_LOR}, {"&&", 2, B_LAND}, {"|", 3, B_OR}, {"^", 4, B_XOR}, {"&", 5, B_AND},
        {"==", 6, B_EQ}, {"!=", 6, B_NE}, {"<", 7, B_LT}, {"<=", 7, B_LE}, {">", 7, B_GT},
        {">=", 7, B_GE}, {"<<", 8, B_SHL}, {">>", 8, B_SHR}, {"+", 9, B_ADD}, {"-", 9, B_SUB},
        {"*", 10, B_MUL}, {"/", 10, B_DIV}, {"%", 10, B_REM}, {"mod", 10, B_MOD}};
    if (t.kind != T_SYM && !(t.kind == T_NAME && t.text == "mod")) return 0;
    for (const E& e : table)
      if (t.text == e.s) { *op = e.op; return e.bp; }
    return 0;
  }

  NodeP leaf(Node::Kind k, int32_t v) {
    NodeP n(new Node);
    n->kind = k; n->value = v;
    return n;
  }

  NodeP expr(int min_bp = 0) {
    NodeP lhs = prefix();
    while (true) {
      uint32_t op;
      int bp = infix_power(cur(), &op);
      if (bp == 0 || bp <= min_bp) break;
      ++p_;
      NodeP rhs = expr(bp);
      NodeP n(new Node);
      n->kind = Node::BINARY; n->op = op; n->l = std::move(lhs); n->r = std::move(rhs);
      lhs = std::move(n);
    }
    return lhs;
  }

  NodeP prefix() {
    const Token& t = cur();
    if (t.kind == T_NUM) { ++p_; return leaf(Node::NUM, (int32_t)(uint32_t)t.num); }
    if (t.kind == T_SYM) {
      uint32_t uop;
      if (t.text == "-") uop = U_NEG;
      else if (t.text == "~") uop = U_BNOT;
      else if (t.text == "!") uop = U_LNOT;
      else if (t.text == "(") {
        ++p_;
        NodeP e = expr();
        sym(")");
        return e;
      } else {
        fail(t, "expected an expression, found '" + t.text + "'");
      }
      ++p_;
      NodeP n(new Node);
      n->kind = Node::UNARY; n->op = uop; n->l = prefix();
      return n;
    }
    if (t.kind != T_NAME) fail(t, "expected an expression, found '" + t.text + "'");
    const std::string& s = t.text;
    static const std::pair<const char*, uint32_t> specials[] = {
        {"lid", SEL_LID}, {"tid", SEL_TID}, {"gid", SEL_GID}, {"wgsize", SEL_WGSIZE},
        {"ngroups", SEL_NGROUPS}, {"nthreads", SEL_NTHREADS}};
    for (auto& sp : specials)
      if (s == sp.first) { ++p_; return leaf(Node::SPECIAL, (int32_t)sp.second); }
    if (s == "size") {
      ++p_;
      sym("(");
      auto it = arrays_.find(cur().kind == T_NAME ? cur().text : std::string());
      if (it == arrays_.end()) fail(cur(), "size() needs an array name");
      ++p_;
      sym(")");
      return leaf(Node::NUM, (int32_t)out_->arrays[it->second].size);
    }
    if (s == "min" || s == "max") {
      uint32_t op = s == "min" ? B_MIN : B_MAX;
      ++p_;
      sym("(");
      NodeP a = expr();
      sym(",");
      NodeP b = expr();
      sym(")");
      NodeP n(new Node);
      n->kind = Node::BINARY; n->op = op; n->l = std::move(a); n->r = std::move(b);
      return n;
    }
    if (vars_.count(s)) { ++p_; return leaf(Node::VAR, vars_[s]); }
    if (scalars_.count(s)) { ++p_; return leaf(Node::SCALAR, scalars_[s]); }
    if (arrays_.count(s)) fail(t, "array '" + s + "' cannot be read inside an expression");
    fail(t, "unknown name '" + s + "'");
  }

  void block(std::vector<Statement>* body, int depth, uint32_t loops) {
    sym("{");
    while (!at_sym("}")) {
      if (cur().kind == T_END) fail(cur(), "expected '}'");
      body->push_back(parse_stmt(depth, loops));
    }
    sym("}");
  }

  Statement parse_stmt(int depth, uint32_t loops) {
    Statement st;
    const Token& t = cur();
    st.line = t.line; st.col = t.col;
    st.pc = out_->n_stmts++;
    if (t.kind != T_NAME) fail(t, "expected a statement, found '" + t.text + "'");
    if (t.text == "barrier") {
      ++p_; sym(";");
      st.kind = Statement::BARRIER;
      return st;
    }
    if (t.text == "assume" || t.text == "assert") {
      st.kind = t.text == "assume" ? Statement::ASSUME : Statement::ASSERT;
      ++p_; sym("("); st.e1 = expr(); sym(")"); sym(";");
      return st;
    }
    if (t.text == "if") {
      if (depth + 1 > (int)MAX_NEST) fail(t, "nesting deeper than 16", true);
      st.kind = Statement::IF;
      ++p_; sym("("); st.e1 = expr(); sym(")");
      block(&st.then_body, depth + 1, loops);
      if (at_name("else")) { ++p_; block(&st.else_body, depth + 1, loops); }
      return st;
    }
    if (t.text == "for") {
      if (depth + 1 > (int)MAX_NEST) fail(t, "nesting deeper than 16", true);
      st.kind = Statement::FOR;
      ++p_;
      const Token& vt = cur();
      if (vt.kind != T_NAME || !vars_.count(vt.text)) fail(vt, "loop variable must be a declared private variable");
      st.var = vars_[vt.text];
      for (int lv : loop_vars_) if (lv == st.var) fail(vt, "loop variable '" + vt.text + "' reused by a nested loop");
      ++p_;
      keyword("in");
      const Token& lt = cur();
      st.lo = int_literal();
      sym("..");
      st.hi = int_literal();
      if (st.lo < INT32_MIN || st.lo > INT32_MAX || st.hi < INT32_MIN || st.hi > INT32_MAX)
        fail(lt, "loop bound out of range");
      st.slot = loops;
      loop_vars_.push_back(st.var);
      block(&st.then_body, depth + 1, loops + 1);
      loop_vars_.pop_back();
      return st;
    }
    auto ait = arrays_.find(t.text);
    if (ait != arrays_.end()) {
      st.kind = Statement::STORE;
      st.arr = ait->second;
      ++p_;
      sym("["); st.e1 = expr(); sym("]");
      sym(":=");
      st.e2 = expr();
      sym(";");
      out_->arrays[st.arr].written = true;
      return st;
    }
    auto vit = vars_.find(t.text);
    if (vit == vars_.end()) {
      if (scalars_.count(t.text)) fail(t, "scalar parameter '" + t.text + "' is read-only");
      fail(t, "unknown name '" + t.text + "'");
    }
    for (int lv : loop_vars_)
      if (lv == vit->second) fail(t, "loop variable '" + t.text + "' assigned inside its loop");
    st.var = vit->second;
    ++p_;
    sym(":=");
    if (cur().kind == T_NAME && arrays_.count(cur().text) && p_ + 1 < t_.size() &&
        t_[p_ + 1].kind == T_SYM && t_[p_ + 1].text == "[") {
      st.kind = Statement::LOAD;
      st.arr = arrays_[cur().text];
      ++p_;
      sym("["); st.e1 = expr(); sym("]"); sym(";");
      return st;
    }
    st.kind = Statement::ASSIGN;
    st.e1 = expr();
    sym(";");
    return st;
  }
};

// ---------------------------------------------------------------------------
// lowering to bytecode
// ---------------------------------------------------------------------------
struct Operand {
  bool imm;
  uint32_t word;
};

class Lowering {
 public:
  explicit Lowering(Compiled* out) : out_(out) {}

  void run(const std::vector<Statement>& body) {
    nvars_ = (uint32_t)out_->vars.size();
    max_reg_ = nvars_;
    for (const Statement& s : body) stmt(s);
    emit(make_hdr(OP_END, false, false, 0, 0, 0), 0, 0, 0);
    out_->nregs = max_reg_ > 0 ? max_reg_ : 1;
  }

 private:
  Compiled* out_;
  uint32_t nvars_ = 0, next_tmp_ = 0, max_reg_ = 0;

  uint32_t here() const { return (uint32_t)(out_->code.size() / 4); }
  uint32_t emit(uint32_t h, uint32_t a, uint32_t b, uint32_t c) {
    uint32_t at = here();
    out_->code.insert(out_->code.end(), {h, a, b, c});
    return at;
  }
  void patch(uint32_t at, int word, uint32_t v) { out_->code[at * 4 + word] = v; }

  uint32_t temp() {
    uint32_t r = nvars_ + next_tmp_++;
    if (r >= MAX_REGS) throw CompileError{1, 1, "expression needs more than 64 registers", true};
    if (r + 1 > max_reg_) max_reg_ = r + 1;
    return r;
  }

  // Evaluate `e`; if it is a leaf return it as an operand, else compute it into
  // `dst` (or a fresh temporary when dst < 0) and return that register.
  Operand value(const Node& e, int dst, uint32_t pc) {
    switch (e.kind) {
      case Node::NUM: return {true, (uint32_t)e.value};
      case Node::VAR: return {false, (uint32_t)e.value};
      case Node::SCALAR: return {false, SEL_SCALAR0 + (uint32_t)e.value};
      case Node::SPECIAL: return {false, (uint32_t)e.value};
      case Node::UNARY: {
        uint32_t save = next_tmp_;
        Operand a = value(*e.l, -1, pc);
        next_tmp_ = save;
        uint32_t d = dst >= 0 ? (uint32_t)dst : temp();
        emit(make_hdr(OP_UN, a.imm, false, e.op, d, pc), a.word, 0, 0);
        return {false, d};
      }
      case Node::BINARY: {
        uint32_t save = next_tmp_;
        Operand a = value(*e.l, -1, pc);
        Operand b = value(*e.r, -1, pc);
        next_tmp_ = save;
        uint32_t d = dst >= 0 ? (uint32_t)dst : temp();
        emit(make_hdr(OP_BIN, a.imm, b.imm, e.op, d, pc), a.word, b.word, 0);
        return {false, d};
      }
    }
    return {true, 0};
  }

  void stmt(const Statement& s) {
    uint32_t pc = s.pc;
    next_tmp_ = 0;
    switch (s.kind) {
      case Statement::ASSIGN: {
        if (s.e1->kind == Node::UNARY || s.e1->kind == Node::BINARY) {
          value(*s.e1, s.var, pc);      // the last operation writes the variable
        } else {
          Operand a = value(*s.e1, -1, pc);
          emit(make_hdr(OP_UN, a.imm, false, U_MOV, (uint32_t)s.var, pc), a.word, 0, 0);
        }
        break;
      }
      case Statement::LOAD: {
        Operand a = value(*s.e1, -1, pc);
        emit(make_hdr(OP_LOAD, a.imm, false, 0, (uint32_t)s.var, pc), a.word, 0, (uint32_t)s.arr);
        break;
      }
      case Statement::STORE: {
        Operand a = value(*s.e1, -1, pc);
        if (!a.imm && a.word >= nvars_ && a.word < MAX_REGS) {
          // keep the index temporary alive while the value is computed
          next_tmp_ = a.word - nvars_ + 1;
        }
        Operand b = value(*s.e2, -1, pc);
        emit(make_hdr(OP_STORE, a.imm, b.imm, 0, 0, pc), a.word, b.word, (uint32_t)s.arr);
        break;
      }
      case Statement::BARRIER:
        emit(make_hdr(OP_BARRIER, false, false, 0, 0, pc), 0, 0, 0);
        break;
      case Statement::ASSUME:
      case Statement::ASSERT: {
        Operand a = value(*s.e1, -1, pc);
        emit(make_hdr(s.kind == Statement::ASSUME ? OP_ASSUME : OP_ASSERT, a.imm, false, 0, 0, pc),
             a.word, 0, 0);
        break;
      }
      case Statement::IF: {
        Operand a = value(*s.e1, -1, pc);
        uint32_t at_if = emit(make_hdr(OP_IF, a.imm, false, 0, 0, pc), a.word, 0, 0);
        for (const Statement& c : s.then_body) stmt(c);
        uint32_t at_else = emit(make_hdr(OP_ELSE, false, false, 0, 0, pc), 0, 0, 0);
        for (const Statement& c : s.else_body) stmt(c);
        uint32_t at_endif = emit(make_hdr(OP_ENDIF, false, false, 0, 0, pc), 0, 0, 0);
        patch(at_if, 2, at_else);
        patch(at_else, 3, at_endif);
        break;
      }
      case Statement::FOR: {
        uint32_t at_for = emit(make_hdr(OP_FOR, true, true, s.slot, (uint32_t)s.var, pc),
                               (uint32_t)(int32_t)s.lo, (uint32_t)(int32_t)s.hi, 0);
        for (const Statement& c : s.then_body) stmt(c);
        emit(make_hdr(OP_ENDFOR, true, true, s.slot, (uint32_t)s.var, pc),
             (uint32_t)(int32_t)s.lo, (uint32_t)(int32_t)s.hi, at_for + 1);
        patch(at_for, 3, here());
        break;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// static bounds per work-item (every branch taken)
// ---------------------------------------------------------------------------
struct Bounds {
  double instr = 0, mem = 0, logged = 0, logged_local = 0, stores = 0, barriers = 0, iters = 0;
  std::vector<double> arr;   // loads/stores per array
};

uint64_t expr_ops(const Node& e) {
  if (e.kind == Node::UNARY) return 1 + expr_ops(*e.l);
  if (e.kind == Node::BINARY) return 1 + expr_ops(*e.l) + expr_ops(*e.r);
  return 0;
}

void bound_block(const std::vector<Statement>& body, const Compiled& c, double mult, Bounds* b) {
  for (const Statement& s : body) {
    switch (s.kind) {
      case Statement::ASSIGN: b->instr += mult * (double)(expr_ops(*s.e1) + 1); break;
      case Statement::LOAD:
      case Statement::STORE: {
        double ops = (double)expr_ops(*s.e1) + (s.e2 ? (double)expr_ops(*s.e2) : 0.0) + 1;
        b->instr += mult * ops;
        b->mem += mult;
        if (b->arr.size() <= (size_t)s.arr) b->arr.resize((size_t)s.arr + 1, 0.0);
        b->arr[(size_t)s.arr] += mult;
        if (c.arrays[s.arr].written) {
          b->logged += mult;
          if (!c.arrays[s.arr].global) b->logged_local += mult;
        }
        if (s.kind == Statement::STORE) b->stores += mult;
        break;
      }
      case Statement::BARRIER: b->instr += mult; b->barriers += mult; break;
      case Statement::ASSUME:
      case Statement::ASSERT: b->instr += mult * (double)(expr_ops(*s.e1) + 1); break;
      case Statement::IF:
        b->instr += mult * (double)(expr_ops(*s.e1) + 3);
        bound_block(s.then_body, c, mult, b);
        bound_block(s.else_body, c, mult, b);
        break;
      case Statement::FOR: {
        double iters = (double)(s.hi > s.lo ? s.hi - s.lo : 0);
        b->instr += mult * (1 + iters);
        b->iters += mult * iters;
        bound_block(s.then_body, c, mult * iters, b);
        break;
      }
    }
  }
}

bool has_barrier(const std::vector<Statement>& body) {
  for (const Statement& s : body) {
    if (s.kind == Statement::BARRIER) return true;
    if ((s.kind == Statement::IF || s.kind == Statement::FOR) &&
        (has_barrier(s.then_body) || has_barrier(s.else_body)))
      return true;
  }
  return false;
}

// Largest number of accesses (per work-item, along any path) between two
// consecutive barriers, counting accesses to arrays selected by `pick`.
struct IntervalBound {
  double open = 0;     // accesses since the last barrier at this point
  double worst = 0;    // largest closed interval so far
};

template <typename Pick>
IntervalBound interval_block(const std::vector<Statement>& body, IntervalBound in, Pick pick) {
  IntervalBound st = in;
  for (const Statement& s : body) {
    switch (s.kind) {
      case Statement::LOAD:
      case Statement::STORE:
        if (pick(s.arr)) st.open += 1;
        break;
      case Statement::BARRIER:
        st.worst = std::max(st.worst, st.open);
        st.open = 0;
        break;
      case Statement::IF: {
        IntervalBound a = interval_block(s.then_body, st, pick);
        IntervalBound b = interval_block(s.else_body, st, pick);
        st.open = std::max(a.open, b.open);
        st.worst = std::max(a.worst, b.worst);
        break;
      }
      case Statement::FOR: {
        const int64_t iters = s.hi > s.lo ? s.hi - s.lo : 0;
        if (iters == 0) break;
        IntervalBound one = interval_block(s.then_body, {0, 0}, pick);
        if (one.worst == 0 && one.open > 0 && !has_barrier(s.then_body)) {
          st.open += one.open * (double)iters;   // no barrier inside: the counts add up
          break;
        }
        if (!has_barrier(s.then_body)) break;
        // a barrier inside: after two iterations the counts repeat
        IntervalBound a = interval_block(s.then_body, st, pick);
        IntervalBound b = iters >= 2 ? interval_block(s.then_body, a, pick) : a;
        st.open = b.open;
        st.worst = std::max(a.worst, b.worst);
        break;
      }
      default:
        break;
    }
  }
  return st;
}

// ---------------------------------------------------------------------------
// static triage features (layout documented with rc_features in rc.h)
// ---------------------------------------------------------------------------
struct Affine {          // index = (a * tid + b) [mod N]
  bool ok = false, has_mod = false;
  int64_t a = 0, b = 0, N = 0;
};

Affine affine_of(const Node& e) {
  Affine r;
  const int64_t lim = (int64_t)1 << 31;
  auto in_range = [&](Affine x) {
    if (x.a > lim || x.a < -lim || x.b > lim || x.b < -lim) x.ok = false;
    return x;
  };
  switch (e.kind) {
    case Node::NUM: r.ok = true; r.b = e.value; return r;
    case Node::SPECIAL: if ((uint32_t)e.value == SEL_TID) { r.ok = true; r.a = 1; } return r;
    case Node::UNARY: {
      if (e.op != U_NEG) return r;
      Affine x = affine_of(*e.l);
      if (!x.ok || x.has_mod) return r;
      x.a = -x.a; x.b = -x.b;
      return in_range(x);
    }
    case Node::BINARY: {
      Affine x = affine_of(*e.l), y = affine_of(*e.r);
      if (!x.ok || !y.ok || x.has_mod || y.has_mod) return r;
      switch (e.op) {
        case B_ADD: r.ok = true; r.a = x.a + y.a; r.b = x.b + y.b; return in_range(r);
        case B_SUB: r.ok = true; r.a = x.a - y.a; r.b = x.b - y.b; return in_range(r);
        case B_MUL:
          if (x.a != 0 && y.a != 0) return r;
          r.ok = true;
          if (x.a == 0) { r.a = x.b * y.a; r.b = x.b * y.b; }
          else { r.a = x.a * y.b; r.b = x.b * y.b; }
          return in_range(r);
        case B_MOD:
        case B_REM:
          if (y.a != 0 || y.b <= 0) return r;
          x.has_mod = true; x.N = y.b;
          return x;
        default: return r;
      }
    }
    default: return r;
  }
}

struct MemStmt {
  bool store;
  int arr;
  Affine idx;
  int64_t ivl;
  bool in_if, in_loop, in_barrier_loop;
};

struct FeatWalk {
  const Compiled* c;
  int64_t counts[8] = {};        // assign, load, store, barrier, assume, assert, if, for
  int64_t ld_g = 0, ld_l = 0, st_g = 0, st_l = 0, n = 0;
  int64_t ivl = 0, mem_in_ivl = 0, max_mem_in_ivl = 0, barriers_in_loops = 0, trip_sum = 0;
  int64_t val_tid = 0, val_other = 0, if_depth = 0, max_if_depth = 0, loop_depth = 0, max_loop_depth = 0;
  int64_t mem_in_if = 0, mem_in_loop = 0, barrier_loop_depth = 0;
  std::vector<MemStmt> mem;

  void walk(const std::vector<Statement>& body) {
    for (const Statement& s : body) {
      ++n;
      counts[(int)s.kind] += 1;
      switch (s.kind) {
        case Statement::LOAD:
        case Statement::STORE: {
          const bool st = s.kind == Statement::STORE;
          const bool g = c->arrays[s.arr].global;
          if (st) (g ? st_g : st_l) += 1; else (g ? ld_g : ld_l) += 1;
          MemStmt m;
          m.store = st;
          m.arr = s.arr;
          m.idx = affine_of(*s.e1);
          m.ivl = ivl;
          m.in_if = if_depth > 0;
          m.in_loop = loop_depth > 0;
          m.in_barrier_loop = barrier_loop_depth > 0;
          mem.push_back(m);
          if (m.in_if) ++mem_in_if;
          if (m.in_loop) ++mem_in_loop;
          ++mem_in_ivl;
          if (st) {
            Affine v = affine_of(*s.e2);
            if (!v.ok) ++val_other;
            else if (v.a != 0) ++val_tid;
          }
          break;
        }
        case Statement::BARRIER:
          if (loop_depth > 0) ++barriers_in_loops;
          max_mem_in_ivl = std::max(max_mem_in_ivl, mem_in_ivl);
          mem_in_ivl = 0;
          ++ivl;
          break;
        case Statement::IF:
          ++if_depth;
          max_if_depth = std::max(max_if_depth, if_depth);
          walk(s.then_body);
          walk(s.else_body);
          --if_depth;
          break;
        case Statement::FOR: {
          trip_sum += s.hi > s.lo ? s.hi - s.lo : 0;
          const bool bl = has_barrier(s.then_body);
          ++loop_depth;
          max_loop_depth = std::max(max_loop_depth, loop_depth);
          if (bl) ++barrier_loop_depth;
          walk(s.then_body);
          if (bl) --barrier_loop_depth;
          --loop_depth;
          break;
        }
        default:
          break;
      }
    }
  }
};

float ratio(int64_t num, int64_t den) { return (float)num / (float)den; }
// a count c on scale k, bounded: c / (c + k)
float squash(int64_t c, int64_t k) { return (float)c / (float)(c + k); }

int64_t emod(int64_t x, int64_t m) { return ((x % m) + m) % m; }

void static_features(const std::vector<Statement>& body, const Compiled& c, float* f) {
  FeatWalk w;
  w.c = &c;
  w.walk(body);
  w.max_mem_in_ivl = std::max(w.max_mem_in_ivl, w.mem_in_ivl);
  const int64_t n = std::max<int64_t>(w.n, 1);
  for (int k = 0; k < 8; ++k) f[k] = ratio(w.counts[k], n);
  f[8] = ratio(w.ld_g, n);
  f[9] = ratio(w.ld_l, n);
  f[10] = ratio(w.st_g, n);
  f[11] = ratio(w.st_l, n);
  f[12] = squash(w.n, 256);
  f[13] = ratio(c.n_global, 8);
  f[14] = ratio(c.n_local, 8);
  f[15] = ratio((int64_t)c.scalars.size(), 16);
  // pairs of memory statements that may touch one cell from two work-items
  int64_t pc[8] = {};
  int64_t meet = 0;   // of the equal-a, different-b pairs: those whose cells meet
  // within 1024 work-items: a*d = (b_q - b_p) mod S for some 1 <= |d| <= 1024
  auto meets = [](int64_t a, int64_t db, int64_t S) {
    for (int64_t d = 1; d <= 1024; ++d)
      if (emod(a * d - db, S) == 0 || emod(-a * d - db, S) == 0) return true;
    return false;
  };
  const size_t M = w.mem.size();
  for (size_t p = 0; p < M; ++p) {
    for (size_t q = p; q < M; ++q) {
      const MemStmt& x = w.mem[p];
      const MemStmt& y = w.mem[q];
      if (x.arr != y.arr || !(x.store || y.store)) continue;
      if (p == q && !x.store) continue;
      if (x.in_barrier_loop || y.in_barrier_loop) { ++pc[7]; continue; }
      if (x.ivl != y.ivl) continue;
      if (p == q) {
        if (!x.idx.ok) ++pc[2];
        else if (x.idx.a == 0) { ++pc[0]; if (x.in_if) ++pc[1]; }
        continue;
      }
      if (!x.idx.ok || !y.idx.ok) { ++pc[6]; continue; }
      if (x.idx.a != y.idx.a) { ++pc[5]; continue; }
      const int64_t S = c.arrays[x.arr].size;
      if (emod(x.idx.b, S) != emod(y.idx.b, S)) {
        ++pc[3];
        if (meets(x.idx.a, emod(y.idx.b - x.idx.b, S), S)) ++meet;
      } else {
        ++pc[4];
      }
    }
  }
  for (int k = 0; k < 8; ++k) f[16 + k] = squash(pc[k], 8);
  f[24] = squash(w.val_tid, 16);
  f[25] = squash(w.val_other, 16);
  f[26] = squash(w.max_if_depth, 16);
  f[27] = squash(w.max_loop_depth, 4);
  f[28] = squash(w.mem_in_if, 16);
  f[29] = squash(w.mem_in_loop, 16);
  {
    std::vector<int64_t> ivls;
    for (const MemStmt& m : w.mem) {
      if (!m.store) continue;
      if (std::find(ivls.begin(), ivls.end(), m.ivl) == ivls.end()) ivls.push_back(m.ivl);
    }
    f[30] = squash((int64_t)ivls.size(), 8);
  }
  f[31] = squash(meet, 8);
  for (size_t k = 0; k < 16; ++k) {
    float* s = f + 32 + 4 * k;
    if (k >= M) { s[0] = s[1] = s[2] = s[3] = 0.f; continue; }
    const MemStmt& m = w.mem[k];
    s[0] = m.store ? 1.f : -1.f;
    if (m.idx.ok) {
      const int64_t S = c.arrays[m.arr].size;
      s[1] = (float)m.idx.a / (float)(1 + (m.idx.a < 0 ? -m.idx.a : m.idx.a));
      s[2] = ratio(emod(m.idx.b, S), S);
    } else {
      s[1] = -2.f;
      s[2] = -2.f;
    }
    s[3] = ratio(m.ivl + 1, 8);
  }
  f[96] = squash(w.counts[Statement::BARRIER], 8);
  f[97] = squash(w.barriers_in_loops, 8);
  f[98] = squash(w.max_mem_in_ivl, 64);
  f[99] = squash(w.trip_sum, 64);
  f[100] = squash((int64_t)M, 64);
  f[101] = squash(w.counts[Statement::STORE], 64);
  {
    std::vector<int> arrs;
    for (const MemStmt& m : w.mem)
      if (m.store && std::find(arrs.begin(), arrs.end(), m.arr) == arrs.end()) arrs.push_back(m.arr);
    f[102] = squash((int64_t)arrs.size(), 8);
  }
  f[103] = 0.f;
}

}  // namespace

bool compile_program(const char* src, size_t len, Compiled* out, std::string* err, bool* is_limit) {
  *out = Compiled();
  *is_limit = false;
  try {
    Parser parser(tokenize(src, len), out);
    std::vector<Statement> body;
    parser.parse_kernel(&body);
    Bounds b;
    bound_block(body, *out, 1.0, &b);
    const double cap = 4.0e18;
    if (b.instr + 1 > 1.0e9) throw CompileError{1, 1, "static bound exceeds 10^9 instructions per work-item", true};
    if (b.stores + 2 > (double)((1u << 22) - 2))
      throw CompileError{1, 1, "static bound exceeds 2^22 store statements per work-group run", true};
    out->dyn_instr = (uint64_t)(b.instr + 1);
    out->dyn_mem = (uint64_t)(b.mem < cap ? b.mem : cap);
    out->dyn_logged_mem = (uint64_t)(b.logged < cap ? b.logged : cap);
    out->dyn_logged_local = (uint64_t)(b.logged_local < cap ? b.logged_local : cap);
    out->dyn_stores = (uint64_t)b.stores;
    out->dyn_mem_array.assign(out->arrays.size(), 0);
    for (size_t a = 0; a < b.arr.size() && a < out->arrays.size(); ++a)
      out->dyn_mem_array[a] = (uint64_t)(b.arr[a] < cap ? b.arr[a] : cap);
    out->max_intervals = (uint64_t)(b.barriers + 1);
    out->dyn_iters = (uint64_t)(b.iters < cap ? b.iters : cap);
    {
      const Compiled& cc = *out;
      IntervalBound lo = interval_block(body, {0, 0}, [&](int a) { return cc.arrays[a].written && !cc.arrays[a].global; });
      IntervalBound al = interval_block(body, {0, 0}, [&](int a) { return cc.arrays[a].written; });
      out->interval_logged_local = std::max(lo.worst, lo.open);
      out->interval_logged_all = std::max(al.worst, al.open);
    }
    static_features(body, *out, out->feat);
    Lowering low(out);
    low.run(body);
    return true;
  } catch (const CompileError& e) {
    *err = std::to_string(e.line) + ":" + std::to_string(e.col) + ": " + e.msg;
    *is_limit = e.limit;
    return false;
  }
}

}  // namespace rc
