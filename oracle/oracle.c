/*
 * oracle.c -- plain, slow, single-threaded CPU oracle of the concrete SIMD
 * race semantics of "Detecting Data Races on OpenCL Kernels with Symbolic
 * Execution" (Distefano, Dubreil).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke entry point and the
 * benchmark's CPU-baseline leg call this code.  It shares no code with the
 * GPU library: it has its own lexer, parser, interpreter and checker.
 *
 * Structure (each part cites the passage it follows):
 *   - lexer/parser:  the kernel language of Section 3 (expressions e, booleans
 *     b, commands Comm, kernel tuple K(Args)), widened to a structured surface
 *     syntax (if/for, expression indices) as the design notes list.
 *   - interpreter:   Section 4 thread-local rules (assign, store, load, assert,
 *     assume, barrier) run for every work-item of a work-group under the
 *     lockstep schedule, one statement at a time; Section 4 global rules give
 *     the barrier: all threads wait, then resume.
 *   - checker:       the race definition of Section 4 and the benign-race
 *     notion of Section 1 (equal-value writes are benign), made concrete as
 *     the pairwise check over each barrier interval's access log.  Pairs are
 *     enumerated naively inside (array, cell) buckets, or over the whole
 *     scope in literal mode.
 */
#include "oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <stdarg.h>
#include <ctype.h>

/* ------------------------------------------------------------------------ */
/* Seeded inputs: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), written from */
/* its published definition: state advances by the golden-ratio increment,  */
/* output is the variant-13 finaliser.  Counter form: the state for          */
/* (stream, idx) is seed + gamma * (stream * 2^32 + idx + 1).                */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ULL * counter;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int32_t orc_seeded_value(uint64_t seed, uint64_t stream, uint64_t idx,
                         int64_t lo, int64_t hi) {
  uint64_t z = splitmix64_at(seed, (stream << 32) + idx + 1);
  uint64_t u = z >> 32;                       /* top 32 bits */
  uint64_t range = (uint64_t)(hi - lo);       /* 1 .. 2^32 */
  uint64_t off = (u * range) >> 32;           /* < range */
  return (int32_t)(uint32_t)((uint64_t)lo + off);
}

/* ------------------------------------------------------------------------ */
/* Errors                                                                    */
/* ------------------------------------------------------------------------ */
static void set_err(char* err, int errlen, const char* fmt, ...) {
  if (!err || errlen <= 0) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(err, (size_t)errlen, fmt, ap);
  va_end(ap);
}

/* ------------------------------------------------------------------------ */
/* Lexer                                                                     */
/* ------------------------------------------------------------------------ */
enum { TK_EOF, TK_INT, TK_ID, TK_P };  /* TK_P: punctuation in tok.text */

typedef struct {
  int kind;
  int64_t ival;
  char text[64];
  int line, col;
} Tok;

typedef struct {
  const char* s;
  size_t pos, len;
  int line, col;
  Tok cur;
  char* err;
  int errlen;
  int failed;
} Lexer;

static const char* PUNCT[] = {
  ":=", "..", "<<", ">>", "<=", ">=", "==", "!=", "&&", "||",
  "[", "]", "(", ")", "{", "}", ";", ",", "+", "-", "*", "/", "%",
  "&", "|", "^", "~", "!", "<", ">", NULL
};

static void lex_fail(Lexer* L, int line, int col, const char* msg) {
  if (!L->failed) set_err(L->err, L->errlen, "%d:%d: %s", line, col, msg);
  L->failed = 1;
}

static void lex_adv_char(Lexer* L) {
  if (L->s[L->pos] == '\n') { L->line++; L->col = 1; } else { L->col++; }
  L->pos++;
}

static void lex_next(Lexer* L) {
  for (;;) {
    while (L->pos < L->len && isspace((unsigned char)L->s[L->pos])) lex_adv_char(L);
    if (L->pos + 1 < L->len && L->s[L->pos] == '/' && L->s[L->pos + 1] == '/') {
      while (L->pos < L->len && L->s[L->pos] != '\n') lex_adv_char(L);
      continue;
    }
    if (L->pos + 1 < L->len && L->s[L->pos] == '/' && L->s[L->pos + 1] == '*') {
      int ln = L->line, cl = L->col;
      lex_adv_char(L); lex_adv_char(L);
      while (L->pos + 1 < L->len && !(L->s[L->pos] == '*' && L->s[L->pos + 1] == '/')) lex_adv_char(L);
      if (L->pos + 1 >= L->len) { lex_fail(L, ln, cl, "unterminated comment"); L->cur.kind = TK_EOF; return; }
      lex_adv_char(L); lex_adv_char(L);
      continue;
    }
    break;
  }
  Tok* t = &L->cur;
  t->line = L->line; t->col = L->col; t->text[0] = 0; t->ival = 0;
  if (L->pos >= L->len) { t->kind = TK_EOF; strcpy(t->text, "<eof>"); return; }
  char c = L->s[L->pos];
  if (isdigit((unsigned char)c)) {
    uint64_t v = 0; int n = 0; int hex = 0;
    if (c == '0' && L->pos + 1 < L->len && (L->s[L->pos + 1] == 'x' || L->s[L->pos + 1] == 'X')) {
      hex = 1; lex_adv_char(L); lex_adv_char(L);
    }
    while (L->pos < L->len) {
      char d = L->s[L->pos]; int dv;
      if (isdigit((unsigned char)d)) dv = d - '0';
      else if (hex && isxdigit((unsigned char)d)) dv = 10 + (tolower((unsigned char)d) - 'a');
      else break;
      v = v * (hex ? 16u : 10u) + (uint64_t)dv;
      if (v > 0xFFFFFFFFULL) { lex_fail(L, t->line, t->col, "integer literal out of range"); v = 0; }
      n++; lex_adv_char(L);
    }
    if (n == 0) lex_fail(L, t->line, t->col, "malformed integer literal");
    if (L->pos < L->len && (isalpha((unsigned char)L->s[L->pos]) || L->s[L->pos] == '_'))
      lex_fail(L, t->line, t->col, "malformed integer literal");
    t->kind = TK_INT; t->ival = (int64_t)v;
    snprintf(t->text, sizeof t->text, "%llu", (unsigned long long)v);
    return;
  }
  if (isalpha((unsigned char)c) || c == '_') {
    int n = 0;
    while (L->pos < L->len && (isalnum((unsigned char)L->s[L->pos]) || L->s[L->pos] == '_')) {
      if (n < 63) t->text[n++] = L->s[L->pos];
      else { lex_fail(L, t->line, t->col, "identifier too long"); }
      lex_adv_char(L);
    }
    t->text[n] = 0; t->kind = TK_ID;
    return;
  }
  for (int i = 0; PUNCT[i]; i++) {
    size_t pl = strlen(PUNCT[i]);
    if (L->pos + pl <= L->len && strncmp(L->s + L->pos, PUNCT[i], pl) == 0) {
      strcpy(t->text, PUNCT[i]); t->kind = TK_P;
      for (size_t k = 0; k < pl; k++) lex_adv_char(L);
      return;
    }
  }
  lex_fail(L, t->line, t->col, "unexpected character");
  t->kind = TK_EOF;
}

/* ------------------------------------------------------------------------ */
/* AST                                                                       */
/* ------------------------------------------------------------------------ */
enum { E_CONST, E_VAR, E_SCALAR, E_TID, E_LID, E_GID, E_WGSIZE, E_NGROUPS,
       E_NTHREADS, E_NEG, E_NOT, E_BNOT, E_BIN };
enum { B_ADD, B_SUB, B_MUL, B_DIV, B_REM, B_MOD, B_AND, B_OR, B_XOR, B_SHL,
       B_SHR, B_LT, B_LE, B_GT, B_GE, B_EQ, B_NE, B_LAND, B_LOR, B_MIN, B_MAX };

typedef struct Expr {
  int kind, op;
  int32_t val;   /* E_CONST value; E_VAR / E_SCALAR index */
  struct Expr *a, *b;
} Expr;

enum { S_ASSIGN, S_LOAD, S_STORE, S_BARRIER, S_ASSUME, S_ASSERT, S_IF, S_FOR };

typedef struct Stmt {
  int kind, pc;
  int var;        /* destination / loop variable */
  int arr;        /* array id (global arrays first, then local arrays) */
  Expr *e1, *e2;  /* index / value / condition */
  struct Stmt** body; int nbody;
  struct Stmt** els;  int nels;
  int64_t lo, hi;  /* for-loop bounds */
} Stmt;

#define MAX_ARRAYS 16
#define MAX_SCALARS 16
#define MAX_VARS 64

struct orc_prog {
  char name[64];
  int n_global, n_local, n_scalars, n_vars;
  char arr_name[MAX_ARRAYS][64];
  int64_t arr_size[MAX_ARRAYS];
  char sc_name[MAX_SCALARS][64];
  char var_name[MAX_VARS][64];
  Stmt** body; int nbody;
  int n_stmts;
  /* arena for cleanup */
  void** allocs; size_t nallocs, capallocs;
};

static void* p_alloc(orc_prog* P, size_t sz) {
  void* m = calloc(1, sz);
  if (!m) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  if (P->nallocs == P->capallocs) {
    P->capallocs = P->capallocs ? 2 * P->capallocs : 256;
    P->allocs = (void**)realloc(P->allocs, P->capallocs * sizeof(void*));
  }
  P->allocs[P->nallocs++] = m;
  return m;
}

void orc_prog_free(orc_prog* P) {
  if (!P) return;
  for (size_t i = 0; i < P->nallocs; i++) free(P->allocs[i]);
  free(P->allocs);
  free(P);
}

/* ------------------------------------------------------------------------ */
/* Parser                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  Lexer L;
  orc_prog* P;
  int loopvars[32]; int nloop;   /* loop variables that may not be assigned */
  int depth;
} Parser;

static const char* KEYWORDS[] = {
  "kernel", "global", "local", "int", "barrier", "assume", "assert", "if",
  "else", "for", "in", "tid", "lid", "gid", "wgsize", "ngroups", "nthreads",
  "size", "min", "max", "mod", NULL
};

static int is_keyword(const char* s) {
  for (int i = 0; KEYWORDS[i]; i++) if (strcmp(s, KEYWORDS[i]) == 0) return 1;
  return 0;
}

static void pfail(Parser* ps, const char* fmt, ...) {
  if (ps->L.failed) return;
  char buf[200];
  va_list ap; va_start(ap, fmt); vsnprintf(buf, sizeof buf, fmt, ap); va_end(ap);
  set_err(ps->L.err, ps->L.errlen, "%d:%d: %s", ps->L.cur.line, ps->L.cur.col, buf);
  ps->L.failed = 1;
}

static int is_p(Parser* ps, const char* p) { return ps->L.cur.kind == TK_P && strcmp(ps->L.cur.text, p) == 0; }
static int is_id(Parser* ps, const char* s) { return ps->L.cur.kind == TK_ID && strcmp(ps->L.cur.text, s) == 0; }
static void expect_p(Parser* ps, const char* p) {
  if (!is_p(ps, p)) { pfail(ps, "expected '%s', found '%s'", p, ps->L.cur.text); return; }
  lex_next(&ps->L);
}
static void expect_id(Parser* ps, const char* s) {
  if (!is_id(ps, s)) { pfail(ps, "expected '%s', found '%s'", s, ps->L.cur.text); return; }
  lex_next(&ps->L);
}

static int find_array(orc_prog* P, const char* n) {
  for (int i = 0; i < P->n_global + P->n_local; i++) if (strcmp(P->arr_name[i], n) == 0) return i;
  return -1;
}
static int find_scalar(orc_prog* P, const char* n) {
  for (int i = 0; i < P->n_scalars; i++) if (strcmp(P->sc_name[i], n) == 0) return i;
  return -1;
}
static int find_var(orc_prog* P, const char* n) {
  for (int i = 0; i < P->n_vars; i++) if (strcmp(P->var_name[i], n) == 0) return i;
  return -1;
}
static int name_taken(orc_prog* P, const char* n) {
  return is_keyword(n) || find_array(P, n) >= 0 || find_scalar(P, n) >= 0 || find_var(P, n) >= 0;
}

static Expr* mk(Parser* ps, int kind, int op, int32_t val, Expr* a, Expr* b) {
  Expr* e = (Expr*)p_alloc(ps->P, sizeof(Expr));
  e->kind = kind; e->op = op; e->val = val; e->a = a; e->b = b;
  return e;
}

static Expr* parse_expr(Parser* ps);

static Expr* parse_primary(Parser* ps) {
  Tok t = ps->L.cur;
  if (ps->L.failed) return mk(ps, E_CONST, 0, 0, NULL, NULL);
  if (t.kind == TK_INT) { lex_next(&ps->L); return mk(ps, E_CONST, 0, (int32_t)(uint32_t)t.ival, NULL, NULL); }
  if (is_p(ps, "(")) { lex_next(&ps->L); Expr* e = parse_expr(ps); expect_p(ps, ")"); return e; }
  if (t.kind == TK_ID) {
    const char* s = t.text;
    if (!strcmp(s, "tid")) { lex_next(&ps->L); return mk(ps, E_TID, 0, 0, NULL, NULL); }
    if (!strcmp(s, "lid")) { lex_next(&ps->L); return mk(ps, E_LID, 0, 0, NULL, NULL); }
    if (!strcmp(s, "gid")) { lex_next(&ps->L); return mk(ps, E_GID, 0, 0, NULL, NULL); }
    if (!strcmp(s, "wgsize")) { lex_next(&ps->L); return mk(ps, E_WGSIZE, 0, 0, NULL, NULL); }
    if (!strcmp(s, "ngroups")) { lex_next(&ps->L); return mk(ps, E_NGROUPS, 0, 0, NULL, NULL); }
    if (!strcmp(s, "nthreads")) { lex_next(&ps->L); return mk(ps, E_NTHREADS, 0, 0, NULL, NULL); }
    if (!strcmp(s, "size")) {
      lex_next(&ps->L); expect_p(ps, "(");
      int a = -1;
      if (ps->L.cur.kind == TK_ID) a = find_array(ps->P, ps->L.cur.text);
      if (a < 0) { pfail(ps, "size() needs an array name"); return mk(ps, E_CONST, 0, 0, NULL, NULL); }
      lex_next(&ps->L); expect_p(ps, ")");
      return mk(ps, E_CONST, 0, (int32_t)ps->P->arr_size[a], NULL, NULL);
    }
    if (!strcmp(s, "min") || !strcmp(s, "max")) {
      int op = !strcmp(s, "min") ? B_MIN : B_MAX;
      lex_next(&ps->L); expect_p(ps, "(");
      Expr* a = parse_expr(ps); expect_p(ps, ",");
      Expr* b = parse_expr(ps); expect_p(ps, ")");
      return mk(ps, E_BIN, op, 0, a, b);
    }
    int v = find_var(ps->P, s);
    if (v >= 0) { lex_next(&ps->L); return mk(ps, E_VAR, 0, v, NULL, NULL); }
    int sc = find_scalar(ps->P, s);
    if (sc >= 0) { lex_next(&ps->L); return mk(ps, E_SCALAR, 0, sc, NULL, NULL); }
    if (find_array(ps->P, s) >= 0) { pfail(ps, "array '%s' cannot be read inside an expression", s); return mk(ps, E_CONST, 0, 0, NULL, NULL); }
    pfail(ps, "unknown name '%s'", s);
    return mk(ps, E_CONST, 0, 0, NULL, NULL);
  }
  pfail(ps, "expected an expression, found '%s'", t.text);
  return mk(ps, E_CONST, 0, 0, NULL, NULL);
}

static Expr* parse_unary(Parser* ps) {
  if (is_p(ps, "-")) { lex_next(&ps->L); return mk(ps, E_NEG, 0, 0, parse_unary(ps), NULL); }
  if (is_p(ps, "~")) { lex_next(&ps->L); return mk(ps, E_BNOT, 0, 0, parse_unary(ps), NULL); }
  if (is_p(ps, "!")) { lex_next(&ps->L); return mk(ps, E_NOT, 0, 0, parse_unary(ps), NULL); }
  return parse_primary(ps);
}

/* binary levels, loosest first */
typedef struct { const char* tok; int op; } OpTok;
static const OpTok LV0[] = {{"||", B_LOR}, {NULL, 0}};
static const OpTok LV1[] = {{"&&", B_LAND}, {NULL, 0}};
static const OpTok LV2[] = {{"|", B_OR}, {NULL, 0}};
static const OpTok LV3[] = {{"^", B_XOR}, {NULL, 0}};
static const OpTok LV4[] = {{"&", B_AND}, {NULL, 0}};
static const OpTok LV5[] = {{"==", B_EQ}, {"!=", B_NE}, {NULL, 0}};
static const OpTok LV6[] = {{"<", B_LT}, {"<=", B_LE}, {">", B_GT}, {">=", B_GE}, {NULL, 0}};
static const OpTok LV7[] = {{"<<", B_SHL}, {">>", B_SHR}, {NULL, 0}};
static const OpTok LV8[] = {{"+", B_ADD}, {"-", B_SUB}, {NULL, 0}};
static const OpTok LV9[] = {{"*", B_MUL}, {"/", B_DIV}, {"%", B_REM}, {"mod", B_MOD}, {NULL, 0}};
static const OpTok* LEVELS[] = {LV0, LV1, LV2, LV3, LV4, LV5, LV6, LV7, LV8, LV9};

static Expr* parse_level(Parser* ps, int lv) {
  if (lv == 10) return parse_unary(ps);
  Expr* a = parse_level(ps, lv + 1);
  for (;;) {
    if (ps->L.failed) return a;
    int found = -1;
    for (int i = 0; LEVELS[lv][i].tok; i++) {
      const char* k = LEVELS[lv][i].tok;
      if ((ps->L.cur.kind == TK_P || ps->L.cur.kind == TK_ID) && strcmp(ps->L.cur.text, k) == 0) { found = LEVELS[lv][i].op; break; }
    }
    if (found < 0) return a;
    lex_next(&ps->L);
    Expr* b = parse_level(ps, lv + 1);
    a = mk(ps, E_BIN, found, 0, a, b);
  }
}

static Expr* parse_expr(Parser* ps) { return parse_level(ps, 0); }

static int parse_int_literal(Parser* ps, int64_t* out) {
  int neg = 0;
  if (is_p(ps, "-")) { neg = 1; lex_next(&ps->L); }
  if (ps->L.cur.kind != TK_INT) { pfail(ps, "expected an integer literal"); return 0; }
  int64_t v = ps->L.cur.ival;
  lex_next(&ps->L);
  *out = neg ? -v : v;
  return 1;
}

static void parse_block(Parser* ps, Stmt*** out, int* n);

static int is_loopvar(Parser* ps, int v) {
  for (int i = 0; i < ps->nloop; i++) if (ps->loopvars[i] == v) return 1;
  return 0;
}

static Stmt* parse_stmt(Parser* ps) {
  orc_prog* P = ps->P;
  Stmt* s = (Stmt*)p_alloc(P, sizeof(Stmt));
  s->pc = P->n_stmts++;
  s->var = -1; s->arr = -1;
  if (is_id(ps, "barrier")) { lex_next(&ps->L); expect_p(ps, ";"); s->kind = S_BARRIER; return s; }
  if (is_id(ps, "assume") || is_id(ps, "assert")) {
    s->kind = is_id(ps, "assume") ? S_ASSUME : S_ASSERT;
    lex_next(&ps->L); expect_p(ps, "("); s->e1 = parse_expr(ps); expect_p(ps, ")"); expect_p(ps, ";");
    return s;
  }
  if (is_id(ps, "if")) {
    s->kind = S_IF;
    lex_next(&ps->L); expect_p(ps, "("); s->e1 = parse_expr(ps); expect_p(ps, ")");
    ps->depth++;
    if (ps->depth > 16) pfail(ps, "nesting deeper than 16");
    parse_block(ps, &s->body, &s->nbody);
    if (is_id(ps, "else")) { lex_next(&ps->L); parse_block(ps, &s->els, &s->nels); }
    ps->depth--;
    return s;
  }
  if (is_id(ps, "for")) {
    s->kind = S_FOR;
    lex_next(&ps->L);
    if (ps->L.cur.kind != TK_ID) { pfail(ps, "expected a loop variable"); return s; }
    s->var = find_var(P, ps->L.cur.text);
    if (s->var < 0) { pfail(ps, "loop variable '%s' is not a declared private variable", ps->L.cur.text); return s; }
    if (is_loopvar(ps, s->var)) { pfail(ps, "loop variable '%s' reused by a nested loop", ps->L.cur.text); return s; }
    lex_next(&ps->L); expect_id(ps, "in");
    parse_int_literal(ps, &s->lo); expect_p(ps, ".."); parse_int_literal(ps, &s->hi);
    if (s->lo < INT32_MIN || s->lo > INT32_MAX || s->hi < INT32_MIN || s->hi > INT32_MAX) pfail(ps, "loop bound out of range");
    ps->depth++;
    if (ps->depth > 16) pfail(ps, "nesting deeper than 16");
    ps->loopvars[ps->nloop++] = s->var;
    parse_block(ps, &s->body, &s->nbody);
    ps->nloop--;
    ps->depth--;
    return s;
  }
  if (ps->L.cur.kind != TK_ID) { pfail(ps, "expected a statement, found '%s'", ps->L.cur.text); return s; }
  char name[64]; strcpy(name, ps->L.cur.text);
  int a = find_array(P, name);
  if (a >= 0) {  /* store */
    s->kind = S_STORE; s->arr = a;
    lex_next(&ps->L); expect_p(ps, "["); s->e1 = parse_expr(ps); expect_p(ps, "]");
    expect_p(ps, ":="); s->e2 = parse_expr(ps); expect_p(ps, ";");
    return s;
  }
  int v = find_var(P, name);
  if (v < 0) {
    if (find_scalar(P, name) >= 0) pfail(ps, "scalar parameter '%s' is read-only", name);
    else pfail(ps, "unknown name '%s'", name);
    return s;
  }
  if (is_loopvar(ps, v)) { pfail(ps, "loop variable '%s' assigned inside its loop", name); return s; }
  lex_next(&ps->L); expect_p(ps, ":=");
  s->var = v;
  if (ps->L.cur.kind == TK_ID && find_array(P, ps->L.cur.text) >= 0) {
    s->kind = S_LOAD; s->arr = find_array(P, ps->L.cur.text);
    lex_next(&ps->L); expect_p(ps, "["); s->e1 = parse_expr(ps); expect_p(ps, "]"); expect_p(ps, ";");
    return s;
  }
  s->kind = S_ASSIGN; s->e1 = parse_expr(ps); expect_p(ps, ";");
  return s;
}

static void parse_block(Parser* ps, Stmt*** out, int* n) {
  expect_p(ps, "{");
  int cap = 8; int cnt = 0;
  Stmt** arr = (Stmt**)p_alloc(ps->P, (size_t)cap * sizeof(Stmt*));
  while (!ps->L.failed && !is_p(ps, "}") && ps->L.cur.kind != TK_EOF) {
    if (cnt == cap) {
      Stmt** na = (Stmt**)p_alloc(ps->P, (size_t)cap * 2 * sizeof(Stmt*));
      memcpy(na, arr, (size_t)cap * sizeof(Stmt*)); arr = na; cap *= 2;
    }
    arr[cnt++] = parse_stmt(ps);
  }
  expect_p(ps, "}");
  *out = arr; *n = cnt;
}

orc_prog* orc_parse(const char* src, char* err, int errlen) {
  orc_prog* P = (orc_prog*)calloc(1, sizeof(orc_prog));
  Parser ps; memset(&ps, 0, sizeof ps);
  ps.P = P;
  ps.L.s = src; ps.L.len = strlen(src); ps.L.line = 1; ps.L.col = 1;
  ps.L.err = err; ps.L.errlen = errlen;
  lex_next(&ps.L);
  expect_id(&ps, "kernel");
  if (ps.L.cur.kind != TK_ID || is_keyword(ps.L.cur.text)) pfail(&ps, "expected the kernel name");
  else { strcpy(P->name, ps.L.cur.text); lex_next(&ps.L); }
  expect_p(&ps, "(");
  int first = 1;
  while (!ps.L.failed && !is_p(&ps, ")")) {
    if (!first) expect_p(&ps, ",");
    first = 0;
    if (is_id(&ps, "global")) {
      lex_next(&ps.L); expect_id(&ps, "int");
      if (ps.L.cur.kind != TK_ID || name_taken(P, ps.L.cur.text)) { pfail(&ps, "bad or duplicate array name"); break; }
      if (P->n_global >= 8) { pfail(&ps, "more than 8 global arrays"); break; }
      if (P->n_local > 0) { pfail(&ps, "internal: locals before globals"); break; }
      int id = P->n_global++;
      strcpy(P->arr_name[id], ps.L.cur.text); lex_next(&ps.L);
      expect_p(&ps, "[");
      int64_t sz = 0; parse_int_literal(&ps, &sz);
      if (!ps.L.failed && (sz < 1 || sz > (1 << 24))) pfail(&ps, "array size must be in [1, 2^24]");
      P->arr_size[id] = sz;
      expect_p(&ps, "]");
    } else if (is_id(&ps, "int")) {
      lex_next(&ps.L);
      if (ps.L.cur.kind != TK_ID || name_taken(P, ps.L.cur.text)) { pfail(&ps, "bad or duplicate scalar name"); break; }
      if (P->n_scalars >= 16) { pfail(&ps, "more than 16 scalar parameters"); break; }
      strcpy(P->sc_name[P->n_scalars++], ps.L.cur.text); lex_next(&ps.L);
    } else { pfail(&ps, "expected a parameter ('global int A[N]' or 'int s')"); break; }
  }
  expect_p(&ps, ")");
  expect_p(&ps, "{");
  /* declarations */
  while (!ps.L.failed) {
    if (is_id(&ps, "local")) {
      lex_next(&ps.L); expect_id(&ps, "int");
      if (ps.L.cur.kind != TK_ID || name_taken(P, ps.L.cur.text)) { pfail(&ps, "bad or duplicate array name"); break; }
      if (P->n_local >= 8) { pfail(&ps, "more than 8 local arrays"); break; }
      int id = P->n_global + P->n_local++;
      strcpy(P->arr_name[id], ps.L.cur.text); lex_next(&ps.L);
      expect_p(&ps, "[");
      int64_t sz = 0; parse_int_literal(&ps, &sz);
      if (!ps.L.failed && (sz < 1 || sz > (1 << 24))) pfail(&ps, "array size must be in [1, 2^24]");
      P->arr_size[id] = sz;
      expect_p(&ps, "]"); expect_p(&ps, ";");
    } else if (is_id(&ps, "int")) {
      lex_next(&ps.L);
      for (;;) {
        if (ps.L.cur.kind != TK_ID || name_taken(P, ps.L.cur.text)) { pfail(&ps, "bad or duplicate variable name"); break; }
        if (P->n_vars >= 32) { pfail(&ps, "more than 32 private variables"); break; }
        strcpy(P->var_name[P->n_vars++], ps.L.cur.text); lex_next(&ps.L);
        if (is_p(&ps, ",")) { lex_next(&ps.L); continue; }
        break;
      }
      expect_p(&ps, ";");
    } else break;
  }
  /* statements until the closing brace */
  int cap = 16, cnt = 0;
  Stmt** arr = (Stmt**)p_alloc(P, (size_t)cap * sizeof(Stmt*));
  while (!ps.L.failed && !is_p(&ps, "}") && ps.L.cur.kind != TK_EOF) {
    if (cnt == cap) {
      Stmt** na = (Stmt**)p_alloc(P, (size_t)cap * 2 * sizeof(Stmt*));
      memcpy(na, arr, (size_t)cap * sizeof(Stmt*)); arr = na; cap *= 2;
    }
    arr[cnt++] = parse_stmt(&ps);
  }
  expect_p(&ps, "}");
  if (!ps.L.failed && ps.L.cur.kind != TK_EOF) pfail(&ps, "trailing input after the kernel");
  if (!ps.L.failed && P->n_stmts > 4096) pfail(&ps, "more than 4096 statements");
  P->body = arr; P->nbody = cnt;
  if (ps.L.failed) { orc_prog_free(P); return NULL; }
  return P;
}

int orc_n_global_arrays(const orc_prog* P) { return P->n_global; }
int orc_n_local_arrays(const orc_prog* P) { return P->n_local; }
int orc_n_scalars(const orc_prog* P) { return P->n_scalars; }
int64_t orc_global_array(const orc_prog* P, int i, char* name, int namelen) {
  if (i < 0 || i >= P->n_global) return -1;
  if (name) snprintf(name, (size_t)namelen, "%s", P->arr_name[i]);
  return P->arr_size[i];
}
int orc_scalar(const orc_prog* P, int i, char* name, int namelen) {
  if (i < 0 || i >= P->n_scalars) return -1;
  if (name) snprintf(name, (size_t)namelen, "%s", P->sc_name[i]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* int32 arithmetic: two's complement, wrapping; the operator table is the   */
/* reading of Section 3's open-ended operator set listed in the design notes.*/
/* ------------------------------------------------------------------------ */
static int32_t wrap(int64_t v) { return (int32_t)(uint32_t)(uint64_t)v; }

static int32_t do_bin(int op, int32_t x, int32_t y, int* divzero) {
  switch (op) {
    case B_ADD: return wrap((int64_t)x + (int64_t)y);
    case B_SUB: return wrap((int64_t)x - (int64_t)y);
    case B_MUL: return wrap((int64_t)x * (int64_t)y);
    case B_DIV:
      if (y == 0) { *divzero = 1; return 0; }
      if (x == INT32_MIN && y == -1) return INT32_MIN;
      return x / y;                                   /* C99: truncates */
    case B_REM:
      if (y == 0) { *divzero = 1; return 0; }
      if (x == INT32_MIN && y == -1) return 0;
      return x % y;                                   /* sign of dividend */
    case B_MOD: {
      if (y == 0) { *divzero = 1; return 0; }
      int64_t r = (int64_t)x % (int64_t)y;
      int64_t ay = y < 0 ? -(int64_t)y : (int64_t)y;
      if (r < 0) r += ay;                             /* Euclidean: 0 <= r < |y| */
      return (int32_t)r;
    }
    case B_AND: return x & y;
    case B_OR: return x | y;
    case B_XOR: return x ^ y;
    case B_SHL: return (int32_t)((uint32_t)x << ((uint32_t)y & 31u));
    case B_SHR: {  /* arithmetic shift written out without relying on >> of negatives */
      uint32_t s = (uint32_t)y & 31u;
      int64_t q = (int64_t)x;
      for (uint32_t k = 0; k < s; k++) q = (q >= 0) ? q / 2 : (q - 1) / 2;
      return (int32_t)q;
    }
    case B_LT: return x < y;
    case B_LE: return x <= y;
    case B_GT: return x > y;
    case B_GE: return x >= y;
    case B_EQ: return x == y;
    case B_NE: return x != y;
    case B_LAND: return (x != 0) && (y != 0);
    case B_LOR: return (x != 0) || (y != 0);
    case B_MIN: return x < y ? x : y;
    case B_MAX: return x > y ? x : y;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Interpreter state                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t array, cell, tid, gid, interval;
  int32_t is_write, value;
} Access;

typedef struct {
  Access* a; size_t n, cap;
} AccessLog;

static void log_push(AccessLog* L, Access x) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 1024;
    L->a = (Access*)realloc(L->a, L->cap * sizeof(Access));
    if (!L->a) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  }
  L->a[L->n++] = x;
}

typedef struct {
  orc_record* r; size_t n, cap;
} RecList;

static void rec_push(RecList* R, orc_record x) {
  if (R->n == R->cap) {
    R->cap = R->cap ? 2 * R->cap : 256;
    R->r = (orc_record*)realloc(R->r, R->cap * sizeof(orc_record));
    if (!R->r) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  }
  R->r[R->n++] = x;
}

typedef struct {
  const orc_prog* P;
  uint32_t G, W, gid;
  uint64_t seed;
  uint32_t instance;
  int flags;
  int32_t scalar_val[MAX_SCALARS];
  /* global memory: initial contents (shared) plus this group's view */
  int32_t* init[MAX_ARRAYS];
  int32_t* view[MAX_ARRAYS];
  unsigned char* written[MAX_ARRAYS];
  /* local arrays of this group */
  int32_t* loc[MAX_ARRAYS];
  /* private variables: vars[v * W + lid] */
  int32_t* vars;
  /* logs */
  AccessLog interval_log;   /* accesses of the current interval */
  AccessLog* inter_log;     /* global-array accesses of all groups */
  uint32_t interval;
  uint64_t n_accesses;
  uint64_t iterations, step_limit;   /* loop iterations started by the group; its limit */
  /* fault of this group */
  int fault_code; uint32_t fault_pc, fault_lid;
  RecList* recs;
  uint32_t n_race_cells, n_benign_cells;
} Group;

enum { ST_OK = 0, ST_OOB = 1, ST_DIV = 2, ST_ASSERT = 3, ST_ASSUME = 4, ST_BARDIV = 5, ST_STEP_LIMIT = 6 };

static int32_t eval(Group* g, const Expr* e, uint32_t lid, int* dz) {
  switch (e->kind) {
    case E_CONST: return e->val;
    case E_VAR: return g->vars[(size_t)e->val * g->W + lid];
    case E_SCALAR: return g->scalar_val[e->val];
    case E_TID: return wrap((int64_t)g->gid * g->W + lid);
    case E_LID: return (int32_t)lid;
    case E_GID: return (int32_t)g->gid;
    case E_WGSIZE: return (int32_t)g->W;
    case E_NGROUPS: return (int32_t)g->G;
    case E_NTHREADS: return wrap((int64_t)g->G * g->W);
    case E_NEG: return wrap(-(int64_t)eval(g, e->a, lid, dz));
    case E_BNOT: return ~eval(g, e->a, lid, dz);
    case E_NOT: return eval(g, e->a, lid, dz) == 0;
    case E_BIN: {
      /* both operands are always evaluated (no short circuit) */
      int32_t x = eval(g, e->a, lid, dz);
      int32_t y = eval(g, e->b, lid, dz);
      return do_bin(e->op, x, y, dz);
    }
  }
  return 0;
}

static int is_global(const Group* g, int arr) { return arr < g->P->n_global; }

static int32_t mem_read(Group* g, int arr, uint32_t cell) {
  if (!is_global(g, arr)) return g->loc[arr][cell];
  if (g->written[arr][cell]) return g->view[arr][cell];
  return g->init[arr][cell];
}

static void mem_write(Group* g, int arr, uint32_t cell, int32_t v) {
  if (!is_global(g, arr)) { g->loc[arr][cell] = v; return; }
  g->view[arr][cell] = v;
  g->written[arr][cell] = 1;
}

/* ------------------------------------------------------------------------ */
/* The race check of one scope: naive pairs inside (array, cell) buckets.    */
/* A pair of accesses is eligible when it is made by two different threads   */
/* (INTRA) or two different work-groups (INTER) and one of them writes.      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int any, rw, wwd, wws;
  uint32_t rw_a, rw_b, wwd_a, wwd_b, wws_a, wws_b;
} PairState;

static void pair_min(int* have, uint32_t* a, uint32_t* b, uint32_t x, uint32_t y) {
  uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
  if (!*have || lo < *a || (lo == *a && hi < *b)) { *a = lo; *b = hi; }
  *have = 1;
}

static void classify_pair(PairState* s, const Access* p, const Access* q, int inter) {
  if (p->array != q->array || p->cell != q->cell) return;
  if (inter ? (p->gid == q->gid) : (p->tid == q->tid)) return;
  if (!p->is_write && !q->is_write) return;
  s->any = 1;
  if (p->is_write && q->is_write) {
    if (p->value != q->value) pair_min(&s->wwd, &s->wwd_a, &s->wwd_b, p->tid, q->tid);
    else pair_min(&s->wws, &s->wws_a, &s->wws_b, p->tid, q->tid);
  } else {
    pair_min(&s->rw, &s->rw_a, &s->rw_b, p->tid, q->tid);
  }
}

static void emit_record(Group* g, const PairState* s, uint32_t array, uint32_t cell, int inter,
                        uint32_t gid, uint32_t interval) {
  if (!s->any) return;
  orc_record r; memset(&r, 0, sizeof r);
  r.instance = g->instance;
  r.gid = inter ? 0xFFFFFFFFu : gid;
  r.interval = inter ? 0 : interval;
  r.array = (uint16_t)array;
  r.cell = cell;
  r.rw_a = r.rw_b = r.ww_a = r.ww_b = 0xFFFFFFFFu;
  uint16_t label = 0;
  if (s->rw) { label |= 1; r.rw_a = s->rw_a; r.rw_b = s->rw_b; }
  if (s->wwd) { label |= 2; r.ww_a = s->wwd_a; r.ww_b = s->wwd_b; }
  if (!label) { label = 4; r.ww_a = s->wws_a; r.ww_b = s->wws_b; }
  r.label = label;
  if (label & 3) g->n_race_cells++; else g->n_benign_cells++;
  rec_push(g->recs, r);
}

/* bucketing key of one access: (array, cell), then its position in the log */
typedef struct { uint32_t array, cell; size_t pos; } CellKey;
static int cmp_cell_key(const void* x, const void* y) {
  const CellKey* a = (const CellKey*)x;
  const CellKey* b = (const CellKey*)y;
  if (a->array != b->array) return a->array < b->array ? -1 : 1;
  if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
  return a->pos < b->pos ? -1 : (a->pos > b->pos ? 1 : 0);
}

static void check_scope(Group* g, const Access* acc, size_t n, int inter,
                        uint32_t gid, uint32_t interval) {
  if (n == 0) return;
  if (g->flags & ORC_LITERAL_PAIRS) {
    /* literal mode: every pair of the scope; collect per (array, cell) */
    /* gather distinct cells first (quadratic, tiny inputs only) */
    size_t* cells = (size_t*)malloc(n * sizeof(size_t)); size_t nc = 0;
    for (size_t i = 0; i < n; i++) {
      int seen = 0;
      for (size_t k = 0; k < nc; k++)
        if (acc[cells[k]].array == acc[i].array && acc[cells[k]].cell == acc[i].cell) { seen = 1; break; }
      if (!seen) cells[nc++] = i;
    }
    for (size_t k = 0; k < nc; k++) {
      PairState s; memset(&s, 0, sizeof s);
      uint32_t A = acc[cells[k]].array, C = acc[cells[k]].cell;
      for (size_t i = 0; i < n; i++)
        for (size_t j = i + 1; j < n; j++)
          if (acc[i].array == A && acc[i].cell == C) classify_pair(&s, &acc[i], &acc[j], inter);
      emit_record(g, &s, A, C, inter, gid, interval);
    }
    free(cells);
    return;
  }
  CellKey* keys = (CellKey*)malloc(n * sizeof(CellKey));
  size_t* idx = (size_t*)malloc(n * sizeof(size_t));
  for (size_t i = 0; i < n; i++) { keys[i].array = acc[i].array; keys[i].cell = acc[i].cell; keys[i].pos = i; }
  qsort(keys, n, sizeof(CellKey), cmp_cell_key);
  for (size_t i = 0; i < n; i++) idx[i] = keys[i].pos;
  free(keys);
  size_t i = 0;
  while (i < n) {
    size_t j = i;
    while (j < n && acc[idx[j]].array == acc[idx[i]].array && acc[idx[j]].cell == acc[idx[i]].cell) j++;
    PairState s; memset(&s, 0, sizeof s);
    /* every eligible pair holds a write: enumerate each unordered pair once, */
    /* from its write (both orders for read+write, p<q for write+write)       */
    for (size_t p = i; p < j; p++) {
      if (!acc[idx[p]].is_write) continue;
      for (size_t q = i; q < j; q++) {
        if (q == p) continue;
        if (acc[idx[q]].is_write && q < p) continue;
        classify_pair(&s, &acc[idx[p]], &acc[idx[q]], inter);
      }
    }
    emit_record(g, &s, acc[idx[i]].array, acc[idx[i]].cell, inter, gid, interval);
    i = j;
  }
  free(idx);
}

/* Closing an interval: the global rule that releases the barrier (Section 4),  */
/* with the race rule made concrete as the pairwise check of the interval log. */
static void close_interval(Group* g) {
  check_scope(g, g->interval_log.a, g->interval_log.n, 0, g->gid, g->interval);
  g->interval_log.n = 0;
  g->interval++;
}

static void record_access(Group* g, int arr, uint32_t cell, uint32_t lid, int is_write, int32_t value) {
  Access x;
  x.array = (uint32_t)arr; x.cell = cell;
  x.tid = g->gid * g->W + lid; x.gid = g->gid; x.interval = g->interval;
  x.is_write = is_write; x.value = is_write ? value : 0;
  log_push(&g->interval_log, x);
  if (is_global(g, arr) && g->G > 1) log_push(g->inter_log, x);
  g->n_accesses++;
}

/* statement results */
enum { RUN_OK = 0, RUN_FAULT = 1 };

static int set_fault(Group* g, const Stmt* s, int code, uint32_t lid) {
  g->fault_code = code; g->fault_pc = (uint32_t)s->pc; g->fault_lid = lid;
  return RUN_FAULT;
}

static int exec_block(Group* g, Stmt* const* body, int n, const unsigned char* mask);

static int any_set(const unsigned char* m, uint32_t W) {
  for (uint32_t i = 0; i < W; i++) if (m[i]) return 1;
  return 0;
}

static int exec_stmt(Group* g, const Stmt* s, const unsigned char* mask) {
  uint32_t W = g->W;
  const orc_prog* P = g->P;
  switch (s->kind) {
    case S_ASSIGN: {   /* v := e  (thread-local assignment rule) */
      int32_t* tmp = (int32_t*)malloc(W * sizeof(int32_t));
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        int dz = 0; tmp[l] = eval(g, s->e1, l, &dz);
        if (dz) { free(tmp); return set_fault(g, s, ST_DIV, l); }
      }
      for (uint32_t l = 0; l < W; l++) if (mask[l]) g->vars[(size_t)s->var * W + l] = tmp[l];
      free(tmp);
      return RUN_OK;
    }
    case S_LOAD: {     /* v := a[e]  (load rule, reading R1 of the notes) */
      int32_t* idx = (int32_t*)malloc(W * sizeof(int32_t));
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        int dz = 0; idx[l] = eval(g, s->e1, l, &dz);
        int code = dz ? ST_DIV : ((idx[l] < 0 || (int64_t)idx[l] >= P->arr_size[s->arr]) ? ST_OOB : 0);
        if (code) { free(idx); return set_fault(g, s, code, l); }
      }
      /* all reads of the statement see the state before it */
      int32_t* val = (int32_t*)malloc(W * sizeof(int32_t));
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        val[l] = mem_read(g, s->arr, (uint32_t)idx[l]);
        record_access(g, s->arr, (uint32_t)idx[l], l, 0, 0);
      }
      for (uint32_t l = 0; l < W; l++) if (mask[l]) g->vars[(size_t)s->var * W + l] = val[l];
      free(idx); free(val);
      return RUN_OK;
    }
    case S_STORE: {    /* a[e] := e'  (store rule); ascending tid, last one stays */
      int32_t* idx = (int32_t*)malloc(W * sizeof(int32_t));
      int32_t* val = (int32_t*)malloc(W * sizeof(int32_t));
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        int dz = 0;
        idx[l] = eval(g, s->e1, l, &dz);
        val[l] = eval(g, s->e2, l, &dz);
        int code = dz ? ST_DIV : ((idx[l] < 0 || (int64_t)idx[l] >= P->arr_size[s->arr]) ? ST_OOB : 0);
        if (code) { free(idx); free(val); return set_fault(g, s, code, l); }
      }
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        mem_write(g, s->arr, (uint32_t)idx[l], val[l]);
        record_access(g, s->arr, (uint32_t)idx[l], l, 1, val[l]);
      }
      free(idx); free(val);
      return RUN_OK;
    }
    case S_ASSUME:
    case S_ASSERT: {   /* assume false -> no continuation; assert false -> error */
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        int dz = 0; int32_t c = eval(g, s->e1, l, &dz);
        if (dz) return set_fault(g, s, ST_DIV, l);
        if (c == 0) return set_fault(g, s, s->kind == S_ASSUME ? ST_ASSUME : ST_ASSERT, l);
      }
      return RUN_OK;
    }
    case S_BARRIER: {  /* every thread of the group must arrive */
      for (uint32_t l = 0; l < W; l++) if (!mask[l]) return set_fault(g, s, ST_BARDIV, l);
      close_interval(g);
      return RUN_OK;
    }
    case S_IF: {
      unsigned char* mt = (unsigned char*)calloc(W, 1);
      unsigned char* me = (unsigned char*)calloc(W, 1);
      for (uint32_t l = 0; l < W; l++) {
        if (!mask[l]) continue;
        int dz = 0; int32_t c = eval(g, s->e1, l, &dz);
        if (dz) { free(mt); free(me); return set_fault(g, s, ST_DIV, l); }
        if (c != 0) mt[l] = 1; else me[l] = 1;
      }
      int r = RUN_OK;
      if (any_set(mt, W)) r = exec_block(g, s->body, s->nbody, mt);
      if (r == RUN_OK && any_set(me, W)) r = exec_block(g, s->els, s->nels, me);
      free(mt); free(me);
      return r;
    }
    case S_FOR: {
      int64_t iters = s->hi - s->lo; if (iters < 0) iters = 0;
      for (int64_t j = 0; j < iters; j++) {
        /* the safety net of reading R13: a group that would start more loop */
        /* iterations than its limit stops here, reported for its first      */
        /* work-item (every work-item of the group reaches the limit)        */
        if (++g->iterations > g->step_limit) return set_fault(g, s, ST_STEP_LIMIT, 0);
        for (uint32_t l = 0; l < W; l++) if (mask[l]) g->vars[(size_t)s->var * W + l] = wrap(s->lo + j);
        int r = exec_block(g, s->body, s->nbody, mask);
        if (r != RUN_OK) return r;
      }
      for (uint32_t l = 0; l < W; l++) if (mask[l]) g->vars[(size_t)s->var * W + l] = wrap(s->lo + iters);
      return RUN_OK;
    }
  }
  return RUN_OK;
}

static int exec_block(Group* g, Stmt* const* body, int n, const unsigned char* mask) {
  for (int i = 0; i < n; i++) {
    int r = exec_stmt(g, body[i], mask);
    if (r != RUN_OK) return r;
  }
  return RUN_OK;
}

/* ------------------------------------------------------------------------ */
/* Canonical record order                                                    */
/* ------------------------------------------------------------------------ */
static int cmp_record(const void* x, const void* y) {
  const orc_record* a = (const orc_record*)x;
  const orc_record* b = (const orc_record*)y;
  if (a->instance != b->instance) return a->instance < b->instance ? -1 : 1;
  /* INTRA scopes (gid, interval) first, INTER (gid = all ones) last */
  if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
  if (a->interval != b->interval) return a->interval < b->interval ? -1 : 1;
  if (a->array != b->array) return a->array < b->array ? -1 : 1;
  if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Driver                                                                    */
/* ------------------------------------------------------------------------ */
int orc_run(const orc_prog* P, uint32_t G, uint32_t W,
            const orc_bind* arrays, int n_arrays,
            const orc_bind* scalars, int n_scalars,
            uint64_t seed, uint32_t instance, int flags, int final_array,
            orc_result* out, char* err, int errlen) {
  return orc_run_limit(P, G, W, arrays, n_arrays, scalars, n_scalars, seed, instance, flags, final_array,
                       ORC_STEP_LIMIT, out, err, errlen);
}

int orc_run_limit(const orc_prog* P, uint32_t G, uint32_t W,
                  const orc_bind* arrays, int n_arrays,
                  const orc_bind* scalars, int n_scalars,
                  uint64_t seed, uint32_t instance, int flags, int final_array, uint64_t step_limit,
                  orc_result* out, char* err, int errlen) {
  memset(out, 0, sizeof *out);
  if (W < 1 || W > 1024 || G < 1 || (uint64_t)G * W >= (1ull << 26)) {
    set_err(err, errlen, "bad launch shape: need 1 <= W <= 1024, G >= 1, G*W < 2^26");
    return -1;
  }
  if (n_arrays != P->n_global || n_scalars != P->n_scalars) {
    set_err(err, errlen, "binding count mismatch: program has %d global arrays and %d scalars",
            P->n_global, P->n_scalars);
    return -1;
  }
  if (final_array >= P->n_global) { set_err(err, errlen, "final_array out of range"); return -1; }
  Group g; memset(&g, 0, sizeof g);
  g.P = P; g.G = G; g.W = W; g.seed = seed; g.instance = instance; g.flags = flags; g.step_limit = step_limit;
  for (int j = 0; j < P->n_scalars; j++) {
    const orc_bind* b = &scalars[j];
    if (b->kind == 1) g.scalar_val[j] = *b->data;
    else {
      if (b->hi - b->lo < 1 || b->hi - b->lo > (1ll << 32)) { set_err(err, errlen, "bad seeded range"); return -1; }
      g.scalar_val[j] = orc_seeded_value(seed, 0x10000u + (uint64_t)j, 0, b->lo, b->hi);
    }
  }
  for (int a = 0; a < P->n_global; a++) {
    const orc_bind* b = &arrays[a];
    int64_t n = P->arr_size[a];
    g.init[a] = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (b->kind == 1) memcpy(g.init[a], b->data, (size_t)n * sizeof(int32_t));
    else {
      if (b->hi - b->lo < 1 || b->hi - b->lo > (1ll << 32)) { set_err(err, errlen, "bad seeded range"); return -1; }
      for (int64_t c = 0; c < n; c++) g.init[a][c] = orc_seeded_value(seed, (uint64_t)a, (uint64_t)c, b->lo, b->hi);
    }
  }
  int32_t* final_mem = NULL;
  if (final_array >= 0) {
    final_mem = (int32_t*)malloc((size_t)P->arr_size[final_array] * sizeof(int32_t));
    memcpy(final_mem, g.init[final_array], (size_t)P->arr_size[final_array] * sizeof(int32_t));
  }
  AccessLog inter_log; memset(&inter_log, 0, sizeof inter_log);
  RecList recs; memset(&recs, 0, sizeof recs);
  g.inter_log = &inter_log; g.recs = &recs;
  unsigned char* full = (unsigned char*)malloc(W);
  memset(full, 1, W);
  int inst_status = 0; uint32_t f_gid = 0xFFFFFFFFu, f_pc = 0xFFFFFFFFu, f_tid = 0xFFFFFFFFu;
  uint32_t total_intervals = 0; uint64_t total_acc = 0;
  g.vars = (int32_t*)malloc((size_t)(P->n_vars ? P->n_vars : 1) * W * sizeof(int32_t));
  /* Each work-group runs on its own view of global memory (initial contents */
  /* plus its own writes); barriers synchronise one work-group.              */
  for (uint32_t gid = 0; gid < G; gid++) {
    g.gid = gid; g.interval = 0; g.n_accesses = 0; g.fault_code = 0; g.iterations = 0;
    memset(g.vars, 0, (size_t)(P->n_vars ? P->n_vars : 1) * W * sizeof(int32_t));
    for (int a = 0; a < P->n_global; a++) {
      g.view[a] = (int32_t*)calloc((size_t)P->arr_size[a], sizeof(int32_t));
      g.written[a] = (unsigned char*)calloc((size_t)P->arr_size[a], 1);
    }
    for (int a = P->n_global; a < P->n_global + P->n_local; a++)
      g.loc[a] = (int32_t*)calloc((size_t)P->arr_size[a], sizeof(int32_t));
    int r = exec_block(&g, P->body, P->nbody, full);
    /* exit, or a fault: the last (possibly partial) interval is closed too */
    close_interval(&g);
    total_intervals += g.interval;
    total_acc += g.n_accesses;
    if (r == RUN_FAULT && f_gid == 0xFFFFFFFFu) {
      inst_status = g.fault_code; f_gid = gid; f_pc = g.fault_pc; f_tid = gid * W + g.fault_lid;
    }
    if (final_mem) {
      for (int64_t c = 0; c < P->arr_size[final_array]; c++)
        if (g.written[final_array][c]) final_mem[c] = g.view[final_array][c];
    }
    for (int a = 0; a < P->n_global; a++) { free(g.view[a]); free(g.written[a]); g.view[a] = NULL; g.written[a] = NULL; }
    for (int a = P->n_global; a < P->n_global + P->n_local; a++) { free(g.loc[a]); g.loc[a] = NULL; }
  }
  /* INTER scope: global-array accesses of different work-groups, whole run */
  if (G > 1) check_scope(&g, inter_log.a, inter_log.n, 1, 0, 0);
  if (recs.n > 1) qsort(recs.r, recs.n, sizeof(orc_record), cmp_record);
  out->records = recs.r; out->n_records = recs.n;
  out->summary.n_accesses = total_acc;
  out->summary.n_race_cells = g.n_race_cells;
  out->summary.n_benign_cells = g.n_benign_cells;
  out->summary.n_intervals = total_intervals;
  out->summary.status = inst_status;
  out->summary.fault_gid = f_gid; out->summary.fault_pc = f_pc; out->summary.fault_tid = f_tid;
  out->summary.flags = 0;
  out->final_mem = final_mem;
  out->final_cells = final_mem ? (uint64_t)P->arr_size[final_array] : 0;
  free(full); free(g.vars); free(g.interval_log.a); free(inter_log.a);
  for (int a = 0; a < P->n_global; a++) free(g.init[a]);
  return 0;
}

void orc_result_free(orc_result* r) {
  if (!r) return;
  free(r->records); free(r->final_mem);
  memset(r, 0, sizeof *r);
}

/* ------------------------------------------------------------------------ */
/* Triage features of one instance                                           */
/* ------------------------------------------------------------------------ */
/*
 * The 128 features are not part of the paper's method: they are the inputs
 * of the learned triage score, defined by the library's documentation of
 * rc_features.  This is that definition written out directly over the
 * oracle's own syntax tree, statement by statement in program order.
 */
typedef struct { int ok, modded; int64_t a, b; } Lin;   /* index = a*tid + b [mod N] */

static Lin lin_bad(void) { Lin r = {0, 0, 0, 0}; return r; }

static Lin lin_check(Lin r) {
  const int64_t big = (int64_t)1 << 31;
  if (r.a > big || r.a < -big || r.b > big || r.b < -big) return lin_bad();
  return r;
}

static Lin lin_of(const Expr* e) {
  Lin r = lin_bad();
  if (e->kind == E_CONST) { r.ok = 1; r.b = e->val; return r; }
  if (e->kind == E_TID) { r.ok = 1; r.a = 1; return r; }
  if (e->kind == E_NEG) {
    Lin x = lin_of(e->a);
    if (!x.ok || x.modded) return lin_bad();
    x.a = -x.a; x.b = -x.b;
    return lin_check(x);
  }
  if (e->kind != E_BIN) return r;
  Lin x = lin_of(e->a), y = lin_of(e->b);
  if (!x.ok || !y.ok || x.modded || y.modded) return r;
  if (e->op == B_ADD) { r.ok = 1; r.a = x.a + y.a; r.b = x.b + y.b; return lin_check(r); }
  if (e->op == B_SUB) { r.ok = 1; r.a = x.a - y.a; r.b = x.b - y.b; return lin_check(r); }
  if (e->op == B_MUL) {
    /* affine only when one factor is a constant */
    if (x.a == 0) { r.ok = 1; r.a = x.b * y.a; r.b = x.b * y.b; return lin_check(r); }
    if (y.a == 0) { r.ok = 1; r.a = x.a * y.b; r.b = x.b * y.b; return lin_check(r); }
    return r;
  }
  if (e->op == B_MOD || e->op == B_REM) {
    if (y.a != 0 || y.b <= 0) return r;
    x.modded = 1;
    return x;
  }
  return r;
}

typedef struct {
  int is_store, arr;
  Lin idx;
  int64_t interval;
  int under_if, under_loop, under_barrier_loop;
} FMem;

typedef struct {
  const orc_prog* P;
  int64_t kind_count[8];
  int64_t n_stmts, loads_g, loads_l, stores_g, stores_l;
  int64_t interval, mem_since_barrier, max_mem_interval, loop_barriers, trips;
  int64_t tid_values, other_values, ifs_open, max_ifs, loops_open, max_loops;
  int64_t mem_under_if, mem_under_loop, barrier_loops_open;
  FMem* mem; int64_t n_mem, cap_mem;
} FState;

static int body_has_barrier(Stmt** b, int n) {
  for (int i = 0; i < n; i++) {
    if (b[i]->kind == S_BARRIER) return 1;
    if (b[i]->kind == S_IF || b[i]->kind == S_FOR)
      if (body_has_barrier(b[i]->body, b[i]->nbody) || body_has_barrier(b[i]->els, b[i]->nels)) return 1;
  }
  return 0;
}

static void fwalk(FState* F, Stmt** b, int n) {
  for (int i = 0; i < n; i++) {
    const Stmt* s = b[i];
    F->n_stmts++;
    F->kind_count[s->kind]++;
    if (s->kind == S_LOAD || s->kind == S_STORE) {
      int global = s->arr < F->P->n_global;
      int st = s->kind == S_STORE;
      if (st && global) F->stores_g++;
      if (st && !global) F->stores_l++;
      if (!st && global) F->loads_g++;
      if (!st && !global) F->loads_l++;
      if (F->n_mem == F->cap_mem) {
        F->cap_mem = F->cap_mem ? 2 * F->cap_mem : 64;
        F->mem = (FMem*)realloc(F->mem, (size_t)F->cap_mem * sizeof(FMem));
      }
      FMem* m = &F->mem[F->n_mem++];
      m->is_store = st;
      m->arr = s->arr;
      m->idx = lin_of(s->e1);
      m->interval = F->interval;
      m->under_if = F->ifs_open > 0;
      m->under_loop = F->loops_open > 0;
      m->under_barrier_loop = F->barrier_loops_open > 0;
      if (m->under_if) F->mem_under_if++;
      if (m->under_loop) F->mem_under_loop++;
      F->mem_since_barrier++;
      if (st) {
        Lin v = lin_of(s->e2);
        if (!v.ok) F->other_values++;
        else if (v.a != 0) F->tid_values++;
      }
    } else if (s->kind == S_BARRIER) {
      if (F->loops_open > 0) F->loop_barriers++;
      if (F->mem_since_barrier > F->max_mem_interval) F->max_mem_interval = F->mem_since_barrier;
      F->mem_since_barrier = 0;
      F->interval++;
    } else if (s->kind == S_IF) {
      F->ifs_open++;
      if (F->ifs_open > F->max_ifs) F->max_ifs = F->ifs_open;
      fwalk(F, s->body, s->nbody);
      fwalk(F, s->els, s->nels);
      F->ifs_open--;
    } else if (s->kind == S_FOR) {
      int with_barrier = body_has_barrier(s->body, s->nbody);
      if (s->hi > s->lo) F->trips += s->hi - s->lo;
      F->loops_open++;
      if (F->loops_open > F->max_loops) F->max_loops = F->loops_open;
      if (with_barrier) F->barrier_loops_open++;
      fwalk(F, s->body, s->nbody);
      if (with_barrier) F->barrier_loops_open--;
      F->loops_open--;
    }
  }
}

static float fdiv(int64_t a, int64_t b) { return (float)a / (float)b; }

/* a count c on scale k, kept bounded: c / (c + k) */
static float fsq(int64_t c, int64_t k) { return (float)c / (float)(c + k); }

static int64_t pos_mod(int64_t x, int64_t m) {
  int64_t r = x % m;
  return r < 0 ? r + m : r;
}

static int64_t ceil_log2(int64_t s) {
  int64_t k = 0;
  while (((int64_t)1 << k) < s) k++;
  return k;
}

int orc_features(const orc_prog* P, uint32_t G, uint32_t W, const orc_bind* arrays, int n_arrays,
                 uint64_t seed, float* f, char* err, int errlen) {
  FState F;
  memset(&F, 0, sizeof F);
  F.P = P;
  for (int k = 0; k < 128; k++) f[k] = 0.0f;
  if (n_arrays < P->n_global) {
    snprintf(err, (size_t)errlen, "every global array needs a binding");
    return -1;
  }
  fwalk(&F, P->body, P->nbody);
  if (F.mem_since_barrier > F.max_mem_interval) F.max_mem_interval = F.mem_since_barrier;
  int64_t n = F.n_stmts > 0 ? F.n_stmts : 1;
  /* statement mix */
  for (int k = 0; k < 8; k++) f[k] = fdiv(F.kind_count[k], n);
  f[8] = fdiv(F.loads_g, n);
  f[9] = fdiv(F.loads_l, n);
  f[10] = fdiv(F.stores_g, n);
  f[11] = fdiv(F.stores_l, n);
  f[12] = fsq(F.n_stmts, 256);
  f[13] = fdiv(P->n_global, 8);
  f[14] = fdiv(P->n_local, 8);
  f[15] = fdiv(P->n_scalars, 16);
  /* candidate conflicting pairs: same array, a store among them, same static
     interval (statements under a loop that holds a barrier counted apart) */
  int64_t self_const = 0, self_const_if = 0, self_other = 0, shifted = 0, aligned = 0;
  int64_t strides = 0, opaque = 0, looped = 0, shifted_meet = 0;
  for (int64_t i = 0; i < F.n_mem; i++) {
    for (int64_t j = i; j < F.n_mem; j++) {
      const FMem* x = &F.mem[i];
      const FMem* y = &F.mem[j];
      if (x->arr != y->arr) continue;
      if (!x->is_store && !y->is_store) continue;
      if (x->under_barrier_loop || y->under_barrier_loop) { looped++; continue; }
      if (x->interval != y->interval) continue;
      if (i == j) {
        if (!x->idx.ok) self_other++;
        else if (x->idx.a == 0) { self_const++; if (x->under_if) self_const_if++; }
        continue;
      }
      if (!x->idx.ok || !y->idx.ok) { opaque++; continue; }
      if (x->idx.a != y->idx.a) { strides++; continue; }
      int64_t S = P->arr_size[x->arr];
      if (pos_mod(x->idx.b, S) == pos_mod(y->idx.b, S)) {
        aligned++;
      } else {
        shifted++;
        /* work-items d apart (1 <= |d| <= 1024) reach one cell when
           a*d and the offset difference agree mod the array size */
        int64_t diff = pos_mod(y->idx.b - x->idx.b, S), d;
        for (d = 1; d <= 1024; d++) {
          if (pos_mod(x->idx.a * d - diff, S) == 0 || pos_mod(-x->idx.a * d - diff, S) == 0) {
            shifted_meet++;
            break;
          }
        }
      }
    }
  }
  f[16] = fsq(self_const, 8);
  f[17] = fsq(self_const_if, 8);
  f[18] = fsq(self_other, 8);
  f[19] = fsq(shifted, 8);
  f[20] = fsq(aligned, 8);
  f[21] = fsq(strides, 8);
  f[22] = fsq(opaque, 8);
  f[23] = fsq(looped, 8);
  f[24] = fsq(F.tid_values, 16);
  f[25] = fsq(F.other_values, 16);
  f[26] = fsq(F.max_ifs, 16);
  f[27] = fsq(F.max_loops, 4);
  f[28] = fsq(F.mem_under_if, 16);
  f[29] = fsq(F.mem_under_loop, 16);
  {
    int64_t distinct = 0;
    for (int64_t i = 0; i < F.n_mem; i++) {
      if (!F.mem[i].is_store) continue;
      int seen = 0;
      for (int64_t j = 0; j < i; j++)
        if (F.mem[j].is_store && F.mem[j].interval == F.mem[i].interval) seen = 1;
      if (!seen) distinct++;
    }
    f[30] = fsq(distinct, 8);
  }
  f[31] = fsq(shifted_meet, 8);
  /* the first 16 memory statements */
  for (int64_t k = 0; k < 16 && k < F.n_mem; k++) {
    const FMem* m = &F.mem[k];
    float* s = f + 32 + 4 * k;
    s[0] = m->is_store ? 1.0f : -1.0f;
    if (m->idx.ok) {
      int64_t mag = m->idx.a < 0 ? -m->idx.a : m->idx.a;
      s[1] = (float)m->idx.a / (float)(1 + mag);
      s[2] = fdiv(pos_mod(m->idx.b, P->arr_size[m->arr]), P->arr_size[m->arr]);
    } else {
      s[1] = -2.0f;
      s[2] = -2.0f;
    }
    s[3] = fdiv(m->interval + 1, 8);
  }
  /* barrier and loop structure */
  f[96] = fsq(F.kind_count[S_BARRIER], 8);
  f[97] = fsq(F.loop_barriers, 8);
  f[98] = fsq(F.max_mem_interval, 64);
  f[99] = fsq(F.trips, 64);
  f[100] = fsq(F.n_mem, 64);
  f[101] = fsq(F.kind_count[S_STORE], 64);
  {
    int64_t distinct = 0;
    for (int64_t i = 0; i < F.n_mem; i++) {
      if (!F.mem[i].is_store) continue;
      int seen = 0;
      for (int64_t j = 0; j < i; j++)
        if (F.mem[j].is_store && F.mem[j].arr == F.mem[i].arr) seen = 1;
      if (!seen) distinct++;
    }
    f[102] = fsq(distinct, 8);
  }
  /* launch shape and array sizes */
  f[104] = fdiv(W, 1024);
  f[105] = fdiv(G, 1024);
  if (P->n_global > 0) f[106] = fdiv(ceil_log2(P->arr_size[0]), 32);
  if (P->n_global > 1) f[107] = fdiv(ceil_log2(P->arr_size[1]), 32);
  {
    int64_t local_cells = 0;
    for (int a = P->n_global; a < P->n_global + P->n_local; a++) local_cells += P->arr_size[a];
    f[108] = fdiv(local_cells, 65536);
  }
  f[109] = fdiv((int64_t)G * (int64_t)W, 1048576);
  /* seed statistics: 8-bin histograms of the first 256 initial cells of
     global arrays 0 and 1 */
  for (int a = 0; a < 2 && a < P->n_global; a++) {
    const orc_bind* b = &arrays[a];
    int64_t cells = P->arr_size[a] < 256 ? P->arr_size[a] : 256;
    int64_t hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t c = 0; c < cells; c++) {
      int bin;
      if (b->kind == 0) {
        int32_t v = orc_seeded_value(seed, (uint64_t)a, (uint64_t)c, b->lo, b->hi);
        /* the draw's offset in [lo, hi), taken mod 2^32 because a range of
           2^32 values wraps in int32, then its eighth of the range */
        uint64_t u = (uint32_t)((uint32_t)v - (uint32_t)(uint64_t)b->lo);
        bin = (int)(u * 8u / (uint64_t)(b->hi - b->lo));
      } else {
        int64_t v = b->data[c];
        bin = (int)((v + 2147483648LL) / 536870912LL);   /* eighths of the int32 range */
      }
      hist[bin]++;
    }
    for (int k = 0; k < 8; k++) f[112 + 8 * a + k] = fdiv(hist[k], 256);
  }
  free(F.mem);
  return 0;
}
