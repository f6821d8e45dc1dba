// capi.cpp -- the rc_* C ABI (include/rc.h): contexts, programs, bindings,
// workspace layout and the pass loop that drives the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/rc.h"
#include "frontend.h"
#include "jit.h"
#include "kernels.h"
#include "mlp.h"
#include "ownership.h"
#include "rc_internal.h"

using namespace rc;
typedef unsigned long long u64;

static_assert(sizeof(rc_record) == 40, "rc_record is 40 bytes");
static_assert(sizeof(rc_summary) == 40, "rc_summary is 40 bytes");

namespace {

thread_local std::string g_err;

// per device: the address of the static workspace (rc_check_static)
std::mutex g_static_ws_mu;
std::vector<void*> g_static_ws;

rc_status fail(rc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(RC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

uint32_t bits_for(u64 count) {   // bits to hold values 0 .. count-1
  uint32_t b = 0;
  while (b < 64 && (1ull << b) < count) ++b;
  return b;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Pending {
  u64* d_n_records;
  u64 cap;
  uint32_t* d_status;
};

}  // namespace

struct rc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool profiling = false;
  std::vector<hipEvent_t> events;            // pool, reused after each read
  size_t events_used = 0;
  std::vector<std::pair<int, size_t>> spans; // (phase, index of the start event)
  struct WsState {
    u64 gen = 0;               // generation this context last wrote to the header
    uint32_t next_epoch = 1;   // first overlay version base not used yet
  };
  std::map<void*, WsState> ws_state;
  std::vector<Pending> pending;
  hipEvent_t upload_done = nullptr;        // last host-to-device table upload
  std::vector<unsigned char> h_call;       // host staging of the call tables
  hipStream_t capture_stream = nullptr;    // private stream used only to capture graphs
  std::vector<hipGraphExec_t> graphs_to_free;   // executable graphs of calls in flight
  bool use_graphs = true;
  u64* last_stats = nullptr;               // log statistics of the last check call (device)
  void* static_ws = nullptr;               // this device's static workspace (rc_check_static)
};

struct rc_prog {
  rc_ctx* ctx = nullptr;
  Compiled c;
  uint32_t G = 0, W = 0;
  bool shaped = false;
  std::vector<ArrayDesc> arrays;     // host copy of the descriptor table
  std::vector<ScalarDesc> scalars;
  std::vector<uint32_t> cellbase, sizes;
  uint32_t n_logged_cells = 0, overlay_cells = 0, lds_local_cells = 0;
  uint32_t lds_log_pref = 0;         // tuning: LDS log entries (0: the library's choice)
  uint32_t radix_bits = 8;           // tuning: digit width of the access-log sort
  uint32_t record_sort = 0;          // tuning: 1 = always sort records by their full key
  uint32_t proofs_off = 0;           // tuning: 1 = no static proof (every written array logged)
  uint32_t global_spills = 0;        // tuning: 1 = spilled intervals always go to the global pass
  bool sc = false;                   // spilled intervals checked by the work-group (current shape)
  uint32_t step_limit = DEFAULT_STEP_LIMIT;   // tuning: loop iterations a work-group may start
  bool never_faults = false;         // proven for the current shape
  uint64_t log_mask = ~0ull;         // intervals whose local-array accesses are logged (ProgDesc)
  uint32_t log_high = 1;
  uint32_t lds_log_cap = 0;          // chosen for the current shape
  // arrays no two work-items share under the current shape (never logged),
  // and the per-item access bounds on the arrays that are logged
  std::vector<uint8_t> owned;
  uint64_t logged_mem = 0, logged_local = 0;
  // per-program kernels (rc_prog_jit): every module compiled so far, one per
  // (width class, launch shape); the one for the current shape, and whether
  // single-program calls use it
  struct JitEntry {
    uint32_t cls;
    JitShape shape;
    hipModule_t mod;
    hipFunction_t fn;
  };
  std::vector<JitEntry> jit_mods;
  hipFunction_t jit_fn = nullptr;
  uint32_t jit_class = ~0u;
  JitShape jit_shape;
  bool jit_on = false;
  // device: code, then tables
  void* d_mem = nullptr;
  size_t off_arrays = 0, off_scalars = 0, off_cellbase = 0, off_size = 0, d_bytes = 0;
  std::vector<unsigned char> h_tables;   // staging for the table upload
};

namespace {

// record a HIP event on the ctx stream when profiling; returns its pool index
rc_status prof_mark(rc_ctx* ctx, hipStream_t st, size_t* idx) {
  if (!ctx->profiling) return RC_OK;
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    ctx->events.push_back(e);
  }
  *idx = ctx->events_used++;
  HIP_TRY(hipEventRecord(ctx->events[*idx], st));
  return RC_OK;
}

struct PhaseTimer {
  rc_ctx* ctx;
  hipStream_t st;
  int phase;
  size_t start = 0;
  bool on;
  PhaseTimer(rc_ctx* c, hipStream_t s, int ph, bool enabled) : ctx(c), st(s), phase(ph), on(enabled && c->profiling) {
    if (on) prof_mark(ctx, st, &start);
  }
  ~PhaseTimer() {
    if (!on) return;
    size_t end = 0;
    if (prof_mark(ctx, st, &end) == RC_OK && end == start + 1) ctx->spans.push_back({phase, start});
  }
};

// ---------------------------------------------------------------------------
// per-program quantities
// ---------------------------------------------------------------------------
// The LDS check uses a per-cell table when the LDS-logged cells are few:
// written local arrays when G > 1 (their log cell keys follow the written
// global arrays'), every written array when G == 1 (keys from 0).
size_t lds_base_bytes(const rc_prog* p) {
  const uint32_t WP = ((p->W + 63) / 64) * 64;
  return ((sizeof(Ctl) + 15) & ~(size_t)15) + (size_t)p->lds_local_cells * 8 + (size_t)p->c.nregs * WP * 4 + 8;
}

// (Only when the table and a minimal log fit in LDS beside the rest.)
void lds_table(const rc_prog* p, uint32_t* base, uint32_t* cells) {
  uint32_t gcells = 0;
  for (size_t i = 0; i < p->c.arrays.size(); ++i) {
    const CompiledArray& a = p->c.arrays[i];
    if (a.global && a.written && !p->owned[i]) gcells += a.size;
  }
  *base = p->G == 1 ? 0u : gcells;
  const uint32_t n = p->n_logged_cells - *base;
  const bool fits = lds_base_bytes(p) + (size_t)n * sizeof(TabCell) + 64 * 16 <= LDS_LIMIT;
  *cells = (n > 0 && n <= TAB_MAX_CELLS && fits) ? n : 0u;
}

size_t lds_fixed_bytes(const rc_prog* p) {
  uint32_t tb, tc;
  lds_table(p, &tb, &tc);
  return lds_base_bytes(p) + (size_t)tc * sizeof(TabCell);
}

// Bytes of one LDS log entry: with the per-cell table an entry packs into
// one word (cell - table base, store flag, local id, value); the sort path
// keeps a sort key, a payload word and the value.
size_t lds_entry_bytes(const rc_prog* p) {
  uint32_t tb, tc;
  lds_table(p, &tb, &tc);
  return tc ? 8u : 16u;
}

// LDS of one work-group; a per-program kernel and the VGPR-file interpreter
// keep the private variables in registers, so they take no LDS there.
size_t lds_bytes(const rc_prog* p, bool vgpr_regs) {
  const uint32_t WP = ((p->W + 63) / 64) * 64;
  const size_t regs = vgpr_regs ? (size_t)p->c.nregs * WP * 4 : 0;
  return lds_fixed_bytes(p) - regs + (size_t)p->lds_log_cap * lds_entry_bytes(p);
}

// Entries of the interval log kept in LDS (a power of two; 0 = none): large
// enough for the program's static per-interval bound when that fits, else as
// large as LDS allows up to 4096 entries (or the tuned size).
uint32_t lds_log_entries(const rc_prog* p) {
  const bool lds_globals = p->G == 1;
  const u64 per_item = p->logged_local + (lds_globals ? p->logged_mem - p->logged_local : 0);
  if (per_item == 0) return 0;
  const size_t fixed = lds_fixed_bytes(p), eb = lds_entry_bytes(p);
  if (fixed + 2 * eb > LDS_LIMIT) return 0;
  uint32_t fit = 2;
  while ((size_t)fit * 2 * eb + fixed <= LDS_LIMIT && fit * 2 <= 65536u) fit *= 2;
  if (p->lds_log_pref) {
    uint32_t t = 2;
    while (t * 2 <= p->lds_log_pref && t * 2 <= fit) t *= 2;
    return t;
  }
  const double bound = (double)p->W * (lds_globals ? p->c.interval_logged_all : p->c.interval_logged_local);
  uint32_t want = 2;
  while (want < bound && want < 65536u) want *= 2;
  if ((double)want >= bound && want <= fit) return want;   // never spills
  return std::min(fit, 4096u);
}

bool lds_logged(const rc_prog* p, uint32_t a) {
  return p->lds_log_cap && p->c.arrays[a].written && !p->owned[a] && (!p->c.arrays[a].global || p->G == 1);
}

// where an array's accesses are logged
uint32_t array_logged(const rc_prog* p, uint32_t a) {
  return !p->c.arrays[a].written || p->owned[a] ? LOG_NONE : (lds_logged(p, a) ? LOG_LDS : LOG_GLOBAL);
}

// an interval's LDS-logged accesses may outgrow the LDS log (static bound)
bool lds_may_spill(const rc_prog* p) {
  const double ib = p->G == 1 ? p->c.interval_logged_all : p->c.interval_logged_local;
  return p->lds_log_cap && (double)p->W * ib > (double)p->lds_log_cap;
}

// log entries one work-group may write to the global log (0: none, the
// program's logged accesses all stay in LDS)
u64 wg_log_need(const rc_prog* p) {
  const u64 lds = p->lds_log_cap ? p->logged_local + (p->G == 1 ? p->logged_mem - p->logged_local : 0) : 0;
  const u64 glob = p->logged_mem - lds;
  // (a one-group program whose spills go to the group check: a trailer per interval)
  return (u64)p->W * (glob + (lds_may_spill(p) ? lds : 0)) + (p->sc ? p->c.max_intervals : 0);
}

// the entries a work-group's region holds: at least one (the global log's
// buffers are never empty)
u64 wg_log_entries(const rc_prog* p) { return std::max<u64>(1, wg_log_need(p)); }

// the words of a work-group's region
u64 wg_region_words(const rc_prog* p) { return wg_log_entries(p); }

// Spilled intervals go to the group check kernel (sc_check) instead of the
// global pass when the program has one group (no INTER scope, every logged
// array in LDS), its intervals may outgrow the LDS log and its cell keys
// fit the packed entries (and so SC_NB_MAX windows of the check).
bool sc_feasible(const rc_prog* p) {
  static_assert((u64)SC_WIN * SC_NB_MAX >= SC_MAX_CELLS, "the group check's windows cover every cell key");
  if (p->global_spills || p->G != 1 || !p->lds_log_cap || !lds_may_spill(p)) return false;
  return p->n_logged_cells >= 1 && p->n_logged_cells <= SC_MAX_CELLS;
}

// the interval log's size for the current shape and tuning, and whether the
// group checks its own spills
void set_log_cap(rc_prog* p) {
  p->lds_log_cap = lds_log_entries(p);
  p->sc = sc_feasible(p);
}

uint32_t width_class(uint32_t W) {
  const uint32_t nw = (W + 63) / 64;
  uint32_t c = 0;
  while ((1u << c) < nw) ++c;
  return c;   // 0..4
}

rc_status check_ready(const rc_prog* p) {
  if (!p->shaped) return fail(RC_E_STATE, "rc_set_ndrange has not been called");
  for (uint32_t a = 0; a < p->c.n_global; ++a)
    if (p->arrays[a].bind == BIND_NONE)
      return fail(RC_E_STATE, "global array '%s' is not bound", p->c.arrays[a].name.c_str());
  for (size_t s = 0; s < p->scalars.size(); ++s)
    if (p->scalars[s].bind == BIND_NONE)
      return fail(RC_E_STATE, "scalar '%s' is not bound", p->c.scalars[s].c_str());
  return RC_OK;
}

// ---------------------------------------------------------------------------
// a call: instances -> chunks under one workspace layout
// ---------------------------------------------------------------------------
struct Need {          // resources of one instance
  u64 log, recs, ovl;
  uint32_t wg;
};

Need need_of(const rc_prog* p) {
  Need n;
  n.wg = p->G;
  n.log = (u64)p->G * wg_region_words(p);
  // A record stands for a cell of one scope with at least two logged
  // accesses (an eligible pair needs two work-items), and the scopes of one
  // kind split the accesses: at most half the logged accesses give INTRA
  // records, and at most half the global ones give INTER records.
  const u64 acc = (u64)p->G * p->W;
  n.recs = std::max<u64>(1, (acc * p->logged_mem + acc * (p->logged_mem - p->logged_local) + 1) / 2);
  n.ovl = (u64)p->G * p->overlay_cells;
  return n;
}

struct Layout {
  // limits of one chunk
  u64 max_log = 0, max_rec = 0, max_ovl = 0;
  uint32_t max_slots = 0, max_wg = 0, max_items_class[N_WCLASS] = {0, 0, 0, 0, 0};
  // key layout
  uint32_t bi = 0, bc = 0, bg = 0, bk = 0, bs = 0, nbits_log = 0, nbits_rec = 0;
  // offsets in the workspace
  size_t header = 0, overlay = 0, tables = 0, progs = 0, slots = 0, chunks = 0, items = 0, recout = 0;
  size_t counters = 0, queue = 0, chunk_index = 0, wg_count = 0, wg_base = 0, tiles = 0;
  size_t inst_acc = 0, inst_fault = 0, inst_int = 0, inst_race = 0, inst_benign = 0, inst_flags = 0;
  size_t lk0 = 0, lv0 = 0, lk1 = 0, lv1 = 0, hist = 0, stage = 0, rk0 = 0, ri0 = 0, rk1 = 0, ri1 = 0;
  size_t longq = 0;
  u64 long_cap = 0;
  // records placed by rank (no global log, so every record comes from an
  // interval closed in LDS): per-(slot, scope) record counts and the scan's
  // partial sums
  bool rank = false, lds_only = false;
  // one-group programs' spilled intervals checked after the interpreter
  // (sc_group_kernel): blocks of the check and their bucket-bound words
  uint32_t sc_blocks = 0;
  size_t sc_ends = 0;
  size_t sc_order = 0;   // per instance of the call: the group check's queue order (chunk-relative slots)
  u64 scope_n = 0;
  size_t scope_cnt = 0, scope_tmp = 0;
  // per-(slot, cell) owner words of the global log (cc_stride cells per
  // slot), when the table is small beside the log it filters
  size_t cc = 0;
  uint32_t cc_stride = 0;
  bool filter = false;
  size_t total = 0;
};

// counters block: [0] log entries, [1] records, [2] status word, [3] long runs
// per-chunk counters: log entries, record slots reserved, status bits,
// queued long runs, record slots left unused, records (reserved - unused)
enum { CNT_LOG = 0, CNT_REC = 1, CNT_STATUS = 2, CNT_LONG = 3, CNT_DEAD = 4, CNT_LIVE = 5, CNT_STATS = 8,
       N_STATS = 7, CNT_WORDS = 16 };

void lay_out(Layout* L, size_t n_progs, size_t n_inst, size_t n_chunks, size_t n_items) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  L->header = take(64);                        // workspace header (validity of the pool)
  L->overlay = take(L->max_ovl * 8);           // the versioned overlay pool
  L->tables = o;
  L->progs = take(n_progs * sizeof(ProgDesc));
  L->slots = take(n_inst * sizeof(SlotDesc));
  L->chunks = take(n_chunks * sizeof(ChunkDesc));
  L->items = take(n_items * 8);
  L->sc_order = take(L->sc_blocks ? n_inst * 4 : 0);
  L->recout = take(sizeof(rc_record_out));
  L->counters = take(CNT_WORDS * 8);
  L->queue = take((N_WCLASS + 1) * 4);   // the classes' queues, then the group check's
  L->sc_ends = take((size_t)L->sc_blocks * SC_NB_MAX * 4);
  L->chunk_index = take(4);
  L->wg_count = take((size_t)L->max_wg * 4);
  L->wg_base = take((size_t)L->max_wg * 8);
  L->tiles = take(((size_t)L->max_wg + 1) * 4);
  L->inst_acc = take((size_t)L->max_slots * 8);
  L->inst_fault = take((size_t)L->max_slots * 8);
  L->inst_int = take((size_t)L->max_slots * 4);
  L->inst_race = take((size_t)L->max_slots * 4);
  L->inst_benign = take((size_t)L->max_slots * 4);
  L->inst_flags = take((size_t)L->max_slots * 4);
  L->lk0 = take(L->max_log * 8);
  L->lv0 = take(L->max_log * 8);
  L->lk1 = take(L->max_log * 8);
  L->lv1 = take(L->max_log * 8);
  L->long_cap = 2 * L->max_log / (SEG_SHORT_RUN + 1) + 2;
  L->longq = take(L->long_cap * 16);
  L->cc = take(L->filter ? (size_t)L->max_slots * L->cc_stride * 4 : 0);
  // (placing records by rank needs no record sort: no second key buffer,
  // no index buffers, no sort histogram)
  const u64 sorted_rec = L->rank ? 0 : L->max_rec;
  L->hist = take(std::max(sort_log_hist_words(L->max_wg, L->max_log), sorted_rec ? sort_hist_words(sorted_rec) : 0) * 4);
  L->stage = take(L->max_rec * sizeof(rc_record));
  L->rk0 = take(L->max_rec * 8);
  L->ri0 = take(sorted_rec * 4);
  L->rk1 = take(sorted_rec * 8);
  L->ri1 = take(sorted_rec * 4);
  L->scope_cnt = take(L->scope_n * 4);
  L->scope_tmp = take(L->rank ? scan_tmp_words(L->scope_n) * 4 : 0);
  L->total = o;
}

struct Call {
  std::vector<rc_prog*> progs;          // distinct programs
  std::vector<uint32_t> inst_prog;      // instance -> program index
  std::vector<uint64_t> inst_seed;
  std::vector<SlotDesc> slots;
  std::vector<ChunkDesc> chunks;
  std::vector<uint32_t> items;          // pairs (instance, gid)
  // the group check's queue, per chunk: its slots (relative to the chunk)
  // in descending static log bound, so the largest spills start first
  std::vector<uint32_t> sc_order;
  Layout L;
  uint32_t classes_used = 0;            // bit c: width class c occurs
  size_t class_lds[N_WCLASS] = {0, 0, 0, 0, 0};
  uint32_t epoch_stride = 1;
  uint32_t radix_bits = 8;              // digit width of the access-log sort
  uint32_t record_sort = 0;             // 1: never place records by rank
  bool jit = false;                     // one program, run by its own kernel
  bool class_vreg[N_WCLASS] = {false, false, false, false, false};   // class interpreted with VGPR registers
};

// Split the instances into chunks whose resources stay under the limits.
void partition(Call& C, const Layout& lim) {
  C.chunks.clear();
  C.sc_order.clear();
  C.slots.assign(C.inst_prog.size(), SlotDesc());
  bool any_sc = false;
  for (const rc_prog* p : C.progs) any_sc = any_sc || p->sc;
  std::vector<std::vector<uint32_t>> class_items(N_WCLASS);
  u64 log = 0, ovl = 0;
  uint32_t wg = 0, n = 0;
  ChunkDesc cur;
  memset(&cur, 0, sizeof cur);
  auto flush = [&](uint32_t next_slot0) {
    cur.n_slots = n;
    cur.n_wg = wg;
    uint32_t at = (uint32_t)(C.items.size() / 2);
    for (uint32_t c = 0; c < N_WCLASS; ++c) {
      cur.item0[c] = at;
      // longest first: cost = width x static instructions
      std::vector<uint32_t>& v = class_items[c];
      std::stable_sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) {
        const rc_prog* pa = C.progs[C.inst_prog[a >> 0]];
        const rc_prog* pb = C.progs[C.inst_prog[b >> 0]];
        return (double)pa->W * (double)pa->c.dyn_instr > (double)pb->W * (double)pb->c.dyn_instr;
      });
      for (uint32_t inst : v) {
        const rc_prog* p = C.progs[C.inst_prog[inst]];
        for (uint32_t g = 0; g < p->G; ++g) { C.items.push_back(inst); C.items.push_back(g); }
      }
      at = (uint32_t)(C.items.size() / 2);
      v.clear();
    }
    cur.item0[N_WCLASS] = at;
    cur.n_items = at - cur.item0[0];
    if (any_sc) {
      // the group check's order: instances with the largest static log
      // bound first (the others are skipped at once)
      const size_t o = C.sc_order.size();
      for (uint32_t k = 0; k < n; ++k) C.sc_order.push_back(k);
      auto cost = [&](uint32_t k) -> u64 {
        const rc_prog* p = C.progs[C.inst_prog[cur.slot0 + k]];
        return p->sc ? wg_log_need(p) : 0u;
      };
      std::stable_sort(C.sc_order.begin() + o, C.sc_order.end(),
                       [&](uint32_t a, uint32_t b) { return cost(a) > cost(b); });
    }
    C.chunks.push_back(cur);
    memset(&cur, 0, sizeof cur);
    cur.slot0 = next_slot0;
    log = ovl = 0;
    wg = n = 0;
  };
  const uint32_t N = (uint32_t)C.inst_prog.size();
  for (uint32_t i = 0; i < N; ++i) {
    const rc_prog* p = C.progs[C.inst_prog[i]];
    const Need nd = need_of(p);
    if (n > 0 && (n + 1 > lim.max_slots || wg + nd.wg > lim.max_wg || log + nd.log > lim.max_log ||
                  ovl + nd.ovl > lim.max_ovl))
      flush(i);
    SlotDesc& s = C.slots[i];
    s.seed = C.inst_seed[i];
    s.log_base = log;
    s.ovl_base = ovl;
    s.prog = C.inst_prog[i];
    s.wg_base = wg;
    class_items[width_class(p->W)].push_back(i);
    log += nd.log;
    ovl += nd.ovl;
    wg += nd.wg;
    ++n;
  }
  if (n > 0) flush(N);
}

// Choose chunk limits so that the layout fits `ws_bytes`, then partition.
// The launch shape of the program's current NDRange and tuning, as the
// device descriptor states it.
JitShape jit_shape_of(const rc_prog* p) {
  JitShape s;
  s.W = p->W;
  s.G = p->G;
  s.n_arrays = (uint32_t)p->c.arrays.size();
  lds_table(p, &s.tab_base, &s.tab_cells);
  if (!p->lds_log_cap) s.tab_cells = 0;
  s.lds_log_cap = p->lds_log_cap;
  s.nospill = p->lds_log_cap && !lds_may_spill(p) ? 1u : 0u;
  s.nofault = p->never_faults ? 1u : 0u;
  s.log_mask = p->log_mask;
  s.log_high = p->log_high;
  for (uint32_t i = 0; i < (uint32_t)p->arrays.size(); ++i) {
    const ArrayDesc& a = p->arrays[i];
    const uint32_t f[JIT_ARRAY_WORDS] = {a.kind, a.size, array_logged(p, i), a.offset, a.cellbase,
                                         (uint32_t)a.own_stride, (uint32_t)a.own_lo, a.own_span, a.nosync};
    s.arrays.insert(s.arrays.end(), f, f + JIT_ARRAY_WORDS);
  }
  return s;
}

bool jit_current(const rc_prog* p) {
  return p->jit_fn && p->jit_class == width_class(p->W) && p->jit_shape == jit_shape_of(p);
}

bool plan(Call& C, size_t ws_bytes, std::string* why) {
  const uint32_t N = (uint32_t)C.inst_prog.size();
  u64 T_log = 0, T_rec = 0, T_ovl = 0, T_wg = 0, M_log = 0, M_rec = 0, M_ovl = 0, M_wg = 0;
  uint32_t bc = 0, bg = 0, bk = 0, bs = 0, max_cells = 0;
  u64 max_stores = 0, items_total = 0;
  for (uint32_t i = 0; i < N; ++i) {
    const Need nd = need_of(C.progs[C.inst_prog[i]]);
    T_log += nd.log; T_rec += nd.recs; T_ovl += nd.ovl; T_wg += nd.wg;
    M_log = std::max(M_log, nd.log); M_rec = std::max(M_rec, nd.recs);
    M_ovl = std::max(M_ovl, nd.ovl); M_wg = std::max<u64>(M_wg, nd.wg);
    items_total += nd.wg;
  }
  C.classes_used = 0;
  C.jit = C.progs.size() == 1 && C.progs[0]->jit_on && jit_current(C.progs[0]);
  // per width class: the VGPR-file interpreter when every program fits it
  // and it keeps more work-groups resident (its registers leave LDS, but it
  // needs more VGPRs)
  bool vreg_ok[N_WCLASS] = {true, true, true, true, true};
  size_t lds_l[N_WCLASS] = {0, 0, 0, 0, 0}, lds_v[N_WCLASS] = {0, 0, 0, 0, 0};
  for (rc_prog* p : C.progs) {
    const uint32_t c = width_class(p->W);
    vreg_ok[c] = vreg_ok[c] && p->c.nregs <= VREG_FILE;
    lds_l[c] = std::max(lds_l[c], lds_bytes(p, false));
    lds_v[c] = std::max(lds_v[c], lds_bytes(p, true));
  }
  for (uint32_t c = 0; c < N_WCLASS; ++c) {
    C.class_vreg[c] = false;
    if (C.jit || !vreg_ok[c] || lds_v[c] == 0) continue;
    const uint32_t threads = 64u << c;
    C.class_vreg[c] = interp_occupancy(threads, lds_v[c], true) > interp_occupancy(threads, lds_l[c], false);
  }
  for (rc_prog* p : C.progs) {
    bc = std::max(bc, bits_for(std::max<u64>(1, p->n_logged_cells)));
    max_cells = std::max(max_cells, p->n_logged_cells);
    bg = std::max(bg, bits_for(p->G));
    bk = std::max(bk, bits_for(p->c.max_intervals));
    bs = std::max(bs, bits_for((u64)p->G * p->c.max_intervals + 1));
    max_stores = std::max<u64>(max_stores, p->c.dyn_stores);
    const uint32_t c = width_class(p->W);
    C.classes_used |= 1u << c;
    C.class_lds[c] = std::max(C.class_lds[c], lds_bytes(p, C.jit || C.class_vreg[c]));
  }
  C.epoch_stride = (uint32_t)std::min<u64>(max_stores + 1, 1u << 22);
  C.radix_bits = C.progs.empty() ? 8u : C.progs[0]->radix_bits;
  C.record_sort = C.progs.empty() ? 0u : C.progs[0]->record_sort;
  bool lds_only = true;   // no program of the call writes the global log
  bool any_sc = false;    // some program's spills go to the group check
  for (const rc_prog* p : C.progs) {
    lds_only = lds_only && (wg_log_need(p) == 0 || p->sc);
    any_sc = any_sc || p->sc;
  }
  if (bc > 32 || bg > 26 || bk > 32) { *why = "sort key fields too wide"; return false; }
  // The fewest chunks that fit: the limits for k chunks are first laid out
  // with a one-chunk table (a lower bound of the total, no partition) and
  // partitioned only when that fits; k grows by an eighth, so the chunks
  // come out within about an eighth of the fewest the budget allows
  for (u64 k = 1;; k = std::max<u64>(k + 1, k + k / 8)) {
    Layout L;
    const u64 per = (N + k - 1) / k;
    L.max_slots = (uint32_t)std::min<u64>(N, per + 1);
    L.max_wg = (uint32_t)std::min<u64>(T_wg, (T_wg + k - 1) / k + M_wg);
    L.max_log = std::min<u64>(T_log, (T_log + k - 1) / k + M_log);
    L.max_rec = std::min<u64>(T_rec, (T_rec + k - 1) / k + M_rec);
    L.max_ovl = std::min<u64>(T_ovl, (T_ovl + k - 1) / k + M_ovl);
    L.max_rec = std::max<u64>(L.max_rec, L.max_log);
    // slots that work-groups reserve in chunks and leave unused: at most a
    // chunk per launched block (a block per work item at most)
    // (and a chunk per block of the group check)
    L.max_rec += (std::min<u64>(L.max_wg, (u64)N_WCLASS * REC_MAX_BLOCKS) + (any_sc ? SC_MAX_BLOCKS : 0)) * REC_CHUNK;
    L.bi = bits_for(L.max_slots);
    L.bc = bc; L.bg = bg; L.bk = bk; L.bs = bs;
    L.nbits_log = L.bi + bc + bg + bk;
    L.nbits_rec = L.bi + bs + bc + 1;   // the top bit is set only in unused slots' keys
    L.cc_stride = std::max<uint32_t>(1, max_cells);
    // The owner filter drops the entries of cells one work-item touched,
    // for the price of an owner word per access and one partition pass.  It
    // pays when accesses are sparse over the cells: at more than one logged
    // access per cell (static bound) most cells are shared and the pass
    // would move nearly everything; the owner table must stay within four
    // words per log entry.
    const u64 owner_words = (u64)L.max_slots * L.cc_stride;
    L.filter = L.max_log >= 4096 && owner_words >= L.max_log && owner_words <= 4 * L.max_log && bg <= 21;
    if (L.nbits_log > 64 || L.nbits_rec > 64) { *why = "sort key wider than 64 bits"; return false; }
    // Without a global log every record comes from an interval closed in
    // LDS, which emits its records in cell-key order: a record's position
    // is then fixed by the record counts of the (slot, scope)s before it
    // and its rank, and the records need no sort.
    L.rank = C.record_sort == 0 && lds_only && L.bi + bs <= 32 && ((u64)L.max_slots << bs) <= (1ull << 26);
    L.scope_n = L.rank ? (u64)L.max_slots << bs : 0;
    L.lds_only = lds_only;
    L.sc_blocks = any_sc ? std::min<uint32_t>(L.max_slots, SC_MAX_BLOCKS) : 0u;
    Layout bound = L;
    lay_out(&bound, C.progs.size(), N, 1, items_total);
    if (bound.total <= ws_bytes) {
      Layout lim = L;
      partition(C, lim);
      lay_out(&L, C.progs.size(), N, C.chunks.size(), C.items.size() / 2);
      if (L.total <= ws_bytes) {
        // class grid sizes: the most items one class has in any chunk
        for (const ChunkDesc& ch : C.chunks)
          for (uint32_t c = 0; c < N_WCLASS; ++c)
            L.max_items_class[c] = std::max(L.max_items_class[c], ch.item0[c + 1] - ch.item0[c]);
        C.L = L;
        return true;
      }
      C.items.clear();
    }
    if (k >= 2 * (u64)N + 2) {
      char b[200];
      snprintf(b, sizeof b, "workspace of %zu bytes is too small: one instance needs %zu", ws_bytes, bound.total);
      *why = b;
      return false;
    }
  }
}

// the per-chunk kernel sequence
rc_status enqueue_chunk(rc_ctx* ctx, const Call& C, char* ws, hipStream_t st, u64* d_n_records,
                        rc_record* d_records, u64 cap, rc_summary* d_summaries, int do_log, bool timed) {
  const Layout& L = C.L;
  u64* cnt = (u64*)(ws + L.counters);
  const ProgDesc* progs = (const ProgDesc*)(ws + L.progs);
  const SlotDesc* slots = (const SlotDesc*)(ws + L.slots);
  const ChunkDesc* chunks = (const ChunkDesc*)(ws + L.chunks);
  const uint32_t* chunk_index = (const uint32_t*)(ws + L.chunk_index);
  {
    PhaseTimer t(ctx, st, 5, timed);
    SetupParams S;
    memset(&S, 0, sizeof S);
    S.chunks = chunks; S.chunk_index = chunk_index; S.counters = cnt; S.queue = (uint32_t*)(ws + L.queue);
    S.inst_acc = (u64*)(ws + L.inst_acc); S.inst_fault = (u64*)(ws + L.inst_fault);
    S.inst_intervals = (uint32_t*)(ws + L.inst_int); S.inst_race = (uint32_t*)(ws + L.inst_race);
    S.inst_benign = (uint32_t*)(ws + L.inst_benign); S.inst_flags = (uint32_t*)(ws + L.inst_flags);
    S.overlay = (u64*)(ws + L.overlay); S.overlay_cells = L.max_ovl; S.max_slots = L.max_slots;
    HIP_TRY(launch_setup(S, st));
    HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.wg_count), L.max_wg, 0u, st));
    if (L.rank) HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.scope_cnt), L.scope_n, 0u, st));
  }
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  {
    PassParams P;
    memset(&P, 0, sizeof P);
    P.progs = progs; P.slots = slots; P.chunks = chunks; P.chunk_index = chunk_index;
    P.items = (const uint32_t*)(ws + L.items); P.queue = (uint32_t*)(ws + L.queue);
    P.bc = L.bc; P.bg = L.bg; P.bk = L.bk; P.bs = L.bs; P.do_log = (uint32_t)do_log;
    P.overlay = (u64*)(ws + L.overlay); P.log_keys = (u64*)(ws + L.lk0); P.log_vals = (u64*)(ws + L.lv0);
    P.wg_count = (uint32_t*)(ws + L.wg_count); P.wg_base = (u64*)(ws + L.wg_base);
    P.inst_acc = (u64*)(ws + L.inst_acc); P.inst_intervals = (uint32_t*)(ws + L.inst_int);
    P.inst_fault = (u64*)(ws + L.inst_fault); P.status_word = (uint32_t*)(cnt + CNT_STATUS);
    P.rec = (rc_record_out*)(ws + L.recout);
    // owner words need no clearing: each is written before it is read
    P.cell_owner = (L.filter && do_log) ? (uint32_t*)(ws + L.cc) : nullptr;
    P.cell_owner_stride = L.cc_stride;
    P.stats = do_log ? cnt + CNT_STATS : nullptr;
    // a call of one program with a compiled kernel runs that kernel; any
    // other call runs the interpreter
    rc_prog* jp = C.jit ? C.progs[0] : nullptr;
    // one timed span per kernel launch (a launch per width class used)
    for (uint32_t c = 0; c < N_WCLASS; ++c) {
      if (!(C.classes_used & (1u << c))) continue;
      PhaseTimer t(ctx, st, 0, timed);
      P.wclass = c;
      const uint32_t threads = 64u << c;
      const size_t lds = C.class_lds[c];
      if (jp && jp->jit_class == c) {
        int occ = 0;
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, jp->jit_fn, (int)threads, lds) != hipSuccess ||
            occ < 1)
          occ = 1;
        const uint32_t blocks =
            std::max<uint32_t>(1, std::min(std::min(L.max_items_class[c], (uint32_t)(cus * occ)), REC_MAX_BLOCKS));
        void* args[] = {&P};
        HIP_TRY(hipModuleLaunchKernel(jp->jit_fn, blocks, 1, 1, threads, 1, 1, (unsigned)lds, st, args, nullptr));
        continue;
      }
      const uint32_t resident = (uint32_t)cus * (uint32_t)interp_occupancy(threads, lds, C.class_vreg[c]);
      const uint32_t blocks = std::max<uint32_t>(1, std::min(std::min(L.max_items_class[c], resident), REC_MAX_BLOCKS));
      HIP_TRY(launch_interp(P, blocks, threads, lds, C.class_vreg[c], st));
    }
    // one-group programs' spilled intervals, checked by the group check
    if (do_log && L.sc_blocks) {
      PhaseTimer t(ctx, st, 2, timed);
      ScParams S;
      memset(&S, 0, sizeof S);
      S.progs = progs; S.slots = slots; S.chunks = chunks; S.chunk_index = chunk_index;
      S.log_keys = P.log_keys; S.log_vals = P.log_vals; S.wg_count = P.wg_count;
      S.queue = P.queue + N_WCLASS;
      S.ends = (uint32_t*)(ws + L.sc_ends);
      S.order = (const uint32_t*)(ws + L.sc_order);
      S.rec = P.rec;
      S.bs = L.bs; S.bc = L.bc;
      const uint32_t blocks =
          std::max<uint32_t>(1, std::min<uint32_t>(L.sc_blocks, (uint32_t)cus * (uint32_t)sc_group_occupancy()));
      HIP_TRY(launch_sc_group(S, blocks, st));
    }
  }
  if (!do_log) return RC_OK;
  int second = 0;
  u64 *lk0 = (u64*)(ws + L.lk0), *lv0 = (u64*)(ws + L.lv0), *lk1 = (u64*)(ws + L.lk1), *lv1 = (u64*)(ws + L.lv1);
  // (a call whose programs keep every logged access in LDS has an empty
  // global log: no log sort, no global pass)
  if (!L.lds_only) {
    PhaseTimer t(ctx, st, 1, timed);
    // Each work-group's log region holds one (instance, group) in execution
    // (so interval) order; a stable sort above the group and interval fields
    // therefore leaves every run of equal full keys, and every (instance,
    // cell) run, contiguous, which is all the check needs.
    HIP_TRY(sort_log(lk0, lv0, lk1, lv1, cnt + CNT_LOG, L.max_log, L.nbits_log, L.bg + L.bk,
                     (const uint32_t*)(ws + L.wg_count),
                     (const u64*)(ws + L.wg_base), (uint32_t*)(ws + L.tiles), L.max_wg, (uint32_t*)(ws + L.hist),
                     C.radix_bits, st, &second, L.filter ? (const uint32_t*)(ws + L.cc) : nullptr, L.cc_stride, L.bc, L.bk));
  }
  if (!L.lds_only) {
    PhaseTimer t(ctx, st, 2, timed);
    SegParams S;
    memset(&S, 0, sizeof S);
    S.keys = second ? lk1 : lk0;
    S.vals = second ? lv1 : lv0;
    S.n_ptr = cnt + CNT_LOG;
    S.bc = L.bc; S.bg = L.bg; S.bk = L.bk; S.bs = L.bs;
    S.progs = progs; S.slots = slots; S.chunks = chunks; S.chunk_index = chunk_index;
    memset(&S.out, 0, sizeof S.out);
    S.out.staging = ws + L.stage; S.out.rec_keys = (u64*)(ws + L.rk0); S.out.rec_idx = (uint32_t*)(ws + L.ri0);
    S.out.rec_count = cnt + CNT_REC; S.out.rec_cap = L.max_rec; S.out.status_word = (uint32_t*)(cnt + CNT_STATUS);
    S.out.rec_dead = cnt + CNT_DEAD;
    S.longq = (u64*)(ws + L.longq);
    S.long_count = cnt + CNT_LONG;
    S.long_cap = L.long_cap;
    HIP_TRY(launch_seg_check(S, L.max_log, st));
  }
  HIP_TRY(launch_clamp(cnt + CNT_REC, L.max_rec, (uint32_t*)(cnt + CNT_STATUS), 2u, st));
  HIP_TRY(launch_live_count(cnt + CNT_REC, cnt + CNT_DEAD, cnt + CNT_LIVE, st));
  int rsecond = 0;
  {
    PhaseTimer t(ctx, st, 3, timed);
    if (L.rank) {
      // each (slot, scope)'s first output position
      HIP_TRY(scan_counts((uint32_t*)(ws + L.scope_cnt), L.scope_n, (uint32_t*)(ws + L.scope_tmp), st));
    } else {
      HIP_TRY(sort_pairs_u32((u64*)(ws + L.rk0), (uint32_t*)(ws + L.ri0), (u64*)(ws + L.rk1),
                             (uint32_t*)(ws + L.ri1), cnt + CNT_REC, L.max_rec, L.nbits_rec,
                             (uint32_t*)(ws + L.hist), st, &rsecond));
    }
  }
  {
    PhaseTimer t(ctx, st, 4, timed);
    GatherParams Gp;
    memset(&Gp, 0, sizeof Gp);
    Gp.staging = (const rc_record_dev*)(ws + L.stage);
    Gp.idx = (const uint32_t*)(ws + (rsecond ? L.ri1 : L.ri0));
    Gp.n_ptr = cnt + CNT_LIVE;   // the unused slots sort after every record
    Gp.stage_cap = L.max_rec;
    Gp.out_base = (u64*)d_n_records;
    Gp.out = (rc_record_dev*)d_records;
    Gp.cap = cap;
    Gp.chunks = chunks; Gp.chunk_index = chunk_index;
    Gp.inst_flags = (uint32_t*)(ws + L.inst_flags);
    Gp.inst_race = (uint32_t*)(ws + L.inst_race);
    Gp.inst_benign = (uint32_t*)(ws + L.inst_benign);
    if (L.rank) {
      Gp.keys = (const u64*)(ws + L.rk0);
      Gp.reserved = cnt + CNT_REC;
      Gp.scope_base = (const uint32_t*)(ws + L.scope_cnt);
      Gp.table_n = L.scope_n;
      Gp.status_word = (uint32_t*)(cnt + CNT_STATUS);
      HIP_TRY(launch_place_out(Gp, L.max_rec, st));
    } else {
      HIP_TRY(launch_gather(Gp, L.max_rec, st));
    }
    FinalParams F;
    memset(&F, 0, sizeof F);
    F.progs = progs; F.slots = slots; F.chunks = chunks; F.chunk_index = chunk_index;
    F.inst_acc = (const u64*)(ws + L.inst_acc);
    F.inst_race = (const uint32_t*)(ws + L.inst_race);
    F.inst_benign = (const uint32_t*)(ws + L.inst_benign);
    F.inst_intervals = (const uint32_t*)(ws + L.inst_int);
    F.inst_flags = (const uint32_t*)(ws + L.inst_flags);
    F.inst_fault = (const u64*)(ws + L.inst_fault);
    F.out = (rc_summary_dev*)d_summaries;
    F.max_slots = L.max_slots;
    HIP_TRY(launch_finalize(F, st));
    HIP_TRY(launch_advance((u64*)d_n_records, cnt + CNT_LIVE, (uint32_t*)(ws + L.chunk_index), st));
  }
  return RC_OK;
}

// Build the call's tables, upload them, and enqueue every chunk.
// no_alloc: the caller cannot allocate (rc_check_static): chunks are
// launched one by one, with no graph and no timing events.
rc_status run_call(rc_ctx* ctx, Call& C, char* ws, size_t ws_bytes, rc_record* d_records, u64 cap,
                   u64* d_n_records, rc_summary* d_summaries, int do_log, uint32_t* epoch_out,
                   bool no_alloc = false) {
  hipStream_t st = ctx->stream;
  std::string why;
  if (!plan(C, ws_bytes, &why)) return fail(RC_E_INVAL, "%s", why.c_str());
  const Layout& L = C.L;
  // overlay versions: one base per chunk, above everything earlier on this workspace
  // The device checks the workspace header and clears the pool unless it
  // holds only cells this context versioned (a cleared pool is valid for any
  // version base, so the host keeps its own sequence).
  rc_ctx::WsState& wst = ctx->ws_state[(void*)ws];
  HIP_TRY(launch_ws_validate((u64*)(ws + L.header), 0x52433147524146ull, (u64)(uintptr_t)ctx, wst.gen,
                             (u64*)(ws + L.overlay), L.max_ovl, (uint32_t*)(ws + L.header + 32), st));
  wst.gen += 1;
  for (ChunkDesc& ch : C.chunks) {
    if (wst.next_epoch + C.epoch_stride >= (1u << 22)) {
      ch.clear_overlay = 1;
      wst.next_epoch = 1;
    }
    ch.epoch = wst.next_epoch;
    wst.next_epoch += C.epoch_stride;
  }
  if (epoch_out) *epoch_out = C.chunks.empty() ? 1u : C.chunks.back().epoch;
  // per-program descriptor tables (bindings and log placement may change between calls)
  if (ctx->upload_done) HIP_TRY(hipEventSynchronize(ctx->upload_done));
  std::vector<ProgDesc> pd(C.progs.size());
  for (size_t i = 0; i < C.progs.size(); ++i) {
    rc_prog* p = C.progs[i];
    for (size_t a = 0; a < p->arrays.size(); ++a) p->arrays[a].logged = array_logged(p, (uint32_t)a);
    unsigned char* h = p->h_tables.data();
    memcpy(h, p->arrays.data(), p->arrays.size() * sizeof(ArrayDesc));
    memcpy(h + (p->off_scalars - p->off_arrays), p->scalars.data(), p->scalars.size() * sizeof(ScalarDesc));
    memcpy(h + (p->off_cellbase - p->off_arrays), p->cellbase.data(), p->cellbase.size() * 4);
    memcpy(h + (p->off_size - p->off_arrays), p->sizes.data(), p->sizes.size() * 4);
    HIP_TRY(hipMemcpyAsync((char*)p->d_mem + p->off_arrays, h, p->h_tables.size(), hipMemcpyHostToDevice, st));
    ProgDesc& D = pd[i];
    memset(&D, 0, sizeof D);
    D.code = (const uint32_t*)p->d_mem;
    D.arrays = (const ArrayDesc*)((char*)p->d_mem + p->off_arrays);
    D.scalars = (const ScalarDesc*)((char*)p->d_mem + p->off_scalars);
    D.cellbase = (const uint32_t*)((char*)p->d_mem + p->off_cellbase);
    D.size = (const uint32_t*)((char*)p->d_mem + p->off_size);
    D.n_arrays = (uint32_t)p->c.arrays.size();
    D.n_global = p->c.n_global;
    D.n_scalars = (uint32_t)p->c.scalars.size();
    // no LDS registers for registers held in VGPRs
    D.nregs = C.jit || C.class_vreg[width_class(p->W)] ? 0u : p->c.nregs;
    D.G = p->G;
    D.W = p->W;
    D.nwaves = (p->W + 63) / 64;
    D.lds_local_cells = p->lds_local_cells;
    D.lds_log_cap = p->lds_log_cap;
    lds_table(p, &D.tab_base, &D.tab_cells);
    if (!p->lds_log_cap) D.tab_cells = 0;
    D.overlay_cells = p->overlay_cells;
    D.NI = (uint32_t)p->c.max_intervals;
    D.wg_log_cap = wg_log_entries(p);
    D.sc = p->sc ? 1u : 0u;
    D.n_cells = p->n_logged_cells;
    D.log_mask = p->log_mask;
    D.log_high = p->log_high;
    // interpreted programs that cannot fault elide group steps (the code's
    // per-instruction flags, set for the current shape)
    D.nf = !C.jit && p->never_faults ? 1u : 0u;
    D.step_limit = p->step_limit;
  }
  rc_record_out R;
  memset(&R, 0, sizeof R);
  u64* cnt = (u64*)(ws + L.counters);
  R.staging = ws + L.stage;
  R.rec_keys = (u64*)(ws + L.rk0);
  R.rec_idx = (uint32_t*)(ws + L.ri0);
  R.rec_count = cnt + CNT_REC;
  R.rec_cap = L.max_rec;
  R.rec_dead = cnt + CNT_DEAD;
  R.status_word = (uint32_t*)(cnt + CNT_STATUS);
  R.rank_keys = L.rank ? 1u : 0u;
  R.scope_cnt = L.rank ? (uint32_t*)(ws + L.scope_cnt) : nullptr;
  // one upload of all call tables (they sit contiguously after the overlay pool)
  const size_t tbytes = L.counters - L.tables;
  ctx->h_call.assign(tbytes, 0);
  unsigned char* h = ctx->h_call.data();
  memcpy(h + (L.progs - L.tables), pd.data(), pd.size() * sizeof(ProgDesc));
  memcpy(h + (L.slots - L.tables), C.slots.data(), C.slots.size() * sizeof(SlotDesc));
  memcpy(h + (L.chunks - L.tables), C.chunks.data(), C.chunks.size() * sizeof(ChunkDesc));
  memcpy(h + (L.items - L.tables), C.items.data(), C.items.size() * 4);
  if (L.sc_blocks) memcpy(h + (L.sc_order - L.tables), C.sc_order.data(), C.sc_order.size() * 4);
  memcpy(h + (L.recout - L.tables), &R, sizeof R);
  HIP_TRY(hipMemcpyAsync(ws + L.tables, h, tbytes, hipMemcpyHostToDevice, st));
  if (!ctx->upload_done) HIP_TRY(hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ctx->upload_done, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.chunk_index), 1, 0u, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(cnt + CNT_STATUS), 1, 0u, st));
  HIP_TRY(launch_fill_u64(cnt + CNT_STATS, N_STATS, 0ull, st));
  if (do_log) ctx->last_stats = cnt + CNT_STATS;
  if (d_n_records) HIP_TRY(launch_fill_u64((u64*)d_n_records, 1, 0ull, st));
  const size_t n_chunks = C.chunks.size();
  // With several chunks and no profiling, capture one chunk's kernels as a
  // graph and replay it; every chunk reads its parameters from device tables.
  if (n_chunks > 1 && ctx->use_graphs && !ctx->profiling && !no_alloc) {
    if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    rc_status s = enqueue_chunk(ctx, C, ws, ctx->capture_stream, d_n_records, d_records, cap, d_summaries, do_log,
                                false);
    hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (s != RC_OK) { if (graph) (void)hipGraphDestroy(graph); return s; }
    if (e != hipSuccess) return fail(RC_E_HIP, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(RC_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    for (size_t c = 0; c < n_chunks; ++c) {
      e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) { (void)hipGraphExecDestroy(exec); return fail(RC_E_HIP, "graph launch: %s", hipGetErrorString(e)); }
    }
    ctx->graphs_to_free.push_back(exec);
    return RC_OK;
  }
  for (size_t c = 0; c < n_chunks; ++c) {
    rc_status s = enqueue_chunk(ctx, C, ws, st, d_n_records, d_records, cap, d_summaries, do_log, !no_alloc);
    if (s) return s;
  }
  return RC_OK;
}

rc_status add_program(Call& C, rc_prog* p, std::map<rc_prog*, uint32_t>& index, uint32_t* out) {
  auto it = index.find(p);
  if (it != index.end()) { *out = it->second; return RC_OK; }
  rc_status s = check_ready(p);
  if (s) return s;
  const uint32_t k = (uint32_t)C.progs.size();
  C.progs.push_back(p);
  index[p] = k;
  *out = k;
  return RC_OK;
}

}  // namespace

extern "C" {

const char* rc_last_error(void) { return g_err.c_str(); }

rc_status rc_ctx_create(int device, void* hip_stream, rc_ctx** out) {
  if (!out) return fail(RC_E_INVAL, "out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(RC_E_HIP, "no HIP device available");
  if (device < 0 || device >= n) return fail(RC_E_INVAL, "device %d out of range (%d devices)", device, n);
  HIP_TRY(hipSetDevice(device));
  // the static workspace's address on this device, once per device (each
  // GPU holds its own copy of the array at its own address)
  void* sws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_ws_mu);
    if (device >= (int)g_static_ws.size()) g_static_ws.resize(device + 1, nullptr);
    if (!g_static_ws[device]) {
      void* addr = nullptr;
      HIP_TRY(static_ws_address(&addr));
      if (!addr) return fail(RC_E_HIP, "the static workspace has no address on device %d", device);
      g_static_ws[device] = addr;
    }
    sws = g_static_ws[device];
  }
  rc_ctx* c = new rc_ctx;
  c->device = device;
  c->static_ws = sws;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return RC_OK;
}

rc_status rc_ctx_destroy(rc_ctx* ctx) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (hipGraphExec_t g : ctx->graphs_to_free) (void)hipGraphExecDestroy(g);
  if (ctx->upload_done) (void)hipEventDestroy(ctx->upload_done);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  delete ctx;
  return RC_OK;
}

rc_status rc_ctx_profile(rc_ctx* ctx, int enable) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  ctx->profiling = enable != 0;
  ctx->spans.clear();
  ctx->events_used = 0;
  return RC_OK;
}

rc_status rc_ctx_profile_read(rc_ctx* ctx, rc_profile* out) {
  if (!ctx || !out) return fail(RC_E_INVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (const auto& sp : ctx->spans) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->events[sp.second], ctx->events[sp.second + 1]));
    out->ms[sp.first] += ms;
    out->launches[sp.first] += 1;
  }
  ctx->spans.clear();
  ctx->events_used = 0;
  return RC_OK;
}

rc_status rc_ctx_set_stream(rc_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  ctx->stream = (hipStream_t)hip_stream;
  return RC_OK;
}

rc_status rc_prog_load(rc_ctx* ctx, const char* src, size_t len, rc_prog** out) {
  if (!ctx || !src || !out) return fail(RC_E_INVAL, "NULL argument");
  rc_prog* p = new rc_prog;
  p->ctx = ctx;
  std::string err;
  bool is_limit = false;
  if (!compile_program(src, len, &p->c, &err, &is_limit)) {
    delete p;
    return fail(is_limit ? RC_E_LIMIT : RC_E_PARSE, "%s", err.c_str());
  }
  const Compiled& c = p->c;
  const uint32_t na = (uint32_t)c.arrays.size();
  p->arrays.assign(na, ArrayDesc());
  p->cellbase.assign(na, 0xFFFFFFFFu);
  p->sizes.assign(na, 0u);
  uint32_t cb = 0, ov = 0, lds = 0;
  for (uint32_t a = 0; a < na; ++a) {
    const CompiledArray& ca = c.arrays[a];
    ArrayDesc& d = p->arrays[a];
    memset(&d, 0, sizeof d);
    d.size = ca.size;
    d.logged = ca.written ? 1u : 0u;
    if (!ca.global) {
      d.kind = AK_LOCAL;
      d.offset = lds;
      lds += ca.size;
    } else if (ca.written) {
      d.kind = AK_GLOBAL_RW;
      d.offset = ov;
      ov += ca.size;
    } else {
      d.kind = AK_GLOBAL_RO;
    }
    if (ca.written) {
      d.cellbase = cb;
      p->cellbase[a] = cb;
      cb += ca.size;
    } else {
      d.cellbase = 0xFFFFFFFFu;
    }
    p->sizes[a] = ca.size;
  }
  p->n_logged_cells = cb;
  p->overlay_cells = ov;
  p->owned.assign(na, 0);
  p->lds_local_cells = lds;
  p->scalars.assign(c.scalars.size(), ScalarDesc());
  for (auto& s : p->scalars) memset(&s, 0, sizeof s);
  // device memory: code + tables (allocated once here; checks allocate nothing)
  size_t o = align_up(c.code.size() * 4, 256);
  p->off_arrays = o;
  o += align_up(na * sizeof(ArrayDesc) + 1, 64);
  p->off_scalars = o;
  o += align_up(p->scalars.size() * sizeof(ScalarDesc) + 1, 64);
  p->off_cellbase = o;
  o += align_up(na * 4 + 1, 64);
  p->off_size = o;
  o += align_up(na * 4 + 1, 64);
  p->d_bytes = o;
  p->h_tables.assign(o - p->off_arrays, 0);
  hipError_t e = hipMalloc(&p->d_mem, o);
  if (e != hipSuccess) {
    delete p;
    return fail(RC_E_HIP, "hipMalloc(program): %s", hipGetErrorString(e));
  }
  e = hipMemcpy(p->d_mem, c.code.data(), c.code.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(p->d_mem);
    delete p;
    return fail(RC_E_HIP, "hipMemcpy(program): %s", hipGetErrorString(e));
  }
  *out = p;
  return RC_OK;
}

rc_status rc_prog_free(rc_prog* p) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  for (const rc_prog::JitEntry& j : p->jit_mods) (void)hipModuleUnload(j.mod);
  if (p->d_mem) (void)hipFree(p->d_mem);
  delete p;
  return RC_OK;
}

rc_status rc_prog_get_info(const rc_prog* p, rc_prog_info* out) {
  if (!p || !out) return fail(RC_E_INVAL, "NULL argument");
  out->n_global_arrays = p->c.n_global;
  out->n_local_arrays = p->c.n_local;
  out->n_scalars = (uint32_t)p->c.scalars.size();
  out->n_vars = (uint32_t)p->c.vars.size();
  out->n_stmts = p->c.n_stmts;
  return RC_OK;
}

rc_status rc_prog_array(const rc_prog* p, uint32_t id, char* name, size_t name_len, uint64_t* cells, int* is_global) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (id >= p->c.arrays.size()) return fail(RC_E_INVAL, "array id %u out of range", id);
  const CompiledArray& a = p->c.arrays[id];
  if (name && name_len) snprintf(name, name_len, "%s", a.name.c_str());
  if (cells) *cells = a.size;
  if (is_global) *is_global = a.global ? 1 : 0;
  return RC_OK;
}

rc_status rc_prog_scalar(const rc_prog* p, uint32_t id, char* name, size_t name_len) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (id >= p->c.scalars.size()) return fail(RC_E_INVAL, "scalar id %u out of range", id);
  if (name && name_len) snprintf(name, name_len, "%s", p->c.scalars[id].c_str());
  return RC_OK;
}

rc_status rc_prog_owned(const rc_prog* p, uint32_t id, int* owned) {
  if (!p || !owned) return fail(RC_E_INVAL, "NULL argument");
  if (!p->shaped) return fail(RC_E_STATE, "rc_set_ndrange has not been called");
  if (id >= p->c.arrays.size()) return fail(RC_E_INVAL, "array id %u out of range", id);
  *owned = p->owned[id] ? 1 : 0;
  return RC_OK;
}

rc_status rc_owned_arrays(const char* src, size_t len, uint32_t num_groups, uint32_t group_size, uint8_t* owned,
                          uint32_t capacity, uint32_t* n_arrays, int* never_faults) {
  if (!src || !n_arrays || (capacity && !owned)) return fail(RC_E_INVAL, "NULL argument");
  if (group_size < 1 || group_size > MAX_WG || num_groups < 1 || (u64)num_groups * group_size >= (1ull << 26))
    return fail(RC_E_INVAL, "launch shape out of range");
  Compiled c;
  std::string err;
  bool is_limit = false;
  if (!compile_program(src, len, &c, &err, &is_limit)) return fail(is_limit ? RC_E_LIMIT : RC_E_PARSE, "%s", err.c_str());
  const Ownership proof = prove_ownership(c, num_groups, group_size);
  const std::vector<OwnedArray>& o = proof.arrays;
  if (never_faults) *never_faults = proof.never_faults && c.dyn_iters <= DEFAULT_STEP_LIMIT ? 1 : 0;
  *n_arrays = (uint32_t)o.size();
  for (uint32_t a = 0; a < capacity && a < o.size(); ++a) owned[a] = o[a].owned ? 1 : (o[a].race_free ? 2 : 0);
  return RC_OK;
}

rc_status rc_log_intervals(const char* src, size_t len, uint32_t num_groups, uint32_t group_size, uint64_t* mask,
                           int* later) {
  if (!src || !mask || !later) return fail(RC_E_INVAL, "NULL argument");
  if (group_size < 1 || group_size > MAX_WG || num_groups < 1 || (u64)num_groups * group_size >= (1ull << 26))
    return fail(RC_E_INVAL, "launch shape out of range");
  Compiled c;
  std::string err;
  bool is_limit = false;
  if (!compile_program(src, len, &c, &err, &is_limit)) return fail(is_limit ? RC_E_LIMIT : RC_E_PARSE, "%s", err.c_str());
  const Ownership proof = prove_ownership(c, num_groups, group_size);
  *mask = proof.local_log_mask;
  *later = proof.local_log_high ? 1 : 0;
  return RC_OK;
}

// Generate, compile and load the program's kernel for its current width
// class and launch shape (synchronous; the runtime compiler takes about a
// second), or take it from the kernels already compiled.
static rc_status jit_build(rc_prog* p) {
  const uint32_t cls = width_class(p->W);
  const JitShape shape = jit_shape_of(p);
  for (const rc_prog::JitEntry& j : p->jit_mods) {
    if (j.cls == cls && j.shape == shape) {
      p->jit_fn = j.fn;
      p->jit_class = cls;
      p->jit_shape = shape;
      p->jit_on = true;
      return RC_OK;
    }
  }
  std::vector<uint32_t> kinds;
  for (const ArrayDesc& a : p->arrays) kinds.push_back(a.kind);
  const std::string src = jit_source(p->c.code, p->c.nregs, 64u << cls, kinds, shape);
  std::vector<char> obj;
  std::string log;
  if (!jit_compile(src, &obj, &log)) {
    p->jit_on = false;
    return fail(RC_E_HIP, "runtime compilation of the program kernel failed: %.900s", log.c_str());
  }
  HIP_TRY(hipSetDevice(p->ctx->device));
  hipModule_t mod = nullptr;
  HIP_TRY(hipModuleLoadData(&mod, obj.data()));
  hipFunction_t fn = nullptr;
  hipError_t e = hipModuleGetFunction(&fn, mod, "rc_jit_kernel");
  if (e != hipSuccess) {
    (void)hipModuleUnload(mod);
    return fail(RC_E_HIP, "hipModuleGetFunction: %s", hipGetErrorString(e));
  }
  p->jit_mods.push_back({cls, shape, mod, fn});
  p->jit_fn = fn;
  p->jit_class = cls;
  p->jit_shape = shape;
  p->jit_on = true;
  return RC_OK;
}

rc_status rc_prog_jit(rc_prog* p, int enable) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (!enable) {
    p->jit_on = false;
    return RC_OK;
  }
  if (!p->shaped) return fail(RC_E_STATE, "set the NDRange before compiling the program kernel");
  return jit_build(p);
}

static rc_status apply_shape(rc_prog* p);

rc_status rc_set_ndrange(rc_prog* p, uint32_t num_groups, uint32_t group_size) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (group_size < 1 || group_size > MAX_WG) return fail(RC_E_LIMIT, "group size must be in [1, 1024]");
  if (num_groups < 1) return fail(RC_E_INVAL, "num_groups must be >= 1");
  if ((u64)num_groups * group_size >= (1ull << 26)) return fail(RC_E_LIMIT, "num_groups * group_size must be < 2^26");
  const uint32_t W = group_size;
  const uint32_t WP = ((W + 63) / 64) * 64;
  const size_t lds = ((sizeof(Ctl) + 15) & ~(size_t)15) + (size_t)p->lds_local_cells * 8 + (size_t)p->c.nregs * WP * 4;
  if (lds > LDS_LIMIT)
    return fail(RC_E_LIMIT, "local arrays and registers need %zu bytes of LDS (limit %u)", lds, LDS_LIMIT);
  if (p->c.max_intervals >= (1ull << 32)) return fail(RC_E_LIMIT, "too many barrier intervals");
  p->G = num_groups;
  p->W = W;
  p->shaped = true;
  return apply_shape(p);
}

// The program's descriptors for its launch shape and tuning: the static
// proofs (none when the tuning turns them off), overlay placement, log cell
// keys and the LDS log size; a per-program kernel for the shape.
static rc_status apply_shape(rc_prog* p) {
  const uint32_t W = p->W;
  Ownership proof;
  if (p->proofs_off) proof.arrays.assign(p->c.arrays.size(), OwnedArray());
  else proof = prove_ownership(p->c, p->G, p->W);
  const std::vector<OwnedArray>& own = proof.arrays;
  // not logged: owned arrays, and local arrays race-free within every interval
  p->owned.assign(own.size(), 0);
  for (size_t a = 0; a < own.size(); ++a) p->owned[a] = own[a].owned || own[a].race_free;
  // overlay words per group: a global rw array owned with a stride keeps its
  // work-items' cells lane by lane (so a wave's accesses to one offset are
  // consecutive words), in own_span * W words instead of one word per cell
  uint32_t ov = 0;
  for (size_t a = 0; a < own.size(); ++a) {
    ArrayDesc& d = p->arrays[a];
    d.own_stride = 0;
    d.own_lo = 0;
    d.own_span = 0;
    if (d.kind != AK_GLOBAL_RW) continue;
    d.offset = ov;
    const u64 span = own[a].stride != 0 ? (u64)(own[a].hi - own[a].lo + 1) : 0;
    if (span != 0 && span * W <= d.size) {
      d.own_stride = (int32_t)own[a].stride;
      d.own_lo = (int32_t)own[a].lo;
      d.own_span = (uint32_t)span;
      ov += (uint32_t)(span * W);
    } else {
      ov += d.size;
    }
  }
  p->overlay_cells = ov;
  // (a program that can reach the loop-iteration limit can stop there)
  p->never_faults = proof.never_faults && p->c.dyn_iters <= p->step_limit;
  p->log_mask = proof.local_log_mask;
  p->log_high = proof.local_log_high ? 1u : 0u;
  for (size_t a = 0; a < own.size(); ++a) {
    ArrayDesc& d = p->arrays[a];
    d.nosync = proof.never_faults && (d.kind == AK_GLOBAL_RO || p->owned[a]) ? 1u : 0u;
  }
  // log cell keys: the written arrays that are not owned, global ones first
  uint32_t cb = 0;
  for (size_t a = 0; a < own.size(); ++a) {
    const bool keyed = p->c.arrays[a].written && !p->owned[a];
    p->arrays[a].cellbase = keyed ? cb : 0xFFFFFFFFu;
    p->cellbase[a] = keyed ? cb : 0xFFFFFFFFu;
    if (keyed) cb += p->c.arrays[a].size;
  }
  p->n_logged_cells = cb;
  p->logged_mem = p->c.dyn_logged_mem;
  p->logged_local = p->c.dyn_logged_local;
  for (size_t a = 0; a < p->owned.size(); ++a) {
    if (!p->owned[a] || !p->c.arrays[a].written) continue;
    p->logged_mem -= std::min(p->logged_mem, p->c.dyn_mem_array[a]);
    if (!p->c.arrays[a].global) p->logged_local -= std::min(p->logged_local, p->c.dyn_mem_array[a]);
  }
  set_log_cap(p);
  // the interpreter's code: load and store instructions of a program that
  // cannot fault carry INSN_NO_STEP where no conflicting access needs their
  // group step
  {
    std::vector<uint32_t> code = p->c.code;
    if (p->never_faults) {
      const std::vector<uint8_t> keep = group_steps(p->c.code, jit_shape_of(p), false);
      for (size_t i = 0; i < keep.size(); ++i) {
        const uint32_t op = code[4 * i] & 63u;
        if ((op == OP_LOAD || op == OP_STORE) && !keep[i]) code[4 * i + 3] |= INSN_NO_STEP;
      }
    }
    HIP_TRY(hipSetDevice(p->ctx->device));
    HIP_TRY(hipMemcpy(p->d_mem, code.data(), code.size() * 4, hipMemcpyHostToDevice));
  }
  // a per-program kernel is compiled for one launch shape
  if (p->jit_on && !jit_current(p)) return jit_build(p);
  return RC_OK;
}

static rc_status check_range(int64_t lo, int64_t hi) {
  if (hi - lo < 1 || hi - lo > (1ll << 32)) return fail(RC_E_INVAL, "seeded range needs 1 <= hi - lo <= 2^32");
  if (lo < INT32_MIN || hi > (int64_t)INT32_MAX + 1) return fail(RC_E_INVAL, "seeded range outside int32");
  return RC_OK;
}

rc_status rc_bind_seeded(rc_prog* p, uint32_t id, int64_t lo, int64_t hi) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (id >= p->c.n_global) return fail(RC_E_INVAL, "array %u is not a global array", id);
  rc_status s = check_range(lo, hi);
  if (s) return s;
  p->arrays[id].bind = BIND_SEEDED;
  p->arrays[id].lo = lo;
  p->arrays[id].hi = hi;
  p->arrays[id].dptr = nullptr;
  return RC_OK;
}

rc_status rc_bind_device(rc_prog* p, uint32_t id, const int32_t* d_cells) {
  if (!p || !d_cells) return fail(RC_E_INVAL, "NULL argument");
  if (id >= p->c.n_global) return fail(RC_E_INVAL, "array %u is not a global array", id);
  p->arrays[id].bind = BIND_DEVICE;
  p->arrays[id].dptr = d_cells;
  return RC_OK;
}

rc_status rc_bind_scalar_seeded(rc_prog* p, uint32_t id, int64_t lo, int64_t hi) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (id >= p->scalars.size()) return fail(RC_E_INVAL, "scalar %u out of range", id);
  rc_status s = check_range(lo, hi);
  if (s) return s;
  p->scalars[id].bind = BIND_SEEDED;
  p->scalars[id].lo = lo;
  p->scalars[id].hi = hi;
  return RC_OK;
}

rc_status rc_bind_scalar(rc_prog* p, uint32_t id, int32_t value) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (id >= p->scalars.size()) return fail(RC_E_INVAL, "scalar %u out of range", id);
  p->scalars[id].bind = BIND_DEVICE;   // a fixed value
  p->scalars[id].value = value;
  return RC_OK;
}

rc_status rc_prog_set_tuning(rc_prog* p, const rc_tuning* t) {
  if (!p || !t) return fail(RC_E_INVAL, "NULL argument");
  if (t->radix_bits > 8) return fail(RC_E_INVAL, "radix_bits must be in 1..8 (0: default)");
  if (t->record_sort > 1) return fail(RC_E_INVAL, "record_sort must be 0 or 1");
  if (t->proofs_off > 1) return fail(RC_E_INVAL, "proofs_off must be 0 or 1");
  if (t->global_spills > 1) return fail(RC_E_INVAL, "global_spills must be 0 or 1");
  p->record_sort = t->record_sort;
  p->global_spills = t->global_spills;
  p->lds_log_pref = t->lds_log_entries;
  p->radix_bits = t->radix_bits ? t->radix_bits : 8;
  const uint32_t limit = t->step_limit ? t->step_limit : DEFAULT_STEP_LIMIT;
  const bool reprove = p->proofs_off != t->proofs_off || p->step_limit != limit;
  p->proofs_off = t->proofs_off;
  p->step_limit = limit;
  if (p->shaped && reprove) return apply_shape(p);
  if (p->shaped) set_log_cap(p);
  if (p->jit_on && p->shaped && !jit_current(p)) return jit_build(p);
  return RC_OK;
}

static std::string bucket_key(const rc_prog* p, int device) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  const double ib = (double)p->W * (p->G == 1 ? p->c.interval_logged_all : p->c.interval_logged_local);
  char b[160];
  snprintf(b, sizeof b, "%s|wclass%u|groups%u|interval%u|cells%u|v2", arch.c_str(), width_class(p->W),
           bits_for(p->G), bits_for((u64)(ib + 1)), bits_for(std::max<uint32_t>(1, p->n_logged_cells)));
  return b;
}

static bool cache_lookup(const char* path, const std::string& key, rc_tuning* t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  const std::string q = "\"" + key + "\"";
  while (std::getline(f, line)) {
    const size_t at = line.find(q);
    if (at == std::string::npos) continue;
    unsigned T = 0, d = 0;
    const size_t a = line.find("\"lds_log_entries\":"), b = line.find("\"radix_bits\":");
    if (a == std::string::npos || b == std::string::npos) return false;
    if (sscanf(line.c_str() + a + 18, "%u", &T) != 1 || sscanf(line.c_str() + b + 13, "%u", &d) != 1) return false;
    memset(t, 0, sizeof *t);
    t->lds_log_entries = T;
    t->radix_bits = d;
    return true;
  }
  return false;
}

static void cache_store(const char* path, const std::string& key, const rc_tuning& t, double ms) {
  std::vector<std::string> entries;
  {
    std::ifstream f(path);
    std::string line;
    const std::string q = "\"" + key + "\"";
    while (f && std::getline(f, line)) {
      if (line.find("\": {") == std::string::npos || line.find(q) != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      entries.push_back(line);
    }
  }
  char b[320];
  snprintf(b, sizeof b, "  \"%s\": {\"lds_log_entries\": %u, \"radix_bits\": %u, \"ms\": %.4f}", key.c_str(),
           t.lds_log_entries, t.radix_bits, ms);
  entries.push_back(b);
  std::ofstream f(path, std::ios::trunc);
  f << "{\n";
  for (size_t i = 0; i < entries.size(); ++i) f << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  f << "}\n";
}

rc_status rc_autotune(rc_prog* p, uint64_t seed0, uint32_t n_seeds, void* d_ws, size_t ws_bytes,
                      const char* cache_path, rc_tuning* chosen) {
  if (!p || !d_ws || !chosen || n_seeds == 0) return fail(RC_E_INVAL, "bad argument");
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  const std::string key = bucket_key(p, ctx->device);
  rc_tuning t;
  if (cache_path && cache_lookup(cache_path, key, &t)) {
    t.record_sort = p->record_sort;
    t.proofs_off = p->proofs_off;
    t.step_limit = p->step_limit;
    t.global_spills = p->global_spills;
    s = rc_prog_set_tuning(p, &t);
    if (s) return s;
    *chosen = t;
    return RC_OK;
  }
  // candidates: LDS log sizes (deduplicated after clamping) x digit widths
  std::vector<rc_tuning> cands;
  std::vector<uint32_t> seen_caps;
  const uint32_t T_opts[] = {0, 256, 1024, 4096, 8192, 16384};
  const uint32_t d_opts[] = {8, 6, 4};
  const uint32_t saved_pref = p->lds_log_pref, saved_bits = p->radix_bits;
  for (uint32_t T : T_opts) {
    p->lds_log_pref = T;
    const uint32_t cap = lds_log_entries(p);
    if (std::find(seen_caps.begin(), seen_caps.end(), cap) != seen_caps.end()) continue;
    seen_caps.push_back(cap);
    for (uint32_t d : d_opts) {
      rc_tuning c;
      memset(&c, 0, sizeof c);
      c.lds_log_entries = T;
      c.radix_bits = d;
      c.record_sort = p->record_sort;
      c.proofs_off = p->proofs_off;
      c.step_limit = p->step_limit;
      c.global_spills = p->global_spills;
      cands.push_back(c);
    }
  }
  p->lds_log_pref = saved_pref;
  p->radix_bits = saved_bits;
  const u64 cap = 1ull << 20;
  rc_record* d_rec = nullptr;
  rc_summary* d_sum = nullptr;
  u64* d_n = nullptr;
  HIP_TRY(hipMalloc(&d_rec, cap * sizeof(rc_record)));
  HIP_TRY(hipMalloc(&d_sum, (size_t)n_seeds * sizeof(rc_summary)));
  HIP_TRY(hipMalloc(&d_n, 8));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<unsigned char> ref_rec, ref_sum, cur_rec, cur_sum;
  u64 ref_n = 0;
  double best = 1e30;
  rc_tuning best_t = cands.empty() ? rc_tuning() : cands[0];
  rc_status result = RC_OK;
  for (size_t i = 0; i < cands.size() && result == RC_OK; ++i) {
    rc_prog_set_tuning(p, &cands[i]);
    double ms_best = 1e30;
    for (int rep = 0; rep < 3 && result == RC_OK; ++rep) {
      (void)hipEventRecord(e0, ctx->stream);
      result = rc_check(p, seed0, n_seeds, d_ws, ws_bytes, d_rec, cap, (uint64_t*)d_n, d_sum);
      (void)hipEventRecord(e1, ctx->stream);
      if (result == RC_OK) result = rc_sync(ctx);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) ms_best = std::min(ms_best, (double)ms);   // the first run warms up
    }
    if (result != RC_OK) break;
    u64 n = 0;
    (void)hipMemcpy(&n, d_n, 8, hipMemcpyDeviceToHost);
    const u64 k = std::min(n, cap);
    cur_rec.resize(k * sizeof(rc_record));
    cur_sum.resize((size_t)n_seeds * sizeof(rc_summary));
    (void)hipMemcpy(cur_rec.data(), d_rec, cur_rec.size(), hipMemcpyDeviceToHost);
    (void)hipMemcpy(cur_sum.data(), d_sum, cur_sum.size(), hipMemcpyDeviceToHost);
    if (i == 0) {
      ref_rec = cur_rec;
      ref_sum = cur_sum;
      ref_n = n;
    } else if (n != ref_n || cur_rec != ref_rec || cur_sum != ref_sum) {
      result = fail(RC_E_HIP, "tuning candidate %zu changed the report: results must not depend on tuning", i);
      break;
    }
    if (ms_best < best) {
      best = ms_best;
      best_t = cands[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_rec);
  (void)hipFree(d_sum);
  (void)hipFree(d_n);
  if (result != RC_OK) {
    rc_tuning back;
    memset(&back, 0, sizeof back);
    back.lds_log_entries = saved_pref;
    back.radix_bits = saved_bits;
    back.record_sort = p->record_sort;
    back.proofs_off = p->proofs_off;
    back.step_limit = p->step_limit;
    back.global_spills = p->global_spills;
    rc_prog_set_tuning(p, &back);
    return result;
  }
  rc_prog_set_tuning(p, &best_t);
  if (cache_path) cache_store(cache_path, key, best_t, best);
  *chosen = best_t;
  return RC_OK;
}

rc_status rc_workspace_size(const rc_prog* p, uint32_t n_seeds, size_t* bytes) {
  if (!p || !bytes) return fail(RC_E_INVAL, "NULL argument");
  if (!p->shaped) return fail(RC_E_STATE, "rc_set_ndrange has not been called");
  Call C;
  C.progs.push_back(const_cast<rc_prog*>(p));
  const uint32_t n = std::max<uint32_t>(1, n_seeds);
  C.inst_prog.assign(n, 0);
  C.inst_seed.assign(n, 0);
  std::string why;
  if (!plan(C, ~(size_t)0, &why)) return fail(RC_E_LIMIT, "%s", why.c_str());
  *bytes = C.L.total;
  return RC_OK;
}

rc_status rc_check(rc_prog* p, uint64_t seed0, uint32_t n_seeds, void* d_ws, size_t ws_bytes,
                   rc_record* d_records, uint64_t cap, uint64_t* d_n_records, rc_summary* d_summaries) {
  if (!p || !d_ws || !d_n_records || !d_summaries) return fail(RC_E_INVAL, "NULL argument");
  if (cap > 0 && !d_records) return fail(RC_E_INVAL, "d_records is NULL with cap > 0");
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  if (n_seeds == 0) {
    HIP_TRY(launch_fill_u64((u64*)d_n_records, 1, 0ull, ctx->stream));
    return RC_OK;
  }
  Call C;
  C.progs.push_back(p);
  C.inst_prog.assign(n_seeds, 0);
  C.inst_seed.resize(n_seeds);
  for (uint32_t j = 0; j < n_seeds; ++j) C.inst_seed[j] = seed0 + j;
  s = run_call(ctx, C, (char*)d_ws, ws_bytes, d_records, cap, (u64*)d_n_records, d_summaries, 1, nullptr);
  if (s) return s;
  ctx->pending.push_back(Pending{(u64*)d_n_records, cap, (uint32_t*)((char*)d_ws + C.L.counters + CNT_STATUS * 8)});
  return RC_OK;
}

rc_status rc_check_static(rc_prog* p, uint64_t seed0, uint32_t n_seeds, rc_record* d_records, uint64_t cap,
                          uint64_t* d_n_records, rc_summary* d_summaries) {
  static_assert(STATIC_WS_BYTES == (size_t)RC_STATIC_WS_BYTES, "static workspace size");
  if (!p || !d_n_records || !d_summaries) return fail(RC_E_INVAL, "NULL argument");
  if (cap > 0 && !d_records) return fail(RC_E_INVAL, "d_records is NULL with cap > 0");
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  if (!ctx->static_ws) return fail(RC_E_STATE, "the context has no static workspace");
  size_t one = 0;
  s = rc_workspace_size(p, 1, &one);
  if (s) return s;
  if (one > STATIC_WS_BYTES)
    return fail(RC_E_INVAL, "one instance needs %zu bytes of workspace, more than the %zu bytes of the static workspace",
                one, STATIC_WS_BYTES);
  HIP_TRY(hipSetDevice(ctx->device));
  if (n_seeds == 0) {
    HIP_TRY(launch_fill_u64((u64*)d_n_records, 1, 0ull, ctx->stream));
    return RC_OK;
  }
  Call C;
  C.progs.push_back(p);
  C.inst_prog.assign(n_seeds, 0);
  C.inst_seed.resize(n_seeds);
  for (uint32_t j = 0; j < n_seeds; ++j) C.inst_seed[j] = seed0 + j;
  char* ws = (char*)ctx->static_ws;
  s = run_call(ctx, C, ws, STATIC_WS_BYTES, d_records, cap, (u64*)d_n_records, d_summaries, 1, nullptr, true);
  if (s) return s;
  ctx->pending.push_back(Pending{(u64*)d_n_records, cap, (uint32_t*)(ws + C.L.counters + CNT_STATUS * 8)});
  return RC_OK;
}

rc_status rc_batch_check(rc_ctx* ctx, rc_prog* const* progs, const uint64_t* seeds, uint32_t n, void* d_ws,
                         size_t ws_bytes, rc_record* d_records, uint64_t cap, uint64_t* d_n_records,
                         rc_summary* d_summaries) {
  if (!ctx || !d_ws || !d_n_records || !d_summaries || (n && (!progs || !seeds)))
    return fail(RC_E_INVAL, "NULL argument");
  if (cap > 0 && !d_records) return fail(RC_E_INVAL, "d_records is NULL with cap > 0");
  HIP_TRY(hipSetDevice(ctx->device));
  if (n == 0) {
    HIP_TRY(launch_fill_u64((u64*)d_n_records, 1, 0ull, ctx->stream));
    return RC_OK;
  }
  Call C;
  std::map<rc_prog*, uint32_t> index;
  C.inst_prog.resize(n);
  C.inst_seed.assign(seeds, seeds + n);
  for (uint32_t i = 0; i < n; ++i) {
    if (!progs[i]) return fail(RC_E_INVAL, "programs[%u] is NULL", i);
    if (progs[i]->ctx != ctx) return fail(RC_E_INVAL, "programs[%u] belongs to another context", i);
    rc_status s = add_program(C, progs[i], index, &C.inst_prog[i]);
    if (s) return s;
  }
  rc_status s = run_call(ctx, C, (char*)d_ws, ws_bytes, d_records, cap, (u64*)d_n_records, d_summaries, 1, nullptr);
  if (s) return s;
  ctx->pending.push_back(Pending{(u64*)d_n_records, cap, (uint32_t*)((char*)d_ws + C.L.counters + CNT_STATUS * 8)});
  return RC_OK;
}

rc_status rc_sync(rc_ctx* ctx) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipError_t e = hipStreamSynchronize(ctx->stream);
  for (hipGraphExec_t g : ctx->graphs_to_free) (void)hipGraphExecDestroy(g);
  ctx->graphs_to_free.clear();
  if (e != hipSuccess) {
    ctx->pending.clear();
    return fail(RC_E_HIP, "stream synchronize: %s", hipGetErrorString(e));
  }
  rc_status result = RC_OK;
  std::string msg;
  for (const Pending& pd : ctx->pending) {
    u64 n = 0;
    uint32_t status = 0;
    e = hipMemcpy(&n, pd.d_n_records, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&status, pd.d_status, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      result = RC_E_HIP;
      msg = std::string("reading check status: ") + hipGetErrorString(e);
      break;
    }
    if (status & 4u) {
      result = RC_E_HIP;
      msg = "internal error: an access left its owned-array placement";
    } else if (status & 8u) {
      result = RC_E_HIP;
      msg = "internal error: a per-program kernel ran on a program of another launch shape";
    } else if (status & 16u) {
      result = RC_E_HIP;
      msg = "internal error: a program proven never to fault faulted";
    } else if (status != 0u) {
      result = RC_E_HIP;
      msg = "internal capacity exceeded (access log or record staging)";
    } else if (n > pd.cap && result == RC_OK) {
      result = RC_E_OVERFLOW;
      char b[160];
      snprintf(b, sizeof b, "%llu race records, capacity %llu", (unsigned long long)n, (unsigned long long)pd.cap);
      msg = b;
    }
  }
  ctx->pending.clear();
  if (result != RC_OK) return fail(result, "%s", msg.c_str());
  return RC_OK;
}

rc_status rc_call_stats(rc_ctx* ctx, rc_stats* out) {
  if (!ctx || !out) return fail(RC_E_INVAL, "NULL argument");
  if (!ctx->last_stats) return fail(RC_E_STATE, "no check call on this context yet");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  u64 v[N_STATS];
  HIP_TRY(hipMemcpy(v, ctx->last_stats, sizeof v, hipMemcpyDeviceToHost));
  out->logged = v[0];
  out->logged_global = v[1];
  out->intervals_spilled = v[2];
  out->intervals = v[3];
  out->instructions = v[4];
  out->wave_instructions = v[5];
  out->global_pass = v[6];
  return RC_OK;
}

rc_status rc_read_final(rc_prog* p, uint64_t seed, uint32_t array_id, int32_t* d_out, void* d_ws, size_t ws_bytes) {
  if (!p || !d_out || !d_ws) return fail(RC_E_INVAL, "NULL argument");
  if (array_id >= p->c.n_global) return fail(RC_E_INVAL, "array %u is not a global array", array_id);
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  Call C;
  C.progs.push_back(p);
  C.inst_prog.assign(1, 0);
  C.inst_seed.assign(1, seed);
  uint32_t epoch = 1;
  s = run_call(ctx, C, (char*)d_ws, ws_bytes, nullptr, 0, nullptr, nullptr, 0, &epoch);
  if (s) return s;
  const ArrayDesc& A = p->arrays[array_id];
  FinalMemParams M;
  memset(&M, 0, sizeof M);
  M.size = A.size;
  M.G = p->G;
  M.overlay_cells = p->overlay_cells;
  M.offset = A.offset;
  M.W = p->W;
  M.own_stride = A.own_stride;
  M.own_lo = A.own_lo;
  M.own_span = A.own_span;
  M.array_id = array_id;
  M.bind = A.bind;
  M.rw = A.kind == AK_GLOBAL_RW ? 1u : 0u;
  M.epoch = epoch;
  M.lo = A.lo;
  M.hi = A.hi;
  M.seed = seed;
  M.dptr = A.dptr;
  M.overlay = (const u64*)((char*)d_ws + C.L.overlay);
  M.out = d_out;
  HIP_TRY(launch_final_merge(M, ctx->stream));
  return RC_OK;
}


// ---- triage features -----------------------------------------------------
static size_t feat_items_bytes(uint32_t n) { return ((size_t)n * sizeof(FeatItem) + 255) & ~(size_t)255; }

rc_status rc_features_workspace_size(uint32_t n, uint32_t n_programs, size_t* bytes) {
  if (!bytes) return fail(RC_E_INVAL, "NULL argument");
  *bytes = feat_items_bytes(n) + (size_t)n_programs * sizeof(FeatProg);
  return RC_OK;
}

static int64_t ceil_log2_u(uint64_t s) {
  int64_t k = 0;
  while (((uint64_t)1 << k) < s) ++k;
  return k;
}

static void fill_feat_prog(const rc_prog* p, FeatProg* F) {
  memset(F, 0, sizeof *F);
  const Compiled& c = p->c;
  for (int k = 0; k < 104; ++k) F->stat[k] = c.feat[k];
  F->stat[104] = (float)p->W / 1024.f;
  F->stat[105] = (float)p->G / 1024.f;
  if (c.n_global > 0) F->stat[106] = (float)ceil_log2_u(c.arrays[0].size) / 32.f;
  if (c.n_global > 1) F->stat[107] = (float)ceil_log2_u(c.arrays[1].size) / 32.f;
  int64_t local_cells = 0;
  for (const CompiledArray& a : c.arrays)
    if (!a.global) local_cells += a.size;
  F->stat[108] = (float)local_cells / 65536.f;
  F->stat[109] = (float)((int64_t)p->G * (int64_t)p->W) / 1048576.f;
  for (uint32_t j = 0; j < 2 && j < c.n_global; ++j) {
    const ArrayDesc& A = p->arrays[j];
    FeatArray& fa = F->arr[j];
    fa.present = 1;
    fa.bind = A.bind;
    fa.size = A.size;
    fa.lo = A.lo;
    fa.hi = A.hi;
    fa.dptr = A.dptr;
  }
}

rc_status rc_features(rc_ctx* ctx, rc_prog* const* progs, const uint64_t* seeds, uint32_t n, float* d_feat,
                      void* d_ws, size_t ws_bytes) {
  if (!ctx || (n && (!progs || !seeds || !d_feat || !d_ws))) return fail(RC_E_INVAL, "NULL argument");
  if (n == 0) return RC_OK;
  if (n > (1u << 26)) return fail(RC_E_LIMIT, "n = %u instances exceeds 2^26", n);
  std::map<const rc_prog*, uint32_t> index;
  std::vector<const rc_prog*> uniq;
  std::vector<FeatItem> items(n);
  for (uint32_t i = 0; i < n; ++i) {
    const rc_prog* p = progs[i];
    if (!p) return fail(RC_E_INVAL, "programs[%u] is NULL", i);
    if (p->ctx != ctx) return fail(RC_E_INVAL, "programs[%u] belongs to another context", i);
    auto it = index.find(p);
    if (it == index.end()) {
      rc_status s = check_ready(p);
      if (s) return s;
      it = index.emplace(p, (uint32_t)uniq.size()).first;
      uniq.push_back(p);
    }
    items[i].seed = seeds[i];
    items[i].prog = it->second;
    items[i].pad = 0;
  }
  const size_t off_progs = feat_items_bytes(n);
  const size_t need = off_progs + uniq.size() * sizeof(FeatProg);
  if (ws_bytes < need)
    return fail(RC_E_INVAL, "workspace of %zu bytes is below the %zu needed for %u instances of %zu programs",
                ws_bytes, need, n, uniq.size());
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  if (ctx->upload_done) HIP_TRY(hipEventSynchronize(ctx->upload_done));
  ctx->h_call.assign(need, 0);
  unsigned char* h = ctx->h_call.data();
  memcpy(h, items.data(), items.size() * sizeof(FeatItem));
  for (size_t k = 0; k < uniq.size(); ++k) fill_feat_prog(uniq[k], (FeatProg*)(h + off_progs) + k);
  HIP_TRY(hipMemcpyAsync(d_ws, h, need, hipMemcpyHostToDevice, st));
  if (!ctx->upload_done) HIP_TRY(hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ctx->upload_done, st));
  HIP_TRY(launch_features((const FeatItem*)d_ws, (const FeatProg*)((char*)d_ws + off_progs), n, d_feat, st));
  return RC_OK;
}

// ---- ranking -----------------------------------------------------------------
struct RankLayout {
  size_t k0, v0, k1, v1, hist, n_ptr, total;
};
static RankLayout rank_layout(uint32_t n) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  RankLayout L;
  size_t o = 0;
  L.k0 = o; o = up(o + (size_t)n * 8);
  L.v0 = o; o = up(o + (size_t)n * 4);
  L.k1 = o; o = up(o + (size_t)n * 8);
  L.v1 = o; o = up(o + (size_t)n * 4);
  L.hist = o; o = up(o + sort_hist_words(n ? n : 1) * 4);
  L.n_ptr = o; o = up(o + 8);
  L.total = o;
  return L;
}

rc_status rc_rank_workspace_size(uint32_t n, size_t* bytes) {
  if (!bytes) return fail(RC_E_INVAL, "NULL argument");
  *bytes = rank_layout(n).total;
  return RC_OK;
}

rc_status rc_rank(rc_ctx* ctx, const float* d_scores, uint32_t n, uint32_t* d_order, void* d_ws, size_t ws_bytes) {
  if (!ctx || (n && (!d_scores || !d_order || !d_ws))) return fail(RC_E_INVAL, "NULL argument");
  if (n == 0) return RC_OK;
  const RankLayout L = rank_layout(n);
  if (ws_bytes < L.total) return fail(RC_E_INVAL, "workspace of %zu bytes is below the %zu needed", ws_bytes, L.total);
  HIP_TRY(hipSetDevice(ctx->device));
  char* ws = (char*)d_ws;
  hipStream_t st = ctx->stream;
  uint32_t idx_bits = 0;
  while (idx_bits < 32 && ((u64)1 << idx_bits) < (u64)n) ++idx_bits;
  HIP_TRY(launch_rank_keys(d_scores, n, idx_bits, (u64*)(ws + L.k0), (uint32_t*)(ws + L.v0), (u64*)(ws + L.n_ptr),
                           st));
  int in_second = 0;
  HIP_TRY(sort_pairs_u32((u64*)(ws + L.k0), (uint32_t*)(ws + L.v0), (u64*)(ws + L.k1), (uint32_t*)(ws + L.v1),
                         (const u64*)(ws + L.n_ptr), n, 32 + idx_bits, (uint32_t*)(ws + L.hist), st, &in_second));
  HIP_TRY(hipMemcpyAsync(d_order, ws + (in_second ? L.v1 : L.v0), (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  return RC_OK;
}

// ---- triage network ------------------------------------------------------
rc_status rc_mlp_workspace_size(uint32_t n, size_t* bytes) {
  if (!bytes) return fail(RC_E_INVAL, "NULL argument");
  *bytes = mlp_ws_bytes(n);
  return RC_OK;
}

static rc_status mlp_args(rc_ctx* ctx, uint32_t n, const void* ws, size_t ws_bytes) {
  if (!ctx || !ws) return fail(RC_E_INVAL, "NULL argument");
  if (n == 0) return fail(RC_E_INVAL, "n must be at least 1");
  if (n > (1u << 26)) return fail(RC_E_LIMIT, "n = %u rows exceeds 2^26", n);
  if (ws_bytes < mlp_ws_bytes(n))
    return fail(RC_E_INVAL, "workspace of %zu bytes is below the %zu needed for %u rows", ws_bytes, mlp_ws_bytes(n),
                n);
  return RC_OK;
}

rc_status rc_mlp_forward(rc_ctx* ctx, const float* d_params, const float* d_feat, uint32_t n, float* d_logits,
                         void* d_ws, size_t ws_bytes) {
  rc_status s = mlp_args(ctx, n, d_ws, ws_bytes);
  if (s) return s;
  if (!d_params || !d_feat || !d_logits) return fail(RC_E_INVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(mlp_forward(d_params, d_feat, n, d_logits, d_ws, ctx->stream));
  return RC_OK;
}

rc_status rc_mlp_grad(rc_ctx* ctx, const float* d_params, const float* d_feat, const float* d_labels,
                      const uint32_t* d_rows, uint32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes) {
  rc_status s = mlp_args(ctx, n, d_ws, ws_bytes);
  if (s) return s;
  if (!d_params || !d_feat || !d_labels || !d_grad || !d_loss) return fail(RC_E_INVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(mlp_grad(d_params, d_feat, d_labels, d_rows, n, d_grad, d_loss, d_ws, ctx->stream));
  return RC_OK;
}

rc_status rc_mlp_train_step(rc_ctx* ctx, float* d_params, float* d_adam_m, float* d_adam_v, uint32_t step,
                            const float* d_feat, const float* d_labels, const uint32_t* d_rows, uint32_t n, float lr,
                            float* d_loss, void* d_ws, size_t ws_bytes) {
  rc_status s = mlp_args(ctx, n, d_ws, ws_bytes);
  if (s) return s;
  if (!d_params || !d_adam_m || !d_adam_v || !d_feat || !d_labels || !d_loss) return fail(RC_E_INVAL, "NULL argument");
  if (step == 0) return fail(RC_E_INVAL, "Adam steps count from 1");
  if (!(lr > 0.f) || !(lr < 1e30f)) return fail(RC_E_INVAL, "learning rate must be positive and finite");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(mlp_train_step(d_params, d_adam_m, d_adam_v, step, d_feat, d_labels, d_rows, n, lr, d_loss, d_ws,
                         ctx->stream));
  return RC_OK;
}

}  // extern "C"
