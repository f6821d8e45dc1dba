// capi.cpp -- the rc_* C ABI (include/rc.h): contexts, programs, bindings,
// workspace layout and the pass loop that drives the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/rc.h"
#include "frontend.h"
#include "kernels.h"
#include "rc_internal.h"

using namespace rc;
typedef unsigned long long u64;

static_assert(sizeof(rc_record) == 40, "rc_record is 40 bytes");
static_assert(sizeof(rc_summary) == 40, "rc_summary is 40 bytes");

namespace {

thread_local std::string g_err;

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
  std::map<void*, std::string> ws_sig;   // workspace -> layout of its persistent part
  std::vector<Pending> pending;
  rc_status deferred = RC_OK;
  std::string deferred_msg;
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
  uint32_t lds_log_pref = 0;         // preferred LDS log entries when a spill is possible (0: default)
  uint32_t lds_log_cap = 0;          // chosen for the current shape
  // device: code, then tables
  void* d_mem = nullptr;
  size_t off_arrays = 0, off_scalars = 0, off_cellbase = 0, off_size = 0, off_recout = 0, d_bytes = 0;
  std::vector<unsigned char> h_tables;   // staging for the async table upload
};

namespace {

// record a HIP event on the ctx stream when profiling; returns its pool index
rc_status prof_mark(rc_ctx* ctx, size_t* idx) {
  if (!ctx->profiling) return RC_OK;
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    ctx->events.push_back(e);
  }
  *idx = ctx->events_used++;
  HIP_TRY(hipEventRecord(ctx->events[*idx], ctx->stream));
  return RC_OK;
}

struct PhaseTimer {
  rc_ctx* ctx;
  int phase;
  size_t start = 0;
  PhaseTimer(rc_ctx* c, int ph) : ctx(c), phase(ph) {
    if (ctx->profiling) prof_mark(ctx, &start);
  }
  ~PhaseTimer() {
    if (!ctx->profiling) return;
    size_t end = 0;
    if (prof_mark(ctx, &end) == RC_OK && end == start + 1) ctx->spans.push_back({phase, start});
  }
};

struct Layout {
  uint32_t n_slots = 0;
  u64 log_cap = 0, rec_cap = 0, wg_log_cap = 0;
  uint32_t bi = 0, bc = 0, bg = 0, bk = 0, bs = 0, nbits_log = 0, nbits_rec = 0;
  uint32_t NI = 0;
  // persistent
  size_t epochs = 0, epoch_used = 0, overlay = 0, persistent_end = 0;
  // per pass
  size_t counters = 0, wg_count = 0, inst_acc = 0, inst_fault = 0, inst_int = 0, inst_race = 0, inst_benign = 0, inst_flags = 0;
  size_t lk0 = 0, lv0 = 0, lk1 = 0, lv1 = 0, hist = 0, stage = 0, rk0 = 0, ri0 = 0, rk1 = 0, ri1 = 0;
  size_t total = 0;
  std::string signature;
};

// counters block: [0] log_count, [1] rec_count, [2] status word (u32 in a u64 slot)
enum { CNT_LOG = 0, CNT_REC = 1, CNT_STATUS = 2, CNT_WORDS = 4 };

bool make_layout(const rc_prog* p, uint32_t n_slots, Layout* L, std::string* why) {
  const Compiled& c = p->c;
  L->n_slots = n_slots;
  const u64 items = (u64)n_slots * p->G * p->W;
  const double logcap = (double)items * (double)c.dyn_logged_mem;
  if (logcap > 4.0e9) { *why = "access-log bound exceeds 4e9 entries for this pass"; return false; }
  L->wg_log_cap = std::max<u64>(1, (u64)p->W * c.dyn_logged_mem);
  L->log_cap = L->wg_log_cap * n_slots * p->G;
  L->rec_cap = L->log_cap;
  L->NI = (uint32_t)std::min<u64>(c.max_intervals, 0xFFFFFFFFull);
  L->bi = bits_for(n_slots);
  L->bc = bits_for(std::max<u64>(1, p->n_logged_cells));
  L->bg = bits_for(p->G);
  L->bk = bits_for(c.max_intervals);
  L->nbits_log = L->bi + L->bc + L->bg + L->bk;
  L->bs = bits_for((u64)p->G * c.max_intervals + 1);
  L->nbits_rec = L->bi + L->bs + L->bc;
  if (L->nbits_log > 64 || L->nbits_rec > 64 || L->bc > 32 || L->bg > 26 || L->bk > 32) {
    *why = "sort key wider than 64 bits";
    return false;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  const u64 ovl = (u64)n_slots * p->G;
  L->epochs = take(ovl * 4);
  L->epoch_used = take(ovl * 4);
  L->overlay = take(ovl * (u64)p->overlay_cells * 8);
  L->persistent_end = o;
  L->counters = take(CNT_WORDS * 8);
  L->wg_count = take((size_t)n_slots * p->G * 4);
  L->inst_acc = take((size_t)n_slots * 8);
  L->inst_fault = take((size_t)n_slots * 8);
  L->inst_int = take((size_t)n_slots * 4);
  L->inst_race = take((size_t)n_slots * 4);
  L->inst_benign = take((size_t)n_slots * 4);
  L->inst_flags = take((size_t)n_slots * 4);
  L->lk0 = take(L->log_cap * 8);
  L->lv0 = take(L->log_cap * 8);
  L->lk1 = take(L->log_cap * 8);
  L->lv1 = take(L->log_cap * 8);
  L->hist = take(std::max(sort_log_hist_words((u64)n_slots * p->G, L->wg_log_cap, L->log_cap),
                          sort_hist_words(L->rec_cap)) * 4);
  L->stage = take(L->rec_cap * sizeof(rc_record));
  L->rk0 = take(L->rec_cap * 8);
  L->ri0 = take(L->rec_cap * 4);
  L->rk1 = take(L->rec_cap * 8);
  L->ri1 = take(L->rec_cap * 4);
  L->total = o;
  char sig[160];
  snprintf(sig, sizeof sig, "%p/%u/%u/%u/%zu", (const void*)p, n_slots, p->G, p->overlay_cells, L->persistent_end);
  L->signature = sig;
  return true;
}

rc_record_out record_out(const Layout& L, char* ws) {
  rc_record_out R;
  memset(&R, 0, sizeof R);
  u64* cnt = (u64*)(ws + L.counters);
  R.staging = ws + L.stage;
  R.rec_keys = (u64*)(ws + L.rk0);
  R.rec_idx = (uint32_t*)(ws + L.ri0);
  R.rec_count = cnt + CNT_REC;
  R.rec_cap = L.rec_cap;
  R.status_word = (uint32_t*)(cnt + CNT_STATUS);
  return R;
}

// LDS bytes of everything except the interval log
size_t lds_fixed_bytes(const rc_prog* p) {
  const uint32_t WP = ((p->W + 63) / 64) * 64;
  return (size_t)p->lds_local_cells * 8 + (size_t)p->c.nregs * WP * 4 + sizeof(Ctl);
}

// Entries of the interval log kept in LDS (a power of two; 0 = none): large
// enough for the program's static bound when that fits, else as large as LDS
// allows up to `pref` entries.
uint32_t lds_log_entries(const rc_prog* p) {
  const bool lds_globals = p->G == 1;
  const u64 per_item = p->c.dyn_logged_local + (lds_globals ? p->c.dyn_logged_mem - p->c.dyn_logged_local : 0);
  if (per_item == 0) return 0;
  const size_t fixed = lds_fixed_bytes(p);
  if (fixed + 32 > LDS_LIMIT) return 0;
  uint32_t fit = 2;
  while ((size_t)fit * 2 * 16 + fixed <= LDS_LIMIT && fit * 2 <= 65536u) fit *= 2;
  const double bound = (double)p->W * (lds_globals ? p->c.interval_logged_all : p->c.interval_logged_local);
  if (p->lds_log_pref) {   // explicit tuning
    uint32_t t = 2;
    while (t * 2 <= p->lds_log_pref && t * 2 <= fit) t *= 2;
    return t;
  }
  const uint32_t pref = 4096u;
  uint32_t want = 2;
  while (want < bound && want < 65536u) want *= 2;
  if ((double)want >= bound && want <= fit) return want;   // never spills
  return std::min(fit, std::max<uint32_t>(pref, 2));
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

rc_status upload_tables(rc_prog* p, hipStream_t st, const rc_record_out* R) {
  unsigned char* h = p->h_tables.data();
  for (size_t a = 0; a < p->arrays.size(); ++a) {
    ArrayDesc& d = p->arrays[a];
    if (!p->c.arrays[a].written) d.logged = LOG_NONE;
    else if (p->lds_log_cap && (!p->c.arrays[a].global || p->G == 1)) d.logged = LOG_LDS;
    else d.logged = LOG_GLOBAL;
  }
  memcpy(h + p->off_arrays - p->off_arrays, p->arrays.data(), p->arrays.size() * sizeof(ArrayDesc));
  if (R) memcpy(h + (p->off_recout - p->off_arrays), R, sizeof *R);
  memcpy(h + (p->off_scalars - p->off_arrays), p->scalars.data(), p->scalars.size() * sizeof(ScalarDesc));
  memcpy(h + (p->off_cellbase - p->off_arrays), p->cellbase.data(), p->cellbase.size() * 4);
  memcpy(h + (p->off_size - p->off_arrays), p->sizes.data(), p->sizes.size() * 4);
  HIP_TRY(hipMemcpyAsync((char*)p->d_mem + p->off_arrays, h, p->h_tables.size(), hipMemcpyHostToDevice, st));
  return RC_OK;
}

rc_status prepare_workspace(rc_prog* p, void* ws, const Layout& L) {
  rc_ctx* ctx = p->ctx;
  auto it = ctx->ws_sig.find(ws);
  if (it == ctx->ws_sig.end() || it->second != L.signature) {
    // fresh (or re-laid-out) workspace: clear epochs, epoch records and overlays
    HIP_TRY(launch_fill_u64((u64*)ws, L.persistent_end / 8, 0ull, ctx->stream));
    ctx->ws_sig[ws] = L.signature;
  }
  return RC_OK;
}

InterpParams interp_params(const rc_prog* p, const Layout& L, char* ws, uint64_t seed0, uint32_t inst_offset,
                           uint32_t n, int do_log) {
  InterpParams P;
  memset(&P, 0, sizeof P);
  P.code = (const uint32_t*)p->d_mem;
  P.n_arrays = (uint32_t)p->c.arrays.size();
  P.n_global = p->c.n_global;
  P.n_scalars = (uint32_t)p->c.scalars.size();
  P.nregs = p->c.nregs;
  P.G = p->G;
  P.W = p->W;
  P.nwaves = (p->W + 63) / 64;
  P.lds_local_cells = p->lds_local_cells;
  P.n_slots = n;
  P.overlay_cells = p->overlay_cells;
  P.max_store_seq = (uint32_t)std::min<u64>(p->c.dyn_stores, (1u << 22));
  P.inst_offset = inst_offset;
  P.seed0 = seed0;
  P.bc = L.bc;
  P.bg = L.bg;
  P.bk = L.bk;
  P.arrays = (const ArrayDesc*)((char*)p->d_mem + p->off_arrays);
  P.scalars = (const ScalarDesc*)((char*)p->d_mem + p->off_scalars);
  P.epochs = (uint32_t*)(ws + L.epochs);
  P.epoch_used = (uint32_t*)(ws + L.epoch_used);
  P.overlay = (u64*)(ws + L.overlay);
  u64* cnt = (u64*)(ws + L.counters);
  P.log_keys = (u64*)(ws + L.lk0);
  P.log_vals = (u64*)(ws + L.lv0);
  P.wg_count = (uint32_t*)(ws + L.wg_count);
  P.wg_log_cap = L.wg_log_cap;
  P.inst_acc = (u64*)(ws + L.inst_acc);
  P.inst_intervals = (uint32_t*)(ws + L.inst_int);
  P.inst_fault = (u64*)(ws + L.inst_fault);
  P.status_word = (uint32_t*)(cnt + CNT_STATUS);
  P.do_log = do_log;
  P.lds_log_cap = p->lds_log_cap;
  P.bs = L.bs;
  P.NI = L.NI;
  P.rec = (rc_record_out*)((char*)p->d_mem + p->off_recout);
  return P;
}

size_t lds_bytes(const rc_prog* p) { return lds_fixed_bytes(p) + (size_t)p->lds_log_cap * 16; }

rc_status reset_pass(const rc_prog* p, const Layout& L, char* ws, hipStream_t st) {
  HIP_TRY(launch_fill_u64((u64*)(ws + L.counters), 2, 0ull, st));   // log and record counters
  HIP_TRY(launch_fill_u64((u64*)(ws + L.inst_acc), L.n_slots, 0ull, st));
  HIP_TRY(launch_fill_u64((u64*)(ws + L.inst_fault), L.n_slots, ~0ull, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.inst_int), L.n_slots, 0u, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.inst_race), L.n_slots, 0u, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.inst_benign), L.n_slots, 0u, st));
  HIP_TRY(launch_fill_u32((uint32_t*)(ws + L.inst_flags), L.n_slots, 0u, st));
  (void)p;
  return RC_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* rc_last_error(void) { return g_err.c_str(); }

rc_status rc_ctx_create(int device, void* hip_stream, rc_ctx** out) {
  if (!out) return fail(RC_E_INVAL, "out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(RC_E_HIP, "no HIP device available");
  if (device < 0 || device >= n) return fail(RC_E_INVAL, "device %d out of range (%d devices)", device, n);
  HIP_TRY(hipSetDevice(device));
  rc_ctx* c = new rc_ctx;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return RC_OK;
}

rc_status rc_ctx_destroy(rc_ctx* ctx) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
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
  p->off_recout = o;
  o += align_up(sizeof(rc_record_out), 64);
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

rc_status rc_set_ndrange(rc_prog* p, uint32_t num_groups, uint32_t group_size) {
  if (!p) return fail(RC_E_INVAL, "prog is NULL");
  if (group_size < 1 || group_size > MAX_WG) return fail(RC_E_LIMIT, "group size must be in [1, 1024]");
  if (num_groups < 1) return fail(RC_E_INVAL, "num_groups must be >= 1");
  if ((u64)num_groups * group_size >= (1ull << 26)) return fail(RC_E_LIMIT, "num_groups * group_size must be < 2^26");
  const uint32_t W = group_size;
  const uint32_t WP = ((W + 63) / 64) * 64;
  const size_t lds = (size_t)p->lds_local_cells * 8 + (size_t)p->c.nregs * WP * 4 + sizeof(Ctl);
  if (lds > LDS_LIMIT)
    return fail(RC_E_LIMIT, "local arrays and registers need %zu bytes of LDS (limit %u)", lds, LDS_LIMIT);
  if (p->c.max_intervals >= (1ull << 32)) return fail(RC_E_LIMIT, "too many barrier intervals");
  p->G = num_groups;
  p->W = W;
  p->shaped = true;
  p->lds_log_cap = lds_log_entries(p);
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
  p->lds_log_pref = t->lds_log_entries;
  if (p->shaped) p->lds_log_cap = lds_log_entries(p);
  return RC_OK;
}

rc_status rc_workspace_size(const rc_prog* p, uint32_t n_seeds, size_t* bytes) {
  if (!p || !bytes) return fail(RC_E_INVAL, "NULL argument");
  if (!p->shaped) return fail(RC_E_STATE, "rc_set_ndrange has not been called");
  Layout L;
  std::string why;
  if (!make_layout(p, std::max<uint32_t>(1, n_seeds), &L, &why)) return fail(RC_E_LIMIT, "%s", why.c_str());
  *bytes = L.total;
  return RC_OK;
}

rc_status rc_check(rc_prog* p, uint64_t seed0, uint32_t n_seeds, void* d_ws, size_t ws_bytes,
                   rc_record* d_records, uint64_t cap, uint64_t* d_n_records, rc_summary* d_summaries) {
  if (!p || !d_ws || !d_n_records || !d_summaries) return fail(RC_E_INVAL, "NULL argument");
  if (cap > 0 && !d_records) return fail(RC_E_INVAL, "d_records is NULL with cap > 0");
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  hipStream_t st = ctx->stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_fill_u64((u64*)d_n_records, 1, 0ull, st));
  if (n_seeds == 0) return RC_OK;
  // largest pass that fits the workspace
  Layout L;
  std::string why;
  uint32_t lo = 1, hi = n_seeds;
  if (!make_layout(p, 1, &L, &why)) return fail(RC_E_LIMIT, "%s", why.c_str());
  if (L.total > ws_bytes)
    return fail(RC_E_INVAL, "workspace of %zu bytes is smaller than the %zu needed for one seed", ws_bytes, L.total);
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    Layout M;
    if (make_layout(p, mid, &M, &why) && M.total <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  make_layout(p, lo, &L, &why);
  char* ws = (char*)d_ws;
  s = prepare_workspace(p, ws, L);
  if (s) return s;
  const rc_record_out R = record_out(L, ws);
  s = upload_tables(p, st, &R);
  if (s) return s;
  u64* cnt = (u64*)(ws + L.counters);
  HIP_TRY(launch_fill_u64(cnt + CNT_STATUS, 1, 0ull, st));
  const size_t lds = lds_bytes(p);
  for (uint32_t off = 0; off < n_seeds; off += L.n_slots) {
    const uint32_t n = std::min(L.n_slots, n_seeds - off);
    {
      PhaseTimer t(ctx, 5);
      s = reset_pass(p, L, ws, st);
      if (s) return s;
    }
    InterpParams P = interp_params(p, L, ws, seed0, off, n, 1);
    {
      PhaseTimer t(ctx, 0);
      HIP_TRY(launch_interp(P, lds, st));
    }
    // sort the access log by (instance, cell, gid, interval)
    int second = 0;
    u64 *lk0 = (u64*)(ws + L.lk0), *lv0 = (u64*)(ws + L.lv0), *lk1 = (u64*)(ws + L.lk1), *lv1 = (u64*)(ws + L.lv1);
    {
      PhaseTimer t(ctx, 1);
      HIP_TRY(sort_log(lk0, lv0, lk1, lv1, cnt + CNT_LOG, L.log_cap, L.nbits_log, (const uint32_t*)(ws + L.wg_count),
                       (u64)n * p->G, L.wg_log_cap, (uint32_t*)(ws + L.hist), st, &second));
    }
    SegParams S;
    memset(&S, 0, sizeof S);
    S.keys = second ? lk1 : lk0;
    S.vals = second ? lv1 : lv0;
    S.n_ptr = cnt + CNT_LOG;
    S.bc = L.bc;
    S.bg = L.bg;
    S.bk = L.bk;
    S.bs = L.bs;
    S.G = p->G;
    S.W = p->W;
    S.NI = L.NI;
    S.n_arrays = (uint32_t)p->c.arrays.size();
    S.n_global = p->c.n_global;
    S.inst_offset = off;
    S.cellbase = (const uint32_t*)((char*)p->d_mem + p->off_cellbase);
    S.size = (const uint32_t*)((char*)p->d_mem + p->off_size);
    S.out = record_out(L, ws);
    {
      PhaseTimer t(ctx, 2);
      HIP_TRY(launch_seg_check(S, L.log_cap, st));
    }
    HIP_TRY(launch_clamp(cnt + CNT_REC, L.rec_cap, (uint32_t*)(cnt + CNT_STATUS), 2u, st));
    // canonical order of the records
    int rsecond = 0;
    {
      PhaseTimer t(ctx, 3);
      HIP_TRY(sort_pairs_u32((u64*)(ws + L.rk0), (uint32_t*)(ws + L.ri0), (u64*)(ws + L.rk1),
                             (uint32_t*)(ws + L.ri1), cnt + CNT_REC, L.rec_cap, L.nbits_rec,
                             (uint32_t*)(ws + L.hist), st, &rsecond));
    }
    PhaseTimer out_timer(ctx, 4);
    GatherParams Gp;
    memset(&Gp, 0, sizeof Gp);
    Gp.staging = (const rc_record_dev*)(ws + L.stage);
    Gp.idx = (const uint32_t*)(ws + (rsecond ? L.ri1 : L.ri0));
    Gp.n_ptr = cnt + CNT_REC;
    Gp.out_base = (u64*)d_n_records;
    Gp.out = (rc_record_dev*)d_records;
    Gp.cap = cap;
    Gp.inst_offset = off;
    Gp.inst_flags = (uint32_t*)(ws + L.inst_flags);
    Gp.inst_race = (uint32_t*)(ws + L.inst_race);
    Gp.inst_benign = (uint32_t*)(ws + L.inst_benign);
    HIP_TRY(launch_gather(Gp, L.rec_cap, st));
    FinalParams F;
    memset(&F, 0, sizeof F);
    F.n_slots = n;
    F.inst_offset = off;
    F.W = p->W;
    F.inst_acc = (const u64*)(ws + L.inst_acc);
    F.inst_race = (const uint32_t*)(ws + L.inst_race);
    F.inst_benign = (const uint32_t*)(ws + L.inst_benign);
    F.inst_intervals = (const uint32_t*)(ws + L.inst_int);
    F.inst_flags = (const uint32_t*)(ws + L.inst_flags);
    F.inst_fault = (const u64*)(ws + L.inst_fault);
    F.out = (rc_summary_dev*)d_summaries;
    HIP_TRY(launch_finalize(F, st));
  }
  ctx->pending.push_back(Pending{(u64*)d_n_records, cap, (uint32_t*)(cnt + CNT_STATUS)});
  return RC_OK;
}

rc_status rc_sync(rc_ctx* ctx) {
  if (!ctx) return fail(RC_E_INVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipError_t e = hipStreamSynchronize(ctx->stream);
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
    if (status != 0u) {
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

rc_status rc_read_final(rc_prog* p, uint64_t seed, uint32_t array_id, int32_t* d_out, void* d_ws, size_t ws_bytes) {
  if (!p || !d_out || !d_ws) return fail(RC_E_INVAL, "NULL argument");
  if (array_id >= p->c.n_global) return fail(RC_E_INVAL, "array %u is not a global array", array_id);
  rc_status s = check_ready(p);
  if (s) return s;
  rc_ctx* ctx = p->ctx;
  hipStream_t st = ctx->stream;
  HIP_TRY(hipSetDevice(ctx->device));
  Layout L;
  std::string why;
  if (!make_layout(p, 1, &L, &why)) return fail(RC_E_LIMIT, "%s", why.c_str());
  if (L.total > ws_bytes) return fail(RC_E_INVAL, "workspace too small (%zu < %zu)", ws_bytes, L.total);
  char* ws = (char*)d_ws;
  s = prepare_workspace(p, ws, L);
  if (s) return s;
  s = upload_tables(p, st, nullptr);
  if (s) return s;
  s = reset_pass(p, L, ws, st);
  if (s) return s;
  InterpParams P = interp_params(p, L, ws, seed, 0, 1, 0);
  HIP_TRY(launch_interp(P, lds_bytes(p), st));
  const ArrayDesc& A = p->arrays[array_id];
  FinalMemParams M;
  memset(&M, 0, sizeof M);
  M.size = A.size;
  M.G = p->G;
  M.overlay_cells = p->overlay_cells;
  M.offset = A.offset;
  M.array_id = array_id;
  M.bind = A.bind;
  M.rw = A.kind == AK_GLOBAL_RW ? 1u : 0u;
  M.lo = A.lo;
  M.hi = A.hi;
  M.seed = seed;
  M.dptr = A.dptr;
  M.overlay = (const u64*)(ws + L.overlay);
  M.epoch_used = (const uint32_t*)(ws + L.epoch_used);
  M.out = d_out;
  HIP_TRY(launch_final_merge(M, st));
  return RC_OK;
}

}  // extern "C"
