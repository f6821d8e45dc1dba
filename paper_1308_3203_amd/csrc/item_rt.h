// item_rt.h -- device runtime of one interpreted work-group ("item"): the
// lockstep protocol (group reductions, faults, the LDS and global access
// logs, the in-LDS interval check) shared by the bytecode interpreter and by
// the per-program kernels compiled at load time.  Self-contained: it is also
// handed to the runtime compiler.
#pragma once
#ifndef __HIPCC_RTC__        // the runtime compiler provides the HIP device API itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

#include "rc_internal.h"

namespace rc {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// seeded inputs: SplitMix64 (Steele, Lea, Flood 2014) in counter form
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + counter * 0x9E3779B97F4A7C15ull;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int32_t seeded_cell(uint64_t seed, uint32_t stream, uint32_t idx,
                                                int64_t lo, int64_t hi) {
  uint64_t hi32 = sm64(seed, ((uint64_t)stream << 32) | ((uint64_t)idx + 1)) >> 32;
  // stream < 2^17 and idx < 2^24: the counter never carries out of the low word
  uint64_t scaled = (hi32 * (uint64_t)(hi - lo)) >> 32;
  return (int32_t)(uint32_t)((uint64_t)lo + scaled);
}

// ---------------------------------------------------------------------------
// int32 operators (two's complement, wrapping; division faults on zero)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t alu_bin(uint32_t op, int32_t x, int32_t y, bool& dz) {
  const uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
  switch (op) {
    case B_ADD: return (int32_t)(ux + uy);
    case B_SUB: return (int32_t)(ux - uy);
    case B_MUL: return (int32_t)(ux * uy);
    case B_DIV:
      if (y == 0) { dz = true; return 0; }
      if (y == -1) return (int32_t)(0u - ux);
      return x / y;
    case B_REM:
      if (y == 0) { dz = true; return 0; }
      if (y == -1) return 0;
      return x % y;
    case B_MOD: {
      // a positive power of two: the result in [0, y) is the low bits of x
      // in two's complement (no division)
      if (y > 0 && (uy & (uy - 1u)) == 0u) return (int32_t)(ux & (uy - 1u));
      if (y == 0) { dz = true; return 0; }
      if (y == -1 || y == 1) return 0;
      int32_t r = x % y;
      if (r < 0) r = (int32_t)((uint32_t)r + (y < 0 ? 0u - uy : uy));
      return r;
    }
    case B_AND: return x & y;
    case B_OR: return x | y;
    case B_XOR: return x ^ y;
    case B_SHL: return (int32_t)(ux << (uy & 31u));
    case B_SHR: return x >> (int32_t)(uy & 31u);
    case B_LT: return x < y;
    case B_LE: return x <= y;
    case B_GT: return x > y;
    case B_GE: return x >= y;
    case B_EQ: return x == y;
    case B_NE: return x != y;
    case B_LAND: return (x != 0) & (y != 0);
    case B_LOR: return (x != 0) | (y != 0);
    case B_MIN: return x < y ? x : y;
    default: return x > y ? x : y;   // B_MAX
  }
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Reads through the constant address space: with a uniform index these are
// scalar loads (the code and descriptor tables are never written by kernels).
struct Insn {
  uint32_t h, a, b, c;
};
template <typename T>
__device__ __forceinline__ T const_load(const void* base, uint32_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) T*)base)[i];
#else
  return ((const T*)base)[i];   // the host pass only parses device code
#endif
}

// An array's descriptor.  A per-program kernel defines RC_JIT_ARRAYS and
// jit_array(), which sets the fields fixed by the program and its launch
// shape to constants the compiler folds (run_items checks them against the
// descriptors it runs on).
__device__ __forceinline__ ArrayDesc array_desc(const ArrayDesc* arrays, uint32_t a) {
  ArrayDesc A = const_load<ArrayDesc>(arrays, a);
#ifdef RC_JIT_ARRAYS
  jit_array(a, A);
#endif
  return A;
}

// fault key: dynamic statement | lid | pc | priority | code  (smaller = earlier)
// priority orders one item's faults inside a statement: DIV, OOB, the rest.
__device__ __forceinline__ u64 fault_key(uint32_t step, uint32_t lid, uint32_t pc, uint32_t code) {
  uint32_t prio = code == F_DIV ? 0u : (code == F_OOB ? 1u : 2u);
  return ((u64)step << 32) | ((u64)lid << 17) | ((u64)pc << 5) | ((u64)prio << 3) | code;
}

// ---------------------------------------------------------------------------
// interval checks (shared by the interpreter's LDS path and the global pass)
// ---------------------------------------------------------------------------
struct Pair {
  uint32_t a, b;
};
__device__ __forceinline__ void pair_take(Pair& best, uint32_t x, uint32_t y) {
  const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
  if (lo < best.a || (lo == best.a && hi < best.b)) { best.a = lo; best.b = hi; }
}

__device__ __forceinline__ uint32_t pay_lid(u64 p) { return (uint32_t)p & 1023u; }
__device__ __forceinline__ bool pay_w(u64 p) { return ((uint32_t)p >> 10) & 1u; }
__device__ __forceinline__ int32_t pay_val(u64 p) { return (int32_t)(uint32_t)(p >> 32); }

// Both scopes are decided by two passes over a cell's accesses: the first
// finds the smallest reader and the smallest writer (with its smallest
// value), the second finds the partners those need.  Every quantity is a
// minimum or an OR, so a pass can be split over lanes and merged.
constexpr uint32_t NONE32 = 0xFFFFFFFFu;

struct Pass1 {            // r1: smallest reader; wmin: (writer id, value ^ sign) minimum
  uint32_t r1;
  u64 wmin;
};
__device__ __forceinline__ Pass1 pass1_init() { return Pass1{NONE32, ~0ull}; }
__device__ __forceinline__ void pass1_add(Pass1& a, uint32_t id, bool w, int32_t v) {
  if (w) {
    const u64 kx = ((u64)id << 32) | ((uint32_t)v ^ 0x80000000u);
    if (kx < a.wmin) a.wmin = kx;
  } else if (id < a.r1) {
    a.r1 = id;
  }
}

// INTRA (ids are lids of one group): partners of r1 / w1
struct Intra2 {
  uint32_t r2, w2, q, multi1;
};
__device__ __forceinline__ Intra2 intra2_init() { return Intra2{NONE32, NONE32, NONE32, 0u}; }
__device__ __forceinline__ void intra2_add(Intra2& a, uint32_t l, bool w, int32_t v, uint32_t r1, uint32_t w1,
                                           int32_t x1) {
  if (w) {
    if (l == w1) { if (v != x1) a.multi1 = 1u; }
    else {
      if (l < a.w2) a.w2 = l;
      if (v != x1 && l < a.q) a.q = l;
    }
  } else if (l != r1 && l < a.r2) {
    a.r2 = l;
  }
}
__device__ bool intra_finish(const Pass1& p1, const Intra2& p2, uint32_t* label, Pair* rw, Pair* ww) {
  const uint32_t r1 = p1.r1, w1 = p1.wmin == ~0ull ? NONE32 : (uint32_t)(p1.wmin >> 32);
  Pair brw = {NONE32, NONE32}, bww = {NONE32, NONE32};
  const uint32_t rs[2] = {r1, p2.r2}, ws[2] = {w1, p2.w2};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      if (rs[i] != NONE32 && ws[j] != NONE32 && rs[i] != ws[j]) pair_take(brw, rs[i], ws[j]);
  bool wwd = false;
  if (p2.multi1 && p2.w2 != NONE32) { bww = {w1, p2.w2}; wwd = true; }
  else if (p2.q != NONE32) { bww = {w1, p2.q}; wwd = true; }
  uint32_t lab = (brw.a != NONE32 ? 1u : 0u) | (wwd ? 2u : 0u);
  if (lab == 0u) {
    if (p2.w2 == NONE32) return false;   // no eligible pair
    lab = 4u;
    bww = {w1, p2.w2};
  }
  *label = lab;
  *rw = brw;
  *ww = bww;
  return true;
}

// INTRA scope over entries [s, e) of one work-group (ids compared by lid);
// get(i) returns entry i's payload: value << 32 | is_write << 10 | lid.
template <typename Get>
__device__ bool intra_check(Get get, u64 s, u64 e, uint32_t* label, Pair* rw, Pair* ww) {
  Pass1 p1 = pass1_init();
  for (u64 i = s; i < e; ++i) {
    const u64 p = get(i);
    pass1_add(p1, pay_lid(p), pay_w(p), pay_val(p));
  }
  const uint32_t w1 = p1.wmin == ~0ull ? NONE32 : (uint32_t)(p1.wmin >> 32);
  const int32_t x1 = (int32_t)((uint32_t)p1.wmin ^ 0x80000000u);
  Intra2 p2 = intra2_init();
  for (u64 i = s; i < e; ++i) {
    const u64 p = get(i);
    intra2_add(p2, pay_lid(p), pay_w(p), pay_val(p), p1.r1, w1, x1);
  }
  return intra_finish(p1, p2, label, rw, ww);
}

// INTER (ids are global tids; pairs must come from different groups)
struct Inter2 {
  uint32_t r1p, w1p, q, A, multi1;
};
__device__ __forceinline__ Inter2 inter2_init() { return Inter2{NONE32, NONE32, NONE32, NONE32, 0u}; }
__device__ __forceinline__ void inter2_add(Inter2& a, uint32_t t, uint32_t g, bool w, int32_t v, uint32_t gr1,
                                           uint32_t w1, uint32_t g1, int32_t x1) {
  if (w) {
    if (t == w1) { if (v != x1) a.multi1 = 1u; }
    if (g != g1) {
      if (t < a.w1p) a.w1p = t;
      if (v != x1 && t < a.q) a.q = t;
    } else if (t != w1 && v != x1 && t < a.A) {
      a.A = t;
    }
  } else if (g != gr1 && t < a.r1p) {
    a.r1p = t;
  }
}
__device__ bool inter_finish(const Pass1& p1, const Inter2& p2, uint32_t W, uint32_t* label, Pair* rw, Pair* ww) {
  const uint32_t r1 = p1.r1, w1 = p1.wmin == ~0ull ? NONE32 : (uint32_t)(p1.wmin >> 32);
  Pair brw = {NONE32, NONE32}, bww = {NONE32, NONE32};
  const uint32_t rs[2] = {r1, p2.r1p}, ws[2] = {w1, p2.w1p};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      if (rs[i] != NONE32 && ws[j] != NONE32 && rs[i] / W != ws[j] / W) pair_take(brw, rs[i], ws[j]);
  bool wwd = false;
  if (p2.multi1 && p2.w1p != NONE32) { bww = {w1, p2.w1p}; wwd = true; }
  else if (p2.q != NONE32) { bww = {w1, p2.q}; wwd = true; }
  else if (p2.A != NONE32 && p2.w1p != NONE32) {
    bww = {p2.A < p2.w1p ? p2.A : p2.w1p, p2.A < p2.w1p ? p2.w1p : p2.A};
    wwd = true;
  }
  uint32_t lab = (brw.a != NONE32 ? 1u : 0u) | (wwd ? 2u : 0u);
  if (lab == 0u) {
    if (p2.w1p == NONE32) return false;
    lab = 4u;
    bww = {w1, p2.w1p};
  }
  *label = lab;
  *rw = brw;
  *ww = bww;
  return true;
}

// INTER scope over records [s, e) of one cell, all groups (global tids).
__device__ bool inter_check(const u64* keys, const u64* vals, u64 s, u64 e, uint32_t bk, uint32_t gmask,
                            uint32_t W, uint32_t* label, Pair* rw, Pair* ww) {
  Pass1 p1 = pass1_init();
  for (u64 i = s; i < e; ++i) {
    const u64 p = vals[i];
    const uint32_t g = (uint32_t)(keys[i] >> bk) & gmask;
    pass1_add(p1, g * W + pay_lid(p), pay_w(p), pay_val(p));
  }
  const uint32_t w1 = p1.wmin == ~0ull ? NONE32 : (uint32_t)(p1.wmin >> 32);
  const int32_t x1 = (int32_t)((uint32_t)p1.wmin ^ 0x80000000u);
  const uint32_t gr1 = p1.r1 == NONE32 ? NONE32 : p1.r1 / W;
  const uint32_t g1 = w1 == NONE32 ? NONE32 : w1 / W;
  Inter2 p2 = inter2_init();
  for (u64 i = s; i < e; ++i) {
    const u64 p = vals[i];
    const uint32_t g = (uint32_t)(keys[i] >> bk) & gmask;
    inter2_add(p2, g * W + pay_lid(p), g, pay_w(p), pay_val(p), gr1, w1, g1, x1);
  }
  return inter_finish(p1, p2, W, label, rw, ww);
}

struct PendingRec {
  uint32_t gid, interval, aid, cell, cellkey, label, lidbase;
  Pair rw, ww;
};

// canonical sort key fields of a record
struct RecKey {
  uint32_t bs, bc, G, NI;
};

// the record of a finished check and its canonical sort key
__device__ __forceinline__ rc_record_dev make_record(const RecKey& K, uint32_t slot, uint32_t instance,
                                                     const PendingRec& p, bool inter, u64* key) {
  const uint32_t NONE = 0xFFFFFFFFu;
  rc_record_dev r;
  r.instance = instance;
  r.gid = inter ? NONE : p.gid;
  r.interval = inter ? 0u : p.interval;
  r.array_label = p.aid | (p.label << 16);
  r.cell = p.cell;
  r.rw_a = p.rw.a == NONE ? NONE : p.rw.a + p.lidbase;
  r.rw_b = p.rw.b == NONE ? NONE : p.rw.b + p.lidbase;
  r.ww_a = p.ww.a == NONE ? NONE : p.ww.a + p.lidbase;
  r.ww_b = p.ww.b == NONE ? NONE : p.ww.b + p.lidbase;
  r.pad = 0;
  const u64 scope = inter ? (u64)K.G * K.NI : (u64)p.gid * K.NI + p.interval;
  *key = ((u64)slot << (K.bs + K.bc)) | (scope << K.bc) | p.cellkey;
  return r;
}

// Pointers read from descriptors in memory are generic to the compiler; these
// casts let it emit global (not flat) memory instructions, which do not hold
// up waits on LDS.
#if defined(__HIP_DEVICE_COMPILE__)
#define RC_GLOBAL(T, ptr) ((__attribute__((address_space(1))) T*)(ptr))
#else
#define RC_GLOBAL(T, ptr) ((T*)(ptr))   // the host pass only parses device code
#endif

// k: the record's rank among the records of its (group, interval) in
// cell-key order (used by rank keys only)
__device__ __forceinline__ void store_record(const rc_record_out& R, const RecKey& K, u64 pos, uint32_t slot,
                                             uint32_t instance, const PendingRec& p, bool inter, uint32_t k = 0) {
  if (pos >= R.rec_cap) {
    __hip_atomic_fetch_or(RC_GLOBAL(uint32_t, R.status_word), 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const uint32_t NONE = 0xFFFFFFFFu;
  rc_record_dev r;
  r.instance = instance;
  r.gid = inter ? NONE : p.gid;
  r.interval = inter ? 0u : p.interval;
  r.array_label = p.aid | (p.label << 16);
  r.cell = p.cell;
  r.rw_a = p.rw.a == NONE ? NONE : p.rw.a + p.lidbase;
  r.rw_b = p.rw.b == NONE ? NONE : p.rw.b + p.lidbase;
  r.ww_a = p.ww.a == NONE ? NONE : p.ww.a + p.lidbase;
  r.ww_b = p.ww.b == NONE ? NONE : p.ww.b + p.lidbase;
  r.pad = 0;
  RC_GLOBAL(rc_record_dev, R.staging)[pos] = r;
  const u64 scope = inter ? (u64)K.G * K.NI : (u64)p.gid * K.NI + p.interval;
  if (R.rank_keys) {
    RC_GLOBAL(u64, R.rec_keys)[pos] = ((((u64)slot << K.bs) | scope) << 32) | k;
  } else {
    RC_GLOBAL(u64, R.rec_keys)[pos] = ((u64)slot << (K.bs + K.bc)) | (scope << K.bc) | p.cellkey;
    RC_GLOBAL(uint32_t, R.rec_idx)[pos] = (uint32_t)pos;
  }
}

// wave-wide allocation of record slots: one atomic per wave
__device__ __forceinline__ u64 wave_reserve(unsigned long long* counter, uint32_t n, uint32_t lane) {
  u64 base = 0;
  if (lane == 0 && n)
    base = __hip_atomic_fetch_add(RC_GLOBAL(unsigned long long, counter), (unsigned long long)n, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t blo = __builtin_amdgcn_readlane((uint32_t)base, 0);
  const uint32_t bhi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), 0);
  return ((u64)bhi << 32) | blo;
}

extern __shared__ __attribute__((aligned(16))) unsigned char rc_smem[];

// Everything one work item (an instance's work-group) needs; uniform.
struct ItemView {
  const uint32_t* code;
  const ArrayDesc* arrays;
  const ScalarDesc* scalars;
  uint32_t n_arrays, n_global, n_scalars, nregs, G, W, nwaves, lds_local_cells;
  uint32_t lds_log_cap, overlay_cells, NI, bc, bg, bk, bs, do_log;
  uint32_t tab_base, tab_cells;
  u64 log_mask;            // intervals whose local-array accesses are logged (ProgDesc)
  uint32_t log_high;
  u64 wg_log_cap;
  u64* log_keys;
  u64* log_vals;
  uint32_t* status_word;
  const rc_record_out* rec;
  u64* inst_acc;
  uint32_t* inst_intervals;
  u64* inst_fault;
  uint32_t* wg_count;
  u64* wg_base;
  uint32_t* cell_owner;    // see PassParams
  uint32_t co_stride;
  u64* stats;              // see PassParams (may be null)
  uint32_t nf;             // elided group steps (ProgDesc::nf)
  uint32_t step_limit;     // loop iterations the group may start
  uint32_t sc;             // spilled intervals go to the group check (ProgDesc)
};

__device__ __forceinline__ TabCell empty_tab_cell() { return TabCell{~0ull, NONE32, NONE32, NONE32, NONE32}; }

// An LDS log entry on the per-cell table path, one word: bits 0-31 the value,
// 32-41 the local id, 42 the store flag, 43-54 the cell's table index.
__device__ __forceinline__ u64 tab_entry(uint32_t trel, bool store, uint32_t l, int32_t v) {
  return ((u64)trel << 43) | ((u64)(store ? 1u : 0u) << 42) | ((u64)l << 32) | (uint32_t)v;
}

// The record of a table cell, if its accesses form one (labels and pairs
// only; the caller adds the location).  q counts w1 too: w1 wrote a second
// value exactly when q == w1.
__device__ __forceinline__ bool tab_cell_finish(const TabCell c, PendingRec* pr) {
  if (c.wmin == ~0ull && c.r1 == NONE32) return false;
  const uint32_t w1 = c.wmin == ~0ull ? NONE32 : (uint32_t)(c.wmin >> 32);
  const bool multi1 = c.q != NONE32 && c.q == w1;
  const Pass1 p1 = {c.r1, c.wmin};
  const Intra2 p2 = {c.r2, c.w2, multi1 ? NONE32 : c.q, multi1 ? 1u : 0u};
  return intra_finish(p1, p2, &pr->label, &pr->rw, &pr->ww);
}

// Record slots for the whole group: this thread's n records are the
// group's records [k, k + n) (threads in order), and the k-th record of the
// group goes to slot k < room ? at + k : jump + (k - room).  The block takes
// the slots from chunks of REC_CHUNK it reserves with one atomic (not one
// per interval): the rest of the current chunk first, then a new one.  Every
// thread of the block calls it.  (n <= 64; the wave's scan is taken
// bit-plane by bit-plane with ballots.)  Returns k.
__device__ __forceinline__ uint32_t reserve_records(Ctl* ctl, const rc_record_out& R, uint32_t n, uint32_t tl,
                                                    uint32_t nthr, u64* room_out, u64* at_out, u64* jump_out) {
  const uint32_t lane = tl & 63u, wave = tl >> 6;
  const u64 below = (1ull << lane) - 1ull;
  uint32_t x = 0, wsum = 0;   // exclusive prefix in the wave, wave total
#pragma unroll
  for (uint32_t b = 0; b < 7; ++b) {
    const u64 m = __ballot((n >> b) & 1u);
    x += (uint32_t)__popcll(m & below) << b;
    wsum += (uint32_t)__popcll(m) << b;
  }
  if (lane == 0) ctl->rec_sum[wave] = wsum;
  __syncthreads();
  const uint32_t nw = nthr >> 6;
  uint32_t before = 0, total = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    const uint32_t v = ctl->rec_sum[w];
    total += v;
    if (w < wave) before += v;
  }
  if (tl == 0) {
    ctl->rec_sum_total = total;
    const u64 room = ctl->rc_end - ctl->rc_cur;
    ctl->rec_base = ctl->rc_cur;               // records [0, room) go here
    ctl->rc_room = room;
    if (total <= room) {
      ctl->rc_cur += total;
      ctl->rc_next = ctl->rc_end;
    } else {
      const u64 more = total - room;           // and the rest to a new chunk
      const u64 take = more > REC_CHUNK ? more : REC_CHUNK;
      const u64 base = __hip_atomic_fetch_add(RC_GLOBAL(unsigned long long, R.rec_count), (unsigned long long)take,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ctl->rc_next = base;
      ctl->rc_cur = base + more;
      ctl->rc_end = base + take;
    }
  }
  __syncthreads();
  *room_out = ctl->rc_room;
  *at_out = ctl->rec_base;
  *jump_out = ctl->rc_next;
  return before + x;
}

// ---------------------------------------------------------------------------
// A spilled interval of a one-group program, checked by one block of the
// group check kernel.  With one group there is no INTER scope, so the
// interval's accesses, in the group's log region as packed words (cell key,
// store flag, lid, value), need only be grouped by cell.  They are bucketed
// by windows of SC_WIN cells into a second buffer (a count, a scan and a
// scatter, LDS counters), and each bucket is checked through a per-cell
// table over its window in LDS: the two passes of min-reductions as LDS
// atomics, a bitmap of the touched cells, then a pass over the touched
// cells in cell order that emits the records and clears the cells again.
// The table therefore stays clean between buckets and intervals (the block
// clears it once).  Buckets are taken in cell order, so the records leave
// in cell-key order with their ranks, as from the LDS path.  Arguments are
// uniform; every thread of the block calls it.
// ---------------------------------------------------------------------------
struct ScEnv {
  u64* src;              // the interval's m packed entries in the region
  u64* dst;              // the same words of the second log buffer
  uint32_t* ends;        // the block's bucket ends (SC_NB_MAX words)
  uint32_t cells, nthr;
  uint32_t slot, instance, interval, n_arrays;
  const ArrayDesc* arrays;
  const rc_record_out* recp;
  RecKey K;
  // LDS: the window table, one array per field of a cell (consecutive
  // cells in consecutive banks), clean; the bitmap, zero
  u64* wmin;
  uint32_t *r1, *r2, *w2, *q;
  uint32_t* bits;        // SC_WORDS words
  uint32_t* cnt;         // LDS: SC_NB_MAX bucket counters
};

__device__ __forceinline__ uint32_t sc_aid(const ScEnv& E, uint32_t ck) {
  uint32_t aid = 0;
  for (uint32_t a = 0; a < E.n_arrays; ++a) {
    const ArrayDesc D = const_load<ArrayDesc>(E.arrays, a);
    if (D.logged == LOG_LDS && ck >= D.cellbase && ck - D.cellbase < D.size) aid = a;
  }
  return aid;
}

// f(e) for every entry e of in[0, n), in rounds of four loads per thread
// (issued together: the passes are bound by memory latency)
template <typename F>
__device__ __forceinline__ void sc_each(const u64* in, u64 n, uint32_t nthr, F f) {
  for (u64 i0 = threadIdx.x; i0 < n; i0 += 4u * (u64)nthr) {
    u64 e[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const u64 i = i0 + (u64)k * nthr;
      ok[k] = i < n;
      e[k] = ok[k] ? in[i] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (ok[k]) f(e[k]);
  }
}

// Bucket in[0, n) by window (cell key >> SC_WIN_BITS) into out, nb
// buckets; E.ends[b] = end of bucket b in out.
__device__ void sc_bucket(const ScEnv& E, const u64* in, u64* out, u64 n, uint32_t nb) {
  const uint32_t tl = threadIdx.x, lane = tl & 63u;
  uint32_t* cnt = E.cnt;
  for (uint32_t i = tl; i < nb; i += E.nthr) cnt[i] = 0u;
  __syncthreads();
  sc_each(in, n, E.nthr, [&](u64 e) { atomicAdd(&cnt[(uint32_t)(e >> 43) >> SC_WIN_BITS], 1u); });
  __syncthreads();
  if (tl < 64u) {   // exclusive scan: lane l takes a contiguous run of counters
    const uint32_t per = (nb + 63u) / 64u, lo = lane * per, hi = lo + per < nb ? lo + per : nb;
    uint32_t sum = 0;
    for (uint32_t j = lo; j < hi; ++j) sum += cnt[j];
    uint32_t run = sum;
    for (uint32_t off = 1; off < 64u; off <<= 1) {
      const uint32_t o = __shfl_up(run, off);
      if (lane >= off) run += o;
    }
    run -= sum;
    for (uint32_t j = lo; j < hi; ++j) {
      const uint32_t c = cnt[j];
      cnt[j] = run;
      run += c;
    }
  }
  __syncthreads();
  sc_each(in, n, E.nthr, [&](u64 e) { out[atomicAdd(&cnt[(uint32_t)(e >> 43) >> SC_WIN_BITS], 1u)] = e; });
  __syncthreads();
  for (uint32_t i = tl; i < nb; i += E.nthr) E.ends[i] = cnt[i];
  // the bucket contents and bounds are read back by other threads of the block
  __threadfence();
  __syncthreads();
}

// Check bucket in[0, n) (cell keys base .. base + SC_WIN - 1) through the
// table; kb = records of the interval so far; returns the new count.  A
// bucket of at least SC_SCAN_MIN entries finishes every cell of the window
// (each thread SC_WIN / nthr consecutive ones); a smaller one finishes the
// cells its bitmap marks (set by the first reader and the first writer of
// each cell).
constexpr uint32_t SC_SCAN_MIN = 256;
__device__ __forceinline__ bool sc_touched(const ScEnv& E, uint32_t c) {
  return E.wmin[c] != ~0ull || E.r1[c] != NONE32;
}
__device__ __forceinline__ TabCell sc_cell(const ScEnv& E, uint32_t c) {
  return TabCell{E.wmin[c], E.r1[c], E.r2[c], E.w2[c], E.q[c]};
}
__device__ __forceinline__ void sc_clear(const ScEnv& E, uint32_t c) {
  E.wmin[c] = ~0ull;
  E.r1[c] = E.r2[c] = E.w2[c] = E.q[c] = NONE32;
}

__device__ uint32_t sc_window(const ScEnv& E, const u64* in, uint32_t n, uint32_t base, uint32_t kb) {
  const uint32_t tl = threadIdx.x;
  Ctl* ctl = reinterpret_cast<Ctl*>(rc_smem);
  const bool scan = n >= SC_SCAN_MIN;
  // Every field only decreases, so an entry whose value is not below the
  // field's current one (a read that may be stale, never below the true
  // value) needs no atomic: a cell that every work-item touches sees few
  // atomics instead of one per lane.  (A cell already touched is not the
  // first touch, so skipping leaves the bitmap right.)
  sc_each(in, n, E.nthr, [&](u64 e) {
    const uint32_t c = (uint32_t)(e >> 43) - base;
    const uint32_t l = (uint32_t)(e >> 32) & 1023u;
    bool first = false;
    if ((e >> 42) & 1u) {
      const u64 v = ((u64)l << 32) | ((uint32_t)e ^ 0x80000000u);
      if (E.wmin[c] > v) first = atomicMin(&E.wmin[c], v) == ~0ull;
    } else if (E.r1[c] > l) {
      first = atomicMin(&E.r1[c], l) == NONE32;
    }
    if (!scan && first) atomicOr(&E.bits[c >> 5], 1u << (c & 31u));
  });
  __syncthreads();
  sc_each(in, n, E.nthr, [&](u64 e) {
    const uint32_t c = (uint32_t)(e >> 43) - base;
    const uint32_t l = (uint32_t)(e >> 32) & 1023u;
    if ((e >> 42) & 1u) {
      const u64 wmin = E.wmin[c];
      if ((uint32_t)e != ((uint32_t)wmin ^ 0x80000000u) && E.q[c] > l) atomicMin(&E.q[c], l);
      if (l != (uint32_t)(wmin >> 32) && E.w2[c] > l) atomicMin(&E.w2[c], l);
    } else if (l != E.r1[c] && E.r2[c] > l) {
      atomicMin(&E.r2[c], l);
    }
  });
  __syncthreads();
  // the cells this thread finishes, in cell order: a count, the group's
  // reservation, then the records; every touched cell is cleared again
  const uint32_t per = SC_WIN / E.nthr;
  const uint32_t c0 = tl * per;
  const uint32_t word = !scan && tl < SC_WORDS ? E.bits[tl] : 0u;
  uint32_t mine = 0;
  if (scan) {
    for (uint32_t c = c0; c < c0 + per; ++c) {
      if (!sc_touched(E, c)) continue;
      PendingRec pr;
      if (tab_cell_finish(sc_cell(E, c), &pr)) ++mine;
    }
  } else {
    for (uint32_t m = word; m; m &= m - 1u) {
      PendingRec pr;
      if (tab_cell_finish(sc_cell(E, tl * 32u + (uint32_t)__ffs(m) - 1u), &pr)) ++mine;
    }
  }
  const rc_record_out R = const_load<rc_record_out>(E.recp, 0);
  u64 room, at0, jump;
  uint32_t k = reserve_records(ctl, R, mine, tl, E.nthr, &room, &at0, &jump);
  auto emit = [&](uint32_t c) {
    const TabCell t = sc_cell(E, c);
    sc_clear(E, c);
    PendingRec pr;
    if (!tab_cell_finish(t, &pr)) return;
    const uint32_t ck = base + c;
    const uint32_t aid = sc_aid(E, ck);
    pr.gid = 0; pr.interval = E.interval; pr.aid = aid;
    pr.cell = ck - const_load<ArrayDesc>(E.arrays, aid).cellbase;
    pr.cellkey = ck; pr.lidbase = 0;
    store_record(R, E.K, k < room ? at0 + k : jump + (k - room), E.slot, E.instance, pr, false, kb + k);
    ++k;
  };
  const uint32_t total = ctl->rec_sum_total;
  if (scan) {
    for (uint32_t c = c0; c < c0 + per; ++c)
      if (sc_touched(E, c)) emit(c);
  } else {
    for (uint32_t m = word; m; m &= m - 1u) emit(tl * 32u + (uint32_t)__ffs(m) - 1u);
    if (tl < SC_WORDS) E.bits[tl] = 0u;
  }
  __syncthreads();   // the table is clean again
  return kb + total;
}

__device__ __forceinline__ uint32_t sc_check(const ScEnv& E, u64 m) {
  const uint32_t nb = (E.cells + SC_WIN - 1u) >> SC_WIN_BITS;
  sc_bucket(E, E.src, E.dst, m, nb);
  uint32_t kb = 0, s = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    const uint32_t e = uni(E.ends[b]);
    if (e - s >= 2u) kb = sc_window(E, E.dst + s, e - s, b << SC_WIN_BITS, kb);
    s = e;
  }
  return kb;
}

// The state of one item on its workgroup (uniform values in scalars, per-lane
// values in vector registers) and the statement semantics of paper Section 4
// as run lockstep: every method is called by every thread of the workgroup
// at the same point of the program.
struct Item {
  ItemView P;
  Ctl* ctl;
  uint32_t slot, instance, gid, epoch_base, wg_index;
  uint64_t seed;
  u64 log_base;
  u64* ovl;
  uint32_t tl, WP, wave, lane, tr;
  uint32_t nthr;           // threads of the block (64 << width class)
  u64 rec_at, rec_jump, rec_room;   // the last record reservation (see group_reserve)
  bool real;
  u64* locc;
  u64* lkey;
  uint32_t* lmeta;
  int32_t* lval;
  int32_t* regs;
  TabCell* tab;
  u64 key_slot;
  u64 log_used;
  uint32_t lds_used;       // entries of the current interval in the LDS log
  bool lds_spilled;        // the current interval moved to the global log
  uint32_t step, last_spc, store_seq, interval, parity, n_acc;
  uint32_t iters;          // loop iterations the group started (uniform)
  uint32_t n_logged;       // this work-item's logged accesses
  uint32_t n_spilled;      // intervals of the group whose log moved to the global log
  uint32_t n_insn;         // instructions the group executed (uniform)
  u64 n_glog;              // entries of spilled intervals (one-group programs: trailers not counted)
  u64 ival_base;           // (one-group programs) region word where the current spilled interval starts
  u64 my_fault;            // earliest fault of this work-item (fault_key order)
  bool faulted;

  // `slot` indexes the chunk's per-instance counters, `instance` the call's.
  __device__ __forceinline__ void init(const ItemView& view, Ctl* c, uint32_t slot_, uint32_t instance_,
                                       uint32_t gid_, uint64_t seed_, u64 log_base_, u64* ovl_,
                                       uint32_t epoch_base_, uint32_t wg_index_, uint32_t nthr_) {
    P = view;
    ctl = c;
    slot = slot_; instance = instance_; gid = gid_; seed = seed_; log_base = log_base_; ovl = ovl_;
    epoch_base = epoch_base_; wg_index = wg_index_;
    tl = threadIdx.x;
    // (a launch parameter, not blockDim.x: reading the block size takes a
    // vector memory load on this target)
    nthr = nthr_;
    WP = P.nwaves * 64u;
    wave = tl >> 6;
    lane = tl & 63u;
    real = tl < P.W;
    tr = tl < WP ? tl : WP - 1u;   // waves past the group read a real lane's registers
    // dynamic LDS after the control block: local array cells (u64), the
    // interval log (T packed words with the table; else T keys, T payload
    // words, T values), registers, table
    locc = reinterpret_cast<u64*>(reinterpret_cast<unsigned char*>(ctl) + ((sizeof(Ctl) + 15) & ~(size_t)15));
    lkey = locc + P.lds_local_cells;
    if (P.tab_cells) {
      lmeta = nullptr;
      lval = nullptr;
      regs = reinterpret_cast<int32_t*>(lkey + P.lds_log_cap);
    } else {
      lmeta = reinterpret_cast<uint32_t*>(lkey + P.lds_log_cap);
      lval = reinterpret_cast<int32_t*>(lmeta + P.lds_log_cap);
      regs = lval + P.lds_log_cap;
    }
    // the per-cell check table (8-byte aligned after the registers)
    // (offset arithmetic from the LDS base, so that the compiler still sees
    // an LDS pointer and emits LDS atomics on the table)
    unsigned char* const lds0 = reinterpret_cast<unsigned char*>(ctl);
    const size_t toff = ((size_t)(reinterpret_cast<unsigned char*>(regs + P.nregs * WP) - lds0) + 7u) & ~(size_t)7u;
    tab = reinterpret_cast<TabCell*>(lds0 + toff);
    const TabCell empty_cell = empty_tab_cell();
    for (uint32_t i = tl; i < P.lds_local_cells; i += nthr) locc[i] = 0ull;
    for (uint32_t i = tl; i < P.nregs * WP; i += nthr) regs[i] = 0;
    for (uint32_t i = tl; i < P.tab_cells; i += nthr) tab[i] = empty_cell;
    if (tl == 0) {
      ctl->fault = ~0ull;
      ctl->lds_cnt[0] = ctl->lds_cnt[1] = 0u;
      ctl->gl_cnt = 0ull;
    }
    if (tl < P.n_scalars) {
      const ScalarDesc S = const_load<ScalarDesc>(P.scalars, tl);
      ctl->uval[SEL_SCALAR0 - SEL_LID + tl] =
          S.bind == BIND_SEEDED ? seeded_cell(seed, 0x10000u + tl, 0, S.lo, S.hi) : S.value;
    }
    if (tl == 0) {
      ctl->uval[SEL_LID - SEL_LID] = 0;
      ctl->uval[SEL_TID - SEL_LID] = (int32_t)(gid * P.W);
      ctl->uval[SEL_GID - SEL_LID] = (int32_t)gid;
      ctl->uval[SEL_WGSIZE - SEL_LID] = (int32_t)P.W;
      ctl->uval[SEL_NGROUPS - SEL_LID] = (int32_t)P.G;
      ctl->uval[SEL_NTHREADS - SEL_LID] = (int32_t)(P.G * P.W);
    }
    __syncthreads();
    key_slot = (u64)slot << (P.bc + P.bg + P.bk);
    log_used = 0;
    lds_used = 0;
    lds_spilled = false;
    step = 0; last_spc = ~0u; store_seq = 0; interval = 0; parity = 0; n_acc = 0;
    n_logged = 0; n_spilled = 0; iters = 0; n_insn = 0; n_glog = 0; ival_base = 0;
    my_fault = ~0ull;
    faulted = false;
  }

  // statements are numbered by execution: a new statement pc starts a new step
  __device__ __forceinline__ void stmt(uint32_t spc) {
    ++n_insn;
    if (spc != last_spc) { ++step; last_spc = spc; }
  }

  // A loop iteration starts (every thread, at the same point): true when
  // the group has started more than its limit, a fault of the whole group
  // (reported for its first work-item; every wave stops here).
  __device__ __forceinline__ bool iter_start(uint32_t spc) {
    if (++iters <= P.step_limit) return false;
    raise(spc, F_STEP_LIMIT);
    return true;
  }

  // lid, tid, gid, wgsize, ngroups, nthreads, scalar parameters
  __device__ __forceinline__ int32_t special(uint32_t w) const {
    switch (w) {
      case SEL_LID: return (int32_t)tl;
      case SEL_TID: return (int32_t)(gid * P.W + tl);
      case SEL_GID: return (int32_t)gid;
      case SEL_WGSIZE: return (int32_t)P.W;
      case SEL_NGROUPS: return (int32_t)P.G;
      case SEL_NTHREADS: return (int32_t)(P.G * P.W);
      default: return ctl->uval[w - SEL_LID];
    }
  }
  // the same for a selector known only at run time (the interpreter): one
  // LDS read and no branch
  __device__ __forceinline__ int32_t special_dyn(uint32_t w) const {
    const uint32_t k = w - SEL_LID;
    return (int32_t)((uint32_t)ctl->uval[k] + (k < 2u ? tl : 0u));
  }

  // Group-wide OR of two per-lane predicates (bits 0, 1) and of "some
  // work-item has a pending fault" (bit 2).  Every wave publishes its word
  // before the barrier and reads all words after it, so all waves decide on
  // the same snapshot.  The words are double-buffered: a wave can only reuse
  // a buffer after the next reduction's barrier, which every reader passes
  // after reading.
  __device__ __forceinline__ uint32_t group_red(bool p0, bool p1, bool sync_always) {
    const u64 b0 = __ballot(p0), b1 = __ballot(p1), bf = __ballot(fault_pending());
    const uint32_t mine = (b0 != 0ull ? 1u : 0u) | (b1 != 0ull ? 2u : 0u) | (bf != 0ull ? 4u : 0u);
    if (P.nwaves == 1) {
      if (sync_always) __syncthreads();
      return uni(mine);
    }
    if (lane == 0) ctl->red[parity][wave] = mine;
    __syncthreads();
    // lane w reads wave w's word: one LDS round trip whatever the width
    const uint32_t x = lane < P.nwaves ? ctl->red[parity][lane] : 0u;
    parity ^= 1u;
#ifdef RC_JIT_NOFAULT
    return (__ballot(x & 1u) != 0ull ? 1u : 0u) | (__ballot(x & 2u) != 0ull ? 2u : 0u);
#else
    return (__ballot(x & 1u) != 0ull ? 1u : 0u) | (__ballot(x & 2u) != 0ull ? 2u : 0u) |
           (__ballot(x & 4u) != 0ull ? 4u : 0u);
#endif
  }

  // The same snapshot reduction for a memory statement: bit 0 of each wave's
  // word is its pending-fault flag, bits 8.. its count of log entries; every
  // wave gets the group total and the count of the waves before it.
  __device__ __forceinline__ bool mem_red(bool rec, u64* brec, uint32_t* prefix, uint32_t* total) {
    const u64 br = __ballot(rec), bf = __ballot(fault_pending());
    *brec = br;
    const uint32_t cnt = (uint32_t)__popcll(br);
    if (P.nwaves == 1) {
      __syncthreads();
      *prefix = 0u;
      *total = uni(cnt);
      return bf != 0ull;
    }
    if (lane == 0) ctl->red[parity][wave] = (bf != 0ull ? 1u : 0u) | (cnt << 8);
    __syncthreads();
    // lane w reads wave w's word; the counts (at most 64: 7 bits) are summed
    // bit-plane by bit-plane with ballots, over all waves and over the waves
    // before this one
    const uint32_t x = lane < P.nwaves ? ctl->red[parity][lane] : 0u;
    parity ^= 1u;
    // inclusive scan of the counts over lanes 0..15 (one DPP row): lane w
    // then holds the entries of waves 0..w
    uint32_t c = x >> 8;
    c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x111, 0xf, 0xf, true);   // row_shr:1
    c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x112, 0xf, 0xf, true);   // row_shr:2
    c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x114, 0xf, 0xf, true);   // row_shr:4
    c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x118, 0xf, 0xf, true);   // row_shr:8
    *total = (uint32_t)__builtin_amdgcn_readlane((int)c, 15);
    *prefix = wave == 0 ? 0u : (uint32_t)__builtin_amdgcn_readlane((int)c, (int)(wave < 16u ? wave - 1u : 15u));
    return __ballot(x & 1u) != 0ull;
  }

  // A per-program kernel of a program proven never to fault (RC_JIT_NOFAULT)
  // has no fault to agree on: a fault there means the proof is wrong, and
  // it is reported as a library error (status bit 4) instead.
  __device__ __forceinline__ bool fault_pending() const {
#ifdef RC_JIT_NOFAULT
    return false;
#else
    return my_fault != ~0ull;
#endif
  }
  __device__ __forceinline__ void raise(uint32_t spc, uint32_t code) {
#ifdef RC_JIT_NOFAULT
    (void)spc;
    (void)code;
    atomicOr(P.status_word, 16u);
#else
    if (P.nf) {   // proven not to fault: a fault means the proof is wrong
      atomicOr(P.status_word, 16u);
      return;
    }
    const u64 k = fault_key(step, tl, spc, code);
    if (k < my_fault) my_fault = k;
#endif
  }

  // The record of a table cell, if its accesses form one (labels and pairs
  // only; the caller adds the location).
  __device__ __forceinline__ static bool tab_finish(const TabCell c, PendingRec* pr) {
    return tab_cell_finish(c, pr);
  }

  // Record slots for the whole group (reserve_records): this thread's n
  // records (n <= 64: a thread finishes at most 4096 / 64 cells) are the
  // group's records [k, k + n), the k-th going to slot_of(k).
  __device__ __forceinline__ uint32_t group_reserve(const rc_record_out& R, uint32_t n) {
    return reserve_records(ctl, R, n, tl, nthr, &rec_room, &rec_at, &rec_jump);
  }
  // the slot of the group's k-th record of the last reservation
  __device__ __forceinline__ u64 slot_of(uint32_t k) const {
    return k < rec_room ? rec_at + k : rec_jump + (k - rec_room);
  }

  // One entry at position pos of the group's global log region: key and
  // payload words (with the owner word when filtering), or for a group that
  // checks its spilled intervals itself (P.sc) one packed word.
  __device__ __forceinline__ void glog_put(u64 pos, u64 ck, uint32_t meta, uint32_t v) {
    if (pos >= P.wg_log_cap) {
      atomicOr(P.status_word, 1u);
      return;
    }
    if (P.sc) {
      P.log_keys[log_base + pos] = tab_entry((uint32_t)ck, (meta & 1024u) != 0u, meta & 1023u, (int32_t)v);
      return;
    }
    P.log_keys[log_base + pos] = key_slot | (((ck << P.bg) | gid) << P.bk) | interval;
    P.log_vals[log_base + pos] = ((u64)v << 32) | meta;
    if (P.cell_owner) P.cell_owner[(u64)slot * P.co_stride + ck] = (gid << 10) | (meta & 1023u);
  }

  // Move LDS log entries [0, count) of the current interval to the group's
  // global log (elided group steps; every thread has passed a barrier since
  // the interval's last access).
  __device__ __forceinline__ void spill_nf(uint32_t count) {
    const u64 base = ((u64)uni((uint32_t)(ctl->gl_cnt >> 32)) << 32) | uni((uint32_t)ctl->gl_cnt);
    __syncthreads();
    if (tl == 0) ctl->gl_cnt = base + count;
    for (uint32_t i = tl; i < count; i += nthr) {
      const u64 pos = base + i;
      const u64 e = lkey[i];
      u64 ck;
      uint32_t meta, v;
      if (P.tab_cells) {
        ck = P.tab_base + (e >> 43);
        meta = (uint32_t)(e >> 32) & 2047u;   // store flag (bit 10) and local id
        v = (uint32_t)e;
      } else {
        ck = e >> 16;
        meta = lmeta[i];
        v = (uint32_t)lval[i];
      }
      glog_put(pos, ck, meta, v);
    }
    __syncthreads();
  }

  // A spilled interval of a one-group program closes: a trailer word after
  // its entries in the group's region, (interval << 32) | entry count,
  // lets the group check kernel find it (sc_group_kernel walks the
  // trailers back from the region's end).  end: the region's words so far.
  __device__ __forceinline__ u64 spill_trailer(u64 end) {
    const u64 count = end - ival_base;
    if (tl == 0) {
      if (end < P.wg_log_cap) P.log_keys[log_base + end] = ((u64)interval << 32) | count;
      else atomicOr(P.status_word, 1u);
    }
    n_glog += count;
    ival_base = end + 1u;
    return end + 1u;
  }

  // Close the current interval on the LDS path: check its log in LDS (by a
  // per-cell table, or by a bitonic sort and runs) and stage the records of
  // the INTRA scope.  Callers have passed a barrier since the interval's last
  // access.
  __device__ __forceinline__ void close_interval() {
#ifdef RC_JIT_ELIDE
    // the interval's entries, from its LDS counter; the next interval's
    // counter was last read at the previous close, before the barrier
    // every thread passed to get here
    const uint32_t n = uni(ctl->lds_cnt[interval & 1u]);
    if (tl == 0) ctl->lds_cnt[(interval + 1u) & 1u] = 0u;
    __syncthreads();
#else
    uint32_t n = lds_used;
    if (P.nf) {
      // elided group steps: the entries from the interval's LDS counter (the
      // next interval's counter was last read at the previous close, before
      // the barrier every thread passed to get here); an interval that
      // outgrew the LDS log moves what it holds to the global log, beside
      // its other entries
      n = uni(ctl->lds_cnt[interval & 1u]);
      if (tl == 0) ctl->lds_cnt[(interval + 1u) & 1u] = 0u;
      __syncthreads();
      if (n > P.lds_log_cap) {
        spill_nf(P.lds_log_cap);
        ++n_spilled;
        if (P.sc) {
          const u64 end = ((u64)uni((uint32_t)(ctl->gl_cnt >> 32)) << 32) | uni((uint32_t)ctl->gl_cnt);
          const u64 next = spill_trailer(end);
          if (tl == 0) ctl->gl_cnt = next;
          __syncthreads();
        }
        return;
      }
    }
#endif
  const bool spilled = lds_spilled;
  lds_used = 0;
  lds_spilled = false;
#ifndef RC_JIT_NOSPILL
  if (spilled && P.sc) {
    log_used = spill_trailer(log_used);
    return;
  }
#endif
  if (spilled || n < 2u) return;
  const rc_record_out R = const_load<rc_record_out>(P.rec, 0);
  const RecKey K = {P.bs, P.bc, P.G, P.NI};
  if (P.tab_cells) {
    // Per-cell table: the two passes of intra_check merged with LDS atomics,
    // then one pass over the table finishes every touched cell and clears it
    // for the next interval.  q counts w1 too: w1 wrote a second value
    // exactly when q == w1.
    for (uint32_t i = tl; i < n; i += nthr) {
      const u64 e = lkey[i];
      TabCell& c = tab[(uint32_t)(e >> 43)];
      const uint32_t l = (uint32_t)(e >> 32) & 1023u;
      // (fields only decrease: an entry not below the current value needs
      // no atomic)
      if ((e >> 42) & 1u) {
        const u64 v = ((u64)l << 32) | ((uint32_t)e ^ 0x80000000u);
        if (c.wmin > v) atomicMin(&c.wmin, v);
      } else if (c.r1 > l) {
        atomicMin(&c.r1, l);
      }
    }
    __syncthreads();
    for (uint32_t i = tl; i < n; i += nthr) {
      const u64 e = lkey[i];
      TabCell& c = tab[(uint32_t)(e >> 43)];
      const uint32_t l = (uint32_t)(e >> 32) & 1023u;
      if ((e >> 42) & 1u) {
        const u64 wmin = c.wmin;
        const uint32_t w1 = (uint32_t)(wmin >> 32);
        if ((uint32_t)e != ((uint32_t)wmin ^ 0x80000000u) && c.q > l) atomicMin(&c.q, l);
        if (l != w1 && c.w2 > l) atomicMin(&c.w2, l);
      } else if (l != c.r1 && c.r2 > l) {
        atomicMin(&c.r2, l);
      }
    }
    __syncthreads();
    // Each thread finishes a run of consecutive cells (so the records leave
    // in cell-key order): a first pass counts its records, the group
    // reserves them with one atomic, a second pass stores them and clears
    // the cells for the next interval.
    // Cells without a record are cleared in the first pass; the second runs
    // only when the group has records.
    const uint32_t per = (P.tab_cells + nthr - 1u) / nthr;
    const uint32_t t0 = tl * per, t1 = min(t0 + per, P.tab_cells);
    uint32_t mine = 0;
    for (uint32_t t = t0; t < t1; ++t) {
      const TabCell c = tab[t];
      if (c.wmin == ~0ull && c.r1 == NONE32) continue;
      PendingRec pr;
      if (tab_finish(c, &pr)) ++mine;
      else tab[t] = empty_tab_cell();
    }
    uint32_t at = group_reserve(R, mine);
    const uint32_t total = ctl->rec_sum_total;
    if (total == 0u) {
      __syncthreads();
      return;
    }
    if (R.rank_keys && tl == 0)
      RC_GLOBAL(uint32_t, R.scope_cnt)[((u64)slot << K.bs) | ((u64)gid * K.NI + interval)] = total;
    for (uint32_t t = t0; t < t1; ++t) {
      const TabCell c = tab[t];
      if (c.wmin == ~0ull && c.r1 == NONE32) continue;
      tab[t] = empty_tab_cell();
      PendingRec pr;
      if (!tab_finish(c, &pr)) continue;
      const uint32_t ck = P.tab_base + t;
      uint32_t aid = 0;
      for (uint32_t a = 0; a < P.n_arrays; ++a) {
        const ArrayDesc D = array_desc(P.arrays, a);
        if (D.logged == LOG_LDS && ck >= D.cellbase && ck - D.cellbase < D.size) aid = a;
      }
      const ArrayDesc D = array_desc(P.arrays, aid);
      pr.gid = gid; pr.interval = interval; pr.aid = aid; pr.cell = ck - D.cellbase;
      pr.cellkey = ck; pr.lidbase = gid * P.W;
      store_record(R, K, slot_of(at), slot, instance, pr, false, at);
      ++at;
    }
    __syncthreads();
    return;
  }
  uint32_t P2 = 2;
  while (P2 < n) P2 <<= 1;
  for (uint32_t i = n + tl; i < P2; i += nthr) lkey[i] = ~0ull;
  __syncthreads();
  for (uint32_t k = 2; k <= P2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tl; i < P2; i += nthr) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const u64 a = lkey[i], b = lkey[ixj];
          if ((a > b) == ((i & k) == 0u)) { lkey[i] = b; lkey[ixj] = a; }
        }
      }
      __syncthreads();
    }
  }
  uint32_t kbase = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += nthr) {
    const uint32_t i = b0 + tl;
    bool has = false;
    PendingRec pr;
    if (i < n) {
      const u64 ck = lkey[i] >> 16;
      if (i == 0 || (lkey[i - 1] >> 16) != ck) {
        uint32_t e = i + 1;
        while (e < n && (lkey[e] >> 16) == ck) ++e;
        if (e - i >= 2u) {
          has = intra_check([&](u64 q) {
                              const uint32_t ix = (uint32_t)lkey[q] & 0xFFFFu;
                              return ((u64)(uint32_t)lval[ix] << 32) | lmeta[ix];
                            }, i, e, &pr.label, &pr.rw, &pr.ww);
          if (has) {
            uint32_t aid = 0;
            for (uint32_t a = 0; a < P.n_arrays; ++a) {
              const ArrayDesc D = array_desc(P.arrays, a);
              if (D.logged == LOG_LDS && ck >= D.cellbase && ck - D.cellbase < D.size) aid = a;
            }
            const ArrayDesc D = array_desc(P.arrays, aid);
            pr.gid = gid; pr.interval = interval; pr.aid = aid; pr.cell = (uint32_t)ck - D.cellbase;
            pr.cellkey = (uint32_t)ck; pr.lidbase = gid * P.W;
          }
        }
      }
    }
    // the round's records in entry (cell-key) order, after the earlier
    // rounds' (kbase)
    const uint32_t at = group_reserve(R, has ? 1u : 0u);
    const uint32_t got = ctl->rec_sum_total;
    if (has) store_record(R, K, slot_of(at), slot, instance, pr, false, kbase + at);
    kbase += got;
  }
  if (R.rank_keys && tl == 0 && kbase)
    RC_GLOBAL(uint32_t, R.scope_cnt)[((u64)slot << K.bs) | ((u64)gid * K.NI + interval)] = kbase;
  __syncthreads();
  }

  // The access itself: a load reads the group's view of the cell (LDS for a
  // local array; for a global array its overlay word when this chunk wrote
  // it, else the input); a store applies with the highest work-item's value
  // staying within one statement (version words compared by atomicMax).
  __device__ __forceinline__ void access(uint32_t op, uint32_t wc, const ArrayDesc& A, int32_t idx, int32_t val,
                                         bool active, int32_t& out) {
    const uint32_t cell = (uint32_t)idx;
    // overlay word of the cell: by cell, or for an owned array by (offset
    // from the work-item's stride, lid), which keeps a wave's words together
    uint32_t word_at = A.offset + cell;
    bool placed = true;
    if (A.kind == AK_GLOBAL_RW && A.own_stride != 0 && active) {
      // (mod 2^32, as the index arithmetic itself)
      const uint32_t o = (uint32_t)idx - (uint32_t)A.own_stride * (gid * P.W + tl) - (uint32_t)A.own_lo;
      placed = o < A.own_span;
      word_at = A.offset + o * P.W + tl;
      if (!placed) atomicOr(P.status_word, 4u);   // the ownership proof does not hold
    }
    if (op == OP_LOAD) {
      if (active) {
        int32_t v;
        if (A.kind == AK_LOCAL) {
          v = (int32_t)(uint32_t)locc[A.offset + cell];
        } else {
          bool have = false;
          v = 0;
          if (A.kind == AK_GLOBAL_RW && placed) {
            u64 w = __hip_atomic_load(&ovl[word_at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(w >> 42) >= epoch_base) { v = (int32_t)(uint32_t)w; have = true; }
          }
          if (!have)
            v = A.bind == BIND_SEEDED ? seeded_cell(seed, wc, cell, A.lo, A.hi) : A.dptr[cell];
        }
        out = v;
        ++n_acc;
      }
    } else {
      ++store_seq;
      if (active) {
        // within one statement the highest work-item's value stays
        const uint32_t ep = A.kind == AK_LOCAL ? store_seq : epoch_base + store_seq;
        const u64 word = ((u64)((ep << 10) | tl) << 32) | (uint32_t)val;
        if (A.kind == AK_LOCAL) atomicMax(&locc[A.offset + cell], word);
        else if (A.own_stride != 0) {   // no other work-item has this word
          if (placed) __hip_atomic_store(&ovl[word_at], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        else atomicMax(&ovl[A.offset + cell], word);
        ++n_acc;
      }
    }
  }

  // Append this lane's entry (when rec) to the global log at a position
  // reserved with one LDS atomic per wave; lanes in `mask` take part.
  __device__ __forceinline__ void glog_append(u64 mask, bool mine, u64 ck, uint32_t meta, int32_t v) {
    if (mask == 0ull) return;
    u64 base = 0;
    if (lane == 0) base = atomicAdd(&ctl->gl_cnt, (u64)__popcll(mask));
    base = ((u64)(uint32_t)__shfl((int)(base >> 32), 0) << 32) | (uint32_t)__shfl((int)(uint32_t)base, 0);
    if (!mine) return;
    const u64 pos = base + (u64)__popcll(mask & ((1ull << lane) - 1ull));
    glog_put(pos, ck, meta, (uint32_t)v);
  }

  // Log an access with elided group steps: an LDS log position from the
  // interval's LDS counter; entries past the LDS log's end, and accesses to
  // arrays logged globally, go to the global log (positions from the
  // group's global counter).  Entry order inside an interval does not
  // matter to the check.  Called by every lane of the wave.
  __device__ __forceinline__ void log_nf(uint32_t op, const ArrayDesc& A, uint32_t cell, int32_t val, bool rec) {
    const u64 br = __ballot(rec);
    if (br == 0ull) return;
    const bool store = op == OP_STORE;
    const uint32_t meta = (store ? 1024u : 0u) | tl;
    const u64 ck = (u64)A.cellbase + cell;
    if (A.logged == LOG_LDS) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&ctl->lds_cnt[interval & 1u], (uint32_t)__popcll(br));
      base = (uint32_t)__shfl((int)base, 0);
      const uint32_t j = base + (uint32_t)__popcll(br & ((1ull << lane) - 1ull));
      const bool over = rec && j >= P.lds_log_cap;
      if (rec && !over) {
        if (P.tab_cells) {
          lkey[j] = tab_entry((uint32_t)ck - P.tab_base, store, tl, val);
        } else {
          lkey[j] = (ck << 16) | j;
          lmeta[j] = meta;
          lval[j] = val;
        }
      }
      glog_append(__ballot(over), over, ck, meta, val);
    } else {
      glog_append(br, rec, ck, meta, val);
    }
  }

  // One load or store statement (op OP_LOAD / OP_STORE on array wc) for the
  // whole group; a load's value goes to `out` on active lanes.  Returns true
  // when the group stops on a fault (the statement then has no effect).
  // KIND >= 0: the array's kind (AK_*) known when the caller is compiled,
  // so only its path is generated; -1: read from the descriptor.
  // SYNC == false (per-program kernels with RC_JIT_ELIDE only): the
  // statement needs no group step, because no access since the group's last
  // synchronisation conflicts with it (a load after a store of the array, or
  // a store after a load); faults cannot occur and LDS log entries are
  // numbered by an LDS counter.
  // keep (interpreter, elided group steps only): whether this statement's
  // group step is kept (INSN_NO_STEP clear).
  template <int KIND = -1, bool SYNC = true>
  __device__ __forceinline__ bool mem(uint32_t op, uint32_t wc, int32_t idx, int32_t val, bool active,
                                      uint32_t spc, int32_t& out, bool keep = true) {
    ArrayDesc A = array_desc(P.arrays, wc);
    if (KIND >= 0) A.kind = (uint32_t)KIND;
    if (KIND == (int)AK_GLOBAL_RO) A.logged = LOG_NONE;   // never written, never logged
    const bool oob = active && (idx < 0 || (uint32_t)idx >= A.size);
#ifdef RC_JIT_NOFAULT
    if (oob) {   // (reported; the access is dropped)
      raise(spc, F_OOB);
      active = false;
    }
#else
    if (oob) {
      if (A.nosync || P.nf) {   // proven in bounds: the proof is wrong (reported; the access is dropped)
        atomicOr(P.status_word, 16u);
        active = false;
      } else {
        raise(spc, F_OOB);
      }
    }
#endif
    // a local array's accesses in an interval the proof shows race-free
    // (no cell written by one work-item and touched by another) can give no
    // record: they are not logged, and (the program cannot fault) need no
    // group step
    const bool quiet = A.kind == AK_LOCAL && A.logged != LOG_NONE &&
                       !(interval < 64u ? ((P.log_mask >> interval) & 1ull) != 0ull : P.log_high != 0u);
    const bool rec = active && P.do_log && A.logged != LOG_NONE && !quiet;
    n_logged += rec ? 1u : 0u;
#ifndef RC_JIT_W
    if (P.nf) {
      // no fault to publish and no entry numbering: synchronise only where
      // an earlier access since the last synchronisation conflicts
      if (keep && !quiet && !A.nosync) __syncthreads();
      access(op, wc, A, idx, val, active, out);
      if (P.do_log && A.logged != LOG_NONE && !quiet) log_nf(op, A, (uint32_t)idx, val, rec);
      return false;
    }
#endif
    // the barrier completes every earlier statement's accesses, publishes
    // pending faults (a faulting statement has no effect) and each wave's
    // number of log entries for this statement; a nosync array needs none
    // of that
    u64 brec = 0;
    uint32_t prefix = 0, total = 0;
    if (!A.nosync && SYNC && !quiet && mem_red(rec, &brec, &prefix, &total)) return true;
    access(op, wc, A, idx, val, active, out);
    const uint32_t cell = (uint32_t)idx;
#ifdef RC_JIT_ELIDE
    if (A.logged == LOG_LDS) {
      const u64 br = __ballot(rec);
      if (br != 0ull) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&ctl->lds_cnt[interval & 1u], (uint32_t)__popcll(br));
        base = (uint32_t)__shfl((int)base, 0);
        if (rec) {
          const uint32_t j = base + (uint32_t)__popcll(br & ((1ull << lane) - 1ull));
          if (j >= P.lds_log_cap) {
            atomicOr(P.status_word, 16u);   // (the static interval bound does not hold)
          } else if (P.tab_cells) {
            lkey[j] = tab_entry(A.cellbase + cell - P.tab_base, op == OP_STORE, tl, val);
          } else {
            lkey[j] = ((u64)(A.cellbase + cell) << 16) | j;
            lmeta[j] = ((op == OP_STORE) ? 1024u : 0u) | tl;
            lval[j] = val;
          }
        }
      }
      return false;
    }
#endif
    if (total != 0u) {
#ifdef RC_JIT_NOSPILL
      // (a per-program kernel of a program whose intervals always fit the
      // LDS log: the log never moves to the global log)
      constexpr bool may_spill = false;
#else
      constexpr bool may_spill = true;
#endif
      bool to_lds = A.logged == LOG_LDS && !(may_spill && lds_spilled);
      if (may_spill && to_lds && lds_used + total > P.lds_log_cap) {
        // the interval outgrows LDS: move its log to the global log, where
        // the global pass checks it
        for (uint32_t i = tl; i < lds_used; i += nthr) {
          const u64 pos = log_used + i;
          const u64 e = lkey[i];
          u64 ck;
          uint32_t meta, v;
          if (P.tab_cells) {
            ck = P.tab_base + (e >> 43);
            meta = (uint32_t)(e >> 32) & 2047u;   // store flag (bit 10) and local id
            v = (uint32_t)e;
          } else {
            ck = e >> 16;
            meta = lmeta[i];
            v = (uint32_t)lval[i];
          }
          glog_put(pos, ck, meta, v);
        }
        log_used += lds_used;
        lds_used = 0;
        lds_spilled = true;
        ++n_spilled;
        to_lds = false;
      }
      const uint32_t below = prefix + (uint32_t)__popcll(brec & ((1ull << lane) - 1ull));
      const uint32_t meta = ((op == OP_STORE) ? 1024u : 0u) | tl;
      if (to_lds) {
        if (rec) {
          const uint32_t j = lds_used + below;
          if (P.tab_cells) {
            lkey[j] = tab_entry(A.cellbase + cell - P.tab_base, op == OP_STORE, tl, val);
          } else {
            lkey[j] = ((u64)(A.cellbase + cell) << 16) | j;
            lmeta[j] = meta;
            lval[j] = val;
          }
        }
        lds_used += total;
      } else {
        if (rec) glog_put(log_used + below, (u64)A.cellbase + cell, meta, (uint32_t)val);
        log_used += total;
      }
    }
    return false;
  }

  // barrier: every work-item of the group must arrive; closes the interval.
  // Returns true when the group stops (a pending fault, or divergence).
  __device__ __forceinline__ bool barrier(bool active, uint32_t spc) {
    const uint32_t r = group_red(real && !active, active, true);
    if (r & 4u) return true;
    if (r & 1u) {
      if (real && !active) raise(spc, F_BARDIV);
      return true;
    }
    if (P.do_log) close_interval();
    ++interval;
    return false;
  }

  // end of the program (true: a pending fault stops the group first)
  __device__ __forceinline__ bool end() { return (group_red(false, false, true) & 4u) != 0u; }

  // Every wave leaves the program at the same point; the earliest fault wins.
  // The last interval (complete, or cut short by the fault) is checked, then
  // the item's counters go to the chunk's per-instance totals.
  __device__ __forceinline__ void finish() {
    if (faulted) {
      if (my_fault != ~0ull) atomicMin(&ctl->fault, my_fault);
      __syncthreads();
    }
    if (P.do_log) close_interval();
#ifndef RC_JIT_W
    if (P.nf) log_used = ctl->gl_cnt;   // (thread 0 reads what the last barrier published)
#endif
    if (tl == 0) {
      P.wg_count[wg_index] = (uint32_t)(log_used < P.wg_log_cap ? log_used : P.wg_log_cap);
      P.wg_base[wg_index] = log_base;
      atomicAdd(&P.inst_intervals[slot], interval + 1u);
      if (faulted) {
        const u64 f = ctl->fault;
        const uint32_t lid = (uint32_t)(f >> 17) & 1023u, fpc = (uint32_t)(f >> 5) & 4095u, code = (uint32_t)f & 7u;
        // instance status: the lowest faulting work-group
        atomicMin(&P.inst_fault[slot], ((u64)gid << 38) | ((u64)fpc << 26) | ((u64)lid << 16) | code);
      }
    }
    // accesses of the group
    u64 acc = n_acc;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if (lane == 0 && acc) atomicAdd(&P.inst_acc[slot], acc);
    // the call's log statistics: logged accesses, those in the global log,
    // intervals moved to the global log, intervals closed
    // (into the block's LDS totals: one global atomic per block and
    // statistic when the block leaves, not one per item)
    if (P.stats) {
      u64 lg = n_logged;
      for (int off = 32; off > 0; off >>= 1) lg += __shfl_down(lg, off);
      if (lane == 0 && lg) atomicAdd(&ctl->stat[0], lg);
      if (tl == 0) {
        // entries for the global pass or (one-group programs) the group
        // check, trailers not counted
        const u64 left = P.sc ? n_glog : (log_used < P.wg_log_cap ? log_used : P.wg_log_cap);
        ctl->stat[1] += left;
        ctl->stat[6] += left;
        ctl->stat[2] += n_spilled;
        ctl->stat[3] += interval + 1u;
        ctl->stat[4] += n_insn;
        ctl->stat[5] += (u64)n_insn * (nthr >> 6);
      }
    }
    __syncthreads();
  }
};

// Persistent loop: the workgroups of one width class take work items (an
// instance's work-group) from the chunk's queue until it is empty; `body`
// runs one item's program on a prepared Item and sets it.faulted when the
// group stopped on a fault.  The queue is ordered longest-first, so stealing
// in order balances the tail.
template <typename Body>
__device__ __forceinline__ void run_items(const PassParams& PP, Body body) {
  Ctl* ctl = reinterpret_cast<Ctl*>(rc_smem);
  const uint32_t ci = const_load<uint32_t>(PP.chunk_index, 0);
  const ChunkDesc C = const_load<ChunkDesc>(PP.chunks, ci);
  // (the class bounds are read from memory: a dynamic index into the loaded
  // descriptor would go through scratch)
  const uint32_t* item0 = PP.chunks[ci].item0;
  const uint32_t i0 = const_load<uint32_t>(item0, PP.wclass), i1 = const_load<uint32_t>(item0, PP.wclass + 1);
  if (i0 == i1) return;
  if (threadIdx.x == 0) {
    ctl->rc_cur = ctl->rc_end = 0ull;   // no record slots yet
    for (int k = 0; k < 7; ++k) ctl->stat[k] = 0ull;
  }
  for (;;) {
    if (threadIdx.x == 0) ctl->item = i0 + atomicAdd(&PP.queue[PP.wclass], 1u);
    __syncthreads();
    const uint32_t item = uni(ctl->item);
    __syncthreads();
    if (item >= i1) {
      // the block's log statistics
      if (PP.stats && threadIdx.x < 7u && ctl->stat[threadIdx.x])
        atomicAdd(&PP.stats[threadIdx.x], ctl->stat[threadIdx.x]);
      // the block's unused record slots
      const rc_record_out R = const_load<rc_record_out>(PP.rec, 0);
      const u64 a = ctl->rc_cur, b = ctl->rc_end;
      const uint32_t nthr = 64u << PP.wclass;
      for (u64 p = a + threadIdx.x; p < b && p < R.rec_cap; p += nthr) RC_GLOBAL(u64, R.rec_keys)[p] = ~0ull;
      if (threadIdx.x == 0 && b > a)
        __hip_atomic_fetch_add(RC_GLOBAL(unsigned long long, R.rec_dead), (unsigned long long)(b - a),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    const uint32_t instance = const_load<uint32_t>(PP.items, 2u * item);
    const uint32_t gid = const_load<uint32_t>(PP.items, 2u * item + 1u);
    const SlotDesc S = const_load<SlotDesc>(PP.slots, instance);
    const ProgDesc D = const_load<ProgDesc>(PP.progs, S.prog);
    ItemView P;
    P.code = D.code; P.arrays = D.arrays; P.scalars = D.scalars;
    P.n_arrays = D.n_arrays; P.n_global = D.n_global; P.n_scalars = D.n_scalars; P.nregs = D.nregs;
    P.G = D.G; P.W = D.W; P.nwaves = D.nwaves; P.lds_local_cells = D.lds_local_cells;
    P.lds_log_cap = D.lds_log_cap; P.overlay_cells = D.overlay_cells; P.NI = D.NI;
    P.tab_base = D.tab_base; P.tab_cells = D.tab_cells;
    P.log_mask = D.log_mask; P.log_high = D.log_high;
    P.bc = PP.bc; P.bg = PP.bg; P.bk = PP.bk; P.bs = PP.bs; P.do_log = PP.do_log;
    P.wg_log_cap = D.wg_log_cap;
    P.log_keys = PP.log_keys; P.log_vals = PP.log_vals; P.status_word = PP.status_word; P.rec = PP.rec;
    P.inst_acc = PP.inst_acc; P.inst_intervals = PP.inst_intervals; P.inst_fault = PP.inst_fault;
    P.wg_count = PP.wg_count; P.wg_base = PP.wg_base;
    P.cell_owner = PP.cell_owner; P.co_stride = PP.cell_owner_stride;
    P.stats = PP.stats;
    P.nf = D.nf;
    P.step_limit = D.step_limit;
    P.sc = D.sc;
#ifdef RC_JIT_W
    // A per-program kernel is compiled for one launch shape: its constants
    // replace the descriptor's fields, so the compiler folds them.  A
    // descriptor of another shape is a library error, reported through the
    // status word; the item is skipped.
    bool same_arrays = true;
#pragma unroll
    for (uint32_t a = 0; a < RC_JIT_NA; ++a) {
      const ArrayDesc X = const_load<ArrayDesc>(D.arrays, a), Y = array_desc(D.arrays, a);
      same_arrays = same_arrays && X.kind == Y.kind && X.size == Y.size && X.logged == Y.logged &&
                    X.offset == Y.offset && X.cellbase == Y.cellbase && X.own_stride == Y.own_stride &&
                    X.own_lo == Y.own_lo && X.own_span == Y.own_span && X.nosync == Y.nosync;
    }
    if (D.W != RC_JIT_W || D.G != RC_JIT_G || D.n_arrays != RC_JIT_NA || D.tab_cells != RC_JIT_TC ||
        D.tab_base != RC_JIT_TB || D.lds_log_cap != RC_JIT_LC || D.log_mask != RC_JIT_LOGMASK ||
        D.log_high != RC_JIT_LOGHIGH || !same_arrays) {
      if (threadIdx.x == 0) {
        atomicOr(PP.status_word, 8u);
        PP.wg_count[S.wg_base + gid] = 0u;   // nothing logged
        PP.wg_base[S.wg_base + gid] = S.log_base + (u64)gid * D.wg_log_cap;
      }
      continue;
    }
    P.W = RC_JIT_W; P.G = RC_JIT_G; P.nwaves = (RC_JIT_W + 63u) / 64u; P.n_arrays = RC_JIT_NA;
    P.tab_cells = RC_JIT_TC; P.tab_base = RC_JIT_TB; P.lds_log_cap = RC_JIT_LC;
    P.log_mask = RC_JIT_LOGMASK; P.log_high = RC_JIT_LOGHIGH;
    P.nf = 0u;
#endif
    Item it;
    it.init(P, ctl, instance - C.slot0, instance, gid, S.seed, S.log_base + (u64)gid * D.wg_log_cap,
            PP.overlay + S.ovl_base + (u64)gid * D.overlay_cells, C.epoch, S.wg_base + gid, 64u << PP.wclass);
    body(it);
    it.finish();
  }
}

}  // namespace rc
