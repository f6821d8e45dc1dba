// kernels.hip -- HIP kernels of the race checker for gfx950.
//
//  * rc_interp_kernel: the lockstep interpreter.  One workgroup runs one
//    work-group of one instance; lane l is work-item l.  Statements run one
//    at a time for the whole work-group (paper Section 4 thread-local rules
//    under the lockstep schedule); a barrier closes an interval (Section 4
//    global rules).  Private variables live in LDS, laid out register-major
//    so a wave reads 64 consecutive dwords.  Every access to an array that
//    the program writes somewhere is appended to the access log.
//  * rs_* / scan_*: stable LSD radix sort (8-bit digits) and exclusive scan.
//  * seg_check_kernel: after the log is sorted by (instance, cell, gid,
//    interval), each run of one cell is checked for eligible pairs (the
//    Section 4 race rule made concrete; Section 1: equal-value writes are
//    benign) with two passes of min-reductions per scope.
//  * rec_gather_kernel / finalize: canonical record order and summaries.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "rc_internal.h"
#include "kernels.h"

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

__device__ __forceinline__ void store_record(const rc_record_out& R, const RecKey& K, u64 pos, uint32_t slot,
                                             uint32_t instance, const PendingRec& p, bool inter) {
  if (pos >= R.rec_cap) { atomicOr(R.status_word, 2u); return; }
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
  reinterpret_cast<rc_record_dev*>(R.staging)[pos] = r;
  const u64 scope = inter ? (u64)K.G * K.NI : (u64)p.gid * K.NI + p.interval;
  R.rec_keys[pos] = ((u64)slot << (K.bs + K.bc)) | (scope << K.bc) | p.cellkey;
  R.rec_idx[pos] = (uint32_t)pos;
}

// wave-wide allocation of record slots: one atomic per wave
__device__ __forceinline__ u64 wave_reserve(unsigned long long* counter, uint32_t n, uint32_t lane) {
  u64 base = 0;
  if (lane == 0 && n) base = atomicAdd(counter, (u64)n);
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
};

// Run one work-group of one instance, lockstep, on the calling workgroup.
// `slot` indexes the chunk's per-instance counters, `instance` the call's.
__device__ __forceinline__ void run_item(const ItemView& P, Ctl* ctl, uint32_t slot, uint32_t instance,
                                         uint32_t gid, uint64_t seed, u64 log_base, u64* ovl,
                                         uint32_t epoch_base, uint32_t wg_index) {
  const uint32_t tl = threadIdx.x;
  const uint32_t WP = P.nwaves * 64u;
  const uint32_t wave = tl >> 6, lane = tl & 63u;
  const bool real = tl < P.W;
  const uint32_t tr = tl < WP ? tl : WP - 1u;   // waves past the group read a real lane's registers

  // dynamic LDS after the control block: local array cells (u64), the
  // interval log (T keys, T payload words, T values), registers
  u64* locc = reinterpret_cast<u64*>(reinterpret_cast<unsigned char*>(ctl) + ((sizeof(Ctl) + 15) & ~(size_t)15));
  u64* lkey = locc + P.lds_local_cells;
  uint32_t* lmeta = reinterpret_cast<uint32_t*>(lkey + P.lds_log_cap);
  int32_t* lval = reinterpret_cast<int32_t*>(lmeta + P.lds_log_cap);
  int32_t* regs = lval + P.lds_log_cap;
  // the per-cell check table (8-byte aligned after the registers)
  TabCell* tab = reinterpret_cast<TabCell*>(
      (reinterpret_cast<uintptr_t>(regs + P.nregs * WP) + 7u) & ~(uintptr_t)7u);
  const TabCell empty_cell = {~0ull, NONE32, NONE32, NONE32, NONE32, 0u, NONE32};

  for (uint32_t i = tl; i < P.lds_local_cells; i += blockDim.x) locc[i] = 0ull;
  for (uint32_t i = tl; i < P.nregs * WP; i += blockDim.x) regs[i] = 0;
  for (uint32_t i = tl; i < P.tab_cells; i += blockDim.x) tab[i] = empty_cell;
  if (tl == 0) ctl->fault = ~0ull;
  if (tl < P.n_scalars) {
    const ScalarDesc S = const_load<ScalarDesc>(P.scalars, tl);
    ctl->scal[tl] = S.bind == BIND_SEEDED ? seeded_cell(seed, 0x10000u + tl, 0, S.lo, S.hi) : S.value;
  }
  __syncthreads();

  const u64 key_slot = (u64)slot << (P.bc + P.bg + P.bk);
  u64 log_used = 0;
  uint32_t lds_used = 0;       // entries of the current interval in the LDS log
  bool lds_spilled = false;    // the current interval moved to the global log
  uint32_t pc = 0, depth = 0, eany = 0, last_spc = ~0u;
  uint32_t step = 0, store_seq = 0, interval = 0, parity = 0;
  uint32_t mbits = real ? 1u : 0u, ebits = 0u;
  uint32_t n_acc = 0;
  u64 my_fault = ~0ull;      // earliest fault of this work-item (fault_key order)
  bool faulted = false;

  auto fetch = [&](bool imm, uint32_t w) -> int32_t {
    if (imm) return (int32_t)w;
    if (w < MAX_REGS) return regs[w * WP + tr];
    switch (w) {
      case SEL_LID: return (int32_t)tl;
      case SEL_TID: return (int32_t)(gid * P.W + tl);
      case SEL_GID: return (int32_t)gid;
      case SEL_WGSIZE: return (int32_t)P.W;
      case SEL_NGROUPS: return (int32_t)P.G;
      case SEL_NTHREADS: return (int32_t)(P.G * P.W);
      default: return ctl->scal[w - SEL_SCALAR0];
    }
  };
  // Group-wide OR of two per-lane predicates (bits 0, 1) and of "some
  // work-item has a pending fault" (bit 2).  Every wave publishes its word
  // before the barrier and reads all words after it, so all waves decide on
  // the same snapshot.  The words are double-buffered: a wave can only reuse
  // a buffer after the next reduction's barrier, which every reader passes
  // after reading.
  auto group_red = [&](bool p0, bool p1, bool sync_always) -> uint32_t {
    const u64 b0 = __ballot(p0), b1 = __ballot(p1), bf = __ballot(my_fault != ~0ull);
    const uint32_t mine = (b0 != 0ull ? 1u : 0u) | (b1 != 0ull ? 2u : 0u) | (bf != 0ull ? 4u : 0u);
    if (P.nwaves == 1) {
      if (sync_always) __syncthreads();
      return uni(mine);
    }
    if (lane == 0) ctl->red[parity][wave] = mine;
    __syncthreads();
    uint32_t acc = 0;
    for (uint32_t w = 0; w < P.nwaves; ++w) acc |= ctl->red[parity][w];
    parity ^= 1u;
    return uni(acc);
  };
  // The same snapshot reduction for a memory statement: bit 0 of each wave's
  // word is its pending-fault flag, bits 8.. its count of log entries; every
  // wave gets the group total and the count of the waves before it.
  auto mem_red = [&](bool rec, u64* brec, uint32_t* prefix, uint32_t* total) -> bool {
    const u64 br = __ballot(rec), bf = __ballot(my_fault != ~0ull);
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
    uint32_t f = 0, tot = 0, pre = 0;
    for (uint32_t w = 0; w < P.nwaves; ++w) {
      const uint32_t x = ctl->red[parity][w];
      f |= x & 1u;
      tot += x >> 8;
      if (w < wave) pre += x >> 8;
    }
    parity ^= 1u;
    *prefix = uni(pre);
    *total = uni(tot);
    return uni(f) != 0u;
  };
  auto raise = [&](uint32_t spc, uint32_t code) {
    const u64 k = fault_key(step, tl, spc, code);
    if (k < my_fault) my_fault = k;
  };

  // Close the current interval on the LDS path: sort its log by cell in LDS
  // (bitonic), then the first entry of every cell's run checks the run
  // (INTRA scope) and records go to the staging area.  Callers have passed a
  // barrier since the interval's last access.
  auto close_interval = [&]() {
    const uint32_t n = lds_used;
    const bool spilled = lds_spilled;
    lds_used = 0;
    lds_spilled = false;
    if (spilled || n < 2u) return;
    const rc_record_out R = const_load<rc_record_out>(P.rec, 0);
    const RecKey K = {P.bs, P.bc, P.G, P.NI};
    if (P.tab_cells) {
      // Per-cell table: the same two passes as intra_check, merged with LDS
      // atomics; the cell's first log entry (the owner) finishes the check
      // and clears the cell for the next interval.
      for (uint32_t i = tl; i < n; i += blockDim.x) {
        TabCell& c = tab[(uint32_t)(lkey[i] >> 16) - P.tab_base];
        const uint32_t meta = lmeta[i];
        const uint32_t l = meta & 1023u;
        if (meta & 1024u) atomicMin(&c.wmin, ((u64)l << 32) | ((uint32_t)lval[i] ^ 0x80000000u));
        else atomicMin(&c.r1, l);
        atomicMin(&c.owner, i);
      }
      __syncthreads();
      for (uint32_t i = tl; i < n; i += blockDim.x) {
        TabCell& c = tab[(uint32_t)(lkey[i] >> 16) - P.tab_base];
        const uint32_t meta = lmeta[i];
        const uint32_t l = meta & 1023u;
        const u64 wmin = c.wmin;
        const uint32_t w1 = wmin == ~0ull ? NONE32 : (uint32_t)(wmin >> 32);
        const int32_t x1 = (int32_t)((uint32_t)wmin ^ 0x80000000u);
        if (meta & 1024u) {
          const int32_t v = lval[i];
          if (l == w1) { if (v != x1) atomicOr(&c.multi1, 1u); }
          else {
            atomicMin(&c.w2, l);
            if (v != x1) atomicMin(&c.q, l);
          }
        } else if (l != c.r1) {
          atomicMin(&c.r2, l);
        }
      }
      __syncthreads();
      for (uint32_t b0 = 0; b0 < n; b0 += blockDim.x) {
        const uint32_t i = b0 + tl;
        bool has = false;
        PendingRec pr;
        if (i < n) {
          const uint32_t ck = (uint32_t)(lkey[i] >> 16);
          TabCell& c = tab[ck - P.tab_base];
          if (c.owner == i) {
            const Pass1 p1 = {c.r1, c.wmin};
            const Intra2 p2 = {c.r2, c.w2, c.q, c.multi1};
            c = empty_cell;
            has = intra_finish(p1, p2, &pr.label, &pr.rw, &pr.ww);
            if (has) {
              uint32_t aid = 0;
              for (uint32_t a = 0; a < P.n_arrays; ++a) {
                const ArrayDesc D = const_load<ArrayDesc>(P.arrays, a);
                if (D.logged == LOG_LDS && ck >= D.cellbase && ck - D.cellbase < D.size) aid = a;
              }
              const ArrayDesc D = const_load<ArrayDesc>(P.arrays, aid);
              pr.gid = gid; pr.interval = interval; pr.aid = aid; pr.cell = ck - D.cellbase;
              pr.cellkey = ck; pr.lidbase = gid * P.W;
            }
          }
        }
        const u64 m = __ballot(has);
        if (m != 0ull) {
          const u64 base = wave_reserve(R.rec_count, (uint32_t)__popcll(m), lane);
          if (has) store_record(R, K, base + (u64)__popcll(m & ((1ull << lane) - 1ull)), slot, instance, pr, false);
        }
      }
      __syncthreads();
      return;
    }
    uint32_t P2 = 2;
    while (P2 < n) P2 <<= 1;
    for (uint32_t i = n + tl; i < P2; i += blockDim.x) lkey[i] = ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= P2; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = tl; i < P2; i += blockDim.x) {
          const uint32_t ixj = i ^ j;
          if (ixj > i) {
            const u64 a = lkey[i], b = lkey[ixj];
            if ((a > b) == ((i & k) == 0u)) { lkey[i] = b; lkey[ixj] = a; }
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t b0 = 0; b0 < n; b0 += blockDim.x) {
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
                const ArrayDesc D = const_load<ArrayDesc>(P.arrays, a);
                if (D.logged == LOG_LDS && ck >= D.cellbase && ck - D.cellbase < D.size) aid = a;
              }
              const ArrayDesc D = const_load<ArrayDesc>(P.arrays, aid);
              pr.gid = gid; pr.interval = interval; pr.aid = aid; pr.cell = (uint32_t)ck - D.cellbase;
              pr.cellkey = (uint32_t)ck; pr.lidbase = gid * P.W;
            }
          }
        }
      }
      const u64 m = __ballot(has);
      if (m != 0ull) {
        const u64 base = wave_reserve(R.rec_count, (uint32_t)__popcll(m), lane);
        if (has) store_record(R, K, base + (u64)__popcll(m & ((1ull << lane) - 1ull)), slot, instance, pr, false);
      }
    }
    __syncthreads();
  };

  for (;;) {
    pc = uni(pc);
    const Insn in = const_load<Insn>(P.code, pc);
    const uint32_t h = in.h, wa = in.a, wb = in.b, wc = in.c;
    const uint32_t op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u, spc = h >> 20;
    const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
    if (spc != last_spc) { ++step; last_spc = spc; }
    const bool active = (mbits >> depth) & 1u;

    if (op == OP_BIN) {
      int32_t x = fetch(fa, wa), y = fetch(fb, wb);
      bool dz = false;
      int32_t r = alu_bin(sub, x, y, dz);
      if (active) {
        regs[dst * WP + tl] = r;
        if (dz) raise(spc, F_DIV);
      }
      ++pc;
    } else if (op == OP_UN) {
      int32_t x = fetch(fa, wa);
      int32_t r = sub == U_MOV ? x : sub == U_NEG ? (int32_t)(0u - (uint32_t)x) : sub == U_BNOT ? ~x : (int32_t)(x == 0);
      if (active) regs[dst * WP + tl] = r;
      ++pc;
    } else if (op == OP_LOAD || op == OP_STORE) {
      const ArrayDesc A = const_load<ArrayDesc>(P.arrays, wc);
      const int32_t idx = fetch(fa, wa);
      const int32_t val = op == OP_STORE ? fetch(fb, wb) : 0;
      if (active && (idx < 0 || (uint32_t)idx >= A.size)) raise(spc, F_OOB);
      const bool rec = active && P.do_log && A.logged != LOG_NONE;
      // the barrier completes every earlier statement's accesses, publishes
      // pending faults (a faulting statement has no effect) and each wave's
      // number of log entries for this statement
      u64 brec;
      uint32_t prefix, total;
      if (mem_red(rec, &brec, &prefix, &total)) { faulted = true; break; }
      const uint32_t cell = (uint32_t)idx;
      if (op == OP_LOAD) {
        if (active) {
          int32_t v;
          if (A.kind == AK_LOCAL) {
            v = (int32_t)(uint32_t)locc[A.offset + cell];
          } else {
            bool have = false;
            v = 0;
            if (A.kind == AK_GLOBAL_RW) {
              u64 w = __hip_atomic_load(&ovl[A.offset + cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if ((uint32_t)(w >> 42) >= epoch_base) { v = (int32_t)(uint32_t)w; have = true; }
            }
            if (!have)
              v = A.bind == BIND_SEEDED ? seeded_cell(seed, wc, cell, A.lo, A.hi) : A.dptr[cell];
          }
          regs[dst * WP + tl] = v;
          ++n_acc;
        }
      } else {
        ++store_seq;
        if (active) {
          // within one statement the highest work-item's value stays
          const uint32_t ep = A.kind == AK_LOCAL ? store_seq : epoch_base + store_seq;
          const u64 word = ((u64)((ep << 10) | tl) << 32) | (uint32_t)val;
          if (A.kind == AK_LOCAL) atomicMax(&locc[A.offset + cell], word);
          else atomicMax(&ovl[A.offset + cell], word);
          ++n_acc;
        }
      }
      if (total != 0u) {
        bool to_lds = A.logged == LOG_LDS && !lds_spilled;
        if (to_lds && lds_used + total > P.lds_log_cap) {
          // the interval outgrows LDS: move its log to the global log, where
          // the global pass checks it
          for (uint32_t i = tl; i < lds_used; i += blockDim.x) {
            const u64 pos = log_used + i;
            const u64 ck = lkey[i] >> 16;
            if (pos < P.wg_log_cap) {
              P.log_keys[log_base + pos] = key_slot | (((ck << P.bg) | gid) << P.bk) | interval;
              P.log_vals[log_base + pos] = ((u64)(uint32_t)lval[i] << 32) | lmeta[i];
            } else {
              atomicOr(P.status_word, 1u);
            }
          }
          log_used += lds_used;
          lds_used = 0;
          lds_spilled = true;
          to_lds = false;
        }
        const uint32_t below = prefix + (uint32_t)__popcll(brec & ((1ull << lane) - 1ull));
        const uint32_t meta = ((op == OP_STORE) ? 1024u : 0u) | tl;
        if (to_lds) {
          if (rec) {
            const uint32_t j = lds_used + below;
            lkey[j] = ((u64)(A.cellbase + cell) << 16) | j;
            lmeta[j] = meta;
            lval[j] = val;
          }
          lds_used += total;
        } else {
          if (rec) {
            const u64 pos = log_used + below;
            if (pos < P.wg_log_cap) {
              P.log_keys[log_base + pos] = key_slot | ((((u64)(A.cellbase + cell) << P.bg) | gid) << P.bk) | interval;
              P.log_vals[log_base + pos] = ((u64)(uint32_t)val << 32) | meta;
            } else {
              atomicOr(P.status_word, 1u);
            }
          }
          log_used += total;
        }
      }
      ++pc;
    } else if (op == OP_IF) {
      const int32_t c = fetch(fa, wa);
      const bool t = active && c != 0, e = active && c == 0;
      const uint32_t d1 = depth + 1u;
      mbits = (mbits & ~(1u << d1)) | ((uint32_t)t << d1);
      ebits = (ebits & ~(1u << d1)) | ((uint32_t)e << d1);
      const uint32_t any = group_red(t, e, false);
      if (any & 4u) { faulted = true; break; }
      depth = d1;
      eany = (eany & ~(1u << d1)) | (((any >> 1) & 1u) << d1);
      pc = (any & 1u) ? pc + 1u : wb;
    } else if (op == OP_ELSE) {
      mbits = (mbits & ~(1u << depth)) | (((ebits >> depth) & 1u) << depth);
      pc = ((eany >> depth) & 1u) ? pc + 1u : wc;
    } else if (op == OP_ENDIF) {
      --depth;
      ++pc;
    } else if (op == OP_FOR) {
      const int32_t lo = (int32_t)wa, hi = (int32_t)wb;
      if (active) regs[dst * WP + tl] = lo;
      if ((int64_t)hi - (int64_t)lo <= 0) {
        pc = wc;
      } else {
        if (lane == 0) ctl->loopctr[wave][sub] = 0u;
        ++pc;
      }
    } else if (op == OP_ENDFOR) {
      const int32_t lo = (int32_t)wa, hi = (int32_t)wb;
      const uint32_t iters = (uint32_t)((int64_t)hi - (int64_t)lo);
      const uint32_t ctr = uni(ctl->loopctr[wave][sub]) + 1u;
      if (lane == 0) ctl->loopctr[wave][sub] = ctr;
      if (active) regs[dst * WP + tl] = (int32_t)((uint32_t)lo + ctr);
      pc = ctr < iters ? wc : pc + 1u;
    } else if (op == OP_BARRIER) {
      // every work-item of the group must arrive (bit 0: some are missing)
      const uint32_t r = group_red(real && !active, active, true);
      if (r & 4u) { faulted = true; break; }
      if (r & 1u) {
        if (real && !active) raise(spc, F_BARDIV);
        faulted = true;
        break;
      }
      if (P.do_log) close_interval();
      ++interval;
      ++pc;
    } else if (op == OP_ASSERT || op == OP_ASSUME) {
      const int32_t c = fetch(fa, wa);
      if (active && c == 0) raise(spc, op == OP_ASSERT ? F_ASSERT : F_ASSUME);
      ++pc;
    } else {  // OP_END
      if (group_red(false, false, true) & 4u) faulted = true;
      break;
    }
  }

  // every wave leaves the loop at the same point; the earliest fault wins.
  // The last interval (complete, or cut short by the fault) is checked.
  if (faulted) {
    if (my_fault != ~0ull) atomicMin(&ctl->fault, my_fault);
    __syncthreads();
  }
  if (P.do_log) close_interval();
  // the last interval (complete, or cut by a fault) is closed
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
  __syncthreads();
}

// Persistent interpreter: the workgroups of one width class take work items
// (an instance's work-group) from the chunk's queue until it is empty.  The
// queue is ordered longest-first, so stealing in order balances the tail.
__global__ __launch_bounds__(1024) void rc_interp_kernel(PassParams PP) {
  Ctl* ctl = reinterpret_cast<Ctl*>(rc_smem);
  const uint32_t ci = const_load<uint32_t>(PP.chunk_index, 0);
  const ChunkDesc C = const_load<ChunkDesc>(PP.chunks, ci);
  const uint32_t i0 = C.item0[PP.wclass], i1 = C.item0[PP.wclass + 1];
  if (i0 == i1) return;
  for (;;) {
    if (threadIdx.x == 0) ctl->item = i0 + atomicAdd(&PP.queue[PP.wclass], 1u);
    __syncthreads();
    const uint32_t item = uni(ctl->item);
    __syncthreads();
    if (item >= i1) break;
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
    P.bc = PP.bc; P.bg = PP.bg; P.bk = PP.bk; P.bs = PP.bs; P.do_log = PP.do_log;
    P.wg_log_cap = D.wg_log_cap;
    P.log_keys = PP.log_keys; P.log_vals = PP.log_vals; P.status_word = PP.status_word; P.rec = PP.rec;
    P.inst_acc = PP.inst_acc; P.inst_intervals = PP.inst_intervals; P.inst_fault = PP.inst_fault;
    P.wg_count = PP.wg_count; P.wg_base = PP.wg_base;
    run_item(P, ctl, instance - C.slot0, instance, gid, S.seed, S.log_base + (u64)gid * D.wg_log_cap,
             PP.overlay + S.ovl_base + (u64)gid * D.overlay_cells, C.epoch, S.wg_base + gid);
  }
}

// ---------------------------------------------------------------------------
// exclusive scan of u32 arrays (three-level, 1024 elements per block)
// ---------------------------------------------------------------------------
constexpr uint32_t SCAN_BLOCK = 1024;

__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* sh, uint32_t* total) {
  // 256 threads: inclusive scan via waves + LDS
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t i = 0; i < w; ++i) before += sh[i];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return before + x - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t* in, uint64_t m, uint32_t* sums) {
  __shared__ uint32_t sh[4];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * 4u;
  uint32_t s = 0;
  for (int k = 0; k < 4; ++k) if (base + k < m) s += in[base + k];
  uint32_t total;
  block_excl_scan_256(s, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_block_kernel(uint32_t* data, uint64_t m, const uint32_t* offs) {
  __shared__ uint32_t sh[4];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * 4u;
  uint32_t v[4];
  uint32_t s = 0;
  for (int k = 0; k < 4; ++k) { v[k] = base + k < m ? data[base + k] : 0u; s += v[k]; }
  uint32_t total;
  uint32_t ex = block_excl_scan_256(s, sh, &total);
  if (offs) ex += offs[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    if (base + k < m) data[base + k] = ex;
    ex += v[k];
  }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits; n lives on the device
// ---------------------------------------------------------------------------
constexpr uint32_t RS_THREADS = 256, RS_ROUNDS = 16, RS_TILE = RS_THREADS * RS_ROUNDS;

// Input of one radix pass: dense (n on the device), or segmented: region r
// starts at entry seg_base[r] and holds seg_count[r] entries; tiles[r] is the
// exclusive prefix of the regions' tile counts (n_regions + 1 words), so each
// block finds its region by binary search and the pass also compacts the
// regions into a dense output.
struct RsIn {
  const u64* n_ptr;
  const uint32_t* seg_count;
  const u64* seg_base;
  const uint32_t* tiles;
  uint32_t n_regions, dbits;   // dbits: digit width of this pass (1..8)
};

__device__ __forceinline__ void rs_tile(const RsIn& in, uint32_t b, u64* start, uint32_t* count) {
  if (in.seg_count == nullptr) {
    const u64 n = *in.n_ptr;
    const u64 t0 = (u64)b * RS_TILE;
    *start = t0;
    *count = t0 >= n ? 0u : (uint32_t)(n - t0 < RS_TILE ? n - t0 : RS_TILE);
    return;
  }
  *start = 0;
  *count = 0;
  if (b >= in.tiles[in.n_regions]) return;
  uint32_t lo = 0, hi = in.n_regions;   // tiles[lo] <= b < tiles[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (in.tiles[mid] <= b) lo = mid; else hi = mid;
  }
  const u64 t0 = (u64)(b - in.tiles[lo]) * RS_TILE;
  const u64 used = in.seg_count[lo];
  *start = in.seg_base[lo] + t0;
  *count = t0 >= used ? 0u : (uint32_t)(used - t0 < RS_TILE ? used - t0 : RS_TILE);
}

__global__ __launch_bounds__(256) void region_tiles_kernel(const uint32_t* counts, uint32_t* tiles, u64 n) {
  const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) tiles[r] = (counts[r] + RS_TILE - 1) / RS_TILE;
  else if (r == n) tiles[r] = 0;
}

// Lanes of a wave holding the same digit (dbits ballots); rank = position
// among them, count = how many.
__device__ __forceinline__ void digit_peers(uint32_t d, bool valid, uint32_t dbits, uint32_t lane,
                                            uint32_t* rank, uint32_t* count) {
  u64 eq = __ballot(valid);
  for (uint32_t b = 0; b < dbits; ++b) {
    const u64 bb = __ballot((d >> b) & 1u);
    eq &= ((d >> b) & 1u) ? bb : ~bb;
  }
  *rank = (uint32_t)__popcll(eq & ((1ull << lane) - 1ull));
  *count = (uint32_t)__popcll(eq);
}

// Digit counts of one tile; one LDS atomic per distinct digit per wave
// (sorted inputs make high digits nearly constant within a tile).
__global__ __launch_bounds__(256) void rs_hist_kernel(const u64* keys, RsIn in, uint32_t shift,
                                                      uint32_t* hist, uint32_t nblocks) {
  __shared__ uint32_t h[256];
  const uint32_t t = threadIdx.x, lane = t & 63u;
  const uint32_t dmask = (1u << in.dbits) - 1u;
  h[t] = 0;
  __syncthreads();
  u64 start;
  uint32_t count;
  rs_tile(in, blockIdx.x, &start, &count);
  for (uint32_t i0 = 0; i0 < count; i0 += RS_THREADS) {
    const uint32_t i = i0 + t;
    const bool valid = i < count;
    const uint32_t d = valid ? (uint32_t)(keys[start + i] >> shift) & dmask : 0u;
    uint32_t rank, cnt;
    digit_peers(d, valid, in.dbits, lane, &rank, &cnt);
    if (valid && rank == 0) atomicAdd(&h[d], cnt);
  }
  __syncthreads();
  if (t <= dmask) hist[(size_t)t * nblocks + blockIdx.x] = h[t];
}

// Stable scatter of one tile: wave w owns the tile's w-th quarter (RS_ROUNDS
// rounds of 64 consecutive entries, kept in registers).  Each wave counts its
// digits, one pass turns the counts into per-wave running offsets, and each
// wave then writes its entries in order.  Two block barriers per tile.
template <typename V>
__global__ __launch_bounds__(256) void rs_scatter_kernel(const u64* kin, const V* vin, u64* kout, V* vout,
                                                         RsIn in, uint32_t shift,
                                                         const uint32_t* offs, uint32_t nblocks) {
  __shared__ uint32_t woff[4][256];
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  u64 start;
  uint32_t count;
  rs_tile(in, blockIdx.x, &start, &count);
  if (count == 0) return;
  const uint32_t dmask = (1u << in.dbits) - 1u;
  for (uint32_t ww = 0; ww < 4; ++ww) woff[ww][t] = 0u;
  __syncthreads();
  const uint32_t wbeg = w * (RS_TILE / 4);
  u64 kr[RS_ROUNDS];
  V vr[RS_ROUNDS];
#pragma unroll
  for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
    const uint32_t i = wbeg + r * 64u + lane;
    const bool valid = i < count;
    kr[r] = valid ? kin[start + i] : 0ull;
    vr[r] = valid ? vin[start + i] : (V)0;
    const uint32_t d = (uint32_t)(kr[r] >> shift) & dmask;
    uint32_t rank, cnt;
    digit_peers(d, valid, in.dbits, lane, &rank, &cnt);
    if (valid && rank == 0) woff[w][d] += cnt;      // one lane per digit: no conflict in the wave
  }
  __syncthreads();
  if (t <= dmask) {
    uint32_t o = offs[(size_t)t * nblocks + blockIdx.x];
    for (uint32_t ww = 0; ww < 4; ++ww) {
      const uint32_t c = woff[ww][t];
      woff[ww][t] = o;
      o += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
    const uint32_t i = wbeg + r * 64u + lane;
    const bool valid = i < count;
    const uint32_t d = (uint32_t)(kr[r] >> shift) & dmask;
    uint32_t rank, cnt;
    digit_peers(d, valid, in.dbits, lane, &rank, &cnt);
    if (valid) {
      const uint32_t base = woff[w][d];
      kout[base + rank] = kr[r];
      vout[base + rank] = vr[r];
      // the new offset depends on the value just read, so the wave's read
      // of this round is complete before any lane advances the counter
      if (rank == 0) woff[w][d] = base + cnt;
    }
  }
}

__global__ __launch_bounds__(256) void sum_u32_kernel(const uint32_t* v, u64 n, u64* out) {
  u64 s = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) s += v[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63u) == 0 && s) atomicAdd(out, s);
}

// ---------------------------------------------------------------------------
// segment check
// ---------------------------------------------------------------------------
// One thread per sorted log entry.  The first entry of a run of equal keys
// checks its INTRA(gid, interval) scope; the first entry of a cell's run
// also checks the INTER scope (global arrays, several groups).
// A run of the sorted log is the entries sharing a key prefix: the full key
// for an INTRA run (instance, cell, group, interval), the key above the group
// and interval fields for an INTER run (instance, cell).  A run of at most
// SEG_SHORT entries is checked by the thread at its head; a longer one is
// queued and checked by a whole workgroup (seg_long_kernel), so a hot cell
// never serialises a wave.
constexpr u64 SEG_SHORT = SEG_SHORT_RUN;

// first index after i whose key differs from keys[i] above `shift` bits
// (galloping then bisection: O(log run length) reads)
__device__ __forceinline__ u64 run_end(const u64* keys, u64 i, u64 n, uint32_t shift) {
  const u64 kk = keys[i] >> shift;
  u64 lo = i, hi = n, step = 1;
  while (true) {
    const u64 probe = i + step;
    if (probe >= n) { hi = n; break; }
    if ((keys[probe] >> shift) != kk) { hi = probe; break; }
    lo = probe;
    step <<= 1;
  }
  while (hi - lo > 1) {
    const u64 mid = lo + (hi - lo) / 2;
    if ((keys[mid] >> shift) == kk) lo = mid; else hi = mid;
  }
  return hi;
}

struct SegHead {          // what a run's first key says about it
  uint32_t slot, instance, gid, interval, aid, cell, cellkey, G, W, NI, n_global;
};
__device__ __forceinline__ SegHead seg_head(const SegParams& S, u64 k) {
  SegHead h;
  const uint32_t low = S.bg + S.bk;
  const uint32_t cmask = S.bc >= 32 ? 0xFFFFFFFFu : ((1u << S.bc) - 1u);
  h.cellkey = (uint32_t)(k >> low) & cmask;
  h.slot = (uint32_t)(k >> (low + S.bc));
  h.gid = (uint32_t)(k >> S.bk) & ((1u << S.bg) - 1u);
  h.interval = (uint32_t)k & ((1u << S.bk) - 1u);
  const ChunkDesc C = S.chunks[*S.chunk_index];
  h.instance = C.slot0 + h.slot;
  const ProgDesc& D = S.progs[S.slots[h.instance].prog];
  h.G = D.G;
  h.W = D.W;
  h.NI = D.NI;
  h.n_global = D.n_global;
  uint32_t aid = 0;
  for (uint32_t a = 0; a < D.n_arrays; ++a) {
    const uint32_t cb = D.cellbase[a];
    if (cb != 0xFFFFFFFFu && h.cellkey >= cb && h.cellkey - cb < D.size[a]) aid = a;
  }
  h.aid = aid;
  h.cell = h.cellkey - D.cellbase[aid];
  return h;
}

__device__ __forceinline__ void push_long(const SegParams& S, u64 s, u64 e, bool inter) {
  const u64 q = atomicAdd(S.long_count, 1ull);
  if (q < S.long_cap) {
    S.longq[2 * q] = s;
    S.longq[2 * q + 1] = e | ((u64)(inter ? 1u : 0u) << 63);
  }
}

__global__ __launch_bounds__(256) void seg_check_kernel(SegParams S) {
  const u64 n = *S.n_ptr;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t low = S.bg + S.bk;
  const uint32_t gmask = (1u << S.bg) - 1u;
  // block-uniform rounds, so the whole wave reaches the ballots below
  for (u64 base = (u64)blockIdx.x * blockDim.x; base < n; base += (u64)gridDim.x * blockDim.x) {
    const u64 i = base + threadIdx.x;
    bool has_intra = false, has_inter = false;
    SegHead H;
    PendingRec pa, pb;
    if (i < n) {
      const u64 k = S.keys[i];
      const bool sub_head = i == 0 || S.keys[i - 1] != k;
      if (sub_head) {
        const bool head = i == 0 || (S.keys[i - 1] >> low) != (k >> low);
        H = seg_head(S, k);
        const u64 e = run_end(S.keys, i, n, 0);
        if (e - i >= 2) {
          if (e - i <= SEG_SHORT) {
            const u64* vals = S.vals;
            has_intra = intra_check([vals](u64 j) { return vals[j]; }, i, e, &pa.label, &pa.rw, &pa.ww);
            pa.gid = H.gid; pa.interval = H.interval; pa.aid = H.aid; pa.cell = H.cell; pa.cellkey = H.cellkey;
            pa.lidbase = H.gid * H.W;
          } else {
            push_long(S, i, e, false);
          }
        }
        if (head && H.G > 1 && H.aid < H.n_global) {
          const u64 f = run_end(S.keys, i, n, low);
          if (f - i >= 2) {
            if (f - i <= SEG_SHORT) {
              has_inter = inter_check(S.keys, S.vals, i, f, S.bk, gmask, H.W, &pb.label, &pb.rw, &pb.ww);
              pb.gid = H.gid; pb.interval = 0; pb.aid = H.aid; pb.cell = H.cell; pb.cellkey = H.cellkey;
              pb.lidbase = 0;
            } else {
              push_long(S, i, f, true);
            }
          }
        }
      }
    }
    const u64 m1 = __ballot(has_intra), m2 = __ballot(has_inter);
    const uint32_t c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
    if (c1 + c2 == 0) continue;
    const u64 rbase = wave_reserve(S.out.rec_count, c1 + c2, lane);
    const u64 below = (1ull << lane) - 1ull;
    RecKey K = {S.bs, S.bc, has_intra || has_inter ? H.G : 1u, has_intra || has_inter ? H.NI : 1u};
    if (has_intra) store_record(S.out, K, rbase + (u64)__popcll(m1 & below), H.slot, H.instance, pa, false);
    if (has_inter) store_record(S.out, K, rbase + c1 + (u64)__popcll(m2 & below), H.slot, H.instance, pb, true);
  }
}

// minimum over the workgroup (256 lanes, 4 waves); sh holds 4 words
__device__ __forceinline__ u64 block_min_u64(u64 v, u64* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, off), hi = __shfl_xor((uint32_t)(v >> 32), off);
    const u64 o = ((u64)hi << 32) | lo;
    v = o < v ? o : v;
  }
  if ((threadIdx.x & 63u) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  u64 r = sh[0];
  for (uint32_t w = 1; w < (blockDim.x >> 6); ++w) r = sh[w] < r ? sh[w] : r;
  __syncthreads();
  return r;
}

// Long runs queued by seg_check_kernel: one workgroup per run, both passes
// split over its lanes and merged with block minima.
__global__ __launch_bounds__(256) void seg_long_kernel(SegParams S) {
  __shared__ u64 sh[4];
  const u64 total = *S.long_count;
  const u64 nq = total < S.long_cap ? total : S.long_cap;
  const uint32_t gmask = (1u << S.bg) - 1u;
  for (u64 q = blockIdx.x; q < nq; q += gridDim.x) {
    const u64 s = S.longq[2 * q], ew = S.longq[2 * q + 1];
    const bool inter = (ew >> 63) != 0;
    const u64 e = ew & ~(1ull << 63);
    const SegHead H = seg_head(S, S.keys[s]);
    Pass1 p1 = pass1_init();
    for (u64 i = s + threadIdx.x; i < e; i += blockDim.x) {
      const u64 p = S.vals[i];
      uint32_t id = pay_lid(p);
      if (inter) id += ((uint32_t)(S.keys[i] >> S.bk) & gmask) * H.W;
      pass1_add(p1, id, pay_w(p), pay_val(p));
    }
    p1.r1 = (uint32_t)block_min_u64(p1.r1, sh);
    p1.wmin = block_min_u64(p1.wmin, sh);
    const uint32_t w1 = p1.wmin == ~0ull ? NONE32 : (uint32_t)(p1.wmin >> 32);
    const int32_t x1 = (int32_t)((uint32_t)p1.wmin ^ 0x80000000u);
    PendingRec pr;
    bool has = false;
    if (!inter) {
      Intra2 p2 = intra2_init();
      for (u64 i = s + threadIdx.x; i < e; i += blockDim.x) {
        const u64 p = S.vals[i];
        intra2_add(p2, pay_lid(p), pay_w(p), pay_val(p), p1.r1, w1, x1);
      }
      p2.r2 = (uint32_t)block_min_u64(p2.r2, sh);
      p2.w2 = (uint32_t)block_min_u64(p2.w2, sh);
      p2.q = (uint32_t)block_min_u64(p2.q, sh);
      p2.multi1 = block_min_u64(p2.multi1 ? 0u : 1u, sh) == 0u ? 1u : 0u;
      if (threadIdx.x == 0) {
        has = intra_finish(p1, p2, &pr.label, &pr.rw, &pr.ww);
        pr.gid = H.gid; pr.interval = H.interval; pr.lidbase = H.gid * H.W;
      }
    } else {
      const uint32_t gr1 = p1.r1 == NONE32 ? NONE32 : p1.r1 / H.W;
      const uint32_t g1 = w1 == NONE32 ? NONE32 : w1 / H.W;
      Inter2 p2 = inter2_init();
      for (u64 i = s + threadIdx.x; i < e; i += blockDim.x) {
        const u64 p = S.vals[i];
        const uint32_t g = (uint32_t)(S.keys[i] >> S.bk) & gmask;
        inter2_add(p2, g * H.W + pay_lid(p), g, pay_w(p), pay_val(p), gr1, w1, g1, x1);
      }
      p2.r1p = (uint32_t)block_min_u64(p2.r1p, sh);
      p2.w1p = (uint32_t)block_min_u64(p2.w1p, sh);
      p2.q = (uint32_t)block_min_u64(p2.q, sh);
      p2.A = (uint32_t)block_min_u64(p2.A, sh);
      p2.multi1 = block_min_u64(p2.multi1 ? 0u : 1u, sh) == 0u ? 1u : 0u;
      if (threadIdx.x == 0) {
        has = inter_finish(p1, p2, H.W, &pr.label, &pr.rw, &pr.ww);
        pr.gid = H.gid; pr.interval = 0; pr.lidbase = 0;
      }
    }
    if (threadIdx.x == 0 && has) {
      pr.aid = H.aid; pr.cell = H.cell; pr.cellkey = H.cellkey;
      const RecKey K = {S.bs, S.bc, H.G, H.NI};
      store_record(S.out, K, atomicAdd(S.out.rec_count, 1ull), H.slot, H.instance, pr, inter);
    }
  }
}

// ---------------------------------------------------------------------------
// ordered output and summaries
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void rec_gather_kernel(GatherParams Gp) {
  const u64 n = *Gp.n_ptr;
  const u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  bool valid = p < n;
  uint32_t slot = 0;
  bool race = false, benign = false;
  if (valid) {
    const rc_record_dev r = Gp.staging[Gp.idx[p]];
    const u64 out = *Gp.out_base + p;
    slot = r.instance - Gp.chunks[*Gp.chunk_index].slot0;
    const uint32_t label = r.array_label >> 16;
    race = (label & 3u) != 0u;
    benign = label == 4u;
    if (out < Gp.cap) Gp.out[out] = r;
    else atomicOr(&Gp.inst_flags[slot], 1u);
  }
  // aggregate per-instance counts over the wave when it holds one instance
  const uint32_t s0 = __builtin_amdgcn_readfirstlane(slot);
  const u64 same = __ballot(!valid || slot == s0);
  if (same == ~0ull) {
    const uint32_t nr = (uint32_t)__popcll(__ballot(race)), nb = (uint32_t)__popcll(__ballot(benign));
    if (lane == 0) {
      if (nr) atomicAdd(&Gp.inst_race[s0], nr);
      if (nb) atomicAdd(&Gp.inst_benign[s0], nb);
    }
  } else if (valid) {
    if (race) atomicAdd(&Gp.inst_race[slot], 1u);
    if (benign) atomicAdd(&Gp.inst_benign[slot], 1u);
  }
}


// entries past a buffer's capacity were dropped (and flagged): later kernels
// see at most `cap`
__global__ void clamp_count_kernel(u64* n_ptr, u64 cap, uint32_t* status, uint32_t bit) {
  if (*n_ptr > cap) {
    *n_ptr = cap;
    *status |= bit;
  }
}

__global__ __launch_bounds__(256) void finalize_kernel(FinalParams F) {
  const ChunkDesc C = F.chunks[*F.chunk_index];
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= C.n_slots) return;
  const uint32_t W = F.progs[F.slots[C.slot0 + s].prog].W;
  rc_summary_dev o;
  o.n_accesses = F.inst_acc[s];
  o.n_race_cells = F.inst_race[s];
  o.n_benign_cells = F.inst_benign[s];
  o.n_intervals = F.inst_intervals[s];
  const u64 f = F.inst_fault[s];
  if (f == ~0ull) {
    o.status = 0;
    o.fault_gid = o.fault_pc = o.fault_tid = 0xFFFFFFFFu;
  } else {
    const uint32_t g = (uint32_t)(f >> 38), fpc = (uint32_t)(f >> 26) & 4095u, lid = (uint32_t)(f >> 16) & 1023u;
    o.status = (int32_t)(f & 7u);
    o.fault_gid = g;
    o.fault_pc = fpc;
    o.fault_tid = g * W + lid;
  }
  o.flags = F.inst_flags[s];
  F.out[C.slot0 + s] = o;
}

// Start of a chunk: clear its counters (and the overlay pool when the
// overlay versions wrap).  One block per 256 instances; block 0 also clears
// the scalar counters.
__global__ __launch_bounds__(256) void chunk_setup_kernel(SetupParams P) {
  const ChunkDesc C = P.chunks[*P.chunk_index];
  const uint32_t t = threadIdx.x;
  if (blockIdx.x == 0 && t < 8) P.counters[t] = 0ull;       // log, records, queue words
  if (blockIdx.x == 0 && t < N_WCLASS) P.queue[t] = 0u;
  for (uint32_t s = blockIdx.x * blockDim.x + t; s < P.max_slots; s += gridDim.x * blockDim.x) {
    P.inst_acc[s] = 0ull;
    P.inst_fault[s] = ~0ull;
    P.inst_intervals[s] = 0u;
    P.inst_race[s] = 0u;
    P.inst_benign[s] = 0u;
    P.inst_flags[s] = 0u;
  }
  if (C.clear_overlay)
    for (u64 c = (u64)blockIdx.x * blockDim.x + t; c < P.overlay_cells; c += (u64)gridDim.x * blockDim.x)
      P.overlay[c] = 0ull;
}

// Start of a call: the workspace header (magic, context, generation, pool
// size) tells whether the overlay pool still holds only versioned cells from
// this context's earlier calls; if not (a new or reused buffer), the pool is
// cleared before anything reads it.
__global__ void ws_validate_kernel(u64* header, u64 magic, u64 ctx_id, u64 gen, u64 pool_cells, uint32_t* dirty) {
  const bool ok = header[0] == magic && header[1] == ctx_id && header[2] == gen && header[3] >= pool_cells;
  *dirty = ok ? 0u : 1u;
  header[0] = magic;
  header[1] = ctx_id;
  header[2] = gen + 1ull;
  header[3] = pool_cells;   // bytes past this pool will hold other data
}

__global__ __launch_bounds__(256) void pool_clear_kernel(u64* pool, u64 cells, const uint32_t* dirty) {
  if (*dirty == 0u) return;
  for (u64 c = (u64)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (u64)gridDim.x * blockDim.x) pool[c] = 0ull;
}

// End of a chunk: advance the output base and the chunk index.
__global__ void chunk_advance_kernel(u64* out_base, const u64* rec_n, uint32_t* chunk_index) {
  *out_base += *rec_n;
  *chunk_index += 1u;
}

__global__ __launch_bounds__(256) void fill_u64_kernel(u64* p, u64 n, u64 v) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = v;
}
__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* p, u64 n, uint32_t v) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = v;
}

// final memory of one global array: highest writing work-group wins
__global__ __launch_bounds__(256) void final_merge_kernel(FinalMemParams M) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M.size) return;
  int32_t v = M.bind == BIND_SEEDED ? seeded_cell(M.seed, M.array_id, c, M.lo, M.hi) : M.dptr[c];
  if (M.rw) {
    for (uint32_t g = 0; g < M.G; ++g) {
      const u64 w = M.overlay[(size_t)g * M.overlay_cells + M.offset + c];
      if ((uint32_t)(w >> 42) >= M.epoch) v = (int32_t)(uint32_t)w;
    }
  }
  M.out[c] = v;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(u64 n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

static void set_lds_attr() {
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rc_interp_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
}

hipError_t launch_interp(const PassParams& P, uint32_t blocks, uint32_t threads, size_t lds_bytes, hipStream_t st) {
  set_lds_attr();
  hipLaunchKernelGGL(rc_interp_kernel, dim3(blocks), dim3(threads), lds_bytes, st, P);
  return hipGetLastError();
}

int interp_occupancy(uint32_t threads, size_t lds_bytes) {
  set_lds_attr();
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rc_interp_kernel, (int)threads, lds_bytes) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_setup(const SetupParams& P, hipStream_t st) {
  uint32_t nb = blocks_for(std::max<u64>(P.max_slots, 1), 256);
  if (nb < 1024) nb = 1024;
  hipLaunchKernelGGL(chunk_setup_kernel, dim3(nb), dim3(256), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_ws_validate(u64* header, u64 magic, u64 ctx_id, u64 gen, u64* pool, u64 pool_cells,
                              uint32_t* dirty, hipStream_t st) {
  hipLaunchKernelGGL(ws_validate_kernel, dim3(1), dim3(1), 0, st, header, magic, ctx_id, gen, pool_cells, dirty);
  uint32_t nb = blocks_for(std::max<u64>(pool_cells, 1), 256);
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(pool_clear_kernel, dim3(nb), dim3(256), 0, st, pool, pool_cells, (const uint32_t*)dirty);
  return hipGetLastError();
}

hipError_t launch_advance(u64* out_base, const u64* rec_n, uint32_t* chunk_index, hipStream_t st) {
  hipLaunchKernelGGL(chunk_advance_kernel, dim3(1), dim3(1), 0, st, out_base, rec_n, chunk_index);
  return hipGetLastError();
}

hipError_t launch_region_tiles(const uint32_t* counts, uint32_t* tiles, u64 n_regions, hipStream_t st) {
  hipLaunchKernelGGL(region_tiles_kernel, dim3(blocks_for(n_regions + 1, 256)), dim3(256), 0, st, counts, tiles,
                     n_regions);
  return hipGetLastError();
}

// exclusive scan in place; tmp needs scan_tmp_words(m) words
size_t scan_tmp_words(u64 m) {
  size_t words = 0;
  while (m > SCAN_BLOCK) {
    m = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    words += m;
  }
  return words + 1;
}

static void scan_excl(uint32_t* data, u64 m, uint32_t* tmp, hipStream_t st) {
  if (m <= SCAN_BLOCK) {
    hipLaunchKernelGGL(scan_block_kernel, dim3(1), dim3(256), 0, st, data, m, (const uint32_t*)nullptr);
    return;
  }
  const uint32_t nb = blocks_for(m, SCAN_BLOCK);
  uint32_t* sums = tmp;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(256), 0, st, (const uint32_t*)data, m, sums);
  scan_excl(sums, nb, tmp + nb, st);
  hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(256), 0, st, data, m, (const uint32_t*)sums);
}

size_t sort_hist_words(u64 cap) {
  const u64 nb = (cap + RS_TILE - 1) / RS_TILE;
  const u64 m = 256ull * (nb ? nb : 1);
  return m + scan_tmp_words(m);
}

// upper bound of the tiles the first (segmented) pass walks
static u64 seg_blocks(u64 n_regions, u64 cap) { return (cap + RS_TILE - 1) / RS_TILE + n_regions; }

size_t sort_log_hist_words(u64 n_regions, u64 cap) {
  const u64 nb = std::max<u64>(seg_blocks(n_regions, cap), (cap + RS_TILE - 1) / RS_TILE);
  const u64 m = 256ull * (nb ? nb : 1);
  return m + scan_tmp_words(std::max<u64>(m, n_regions + 1));
}

template <typename V>
static hipError_t sort_pairs_impl(u64* k0, V* v0, u64* k1, V* v1, const u64* n_ptr, u64 cap, uint32_t nbits,
                                  const uint32_t* seg_count, const u64* seg_base, const uint32_t* tiles,
                                  u64 n_regions, uint32_t* hist, uint32_t dbits, hipStream_t st,
                                  int* result_in_second, uint32_t start_bit = 0) {
  u64 *ka = k0, *kb = k1;
  V *va = v0, *vb = v1;
  int passes = 0;
  if (dbits < 1 || dbits > 8) dbits = 8;
  // passes of dbits each over bits [start_bit, nbits); a segmented input
  // always takes at least one pass, which also makes it dense
  const uint32_t want = seg_count ? std::max(nbits, start_bit + 1) : nbits;
  for (uint32_t shift = start_bit; shift < want; shift += dbits) {
    RsIn in;
    memset(&in, 0, sizeof in);
    in.n_ptr = n_ptr;
    in.dbits = dbits;
    u64 nbl;
    if (passes == 0 && seg_count) {
      in.seg_count = seg_count;
      in.seg_base = seg_base;
      in.tiles = tiles;
      in.n_regions = (uint32_t)n_regions;
      nbl = seg_blocks(n_regions, cap);
    } else {
      nbl = blocks_for(cap ? cap : 1, RS_TILE);
    }
    const uint32_t nb = (uint32_t)(nbl ? nbl : 1);
    const u64 m = (1ull << dbits) * nb;
    uint32_t* tmp = hist + m;
    hipLaunchKernelGGL(rs_hist_kernel, dim3(nb), dim3(RS_THREADS), 0, st, (const u64*)ka, in, shift, hist, nb);
    scan_excl(hist, m, tmp, st);
    hipLaunchKernelGGL(rs_scatter_kernel<V>, dim3(nb), dim3(RS_THREADS), 0, st, (const u64*)ka, (const V*)va, kb,
                       vb, in, shift, (const uint32_t*)hist, nb);
    u64* tk = ka; ka = kb; kb = tk;
    V* tv = va; va = vb; vb = tv;
    ++passes;
  }
  *result_in_second = passes & 1;
  return hipGetLastError();
}

hipError_t sort_log(u64* k0, u64* v0, u64* k1, u64* v1, const u64* n_ptr, u64 cap, uint32_t nbits,
                    uint32_t start_bit, const uint32_t* seg_count, const u64* seg_base, uint32_t* tiles,
                    u64 n_regions, uint32_t* hist, uint32_t dbits, hipStream_t st, int* in_second) {
  // the number of entries, and the regions' tile prefix
  hipLaunchKernelGGL(sum_u32_kernel, dim3(n_regions > 65536 ? 1024 : (uint32_t)blocks_for(n_regions, 256)),
                     dim3(256), 0, st, seg_count, n_regions, (u64*)n_ptr);
  hipLaunchKernelGGL(region_tiles_kernel, dim3(blocks_for(n_regions + 1, 256)), dim3(256), 0, st, seg_count,
                     tiles, n_regions);
  scan_excl(tiles, n_regions + 1, hist, st);
  return sort_pairs_impl<u64>(k0, v0, k1, v1, n_ptr, cap, nbits, seg_count, seg_base, tiles, n_regions, hist, dbits,
                              st, in_second, start_bit);
}
hipError_t sort_pairs_u32(u64* k0, uint32_t* v0, u64* k1, uint32_t* v1, const u64* n_ptr, u64 cap,
                          uint32_t nbits, uint32_t* hist, hipStream_t st, int* in_second) {
  return sort_pairs_impl<uint32_t>(k0, v0, k1, v1, n_ptr, cap, nbits, nullptr, nullptr, nullptr, 0, hist, 8, st,
                                   in_second);
}

hipError_t launch_seg_check(const SegParams& S, u64 cap, hipStream_t st) {
  // the entry count is on the device: a fixed grid walks it in rounds
  uint32_t blocks = blocks_for(cap ? cap : 1, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(seg_check_kernel, dim3(blocks), dim3(256), 0, st, S);
  uint32_t lblocks = (uint32_t)std::min<u64>(S.long_cap ? S.long_cap : 1, 2048);
  hipLaunchKernelGGL(seg_long_kernel, dim3(lblocks), dim3(256), 0, st, S);
  return hipGetLastError();
}
hipError_t launch_gather(const GatherParams& G, u64 cap, hipStream_t st) {
  hipLaunchKernelGGL(rec_gather_kernel, dim3(blocks_for(cap ? cap : 1, 256)), dim3(256), 0, st, G);
  return hipGetLastError();
}
hipError_t launch_finalize(const FinalParams& F, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(std::max<u64>(F.max_slots, 1), 256)), dim3(256), 0, st, F);
  return hipGetLastError();
}
hipError_t launch_fill_u64(u64* p, u64 n, u64 v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t nb = blocks_for(n, 256);
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(nb), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, u64 n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t nb = blocks_for(n, 256);
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(nb), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_clamp(u64* n_ptr, u64 cap, uint32_t* status, uint32_t bit, hipStream_t st) {
  hipLaunchKernelGGL(clamp_count_kernel, dim3(1), dim3(1), 0, st, n_ptr, cap, status, bit);
  return hipGetLastError();
}
hipError_t launch_final_merge(const FinalMemParams& M, hipStream_t st) {
  hipLaunchKernelGGL(final_merge_kernel, dim3(blocks_for(M.size, 256)), dim3(256), 0, st, M);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// triage features: one wave per instance copies the program's static part and
// bins the first 256 initial cells of global arrays 0 and 1 into eighths of
// their value range (seeded: [lo, hi); bound buffers: the int32 range)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void features_kernel(const FeatItem* items, const FeatProg* progs, uint32_t n,
                                                       float* out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t i = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  if (i >= n) return;
  const FeatItem it = items[i];
  const FeatProg* P = progs + it.prog;
  float* row = out + i * N_FEAT;
  for (uint32_t k = lane; k < (uint32_t)N_FEAT_STATIC; k += 64u) row[k] = P->stat[k];
  for (uint32_t j = 0; j < 2; ++j) {
    const FeatArray A = P->arr[j];
    uint32_t count = 0;   // lane b < 8 counts bin b
    if (A.present) {
      const uint32_t cells = A.size < 256u ? A.size : 256u;
      for (uint32_t c0 = 0; c0 < cells; c0 += 64u) {
        const uint32_t c = c0 + lane;
        int bin = -1;
        if (c < cells) {
          if (A.bind == BIND_SEEDED) {
            // offset of the draw in [lo, hi) mod 2^32 (a 2^32-wide range wraps in int32)
            const uint32_t u = (uint32_t)seeded_cell(it.seed, j, c, A.lo, A.hi) - (uint32_t)(uint64_t)A.lo;
            bin = (int)((uint64_t)u * 8ull / (uint64_t)(A.hi - A.lo));
          } else {
            bin = (int)(((uint32_t)A.dptr[c] ^ 0x80000000u) >> 29);
          }
        }
        for (int b = 0; b < 8; ++b) {
          const uint64_t m = __ballot(bin == b);
          if (lane == (uint32_t)b) count += (uint32_t)__popcll(m);
        }
      }
    }
    if (lane < 8u) row[N_FEAT_STATIC + 8u * j + lane] = (float)count / 256.f;
  }
}

hipError_t launch_features(const FeatItem* items, const FeatProg* progs, uint32_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(features_kernel, dim3((n + 3u) / 4u), dim3(256), 0, st, items, progs, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ranking keys: score descending, then index ascending, as one u64
// ---------------------------------------------------------------------------
// key = (descending score) << idx_bits | index, so a sort by the low
// 32 + idx_bits bits orders by score, then index
__global__ __launch_bounds__(256) void rank_keys_kernel(const float* scores, uint32_t n, uint32_t idx_bits, u64* keys,
                                                        uint32_t* vals, u64* n_ptr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *n_ptr = n;
  if (i >= n) return;
  const float f = scores[i];
  uint32_t b = __float_as_uint(f);
  // monotone map of float order onto u32 order; NaN ranks below every number
  uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  if (f != f) asc = 0u;
  keys[i] = ((u64)(~asc) << idx_bits) | i;
  vals[i] = i;
}

hipError_t launch_rank_keys(const float* scores, uint32_t n, uint32_t idx_bits, u64* keys, uint32_t* vals,
                            u64* n_ptr, hipStream_t st) {
  hipLaunchKernelGGL(rank_keys_kernel, dim3(blocks_for(n ? n : 1, 256)), dim3(256), 0, st, scores, n, idx_bits, keys,
                     vals, n_ptr);
  return hipGetLastError();
}

}  // namespace rc
