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

#include "item_rt.h"
#include "kernels.h"

namespace rc {

// The bytecode interpreter: one item's program, instruction by instruction,
// on the Item runtime.  Private variables live in LDS (register-major, so a
// wave reads 64 consecutive dwords); control flow keeps a mask bit per
// nesting depth.
// NR == 0: private variables in LDS (regs[r * WP + lid]); NR > 0: in a
// register file of NR VGPRs per lane, indexed by the instruction's (uniform)
// register number, for programs with at most NR registers.
template <int NR>
__device__ __forceinline__ void interp_item(Item& it) {
  const ItemView& P = it.P;
  int32_t* regs = it.regs;
  const uint32_t WP = it.WP, tl = it.tl, tr = it.tr, lane = it.lane, wave = it.wave;
  Ctl* ctl = it.ctl;
  uint32_t pc = 0, depth = 0, eany = 0;
  uint32_t mbits = it.real ? 1u : 0u, ebits = 0u;
  (void)lane;
  (void)WP;
  (void)tr;
  int32_t vr[NR > 0 ? NR : 1];
#pragma unroll
  for (int i = 0; i < (NR > 0 ? NR : 1); ++i) vr[i] = 0;
  auto rd = [&](uint32_t w) -> int32_t {
    if constexpr (NR > 0) return vr[w < (uint32_t)NR ? w : (uint32_t)(NR - 1)];
    else return regs[w * WP + tr];
  };
  auto wr = [&](uint32_t w, int32_t v) {
    if constexpr (NR > 0) vr[w < (uint32_t)NR ? w : (uint32_t)(NR - 1)] = v;
    else regs[w * WP + tl] = v;
  };

  auto fetch = [&](bool imm, uint32_t w) -> int32_t {
    if (imm) return (int32_t)w;
    if (w < MAX_REGS) return rd(w);
    return it.special_dyn(w);
  };

  for (;;) {
    pc = uni(pc);
    const Insn in = const_load<Insn>(P.code, pc);
    const uint32_t h = in.h, wa = in.a, wb = in.b, wc = in.c;
    const uint32_t op = h & 63u, sub = (h >> 8) & 63u, dst = (h >> 14) & 63u, spc = h >> 20;
    const bool fa = (h >> 6) & 1u, fb = (h >> 7) & 1u;
    it.stmt(spc);
    const bool active = (mbits >> depth) & 1u;

    if (op == OP_BIN || op == OP_UN) {
      // a run of arithmetic instructions (an expression's nodes) in a loop
      // of its own: the mask does not change inside it, and the state the
      // rest of the interpreter carries stays out of it
      uint32_t hh = h, xa = wa, xb = wb, hop = op, hsub = sub, hdst = dst, hspc = spc;
      bool ffa = fa, ffb = fb;
      for (;;) {
        const int32_t x = fetch(ffa, xa);
        int32_t r;
        if (hop == OP_BIN) {
          const int32_t y = fetch(ffb, xb);
          bool dz = false;
          r = alu_bin(hsub, x, y, dz);
          if (active && dz) it.raise(hspc, F_DIV);
        } else {
          r = hsub == U_MOV ? x : hsub == U_NEG ? (int32_t)(0u - (uint32_t)x) : hsub == U_BNOT ? ~x : (int32_t)(x == 0);
        }
        if (active) wr(hdst, r);
        ++pc;
        const Insn nx = const_load<Insn>(P.code, pc);
        hh = nx.h;
        hop = hh & 63u;
        if (hop != OP_BIN && hop != OP_UN) break;
        xa = nx.a; xb = nx.b;
        hsub = (hh >> 8) & 63u; hdst = (hh >> 14) & 63u; hspc = hh >> 20;
        ffa = (hh >> 6) & 1u; ffb = (hh >> 7) & 1u;
        it.stmt(hspc);
      }
    } else if (op == OP_LOAD || op == OP_STORE) {
      const int32_t idx = fetch(fa, wa);
      const int32_t val = op == OP_STORE ? fetch(fb, wb) : 0;
      int32_t v = 0;
      if (it.mem(op, wc & ~INSN_NO_STEP, idx, val, active, spc, v, (wc & INSN_NO_STEP) == 0u)) {
        it.faulted = true;
        break;
      }
      if (op == OP_LOAD && active) wr(dst, v);
      ++pc;
    } else if (op == OP_IF) {
      const int32_t c = fetch(fa, wa);
      const bool t = active && c != 0, e = active && c == 0;
      const uint32_t d1 = depth + 1u;
      mbits = (mbits & ~(1u << d1)) | ((uint32_t)t << d1);
      ebits = (ebits & ~(1u << d1)) | ((uint32_t)e << d1);
      const uint32_t any = it.group_red(t, e, false);
      if (any & 4u) { it.faulted = true; break; }
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
      if (active) wr(dst, lo);
      if ((int64_t)hi - (int64_t)lo <= 0) {
        pc = wc;
      } else {
        if (it.iter_start(spc)) { it.faulted = true; break; }
        if (it.lane == 0) ctl->loopctr[wave][sub] = 0u;
        ++pc;
      }
    } else if (op == OP_ENDFOR) {
      const int32_t lo = (int32_t)wa, hi = (int32_t)wb;
      const uint32_t iters = (uint32_t)((int64_t)hi - (int64_t)lo);
      const uint32_t ctr = uni(ctl->loopctr[wave][sub]) + 1u;
      if (it.lane == 0) ctl->loopctr[wave][sub] = ctr;
      if (active) wr(dst, (int32_t)((uint32_t)lo + ctr));
      if (ctr < iters && it.iter_start(spc)) { it.faulted = true; break; }
      pc = ctr < iters ? wc : pc + 1u;
    } else if (op == OP_BARRIER) {
      if (it.barrier(active, spc)) { it.faulted = true; break; }
      ++pc;
    } else if (op == OP_ASSERT || op == OP_ASSUME) {
      const int32_t c = fetch(fa, wa);
      if (active && c == 0) it.raise(spc, op == OP_ASSERT ? F_ASSERT : F_ASSUME);
      ++pc;
    } else {  // OP_END
      if (it.end()) it.faulted = true;
      break;
    }
  }
}

__global__ __launch_bounds__(1024) void rc_interp_kernel(PassParams PP) {
  run_items(PP, [](Item& it) { interp_item<0>(it); });
}

// the same for calls whose programs all have at most 16 registers
__global__ __launch_bounds__(1024) void rc_interp_vreg_kernel(PassParams PP) {
  run_items(PP, [](Item& it) { interp_item<VREG_FILE>(it); });
}

// ---------------------------------------------------------------------------
// Spilled intervals of one-group programs (ProgDesc::sc), after the
// interpreter: persistent blocks take the chunk's instances from a queue,
// in the planner's order (largest static log bound first);
// for each one whose program has sc set, the block walks its region's
// trailers back from the end, checks every spilled interval in LDS
// (sc_check), and sets the region's count to zero.  Its records carry the interval's ranks and counts like those
// of an interval closed in LDS.  LDS: the control block, then the work area.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SC_THREADS) void sc_group_kernel(ScParams S) {
  Ctl* ctl = reinterpret_cast<Ctl*>(rc_smem);
  const uint32_t tl = threadIdx.x;
  const ChunkDesc C = const_load<ChunkDesc>(S.chunks, const_load<uint32_t>(S.chunk_index, 0));
  const rc_record_out R = const_load<rc_record_out>(S.rec, 0);
  if (tl == 0) ctl->rc_cur = ctl->rc_end = 0ull;   // no record slots yet
  // the work area: the window table, field by field (cleared once, kept
  // clean), the touched-cell bitmap, the bucket counters
  u64* wmin = reinterpret_cast<u64*>(rc_smem + SC_CTL_BYTES);
  uint32_t* r1 = reinterpret_cast<uint32_t*>(wmin + SC_WIN);
  uint32_t* r2 = r1 + SC_WIN;
  uint32_t* w2 = r2 + SC_WIN;
  uint32_t* q = w2 + SC_WIN;
  uint32_t* bits = q + SC_WIN;
  uint32_t* cnt = bits + SC_WORDS;
  for (uint32_t i = tl; i < SC_WIN; i += SC_THREADS) {
    wmin[i] = ~0ull;
    r1[i] = r2[i] = w2[i] = q[i] = NONE32;
  }
  for (uint32_t i = tl; i < SC_WORDS; i += SC_THREADS) bits[i] = 0u;
  __syncthreads();
  for (;;) {
    if (tl == 0) ctl->item = atomicAdd(S.queue, 1u);
    __syncthreads();
    const uint32_t taken = uni(ctl->item);
    __syncthreads();
    if (taken >= C.n_slots) {
      // the block's unused record slots
      const u64 a = ctl->rc_cur, b = ctl->rc_end;
      for (u64 q = a + tl; q < b && q < R.rec_cap; q += SC_THREADS) RC_GLOBAL(u64, R.rec_keys)[q] = ~0ull;
      if (tl == 0 && b > a)
        __hip_atomic_fetch_add(RC_GLOBAL(unsigned long long, R.rec_dead), (unsigned long long)(b - a),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // the chunk's slots largest static log bound first
    const uint32_t rel = const_load<uint32_t>(S.order, C.slot0 + taken);
    const uint32_t instance = C.slot0 + rel;
    const SlotDesc Sd = const_load<SlotDesc>(S.slots, instance);
    const ProgDesc D = const_load<ProgDesc>(S.progs, Sd.prog);
    if (!D.sc) continue;
    u64 pos = uni(S.wg_count[Sd.wg_base]);
    if (pos == 0u) continue;
    u64* region = S.log_keys + Sd.log_base;
    ScEnv E;
    E.ends = S.ends + (u64)blockIdx.x * SC_NB_MAX;
    E.cells = D.n_cells;
    E.nthr = SC_THREADS;
    E.wmin = wmin; E.r1 = r1; E.r2 = r2; E.w2 = w2; E.q = q;
    E.bits = bits;
    E.cnt = cnt;
    E.slot = rel;
    E.instance = instance;
    E.n_arrays = D.n_arrays;
    E.arrays = D.arrays;
    E.recp = S.rec;
    E.K = RecKey{S.bs, S.bc, D.G, D.NI};
    while (pos > 0u) {
      const u64 t = region[pos - 1u];
      const uint32_t cnt = uni((uint32_t)t), interval = uni((uint32_t)(t >> 32));
      if ((u64)cnt >= pos) break;   // (a region that overflowed: already reported)
      const u64 start = pos - 1u - cnt;
      E.src = region + start;
      E.dst = S.log_vals + Sd.log_base + start;
      E.interval = interval;
      const uint32_t kb = cnt >= 2u ? sc_check(E, cnt) : 0u;
      if (R.rank_keys && tl == 0 && kb)
        RC_GLOBAL(uint32_t, R.scope_cnt)[((u64)rel << S.bs) | interval] = kb;
      pos = start;
    }
    // the region is consumed: in a call that also has a global pass (other
    // programs log globally), that pass must not take its packed words for
    // (key, payload) entries
    __syncthreads();   // (every thread has read the count)
    if (tl == 0) S.wg_count[Sd.wg_base] = 0u;
  }
}

// LDS of a group check block: control block, window table (8 + 4 x 4 bytes
// a cell), bitmap, counters
constexpr size_t SC_LDS_BYTES = SC_CTL_BYTES + SC_WIN * 24u + SC_WORDS * 4 + SC_NB_MAX * 4;

hipError_t launch_sc_group(const ScParams& S, uint32_t blocks, hipStream_t st) {
  hipLaunchKernelGGL(sc_group_kernel, dim3(blocks), dim3(SC_THREADS), SC_LDS_BYTES, st, S);
  return hipGetLastError();
}

int sc_group_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sc_group_kernel, (int)SC_THREADS, SC_LDS_BYTES) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

// ---------------------------------------------------------------------------
// exclusive scan of u32 arrays (three-level, 1024 elements per block)
// ---------------------------------------------------------------------------
constexpr uint32_t SCAN_BLOCK = 1024;

__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* sh, uint32_t* total) {
  // the values of the first 256 threads (any threads beyond hold 0): scan
  // via waves + LDS; sh holds a word per wave of the block
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

// length of level `level` of a scan whose level-0 length is *m_ptr: each
// level holds one sum per SCAN_BLOCK elements of the level below
__device__ __forceinline__ uint64_t scan_level_len(const u64* m_ptr, uint32_t level) {
  uint64_t m = *m_ptr;
  for (uint32_t l = 0; l < level; ++l) m = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
  return m;
}

// The same two steps when the length is known only on the device; a fixed
// grid walks the level's blocks.
__global__ __launch_bounds__(256) void scan_reduce_dev_kernel(const uint32_t* in, const u64* m_ptr,
                                                              uint32_t level, uint32_t* sums) {
  __shared__ uint32_t sh[4];
  const uint64_t m = scan_level_len(m_ptr, level);
  for (uint64_t j = blockIdx.x; j * SCAN_BLOCK < m; j += gridDim.x) {
    const uint64_t base = j * SCAN_BLOCK + threadIdx.x * 4u;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) if (base + k < m) s += in[base + k];
    uint32_t total;
    block_excl_scan_256(s, sh, &total);
    if (threadIdx.x == 0) sums[j] = total;
  }
}

__global__ __launch_bounds__(256) void scan_block_dev_kernel(uint32_t* data, const u64* m_ptr, uint32_t level,
                                                             const uint32_t* offs) {
  __shared__ uint32_t sh[4];
  const uint64_t m = scan_level_len(m_ptr, level);
  for (uint64_t j = blockIdx.x; j * SCAN_BLOCK < m; j += gridDim.x) {
    const uint64_t base = j * SCAN_BLOCK + threadIdx.x * 4u;
    uint32_t v[4];
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) { v[k] = base + k < m ? data[base + k] : 0u; s += v[k]; }
    uint32_t total;
    uint32_t ex = block_excl_scan_256(s, sh, &total);
    if (offs) ex += offs[j];
    for (int k = 0; k < 4; ++k) {
      if (base + k < m) data[base + k] = ex;
      ex += v[k];
    }
  }
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
// the LDS-staged scatter ranks a tile with 512 threads (8 waves, 8 rounds):
// its 70 KB of LDS allow two blocks, 16 waves, per CU
constexpr uint32_t RSL_THREADS = 512, RSL_WAVES = RSL_THREADS / 64, RSL_ROUNDS = RS_TILE / RSL_THREADS;

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
  // filter pass: the 1-bit digit is 0 for entries of cells whose owner word
  // says OWNER_SHARED (kept) and 1 otherwise; the cell key is key >> keep_low
  // (keep_bc bits), the slot the bits above it
  const uint32_t* keep;
  uint32_t keep_stride, keep_low, keep_bc, keep_bk;
};

__device__ __forceinline__ uint32_t rs_digit(const RsIn& in, u64 k, uint32_t shift, uint32_t dmask) {
  if (in.keep) {
    const u64 cmask = in.keep_bc >= 32 ? 0xFFFFFFFFull : ((1ull << in.keep_bc) - 1ull);
    const u64 cell = (k >> in.keep_low) & cmask;
    const u64 slot = k >> (in.keep_low + in.keep_bc);
    return in.keep[slot * in.keep_stride + cell] == OWNER_SHARED ? 0u : 1u;
  }
  return (uint32_t)(k >> shift) & dmask;
}

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

// tiles of a pass: the dense entry count in tiles, or the regions' total
__device__ __forceinline__ uint32_t rs_ntiles(const RsIn& in) {
  if (in.seg_count == nullptr) return (uint32_t)((*in.n_ptr + RS_TILE - 1) / RS_TILE);
  return in.tiles[in.n_regions];
}

// length of a pass's digit-major histogram, (2^dbits) x tiles, for the
// device-sized scan
__global__ void rs_hist_len_kernel(RsIn in, u64* m_out) {
  *m_out = (u64)(1u << in.dbits) * rs_ntiles(in);
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

// Count one wave round's digits into LDS counters: an atomic per lane, or
// one for the round when its lanes all hold the same digit (sorted inputs
// make high digits nearly constant within a tile).  Counts need no ranks.
__device__ __forceinline__ void wave_count_digits(uint32_t* cnt, uint32_t d, bool valid, uint32_t lane) {
  const u64 vm = __ballot(valid);
  if (vm == 0ull) return;
  const uint32_t first = (uint32_t)__ffsll((long long)vm) - 1u;
  const uint32_t d0 = __builtin_amdgcn_readlane(d, first);
  if (__ballot(valid && d != d0) == 0ull) {
    if (lane == first) atomicAdd(&cnt[d0], (uint32_t)__popcll(vm));
  } else if (valid) {
    atomicAdd(&cnt[d], 1u);
  }
}

// Digit counts of one tile: an LDS atomic per entry, or one per wave round
// whose lanes all hold the same digit.
// The histogram is digit-major over the pass's live tiles (the count read
// on the device), so its scan and the grids scale with the entries, not
// with the capacity; a fixed grid walks the tiles.
__global__ __launch_bounds__(256) void rs_hist_kernel(const u64* keys, RsIn in, uint32_t shift, uint32_t* hist) {
  __shared__ uint32_t h[256];
  const uint32_t t = threadIdx.x, lane = t & 63u;
  const uint32_t dmask = (1u << in.dbits) - 1u;
  const uint32_t nt = rs_ntiles(in);
  for (uint32_t b = blockIdx.x; b < nt; b += gridDim.x) {
    h[t] = 0;
    __syncthreads();
    u64 start;
    uint32_t count;
    rs_tile(in, b, &start, &count);
    // the tile's keys are loaded before any is counted, so each thread has
    // all its loads in flight at once (the pass is bound by memory latency)
    u64 kr[RS_ROUNDS];
#pragma unroll
    for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
      const uint32_t i = r * RS_THREADS + t;
      kr[r] = i < count ? keys[start + i] : 0ull;
    }
#pragma unroll
    for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
      const bool valid = r * RS_THREADS + t < count;
      wave_count_digits(h, valid ? rs_digit(in, kr[r], shift, dmask) : 0u, valid, lane);
    }
    __syncthreads();
    if (t <= dmask) hist[(size_t)t * nt + b] = h[t];
    __syncthreads();
  }
}

// Stable scatter of one tile: wave w owns the tile's w-th quarter (RS_ROUNDS
// rounds of 64 consecutive entries, kept in registers).  Each wave counts its
// digits, one pass turns the counts into per-wave running offsets, and each
// wave then writes its entries in order.  Two block barriers per tile.
template <typename V>
__global__ __launch_bounds__(256) void rs_scatter_kernel(const u64* kin, const V* vin, u64* kout, V* vout,
                                                         RsIn in, uint32_t shift, const uint32_t* offs) {
  __shared__ uint32_t woff[4][256];
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  const uint32_t nt = rs_ntiles(in);
  for (uint32_t b = blockIdx.x; b < nt; b += gridDim.x) {
  u64 start;
  uint32_t count;
  rs_tile(in, b, &start, &count);
  const uint32_t dmask = (1u << in.dbits) - 1u;
  for (uint32_t ww = 0; ww < 4; ++ww) woff[ww][t] = 0u;
  __syncthreads();
  const uint32_t wbeg = w * (RS_TILE / 4);
  u64 kr[RS_ROUNDS];
  V vr[RS_ROUNDS];
  // all loads of the wave's rounds first, then the counting
#pragma unroll
  for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
    const uint32_t i = wbeg + r * 64u + lane;
    const bool valid = i < count;
    kr[r] = valid ? kin[start + i] : 0ull;
    vr[r] = valid ? vin[start + i] : (V)0;
  }
#pragma unroll
  for (uint32_t r = 0; r < RS_ROUNDS; ++r) {
    const uint32_t i = wbeg + r * 64u + lane;
    const bool valid = i < count;
    wave_count_digits(woff[w], valid ? rs_digit(in, kr[r], shift, dmask) : 0u, valid, lane);
  }
  __syncthreads();
  if (t <= dmask) {
    uint32_t o = offs[(size_t)t * nt + b];
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
    const uint32_t d = valid ? rs_digit(in, kr[r], shift, dmask) : 0u;
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
  __syncthreads();   // woff is reset for the next tile
  }
}

// The same scatter staged through LDS: wave w owns the tile's w-th
// quarter (RS_ROUNDS rounds of 64 consecutive entries, kept in registers).
// Each wave counts its digits; one pass turns the counts into the tile's
// digit order (a local, stable counting sort into LDS); the block then
// writes the tile out in that order, so consecutive threads write
// consecutive addresses of one digit's run.  Dynamic LDS: RS_TILE keys,
// values and digits.
template <typename V>
__global__ __launch_bounds__(RSL_THREADS) void rs_scatter_lds_kernel(const u64* kin, const V* vin, u64* kout, V* vout,
                                                             RsIn in, uint32_t shift, const uint32_t* offs) {
  __shared__ uint32_t woff[RSL_WAVES][256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t sh[RSL_WAVES];
  u64* lkey = reinterpret_cast<u64*>(rc_smem);
  V* lval = reinterpret_cast<V*>(lkey + RS_TILE);
  uint8_t* ldig = reinterpret_cast<uint8_t*>(lval + RS_TILE);
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  const uint32_t nt = rs_ntiles(in);
  const uint32_t dmask = (1u << in.dbits) - 1u;
  for (uint32_t b = blockIdx.x; b < nt; b += gridDim.x) {
    u64 start;
    uint32_t count;
    rs_tile(in, b, &start, &count);
    for (uint32_t i = t; i < RSL_WAVES * 256u; i += RSL_THREADS) (&woff[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t wbeg = w * (RS_TILE / RSL_WAVES);
    u64 kr[RSL_ROUNDS];
    V vr[RSL_ROUNDS];
    uint32_t dr[RSL_ROUNDS];
    // all loads of the wave's rounds first, then the counting
#pragma unroll
    for (uint32_t r = 0; r < RSL_ROUNDS; ++r) {
      const uint32_t i = wbeg + r * 64u + lane;
      const bool valid = i < count;
      kr[r] = valid ? kin[start + i] : 0ull;
      vr[r] = valid ? vin[start + i] : (V)0;
    }
#pragma unroll
    for (uint32_t r = 0; r < RSL_ROUNDS; ++r) {
      const uint32_t i = wbeg + r * 64u + lane;
      const bool valid = i < count;
      dr[r] = valid ? rs_digit(in, kr[r], shift, dmask) : 0u;
      wave_count_digits(woff[w], dr[r], valid, lane);
    }
    __syncthreads();
    // tile-local start of each digit (scan over the digits), then each
    // wave's start within it; gbase maps a local position to the output
    {
      uint32_t c = 0;
      if (t <= dmask)
        for (uint32_t ww = 0; ww < RSL_WAVES; ++ww) c += woff[ww][t];
      // (threads from 256 on hold no digit and add nothing: the scan of
      // the first 256 is exact)
      uint32_t total;
      const uint32_t lstart = block_excl_scan_256(c, sh, &total);
      if (t <= dmask) {
        gbase[t] = offs[(size_t)t * nt + b] - lstart;
        uint32_t o = lstart;
        for (uint32_t ww = 0; ww < RSL_WAVES; ++ww) {
          const uint32_t n = woff[ww][t];
          woff[ww][t] = o;
          o += n;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < RSL_ROUNDS; ++r) {
      const uint32_t i = wbeg + r * 64u + lane;
      const bool valid = i < count;
      uint32_t rank, cnt;
      digit_peers(dr[r], valid, in.dbits, lane, &rank, &cnt);
      if (valid) {
        const uint32_t base = woff[w][dr[r]];
        lkey[base + rank] = kr[r];
        lval[base + rank] = vr[r];
        // (the filter pass's digit comes from the owner table; any other
        // pass's digit is read off the key again below)
        if (in.keep) ldig[base + rank] = (uint8_t)dr[r];
        // the new offset depends on the value just read, so the wave's read
        // of this round is complete before any lane advances the counter
        if (rank == 0) woff[w][dr[r]] = base + cnt;
      }
    }
    __syncthreads();
    for (uint32_t p = t; p < count; p += RSL_THREADS) {
      const u64 k = lkey[p];
      const uint32_t d = in.keep ? (uint32_t)ldig[p] : (uint32_t)(k >> shift) & dmask;
      kout[gbase[d] + p] = k;
      vout[gbase[d] + p] = lval[p];
    }
    __syncthreads();   // the LDS tile and woff are reused for the next tile
  }
}

// dynamic LDS of the scatter: keys, values and digits of one tile
template <typename V>
constexpr size_t rs_scatter_lds() { return (size_t)RS_TILE * (sizeof(u64) + sizeof(V) + 1); }

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
  const ChunkDesc C = const_load<ChunkDesc>(S.chunks, const_load<uint32_t>(S.chunk_index, 0));
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

// Segmented inclusive minimum over the lanes of a wave: `heads` has a bit
// per lane that starts a run; each lane ends with the minimum of its run up
// to itself, so a run's last lane holds the run's minimum.  A scan with DPP
// moves: shifts by 1, 2, 4 and 8 lanes inside each row of 16, then row 0's
// and row 2's last lanes into rows 1 and 3, and lane 31 into rows 2 and 3.
// A lane takes the value it receives unless a run starts between the two,
// and lanes that receive nothing get the identity.  Whether a run starts
// between them depends on `heads` only: SegMasks holds it per step as an
// all-ones word (take nothing) or zero, built once by the same moves and
// shared by every scan over the same runs, so a step is a move, an OR and
// a minimum.
// DPP controls: row_shr:n is 0x110 + n, row_bcast:15 0x142, row_bcast:31 0x143
struct SegMasks {
  uint32_t m[6];
};
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t seg_mask_step(uint32_t m) {
  return m | (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ SegMasks seg_masks(u64 heads, uint32_t lane) {
  SegMasks M;
  M.m[0] = ((heads >> lane) & 1ull) ? ~0u : 0u;
  M.m[1] = seg_mask_step<0x111, 0xF>(M.m[0]);
  M.m[2] = seg_mask_step<0x112, 0xF>(M.m[1]);
  M.m[3] = seg_mask_step<0x114, 0xF>(M.m[2]);
  M.m[4] = seg_mask_step<0x118, 0xF>(M.m[3]);
  M.m[5] = seg_mask_step<0x142, 0xA>(M.m[4]);
  return M;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_min_step(uint32_t& v, uint32_t m) {
  const uint32_t vo = (uint32_t)__builtin_amdgcn_update_dpp((int)NONE32, (int)v, CTRL, ROWS, 0xF, false) | m;
  v = vo < v ? vo : v;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_min_step64(u64& v, uint32_t m) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)NONE32, (int)(uint32_t)v, CTRL, ROWS, 0xF, false) | m;
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)NONE32, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false) | m;
  const u64 vo = ((u64)hi << 32) | lo;
  v = vo < v ? vo : v;
}
__device__ __forceinline__ uint32_t seg_min_u32(uint32_t v, const SegMasks& M) {
  seg_min_step<0x111, 0xF>(v, M.m[0]);
  seg_min_step<0x112, 0xF>(v, M.m[1]);
  seg_min_step<0x114, 0xF>(v, M.m[2]);
  seg_min_step<0x118, 0xF>(v, M.m[3]);
  seg_min_step<0x142, 0xA>(v, M.m[4]);
  seg_min_step<0x143, 0xC>(v, M.m[5]);
  return v;
}
__device__ __forceinline__ u64 seg_min_u64(u64 v, const SegMasks& M) {
  seg_min_step64<0x111, 0xF>(v, M.m[0]);
  seg_min_step64<0x112, 0xF>(v, M.m[1]);
  seg_min_step64<0x114, 0xF>(v, M.m[2]);
  seg_min_step64<0x118, 0xF>(v, M.m[3]);
  seg_min_step64<0x142, 0xA>(v, M.m[4]);
  seg_min_step64<0x143, 0xC>(v, M.m[5]);
  return v;
}
__device__ __forceinline__ u64 shfl_u64(u64 v, uint32_t src) {
  const uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
  return ((u64)hi << 32) | lo;
}

// Both passes of the runs that lie inside the wave's window, for one scope:
// `heads` marks run starts (bit 64 of the window = the entry after it, when
// a run reaches the window's end it is not complete here and is skipped by
// the caller), id = lid (INTRA) or gid << 10 | lid (INTER; ids of one group
// share id >> 10).  Every lane returns its run's reductions; `inter` selects
// the rules.
struct RunSums {
  Pass1 p1;
  uint32_t a, b, q, A, multi1;   // INTRA: r2, w2, q; INTER: r1', w1', q, A
};
__device__ __forceinline__ RunSums window_runs(bool valid, uint32_t id, bool w, int32_t v, u64 heads,
                                               uint32_t last, uint32_t lane, bool inter) {
  RunSums r;
  // pass 1
  uint32_t r1 = valid && !w ? id : NONE32;
  u64 wm = valid && w ? (((u64)id << 32) | ((uint32_t)v ^ 0x80000000u)) : ~0ull;
  const SegMasks M = seg_masks(heads, lane);
  r1 = __shfl(seg_min_u32(r1, M), last);
  wm = shfl_u64(seg_min_u64(wm, M), last);
  r.p1.r1 = r1;
  r.p1.wmin = wm;
  const uint32_t w1 = wm == ~0ull ? NONE32 : (uint32_t)(wm >> 32);
  const int32_t x1 = (int32_t)((uint32_t)wm ^ 0x80000000u);
  // pass 2
  uint32_t a = NONE32, b = NONE32, q = NONE32, A = NONE32;
  bool m1 = false;
  if (valid) {
    if (!inter) {
      if (w) {
        if (id == w1) { if (v != x1) m1 = true; }
        else {
          b = id;
          if (v != x1) q = id;
        }
      } else if (id != r1) {
        a = id;
      }
    } else {
      const uint32_t g = id >> 10, g1 = w1 == NONE32 ? NONE32 : w1 >> 10, gr1 = r1 == NONE32 ? NONE32 : r1 >> 10;
      if (w) {
        if (id == w1 && v != x1) m1 = true;
        if (g != g1) {
          b = id;
          if (v != x1) q = id;
        } else if (id != w1 && v != x1) {
          A = id;
        }
      } else if (g != gr1) {
        a = id;
      }
    }
  }
  r.a = __shfl(seg_min_u32(a, M), last);
  r.b = __shfl(seg_min_u32(b, M), last);
  r.q = __shfl(seg_min_u32(q, M), last);
  r.A = inter ? __shfl(seg_min_u32(A, M), last) : NONE32;
  // OR over the run: the run's lanes are [first, last]
  const u64 mm = __ballot(m1);
  // the run's first lane: the last head at or below this lane (lane 0 when
  // the run began in an earlier window)
  const u64 below_heads = heads & (lane == 63u ? ~0ull : ((2ull << lane) - 1ull));
  const uint32_t first = below_heads ? 63u - (uint32_t)__clzll(below_heads) : 0u;
  const u64 run_mask = (last >= 63u ? ~0ull : ((2ull << last) - 1ull)) & ~((1ull << first) - 1ull);
  r.multi1 = (mm & run_mask) != 0ull ? 1u : 0u;
  return r;
}

// Convert INTER ids (gid << 10 | lid) of a finished check to global tids.
__device__ __forceinline__ uint32_t id_to_tid(uint32_t id, uint32_t W) {
  return id == NONE32 ? NONE32 : (id >> 10) * W + (id & 1023u);
}

// One wave per window of 64 sorted entries.  Runs that start and end inside
// the window are checked by lane reductions; a run that starts inside and
// reaches past the window is checked by its first lane as before (serially
// when short, else queued for seg_long_kernel).  Runs that start before the
// window belong to an earlier window.
// Records of one wave, staged in LDS and handed to the global staging area
// in batches, so the shared record counter sees one atomic per batch.
constexpr uint32_t WREC = 128;
struct WaveRecs {
  uint32_t words[WREC][10];   // rc_record_dev
  u64 keys[WREC];
};

__device__ __forceinline__ void flush_wave_recs(const rc_record_out& R, WaveRecs& B, uint32_t count,
                                                uint32_t lane) {
  if (count == 0) return;
  const u64 base = wave_reserve(R.rec_count, count, lane);
  uint32_t* dst = reinterpret_cast<uint32_t*>(R.staging);
  bool over = false;
  for (uint32_t j = lane; j < count * 10u; j += 64u) {
    const u64 pos = base + j / 10u;
    if (pos < R.rec_cap) dst[pos * 10u + j % 10u] = B.words[j / 10u][j % 10u];
    else over = true;
  }
  for (uint32_t j = lane; j < count; j += 64u) {
    const u64 pos = base + j;
    if (pos < R.rec_cap) {
      R.rec_keys[pos] = B.keys[j];
      R.rec_idx[pos] = (uint32_t)pos;
    }
  }
  if (__ballot(over) != 0ull && lane == 0) atomicOr(R.status_word, 2u);
}

__global__ __launch_bounds__(256) void seg_check_kernel(SegParams S) {
  __shared__ WaveRecs wrecs[4];
  const u64 n = *S.n_ptr;
  const uint32_t lane = threadIdx.x & 63u;
  WaveRecs& B = wrecs[threadIdx.x >> 6];
  uint32_t staged = 0;        // records in this wave's buffer (uniform)
  const uint32_t low = S.bg + S.bk;
  const uint32_t gmask = (1u << S.bg) - 1u;
  const u64 waves = (u64)gridDim.x * (blockDim.x >> 6);
  for (u64 win = (u64)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); win * 64u < n; win += waves) {
    const u64 i = win * 64u + lane;
    const bool valid = i < n;
    const u64 k = valid ? S.keys[i] : ~0ull;
    const u64 p = valid ? S.vals[i] : 0ull;
    const u64 kprev = (i == 0 || lane != 0) ? ~0ull : S.keys[i - 1];
    const u64 kleft = shfl_u64(k, (lane + 63u) & 63u);   // every lane takes part
    const u64 kp = lane == 0 ? kprev : kleft;
    const bool first_entry = i == 0;
    const bool sub_head = valid && (first_entry || kp != k);
    const bool head = valid && (first_entry || (kp >> low) != (k >> low));
    // the entry after the window decides whether the last runs are complete
    const u64 knext = lane == 63u ? (i + 1 < n ? S.keys[i + 1] : ~0ull) : 0ull;
    const u64 kafter = __shfl(knext, 63u);
    const u64 hsub = __ballot(sub_head), hcell = __ballot(head);
    const u64 vmask = __ballot(valid);
    // run bounds of this lane: [its run's first lane, its run's last lane]
    const u64 above = lane == 63u ? 0ull : ~((2ull << lane) - 1ull);    // lanes after this one
    const uint32_t nsub = (uint32_t)__ffsll((long long)(hsub & above));    // 1 + next run start, or 0
    const uint32_t ncell = (uint32_t)__ffsll((long long)(hcell & above));
    const uint32_t nvalid = 64u - (uint32_t)__clzll(vmask);   // valid lanes
    uint32_t last_sub = nsub ? nsub - 2u : nvalid - 1u;
    uint32_t last_cell = ncell ? ncell - 2u : nvalid - 1u;
    // does the lane's run continue past the window?
    const u64 klast = __shfl(k, 63u);
    const bool open_sub = nsub == 0u && nvalid == 64u && i + (63u - lane) + 1u < n && kafter == klast;
    const bool open_cell = ncell == 0u && nvalid == 64u && i + (63u - lane) + 1u < n &&
                           (kafter >> low) == (klast >> low);
    const bool w = pay_w(p);
    const int32_t v = pay_val(p);
    const uint32_t lid = pay_lid(p);
    const uint32_t g = (uint32_t)(k >> S.bk) & gmask;
    const uint32_t len_sub = last_sub + 1u - lane, len_cell = last_cell + 1u - lane;
    const bool want_intra = sub_head && (open_sub || len_sub >= 2u);
    const bool want_inter = head && (open_cell || len_cell >= 2u);
    // the lane reductions of a scope only where some run of it ends in the
    // window with two entries or more (the conditions are wave-uniform)
    RunSums ri, rx;
    if (__ballot(want_intra && !open_sub) != 0ull)
      ri = window_runs(valid, lid, w, v, hsub, last_sub, lane, false);
    if (__ballot(want_inter && !open_cell) != 0ull)
      rx = window_runs(valid, (g << 10) | lid, w, v, hcell, last_cell, lane, true);
    bool has_intra = false, has_inter = false;
    SegHead H;
    PendingRec pa, pb;
    if (want_intra || want_inter) {
      H = seg_head(S, k);
      if (want_intra) {
        if (!open_sub) {
          const Intra2 p2 = {ri.a, ri.b, ri.q, ri.multi1};
          has_intra = intra_finish(ri.p1, p2, &pa.label, &pa.rw, &pa.ww);
        } else {
          const u64 e = run_end(S.keys, i, n, 0);
          if (e - i <= SEG_SHORT) {
            const u64* vals = S.vals;
            has_intra = intra_check([vals](u64 j) { return vals[j]; }, i, e, &pa.label, &pa.rw, &pa.ww);
          } else {
            push_long(S, i, e, false);
          }
        }
        pa.gid = H.gid; pa.interval = H.interval; pa.aid = H.aid; pa.cell = H.cell; pa.cellkey = H.cellkey;
        pa.lidbase = H.gid * H.W;
      }
      if (want_inter && H.G > 1 && H.aid < H.n_global) {
        if (!open_cell) {
          Pass1 p1 = rx.p1;
          p1.r1 = id_to_tid(p1.r1, H.W);
          const uint32_t w1 = p1.wmin == ~0ull ? NONE32 : id_to_tid((uint32_t)(p1.wmin >> 32), H.W);
          if (w1 != NONE32) p1.wmin = ((u64)w1 << 32) | (uint32_t)p1.wmin;
          const Inter2 p2 = {id_to_tid(rx.a, H.W), id_to_tid(rx.b, H.W), id_to_tid(rx.q, H.W),
                             id_to_tid(rx.A, H.W), rx.multi1};
          has_inter = inter_finish(p1, p2, H.W, &pb.label, &pb.rw, &pb.ww);
        } else {
          const u64 f = run_end(S.keys, i, n, low);
          if (f - i <= SEG_SHORT) {
            has_inter = inter_check(S.keys, S.vals, i, f, S.bk, gmask, H.W, &pb.label, &pb.rw, &pb.ww);
          } else {
            push_long(S, i, f, true);
          }
        }
        pb.gid = H.gid; pb.interval = 0; pb.aid = H.aid; pb.cell = H.cell; pb.cellkey = H.cellkey;
        pb.lidbase = 0;
      }
    }
    const u64 m1 = __ballot(has_intra), m2 = __ballot(has_inter);
    const uint32_t c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
    if (c1 + c2 == 0) continue;
    if (staged + c1 + c2 > WREC) {     // at most 128 per window: make room first
      flush_wave_recs(S.out, B, staged, lane);
      staged = 0;
    }
    const u64 below = (1ull << lane) - 1ull;
    RecKey K = {S.bs, S.bc, has_intra || has_inter ? H.G : 1u, has_intra || has_inter ? H.NI : 1u};
    if (has_intra) {
      const uint32_t j = staged + (uint32_t)__popcll(m1 & below);
      const rc_record_dev r = make_record(K, H.slot, H.instance, pa, false, &B.keys[j]);
      const uint32_t* w = reinterpret_cast<const uint32_t*>(&r);
      for (int q = 0; q < 10; ++q) B.words[j][q] = w[q];
    }
    if (has_inter) {
      const uint32_t j = staged + c1 + (uint32_t)__popcll(m2 & below);
      const rc_record_dev r = make_record(K, H.slot, H.instance, pb, true, &B.keys[j]);
      const uint32_t* w = reinterpret_cast<const uint32_t*>(&r);
      for (int q = 0; q < 10; ++q) B.words[j][q] = w[q];
    }
    staged += c1 + c2;
    if (staged >= WREC / 2) {
      flush_wave_recs(S.out, B, staged, lane);
      staged = 0;
    }
  }
  flush_wave_recs(S.out, B, staged, lane);
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
  const uint32_t lane = threadIdx.x & 63u;
  const u64 out0 = *Gp.out_base;
  const uint32_t slot0 = Gp.chunks[*Gp.chunk_index].slot0;
  // each wave walks one contiguous range of the sorted records in rounds of
  // 64 (the count is on the device); the records of an instance are
  // consecutive, so a wave adds up the instance counts of its rounds while
  // they stay on one instance and touches the shared counters only when the
  // instance changes: a call of few instances sees few atomics on them
  const u64 waves = (u64)gridDim.x * (blockDim.x >> 6);
  const u64 n_rounds = (n + 63u) / 64u, per = (n_rounds + waves - 1u) / waves;
  const u64 wid = (u64)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const u64 r_end = (wid + 1u) * per < n_rounds ? (wid + 1u) * per : n_rounds;
  uint32_t acc_slot = NONE32, acc_race = 0, acc_benign = 0;   // wave-uniform
  auto flush = [&]() {
    if (acc_slot != NONE32 && lane == 0) {
      if (acc_race) atomicAdd(&Gp.inst_race[acc_slot], acc_race);
      if (acc_benign) atomicAdd(&Gp.inst_benign[acc_slot], acc_benign);
    }
    acc_slot = NONE32;
    acc_race = acc_benign = 0;
  };
  for (u64 rd = wid * per; rd < r_end; ++rd) {
    const u64 p = rd * 64u + lane;
    bool valid = p < n;
    uint32_t slot = 0;
    bool race = false, benign = false;
    uint32_t ix = 0;
    if (valid) {
      ix = Gp.idx[p];
      valid = ix < Gp.stage_cap;   // (only an overflowed staging leaves a hole)
    }
    if (valid) {
      const rc_record_dev r = Gp.staging[ix];
      const u64 out = out0 + p;
      slot = r.instance - slot0;
      const uint32_t label = r.array_label >> 16;
      race = (label & 3u) != 0u;
      benign = label == 4u;
      if (out < Gp.cap) Gp.out[out] = r;
      else atomicOr(&Gp.inst_flags[slot], 1u);
    }
    const u64 vm = __ballot(valid);
    if (vm == 0ull) continue;
    const uint32_t s0 = __builtin_amdgcn_readlane(slot, (uint32_t)__ffsll((long long)vm) - 1u);
    const u64 same = __ballot(!valid || slot == s0);
    if (same == ~0ull) {
      if (s0 != acc_slot) {
        flush();
        acc_slot = s0;
      }
      acc_race += (uint32_t)__popcll(__ballot(race));
      acc_benign += (uint32_t)__popcll(__ballot(benign));
    } else {
      flush();
      if (valid) {
        if (race) atomicAdd(&Gp.inst_race[slot], 1u);
        if (benign) atomicAdd(&Gp.inst_benign[slot], 1u);
      }
    }
  }
  flush();
}


__global__ __launch_bounds__(256) void rec_place_out_kernel(GatherParams Gp) {
  const u64 n = *Gp.reserved < Gp.stage_cap ? *Gp.reserved : Gp.stage_cap;
  const u64 out0 = *Gp.out_base;
  const uint32_t slot0 = Gp.chunks[*Gp.chunk_index].slot0;
  const uint32_t lane = threadIdx.x & 63u;
  for (u64 base = (u64)blockIdx.x * 256u; base < n; base += (u64)gridDim.x * 256u) {
    const u64 p = base + threadIdx.x;
    bool valid = false;
    uint32_t slot = 0;
    bool race = false, benign = false;
    if (p < n) {
      const u64 k = Gp.keys[p];
      if (k != ~0ull) {   // (not a reserved slot left unused)
        const u64 t = k >> 32;
        const u64 f = t < Gp.table_n ? (u64)Gp.scope_base[t] + (uint32_t)k : Gp.stage_cap;
        if (f < Gp.stage_cap) {
          valid = true;
          const rc_record_dev r = Gp.staging[p];
          slot = r.instance - slot0;
          const uint32_t label = r.array_label >> 16;
          race = (label & 3u) != 0u;
          benign = label == 4u;
          const u64 out = out0 + f;
          if (out < Gp.cap) Gp.out[out] = r;
          else atomicOr(&Gp.inst_flags[slot], 1u);
        } else {
          atomicOr(Gp.status_word, 2u);
        }
      }
    }
    // per-instance counts: one atomic per instance the wave holds (staged
    // slots come in chunks, so a wave spans few instances)
    u64 rem = __ballot(valid);
    const u64 rm = __ballot(race), bm = __ballot(benign);
    while (rem != 0ull) {
      const uint32_t s0 = (uint32_t)__shfl((int)slot, (int)__builtin_ctzll(rem));
      const u64 m = __ballot(valid && slot == s0);
      const uint32_t nr = (uint32_t)__popcll(rm & m), nb = (uint32_t)__popcll(bm & m);
      if (lane == 0) {
        if (nr) atomicAdd(&Gp.inst_race[s0], nr);
        if (nb) atomicAdd(&Gp.inst_benign[s0], nb);
      }
      rem &= ~m;
    }
  }
}

// entries past a buffer's capacity were dropped (and flagged): later kernels
// see at most `cap`
__global__ void live_count_kernel(const u64* reserved, const u64* unused, u64* live) {
  *live = *reserved > *unused ? *reserved - *unused : 0ull;
}

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
  if (blockIdx.x == 0 && t <= N_WCLASS) P.queue[t] = 0u;   // the classes' queues and the group check's
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
  if (M.rw && M.own_stride != 0) {
    // an owned array: the one work-item whose cells include c, if any
    const int64_t S = M.own_stride, lo = M.own_lo, cc = c;
    int64_t t;
    if (S > 0) t = (cc - lo) >= 0 ? (cc - lo) / S : -(((lo - cc) + S - 1) / S);
    else t = (lo - cc) >= 0 ? ((lo - cc) + (-S) - 1) / (-S) : -((cc - lo) / (-S));
    const int64_t o = cc - S * t - lo;
    if (t >= 0 && t < (int64_t)M.G * M.W && o >= 0 && o < (int64_t)M.own_span) {
      const uint64_t g = (uint64_t)t / M.W, l = (uint64_t)t % M.W;
      const u64 w = M.overlay[g * M.overlay_cells + M.offset + (uint64_t)o * M.W + l];
      if ((uint32_t)(w >> 42) >= M.epoch) v = (int32_t)(uint32_t)w;
    }
  } else if (M.rw) {
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
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rc_interp_vreg_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
}

hipError_t launch_interp(const PassParams& P, uint32_t blocks, uint32_t threads, size_t lds_bytes, bool vreg,
                         hipStream_t st) {
  set_lds_attr();
  if (vreg)
    hipLaunchKernelGGL(rc_interp_vreg_kernel, dim3(blocks), dim3(threads), lds_bytes, st, P);
  else
    hipLaunchKernelGGL(rc_interp_kernel, dim3(blocks), dim3(threads), lds_bytes, st, P);
  return hipGetLastError();
}

int interp_occupancy(uint32_t threads, size_t lds_bytes, bool vreg) {
  set_lds_attr();
  int n = 0;
  const hipError_t e =
      vreg ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rc_interp_vreg_kernel, (int)threads, lds_bytes)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rc_interp_kernel, (int)threads, lds_bytes);
  if (e != hipSuccess) return 1;
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

// The same scan when the level-0 length is on the device (*m_ptr <= max_m).
static void scan_excl_dev(uint32_t* data, const u64* m_ptr, uint32_t level, u64 max_m, uint32_t* tmp,
                          hipStream_t st) {
  if (max_m <= SCAN_BLOCK) {
    hipLaunchKernelGGL(scan_block_dev_kernel, dim3(1), dim3(256), 0, st, data, m_ptr, level,
                       (const uint32_t*)nullptr);
    return;
  }
  const u64 nb = (max_m + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const uint32_t grid = (uint32_t)std::min<u64>(nb, 2048);
  uint32_t* sums = tmp;
  hipLaunchKernelGGL(scan_reduce_dev_kernel, dim3(grid), dim3(256), 0, st, (const uint32_t*)data, m_ptr, level, sums);
  scan_excl_dev(sums, m_ptr, level + 1, nb, tmp + nb, st);
  hipLaunchKernelGGL(scan_block_dev_kernel, dim3(grid), dim3(256), 0, st, data, m_ptr, level, (const uint32_t*)sums);
}

// grid of the tile-walking sort kernels
static uint32_t rs_grid(u64 max_tiles) { return (uint32_t)std::max<u64>(1, std::min<u64>(max_tiles, 4096)); }

// hist region of a sort: the device-side histogram length (2 words), the
// histogram (256 x tiles) and the scan's partial sums
size_t sort_hist_words(u64 cap) {
  const u64 nb = (cap + RS_TILE - 1) / RS_TILE;
  const u64 m = 256ull * (nb ? nb : 1);
  return 2 + m + scan_tmp_words(m);
}

// upper bound of the tiles the first (segmented) pass walks
static u64 seg_blocks(u64 n_regions, u64 cap) { return (cap + RS_TILE - 1) / RS_TILE + n_regions; }

size_t sort_log_hist_words(u64 n_regions, u64 cap) {
  const u64 nb = std::max<u64>(seg_blocks(n_regions, cap), (cap + RS_TILE - 1) / RS_TILE);
  const u64 m = 256ull * (nb ? nb : 1);
  return 2 + m + scan_tmp_words(std::max<u64>(m, n_regions + 1));
}

// Second owner pass over the log regions: the interpreter stored, for every
// logged access, its work-item id into the cell's owner word (one of the
// stores survives).  An entry whose id differs from the stored one marks the
// cell shared; a cell touched by a single work-item keeps its id.
__global__ __launch_bounds__(256) void mark_shared_kernel(const u64* keys, const u64* vals, RsIn in) {
  const u64 cmask = in.keep_bc >= 32 ? 0xFFFFFFFFull : ((1ull << in.keep_bc) - 1ull);
  const uint32_t gmask = in.keep_low > in.keep_bk ? ((1u << (in.keep_low - in.keep_bk)) - 1u) : 0u;
  const uint32_t nt = rs_ntiles(in);
  for (uint32_t b = blockIdx.x; b < nt; b += gridDim.x) {
    u64 start;
    uint32_t count;
    rs_tile(in, b, &start, &count);
    for (uint32_t i = threadIdx.x; i < count; i += RS_THREADS) {
      const u64 k = keys[start + i];
      const u64 cell = (k >> in.keep_low) & cmask;
      const u64 slot = k >> (in.keep_low + in.keep_bc);
      const uint32_t id = ((((uint32_t)(k >> in.keep_bk)) & gmask) << 10) | ((uint32_t)vals[start + i] & 1023u);
      uint32_t* w = (uint32_t*)&in.keep[slot * in.keep_stride + cell];
      if (*w != id) *w = OWNER_SHARED;
    }
  }
}

// after a filter pass: the exclusive digit-major scan holds the number of
// kept (digit 0) entries at the first digit-1 slot
__global__ void kept_count_kernel(const uint32_t* hist, RsIn in, u64* n_ptr) {
  const uint32_t nt = rs_ntiles(in);
  *n_ptr = nt ? hist[nt] : 0ull;
}

template <typename V>
static hipError_t sort_pairs_impl(u64* k0, V* v0, u64* k1, V* v1, const u64* n_ptr, u64 cap, uint32_t nbits,
                                  const uint32_t* seg_count, const u64* seg_base, const uint32_t* tiles,
                                  u64 n_regions, uint32_t* hist, uint32_t dbits, hipStream_t st,
                                  int* result_in_second, uint32_t start_bit = 0, const RsIn* filter = nullptr,
                                  bool lds_scatter = false) {
  u64 *ka = k0, *kb = k1;
  V *va = v0, *vb = v1;
  int passes = 0;
  if (dbits < 1 || dbits > 8) dbits = 8;
  // the histogram's live length (written on the device each pass), then the
  // histogram and the scan's partial sums
  u64* mlen = reinterpret_cast<u64*>(hist);
  uint32_t* hst = hist + 2;
  if (filter && seg_count) {
    // stable partition of the regions: entries of cells touched at least
    // twice first, in region order; the rest is dropped
    RsIn in = *filter;
    in.n_ptr = n_ptr;
    in.dbits = 1;
    in.seg_count = seg_count;
    in.seg_base = seg_base;
    in.tiles = tiles;
    in.n_regions = (uint32_t)n_regions;
    const u64 nb = std::max<u64>(1, seg_blocks(n_regions, cap));
    const uint32_t grid = rs_grid(nb);
    uint32_t* tmp = hst + 2ull * nb;
    hipLaunchKernelGGL(mark_shared_kernel, dim3(grid), dim3(RS_THREADS), 0, st, (const u64*)ka, (const u64*)va, in);
    hipLaunchKernelGGL(rs_hist_kernel, dim3(grid), dim3(RS_THREADS), 0, st, (const u64*)ka, in, 0u, hst);
    hipLaunchKernelGGL(rs_hist_len_kernel, dim3(1), dim3(1), 0, st, in, mlen);
    scan_excl_dev(hst, mlen, 0, 2ull * nb, tmp, st);
    hipLaunchKernelGGL(rs_scatter_kernel<V>, dim3(grid), dim3(RS_THREADS), 0, st, (const u64*)ka, (const V*)va, kb,
                       vb, in, 0u, (const uint32_t*)hst);
    hipLaunchKernelGGL(kept_count_kernel, dim3(1), dim3(1), 0, st, (const uint32_t*)hst, in, (u64*)n_ptr);
    u64* tk = ka; ka = kb; kb = tk;
    V* tv = va; va = vb; vb = tv;
    ++passes;
    seg_count = nullptr;     // the rest is dense
  }
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
    const u64 nb = nbl ? nbl : 1;
    const uint32_t grid = rs_grid(nb);
    const u64 m = (1ull << dbits) * nb;
    uint32_t* tmp = hst + m;
    hipLaunchKernelGGL(rs_hist_kernel, dim3(grid), dim3(RS_THREADS), 0, st, (const u64*)ka, in, shift, hst);
    hipLaunchKernelGGL(rs_hist_len_kernel, dim3(1), dim3(1), 0, st, in, mlen);
    scan_excl_dev(hst, mlen, 0, m, tmp, st);
    // passes over full tiles of scattered digits go through LDS (one
    // contiguous run per digit and tile); region passes whose regions
    // average under half a tile, and nearly ordered record keys, scatter
    // directly
    const bool short_regions = in.seg_count && cap < (u64)n_regions * (RS_TILE / 2);
    if (lds_scatter && !short_regions)
      hipLaunchKernelGGL(rs_scatter_lds_kernel<V>, dim3(grid), dim3(RSL_THREADS), rs_scatter_lds<V>(), st,
                         (const u64*)ka, (const V*)va, kb, vb, in, shift, (const uint32_t*)hst);
    else
      hipLaunchKernelGGL(rs_scatter_kernel<V>, dim3(grid), dim3(RS_THREADS), 0, st, (const u64*)ka, (const V*)va, kb,
                         vb, in, shift, (const uint32_t*)hst);
    u64* tk = ka; ka = kb; kb = tk;
    V* tv = va; va = vb; vb = tv;
    ++passes;
  }
  *result_in_second = passes & 1;
  return hipGetLastError();
}

hipError_t sort_log(u64* k0, u64* v0, u64* k1, u64* v1, const u64* n_ptr, u64 cap, uint32_t nbits,
                    uint32_t start_bit, const uint32_t* seg_count, const u64* seg_base, uint32_t* tiles,
                    u64 n_regions, uint32_t* hist, uint32_t dbits, hipStream_t st, int* in_second,
                    const uint32_t* keep, uint32_t keep_stride, uint32_t keep_bc, uint32_t keep_bk) {
  // the number of entries, and the regions' tile prefix
  hipLaunchKernelGGL(sum_u32_kernel, dim3(n_regions > 65536 ? 1024 : (uint32_t)blocks_for(n_regions, 256)),
                     dim3(256), 0, st, seg_count, n_regions, (u64*)n_ptr);
  hipLaunchKernelGGL(region_tiles_kernel, dim3(blocks_for(n_regions + 1, 256)), dim3(256), 0, st, seg_count,
                     tiles, n_regions);
  scan_excl(tiles, n_regions + 1, hist, st);
  RsIn f;
  memset(&f, 0, sizeof f);
  f.keep = keep;
  f.keep_stride = keep_stride;
  f.keep_low = start_bit;
  f.keep_bc = keep_bc;
  f.keep_bk = keep_bk;
  return sort_pairs_impl<u64>(k0, v0, k1, v1, n_ptr, cap, nbits, seg_count, seg_base, tiles, n_regions, hist, dbits,
                              st, in_second, start_bit, keep ? &f : nullptr, true);
}
hipError_t sort_pairs_u32(u64* k0, uint32_t* v0, u64* k1, uint32_t* v1, const u64* n_ptr, u64 cap,
                          uint32_t nbits, uint32_t* hist, hipStream_t st, int* in_second) {
  return sort_pairs_impl<uint32_t>(k0, v0, k1, v1, n_ptr, cap, nbits, nullptr, nullptr, nullptr, 0, hist, 8, st,
                                   in_second);
}

hipError_t scan_counts(uint32_t* counts, u64 n, uint32_t* tmp, hipStream_t st) {
  scan_excl(counts, n, tmp, st);
  return hipGetLastError();
}

hipError_t launch_seg_check(const SegParams& S, u64 cap, hipStream_t st) {
  // the entry count is on the device: a fixed grid walks it in rounds
  uint32_t blocks = blocks_for(cap ? cap : 1, 256);   // 4 windows of 64 entries per block
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(seg_check_kernel, dim3(blocks), dim3(256), 0, st, S);
  uint32_t lblocks = (uint32_t)std::min<u64>(S.long_cap ? S.long_cap : 1, 2048);
  hipLaunchKernelGGL(seg_long_kernel, dim3(lblocks), dim3(256), 0, st, S);
  return hipGetLastError();
}
hipError_t launch_gather(const GatherParams& G, u64 cap, hipStream_t st) {
  hipLaunchKernelGGL(rec_gather_kernel, dim3((uint32_t)std::min<u64>(blocks_for(cap ? cap : 1, 256), 2048)),
                     dim3(256), 0, st, G);
  return hipGetLastError();
}
hipError_t launch_place_out(const GatherParams& G, u64 stage_cap, hipStream_t st) {
  hipLaunchKernelGGL(rec_place_out_kernel, dim3((uint32_t)std::min<u64>(blocks_for(stage_cap ? stage_cap : 1, 256), 8192)),
                     dim3(256), 0, st, G);
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
hipError_t launch_live_count(const u64* reserved, const u64* unused, u64* live, hipStream_t st) {
  hipLaunchKernelGGL(live_count_kernel, dim3(1), dim3(1), 0, st, reserved, unused, live);
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

// ---------------------------------------------------------------------------
// The workspace of rc_check_static, for callers that cannot allocate: a
// fixed array of device memory, one copy per GPU, held until the process
// ends.  On the host the array's name is only a handle, never an address:
// host code reaches the memory through the address hipGetSymbolAddress
// returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

hipError_t static_ws_address(void** out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

}  // namespace rc
