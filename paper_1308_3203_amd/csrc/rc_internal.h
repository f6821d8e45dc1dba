// rc_internal.h -- bytecode format, compiled-program description and the
// parameter blocks shared by the host front end and the HIP kernels.
#pragma once
#include <stdint.h>

namespace rc {

// ---------------------------------------------------------------------------
// Bytecode: every instruction is four 32-bit words {hdr, a, b, c}, so the
// interpreter fetches one with a single 16-byte scalar load.
//   hdr = op:6 | fa:1 | fb:1 | sub:6 | dst:6 | pc:12      (low bits first)
//   fa / fb: operand a / b is an immediate (else a source selector)
// ---------------------------------------------------------------------------
enum Op : uint32_t {
  OP_BIN = 1,     // R[dst] = a <sub> b
  OP_UN = 2,      // R[dst] = <sub> a
  OP_LOAD = 3,    // R[dst] = array c [a]
  OP_STORE = 4,   // array c [a] = b
  OP_IF = 5,      // cond a; b = index of the matching OP_ELSE
  OP_ELSE = 6,    // c = index of the matching OP_ENDIF
  OP_ENDIF = 7,
  OP_FOR = 8,     // var dst, slot sub, lo a, hi b, c = index after OP_ENDFOR
  OP_ENDFOR = 9,  // var dst, slot sub, lo a, hi b, c = index of the first body instruction
  OP_BARRIER = 10,
  OP_ASSERT = 11, // cond a
  OP_ASSUME = 12, // cond a
  OP_END = 13,
};

enum BinOp : uint32_t {
  B_ADD, B_SUB, B_MUL, B_DIV, B_REM, B_MOD, B_AND, B_OR, B_XOR, B_SHL, B_SHR,
  B_LT, B_LE, B_GT, B_GE, B_EQ, B_NE, B_LAND, B_LOR, B_MIN, B_MAX, B_COUNT
};
enum UnOp : uint32_t { U_MOV, U_NEG, U_BNOT, U_LNOT };

// source selectors (operands that are not immediates)
enum : uint32_t {
  MAX_REGS = 64,
  SEL_LID = 64, SEL_TID = 65, SEL_GID = 66, SEL_WGSIZE = 67, SEL_NGROUPS = 68,
  SEL_NTHREADS = 69, SEL_SCALAR0 = 96,
};

inline uint32_t make_hdr(uint32_t op, bool fa, bool fb, uint32_t sub, uint32_t dst, uint32_t pc) {
  return (op & 63u) | (uint32_t(fa) << 6) | (uint32_t(fb) << 7) | ((sub & 63u) << 8) |
         ((dst & 63u) << 14) | ((pc & 4095u) << 20);
}

// fault codes (rc_summary.status)
enum : uint32_t { F_OK = 0, F_OOB = 1, F_DIV = 2, F_ASSERT = 3, F_ASSUME = 4, F_BARDIV = 5, F_STEP_LIMIT = 6 };
constexpr uint32_t DEFAULT_STEP_LIMIT = 1u << 24;

// limits
enum : uint32_t {
  MAX_GLOBAL_ARRAYS = 8, MAX_LOCAL_ARRAYS = 8, MAX_ARRAYS = 16, MAX_SCALARS = 16,
  MAX_VARS = 32, MAX_STMTS = 4096, MAX_NEST = 16, MAX_WG = 1024, MAX_WAVES = 16,
};

// array kinds as the interpreter sees them
enum : uint32_t {
  AK_LOCAL = 0,        // work-group local array in LDS (u64 cells: version | value)
  AK_GLOBAL_RW = 1,    // written global array: per-group overlay in the workspace
  AK_GLOBAL_RO = 2,    // never-written global array: read its input directly
};
enum : uint32_t { BIND_NONE = 0, BIND_SEEDED = 1, BIND_DEVICE = 2 };
// Where an array's accesses are logged.  Arrays never written cannot pair.
// Local arrays, and global arrays when there is one work-group, pair only
// inside a work-group interval: their log stays in LDS and is checked at the
// barrier.  Global arrays with several work-groups also pair across groups
// (INTER scope): their accesses go to the global log.
enum : uint32_t { LOG_NONE = 0, LOG_GLOBAL = 1, LOG_LDS = 2 };

struct ArrayDesc {        // 64 bytes
  uint32_t kind;          // AK_*
  uint32_t size;          // cells
  uint32_t logged;        // LOG_NONE, LOG_GLOBAL or LOG_LDS (see below)
  uint32_t bind;          // BIND_* (global arrays)
  int64_t lo, hi;         // seeded range
  const int32_t* dptr;    // device binding
  uint32_t offset;        // LDS cell offset (local) or overlay cell offset (global rw)
  uint32_t cellbase;      // first cell key of this array in the log key space
  // a global rw array whose cells each belong to one work-item (own_stride
  // != 0): cell own_stride * tid + o sits at overlay word (o - own_lo) * W +
  // lid of its group's region, which holds own_span * W words
  int32_t own_stride, own_lo;
  uint32_t own_span;
  // the program cannot fault, and the array is read-only or owned: its
  // accesses need no group step (no fault to publish, no log, no other
  // work-item's cell)
  uint32_t nosync;
};

struct ScalarDesc {
  uint32_t bind;          // BIND_SEEDED or fixed value
  int32_t value;
  int64_t lo, hi;
};

// ---------------------------------------------------------------------------
// A check call is a list of instances (program, seed).  It runs in chunks;
// every chunk uses the same workspace layout, and all per-chunk parameters
// live in device tables, so the kernel sequence of one chunk is the same for
// every chunk (and is captured once as a HIP graph).
// ---------------------------------------------------------------------------
struct ProgDesc {                 // one program of the call
  const uint32_t* code;           // 4 words per instruction
  const ArrayDesc* arrays;
  const ScalarDesc* scalars;
  const uint32_t* cellbase;       // per array: first log cell key (0xFFFFFFFF: not logged)
  const uint32_t* size;           // per array: cells
  uint32_t n_arrays, n_global, n_scalars, nregs;
  uint32_t G, W, nwaves, lds_local_cells;
  uint32_t lds_log_cap, overlay_cells, NI;
  // interpreted with elided group steps: the program cannot fault, and a
  // memory statement synchronises the group only when its instruction
  // says so (bit 31 of its array word clear); log entries take their
  // positions from LDS counters (see Item::mem_nf)
  uint32_t nf;
  uint64_t wg_log_cap;            // log entries reserved per work-group
  // LDS interval check by a per-cell table instead of a sort: table entry of
  // log cell key ck is ck - tab_base; tab_cells = 0 selects the sort
  uint32_t tab_base, tab_cells;
  // intervals whose local-array accesses are logged: interval k < 64 when
  // bit k of log_mask is set, every later one when log_high != 0 (all set
  // unless a proof shows the other intervals race-free)
  uint32_t log_high;
  uint32_t step_limit;            // loop iterations a work-group may start (then F_STEP_LIMIT)
  uint64_t log_mask;
  // spilled intervals of a one-group program checked by the group check
  // kernel (sc_group_kernel) instead of the global pass: sc != 0; n_cells
  // log cell keys.  The group's region then holds, per spilled interval,
  // its entries as packed words and a trailer (interval << 32 | count).
  uint32_t sc, n_cells;
};
// (one-group programs) spilled intervals: log entries are packed words (cell
// key:21 | store:1 | lid:10 | value:32, as tab_entry), at most SC_MAX_CELLS
// cell keys, so at most SC_NB_MAX windows of SC_WIN cells in the check
constexpr uint32_t SC_MAX_CELLS = 1u << 21;
constexpr uint32_t SC_NB_MAX = 1024;
constexpr uint32_t SC_WIN_BITS = 11, SC_WIN = 1u << SC_WIN_BITS;   // cells per table window of the check
constexpr uint32_t SC_WORDS = SC_WIN / 32u;                        // bitmap words of a window

// one cell's running check state in the LDS table (24 bytes)
struct TabCell {
  unsigned long long wmin;   // (writer lid, value ^ sign) minimum
  uint32_t r1, r2, w2;       // smallest reader; second reader; smallest writer other than w1
  uint32_t q;                // smallest writer of a value other than x1 (w1 included)
};
constexpr uint32_t TAB_MAX_CELLS = 4096;

struct SlotDesc {                 // one instance of the call
  uint64_t seed;
  uint64_t log_base;              // first log entry of its group 0 (in the chunk's log)
  uint64_t ovl_base;              // first overlay cell of its group 0 (in the chunk's pool)
  uint32_t prog;                  // index into the call's program table
  uint32_t wg_base;               // index of its group 0 among the chunk's work-groups
};

constexpr uint32_t N_WCLASS = 5;  // work-group widths up to 64, 128, 256, 512, 1024

struct ChunkDesc {
  uint32_t slot0, n_slots;        // instances [slot0, slot0 + n_slots) of the call
  uint32_t n_wg, n_items;
  uint32_t item0[N_WCLASS + 1];   // items of width class c: [item0[c], item0[c+1])
  uint32_t epoch;                 // overlay version base of this chunk
  uint32_t clear_overlay;         // versions wrapped: clear the pool first
};

// Parameters of the interpreter launches of a call (constant for the call).
struct PassParams {
  const ProgDesc* progs;
  const SlotDesc* slots;
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;    // device: the chunk being processed
  const uint32_t* items;          // (instance, gid) pairs, per chunk and class, longest first
  uint32_t* queue;                // [N_WCLASS] work-stealing counters
  uint32_t wclass, bc, bg, bk, bs, do_log;
  unsigned long long* overlay;    // overlay pool of the chunk
  unsigned long long* log_keys;   // access log (one region per work-group)
  unsigned long long* log_vals;
  uint32_t* wg_count;             // [work-group] log entries written
  unsigned long long* wg_base;    // [work-group] first entry of its region
  unsigned long long* inst_acc;   // [chunk slot] accesses
  uint32_t* inst_intervals;       // [chunk slot]
  unsigned long long* inst_fault; // [chunk slot] min (gid, pc, lid, code) key
  uint32_t* status_word;          // bit 0: internal log overflow
  struct rc_record_out* rec;      // record staging
  // owner word per (chunk slot, log cell key) of the global log, or null:
  // every logged access stores its work-item id (gid << 10 | lid) there;
  // the log sort later keeps only cells touched by two work-items (no other
  // cell can hold an eligible pair in any scope)
  uint32_t* cell_owner;
  uint32_t cell_owner_stride, pad_co;
  // the call's log statistics (summed over chunks), or null: [0] logged
  // accesses, [1] entries written to the global log, [2] intervals whose LDS
  // log moved to the global log, [3] intervals closed, [4] instructions
  // executed (per work-group), [5] the same times the block's waves, [6]
  // global log entries left to the global pass
  unsigned long long* stats;
};
constexpr uint32_t OWNER_SHARED = 0xFFFFFFFFu;

struct rc_record_dev {      // same bytes as rc_record
  uint32_t instance, gid, interval, array_label, cell, rw_a, rw_b, ww_a, ww_b, pad;
};

// Record output shared by the interval checks (interpreter and global pass).
struct rc_record_out {
  void* staging;                       // rc_record[rec_cap]
  unsigned long long* rec_keys;        // canonical sort key per staged record
  uint32_t* rec_idx;
  unsigned long long* rec_count;
  unsigned long long rec_cap;
  uint32_t* status_word;               // bit 1: staging capacity exceeded
  // slots reserved by work-groups in chunks and left unused: their keys
  // are REC_DEAD_KEY (sorted after every record) and they are counted here
  unsigned long long* rec_dead;
  // rank_keys != 0: every record comes from an interval closed in LDS, and
  // its key is (slot << bs | scope) << 32 | its rank among the records of
  // that (group, interval), which are emitted in cell-key order; the
  // closing work-group stores the count of those records in
  // scope_cnt[slot << bs | scope].  0: the key is the full canonical key.
  uint32_t* scope_cnt;
  uint32_t rank_keys, pad_rk;
};
// interpreter work-groups reserve record slots REC_CHUNK at a time; a launch
// runs at most REC_MAX_BLOCKS blocks per width class, so at most
// N_WCLASS * REC_MAX_BLOCKS * REC_CHUNK reserved slots stay unused
constexpr unsigned long long REC_CHUNK = 64;
constexpr uint32_t REC_MAX_BLOCKS = 4096;

// LDS control block of the interpreter (after the local cells and registers)
struct Ctl {
  unsigned long long fault;             // min fault key of the group (~0 = none)
  unsigned long long rec_base;          // the group's record reservation
  unsigned long long rc_cur, rc_end;    // the block's reserved record slots [cur, end)
  unsigned long long rc_next, rc_room;  // a reservation: rc_room slots at rec_base, the rest at rc_next
  uint32_t red[2][MAX_WAVES];           // per-wave reduction words, double-buffered
  uint32_t rec_sum[MAX_WAVES];          // per-wave record counts of a reservation
  uint32_t rec_sum_total, pad2;         // and their sum
  uint32_t item;                        // work item taken by the group
  uint32_t pad;
  // (the group check kernel uses the fields above and puts its work area
  // where the next one starts)
  // the interpreter's special operands by selector (SEL_LID ...): lid and
  // tid add the work-item's lid to words 0 and 1; the scalar parameters
  // follow at SEL_SCALAR0
  int32_t uval[SEL_SCALAR0 - SEL_LID + MAX_SCALARS];
  uint32_t loopctr[MAX_WAVES][MAX_NEST];
  uint32_t lds_cnt[2];                  // LDS log entries of the even / odd intervals
                                        // (elided group steps)
  unsigned long long gl_cnt;            // global log entries of the group (elided group steps)
  // the call's log statistics (PassParams::stats) summed over the block's
  // items, added to the call's totals once, when the block leaves
  unsigned long long stat[7];
};
// bit of a load / store instruction's array word: the interpreter skips the
// statement's group step (programs interpreted with elided steps only)
constexpr uint32_t INSN_NO_STEP = 0x80000000u;

constexpr uint32_t LDS_LIMIT = 160u * 1024u;

// triage features: per program the shape- and seed-independent part plus the
// two arrays whose initial cells are summarised; per instance a program index
// and a seed
constexpr int N_FEAT = 128, N_FEAT_STATIC = 112;
struct FeatArray {       // 32 bytes
  uint32_t present, bind, size, pad;
  int64_t lo, hi;
  const int32_t* dptr;
};
struct FeatProg {        // 512 bytes
  float stat[N_FEAT_STATIC];
  FeatArray arr[2];
};
struct FeatItem {        // 16 bytes
  uint64_t seed;
  uint32_t prog, pad;
};

}  // namespace rc
