/*
 * rc.h -- C ABI of the MI355X concrete race checker.
 *
 * The library runs kernels written in the minimal kernel language of the
 * paper (Section 3: expressions, booleans, commands assign/store/load/barrier/
 * assume/assert, kernel tuple K(Args) = (tid, C, ->, Locals)) under the
 * concrete SIMD semantics of Section 4, for every work-item of every
 * work-group, over many seeded inputs, and reports the non-benign data races
 * of every barrier interval (Section 4 race rule; Section 1 benign races:
 * equal-value writes are not flagged).
 *
 * Conventions
 *   - Every function returns rc_status; 0 is success, negative is an error.
 *     No function throws or aborts.  rc_last_error() returns a thread-local
 *     message describing the last failure on the calling thread.
 *   - The library owns rc_ctx and rc_prog objects.  The caller owns every
 *     device buffer (workspace, records, counters, summaries, bound arrays)
 *     and passes plain device pointers; the library never frees them.
 *   - Work is enqueued on the context's HIP stream (borrowed from the caller,
 *     or the null stream).  rc_check returns once the work is enqueued;
 *     rc_sync waits and reports deferred device errors.
 *   - One rc_ctx per host thread.  An rc_prog must not be modified (bound,
 *     re-shaped) while a check using it is in flight.
 */
#ifndef RC_H
#define RC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RC_OK = 0,
  RC_E_INVAL = -1,    /* bad argument (null pointer, out-of-range id or size)  */
  RC_E_PARSE = -2,    /* program text rejected; message is "line:col: ..."     */
  RC_E_LIMIT = -3,    /* program or launch exceeds a documented limit         */
  RC_E_STATE = -4,    /* call out of order (no NDRange, unbound input, ...)   */
  RC_E_OVERFLOW = -5, /* more race records than the caller's capacity         */
  RC_E_HIP = -6       /* HIP runtime or device failure                        */
} rc_status;

/* Message for the last failing call on this thread ("" if none). */
const char* rc_last_error(void);

typedef struct rc_ctx rc_ctx;
typedef struct rc_prog rc_prog;

/* Runtime fault of one instance (paper Section 4: runtime error / no
 * continuation).  These are results, not API errors. */
enum {
  RC_STATUS_OK = 0,
  RC_STATUS_OOB = 1,                /* index outside [0, size(a))           */
  RC_STATUS_DIV_ZERO = 2,           /* '/', '%' or 'mod' by zero            */
  RC_STATUS_ASSERT = 3,             /* assert(b) with b false               */
  RC_STATUS_ASSUME = 4,             /* assume(b) with b false               */
  RC_STATUS_BARRIER_DIVERGENCE = 5, /* barrier reached by part of a group   */
  RC_STATUS_STEP_LIMIT = 6          /* the work-group would start more loop
                                       iterations (summed over its loops)
                                       than its limit (rc_tuning.step_limit,
                                       2^24 by default): it stops at that for
                                       statement, reported for its first
                                       work-item (a safety net; Section 4
                                       has no such rule)                    */
};

/* Record labels (bit set).  A record is a race when bit 1 or 2 is set. */
enum { RC_LABEL_RW = 1, RC_LABEL_WW_DIFF = 2, RC_LABEL_BENIGN = 4 };

#define RC_NONE 0xFFFFFFFFu

/*
 * One (instance, scope, array, cell) with an eligible pair of accesses.
 * Scope INTRA(gid, interval): accesses of one work-group between two barriers;
 * scope INTER (gid = RC_NONE, interval = 0): global-array accesses of
 * different work-groups over the whole run.  Pairs: two different work-items
 * (INTRA) or work-groups (INTER), at least one writing.  rw_a < rw_b is the
 * lexicographically smallest read/write pair; ww_a < ww_b the smallest
 * different-value write pair of a race, or the smallest equal-value write pair
 * of a benign record.  Absent pairs are RC_NONE.  Thread ids are global:
 * gid * group_size + local id.   40 bytes.
 */
typedef struct {
  uint32_t instance;   /* index of the seed in the call: seed = seed0 + instance */
  uint32_t gid;        /* INTRA: work-group id; INTER: RC_NONE                 */
  uint32_t interval;   /* INTRA: interval index in the group; INTER: 0         */
  uint16_t array;      /* array id (global arrays first, then local arrays)    */
  uint16_t label;      /* RC_LABEL_* bits                                      */
  uint32_t cell;
  uint32_t rw_a, rw_b;
  uint32_t ww_a, ww_b;
  uint32_t pad;        /* 0 */
} rc_record;

/* Per-instance summary.   40 bytes. */
typedef struct {
  uint64_t n_accesses;     /* loads + stores executed (faulted statements excluded) */
  uint32_t n_race_cells;   /* records with RW or WW_DIFF                      */
  uint32_t n_benign_cells; /* records labelled BENIGN                         */
  uint32_t n_intervals;    /* intervals closed, summed over work-groups       */
  int32_t status;          /* RC_STATUS_* of the lowest faulting work-group   */
  uint32_t fault_gid, fault_pc, fault_tid; /* RC_NONE when status is OK       */
  uint32_t flags;          /* bit 0: this instance's records were truncated   */
} rc_summary;

typedef struct {
  uint32_t n_global_arrays, n_local_arrays, n_scalars, n_vars, n_stmts;
} rc_prog_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * borrowed from the caller (NULL: the null stream); it must outlive the ctx. */
rc_status rc_ctx_create(int device, void* hip_stream, rc_ctx** out);
rc_status rc_ctx_destroy(rc_ctx* ctx);
/* Replace the borrowed stream (same rules as rc_ctx_create). */
rc_status rc_ctx_set_stream(rc_ctx* ctx, void* hip_stream);

/* Per-phase device time of the work enqueued while profiling is on, measured
 * with HIP events on the context's stream.  Phases: 0 interpretation, 1 log
 * sort, 2 interval check, 3 record sort, 4 ordered output and summaries,
 * 5 per-pass setup. */
#define RC_N_PHASES 6
typedef struct {
  double ms[8];          /* summed elapsed time per phase                   */
  uint32_t launches[8];  /* number of timed spans per phase                 */
} rc_profile;
/* Start (enable = 1) or stop (0) timing; starting clears earlier timings. */
rc_status rc_ctx_profile(rc_ctx* ctx, int enable);
/* Wait for the stream and return the timings gathered so far (then clear). */
rc_status rc_ctx_profile_read(rc_ctx* ctx, rc_profile* out);

/* ---- program ------------------------------------------------------------ */

/* Parse, validate and compile program text (Section 3 language; the surface
 * syntax is given in the repository's design notes).  `len` bytes of `src`
 * are read; the text need not be NUL-terminated.  RC_E_PARSE carries
 * "line:col: message"; RC_E_LIMIT reports an exceeded limit.  The program
 * starts with no launch shape and no bindings.  The one device allocation
 * outside the caller's workspace: the program's bytecode and descriptor
 * tables (a few KB, hipMalloc here, freed by rc_prog_free), so that the
 * checks themselves allocate nothing; RC_E_HIP if it fails. */
rc_status rc_prog_load(rc_ctx* ctx, const char* src, size_t len, rc_prog** out);
rc_status rc_prog_free(rc_prog* prog);
rc_status rc_prog_get_info(const rc_prog* prog, rc_prog_info* out);
/* Array `array_id`: name (NUL-terminated, truncated to name_len), number of
 * cells, and whether it is global (1) or work-group local (0). */
rc_status rc_prog_array(const rc_prog* prog, uint32_t array_id, char* name, size_t name_len,
                        uint64_t* cells, int* is_global);
rc_status rc_prog_scalar(const rc_prog* prog, uint32_t scalar_id, char* name, size_t name_len);

/* Launch shape (Section 2: work-groups of work-items).  1 <= group_size <= 1024,
 * num_groups >= 1, num_groups * group_size < 2^26; RC_E_LIMIT when the
 * program's static bounds exceed the library's limits for this shape. */
rc_status rc_set_ndrange(rc_prog* prog, uint32_t num_groups, uint32_t group_size);

/* *owned = 1 when, under the current launch shape, array `array_id` can
 * carry no record (every record pairs two work-items, Section 4), so its
 * accesses are not logged; 0 when that is not proven.  Either no two
 * work-items can touch a common cell of the array (every index is
 * S * tid + o for one stride S != 0 and offsets o in a range shorter than
 * |S|, with indices followed through + - * << by constants over gid, lid,
 * tid, the shape constants and loop counters, in int32 without wrapping; or,
 * when no index or branch depends on the inputs, every work-item's cells are
 * enumerated), or, for a local array of a program that cannot fault, no cell
 * is written by one work-item and touched by another within a barrier
 * interval of a group.  Results never depend on it.  RC_E_STATE before
 * rc_set_ndrange. */
rc_status rc_prog_owned(const rc_prog* prog, uint32_t array_id, int* owned);

/* The same proof on program text, host only (no context, no device), under
 * num_groups groups of group_size work-items: *n_arrays receives the
 * program's array count (global arrays first, then local arrays, in
 * declaration order) and owned[a] is written for the first
 * min(capacity, *n_arrays) arrays: 1 when no two work-items can touch a
 * common cell, 2 for a local array that is not that but is race-free within
 * every interval (see rc_prog_owned), else 0; owned may be NULL when
 * capacity is 0.
 * never_faults (may be NULL) receives 1 when no input can make the program
 * fault: its accesses and branches do not depend on loaded values or scalar
 * parameters, and enumerating every work-item finds every access in bounds,
 * no division by zero, every assert and assume holding and no barrier passed
 * by only part of a group (or value ranges show the same for every input),
 * and no work-group can start more loop iterations than the default step
 * limit.  Accesses to read-only and owned arrays of such a
 * program skip the group step of a memory statement.  RC_E_PARSE /
 * RC_E_LIMIT as rc_prog_load, RC_E_INVAL for a shape outside
 * rc_set_ndrange's range. */
rc_status rc_owned_arrays(const char* src, size_t len, uint32_t num_groups, uint32_t group_size,
                          uint8_t* owned, uint32_t capacity, uint32_t* n_arrays, int* never_faults);

/* The barrier intervals in which local-array accesses are logged, from the
 * same enumeration, host only: bit k of *mask for interval k < 64 (the
 * accesses after k barriers), *later = 1 when every later interval is.
 * An interval is left out only when the program cannot fault and, in every
 * group, no cell of a local array is written by one work-item and touched
 * by another in it (INTRA records of local arrays, Section 4, need such a
 * pair); all bits are set when that is not proven.  Errors as
 * rc_owned_arrays. */
rc_status rc_log_intervals(const char* src, size_t len, uint32_t num_groups, uint32_t group_size, uint64_t* mask,
                           int* later);

/* Inputs (Section 3 K(Args): arguments passed by the host).  A global array is
 * bound either to seeded values U[lo, hi) (1 <= hi - lo <= 2^32; instance j's
 * seed is seed0 + j) or to caller-owned device memory of size(array) int32
 * cells, read-only to the library, identical for every seed, and alive until
 * the check completes.  Scalars likewise (seeded or a fixed value). */
rc_status rc_bind_seeded(rc_prog* prog, uint32_t array_id, int64_t lo, int64_t hi);
rc_status rc_bind_device(rc_prog* prog, uint32_t array_id, const int32_t* d_cells);
rc_status rc_bind_scalar_seeded(rc_prog* prog, uint32_t scalar_id, int64_t lo, int64_t hi);
rc_status rc_bind_scalar(rc_prog* prog, uint32_t scalar_id, int32_t value);

/* Implementation tuning (never changes results).  lds_log_entries: size of
 * the per-work-group interval log kept in LDS (rounded down to a power of
 * two and clamped to what LDS holds; 0 = the library's choice).  Intervals
 * larger than it are checked by the global pass instead.  radix_bits: digit
 * width of the global access-log sort, 1..8 (0 = 8).  record_sort: 0 = the
 * library's choice (a call with no global access log places each record by
 * the record counts of the (instance, group, interval)s before it and its
 * rank within its own, with no sort); 1 = always radix-sort the records by
 * their full canonical key.  proofs_off: 0 = the library proves, per launch
 * shape, which arrays can carry no record and whether the program can fault
 * (see rc_prog_owned and rc_log_intervals) and skips the logs and group
 * steps those proofs make unnecessary; 1 = no proof: every access to a
 * written array is logged and checked (the reports are the same).
 * step_limit: loop iterations one work-group may start before it stops
 * with RC_STATUS_STEP_LIMIT (0 = 2^24); unlike the other fields it is part
 * of the semantics, not a tuning, and rc_autotune keeps it.
 * global_spills: 0 = the library's choice (a program of one work-group
 * whose interval outgrows the LDS log has that interval checked after the
 * interpreter by a block per instance, from the group's log region, with
 * no log sort); 1 = such intervals always go to the global pass (log sort
 * and segmented check).  A batch uses radix_bits and
 * record_sort of its first instance's program; rc_autotune keeps
 * record_sort, proofs_off and global_spills. */
typedef struct {
  uint32_t lds_log_entries;
  uint32_t radix_bits;
  uint32_t record_sort;
  uint32_t proofs_off;
  uint32_t step_limit;
  uint32_t global_spills;
  uint32_t reserved[2];
} rc_tuning;
rc_status rc_prog_set_tuning(rc_prog* prog, const rc_tuning* tuning);

/*
 * Autotuner.  Times candidate tunings (LDS interval-log sizes x radix digit
 * widths) on a calibration slice (seeds seed0 .. seed0 + n_seeds - 1, checked
 * with d_ws), verifies that every candidate reports identical records and
 * summaries (RC_E_HIP if not), applies the fastest to `prog` and returns it in
 * *chosen.  With cache_path non-NULL the choice is stored in that JSON file
 * under the program's shape bucket (device, work-group width class, groups,
 * interval size, logged cells); a later call for the same bucket applies the
 * cached choice without timing.  Allocates its own scratch buffers (an
 * offline tool, not for use inside a capture).
 */
rc_status rc_autotune(rc_prog* prog, uint64_t seed0, uint32_t n_seeds, void* d_ws, size_t ws_bytes,
                      const char* cache_path, rc_tuning* chosen);

/*
 * Per-program kernel.  enable != 0: translate the program's bytecode into a
 * kernel of its own (private variables in registers, no instruction
 * dispatch) and compile it for gfx950 with the runtime compiler (about a
 * second, synchronous); rc_check calls of this program then run it.  Results
 * are identical to the interpreter's.  Needs the NDRange.  The kernel is
 * specialised for the launch shape (work-group size, number of groups, the
 * LDS log size the tuning picks): rc_set_ndrange and rc_prog_set_tuning on a
 * program with the kernel enabled compile one for the new shape, or take one
 * compiled earlier for it (kept until rc_prog_free).  rc_batch_check calls
 * that mix programs always interpret.  enable == 0: back to the interpreter.
 * RC_E_HIP with the compiler's log if compilation fails.
 */
rc_status rc_prog_jit(rc_prog* prog, int enable);

/* ---- checking ----------------------------------------------------------- */

/* Workspace bytes needed to check `n_seeds` instances in one pass.  Smaller
 * workspaces (at least rc_workspace_size(prog, 1)) are accepted by rc_check,
 * which then processes the seeds in several passes. */
rc_status rc_workspace_size(const rc_prog* prog, uint32_t n_seeds, size_t* bytes);

/*
 * Check instances seed0 .. seed0 + n_seeds - 1 (asynchronous on the ctx stream).
 *   d_ws        caller-owned device workspace (>= rc_workspace_size(prog, 1)).
 *               The library keeps state in it between calls: pass the same
 *               buffer unmodified, or a fresh one (first use clears it).
 *   d_records   caller-owned array of `cap` rc_record; records are written in
 *               canonical order: instance, then INTRA scopes by (gid,
 *               interval, array, cell), then INTER by (array, cell).
 *   d_n_records caller-owned device uint64: total number of records.  If it
 *               exceeds cap, only the first cap are written, the affected
 *               summaries have flags bit 0, and rc_sync returns RC_E_OVERFLOW.
 *   d_summaries caller-owned array of n_seeds rc_summary.
 * Errors detectable on the host (unbound input, no NDRange, workspace too
 * small, null pointers) are returned synchronously.
 */
rc_status rc_check(rc_prog* prog, uint64_t seed0, uint32_t n_seeds,
                   void* d_ws, size_t ws_bytes,
                   rc_record* d_records, uint64_t cap, uint64_t* d_n_records,
                   rc_summary* d_summaries);

/*
 * rc_check for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same check, with the library's static workspace in place of d_ws.
 * That workspace is a fixed array of RC_STATIC_WS_BYTES in device memory,
 * one copy per GPU, held from the first rc_ctx_create on that GPU until the
 * process ends.  The call allocates nothing: it launches its chunks one by
 * one on the ctx stream (no graph, no timing events; rc_ctx_profile does
 * not see it) and keeps its state in the static workspace between calls,
 * like a d_ws passed unmodified.  Every call on one GPU, from any context,
 * uses the same array: calls whose work overlaps on one GPU (other streams,
 * other contexts, other host threads) race and must be serialised by the
 * caller.  RC_E_INVAL, with the sizes in the message, when one instance
 * needs more workspace than RC_STATIC_WS_BYTES (rc_workspace_size(prog,
 * 1)); more seeds than fit at once run in several passes.  Other arguments,
 * results and errors as rc_check.
 */
#define RC_STATIC_WS_BYTES (256u << 20)
rc_status rc_check_static(rc_prog* prog, uint64_t seed0, uint32_t n_seeds,
                          rc_record* d_records, uint64_t cap, uint64_t* d_n_records,
                          rc_summary* d_summaries);

/*
 * Check a list of instances of possibly different programs (all loaded on
 * `ctx`, shaped and bound): instance i runs programs[i] with seed seeds[i].
 * Records and summaries follow the list order (record.instance = i); other
 * arguments and rules as rc_check.  The instances run in chunks of
 * consecutive list entries that fit the workspace, in list order: a caller
 * that wants an order (the triage ranking, say) permutes the list.  Inside a
 * chunk, persistent workgroups take (instance, group) work items from a
 * queue ordered longest first.
 */
rc_status rc_batch_check(rc_ctx* ctx, rc_prog* const* programs, const uint64_t* seeds, uint32_t n,
                         void* d_ws, size_t ws_bytes,
                         rc_record* d_records, uint64_t cap, uint64_t* d_n_records,
                         rc_summary* d_summaries);

/* Wait for the ctx stream; returns RC_E_OVERFLOW or RC_E_HIP for deferred
 * failures of earlier rc_check calls on this ctx, then clears them. */
rc_status rc_sync(rc_ctx* ctx);

/* Log statistics of the last rc_check / rc_batch_check call on the context
 * (waits for the stream; the workspace of that call must not have been
 * reused since).  logged: accesses appended to an interval log (accesses
 * to arrays never written, and those the static proofs exempt, are not
 * logged); logged_global: entries written to the global access log (arrays
 * logged there, and intervals that outgrew the LDS log); intervals_spilled:
 * intervals whose LDS log moved to the global log; intervals: intervals
 * closed, summed over work-groups and instances; instructions: bytecode
 * instructions executed, counted once per work-group (the lockstep group
 * runs each one for all its work-items); wave_instructions: the same
 * times the wavefronts that ran each work-group (a work-group runs on a
 * block of 64, 128, 256, 512 or 1024 lanes, and every wave of the block
 * takes every instruction); global_pass: the entries of logged_global
 * checked after the interpreter (by the global pass, or for one-group
 * programs by the per-instance check of spilled intervals); it equals
 * logged_global.  RC_E_STATE
 * before the first check call. */
typedef struct {
  uint64_t logged, logged_global, intervals_spilled, intervals;
  uint64_t instructions, wave_instructions, global_pass;
} rc_stats;
rc_status rc_call_stats(rc_ctx* ctx, rc_stats* out);

/* Final contents of global array `array_id` for one seed (asynchronous):
 * per cell, the value left by the highest work-group that wrote it, else the
 * initial value.  d_out holds size(array) int32 cells. */
rc_status rc_read_final(rc_prog* prog, uint64_t seed, uint32_t array_id, int32_t* d_out,
                        void* d_ws, size_t ws_bytes);

/* ---- triage network ------------------------------------------------------
 * A learned score that orders (program, seed) instances by how likely the
 * exact check is to find a race in them, so a sweep can check the likely ones
 * first.  It is not part of the paper's method and never changes a report:
 * every instance that is checked is checked exactly.
 *
 * Network (fp32): logit = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 for a
 * feature row x of RC_MLP_IN floats.  Parameters are one flat device vector
 * of RC_MLP_PARAMS floats: W1 [256][128] row-major, b1 [256], W2 [256][256],
 * b2 [256], w3 [256], b3 [1].  Loss: mean over rows of the binary
 * cross-entropy on logits, softplus(z) - y z, labels y in {0, 1}.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * counted from 1).  Feature rows are row-major [n][RC_MLP_IN] floats.
 * All buffers are caller-owned device memory; work is asynchronous on the
 * ctx stream; n must be >= 1; the workspace must hold
 * rc_mlp_workspace_size(n) bytes (RC_E_INVAL otherwise).
 */
/*
 * Triage features: RC_FEATURES floats per instance (programs[i], seeds[i]),
 * written row-major to d_feat [n][RC_FEATURES].  Every value is a ratio of
 * integers computed in fp32 (exactly reproducible).  "Memory statements" are
 * the loads and stores in program order (statements in both branches of an
 * if, loop bodies once); a statement's static interval is the number of
 * barrier statements before it in that order.  An index expression is affine
 * when it is built from integer literals, size(A), tid, unary -, + and -, and
 * * with a constant factor, optionally under one outer mod or % by a positive
 * constant; it then reads (a*tid + b) [mod N] (intermediate |a|,|b| <= 2^31,
 * else not affine).  b is reduced into [0, size(A)).  A count c "/k" below
 * stands for the bounded c / (c + k).
 *   [0..8)    exact ratios statement count / #statements: assign, load,
 *             store, barrier, assume, assert, if, for
 *   [8..12)   loads of global, loads of local, stores to global, stores to
 *             local arrays / #statements (exact ratios, as [0..8))
 *   [12..16)  #statements/256, then exact ratios #global arrays / 8,
 *             #local arrays / 8, #scalars / 16
 *   [16..24)  /8 each, over pairs {p, q} of memory statements on one array,
 *             at least one a store, in one static interval, p = q allowed
 *             for a store ("self"):  self with a == 0; of those, under an if;
 *             self not affine; p != q affine with equal a and different b;
 *             equal a and equal b; different a; p != q with one not affine;
 *             pairs with p or q under a loop holding a barrier (any interval)
 *   [24..32)  stores whose value is affine with a != 0 (/16); stores whose
 *             value is not affine (/16); deepest if nesting (/16); deepest
 *             loop nesting (/4); memory statements under an if (/16), under a
 *             loop (/16); distinct static intervals holding a store (/8);
 *             of the pairs with equal a and different b, those whose cells
 *             meet within 1024 work-items: a*d = b_q - b_p (mod size(A)) for
 *             some 1 <= |d| <= 1024 (/8)
 *   [32..96)  memory statements k = 0..15, 4 each (zeros when absent):
 *             store ? 1 : -1;  affine ? a / (1+|a|) : -2;  affine ? b / size
 *             : -2;  (interval+1) / 8 (all three exact ratios)
 *   [96..104) barriers/8, barriers under loops/8, most memory statements in
 *             one static interval/64, sum of loop trip counts/64, memory
 *             statements/64, stores/64, distinct arrays stored to/8, 0
 *   [104..112) exact ratios: W / 1024, G / 1024, ceil(log2 size) of global
 *             arrays 0 and 1 / 32 (0 if absent), local cells / 65536,
 *             G*W / 2^20, 0, 0
 *   [112..128) for global arrays 0 and 1 (zeros if absent): counts of the
 *             first min(size, 256) initial cells in 8 bins, exact / 256; seeded
 *             bindings bin floor(8 u / (hi - lo)) with u = (v - lo) mod 2^32
 *             the draw's offset in the range, bound buffers bin
 *             floor((v + 2^31) / 2^29)
 * Programs must be shaped and bound; the workspace holds
 * rc_features_workspace_size(n, number of distinct programs) bytes.
 * Asynchronous on the ctx stream.
 */
#define RC_FEATURES 128
rc_status rc_features_workspace_size(uint32_t n, uint32_t n_programs, size_t* bytes);
rc_status rc_features(rc_ctx* ctx, rc_prog* const* programs, const uint64_t* seeds, uint32_t n, float* d_feat,
                      void* d_ws, size_t ws_bytes);

/*
 * Visiting order of a triage sweep: d_order[k] = index of the k-th largest
 * score (ties by ascending index; NaN ranks last).  d_order holds n uint32;
 * the workspace holds rc_rank_workspace_size(n) bytes.  Asynchronous.
 */
rc_status rc_rank_workspace_size(uint32_t n, size_t* bytes);
rc_status rc_rank(rc_ctx* ctx, const float* d_scores, uint32_t n, uint32_t* d_order, void* d_ws, size_t ws_bytes);

#define RC_MLP_IN 128
#define RC_MLP_HIDDEN 256
#define RC_MLP_PARAMS 99073

rc_status rc_mlp_workspace_size(uint32_t n, size_t* bytes);

/* d_logits[i] = network(d_feat[i]) for i < n. */
rc_status rc_mlp_forward(rc_ctx* ctx, const float* d_params, const float* d_feat, uint32_t n, float* d_logits,
                         void* d_ws, size_t ws_bytes);

/* d_grad (RC_MLP_PARAMS floats, same layout as the parameters) = gradient of
 * the mean loss over the minibatch; *d_loss = that loss.  The minibatch is
 * rows d_rows[0..n) of d_feat / d_labels (each < the caller's row count), or
 * rows 0..n-1 when d_rows is NULL. */
rc_status rc_mlp_grad(rc_ctx* ctx, const float* d_params, const float* d_feat, const float* d_labels,
                      const uint32_t* d_rows, uint32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes);

/* One Adam step on the mean loss of the minibatch (rows as rc_mlp_grad):
 * updates d_params and the moment vectors d_adam_m, d_adam_v (RC_MLP_PARAMS
 * floats each, zero before step 1) in place; *d_loss = the loss before the
 * update.  step >= 1. */
rc_status rc_mlp_train_step(rc_ctx* ctx, float* d_params, float* d_adam_m, float* d_adam_v, uint32_t step,
                            const float* d_feat, const float* d_labels, const uint32_t* d_rows, uint32_t n, float lr,
                            float* d_loss, void* d_ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif
