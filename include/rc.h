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
  RC_STATUS_BARRIER_DIVERGENCE = 5  /* barrier reached by part of a group   */
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
 * starts with no launch shape and no bindings. */
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
 * width of the global access-log sort, 1..8 (0 = 8); a batch uses the value
 * of its first instance's program. */
typedef struct {
  uint32_t lds_log_entries;
  uint32_t radix_bits;
  uint32_t reserved[6];
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
 * Check a list of instances of possibly different programs (all loaded on
 * `ctx`, shaped and bound): instance i runs programs[i] with seed seeds[i].
 * Records and summaries follow the list order (record.instance = i); other
 * arguments and rules as rc_check.  The instances run in chunks that fit the
 * workspace; inside a chunk, persistent workgroups take (instance, group)
 * work items from a queue ordered longest first.
 */
rc_status rc_batch_check(rc_ctx* ctx, rc_prog* const* programs, const uint64_t* seeds, uint32_t n,
                         void* d_ws, size_t ws_bytes,
                         rc_record* d_records, uint64_t cap, uint64_t* d_n_records,
                         rc_summary* d_summaries);

/* Wait for the ctx stream; returns RC_E_OVERFLOW or RC_E_HIP for deferred
 * failures of earlier rc_check calls on this ctx, then clears them. */
rc_status rc_sync(rc_ctx* ctx);

/* Final contents of global array `array_id` for one seed (asynchronous):
 * per cell, the value left by the highest work-group that wrote it, else the
 * initial value.  d_out holds size(array) int32 cells. */
rc_status rc_read_final(rc_prog* prog, uint64_t seed, uint32_t array_id, int32_t* d_out,
                        void* d_ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif
