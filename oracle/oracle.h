/*
 * oracle.h -- plain single-threaded CPU oracle for the concrete SIMD race
 * semantics.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point
 * and the benchmark's CPU-baseline leg are the only callers.  The product
 * (GPU) path never links, imports or executes anything under oracle/.
 *
 * What it computes follows the paper's concrete semantics (Section 4,
 * thread-local rules, global rules, race definition) under the readings
 * listed in the repository design notes; the race check is the naive
 * pairwise definition written out.
 */
#ifndef RC_ORACLE_H
#define RC_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One binding for a global array or a scalar parameter. */
typedef struct {
  int32_t kind;        /* 0 = seeded uniform [lo, hi), 1 = explicit data */
  int32_t pad;
  int64_t lo, hi;      /* seeded range, 1 <= hi-lo <= 2^32 */
  const int32_t* data; /* explicit: array cells (size of the array) or &scalar */
} orc_bind;

/* Race record: same 40-byte layout as the library's rc_record. */
typedef struct {
  uint32_t instance, gid, interval;
  uint16_t array, label;
  uint32_t cell, rw_a, rw_b, ww_a, ww_b, pad;
} orc_record;

typedef struct {
  uint64_t n_accesses;
  uint32_t n_race_cells, n_benign_cells, n_intervals;
  int32_t status;
  uint32_t fault_gid, fault_pc, fault_tid, flags;
} orc_summary;

typedef struct {
  orc_record* records;
  uint64_t n_records;
  orc_summary summary;
  int32_t* final_mem;     /* optional: final contents of one global array */
  uint64_t final_cells;
} orc_result;

/* Program introspection (parsing only). Returns NULL on error (message in err). */
typedef struct orc_prog orc_prog;
orc_prog* orc_parse(const char* src, char* err, int errlen);
void orc_prog_free(orc_prog*);
int orc_n_global_arrays(const orc_prog*);
int orc_n_scalars(const orc_prog*);
int orc_n_local_arrays(const orc_prog*);
/* name + size of global array i (array id i); returns size */
int64_t orc_global_array(const orc_prog*, int i, char* name, int namelen);
int orc_scalar(const orc_prog*, int i, char* name, int namelen);

/* flags */
#define ORC_LITERAL_PAIRS 1   /* check every pair of the scope, no bucketing */

/*
 * Run one instance: G work-groups of W work-items, one seed.  arrays[i] binds
 * global array id i, scalars[j] binds scalar j.  final_array >= 0 asks for the
 * final contents of that global array (merge rule: highest writing gid).
 * Returns 0, or -1 with a message in err (parse error, bad launch, unbound).
 */
int orc_run(const orc_prog* p, uint32_t G, uint32_t W,
            const orc_bind* arrays, int n_arrays,
            const orc_bind* scalars, int n_scalars,
            uint64_t seed, uint32_t instance, int flags, int final_array,
            orc_result* out, char* err, int errlen);
/* The same with the group's loop-iteration limit (reading R13's safety
 * net: a work-group that would start more loop iterations, summed over all
 * its loops, stops with status 6 at that for statement, reported for its
 * first work-item).  orc_run uses ORC_STEP_LIMIT. */
#define ORC_STEP_LIMIT (1ull << 24)
int orc_run_limit(const orc_prog* p, uint32_t G, uint32_t W,
                  const orc_bind* arrays, int n_arrays,
                  const orc_bind* scalars, int n_scalars,
                  uint64_t seed, uint32_t instance, int flags, int final_array, uint64_t step_limit,
                  orc_result* out, char* err, int errlen);
void orc_result_free(orc_result*);

/*
 * The 128 triage features of one instance (inputs of the learned score that
 * orders a sweep; not part of the paper's method), as the library documents
 * them for rc_features.  Returns 0, or -1 with a message in err.
 */
int orc_features(const orc_prog* p, uint32_t G, uint32_t W, const orc_bind* arrays, int n_arrays,
                 uint64_t seed, float* out128, char* err, int errlen);

/* The seeded input generator, exposed for tests of its published definition. */
int32_t orc_seeded_value(uint64_t seed, uint64_t stream, uint64_t idx,
                         int64_t lo, int64_t hi);

#ifdef __cplusplus
}
#endif
#endif
