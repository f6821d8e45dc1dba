// kernels.h -- parameter blocks and host launchers of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc_internal.h"

namespace rc {

struct rc_record_dev {      // same bytes as rc_record
  uint32_t instance, gid, interval, array_label, cell, rw_a, rw_b, ww_a, ww_b, pad;
};
struct rc_summary_dev {     // same bytes as rc_summary
  unsigned long long n_accesses;
  uint32_t n_race_cells, n_benign_cells, n_intervals;
  int32_t status;
  uint32_t fault_gid, fault_pc, fault_tid, flags;
};
static_assert(sizeof(rc_record_dev) == 40, "record layout");
static_assert(sizeof(rc_summary_dev) == 40, "summary layout");

struct SegParams {
  const unsigned long long* keys;   // sorted log keys
  const unsigned long long* vals;   // payloads in the same order
  const unsigned long long* n_ptr;  // number of log entries
  uint32_t bc, bg, bk, bs;          // key field widths; bs = scope bits of record keys
  uint32_t G, W, NI, n_arrays, n_global, inst_offset;
  const uint32_t* cellbase;         // per array, 0xFFFFFFFF when not logged
  const uint32_t* size;
  rc_record_out out;
};

struct GatherParams {
  const rc_record_dev* staging;
  const uint32_t* idx;              // sorted order of staged records
  const unsigned long long* n_ptr;  // staged records
  unsigned long long* out_base;     // records written by earlier passes (caller's counter)
  rc_record_dev* out;
  unsigned long long cap;
  uint32_t inst_offset;
  uint32_t* inst_flags;
  uint32_t* inst_race;
  uint32_t* inst_benign;
};

struct FinalParams {
  uint32_t n_slots, inst_offset, W, pad;
  const unsigned long long* inst_acc;
  const uint32_t* inst_race;
  const uint32_t* inst_benign;
  const uint32_t* inst_intervals;
  const uint32_t* inst_flags;
  const unsigned long long* inst_fault;
  rc_summary_dev* out;
};

struct FinalMemParams {
  uint32_t size, G, overlay_cells, offset, array_id, bind, rw, pad;
  int64_t lo, hi;
  uint64_t seed;
  const int32_t* dptr;
  const unsigned long long* overlay;   // overlays of slot 0, groups 0..G-1
  const uint32_t* epoch_used;          // [G]
  int32_t* out;
};

hipError_t launch_interp(const InterpParams& P, size_t lds_bytes, hipStream_t st);
size_t scan_tmp_words(unsigned long long m);
size_t sort_hist_words(unsigned long long cap);
size_t sort_log_hist_words(unsigned long long n_seg, unsigned long long R, unsigned long long cap);
// Sort the access log: regions of seg_R entries (seg_count[r] used in region
// r) become one dense array sorted by the low nbits of the key; *n_ptr (zero
// on entry) receives the number of entries.
hipError_t sort_log(unsigned long long* k0, unsigned long long* v0, unsigned long long* k1, unsigned long long* v1,
                    const unsigned long long* n_ptr, unsigned long long cap, uint32_t nbits,
                    const uint32_t* seg_count, unsigned long long n_seg, unsigned long long seg_R, uint32_t* hist,
                    hipStream_t st, int* in_second);
hipError_t sort_pairs_u32(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1,
                          const unsigned long long* n_ptr, unsigned long long cap, uint32_t nbits,
                          uint32_t* hist, hipStream_t st, int* in_second);
hipError_t launch_seg_check(const SegParams& S, unsigned long long cap, hipStream_t st);
hipError_t launch_gather(const GatherParams& G, unsigned long long cap, hipStream_t st);
hipError_t launch_finalize(const FinalParams& F, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, unsigned long long n, uint32_t v, hipStream_t st);
hipError_t launch_final_merge(const FinalMemParams& M, hipStream_t st);
hipError_t launch_clamp(unsigned long long* n_ptr, unsigned long long cap, uint32_t* status, uint32_t bit,
                        hipStream_t st);

}  // namespace rc
