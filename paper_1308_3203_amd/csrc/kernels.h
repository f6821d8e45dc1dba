// kernels.h -- parameter blocks and host launchers of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc_internal.h"

namespace rc {

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
  const ProgDesc* progs;
  const SlotDesc* slots;
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;
  rc_record_out out;
  unsigned long long* longq;        // queued long runs: (start, end | inter << 63)
  unsigned long long* long_count;   // zero at chunk start
  unsigned long long long_cap;      // queue capacity in runs
};
// runs longer than this go to the queue; the queue needs at most
// 2 * entries / (SEG_SHORT_RUN + 1) + 2 slots
constexpr unsigned long long SEG_SHORT_RUN = 64;

struct GatherParams {
  const rc_record_dev* staging;
  const uint32_t* idx;              // sorted order of staged records
  const unsigned long long* n_ptr;  // staged records
  unsigned long long stage_cap;     // staged record slots
  unsigned long long* out_base;     // records written by earlier chunks (caller's counter)
  rc_record_dev* out;
  unsigned long long cap;
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;
  uint32_t* inst_flags;
  uint32_t* inst_race;
  uint32_t* inst_benign;
  // records placed by rank (launch_place_out): the staged slots' keys,
  // their count (reserved slots) and the scanned per-(slot, scope) counts
  const unsigned long long* keys;
  const unsigned long long* reserved;
  const uint32_t* scope_base;
  unsigned long long table_n;
  uint32_t* status_word;
};

struct FinalParams {
  const ProgDesc* progs;
  const SlotDesc* slots;
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;
  const unsigned long long* inst_acc;
  const uint32_t* inst_race;
  const uint32_t* inst_benign;
  const uint32_t* inst_intervals;
  const uint32_t* inst_flags;
  const unsigned long long* inst_fault;
  rc_summary_dev* out;
  uint32_t max_slots, pad;
};

struct SetupParams {
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;
  unsigned long long* counters;     // 8 words
  uint32_t* queue;                  // [N_WCLASS]
  unsigned long long* inst_acc;
  unsigned long long* inst_fault;
  uint32_t* inst_intervals;
  uint32_t* inst_race;
  uint32_t* inst_benign;
  uint32_t* inst_flags;
  unsigned long long* overlay;
  unsigned long long overlay_cells;
  uint32_t max_slots, pad;
};

struct FinalMemParams {
  uint32_t size, G, overlay_cells, offset, array_id, bind, rw, epoch;
  uint32_t W, own_span;
  int32_t own_stride, own_lo;   // placement of an owned array (ArrayDesc)
  int64_t lo, hi;
  uint64_t seed;
  const int32_t* dptr;
  const unsigned long long* overlay;   // overlays of the instance, groups 0..G-1
  int32_t* out;
};

// Spilled intervals of one-group programs, checked after the interpreter
// (sc_group_kernel): the chunk's instances from queue (zeroed by the chunk
// setup), per block SC_NB_MAX u32 of bucket bounds at ends.
struct ScParams {
  const ProgDesc* progs;
  const SlotDesc* slots;
  const ChunkDesc* chunks;
  const uint32_t* chunk_index;
  unsigned long long* log_keys;   // the regions: packed entries and trailers
  unsigned long long* log_vals;   // the same regions, second buffer
  uint32_t* wg_count;             // [work-group] region words written (zeroed once checked)
  uint32_t* queue;
  uint32_t* ends;
  const uint32_t* order;          // [call instance] chunk-relative slots in queue order, per chunk
  const rc_record_out* rec;
  uint32_t bs, bc;
};
constexpr uint32_t SC_THREADS = 512;
// the group check's part of the control block: the queue item and the record
// reservation words, which come first in Ctl; its work area starts after them
constexpr uint32_t SC_CTL_BYTES = (uint32_t)((offsetof(Ctl, uval) + 15) & ~(size_t)15);
static_assert(offsetof(Ctl, item) < offsetof(Ctl, uval) && offsetof(Ctl, rc_room) < offsetof(Ctl, uval) &&
                  offsetof(Ctl, rec_sum_total) < offsetof(Ctl, uval),
              "the group check's control fields must precede its work area");
constexpr uint32_t SC_MAX_BLOCKS = 1024;
hipError_t launch_sc_group(const ScParams& S, uint32_t blocks, hipStream_t st);
int sc_group_occupancy();

// vreg: the interpreter variant with the private variables in a 16-entry
// VGPR file (every program of the call has at most 16 registers)
constexpr uint32_t VREG_FILE = 16;
hipError_t launch_interp(const PassParams& P, uint32_t blocks, uint32_t threads, size_t lds_bytes, bool vreg,
                         hipStream_t st);
int interp_occupancy(uint32_t threads, size_t lds_bytes, bool vreg);
hipError_t launch_setup(const SetupParams& P, hipStream_t st);
hipError_t launch_ws_validate(unsigned long long* header, unsigned long long magic, unsigned long long ctx_id,
                              unsigned long long gen, unsigned long long* pool, unsigned long long pool_cells,
                              uint32_t* dirty, hipStream_t st);
hipError_t launch_advance(unsigned long long* out_base, const unsigned long long* rec_n, uint32_t* chunk_index,
                          hipStream_t st);
size_t scan_tmp_words(unsigned long long m);
size_t sort_hist_words(unsigned long long cap);
size_t sort_log_hist_words(unsigned long long n_regions, unsigned long long cap);
// Sort the access log: region r (seg_count[r] entries from seg_base[r])
// becomes part of one dense array, stably sorted by key bits
// [start_bit, nbits); *n_ptr (zero on entry) receives the number of entries;
// tiles holds n_regions + 1 words of scratch.  Bits below start_bit keep the
// regions' order (region by region, each in its own order).  With `keep`
// (owner words per (slot, cell key), keep_stride cells per slot, the cell key
// of keep_bc bits at start_bit, group and interval fields below it, the
// interval keep_bk bits wide), entries of cells touched by one work-item only
// are dropped first and *n_ptr becomes the number kept.
hipError_t sort_log(unsigned long long* k0, unsigned long long* v0, unsigned long long* k1, unsigned long long* v1,
                    const unsigned long long* n_ptr, unsigned long long cap, uint32_t nbits, uint32_t start_bit,
                    const uint32_t* seg_count, const unsigned long long* seg_base, uint32_t* tiles,
                    unsigned long long n_regions, uint32_t* hist, uint32_t dbits, hipStream_t st, int* in_second,
                    const uint32_t* keep = nullptr, uint32_t keep_stride = 0, uint32_t keep_bc = 0,
                    uint32_t keep_bk = 0);
hipError_t sort_pairs_u32(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1,
                          const unsigned long long* n_ptr, unsigned long long cap, uint32_t nbits,
                          uint32_t* hist, hipStream_t st, int* in_second);
hipError_t launch_seg_check(const SegParams& S, unsigned long long cap, hipStream_t st);
hipError_t launch_gather(const GatherParams& G, unsigned long long cap, hipStream_t st);
hipError_t launch_finalize(const FinalParams& F, hipStream_t st);
hipError_t launch_region_tiles(const uint32_t* counts, uint32_t* tiles, unsigned long long n_regions, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long n, unsigned long long v, hipStream_t st);
// exclusive scan in place of counts[n]; tmp holds scan_tmp_words(n) words
hipError_t scan_counts(uint32_t* counts, unsigned long long n, uint32_t* tmp, hipStream_t st);
// Records with rank keys, in one pass over the staged slots: each live
// record goes straight to its output position (the scanned count of its
// (slot, scope) plus its rank), with the per-instance race and benign
// counts; a key outside the table or a position past the staging sets
// status bit 1.
hipError_t launch_place_out(const GatherParams& G, unsigned long long stage_cap, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, unsigned long long n, uint32_t v, hipStream_t st);
hipError_t launch_final_merge(const FinalMemParams& M, hipStream_t st);
hipError_t launch_rank_keys(const float* scores, uint32_t n, uint32_t idx_bits, unsigned long long* keys,
                            uint32_t* vals, unsigned long long* n_ptr, hipStream_t st);
hipError_t launch_features(const FeatItem* items, const FeatProg* progs, uint32_t n, float* out, hipStream_t st);
hipError_t launch_live_count(const unsigned long long* reserved, const unsigned long long* unused,
                             unsigned long long* live, hipStream_t st);
hipError_t launch_clamp(unsigned long long* n_ptr, unsigned long long cap, uint32_t* status, uint32_t bit,
                        hipStream_t st);

// Bytes of the static workspace (rc_check_static) and its address on the
// current device.
constexpr size_t STATIC_WS_BYTES = (size_t)256 << 20;
hipError_t static_ws_address(void** out);

}  // namespace rc
