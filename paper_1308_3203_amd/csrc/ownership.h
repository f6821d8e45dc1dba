// ownership.h -- arrays whose cells each belong to a single work-item.
//
// Every record of the check (the race rule of the global semantics, paper
// Section 4, as checked here per cell) pairs accesses of two different
// work-items to one cell.  When the program's index expressions show that no
// two work-items can ever touch a common cell of an array, that array can
// carry no record, and its accesses need no log.  This pass proves it for
// index expressions that are affine in the work-item id.
#pragma once
#include <stdint.h>

#include <vector>

#include "frontend.h"

namespace rc {

// For an NDRange of G groups of W work-items: owned[a] = 1 when every load
// and store of array a touches a cell S * tid + o, with one stride S != 0 for
// all of the array's accesses and every offset o in one range [lo, hi] with
// hi - lo < |S| (tid = gid * W + lid).  The proof follows the bytecode:
// private variables start at 0, each register holds an affine form in gid,
// lid and the loop counters (each with its known range) or is unknown, the
// two branches of an if are joined, and a loop's entry state is iterated to
// a fixed point.  Every intermediate value must stay inside int32 for all
// values of its symbols, so the forms compute exactly what the wrapping
// int32 arithmetic does.  Loads, scalar parameters and any operation other
// than +, -, negation, multiplication by a constant and a left shift by a
// constant give an unknown value.  With one work-item every array is owned.
//
// For an owned array with stride != 0 every cell touched is stride * tid + o
// with o in [lo, hi] (hi - lo < |stride|), so a work-item's cells can be
// placed by (o - lo, lid) instead of by cell.  stride == 0: owned with no
// such placement (the array is never accessed, or there is one work-item).
//
// race_free (local arrays, by the enumeration below): within every barrier
// interval of every group, no cell is written by one work-item and read or
// written by another.  Every record of an INTRA scope pairs two such
// accesses, and a local array has no INTER scope, so such an array can
// carry no record either: its accesses need no log, and (in a program that
// cannot fault) no group step, since no work-item reads within an interval
// what another writes.
struct OwnedArray {
  uint8_t owned = 0;
  uint8_t race_free = 0;
  int64_t stride = 0, lo = 0, hi = 0;
};

// never_faults: when the accesses and branches do not depend on the inputs,
// the enumeration also sees every statement of every work-item; no access
// out of bounds, no division by zero and no failing assert or assume means
// no input can make the program fault.
//
// local_log_mask / local_log_high: the barrier intervals (k < 64 by bit k,
// all later ones by local_log_high) in which some group has a local-array
// cell written by one work-item and touched by another, in a program that
// cannot fault.  Only those intervals can give records on local arrays;
// all bits stay set when that is not proven.
struct Ownership {
  std::vector<OwnedArray> arrays;
  bool never_faults = false;
  uint64_t local_log_mask = ~0ull;
  bool local_log_high = true;
};
Ownership prove_ownership(const Compiled& c, uint32_t G, uint32_t W);

}  // namespace rc
