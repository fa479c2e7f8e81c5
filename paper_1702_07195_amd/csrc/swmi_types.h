// Plain data shared by the HIP kernels, the host side of the C ABI and the host-only
// search planner (no HIP types here, so the planner also builds with a host compiler).
#pragma once

#include <stdint.h>

namespace swmi {

// Residue code reserved for padding.  Its substitution score against every query
// residue is kPadScore (<= 0), so padded columns or rows never raise a score.
constexpr int kPadCode = 31;  // 0x1f: four padding codes fill a dword as 0x1f1f1f1f
constexpr int kCodes = 32;          // profile rows per query position (codes 0..31)
constexpr int kPadScore = -127;
constexpr int kGroup = 64;          // database sequences per group (one per lane)
constexpr int kColChunk = 4;        // residues per lane per dword in the packed layout
constexpr int kSat16 = 32767;       // int16 saturation value (overflow flag)

// One group of up to 64 length-sorted database sequences.  Residues live in the packed
// buffer at `base`, laid out [ncols/4][64 lanes][4 residues]; `ncols` is the padded
// width (a multiple of 4, at least max length + 2, so the last two columns are padding).
struct GroupDesc {
  int64_t base;
  int32_t ncols;
  int32_t first;   // sorted position of lane 0 (sequence `first + lane`)
  int32_t count;   // live lanes (<= 64)
  int32_t maxlen;
};

// One (query, database sequence) pair -- or one segment of its query bands -- for the
// int32 intra-task kernel.  Residue of column c sits at
// packed[base + (c >> 2) * cstride + (c & 3)].  A long pair may be split into segments
// of consecutive query bands [band0, band1) that run on different workgroups: segment
// j reads the bottom row of segment j - 1 from xbnd[xin ..] once the progress counter
// xprog[prog_in] says it is there, and publishes its own bottom row to xbnd[xout ..] and
// xprog[prog_out]; -1 marks "no neighbour".
struct PairItem {
  int64_t base;
  int32_t cstride;  // 256 for a sequence inside a group, 4 for a contiguous one
  int32_t len;
  int32_t out;      // index into the score array (caller's database order)
  int32_t query;    // query index (batched search), 0 otherwise
  int32_t band0, band1;
  int64_t xin, xout;
  int32_t prog_in, prog_out;
  int32_t segment, nsegments;
};

// A sequence kept out of the groups (longer than the intra-task threshold), stored
// contiguously in the packed buffer at `base`.
struct LongSeq {
  int64_t base;
  int32_t len;
  int32_t orig;  // caller's index
};

// Per-query data used by both kernels.
struct QueryDesc {
  int64_t qp16;      // element offset of this query's strip profile in the int16 arena
  int64_t qp8;       // byte offset of this query's [32][mrows] int8 profile in the arena
  int32_t m;         // query length
  int32_t nstrips;   // inter-task strips (2*T rows each)
  int32_t mrows;     // rows of the intra-task profile (multiple of 64 * R)
  int32_t nbands;    // intra-task bands of 64 * R rows
  int64_t out;       // element offset of this query's scores in the output array
};

// Counters in device memory, cleared by the profile kernel at the start of a search.
struct Counters {
  int32_t inter_next;     // next inter-task work item
  int32_t flagged;        // number of saturated pairs appended to the recompute list
  int32_t intra_next;     // next wide intra-task item (long list)
  int32_t recompute_next; // next wide intra-task item (recompute list)
  int32_t intra_narrow;   // next narrow intra-task item (long list)
  int32_t recompute_narrow;  // next narrow intra-task item (recompute list)
  int32_t error;          // set if a bounded wait between segments ran out
  int32_t crit_next;      // next wide item of the critical-pair list
  int32_t crit_narrow;    // (unused: that list has no narrow items)
  int32_t rescan_next;    // next chunk of the pass over an overflowed recompute list
  int32_t inter_wide;     // next of the widest inter-task items (full-width-slot waves)
};

// Two queries sharing the lanes of the two-query inter-task kernel (batched searches).
struct QueryPair {
  int64_t qp2;       // dword offset of the pair profile in the arena
  int32_t qa, qb;    // query indices; qb = -1 when qa has no partner
  int32_t nstrips;   // strips of T rows (the longer query decides)
  int32_t pad;
};

// One admitted unit of work, in host memory (record r lives in slot r % nrec).
struct ServeRecord {
  int64_t out_a;     // element offset of query a's score row in the score arena
  int64_t out_b;     // query b's row, or -1 (one query per lane)
  int32_t ma, mb;    // query lengths (mb = 0 without query b)
  int32_t kind;      // 1: one query per lane (strips of 2 * T1 rows); 2: two per lane (T2 rows)
  int32_t nstrips;   // strips of the record's kind
};

// Top-k selection state (device memory); prefix/remaining start at 0/k, count at 0.
struct TopkState {
  uint64_t prefix;     // high digits of the k-th largest key found so far
  uint32_t remaining;  // rank of the k-th key within the keys matching the prefix
  uint32_t count;      // keys collected
};
constexpr int kTopkMax = 4096;

// Kernel shapes the planner relies on.
constexpr int kServeT1 = 24;  // strip half-height of one-query records
constexpr int kServeT2 = 28;  // strip height of two-query records
constexpr int kIntraR = 16;
constexpr int kIntraBuf = 4;     // profile-row buffers per lane, two-pair path at R = 16
constexpr int kIntraWaves = 8;
constexpr int kCritR = 8;        // rows per lane of the critical-pair launch
constexpr int kCritWaves = 4;    // waves per workgroup of the critical-pair launch
constexpr int kNarrowWaves = 4;  // waves per workgroup of a throughput-bound main intra launch
constexpr int kIntraLag = 3;   // chunks between consecutive bands (see kernels.hip)
// Band-boundary rows (the bottom row of a band, read as the top row of the next) start
// kBndLead entries into their buffers, and a buffer holds at least n + 127 entries past
// its start for a sequence of n residues: the lane that writes the bottom row then stores
// at every step, also for the columns -63 .. -1 and n .. n + 62 its sweep passes
// through, which nothing reads.
constexpr int kBndLead = 64;
constexpr int kSpinLimit = 1 << 24;  // default polls before a wait between segments gives up

}  // namespace swmi
