// Internal declarations shared by the HIP kernels (kernels.hip) and the host side of the
// C ABI (api.hip).  Not installed; the public interface is include/swmi.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "swmi_types.h"

struct sw_db;

namespace swmi {

struct InterArgs {
  const uint8_t *packed;
  const GroupDesc *groups;
  int32_t ngroups;
  int32_t nqueries;
  const QueryDesc *queries;
  const int32_t *qorder;     // queries of a group in visiting order (longest first)
  const int16_t *qp16;
  const int32_t *perm;       // sorted position -> caller's index
  const int32_t *lens;       // sorted position -> length
  int32_t goe, ge;
  int32_t *scores;
  PairItem *flagged;
  Counters *ctr;
  uint32_t *bnd;             // boundary scratch, one slot per persistent wave
  int64_t bnd_slot_words;    // dwords per slot of the first big_waves waves (>= 64 * widest
                             // group's columns)
  int64_t small_slot_words;  // dwords per slot of the other waves (>= 64 * the columns of
                             // every item from wide_items on)
  int32_t big_waves;         // waves with full-width slots; they take items [0, wide_items)
  int32_t wide_items;        // the widest groups' items (0: one slot class, one counter)
  int32_t recompute_all;
  int32_t nitems;            // ngroups * nqueries
  int32_t prio_cols;         // items of groups at least this wide run at raised wave priority
  int32_t flag_cap;          // recompute-list entries; pairs beyond it are marked kSat16
};

struct Inter2Args {
  const uint8_t *packed;
  const GroupDesc *groups;
  int32_t ngroups;
  int32_t npairs;
  const QueryPair *pairs;    // longest first
  const QueryDesc *queries;  // per query: score offset and intra-task bands (recompute)
  const uint32_t *qp2;
  const int32_t *perm;       // sorted position -> caller's index
  const int32_t *lens;       // sorted position -> length
  int32_t goe, ge;
  int32_t *scores;
  PairItem *flagged;
  Counters *ctr;
  uint32_t *bnd;             // boundary scratch, one slot per persistent wave
  int64_t bnd_slot_words;    // dwords per slot of the first big_waves waves (>= 128 * widest
                             // group's columns)
  int64_t small_slot_words;  // dwords per slot of the other waves (>= 128 * the columns of
                             // every item from wide_items on)
  int32_t big_waves;         // waves with full-width slots; they take items [0, wide_items)
  int32_t wide_items;        // the widest groups' items (0: one slot class, one counter)
  int32_t recompute_all;
  int32_t nitems;            // ngroups * npairs
  int32_t prio_cols;         // items of groups at least this wide run at raised wave priority
  int32_t flag_cap;          // recompute-list entries; pairs beyond it are marked kSat16
};

struct IntraArgs {
  const uint8_t *packed;
  const PairItem *items;     // static list (long sequences) or recompute list
  const int32_t *count_dev;  // if non-null, the item count is read here (recompute list)
  int32_t count;             // otherwise the item count
  int32_t *next;             // work counter of the wide items
  int32_t *next_narrow;      // work counter of the narrow items
  int32_t n_wide;            // items [0, n_wide) take a whole workgroup each
  const QueryDesc *queries;
  const int8_t *qp8;
  int32_t goe, ge;
  int32_t *scores;
  int2 *bnd;                 // band boundary scratch, one slot per persistent workgroup
  int64_t bnd_slot_elems;    // int2 elements per slot (>= 2 * waves * bnd_stride)
  int32_t bnd_stride;        // int2 elements per band buffer (>= max len + 128)
  int2 *xbnd;                // boundary rows between segments of split pairs
  int32_t *xprog;            // columns published per segment boundary
  int32_t *xfin;             // 1 once the segment before the boundary has finished
  int32_t *xmax;             // maximum of H so far, passed along the segments of a pair
  int32_t *error;            // Counters::error
  const PairItem *second;    // per item: the second pair of a two-pair item (len >= 0),
                             // or len < 0; NULL when every item is a single pair
  PairItem *flagged;         // recompute list for two-pair halves that may have saturated
  int32_t *flag_count;       // Counters::flagged
  int32_t spin_limit;        // polls before a wait between segments gives up (sets *error)
  int32_t flag_cap;          // recompute-list entries; pairs beyond it are marked kSat16
  int32_t wide_prio;         // wave priority of the wide phase (0, 2 or 3); narrow is 0
  int32_t chain;             // non-zero: narrow items may run as chained bands
};

// The pass over a recompute list that overflowed: every (query, sequence) whose score
// holds the mark kSat16 is recomputed in int32.
struct RescanArgs {
  IntraArgs ia;              // pair sweeps (packed, profiles, penalties, scores, band rings)
  const GroupDesc *groups;
  int32_t ngroups;
  const int32_t *perm;       // sorted position -> caller's index
  const int32_t *lens;       // sorted position -> length
  const LongSeq *longs;   // sequences kept out of the groups
  int32_t nlongs;
  int32_t nqueries;
  const int32_t *count;      // Counters::flagged (entries the kernels tried to append)
  int32_t *next;             // Counters::rescan_next
};

struct ProfileArgs {
  const uint8_t *query;      // concatenated queries
  const int64_t *qoff;       // query offsets (nqueries + 1)
  const QueryDesc *queries;
  int32_t nqueries;
  const int32_t *matrix;     // alphabet x alphabet
  int32_t alphabet;
  int32_t T;                 // inter-task half-strip rows
  int16_t *qp16;
  int8_t *qp8;
  Counters *ctr;
  int32_t *zero;             // an int32 array cleared with the counters (segment progress)
  int64_t nzero;
  int32_t *scores;           // score rows (QueryDesc::out); an empty query's row is zeroed
  int64_t n_seqs;            // scores per row
};

struct Profile2Args {
  const uint8_t *query;      // concatenated queries
  const int64_t *qoff;       // query offsets (nqueries + 1)
  const QueryPair *pairs;
  int32_t npairs;
  const int32_t *matrix;     // alphabet x alphabet
  int32_t alphabet;
  int32_t T;                 // strip rows
  uint32_t *qp2;
};

struct PackArgs {
  const uint8_t *raw;        // concatenated residues in caller order
  const int64_t *offsets;    // caller offsets
  const int32_t *perm;       // sorted position -> caller index
  const GroupDesc *groups;
  int32_t ngroups;
  uint8_t *packed;
};

// ---- Serving session (continuous batching): one persistent launch whose work list grows
// while it runs.  The host appends records (one query, or two queries sharing the lanes)
// and publishes them through a doorbell in host memory; work item i is group
// ngroups - 1 - (i % ngroups) of record i / ngroups, so a record's items follow those of
// the records published before it.

struct ServeArgs {
  const uint8_t *packed;
  const GroupDesc *groups;
  int32_t ngroups;
  const int32_t *perm;          // sorted position -> caller's index
  int32_t goe, ge;
  const int32_t *matrix;        // device, alphabet x alphabet
  int32_t alphabet;
  int32_t nrec;                 // record slots
  int32_t qcap;                 // bytes per query in a slot (a multiple of 64)
  const ServeRecord *records;   // host, nrec records
  const uint8_t *qstage;        // host, per slot: query a at [0, qcap), query b at [qcap, 2 qcap),
                                // each padded with kPadCode to a multiple of 64 bytes
  int32_t *scores;              // device, score rows (written through to memory: the host
                                // copies a record's rows out once it is complete)
  const int32_t *doorbell;      // host: 2 * (records published) + (1 once closed)
  int32_t *complete;            // host, per slot: r + 1 once record r is complete
  int32_t *hsat;                // host, per slot: saturation bits of the completed record
                                // (1: query a, 2: query b), written before `complete`
  int32_t *hprog;               // host, per polling workgroup: the last item it claimed
  int32_t *mirror;              // device: largest doorbell value a polling wave has seen
  int32_t *claim;               // device: next work item
  int32_t *done;                // device, per slot: items finished
  int32_t *satf;                // device, per slot: saturation bits so far
  int32_t *error;               // device: set when a wait timed out
  uint8_t *qcache;              // device, per wave: 2 * qcap bytes (the current record's queries)
  uint32_t *bnd;                // strip-boundary scratch, one slot per wave
  int64_t bnd_slot_words;       // dwords per slot (>= 128 * widest group's columns)
  int32_t npoll;                // workgroups [0, npoll) read the host doorbell; the others
                                // read its device mirror
  int32_t prio_cols;            // items of groups at least this wide run at raised wave priority
  int64_t timeout_ticks;        // wall-clock ticks a wave waits for work before giving up
};

struct TopkArgs {
  const int32_t *scores;  // n scores in the caller's order
  int64_t n;
  int32_t k;              // 1..min(n, kTopkMax)
  TopkState *state;
  uint32_t *hist;         // 256 counters, zero on entry
  uint64_t *list;         // k keys
  int32_t *hit_index;     // k results (device)
  int32_t *hit_score;
};

// Launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_topk(const TopkArgs &a, hipStream_t s);
hipError_t launch_profile(const ProfileArgs &a, hipStream_t s);
hipError_t launch_pack(const PackArgs &a, hipStream_t s);
hipError_t launch_inter16(const InterArgs &a, int T, int grid, hipStream_t s);
hipError_t launch_profile2(const Profile2Args &a, hipStream_t s);
hipError_t launch_inter16q2(const Inter2Args &a, int T, int grid, hipStream_t s);
// per_cu: the most workgroups of this launch that may share a compute unit (LDS reserved).
hipError_t launch_intra32(const IntraArgs &a, int R, int waves, int grid, hipStream_t s,
                          int per_cu);
hipError_t launch_serve(const ServeArgs &a, int grid, hipStream_t s);
hipError_t launch_rescan(const RescanArgs &a, int grid, hipStream_t s);
int serve_max_blocks_per_cu();

// Device a loaded database lives on (api.hip; the handle is opaque elsewhere).
int db_device(const struct ::sw_db *db);

// Strip heights compiled for the inter-task kernel, and band rows per lane for the
// intra-task kernel.
bool inter16_supported(int T);
int inter16_max_blocks_per_cu(int T);
bool inter16q2_supported(int T);  // strip heights of the pair kernel (also 28)
int inter16q2_max_blocks_per_cu(int T);

}  // namespace swmi
