// Internal declarations shared by the HIP kernels (kernels.hip) and the host side of the
// C ABI (api.hip).  Not installed; the public interface is include/swmi.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct sw_db;

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
  int32_t pad;
};

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
  int64_t bnd_slot_words;    // dwords per slot
  int32_t recompute_all;
  int32_t nitems;            // ngroups * nqueries
  int32_t prio_cols;         // items of groups at least this wide run at raised wave priority
};

// Two queries sharing the lanes of the two-query inter-task kernel (batched searches).
struct QueryPair {
  int64_t qp2;       // dword offset of the pair profile in the arena
  int32_t qa, qb;    // query indices; qb = -1 when qa has no partner
  int32_t nstrips;   // strips of T rows (the longer query decides)
  int32_t pad;
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
  int64_t bnd_slot_words;    // dwords per slot (>= 128 * widest group's columns)
  int32_t recompute_all;
  int32_t nitems;            // ngroups * npairs
  int32_t prio_cols;         // items of groups at least this wide run at raised wave priority
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

// One admitted unit of work, in host memory (record r lives in slot r % nrec).
struct ServeRecord {
  int64_t out_a;     // element offset of query a's score row in the score arena
  int64_t out_b;     // query b's row, or -1 (one query per lane)
  int32_t ma, mb;    // query lengths (mb = 0 without query b)
  int32_t kind;      // 1: one query per lane (strips of 2 * T1 rows); 2: two per lane (T2 rows)
  int32_t nstrips;   // strips of the record's kind
};

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

// Top-k selection state (device memory); prefix/remaining start at 0/k, count at 0.
struct TopkState {
  uint64_t prefix;     // high digits of the k-th largest key found so far
  uint32_t remaining;  // rank of the k-th key within the keys matching the prefix
  uint32_t count;      // keys collected
};
constexpr int kTopkMax = 4096;

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
hipError_t launch_intra32(const IntraArgs &a, int R, int waves, int grid, hipStream_t s);
hipError_t launch_serve(const ServeArgs &a, int grid, hipStream_t s);
int serve_max_blocks_per_cu();
constexpr int kServeT1 = 24;  // strip half-height of one-query records
constexpr int kServeT2 = 28;  // strip height of two-query records

// Device a loaded database lives on (api.hip; the handle is opaque elsewhere).
int db_device(const struct ::sw_db *db);

// Strip heights compiled for the inter-task kernel, and band rows per lane for the
// intra-task kernel.
bool inter16_supported(int T);
int inter16_max_blocks_per_cu(int T);
bool inter16q2_supported(int T);  // strip heights of the pair kernel (also 28)
int inter16q2_max_blocks_per_cu(int T);
constexpr int kIntraR = 16;
constexpr int kIntraBuf = 4;     // profile-row buffers per lane, two-pair path at R = 16
constexpr int kIntraWaves = 8;
constexpr int kCritR = 8;        // rows per lane of the critical-pair launch
constexpr int kCritWaves = 4;    // waves per workgroup of the critical-pair launch
constexpr int kNarrowWaves = 4;  // waves per workgroup of a throughput-bound main intra launch
constexpr int kIntraLag = 3;   // chunks between consecutive bands (see kernels.hip)
constexpr int kSpinLimit = 1 << 24;  // default polls before a wait between segments gives up

}  // namespace swmi
