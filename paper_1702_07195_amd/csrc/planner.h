// Host-side planner of a search (planner.cpp): pure host code, no HIP types, so that it
// builds with a host compiler too.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/swmi.h"
#include "swmi_types.h"

namespace swmi {

// A read-only array view.
template <class T> struct Span {
  const T *p = nullptr;
  size_t n = 0;
  const T *begin() const { return p; }
  const T *end() const { return p + n; }
  size_t size() const { return n; }
  bool empty() const { return n == 0; }
  const T &operator[](size_t i) const { return p[i]; }
};

// What the planner reads of a loaded database (the host copies sw_db_load keeps).
struct DbView {
  int num_cu = 0;
  int32_t alphabet = 0;
  int64_t n_seqs = 0;
  int32_t ngroups = 0;
  int32_t max_ncols = 0;       // widest group (columns incl. padding)
  int32_t max_len = 0;         // longest sequence overall
  int64_t short_residues = 0;  // residues in groups
  int64_t packed_bytes = 0;    // size of the packed residue buffer
  const GroupDesc *groups = nullptr;   // ngroups, shortest first
  const int32_t *perm = nullptr;       // sorted position -> caller's index (n_seqs)
  const int32_t *lens = nullptr;       // sorted position -> length (sequences in groups)
  const int64_t *group_res = nullptr;  // residues in groups [0, g), for g = 0 .. ngroups
  Span<LongSeq> longs;                 // longest first
};

// The knob values a search reads (see SW_KNOB_* in include/swmi.h).
struct Knobs {
  int64_t strip_rows = 0, grid_waves = 0, route_len = 0, wide_len = 0, max_segments = 0,
          intra_rows = 0, intra_pairs = 1, query_pairs = 1, main_waves = 0, mem_cap_mb = 0,
          flag_cap = 0, crit_rows = 0, crit_share = 0;
};

// Recompute-list entries when SW_KNOB_FLAG_CAP is 0 (pairs beyond them are found by the
// overflow pass).
constexpr int64_t kFlagCap = 1 << 20;

// Resident workgroups (one wave each) per compute unit of the inter-task kernels, by strip
// height; 0 for a height that is not compiled.
constexpr int kMaxStripRows = 40;
struct Occupancy {
  int inter16[kMaxStripRows + 1] = {};
  int inter16q2[kMaxStripRows + 1] = {};
};

// Everything one launch sequence needs, decided on the host.
struct Plan {
  int T = 32;                    // inter-task strip rows (half-strip for one query per lane)
  bool q2 = false;               // two queries per lane (k_inter16q2)
  int R = kIntraR;               // rows per lane of the long-pair intra-task launch
  int main_waves = kIntraWaves;  // waves per workgroup of that launch (8, or 4)
  int main_per_cu = 1;           // its workgroups per compute unit (8 waves: 1; 4 waves: 2
                                 // beside a critical-pair launch, else 3)
  bool throughput_bound = false; // the intra-task search is estimated throughput-bound
  int per_cu = 0;                // inter-task workgroups per compute unit
  std::vector<int64_t> lens;     // query lengths
  std::vector<int32_t> qorder;   // queries longest first
  std::vector<int32_t> nbandsR;  // query bands of 64R rows
  int64_t xbnd_elems = 0;  // int2 elements of the boundary rows between pair segments
  int32_t nprog = 0;       // progress counters of those boundaries
  int32_t ngroups_inter = 0;
  int32_t n_wide = 0;
  int64_t nduos = 0;  // two-pair items (their halves may be flagged for recompute)
  int64_t nitems16 = 0;
  int grid16 = 0;
  int grid_long = 0;
  int grid_re = 0;
  int grid_crit = 0;
  int grid32 = 0;
  std::vector<QueryDesc> qd;
  std::vector<PairItem> longitems;
  std::vector<PairItem> second;     // per long item: its second pair (two-pair items) or len -1
  std::vector<PairItem> crititems;  // segments of critical pairs, in bands of 64 * crit_R rows
  int crit_R = 0;                   // rows per lane of the critical-pair launch (0: none)
  int64_t qp16_elems = 0, qp8_elems = 0;
  std::vector<QueryPair> pairs;  // two-query inter-task kernel (empty: k_inter16)
  int64_t qp2_elems = 0;         // dwords of the pair profiles
  int64_t stats[SW_SEARCH_NSTATS] = {};  // see sw_search_stats
  // workspace sizes
  int64_t qbytes = 0;         // concatenated query residues
  size_t bnd16_slot = 0;      // dwords per inter-task wave's boundary slot (the widest group)
  // On a database whose widest groups would make one slot per wave too large: the first
  // big_waves waves have slots of bnd16_slot dwords and take the wide_items widest items
  // first; the other waves' slots have bnd16_small dwords.
  int32_t big_waves = 0;
  int64_t wide_items = 0;
  size_t bnd16_small = 0;
  int32_t bnd32_stride = 0;   // int2 elements per intra-task band buffer
  // Band rings of the intra-task launches, int2 elements per workgroup (max(W + 1, 2W)
  // band buffers for W waves): the main launch's grid_long slots, then the recompute
  // launch's grid_re, then the critical-pair launch's grid_crit.
  size_t bnd32_slot = 0, bnd32_slot_re = 0, bnd32_slot_crit = 0;
  size_t bnd32_off_re = 0, bnd32_off_crit = 0, bnd32_elems = 0;
  size_t need_flagged = 0;    // recompute-list entries
  size_t need_bytes = 0;      // device bytes of the whole workspace
  // staging layout: byte offsets of the parts of the per-call input block
  size_t off_qoff = 0, off_qd = 0, off_mx = 0, off_qo = 0, off_li = 0, off_se = 0,
         off_cr = 0, off_pr = 0, stage_bytes = 0;
};

// Dwords of all inter-task boundary slots: big_waves slots of bnd16_slot, then the others
// of bnd16_small.
inline size_t bnd16_words(const Plan &p) {
  const size_t big = (size_t)std::max(0, std::min(p.big_waves, p.grid16));
  return big * p.bnd16_slot + ((size_t)std::max(0, p.grid16) - big) * p.bnd16_small;
}

// Plan a search of nq queries (offsets qoff[0..nq]) against the database.
Plan make_plan(const DbView &db, const int64_t *qoff, int64_t nq, const Knobs &k,
               const Occupancy &occ);

}  // namespace swmi
