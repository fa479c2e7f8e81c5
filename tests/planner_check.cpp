// CPU check of the search planner (paper_1702_07195_amd/csrc/planner.cpp), built with
// address and undefined-behaviour sanitizers by tests/test_planner_cpu.py.
//
// Random databases (shaped exactly as sw_db_load shapes them: length-sorted groups of 64,
// the longest sequences kept apart), random query sets (empty, short and very long
// queries) and random knob settings are planned on devices of 4 to 256 compute units,
// and every plan must
//   - cover every (query, database sequence) pair exactly once: through an inter-task
//     group item, or through one intra-task item (a single pair, half of a two-pair item,
//     or one complete chain of segments in the main or the critical-pair list);
//   - chain the segments of a split pair in order, each reading only the boundary its
//     predecessor (earlier in the same list) writes;
//   - keep every offset inside its buffer (profiles, score rows, packed residues, segment
//     boundaries and progress counters, query bands, the staging block).
// Prints "planner ok: <cases>" and exits 0, or prints the first violation and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../paper_1702_07195_amd/csrc/planner.h"

using namespace swmi;

namespace {

std::string g_case;
int64_t n_split_duos = 0;  // segments of split two-pair items seen

[[noreturn]] void fail(const std::string &msg) {
  std::printf("planner check failed (%s): %s\n", g_case.c_str(), msg.c_str());
  std::exit(1);
}

#define CHECK(cond, msg)                \
  do {                                  \
    if (!(cond)) fail(std::string(msg)); \
  } while (0)

// A database as sw_db_load lays it out.
struct Db {
  std::vector<int64_t> len;  // caller order
  std::vector<GroupDesc> groups;
  std::vector<int32_t> perm, lens;
  std::vector<int64_t> group_res;
  std::vector<LongSeq> longs;
  DbView view;
};

Db make_db(const std::vector<int64_t> &len, int64_t intra_min_len, int num_cu, int alphabet) {
  Db d;
  d.len = len;
  const int64_t n = (int64_t)len.size();
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return len[x] < len[y]; });
  int64_t n_short = 0;
  while (n_short < n && len[order[n_short]] <= intra_min_len) ++n_short;
  int64_t bytes = 0, short_res = 0;
  int32_t max_ncols = 0;
  for (int64_t f = 0; f < n_short; f += 64) {
    GroupDesc g;
    g.first = (int32_t)f;
    g.count = (int32_t)std::min<int64_t>(64, n_short - f);
    g.maxlen = (int32_t)len[order[f + g.count - 1]];
    g.ncols = ((g.maxlen + 2 + 3) / 4) * 4;
    g.base = bytes;
    bytes += (int64_t)g.ncols * 64;
    max_ncols = std::max(max_ncols, g.ncols);
    d.groups.push_back(g);
  }
  d.group_res.assign(d.groups.size() + 1, 0);
  for (size_t g = 0; g < d.groups.size(); ++g) {
    int64_t r = 0;
    for (int32_t l = 0; l < d.groups[g].count; ++l) r += len[order[d.groups[g].first + l]];
    d.group_res[g + 1] = d.group_res[g] + r;
  }
  short_res = d.group_res.back();
  d.lens.assign((size_t)std::max<int64_t>(1, n_short), 0);
  for (int64_t p = 0; p < n_short; ++p) d.lens[p] = (int32_t)len[order[p]];
  for (int64_t p = n - 1; p >= n_short; --p) {
    LongSeq L;
    L.base = bytes;
    L.len = (int32_t)len[order[p]];
    L.orig = order[p];
    bytes += ((L.len + 4 + 3) / 4) * 4;
    d.longs.push_back(L);
  }
  d.perm = order;
  DbView &v = d.view;
  v.num_cu = num_cu;
  v.alphabet = alphabet;
  v.n_seqs = n;
  v.ngroups = (int32_t)d.groups.size();
  v.max_ncols = max_ncols;
  v.max_len = n ? (int32_t)len[order[n - 1]] : 0;
  v.short_residues = short_res;
  v.packed_bytes = std::max<int64_t>(bytes, 4);
  v.groups = d.groups.data();
  v.perm = d.perm.data();
  v.lens = d.lens.data();
  v.group_res = d.group_res.data();
  v.longs.p = d.longs.data();
  v.longs.n = d.longs.size();
  return d;
}

int64_t nbands_of(int64_t m, int R) { return (m + 64 * R - 1) / (64 * R); }

// Check one list of intra-task items (main or critical, with rows per lane R); counts the
// pairs it covers into `cover` ((query, caller index) -> count).
void check_items(const Plan &p, const Db &d, const std::vector<PairItem> &items,
                 const std::vector<PairItem> *second, int R, int64_t nq,
                 std::map<std::pair<int, int>, int> &cover, std::vector<int> &prog_writers,
                 std::vector<int> &prog_readers,
                 std::vector<std::pair<int64_t, int64_t>> &extents, const char *list) {
  const std::string L(list);
  std::map<int32_t, size_t> writer_at;  // progress counter -> index of its writer
  for (size_t i = 0; i < items.size(); ++i) {
    const PairItem &it = items[i];
    CHECK(it.query >= 0 && it.query < nq, L + ": query index");
    const int64_t m = p.lens[(size_t)it.query];
    CHECK(m > 0, L + ": an item for an empty query");
    const int64_t nb = nbands_of(m, R);
    CHECK(it.band0 >= 0 && it.band0 < it.band1 && it.band1 <= nb, L + ": bands out of range");
    CHECK(it.len >= 0 && it.out >= 0 && it.out < d.view.n_seqs, L + ": sequence");
    CHECK(d.len[(size_t)it.out] == it.len, L + ": length of the caller's sequence");
    // residues inside the packed buffer
    if (it.cstride == 4) {
      CHECK(it.base >= 0 && it.base + it.len <= d.view.packed_bytes, L + ": long residues");
    } else {
      CHECK(it.cstride == 256, L + ": column stride");
      if (it.len > 0) {
        const int64_t last = it.base + ((int64_t)(it.len - 1) >> 2) * 256 + 3;
        CHECK(it.base >= 0 && last < d.view.packed_bytes, L + ": group residues");
      }
    }
    // A segment's bottom-row writer (lane 63 of the last band) stores at every step, the
    // columns -63 .. len + 62, kBndLead entries into the boundary; the next segment reads
    // columns 0 .. len - 1 of it.
    const int64_t reach_lo = kBndLead - 63, reach_hi = kBndLead + (int64_t)it.len + 62;
    // segment chain
    CHECK(it.nsegments >= 1 && it.segment >= 0 && it.segment < it.nsegments, L + ": segment");
    if (it.segment == 0) {
      CHECK(it.xin < 0 && it.prog_in < 0 && it.band0 == 0, L + ": first segment reads nothing");
    } else {
      CHECK(it.xin >= 0 && it.xin + kBndLead + it.len <= p.xbnd_elems, L + ": boundary read range");
      CHECK(it.prog_in >= 0 && it.prog_in < p.nprog, L + ": progress counter read");
      auto w = writer_at.find(it.prog_in);
      CHECK(w != writer_at.end(), L + ": waits for a segment that is not earlier in the list");
      const PairItem &prev = items[w->second];
      CHECK(prev.out == it.out && prev.query == it.query && prev.segment == it.segment - 1 &&
                prev.band1 == it.band0 && prev.xout == it.xin && prev.nsegments == it.nsegments,
            L + ": segment chain");
      prog_readers[(size_t)it.prog_in] += 1;
    }
    if (it.segment + 1 < it.nsegments) {
      CHECK(it.xout + reach_lo >= 0 && it.xout + reach_hi < p.xbnd_elems,
            L + ": boundary write range");
      extents.emplace_back(it.xout + reach_lo, it.xout + reach_hi);
      CHECK(it.prog_out >= 0 && it.prog_out < p.nprog, L + ": progress counter write");
      CHECK(!writer_at.count(it.prog_out), L + ": progress counter written twice");
      writer_at[it.prog_out] = i;
      prog_writers[(size_t)it.prog_out] += 1;
    } else {
      CHECK(it.xout < 0 && it.prog_out < 0 && it.band1 == nb, L + ": last segment ends the query");
      cover[{it.query, it.out}] += 1;  // a complete pair (or chain)
    }
    if (second && (*second)[i].len >= 0) {
      // the second pair of a two-pair item shares the first one's rows, segment and
      // boundary rows (it has none of its own)
      const PairItem &b = (*second)[i];
      CHECK(b.segment == it.segment && b.nsegments == it.nsegments,
            L + ": the two pairs of an item are the same segment");
      CHECK(b.query == it.query && b.band0 == it.band0 && b.band1 == it.band1,
            L + ": the two pairs of an item share the query rows");
      CHECK(b.len <= it.len, L + ": the first pair of a two-pair item is the longer");
      CHECK(b.out >= 0 && b.out < d.view.n_seqs && d.len[(size_t)b.out] == b.len,
            L + ": second pair's sequence");
      if (it.segment > 0) {
        const PairItem &pb = (*second)[writer_at[it.prog_in]];
        CHECK(pb.out == b.out && pb.segment == b.segment - 1,
              L + ": the second pair's segment chain");
      }
      if (b.segment + 1 == b.nsegments) cover[{b.query, b.out}] += 1;
      n_split_duos += it.nsegments > 1;
    }
  }
}

void check_plan(const Plan &p, const Db &d, const std::vector<int64_t> &qoff, int64_t nq) {
  const DbView &v = d.view;
  CHECK((int64_t)p.lens.size() == nq && (int64_t)p.qd.size() == nq, "per-query vectors");
  // profiles and score rows
  for (int64_t q = 0; q < nq; ++q) {
    const QueryDesc &qd = p.qd[(size_t)q];
    CHECK(qd.m == qoff[q + 1] - qoff[q], "query length");
    CHECK(qd.out == q * v.n_seqs, "score row offset");
    CHECK(qd.qp16 >= 0 && qd.qp16 + (int64_t)qd.nstrips * kCodes * 2 * p.T <= p.qp16_elems,
          "one-query profile range");
    CHECK((int64_t)qd.nstrips * 2 * p.T >= (p.q2 ? 0 : qd.m), "strips cover the query");
    CHECK(qd.mrows >= qd.m && qd.mrows == qd.nbands * 64 * kIntraR, "intra-task profile rows");
    CHECK(qd.qp8 >= 0 && qd.qp8 + (int64_t)kCodes * qd.mrows <= p.qp8_elems,
          "intra-task profile range");
  }
  // query pairs of the two-query kernel: every query once
  std::vector<int> in_pair((size_t)nq, 0);
  if (p.q2) {
    for (const QueryPair &qp : p.pairs) {
      CHECK(qp.qa >= 0 && qp.qa < nq && qp.qb < nq, "pair members");
      in_pair[(size_t)qp.qa] += 1;
      if (qp.qb >= 0) {
        in_pair[(size_t)qp.qb] += 1;
        CHECK(p.lens[(size_t)qp.qb] <= p.lens[(size_t)qp.qa], "the longer query of a pair first");
      }
      CHECK((int64_t)qp.nstrips * p.T >= p.lens[(size_t)qp.qa], "pair strips cover both");
      CHECK(qp.qp2 >= 0 && qp.qp2 + (int64_t)qp.nstrips * kCodes * p.T <= p.qp2_elems,
            "pair profile range");
    }
    for (int64_t q = 0; q < nq; ++q) CHECK(in_pair[(size_t)q] == 1, "query in exactly one pair");
  } else {
    CHECK(p.pairs.empty(), "pairs without the two-query kernel");
  }
  // coverage
  CHECK(p.ngroups_inter >= 0 && p.ngroups_inter <= v.ngroups, "routed groups");
  const int64_t units = p.q2 ? (int64_t)p.pairs.size() : nq;
  CHECK(p.nitems16 == (int64_t)p.ngroups_inter * units, "inter-task items");
  std::map<std::pair<int, int>, int> cover;
  std::vector<int> writers((size_t)std::max(0, p.nprog), 0), readers((size_t)std::max(0, p.nprog), 0);
  CHECK(p.second.size() == p.longitems.size(), "one second entry per main item");
  std::vector<std::pair<int64_t, int64_t>> extents;  // boundary entries each writer touches
  check_items(p, d, p.longitems, &p.second, p.R, nq, cover, writers, readers, extents,
              "main list");
  CHECK(p.crititems.empty() || p.crit_R == 4 || p.crit_R == 8, "critical rows per lane");
  check_items(p, d, p.crititems, nullptr, p.crit_R ? p.crit_R : kCritR, nq, cover, writers,
              readers, extents, "critical list");
  std::sort(extents.begin(), extents.end());
  for (size_t k = 1; k < extents.size(); ++k)
    CHECK(extents[k].first > extents[k - 1].second, "two segment boundaries overlap");
  for (int32_t k = 0; k < p.nprog; ++k)
    CHECK(writers[(size_t)k] == 1 && readers[(size_t)k] == 1, "each boundary written and read once");
  for (int64_t q = 0; q < nq; ++q) {
    const bool empty = p.lens[(size_t)q] == 0;
    for (int32_t g = 0; g < v.ngroups; ++g) {
      const GroupDesc &gd = v.groups[g];
      for (int32_t l = 0; l < gd.count; ++l) {
        const int orig = v.perm[gd.first + l];
        const int c = cover.count({(int)q, orig}) ? cover[{(int)q, orig}] : 0;
        if (g < p.ngroups_inter)
          CHECK(c == 0, "a sequence of an inter-task group also has an intra-task item");
        else
          CHECK(c == (empty ? 0 : 1), "a routed sequence not covered exactly once");
      }
    }
    for (const LongSeq &L : v.longs) {
      const int c = cover.count({(int)q, L.orig}) ? cover[{(int)q, L.orig}] : 0;
      CHECK(c == (empty ? 0 : 1), "a long sequence not covered exactly once");
    }
  }
  // launch geometry
  CHECK((p.nitems16 > 0) == (p.grid16 > 0) || p.nitems16 == 0, "inter-task grid");
  CHECK(p.grid16 <= std::max<int64_t>(1, p.nitems16), "inter-task grid beyond its items");
  CHECK(p.longitems.empty() || p.grid_long > 0, "main intra-task grid");
  CHECK(p.crititems.empty() || p.grid_crit > 0, "critical-pair grid");
  CHECK(p.grid32 == p.grid_long + p.grid_re + p.grid_crit, "intra-task slots");
  CHECK(p.main_waves == 4 || p.main_waves == 8, "main waves");
  CHECK(p.R == 2 || p.R == 4 || p.R == 8 || p.R == 16, "rows per lane");
  // workspace and staging
  CHECK(p.need_flagged >= 1, "recompute list");
  // inter-task boundary slots: every item's group fits the slot of every wave that may
  // take it (items [0, wide_items) only the big-slot waves, the others every wave)
  {
    const size_t wpc = 64 * (p.q2 ? 2 : 1);
    int32_t inter_cols = 0;
    for (int32_t g = 0; g < p.ngroups_inter; ++g) inter_cols = std::max(inter_cols, v.groups[g].ncols);
    CHECK(p.bnd16_slot >= (size_t)inter_cols * wpc, "inter-task boundary slot");
    if (p.big_waves > 0) {
      CHECK(p.big_waves <= p.grid16 && p.wide_items > 0 && p.wide_items < p.nitems16 &&
                p.wide_items % units == 0, "two classes of boundary slots");
      const int32_t g_small = p.ngroups_inter - 1 - (int32_t)(p.wide_items / units);
      for (int32_t g = 0; g <= g_small; ++g)
        CHECK((size_t)v.groups[g].ncols * wpc <= p.bnd16_small, "a group wider than the small slots");
      CHECK(bnd16_words(p) == (size_t)p.big_waves * p.bnd16_slot +
                                  (size_t)(p.grid16 - p.big_waves) * p.bnd16_small,
            "boundary slot words");
    } else {
      CHECK(p.wide_items == 0 && p.bnd16_small == p.bnd16_slot, "one class of boundary slots");
    }
  }
  // a band buffer holds the bottom row's reach, kBndLead entries in (see above)
  CHECK(p.bnd32_stride >= kBndLead + v.max_len + 63, "band buffer");
  // band rings: a workgroup of W waves needs max(W + 1, 2W) band buffers, and the three
  // launches' slot ranges follow one another
  auto ring = [&](int w) { return (size_t)std::max(w + 1, 2 * w) * p.bnd32_stride; };
  CHECK(p.bnd32_slot >= ring(p.main_waves), "main band ring");
  CHECK(p.bnd32_slot_re >= ring(kIntraWaves), "recompute band ring");
  CHECK(p.bnd32_slot_crit >= ring(kCritWaves), "critical-pair band ring");
  CHECK(p.bnd32_off_re >= (size_t)p.grid_long * p.bnd32_slot, "band rings overlap");
  CHECK(p.bnd32_off_crit >= p.bnd32_off_re + (size_t)p.grid_re * p.bnd32_slot_re,
        "band rings overlap");
  CHECK(p.bnd32_elems >= p.bnd32_off_crit + (size_t)p.grid_crit * p.bnd32_slot_crit,
        "band rings beyond the buffer");
  CHECK(p.main_per_cu == (p.main_waves == 8 ? 1 : (p.crititems.empty() ? 3 : 2)),
        "main workgroups per CU");
  CHECK(p.grid_long <= (int64_t)std::max(1, v.num_cu) * p.main_per_cu, "main grid per CU");
  CHECK(p.grid_crit <= std::max(1, v.num_cu), "critical-pair grid per CU");
  const size_t parts[][2] = {
      {0, (size_t)p.qbytes},
      {p.off_qoff, (size_t)(nq + 1) * 8},
      {p.off_qd, (size_t)nq * sizeof(QueryDesc)},
      {p.off_mx, (size_t)v.alphabet * v.alphabet * 4},
      {p.off_qo, (size_t)nq * 4},
      {p.off_li, p.longitems.size() * sizeof(PairItem)},
      {p.off_se, p.second.size() * sizeof(PairItem)},
      {p.off_cr, p.crititems.size() * sizeof(PairItem)},
      {p.off_pr, p.pairs.size() * sizeof(QueryPair)}};
  size_t end = 0;
  for (const auto &part : parts) {
    CHECK(part[0] % 64 == 0 && part[0] >= end, "staging part overlaps the one before");
    end = part[0] + part[1];
  }
  CHECK(end <= p.stage_bytes, "staging block too small");
}

}  // namespace

int main() {
  std::mt19937_64 rng(1702);
  Occupancy occ;
  const int inter16[] = {8, 16, 24, 32, 40}, inter16_blocks[] = {24, 16, 12, 8, 8};
  const int q2[] = {8, 16, 24, 28, 32, 40}, q2_blocks[] = {24, 16, 12, 12, 8, 8};
  for (int k = 0; k < 5; ++k) occ.inter16[inter16[k]] = inter16_blocks[k];
  for (int k = 0; k < 6; ++k) occ.inter16q2[q2[k]] = q2_blocks[k];
  auto pick = [&](std::initializer_list<int64_t> xs) {
    return *(xs.begin() + (size_t)(rng() % xs.size()));
  };
  std::lognormal_distribution<double> logn(std::log(200.0), 0.9);
  const int cases = 3000;
  int64_t n_split = 0, n_crit = 0, n_duo = 0, n_routed = 0, n_q2 = 0, n_slots2 = 0;
  for (int c = 0; c < cases; ++c) {
    g_case = "case " + std::to_string(c);
    const int num_cu = (int)pick({1, 4, 16, 256});
    const int64_t n = (int64_t)pick({0, 1, 5, 64, 65, 300, 2000});
    std::vector<int64_t> len((size_t)n);
    for (auto &x : len) {
      const int kind = (int)(rng() % 20);
      x = kind == 0 ? 0 : kind == 1 ? (int64_t)(10000 + rng() % 30000)
                                    : std::min<int64_t>(8000, (int64_t)logn(rng));
    }
    const int64_t intra_min = pick({8192, 500, 1 << 30});
    Db d = make_db(len, intra_min, num_cu, (int)pick({4, 20, 24}));
    const int64_t nq = (int64_t)pick({0, 1, 2, 3, 7});
    std::vector<int64_t> qoff(1, 0);
    for (int64_t q = 0; q < nq; ++q) {
      const int kind = (int)(rng() % 10);
      const int64_t m = kind == 0 ? 0 : kind == 1 ? (int64_t)(5000 + rng() % 35000)
                                                  : (int64_t)(1 + rng() % 1500);
      qoff.push_back(qoff.back() + m);
    }
    Knobs k;
    k.strip_rows = pick({0, 0, 16, 24, 28, 40, 12});
    k.grid_waves = pick({0, 0, 1, 3});
    k.route_len = pick({0, 0, 1, 300, 1 << 30});
    k.wide_len = pick({0, 0, 100, 5000});
    k.max_segments = pick({0, 0, 1, 3});
    k.intra_rows = pick({0, 0, 2, 4, 8, 16});
    k.intra_pairs = pick({1, 1, 0, 2});
    k.query_pairs = pick({1, 1, 0});
    k.main_waves = pick({0, 0, 4, 8});
    k.crit_rows = pick({0, 0, 4, 8});
    k.crit_share = pick({0, 0, 10, 30, 100});
    g_case += " n=" + std::to_string(n) + " nq=" + std::to_string(nq) + " cu=" +
              std::to_string(num_cu);
    const Plan p = make_plan(d.view, qoff.data(), nq, k, occ);
    check_plan(p, d, qoff, nq);
    n_split += p.nprog > 0;
    n_crit += !p.crititems.empty();
    n_duo += p.nduos > 0;
    n_routed += p.ngroups_inter < d.view.ngroups;
    n_q2 += p.q2;
    n_slots2 += p.big_waves > 0;
  }
  // batches of 64 queries against databases that fill the device: the two-query kernel's
  // boundary slots then come in two classes
  for (int c = 0; c < 6; ++c) {
    g_case = "batch case " + std::to_string(c);
    const int64_t n = (int64_t)pick({6000, 12000, 20000});
    std::vector<int64_t> len((size_t)n);
    for (auto &x : len) x = std::max<int64_t>(10, std::min<int64_t>(8000, (int64_t)logn(rng)));
    Db d = make_db(len, 8192, 256, 24);
    std::vector<int64_t> qoff(1, 0);
    for (int q = 0; q < 64; ++q) qoff.push_back(qoff.back() + 50 + (int64_t)(rng() % 4951));
    Knobs k;
    k.strip_rows = pick({0, 28, 24});
    const Plan p = make_plan(d.view, qoff.data(), 64, k, occ);
    check_plan(p, d, qoff, 64);
    n_q2 += p.q2;
    n_slots2 += p.big_waves > 0;
  }
  // Rows per lane on a database shaped like the long-sequence mix (9,900 log-normal
  // sequences of median 300 and 100 of 10,000-35,000 residues): the choices measured
  // fastest on MI355X for queries of 144 to 35,000 residues (300: R = 2, 1000: 4,
  // 2005: 8, 5478 and 35000: 16, 5478 with a critical-pair launch and four-wave
  // workgroups).
  {
    g_case = "long-mix rows per lane";
    std::mt19937_64 r2(35000);
    std::lognormal_distribution<double> ln300(std::log(300.0), 0.8);
    std::vector<int64_t> len;
    for (int i = 0; i < 9900; ++i)
      len.push_back(std::max<int64_t>(10, std::min<int64_t>(8000, (int64_t)ln300(r2))));
    for (int i = 0; i < 99; ++i) len.push_back(10000 + (int64_t)(r2() % 25001));
    len.push_back(35000);
    Db d = make_db(len, 8192, 256, 24);
    const int64_t ms[] = {300, 1000, 2005, 5478, 35000};
    const int want[] = {2, 4, 8, 16, 16};
    for (int i = 0; i < 5; ++i) {
      const int64_t qoff[2] = {0, ms[i]};
      const Plan p = make_plan(d.view, qoff, 1, Knobs{}, occ);
      check_plan(p, d, std::vector<int64_t>(qoff, qoff + 2), 1);
      if (p.R != want[i])
        std::fprintf(stderr, "long mix, %lld-row query: R = %d (want %d)\n", (long long)ms[i],
                     p.R, want[i]);
      CHECK(p.R == want[i], "rows per lane on the long mix");
    }
  }
  // the random cases must reach every kind of item
  if (!n_split || !n_crit || !n_duo || !n_routed || !n_q2 || !n_split_duos || !n_slots2)
    fail("a kind of item never planned");
  std::printf("planner ok: %d cases (split pairs %lld, critical pairs %lld, two-pair items "
              "%lld, split two-pair segments %lld, routed groups %lld, query pairs %lld, two "
              "classes of boundary slots %lld)\n", cases,
              (long long)n_split, (long long)n_crit, (long long)n_duo, (long long)n_split_duos,
              (long long)n_routed, (long long)n_q2, (long long)n_slots2);
  return 0;
}
