// Host-side planning of a search: strip height, routing of long groups to the intra-task
// kernel, rows per lane, intra-task work items (split pairs, critical pairs, two-pair
// items), launch geometry, workspace sizes and the staging layout.  Pure host code (no
// HIP calls): the library calls it before every launch sequence, and a CPU test builds
// it on its own, with address and undefined-behaviour sanitizers, to check that every
// (query, sequence) pair is covered exactly once, that split pairs chain only backwards
// and that every offset fits its buffer.
#include "planner.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <utility>

namespace swmi {

// the boundary rows below leave room for their writers' reach (kBndLead before column 0)
static_assert(kBndLead == 64, "boundary padding of 128 entries per row assumes a lead of 64");

namespace {

// Rows per lane of the intra-task kernel for one search.  Its band is 64R query rows,
// and a step (one anti-diagonal of a band) issues about 7.5 R + 14 instructions: the
// lane's per-step overhead (residue and boundary shifts, the profile request) is paid
// once per R rows, so over many bands R = 16 issues the fewest instructions per cell.
// But a pair of n columns is swept in about n steps whatever R, its bands pipelined
// kIntraLag chunks of 64 steps apart, so with few bands the step time of the longest
// pair sets the search's critical path, and shorter steps win.  For each R in
// {16, 8, 4, 2} the search time is estimated as the larger of
//   - the throughput time: every intra-task pair's bands of 64R rows at the kernel's
//     rate, about 3.6e12 cells/s at R = 16 on MI355X, scaling as R / (7.5 R + 14); a
//     query with more bands than a workgroup has waves is swept in several rounds, where
//     short steps measured less efficient (0.77 at R = 8, 0.34 at R = 4, on a 35,000-row
//     query; 0.15 assumed at R = 2), and R = 2 reached 0.45 of that rate even with few
//     bands (a 1,000-row query over 6.4e6 residues), and
//   - the longest pair's path: n + 63 steps per band of a wave alone on its SIMD, about
//     0.083 + 0.0118 R us (measured 0.13, 0.17 and 0.27 us at R = 4, 8 and 16); several
//     bands (a pair at least `wide_len` long) are a pipeline of a workgroup's waves,
//     alone on their SIMDs up to four bands and 1.66 times slower beyond (two waves per
//     SIMD), and a pair of more than four bands at R > kCritR may instead run at kCritR
//     rows in the critical-pair launch (segments of four bands, one wave per SIMD),
// and the smallest estimate wins, a tie going to the larger R (R = 16 and 8 tie when
// both leave the longest pairs to the critical-pair launch, and 16 measured faster
// there).  (With step times priced from instruction counts, the 2005-row query over the
// long-sequence mix took R = 4, 7.5 ms, against 6.2 ms at R = 8, which it now takes.)  R = 2 is weighed only when the path at R = 4 exceeds a millisecond: below
// that, per-search costs the estimate leaves out dominate, and R = 2 measured no faster
// (a 144-row query over 2,000 sequences of at most 2,000 residues).  (Measured on the
// long-sequence mix, whose longest sequence has 35,000 residues: queries of 300 and
// 1,000 residues ran 1.8 and 2.8 times faster at R = 4 than at the R an instruction
// count alone picks.)
int choose_R(const std::vector<int64_t> &lens, double intra_res, int64_t n_max,
             int64_t wide_len, int num_cu, const Knobs &k, bool *throughput_bound) {
  auto step_scale = [](int R) { return (7.5 * R + 14.0) / (7.5 * 16 + 14.0); };
  auto bands = [](int64_t m, int R) { return (m + 64 * R - 1) / (64 * R); };
  // anti-diagonal step of a wave alone on its SIMD (MI355X: about 0.13, 0.17 and 0.27 us
  // at R = 4, 8 and 16); two waves on a SIMD take 1.66 times as long
  auto step_alone = [](int R) { return 0.083e-6 + 0.0118e-6 * R; };
  auto pipe = [&](int64_t m, int R, int waves) {  // a band pipeline of `waves` waves
    const int64_t b = bands(m, R);
    const double chunks = (double)((n_max + 126) / 64 + (int64_t)kIntraLag * (b - 1));
    return chunks * 64 * step_alone(R) * (std::min<int64_t>(b, waves) > 4 ? 1.66 : 1.0);
  };
  // (throughput time, longest path) at R
  auto estimate = [&](int R, double &thr, double &path) {
    const double rate = 3.6e12 * (R / 16.0) / step_scale(R) * (std::max(1, num_cu) / 256.0);
    const double eff_rounds = R == 16 ? 1.0 : (R == 8 ? 0.77 : (R == 4 ? 0.34 : 0.15));
    const double eff_few = R == 2 ? 0.45 : 1.0;
    thr = 0;
    path = 0;
    for (int64_t m : lens) {
      if (m == 0) continue;
      const int64_t b = bands(m, R);
      thr += (double)b * 64 * R * intra_res / (rate * (b > kIntraWaves ? eff_rounds : eff_few));
      double t;
      if (b >= 2 && n_max >= wide_len) {
        t = pipe(m, R, kIntraWaves);
        // a pair of more than four bands may be split into the critical-pair launch
        if (R > kCritR && b > kCritWaves) t = std::min(t, pipe(m, kCritR, kCritWaves));
      } else {
        t = (double)b * (double)(n_max + 63) * step_alone(R);
      }
      path = std::max(path, t);
    }
  };
  int best = kIntraR;
  const int64_t forced = k.intra_rows;
  if (forced == 2 || forced == 4 || forced == 8 || forced == 16) {
    best = (int)forced;
  } else if (n_max > 0 && intra_res > 0) {
    double best_cost = 1e300, path4 = 0;
    for (int R : {16, 8, 4, 2}) {
      if (R == 2 && path4 < 1e-3) break;
      double thr, path;
      estimate(R, thr, path);
      if (R == 4) path4 = path;
      const double cost = std::max(thr, path);
      if (cost < best_cost * 0.999) {
        best_cost = cost;
        best = R;
      }
    }
  }
  double thr = 0, path = 0;
  if (n_max > 0 && intra_res > 0) estimate(best, thr, path);
  *throughput_bound = thr >= 1.2 * path;
  return best;
}

// Strip half-height T for the inter-task kernel: the fewest padded query rows, weighted
// by the measured relative per-cell speed of each compiled height on gfx950 (T = 24 runs
// at three waves per SIMD and was fastest on the full-scale search).  The pair kernel
// (`pairs`) also has T = 28, still at three waves per SIMD and 2% faster on the batched
// search; its per-strip row count is T, and `lens` then holds twice each pair's rows.
int choose_T(const std::vector<int64_t> &lens, const Knobs &k, const Occupancy &occ,
             bool pairs = false) {
  const int64_t forced = k.strip_rows;
  if (forced > 0 && forced <= kMaxStripRows &&
      (pairs ? occ.inter16q2[forced] : occ.inter16[forced]) > 0)
    return (int)forced;
  struct Cand { int T; double speed; };
  static const Cand single[] = {{24, 1.0}, {40, 0.985}, {32, 0.968}, {16, 0.89}};
  static const Cand paired[] = {{28, 1.02}, {24, 1.0}, {40, 0.98}, {32, 0.962}, {16, 0.938}};
  const Cand *cands = pairs ? paired : single;
  const int ncand = pairs ? 5 : 4;
  int best = 24;
  double best_cost = 1e300;
  for (int k = 0; k < ncand; ++k) {
    const Cand &c = cands[k];
    double cost = 0;
    for (int64_t m : lens) cost += (double)((m + 2 * c.T - 1) / (2 * c.T)) * 2.0 * c.T;
    cost /= c.speed;
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best = c.T;
    }
  }
  return best;
}

// One plan with the given knobs (make_plan below may plan twice).
Plan plan_with(const DbView &db, const int64_t *qoff, int64_t nq, const Knobs &k,
               const Occupancy &occ) {
  Plan p;
  const int A = db.alphabet;
  std::vector<int64_t> &lens = p.lens;
  lens.resize((size_t)nq);
  for (int64_t q = 0; q < nq; ++q) lens[q] = qoff[q + 1] - qoff[q];
  // inter-task items visit each group's queries longest first
  std::vector<int32_t> &qorder = p.qorder;
  qorder.resize((size_t)nq);
  std::iota(qorder.begin(), qorder.end(), 0);
  std::stable_sort(qorder.begin(), qorder.end(),
                   [&](int32_t x, int32_t y) { return lens[x] > lens[y]; });
  // A batched search pairs its queries (longest first) in the two-query inter-task
  // kernel, whose strips hold T rows of both; the strip height is chosen on the padded
  // rows of the pairs.
  const bool q2 = p.q2 = k.query_pairs != 0 && nq >= 2;
  if (q2) {
    std::vector<int64_t> pair_rows;
    for (int64_t k = 0; k < nq; k += 2) {
      QueryPair qp;
      qp.qa = qorder[(size_t)k];
      qp.qb = k + 1 < nq ? qorder[(size_t)k + 1] : -1;
      qp.qp2 = 0;
      qp.nstrips = 0;
      qp.pad = 0;
      p.pairs.push_back(qp);
      pair_rows.push_back(2 * lens[(size_t)qp.qa]);  // ceil(2m / 2T) * 2T = 2T ceil(m / T)
    }
    p.T = choose_T(pair_rows, k, occ, true);
  } else {
    p.T = choose_T(lens, k, occ);
  }
  const int band = 64 * kIntraR;
  p.qd.resize((size_t)nq);
  for (int64_t q = 0; q < nq; ++q) {
    QueryDesc &d = p.qd[q];
    d.m = (int32_t)lens[q];
    d.nstrips = q2 ? 0 : (int32_t)((lens[q] + 2 * p.T - 1) / (2 * p.T));
    d.nbands = (int32_t)((lens[q] + band - 1) / band);
    d.mrows = d.nbands * band;
    d.qp16 = p.qp16_elems;
    d.qp8 = p.qp8_elems;
    d.out = q * db.n_seqs;
    p.qp16_elems += (int64_t)d.nstrips * kCodes * 2 * p.T;
    p.qp8_elems += (int64_t)kCodes * d.mrows;
  }
  for (QueryPair &qp : p.pairs) {
    qp.nstrips = (int32_t)((lens[(size_t)qp.qa] + p.T - 1) / p.T);
    qp.qp2 = p.qp2_elems;
    p.qp2_elems += (int64_t)qp.nstrips * kCodes * p.T;
  }
  const int64_t nunits = q2 ? (int64_t)p.pairs.size() : nq;  // inter-task items per group
  // launch geometry of the inter-task kernel
  int per_cu = (int)k.grid_waves;
  if (per_cu <= 0)
    per_cu = std::max(1, q2 ? occ.inter16q2[p.T] : occ.inter16[p.T]);
  p.per_cu = per_cu;
  const int64_t lanes = (int64_t)per_cu * db.num_cu * 64;

  // Route the longest groups to the intra-task kernel.  One lane runs a whole alignment
  // in the inter-task kernel, so a group of length L costs about L * m on one wave; keep
  // L below twice the average number of residues per lane (weighted by the number of
  // equally long queries), else that wave becomes the critical path.
  // (paired queries: a lane runs both queries of a pair at once, so a pair counts once)
  int64_t sum_m = 0, max_m = 1;
  for (int64_t q = 0; q < nq; ++q) max_m = std::max(max_m, lens[q]);
  if (q2)
    for (const QueryPair &qp : p.pairs) sum_m += lens[(size_t)qp.qa];
  else
    for (int64_t q = 0; q < nq; ++q) sum_m += lens[q];
  const double weight = (double)sum_m / (double)max_m;
  int64_t route = (int64_t)(2.0 * (double)db.short_residues * weight / (double)lanes);
  route = std::max<int64_t>(route, 64);
  const int64_t forced_route = k.route_len;
  if (forced_route > 0) route = forced_route;
  int32_t ninter = db.ngroups;
  while (ninter > 0 && db.groups[ninter - 1].maxlen > route) --ninter;
  p.ngroups_inter = ninter;

  // rows per lane of the intra-task kernel, from the pairs it gets (long sequences and
  // routed groups, the latter estimated at their longest sequence)
  const int64_t wide_len = k.wide_len > 0 ? k.wide_len
                                                      : (int64_t)64 * 6 * kIntraLag;
  {
    double intra_res = 0;
    int64_t n_max = 0;
    for (const auto &L : db.longs) {
      intra_res += L.len;
      n_max = std::max<int64_t>(n_max, L.len);
    }
    for (int32_t g = ninter; g < db.ngroups; ++g) {
      intra_res += (double)db.groups[g].count * db.groups[g].maxlen;
      n_max = std::max<int64_t>(n_max, db.groups[g].maxlen);
    }
    // A throughput-bound search (estimated throughput time at least 1.2 times the
    // longest path) runs four-wave workgroups, two per CU: the same occupancy, and one
    // fits beside a critical-pair workgroup (an 8-wave one does not).  Otherwise
    // eight-wave workgroups give a pair's few band waves a SIMD each (the rest of the
    // workgroup idles).  (Long-sequence mix on MI355X: 5478-residue query 14.7 -> 10.8
    // ms with four-wave workgroups; a 2005-residue query, at a ratio of 1.1, 8.2 -> 9.3.)
    bool throughput_bound = false;
    p.R = choose_R(lens, intra_res, n_max, wide_len, db.num_cu, k, &throughput_bound);
    p.throughput_bound = throughput_bound;
    const int64_t mw = k.main_waves;
    p.main_waves = (mw == 4 || mw == 8) ? (int)mw : (throughput_bound ? kNarrowWaves : kIntraWaves);
  }
  p.nbandsR.resize((size_t)nq);
  for (int64_t q = 0; q < nq; ++q)
    p.nbandsR[q] = (int32_t)((lens[q] + 64 * p.R - 1) / (64 * p.R));

  // intra-task items: long sequences and the sequences of routed groups, for every query;
  // "wide" (a whole workgroup per pair) when the pair has several bands and enough
  // columns to fill the band pipeline, else "narrow" (one wave per pair); each part
  // longest first
  std::vector<std::pair<double, PairItem>> wide, narrow;
  auto add_item = [&](int64_t base, int32_t cstride, int32_t len, int32_t orig, int64_t q) {
    PairItem it;
    it.base = base;
    it.cstride = cstride;
    it.len = len;
    it.out = orig;
    it.query = (int32_t)q;
    it.band0 = 0;
    it.band1 = p.nbandsR[q];
    it.xin = it.xout = -1;
    it.prog_in = it.prog_out = -1;
    it.segment = 0;
    it.nsegments = 1;
    const double cost = (double)len * (double)lens[q];
    const bool is_wide = len >= wide_len && p.nbandsR[q] >= 2;
    (is_wide ? wide : narrow).emplace_back(cost, it);
  };
  for (int64_t q = 0; q < nq; ++q) {
    if (lens[q] == 0) continue;
    for (const auto &L : db.longs) add_item(L.base, 4, L.len, L.orig, q);
    for (int32_t g = ninter; g < db.ngroups; ++g) {
      const GroupDesc &gd = db.groups[g];
      for (int32_t l = 0; l < gd.count; ++l)
        add_item(gd.base + 4 * l, 256, db.lens[gd.first + l], db.perm[gd.first + l], q);
    }
  }
  auto by_cost = [](const std::pair<double, PairItem> &x, const std::pair<double, PairItem> &y) {
    return x.first > y.first;
  };
  std::stable_sort(wide.begin(), wide.end(), by_cost);
  std::stable_sort(narrow.begin(), narrow.end(), by_cost);
  // Critical path of the longest pairs.  A workgroup sweeps its bands in rounds of its
  // W = p.main_waves waves, so a pair of nb bands takes about ceil(nb / W) sweeps of its
  // columns; cut into segments of at most W consecutive bands on workgroups of
  // their own, the bands form one pipeline (nc + kIntraLag * (nb - 1) chunks), and with at
  // most 4 bands per segment each band's wave has a SIMD to itself.  A pair is split as
  // little as keeps its estimated time within half the estimated time of the whole
  // intra-task search (a pair may be claimed only after other work has run); 4-band
  // segments, which leave half a compute unit idle, only when even the full pipeline
  // would outlast the whole search.  Segments of a pair are consecutive in the list, so
  // segment j is always claimed after segment j - 1 (the only one it waits for).
  //   (one step of a wave with R = 16: about 0.5 us with two waves per SIMD, 0.25 us
  //   alone; the kernel then sustains about 2.5e12 cells/s over the whole chip: MI355X
  //   measurements; both scale with the instructions per step, 7.5 R + 14)
  double intra_cells = 0;
  for (auto &x : wide) intra_cells += x.first;
  for (auto &x : narrow) intra_cells += x.first;
  const double step_scale = (7.5 * p.R + 14.0) / (7.5 * 16 + 14.0);
  const double t_search = intra_cells / (2.5e12 * (p.R / 16.0) / step_scale) *
                          (256.0 / std::max(1, db.num_cu));
  const double t_step = 0.5e-6 * step_scale;
  const int64_t cap = k.max_segments;
  // Narrow pairs of the same query can run two per wave as one packed int16 item
  // (consecutive in cost order, so of similar length).  Such an item does two pairs'
  // cells per step at about 1.45 times the single step's time, which pays when the
  // search is throughput-bound and hurts the critical path when it is not, so pairing
  // is used only when there are at least two narrow items per wave slot, and only for
  // items whose paired time stays under a quarter of the estimated search time.  Wide
  // pairs stay single, in int32.  (Knob value 2 pairs every unsplit pair, wide ones
  // included: a test setting.)
  const int64_t pair_mode = k.intra_pairs;
  const bool pair_all = pair_mode == 2;
  const bool pair_narrow = pair_mode == 1 &&
                           narrow.size() >= 2 * (size_t)std::max(1, db.num_cu) * kIntraWaves;
  const bool pair_wide = pair_mode == 1 && wide.size() >= 2 * (size_t)std::max(1, db.num_cu);
  const bool pairs16 = pair_all || pair_narrow || pair_wide;
  PairItem none;
  std::memset(&none, 0, sizeof(none));
  none.len = -1;
  none.out = -1;
  std::vector<int64_t> pending((size_t)nq, -1);  // index in longitems of an unpaired item
  auto emit = [&](const PairItem &it, bool pairable) {
    if (pairs16 && pairable) {
      int64_t &pend = pending[(size_t)it.query];
      if (pend >= 0) {
        p.second[(size_t)pend] = it;
        pend = -1;
        ++p.nduos;
        return;
      }
      pend = (int64_t)p.longitems.size();
    }
    p.longitems.push_back(it);
    p.second.push_back(none);
  };
  // Segments of a split pair (and, for a two-pair item, of its second pair, which shares
  // the first one's bands and boundary rows) are appended consecutively, so segment j is
  // always claimed after segment j - 1.
  // Each boundary row holds kBndLead entries before column 0 and at least 63 after column
  // len - 1: its writer stores the columns -63 .. len + 62 its sweep passes through.
  auto push_segments = [&](const PairItem &it, const PairItem *second, int32_t S) {
    const int32_t nb = it.band1;
    const int64_t npad = (((int64_t)it.len + 63) / 64) * 64 + 128;
    for (int32_t j = 0; j < S; ++j) {
      PairItem sg = it;
      sg.band0 = (int32_t)((int64_t)nb * j / S);
      sg.band1 = (int32_t)((int64_t)nb * (j + 1) / S);
      sg.segment = j;
      sg.nsegments = S;
      if (j > 0) {
        sg.xin = p.xbnd_elems - npad;
        sg.prog_in = p.nprog - 1;
      }
      if (j + 1 < S) {
        sg.xout = p.xbnd_elems;
        sg.prog_out = p.nprog;
        p.xbnd_elems += npad;
        p.nprog += 1;
      }
      p.longitems.push_back(sg);
      if (second) {
        PairItem sb = *second;
        sb.band0 = sg.band0;
        sb.band1 = sg.band1;
        sb.segment = j;
        sb.nsegments = S;
        p.second.push_back(sb);
        ++p.nduos;
      } else {
        p.second.push_back(none);
      }
    }
  };
  // Split pairs (the costliest, claimed first), then the unsplit wide ones.  When the
  // search is throughput-bound, consecutive split pairs of the same query, bands and
  // segment count run two per workgroup in packed int16 (each step about 1.45 times a
  // single one's, for twice the cells) if the paired pipeline stays within half the
  // estimated search time.
  struct Split {
    PairItem it;
    int32_t S;
    bool pairable;
  };
  std::vector<Split> splits;
  std::vector<PairItem> singles;
  std::vector<bool> singles_pairable;
  // The longest band pipeline of the split and critical pairs seen so far (wide pairs come
  // longest first): an item whose paired time stays within 0.6 of it, or within a quarter
  // of the estimated search time, is short enough to pair.  (Long-sequence mix on
  // MI355X: the 5478-residue query, whose split pairs' pipelines take about 9 ms of a
  // 10.4 ms search, 10.4 -> 10.2 ms with its longer narrow and wide pairs paired; the
  // 35000-residue query keeps the quarter, since pairing its longest narrow items, 35
  // bands swept by one wave, only lengthened the tail: 53.7 -> 55.9 ms.)
  double max_path = 0;
  auto pair_limit = [&]() { return std::max(0.25 * t_search, 0.6 * max_path); };
  for (auto &x : wide) {
    const PairItem &it = x.second;
    const int32_t nb = it.band1;
    const int64_t nc = ((int64_t)it.len + 126) / 64;
    const int64_t nce = std::max<int64_t>(nc, (int64_t)kIntraLag * p.main_waves);
    const int64_t lastb = nb - 1;
    const double whole = (double)((lastb / p.main_waves) * nce + kIntraLag * (lastb % p.main_waves) + nc);
    const double piped = (double)(nc + (int64_t)kIntraLag * lastb);
    const int32_t s8 = (nb + p.main_waves - 1) / p.main_waves, s4 = (nb + 3) / 4;
    int32_t S = 1;
    if (whole * 64 * t_step > 0.5 * t_search) S = piped * 64 * t_step <= t_search ? s8 : s4;
    if (cap > 0) S = std::min<int32_t>(S, (int32_t)cap);
    S = std::max<int32_t>(1, std::min(S, nb));
    if (S == 1) {
      singles.push_back(it);
      singles_pairable.push_back(pair_all || (pair_wide && 1.45 * whole * 64 * t_step <= pair_limit()));
      continue;
    }
    // A pair whose full pipeline would outlast the search sets its critical path; with
    // bands of 64 * kCritR rows a step takes 7.5 kCritR + 14 instructions instead of
    // 7.5 R + 14, over more, shorter bands, so such pairs get a launch of their own with
    // that height (segments of kCritWaves bands, one wave per SIMD) when it shortens their
    // pipeline.
    // (A wave alone on its SIMD steps in about 0.76 of t_step: 0.38 us at R = 16 on
    // MI355X, where latency keeps a step at about 1.7 times its instruction time.)
    // Rows per lane of that launch: 8 (bands of 512 rows), or 4 when SW_KNOB_CRIT_ROWS
    // asks for it.  (With 4 the step issues fewer instructions but the long mix's
    // 5478-residue query measured slower, 2,642 against 3,048 GCUPS: a step alone on its
    // SIMD is bound by latency, not by its instruction count.)
    p.crit_R = k.crit_rows > 0 ? (int)k.crit_rows : kCritR;
    const int Rc = p.crit_R;
    // (default share 20%: on the long mix the 5478-residue query ran 9.68-9.71 ms against
    // 9.87-9.90 with 50%; the other queries measured the same)
    const double share = k.crit_share > 0 ? (double)k.crit_share / 100.0 : 0.2;
    if (S == s4 && p.R > Rc && k.intra_rows == 0 && cap == 0 &&
        piped * 64 * 0.76 * t_step > share * t_search) {  // still critical with a SIMD per wave
      const int32_t nbc = (int32_t)((lens[it.query] + 64 * Rc - 1) / (64 * Rc));
      const double piped_c = (double)(nc + (int64_t)kIntraLag * (nbc - 1));
      const double step_c = (7.5 * Rc + 14.0) / (7.5 * p.R + 14.0);
      if (piped_c * step_c < piped) {
        const int32_t Sc = (nbc + kCritWaves - 1) / kCritWaves;
        const int64_t npad = (((int64_t)it.len + 63) / 64) * 64 + 128;
        for (int32_t j = 0; j < Sc; ++j) {
          PairItem sg = it;
          sg.band0 = (int32_t)((int64_t)nbc * j / Sc);
          sg.band1 = (int32_t)((int64_t)nbc * (j + 1) / Sc);
          sg.segment = j;
          sg.nsegments = Sc;
          if (j > 0) {
            sg.xin = p.xbnd_elems - npad;
            sg.prog_in = p.nprog - 1;
          }
          if (j + 1 < Sc) {
            sg.xout = p.xbnd_elems;
            sg.prog_out = p.nprog;
            p.xbnd_elems += npad;
            p.nprog += 1;
          }
          p.crititems.push_back(sg);
        }
        max_path = std::max(max_path, piped_c * 64 * 0.76 * t_step * step_c);
        continue;
      }
    }
    max_path = std::max(max_path, piped * 64 * t_step);
    const bool pairable = pair_all || (pair_mode == 1 && p.throughput_bound &&
                                       1.45 * piped * 64 * t_step <= 0.5 * t_search);
    splits.push_back({it, S, pairable});
  }
  for (size_t i = 0; i < splits.size(); ++i) {
    const Split &a = splits[i];
    if (a.pairable && i + 1 < splits.size()) {
      const Split &b = splits[i + 1];
      if (b.pairable && b.it.query == a.it.query && b.it.band1 == a.it.band1 && b.S == a.S) {
        push_segments(a.it, &b.it, a.S);
        ++i;
        continue;
      }
    }
    push_segments(a.it, nullptr, a.S);
  }
  for (size_t i = 0; i < singles.size(); ++i) emit(singles[i], singles_pairable[i]);
  p.n_wide = (int32_t)p.longitems.size();
  std::fill(pending.begin(), pending.end(), -1);  // wide and narrow items are not mixed
  for (auto &x : narrow) {
    const PairItem &it = x.second;
    const double single = (double)it.band1 * (double)((it.len + 126) / 64) * 64 * t_step;
    emit(it, pair_all || (pair_narrow && 1.45 * single <= pair_limit()));
  }

  const int64_t nitems16 = p.nitems16 = (int64_t)ninter * nunits;
  p.grid16 = (int)std::min<int64_t>(nitems16, (int64_t)per_cu * db.num_cu);
  {
    // algorithmic cells (query rows x unpadded residues) of each launch
    int64_t sum_all = 0;
    for (int64_t q = 0; q < nq; ++q) sum_all += lens[q];
    auto rows_of = [&](const PairItem &it, int R) {
      const int64_t m = lens[(size_t)it.query];
      return std::min<int64_t>(m, (int64_t)it.band1 * 64 * R) - (int64_t)it.band0 * 64 * R;
    };
    int64_t c32 = 0, c16 = 0, ccrit = 0;
    for (size_t k = 0; k < p.longitems.size(); ++k) {
      const PairItem &it = p.longitems[k];
      if (p.second[k].len >= 0)
        c16 += (int64_t)(it.len + p.second[k].len) * rows_of(it, p.R);
      else
        c32 += (int64_t)it.len * rows_of(it, p.R);
    }
    for (const PairItem &it : p.crititems) ccrit += (int64_t)it.len * rows_of(it, p.crit_R);
    int64_t *st = p.stats;
    st[SW_ST_CELLS_INTER16] = sum_all * db.group_res[(size_t)ninter];
    st[SW_ST_CELLS_INTRA32] = c32;
    st[SW_ST_CELLS_INTRA16] = c16;
    st[SW_ST_CELLS_CRIT] = ccrit;
    st[SW_ST_INTRA_ROWS] = p.R;
    st[SW_ST_MAIN_WAVES] = p.main_waves;
    st[SW_ST_ROUTED_GROUPS] = db.ngroups - ninter;
    st[SW_ST_STRIP_ROWS] = p.T;
    st[SW_ST_QUERY_PAIRS] = q2 ? 1 : 0;
  }
  // Persistent workgroups per compute unit of the main launch: one of eight waves (two
  // per SIMD), or four-wave ones: two beside a critical-pair launch (whose workgroup
  // takes the third slot; a third main workgroup there slowed the critical waves by
  // 10-15%), else three (three waves per SIMD: the 35000-residue query over the
  // long-sequence mix on MI355X, 49.2-50.0 ms against 50.1-50.9 with two and 51.2-51.4
  // with one eight-wave workgroup).  Four waves per SIMD (two eight-wave workgroups)
  // measured slower and erratic: the per-step profile gathers touch one cache line per
  // lane.  Each launch reserves LDS so that no more than that many share a CU.
  const int64_t n_narrow = (int64_t)p.longitems.size() - p.n_wide;
  p.main_per_cu = p.main_waves == kIntraWaves ? 1 : (p.crititems.empty() ? 3 : 2);
  // The critical pairs' launch (a workgroup of kCritWaves waves per CU, one band and one
  // wave per SIMD) is enqueued first and gets its CUs first; the main launch's
  // workgroups that find no room start as the critical workgroups finish.
  p.grid_crit = (int)std::min<int64_t>((int64_t)p.crititems.size(), std::max(1, db.num_cu));
  p.grid_long = (int)std::min<int64_t>((int64_t)p.n_wide + (n_narrow + p.main_waves - 1) / p.main_waves,
                                       (int64_t)db.num_cu * p.main_per_cu);
  // the recompute list is usually empty; a quarter of the CUs is plenty when it is not,
  // and nothing is launched when no kernel can append to it
  const bool may_flag = (nitems16 > 0 && p.grid16 > 0) || p.nduos > 0;
  p.grid_re = (may_flag && nq > 0) ? std::max(1, db.num_cu / 4) : 0;
  p.grid32 = p.grid_long + p.grid_re + p.grid_crit;

  // workspace sizes
  p.qbytes = qoff[nq];
  // Inter-task boundary slots, one per persistent wave, as wide as the widest group the
  // kernel gets (one dword per lane and column, two in the two-query kernel).  When one
  // such slot per wave would pass kSlotBudget, the widest groups -- those holding at most
  // a sixteenth of the inter-task work -- are left to an eighth of the waves, which take
  // them first (they are the longest items) and keep full-width slots; the other waves'
  // slots only need the width of the widest remaining group.  (The 6e6-sequence database:
  // 6.3 GB of slots as one class for one query per lane and 12.6 GB for a 64-query
  // batch, about 1.7 and 3.4 GB as two.)
  int32_t inter_cols = 0;
  for (int32_t g = 0; g < p.ngroups_inter; ++g) inter_cols = std::max(inter_cols, db.groups[g].ncols);
  const size_t words_per_col = 64 * (q2 ? 2 : 1);
  p.bnd16_slot = std::max<size_t>(1, (size_t)inter_cols * words_per_col);  // dwords
  p.bnd16_small = p.bnd16_slot;
  p.big_waves = 0;
  p.wide_items = 0;
  constexpr size_t kSlotBudget = size_t(1) << 30;
  if (p.grid16 >= 64 && (size_t)p.grid16 * p.bnd16_slot * 4 > kSlotBudget) {
    double total = 0;
    for (int32_t g = 0; g < p.ngroups_inter; ++g) total += (double)db.groups[g].ncols;
    int32_t nwide = 0;  // widest groups taken by the big-slot waves
    double wide_work = 0;
    for (int32_t g = p.ngroups_inter - 1; g > 0; --g) {
      if (wide_work + db.groups[g].ncols > total / 16) break;
      wide_work += db.groups[g].ncols;
      ++nwide;
    }
    const int32_t small_cols = p.ngroups_inter - nwide > 0 ? db.groups[p.ngroups_inter - 1 - nwide].ncols : 0;
    if (nwide > 0 && small_cols < inter_cols) {
      p.big_waves = std::max(1, p.grid16 / 8);
      p.wide_items = (int64_t)nwide * nunits;
      p.bnd16_small = std::max<size_t>(1, (size_t)small_cols * words_per_col);
    }
  }
  p.stats[SW_ST_BIG_WAVES] = p.big_waves;
  p.bnd32_stride = ((db.max_len + 128 + 63) / 64) * 64;  // >= kBndLead + max_len + 63
  auto ring = [&](int w) { return (size_t)std::max(w + 1, 2 * w) * p.bnd32_stride; };
  p.bnd32_slot = ring(p.main_waves);
  p.bnd32_slot_re = ring(kIntraWaves);
  p.bnd32_slot_crit = ring(kCritWaves);
  p.bnd32_off_re = (size_t)p.grid_long * p.bnd32_slot;
  p.bnd32_off_crit = p.bnd32_off_re + (size_t)p.grid_re * p.bnd32_slot_re;
  p.bnd32_elems = p.bnd32_off_crit + (size_t)p.grid_crit * p.bnd32_slot_crit;
  // saturated pairs: any database sequence, from either kernel, up to the list's capacity
  // (the pairs beyond it are marked in the scores and found by the overflow pass)
  const int64_t list_cap = k.flag_cap > 0 ? k.flag_cap : kFlagCap;
  p.need_flagged = (size_t)std::max<int64_t>(1, std::min<int64_t>(db.n_seqs * nq, list_cap));
  p.need_bytes = (size_t)p.qbytes + 64 + (nq + 1) * 8 + nq * sizeof(QueryDesc) + A * A * 4 +
                 (size_t)p.qp16_elems * 2 + (size_t)p.qp2_elems * 4 + (size_t)p.qp8_elems +
                 sizeof(Counters) + p.pairs.size() * sizeof(QueryPair) +
                 p.need_flagged * sizeof(PairItem) +
                 (2 * p.longitems.size() + p.crititems.size()) * sizeof(PairItem) +
                 bnd16_words(p) * 4 + p.bnd32_elems * 8 +
                 (size_t)p.xbnd_elems * 8 + (size_t)p.nprog * 12;
  // small per-call inputs, staged in one block (64-byte aligned parts)
  auto up = [](size_t x) { return (x + 63) & ~size_t(63); };
  p.off_qoff = up((size_t)p.qbytes);
  p.off_qd = p.off_qoff + up((size_t)(nq + 1) * 8);
  p.off_mx = p.off_qd + up(nq * sizeof(QueryDesc));
  p.off_qo = p.off_mx + up((size_t)A * A * 4);
  p.off_li = p.off_qo + up(nq * sizeof(int32_t));
  p.off_se = p.off_li + up(p.longitems.size() * sizeof(PairItem));
  p.off_cr = p.off_se + up(p.second.size() * sizeof(PairItem));
  p.off_pr = p.off_cr + up(p.crititems.size() * sizeof(PairItem));
  p.stage_bytes = p.off_pr + p.pairs.size() * sizeof(QueryPair) + 64;
  return p;
}

}  // namespace

Plan make_plan(const DbView &db, const int64_t *qoff, int64_t nq, const Knobs &k,
               const Occupancy &occ) {
  return plan_with(db, qoff, nq, k, occ);
}

}  // namespace swmi
