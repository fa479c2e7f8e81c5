// Host side of the C ABI declared in include/swmi.h: argument checks, database
// pre-processing (Section 4: sort by length, group by lane count, pad), device
// workspaces, and the launch sequence of one search.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/swmi.h"
#include "planner.h"
#include "swmi_internal.h"

#define SW_API extern "C" __attribute__((visibility("default")))

using namespace swmi;

namespace {

std::atomic<int64_t> g_knob_intra_min_len{8192};
std::atomic<int64_t> g_knob_recompute_all{0};
std::atomic<int64_t> g_knob_strip_rows{0};
std::atomic<int64_t> g_knob_grid_waves{0};
std::atomic<int64_t> g_knob_mem_cap_mb{0};
std::atomic<int64_t> g_knob_route_len{0};
std::atomic<int64_t> g_knob_wide_len{0};
std::atomic<int64_t> g_knob_max_segments{0};
std::atomic<int64_t> g_knob_intra_rows{0};
std::atomic<int64_t> g_knob_intra_pairs{1};
std::atomic<int64_t> g_knob_spin_limit{0};
std::atomic<int64_t> g_knob_query_pairs{1};
std::atomic<int64_t> g_knob_main_waves{0};
std::atomic<int64_t> g_knob_prio_cols{0};
std::atomic<int64_t> g_knob_flag_cap{0};
std::atomic<int64_t> g_knob_crit_rows{0};
std::atomic<int64_t> g_knob_crit_share{0};
std::atomic<int64_t> g_knob_intra_prio{1};
std::atomic<int64_t> g_knob_intra_chain{1};

// Group width from which an inter-task item runs at raised wave priority: a wave sweeping
// a group of ncols columns spends about 64 * ncols * waves / residues of the launch's
// time on it (waves sharing the chip evenly), so items past a quarter of the launch start
// first and get their SIMD's issue slots first, which keeps them off the critical path.
int32_t prio_cols_for(int64_t residues, int64_t waves) {
  const int64_t forced = g_knob_prio_cols.load();
  if (forced > 0) return (int32_t)std::min<int64_t>(forced, INT32_MAX);
  const int64_t c = residues / std::max<int64_t>(1, 256 * waves);
  return (int32_t)std::min<int64_t>(std::max<int64_t>(c, 64), INT32_MAX);
}

struct HipFail {
  hipError_t err;
};

inline void hip_check(hipError_t e) {
  if (e != hipSuccess) throw HipFail{e};
}

// A device buffer that only grows.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
};

struct HostBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  void release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
};

// Per-call device state.  A workspace is reused only after `done` has completed, so a
// call never overwrites buffers that earlier work on the device may still read.
struct Workspace {
  hipStream_t own = nullptr;    // stream used by the blocking calls
  hipStream_t aux = nullptr;    // second stream for the long-sequence kernel
  hipStream_t crit = nullptr;   // third stream for the critical pairs (finer bands)
  hipEvent_t done = nullptr, fork = nullptr, join = nullptr, join_crit = nullptr;
  hipEvent_t t0[3] = {}, t1[3] = {};  // kernel timing: inter-task, long intra, recompute
  bool timed[3] = {false, false, false};
  bool busy = false;
  uint64_t last_use = 0;  // order in which workspaces were last handed out
  // `inputs` holds the per-call host data (queries, offsets, query descriptors,
  // matrix, query order, intra-task items) in the layout of `staging`, so one copy
  // moves it to the device
  DevBuf inputs, qp16, qp8, ctr, flagged, bnd16, bnd32, xbnd, xprog, scores;
  HostBuf staging;
  size_t total_bytes() const {
    return inputs.bytes + qp16.bytes + qp8.bytes + ctr.bytes + flagged.bytes + bnd16.bytes +
           bnd32.bytes + xbnd.bytes + xprog.bytes + scores.bytes;
  }
};

}  // namespace

// Timing events created when timing is turned on (two per timed launch).
constexpr size_t kTimingSpares = 256;

struct sw_db {
  int device = 0;
  int num_cu = 0;
  int64_t n_seqs = 0;
  int32_t alphabet = 0;
  int64_t n_short = 0;
  int32_t ngroups = 0;
  int32_t max_ncols = 0;      // widest group (columns incl. padding)
  int32_t max_len = 0;        // longest sequence overall
  int64_t residues = 0;       // unpadded residue total
  DevBuf packed, groups, perm, lens, dlongs;
  std::vector<LongSeq> longs;  // sorted by decreasing length (device copy: dlongs)
  std::vector<GroupDesc> hgroups;   // host copy of the group table
  std::vector<int32_t> hperm;       // host copy: sorted position -> caller index
  std::vector<int32_t> hlens;       // host copy: sorted position -> length
  int64_t short_residues = 0;       // residues in groups
  std::vector<int64_t> group_res;   // residues in groups [0, g), g = 0 .. ngroups
  int64_t last_stats[SW_SEARCH_NSTATS] = {};  // sw_search_stats of the latest search (under mu)
  std::mutex mu;
  std::vector<Workspace *> pool;
  uint64_t pool_uses = 0;
  std::atomic<bool> timing{false};
  std::mutex topk_mu;
  DevBuf topk_scratch;  // TopkState, 256 counters, kTopkMax keys, 2 x kTopkMax results
  struct TimedLaunch {
    int kind;
    hipEvent_t e0, e1;
  };
  std::vector<TimedLaunch> timing_events;
  std::vector<hipEvent_t> spare_events;  // read timing events, reused by later searches
  int64_t timing_launches[3] = {0, 0, 0};
  double timing_ms[3] = {0.0, 0.0, 0.0};
};

int swmi::db_device(const sw_db *db) { return db->device; }

namespace {

int map_hip(hipError_t e) {
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SW_ENOMEM : SW_EDEVICE;
}

// Runs the body of an entry point: no exception crosses the C ABI (a HIP failure maps to
// its code, an allocation failure to SW_ENOMEM, anything else, such as std::system_error
// from a lock or a thread, to SW_EDEVICE).
template <class F> int abi_guard(F &&body) noexcept {
  try {
    return body();
  } catch (const HipFail &f) {
    return map_hip(f.err);
  } catch (const std::bad_alloc &) {
    return SW_ENOMEM;
  } catch (...) {
    return SW_EDEVICE;
  }
}

template <class F> void abi_guard_void(F &&body) noexcept {
  try {
    body();
  } catch (...) {
  }
}

void grow(DevBuf &b, size_t bytes) {
  if (bytes <= b.bytes) return;
  b.release();
  size_t want = std::max<size_t>(bytes, 256);
  hip_check(hipMalloc(&b.ptr, want));
  b.bytes = want;
}

void grow_host(HostBuf &b, size_t bytes) {
  if (bytes <= b.bytes) return;
  b.release();
  size_t want = std::max<size_t>(bytes, 4096);
  hip_check(hipHostMalloc(&b.ptr, want, hipHostMallocDefault));
  b.bytes = want;
}

void destroy_workspace(Workspace *w) {
  if (w->own) (void)hipStreamSynchronize(w->own);
  if (w->aux) (void)hipStreamSynchronize(w->aux);
  if (w->crit) (void)hipStreamSynchronize(w->crit);
  for (DevBuf *b : {&w->inputs, &w->qp16, &w->qp8, &w->ctr, &w->flagged, &w->bnd16, &w->bnd32,
                    &w->xbnd, &w->xprog, &w->scores})
    b->release();
  w->staging.release();
  for (hipEvent_t e : {w->done, w->fork, w->join, w->join_crit, w->t0[0], w->t1[0], w->t0[1], w->t1[1],
                       w->t0[2], w->t1[2]})
    if (e) (void)hipEventDestroy(e);
  if (w->own) (void)hipStreamDestroy(w->own);
  if (w->aux) (void)hipStreamDestroy(w->aux);
  if (w->crit) (void)hipStreamDestroy(w->crit);
  delete w;
}

// A workspace with its streams and events (buffers grow on first use).
Workspace *new_workspace() {
  Workspace *w = new Workspace();
  try {
    hip_check(hipStreamCreateWithFlags(&w->own, hipStreamNonBlocking));
    hip_check(hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking));
    hip_check(hipStreamCreateWithFlags(&w->crit, hipStreamNonBlocking));
    hip_check(hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
    hip_check(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
    hip_check(hipEventCreateWithFlags(&w->join, hipEventDisableTiming));
    hip_check(hipEventCreateWithFlags(&w->join_crit, hipEventDisableTiming));
    for (int k = 0; k < 3; ++k) {
      hip_check(hipEventCreate(&w->t0[k]));
      hip_check(hipEventCreate(&w->t1[k]));
    }
    hip_check(hipEventRecord(w->done, w->own));
  } catch (...) {
    destroy_workspace(w);
    throw;
  }
  return w;
}

Workspace *acquire(sw_db *db) {
  std::lock_guard<std::mutex> lk(db->mu);
  for (Workspace *w : db->pool) {
    if (!w->busy && hipEventQuery(w->done) == hipSuccess) {
      w->busy = true;
      w->last_use = ++db->pool_uses;
      return w;
    }
  }
  // Two workspaces let a host thread enqueue one search while the previous one runs;
  // beyond that a call waits for the older idle workspace to finish, which keeps the
  // device fed (the newer search is still queued) and costs less than sizing a new
  // workspace.  A new one is still created if every workspace is held by a concurrent
  // call.
  if (db->pool.size() >= 2) {
    Workspace *oldest = nullptr;
    for (Workspace *w : db->pool)
      if (!w->busy && (!oldest || w->last_use < oldest->last_use)) oldest = w;
    if (oldest) {
      hip_check(hipEventSynchronize(oldest->done));
      oldest->busy = true;
      oldest->last_use = ++db->pool_uses;
      return oldest;
    }
  }
  Workspace *w = new_workspace();
  w->busy = true;
  w->last_use = ++db->pool_uses;
  db->pool.push_back(w);
  return w;
}

void release(sw_db *db, Workspace *w) {
  std::lock_guard<std::mutex> lk(db->mu);
  w->busy = false;
}

int validate_search(const sw_db *db, const int32_t *matrix, int32_t gap_open,
                    int32_t gap_extend) {
  if (!db) return SW_ENODB;
  if (!matrix) return SW_EINVAL;
  if (gap_open < 0 || gap_extend < 0) return SW_EINVAL;
  if ((int64_t)gap_open + gap_extend > SW_MAX_GOE) return SW_EINVAL;
  const int A = db->alphabet;
  for (int i = 0; i < A * A; ++i)
    if (matrix[i] > SW_MAX_ABS_SCORE || matrix[i] < -SW_MAX_ABS_SCORE) return SW_EINVAL;
  return SW_OK;
}

int validate_query(const sw_db *db, const uint8_t *q, int64_t m) {
  if (m < 0 || m > SW_MAX_QUERY_LEN) return SW_EINVAL;
  if (m > 0 && !q) return SW_EINVAL;
  for (int64_t i = 0; i < m; ++i)
    if (q[i] >= db->alphabet) return SW_EINVAL;
  return SW_OK;
}

// The knob values and kernel occupancies a search plans with.
Knobs knob_snapshot() {
  Knobs k;
  k.strip_rows = g_knob_strip_rows.load();
  k.grid_waves = g_knob_grid_waves.load();
  k.route_len = g_knob_route_len.load();
  k.wide_len = g_knob_wide_len.load();
  k.max_segments = g_knob_max_segments.load();
  k.intra_rows = g_knob_intra_rows.load();
  k.intra_pairs = g_knob_intra_pairs.load();
  k.query_pairs = g_knob_query_pairs.load();
  k.main_waves = g_knob_main_waves.load();
  k.mem_cap_mb = g_knob_mem_cap_mb.load();
  k.flag_cap = g_knob_flag_cap.load();
  k.crit_rows = g_knob_crit_rows.load();
  k.crit_share = g_knob_crit_share.load();
  return k;
}

const Occupancy &occupancy() {
  static const Occupancy occ = [] {
    Occupancy o;
    for (int T = 1; T <= kMaxStripRows; ++T) {
      if (inter16_supported(T)) o.inter16[T] = inter16_max_blocks_per_cu(T);
      if (inter16q2_supported(T)) o.inter16q2[T] = inter16q2_max_blocks_per_cu(T);
    }
    return o;
  }();
  return occ;
}

DbView db_view(const sw_db *db) {
  DbView v;
  v.num_cu = db->num_cu;
  v.alphabet = db->alphabet;
  v.n_seqs = db->n_seqs;
  v.ngroups = db->ngroups;
  v.max_ncols = db->max_ncols;
  v.max_len = db->max_len;
  v.short_residues = db->short_residues;
  v.packed_bytes = (int64_t)db->packed.bytes;
  v.groups = db->hgroups.data();
  v.perm = db->hperm.data();
  v.lens = db->hlens.data();
  v.group_res = db->group_res.data();
  v.longs.p = db->longs.data();
  v.longs.n = db->longs.size();
  return v;
}

// Enqueue one (possibly batched) search on `s`.  Queries are host memory; scores go to
// `scores_dev` (n_queries x n_seqs).  The caller owns `w` until `done` is recorded.
void enqueue_search(sw_db *db, Workspace *w, const uint8_t *queries, const int64_t *qoff,
                    int64_t nq, const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t *scores_dev, hipStream_t s, bool allow_timing = true) {
  // the caller has made db->device current (no device switch while a graph is captured)
  const int A = db->alphabet;
  const Knobs knobs = knob_snapshot();
  const Plan p = make_plan(db_view(db), qoff, nq, knobs, occupancy());
  const bool q2 = p.q2;
  const int64_t nitems16 = p.nitems16;
  const std::vector<int32_t> &qorder = p.qorder;
  const int64_t qbytes = p.qbytes;
  const size_t bnd16_slot = p.bnd16_slot, bnd32_slot = p.bnd32_slot;
  const int bnd32_stride = p.bnd32_stride;
  const size_t need_flagged = p.need_flagged;
  if (knobs.mem_cap_mb > 0 &&
      (int64_t)(std::max(p.need_bytes, w->total_bytes()) >> 20) > knobs.mem_cap_mb)
    throw HipFail{hipErrorOutOfMemory};
  // small per-call inputs, staged through pinned memory (reused only after `done`) and
  // copied to the device in one transfer
  const size_t off_qoff = p.off_qoff, off_qd = p.off_qd, off_mx = p.off_mx, off_qo = p.off_qo,
               off_li = p.off_li, off_se = p.off_se, off_cr = p.off_cr, off_pr = p.off_pr,
               stage_bytes = p.stage_bytes;
  grow(w->inputs, stage_bytes);
  // (the int16 strip profiles of k_inter16, or the pair profiles of the two-query kernel)
  grow(w->qp16, (size_t)std::max<int64_t>({16, p.qp16_elems * 2, p.qp2_elems * 4}));
  grow(w->qp8, (size_t)std::max<int64_t>(16, p.qp8_elems));
  grow(w->ctr, sizeof(Counters));
  grow(w->flagged, need_flagged * sizeof(PairItem));
  grow(w->bnd16, std::max<size_t>(1, bnd16_words(p)) * 4);
  grow(w->bnd32, std::max<size_t>(1, p.bnd32_elems) * 8);
  grow(w->xbnd, (size_t)std::max<int64_t>(1, p.xbnd_elems) * 8);
  // per segment boundary: progress, finished flag (both cleared per search), maximum
  grow(w->xprog, (size_t)std::max<int32_t>(1, p.nprog) * 12);

  grow_host(w->staging, stage_bytes);
  uint8_t *st = (uint8_t *)w->staging.ptr;
  if (qbytes) std::memcpy(st, queries, (size_t)qbytes);
  std::memcpy(st + off_qoff, qoff, (size_t)(nq + 1) * 8);
  if (nq) std::memcpy(st + off_qd, p.qd.data(), nq * sizeof(QueryDesc));
  std::memcpy(st + off_mx, matrix, (size_t)A * A * 4);
  if (nq) std::memcpy(st + off_qo, qorder.data(), nq * sizeof(int32_t));
  if (!p.longitems.empty()) {
    std::memcpy(st + off_li, p.longitems.data(), p.longitems.size() * sizeof(PairItem));
    std::memcpy(st + off_se, p.second.data(), p.second.size() * sizeof(PairItem));
  }
  if (!p.crititems.empty())
    std::memcpy(st + off_cr, p.crititems.data(), p.crititems.size() * sizeof(PairItem));
  if (!p.pairs.empty())
    std::memcpy(st + off_pr, p.pairs.data(), p.pairs.size() * sizeof(QueryPair));
  hip_check(hipMemcpyAsync(w->inputs.ptr, st, stage_bytes, hipMemcpyHostToDevice, s));
  uint8_t *din = (uint8_t *)w->inputs.ptr;
  const uint8_t *d_queries = din;
  const int64_t *d_qoff = (const int64_t *)(din + off_qoff);
  const QueryDesc *d_qdesc = (const QueryDesc *)(din + off_qd);
  const int32_t *d_matrix = (const int32_t *)(din + off_mx);
  const int32_t *d_qorder = (const int32_t *)(din + off_qo);
  const PairItem *d_items = (const PairItem *)(din + off_li);
  const PairItem *d_second = (const PairItem *)(din + off_se);
  const PairItem *d_crit = (const PairItem *)(din + off_cr);
  const QueryPair *d_pairs = (const QueryPair *)(din + off_pr);

  Counters *ctr = (Counters *)w->ctr.ptr;
  ProfileArgs pa;
  pa.query = d_queries;
  pa.qoff = d_qoff;
  pa.queries = d_qdesc;
  pa.nqueries = (int32_t)nq;
  pa.matrix = d_matrix;
  pa.alphabet = A;
  pa.T = p.T;
  pa.qp16 = (int16_t *)w->qp16.ptr;
  pa.qp8 = (int8_t *)w->qp8.ptr;
  pa.ctr = ctr;
  pa.zero = (int32_t *)w->xprog.ptr;
  pa.nzero = 2 * (int64_t)std::max<int32_t>(1, p.nprog);
  pa.scores = scores_dev;
  pa.n_seqs = db->n_seqs;
  if (nq > 0) hip_check(launch_profile(pa, s));
  if (q2 && nitems16 > 0) {
    Profile2Args pb;
    pb.query = d_queries;
    pb.qoff = d_qoff;
    pb.pairs = d_pairs;
    pb.npairs = (int32_t)p.pairs.size();
    pb.matrix = d_matrix;
    pb.alphabet = A;
    pb.T = p.T;
    pb.qp2 = (uint32_t *)w->qp16.ptr;
    hip_check(launch_profile2(pb, s));
  }

  // long sequences: intra-task kernel on the auxiliary stream, concurrent with the sweep
  // (enqueued after the inter-task launch, whose few waves are then dispatched first);
  // with no inter-task launch to run beside, on the search's own stream (a fork and a
  // join between streams cost a latency-bound search about 5% of its time)
  const bool main_aside = p.grid_long > 0 && p.grid16 > 0;
  hipStream_t main_stream = main_aside ? w->aux : s;
  auto launch_main = [&]() {
    if (p.grid_long <= 0) return;
    if (main_aside) hip_check(hipStreamWaitEvent(w->aux, w->fork, 0));
    IntraArgs ia;
    ia.packed = (const uint8_t *)db->packed.ptr;
    ia.items = d_items;
    ia.count_dev = nullptr;
    ia.count = (int32_t)p.longitems.size();
    ia.next = &ctr->intra_next;
    ia.next_narrow = &ctr->intra_narrow;
    ia.n_wide = p.n_wide;
    ia.queries = d_qdesc;
    ia.qp8 = (const int8_t *)w->qp8.ptr;
    ia.goe = gap_open + gap_extend;
    ia.ge = gap_extend;
    ia.scores = scores_dev;
    ia.bnd = (int2 *)w->bnd32.ptr;
    ia.bnd_slot_elems = (int64_t)bnd32_slot;
    ia.bnd_stride = bnd32_stride;
    ia.xbnd = (int2 *)w->xbnd.ptr;
    ia.xprog = (int32_t *)w->xprog.ptr;
    ia.xfin = (int32_t *)w->xprog.ptr + std::max<int32_t>(1, p.nprog);
    ia.xmax = (int32_t *)w->xprog.ptr + 2 * std::max<int32_t>(1, p.nprog);
    ia.error = &ctr->error;
    ia.second = d_second;
    ia.flagged = (PairItem *)w->flagged.ptr;
    ia.flag_count = &ctr->flagged;
    ia.spin_limit = g_knob_spin_limit.load() > 0 ? (int32_t)g_knob_spin_limit.load() : kSpinLimit;
    ia.flag_cap = (int32_t)need_flagged;
    ia.wide_prio = g_knob_intra_prio.load() ? 2 : 0;
    ia.chain = g_knob_intra_chain.load() ? 1 : 0;
    const bool timed = allow_timing && db->timing.load();
    if (timed) hip_check(hipEventRecord(w->t0[1], main_stream));
    hip_check(launch_intra32(ia, p.R, p.main_waves, p.grid_long, main_stream, p.main_per_cu));
    if (timed) {
      hip_check(hipEventRecord(w->t1[1], main_stream));
      w->timed[1] = true;
    }
    if (main_aside) hip_check(hipEventRecord(w->join, w->aux));
  };

  if (main_aside || p.grid_crit > 0) hip_check(hipEventRecord(w->fork, s));
  // critical pairs first (their workgroups are dispatched before the main launch's),
  // on a stream of their own, with finer bands
  if (p.grid_crit > 0) {
    hip_check(hipStreamWaitEvent(w->crit, w->fork, 0));
    IntraArgs ca;
    ca.packed = (const uint8_t *)db->packed.ptr;
    ca.items = d_crit;
    ca.count_dev = nullptr;
    ca.count = (int32_t)p.crititems.size();
    ca.next = &ctr->crit_next;
    ca.next_narrow = &ctr->crit_narrow;
    ca.n_wide = ca.count;
    ca.queries = d_qdesc;
    ca.qp8 = (const int8_t *)w->qp8.ptr;
    ca.goe = gap_open + gap_extend;
    ca.ge = gap_extend;
    ca.scores = scores_dev;
    ca.bnd = (int2 *)w->bnd32.ptr + p.bnd32_off_crit;
    ca.bnd_slot_elems = (int64_t)p.bnd32_slot_crit;
    ca.bnd_stride = bnd32_stride;
    ca.xbnd = (int2 *)w->xbnd.ptr;
    ca.xprog = (int32_t *)w->xprog.ptr;
    ca.xfin = (int32_t *)w->xprog.ptr + std::max<int32_t>(1, p.nprog);
    ca.xmax = (int32_t *)w->xprog.ptr + 2 * std::max<int32_t>(1, p.nprog);
    ca.error = &ctr->error;
    ca.second = nullptr;
    ca.flagged = nullptr;
    ca.flag_count = nullptr;
    ca.spin_limit = g_knob_spin_limit.load() > 0 ? (int32_t)g_knob_spin_limit.load() : kSpinLimit;
    ca.flag_cap = (int32_t)need_flagged;
    ca.wide_prio = g_knob_intra_prio.load() ? 3 : 0;
    ca.chain = g_knob_intra_chain.load() ? 1 : 0;
    hip_check(launch_intra32(ca, p.crit_R, kCritWaves, p.grid_crit, w->crit, 2));
    hip_check(hipEventRecord(w->join_crit, w->crit));
  }
  // An inter-task launch of fewer items than the chip has SIMDs, beside the intra-task
  // launches, has its waves share SIMDs with theirs; at raised priority it finishes first
  // instead of last.  (Long-sequence mix, 5478-residue query, on MI355X: its three items
  // took 4.2-12.4 ms beside a search of about 11 ms, ending last when dispatched late.)
  const bool inter_beside_intra =
      (p.grid_long > 0 || p.grid_crit > 0) && nitems16 < 4LL * std::max(1, db->num_cu);
  if (nq > 0) {
    const bool timed = allow_timing && db->timing.load();
    if (timed && p.grid16 > 0) hip_check(hipEventRecord(w->t0[0], s));
    if (q2) {
      Inter2Args ia;
      ia.packed = (const uint8_t *)db->packed.ptr;
      ia.groups = (const GroupDesc *)db->groups.ptr;
      ia.ngroups = p.ngroups_inter;
      ia.npairs = (int32_t)p.pairs.size();
      ia.pairs = d_pairs;
      ia.queries = d_qdesc;
      ia.qp2 = (const uint32_t *)w->qp16.ptr;
      ia.perm = (const int32_t *)db->perm.ptr;
      ia.lens = (const int32_t *)db->lens.ptr;
      ia.goe = gap_open + gap_extend;
      ia.ge = gap_extend;
      ia.scores = scores_dev;
      ia.flagged = (PairItem *)w->flagged.ptr;
      ia.ctr = ctr;
      ia.bnd = (uint32_t *)w->bnd16.ptr;
      ia.bnd_slot_words = (int64_t)bnd16_slot;
      ia.small_slot_words = (int64_t)p.bnd16_small;
      ia.big_waves = p.big_waves;
      ia.wide_items = (int32_t)p.wide_items;
      ia.recompute_all = g_knob_recompute_all.load() ? 1 : 0;
      ia.nitems = (int32_t)nitems16;
      ia.prio_cols = inter_beside_intra
                         ? 1
                         : prio_cols_for(db->group_res[(size_t)p.ngroups_inter], p.grid16);
      ia.flag_cap = (int32_t)need_flagged;
      hip_check(launch_inter16q2(ia, p.T, p.grid16, s));
    } else {
      InterArgs ia;
      ia.packed = (const uint8_t *)db->packed.ptr;
      ia.groups = (const GroupDesc *)db->groups.ptr;
      ia.ngroups = p.ngroups_inter;
      ia.nqueries = (int32_t)nq;
      ia.queries = d_qdesc;
      ia.qorder = d_qorder;
      ia.qp16 = (const int16_t *)w->qp16.ptr;
      ia.perm = (const int32_t *)db->perm.ptr;
      ia.lens = (const int32_t *)db->lens.ptr;
      ia.goe = gap_open + gap_extend;
      ia.ge = gap_extend;
      ia.scores = scores_dev;
      ia.flagged = (PairItem *)w->flagged.ptr;
      ia.ctr = ctr;
      ia.bnd = (uint32_t *)w->bnd16.ptr;
      ia.bnd_slot_words = (int64_t)bnd16_slot;
      ia.small_slot_words = (int64_t)p.bnd16_small;
      ia.big_waves = p.big_waves;
      ia.wide_items = (int32_t)p.wide_items;
      ia.recompute_all = g_knob_recompute_all.load() ? 1 : 0;
      ia.nitems = (int32_t)nitems16;
      ia.prio_cols = inter_beside_intra
                         ? 1
                         : prio_cols_for(db->group_res[(size_t)p.ngroups_inter], p.grid16);
      ia.flag_cap = (int32_t)need_flagged;
      hip_check(launch_inter16(ia, p.T, p.grid16, s));
    }
    if (timed && p.grid16 > 0) {
      hip_check(hipEventRecord(w->t1[0], s));
      w->timed[0] = true;
    }
  }
  launch_main();
  if (nq > 0) {
    const bool timed = allow_timing && db->timing.load();
    // exact int32 recompute of the saturated alignments of both kernels (count read on
    // the device), after the long-pair kernel; it uses the boundary slots after that
    // kernel's
    if (main_aside) hip_check(hipStreamWaitEvent(s, w->join, 0));
    if (p.grid_crit > 0) hip_check(hipStreamWaitEvent(s, w->join_crit, 0));
    IntraArgs ra;
    ra.packed = (const uint8_t *)db->packed.ptr;
    ra.items = (const PairItem *)w->flagged.ptr;
    ra.count_dev = &ctr->flagged;
    ra.count = 0;
    ra.next = &ctr->recompute_next;
    ra.next_narrow = &ctr->recompute_narrow;
    ra.n_wide = 0;
    ra.queries = d_qdesc;
    ra.qp8 = (const int8_t *)w->qp8.ptr;
    ra.goe = gap_open + gap_extend;
    ra.ge = gap_extend;
    ra.scores = scores_dev;
    ra.bnd = (int2 *)w->bnd32.ptr + p.bnd32_off_re;
    ra.bnd_slot_elems = (int64_t)p.bnd32_slot_re;
    ra.bnd_stride = bnd32_stride;
    ra.xbnd = (int2 *)w->xbnd.ptr;
    ra.xprog = (int32_t *)w->xprog.ptr;
    ra.xfin = (int32_t *)w->xprog.ptr + std::max<int32_t>(1, p.nprog);
    ra.xmax = (int32_t *)w->xprog.ptr + 2 * std::max<int32_t>(1, p.nprog);
    ra.error = &ctr->error;
    ra.second = nullptr;
    ra.flagged = nullptr;
    ra.flag_count = nullptr;
    ra.spin_limit = kSpinLimit;
    ra.flag_cap = (int32_t)need_flagged;
    ra.wide_prio = 0;
    ra.chain = g_knob_intra_chain.load() ? 1 : 0;
    if (timed && p.grid_re > 0) hip_check(hipEventRecord(w->t0[2], s));
    hip_check(launch_intra32(ra, kIntraR, kIntraWaves, p.grid_re, s, 1));
    if (timed && p.grid_re > 0) {
      hip_check(hipEventRecord(w->t1[2], s));
      w->timed[2] = true;
    }
    // pairs that did not fit the recompute list (nothing to do unless it overflowed)
    if (p.grid_re > 0) {
      RescanArgs rs;
      rs.ia = ra;
      rs.groups = (const GroupDesc *)db->groups.ptr;
      rs.ngroups = db->ngroups;
      rs.perm = (const int32_t *)db->perm.ptr;
      rs.lens = (const int32_t *)db->lens.ptr;
      rs.longs = (const LongSeq *)db->dlongs.ptr;
      rs.nlongs = (int32_t)db->longs.size();
      rs.nqueries = (int32_t)nq;
      rs.count = &ctr->flagged;
      rs.next = &ctr->rescan_next;
      hip_check(launch_rescan(rs, p.grid_re * kIntraWaves, s));
    }
  }
  if (main_aside) hip_check(hipStreamWaitEvent(s, w->join, 0));
  if (p.grid_crit > 0) hip_check(hipStreamWaitEvent(s, w->join_crit, 0));
  std::lock_guard<std::mutex> lk(db->mu);
  std::memcpy(db->last_stats, p.stats, sizeof(p.stats));
}

int64_t total_of(const int64_t *offsets, int64_t n) { return offsets[n]; }

}  // namespace

// ------------------------------------------------------------------------ ABI
SW_API const char *sw_strerror(int code) {
  switch (code) {
    case SW_OK: return "success";
    case SW_EINVAL: return "invalid argument";
    case SW_ENOMEM: return "out of device memory (admission refused)";
    case SW_EDEVICE: return "HIP device error or no usable gfx950 device";
    case SW_ENODB: return "no database loaded";
    default: return "unknown error";
  }
}

SW_API int sw_set_knob(int32_t knob, int64_t value) {
  switch (knob) {
    case SW_KNOB_INTRA_MIN_LEN: if (value < 0) return SW_EINVAL; g_knob_intra_min_len = value; return SW_OK;
    case SW_KNOB_RECOMPUTE_ALL: g_knob_recompute_all = value; return SW_OK;
    case SW_KNOB_STRIP_ROWS:
      if (value != 0 && !inter16_supported((int)value) && !inter16q2_supported((int)value))
        return SW_EINVAL;
      g_knob_strip_rows = value; return SW_OK;
    case SW_KNOB_GRID_WAVES: if (value < 0 || value > 64) return SW_EINVAL; g_knob_grid_waves = value; return SW_OK;
    case SW_KNOB_MEM_CAP_MB: if (value < 0) return SW_EINVAL; g_knob_mem_cap_mb = value; return SW_OK;
    case SW_KNOB_ROUTE_LEN: if (value < 0) return SW_EINVAL; g_knob_route_len = value; return SW_OK;
    case SW_KNOB_WIDE_LEN: if (value < 0) return SW_EINVAL; g_knob_wide_len = value; return SW_OK;
    case SW_KNOB_MAX_SEGMENTS: if (value < 0) return SW_EINVAL; g_knob_max_segments = value; return SW_OK;
    case SW_KNOB_INTRA_ROWS:
      if (value != 0 && value != 2 && value != 4 && value != 8 && value != 16) return SW_EINVAL;
      g_knob_intra_rows = value;
      return SW_OK;
    case SW_KNOB_INTRA_PAIRS: if (value < 0 || value > 2) return SW_EINVAL; g_knob_intra_pairs = value; return SW_OK;
    case SW_KNOB_SPIN_LIMIT:
      if (value < 0 || value > kSpinLimit) return SW_EINVAL;
      g_knob_spin_limit = value;
      return SW_OK;
    case SW_KNOB_QUERY_PAIRS: if (value < 0 || value > 1) return SW_EINVAL; g_knob_query_pairs = value; return SW_OK;
    case SW_KNOB_MAIN_WAVES:
      if (value != 0 && value != 4 && value != 8) return SW_EINVAL;
      g_knob_main_waves = value;
      return SW_OK;
    case SW_KNOB_PRIO_COLS: if (value < 0) return SW_EINVAL; g_knob_prio_cols = value; return SW_OK;
    case SW_KNOB_FLAG_CAP:
      if (value < 0 || value > INT32_MAX) return SW_EINVAL;
      g_knob_flag_cap = value;
      return SW_OK;
    case SW_KNOB_CRIT_ROWS:
      if (value != 0 && value != 4 && value != 8) return SW_EINVAL;
      g_knob_crit_rows = value;
      return SW_OK;
    case SW_KNOB_CRIT_SHARE:
      if (value < 0 || value > 100) return SW_EINVAL;
      g_knob_crit_share = value;
      return SW_OK;
    case SW_KNOB_INTRA_PRIO:
      if (value != 0 && value != 1) return SW_EINVAL;
      g_knob_intra_prio = value;
      return SW_OK;
    case SW_KNOB_INTRA_CHAIN:
      if (value != 0 && value != 1) return SW_EINVAL;
      g_knob_intra_chain = value;
      return SW_OK;
    default: return SW_EINVAL;
  }
}

SW_API int64_t sw_get_knob(int32_t knob) {
  switch (knob) {
    case SW_KNOB_INTRA_MIN_LEN: return g_knob_intra_min_len.load();
    case SW_KNOB_RECOMPUTE_ALL: return g_knob_recompute_all.load();
    case SW_KNOB_STRIP_ROWS: return g_knob_strip_rows.load();
    case SW_KNOB_GRID_WAVES: return g_knob_grid_waves.load();
    case SW_KNOB_MEM_CAP_MB: return g_knob_mem_cap_mb.load();
    case SW_KNOB_ROUTE_LEN: return g_knob_route_len.load();
    case SW_KNOB_WIDE_LEN: return g_knob_wide_len.load();
    case SW_KNOB_MAX_SEGMENTS: return g_knob_max_segments.load();
    case SW_KNOB_INTRA_ROWS: return g_knob_intra_rows.load();
    case SW_KNOB_INTRA_PAIRS: return g_knob_intra_pairs.load();
    case SW_KNOB_SPIN_LIMIT: return g_knob_spin_limit.load();
    case SW_KNOB_QUERY_PAIRS: return g_knob_query_pairs.load();
    case SW_KNOB_MAIN_WAVES: return g_knob_main_waves.load();
    case SW_KNOB_PRIO_COLS: return g_knob_prio_cols.load();
    case SW_KNOB_FLAG_CAP: return g_knob_flag_cap.load();
    case SW_KNOB_CRIT_ROWS: return g_knob_crit_rows.load();
    case SW_KNOB_CRIT_SHARE: return g_knob_crit_share.load();
    case SW_KNOB_INTRA_PRIO: return g_knob_intra_prio.load();
    case SW_KNOB_INTRA_CHAIN: return g_knob_intra_chain.load();
    default: return SW_EINVAL;
  }
}

SW_API int sw_db_load(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs,
                      int32_t alphabet, sw_db **out) {
  return abi_guard([&]() -> int {
    if (!out || !offsets || n_seqs < 0) return SW_EINVAL;
    if (alphabet < 1 || alphabet > SW_MAX_ALPHABET) return SW_EINVAL;
    if (n_seqs > INT32_MAX / 2) return SW_EINVAL;
    if (offsets[0] != 0) return SW_EINVAL;
    for (int64_t k = 0; k < n_seqs; ++k) {
      if (offsets[k + 1] < offsets[k]) return SW_EINVAL;
      if (offsets[k + 1] - offsets[k] > (int64_t)INT32_MAX / 2) return SW_EINVAL;
    }
    const int64_t total = total_of(offsets, n_seqs);
    if (total > 0 && !residues) return SW_EINVAL;
    for (int64_t i = 0; i < total; ++i)
      if (residues[i] >= alphabet) return SW_EINVAL;

    sw_db *db = new (std::nothrow) sw_db();
    if (!db) return SW_ENOMEM;
    void *d_raw = nullptr, *d_off = nullptr;
    try {
      int ndev = 0;
      if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw HipFail{hipErrorNoDevice};
      hip_check(hipGetDevice(&db->device));
      hipDeviceProp_t prop;
      hip_check(hipGetDeviceProperties(&prop, db->device));
      if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) throw HipFail{hipErrorNoBinaryForGpu};
      db->num_cu = prop.multiProcessorCount;
      db->n_seqs = n_seqs;
      db->alphabet = alphabet;
      db->residues = total;

      // Section 4: sort by length (ascending, stable), route the longest sequences to the
      // intra-task kernel, group the rest 64 at a time and pad each group to its longest.
      std::vector<int32_t> order((size_t)n_seqs);
      std::iota(order.begin(), order.end(), 0);
      auto len_of = [&](int32_t k) { return offsets[k + 1] - offsets[k]; };
      std::stable_sort(order.begin(), order.end(),
                       [&](int32_t x, int32_t y) { return len_of(x) < len_of(y); });
      const int64_t lmax = g_knob_intra_min_len.load();
      int64_t n_short = 0;
      while (n_short < n_seqs && len_of(order[n_short]) <= lmax) ++n_short;
      db->n_short = n_short;
      db->max_len = n_seqs ? (int32_t)len_of(order[n_seqs - 1]) : 0;

      std::vector<GroupDesc> groups;
      int64_t bytes = 0;
      for (int64_t f = 0; f < n_short; f += kGroup) {
        GroupDesc g;
        g.first = (int32_t)f;
        g.count = (int32_t)std::min<int64_t>(kGroup, n_short - f);
        g.maxlen = (int32_t)len_of(order[f + g.count - 1]);
        g.ncols = ((g.maxlen + 2 + 3) / 4) * 4;
        g.base = bytes;
        bytes += (int64_t)g.ncols * 64;
        db->max_ncols = std::max(db->max_ncols, g.ncols);
        groups.push_back(g);
      }
      db->ngroups = (int32_t)groups.size();
      for (int64_t p = 0; p < n_short; ++p) db->short_residues += len_of(order[p]);
      db->group_res.assign(groups.size() + 1, 0);
      for (size_t g = 0; g < groups.size(); ++g) {
        int64_t r = 0;
        for (int32_t l = 0; l < groups[g].count; ++l) r += len_of(order[groups[g].first + l]);
        db->group_res[g + 1] = db->group_res[g] + r;
      }
      std::vector<int32_t> lens((size_t)std::max<int64_t>(1, n_short));
      for (int64_t p = 0; p < n_short; ++p) lens[p] = (int32_t)len_of(order[p]);
      for (int64_t p = n_seqs - 1; p >= n_short; --p) {  // longest first
        LongSeq L;
        L.base = bytes;
        L.len = (int32_t)len_of(order[p]);
        L.orig = order[p];
        bytes += ((L.len + 4 + 3) / 4) * 4;
        db->longs.push_back(L);
      }

      grow(db->packed, (size_t)std::max<int64_t>(bytes, 4));
      grow(db->groups, std::max<size_t>(1, groups.size()) * sizeof(GroupDesc));
      grow(db->perm, (size_t)std::max<int64_t>(1, n_seqs) * 4);
      grow(db->lens, lens.size() * 4);
      if (!groups.empty())
        hip_check(hipMemcpy(db->groups.ptr, groups.data(), groups.size() * sizeof(GroupDesc),
                            hipMemcpyHostToDevice));
      if (n_seqs)
        hip_check(hipMemcpy(db->perm.ptr, order.data(), (size_t)n_seqs * 4, hipMemcpyHostToDevice));
      grow(db->dlongs, std::max<size_t>(1, db->longs.size()) * sizeof(LongSeq));
      if (!db->longs.empty())
        hip_check(hipMemcpy(db->dlongs.ptr, db->longs.data(), db->longs.size() * sizeof(LongSeq),
                            hipMemcpyHostToDevice));
      hip_check(hipMemcpy(db->lens.ptr, lens.data(), lens.size() * 4, hipMemcpyHostToDevice));

      if (total > 0) {
        hip_check(hipMalloc(&d_raw, (size_t)total));
        hip_check(hipMalloc(&d_off, (size_t)(n_seqs + 1) * 8));
        hip_check(hipMemcpy(d_raw, residues, (size_t)total, hipMemcpyHostToDevice));
        hip_check(hipMemcpy(d_off, offsets, (size_t)(n_seqs + 1) * 8, hipMemcpyHostToDevice));
        PackArgs pa;
        pa.raw = (const uint8_t *)d_raw;
        pa.offsets = (const int64_t *)d_off;
        pa.perm = (const int32_t *)db->perm.ptr;
        pa.groups = (const GroupDesc *)db->groups.ptr;
        pa.ngroups = db->ngroups;
        pa.packed = (uint8_t *)db->packed.ptr;
        hip_check(launch_pack(pa, nullptr));
        for (const auto &L : db->longs) {
          const int64_t padded = ((L.len + 4 + 3) / 4) * 4;
          hip_check(hipMemsetD8((hipDeviceptr_t)((uint8_t *)db->packed.ptr + L.base), kPadCode,
                                (size_t)padded));
          hip_check(hipMemcpy((uint8_t *)db->packed.ptr + L.base,
                              (const uint8_t *)d_raw + offsets[L.orig], (size_t)L.len,
                              hipMemcpyDeviceToDevice));
        }
        hip_check(hipDeviceSynchronize());
        hip_check(hipFree(d_raw));
        d_raw = nullptr;
        hip_check(hipFree(d_off));
        d_off = nullptr;
      }
      db->hgroups = std::move(groups);
      db->hperm = std::move(order);
      db->hlens = std::move(lens);
    } catch (const HipFail &f) {
      if (d_raw) (void)hipFree(d_raw);
      if (d_off) (void)hipFree(d_off);
      db->packed.release(); db->groups.release(); db->perm.release(); db->lens.release();
      db->dlongs.release();
      delete db;
      return f.err == hipErrorNoDevice || f.err == hipErrorNoBinaryForGpu ? SW_EDEVICE
                                                                        : map_hip(f.err);
    } catch (const std::bad_alloc &) {
      if (d_raw) (void)hipFree(d_raw);
      if (d_off) (void)hipFree(d_off);
      db->packed.release(); db->groups.release(); db->perm.release(); db->lens.release();
      db->dlongs.release();
      delete db;
      return SW_ENOMEM;
    }
    *out = db;
    return SW_OK;
  });
}

SW_API int64_t sw_db_size(const sw_db *db) { return db ? db->n_seqs : SW_ENODB; }

SW_API void sw_db_free(sw_db *db) {
  abi_guard_void([&]() {
    if (!db) return;
    (void)hipSetDevice(db->device);
    for (Workspace *w : db->pool) destroy_workspace(w);
    for (auto &e : db->timing_events) {
      (void)hipEventDestroy(e.e0);
      (void)hipEventDestroy(e.e1);
    }
    for (hipEvent_t e : db->spare_events) (void)hipEventDestroy(e);
    db->packed.release(); db->groups.release(); db->perm.release(); db->lens.release();
    db->dlongs.release();
    db->topk_scratch.release();
    delete db;
  });
}

namespace {

// An event for timing: a spare one already read, else a new one (caller holds db->mu).
hipEvent_t timing_event(sw_db *db) {
  if (!db->spare_events.empty()) {
    hipEvent_t e = db->spare_events.back();
    db->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Hand the workspace's recorded timing events to the database (they are read by
// sw_timing_read_kernel and then kept as spares) and give the workspace other ones.
void hand_over_timing(sw_db *db, Workspace *w) {
  std::lock_guard<std::mutex> lk(db->mu);
  for (int k = 0; k < 3; ++k) {
    if (!w->timed[k]) continue;
    w->timed[k] = false;
    hipEvent_t a = timing_event(db);
    if (!a) continue;
    hipEvent_t b = timing_event(db);
    if (!b) {
      db->spare_events.push_back(a);
      continue;
    }
    db->timing_events.push_back({k, w->t0[k], w->t1[k]});
    w->t0[k] = a;
    w->t1[k] = b;
  }
}

int run_search(const sw_db *cdb, const uint8_t *queries, const int64_t *qoff, int64_t nq,
               const int32_t *matrix, int32_t gap_open, int32_t gap_extend, int32_t *host_out,
               int32_t *dev_out, hipStream_t stream) {
  sw_db *db = const_cast<sw_db *>(cdb);
  Workspace *w = nullptr;
  try {
    hip_check(hipSetDevice(db->device));
    w = acquire(db);
    const size_t nscores = (size_t)nq * db->n_seqs;
    hipStream_t s = dev_out ? stream : w->own;
    int32_t *scores = dev_out;
    if (!scores) {
      grow(w->scores, std::max<size_t>(1, nscores) * 4);
      scores = (int32_t *)w->scores.ptr;
    }
    if (nscores > 0) {
      enqueue_search(db, w, queries, qoff, nq, matrix, gap_open, gap_extend, scores, s);
    }
    if (host_out) {
      // the error flag first, so that a failed search leaves scores_out untouched
      int32_t err = 0;
      if (nscores > 0 && w->ctr.ptr) {
        hip_check(hipMemcpyAsync(&err, &((Counters *)w->ctr.ptr)->error, 4,
                                 hipMemcpyDeviceToHost, s));
        hip_check(hipStreamSynchronize(s));
      }
      if (err) throw HipFail{hipErrorLaunchTimeOut};
      if (nscores > 0)
        hip_check(hipMemcpyAsync(host_out, scores, nscores * 4, hipMemcpyDeviceToHost, s));
      hip_check(hipEventRecord(w->done, s));
      hip_check(hipStreamSynchronize(s));
    } else {
      hip_check(hipEventRecord(w->done, s));
    }
    hand_over_timing(db, w);
    release(db, w);
    return SW_OK;
  } catch (const HipFail &f) {
    if (w) {
      (void)hipDeviceSynchronize();
      release(db, w);
    }
    return map_hip(f.err);
  } catch (const std::bad_alloc &) {
    if (w) release(db, w);
    return SW_ENOMEM;
  }
}

}  // namespace

SW_API int sw_search(const sw_db *db, const uint8_t *query, int32_t query_len,
                     const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                     int32_t *scores_out) {
  return abi_guard([&]() -> int {
    int rc = validate_search(db, matrix, gap_open, gap_extend);
    if (rc) return rc;
    if (!scores_out && db->n_seqs > 0) return SW_EINVAL;
    if ((rc = validate_query(db, query, query_len))) return rc;
    const int64_t qoff[2] = {0, query_len};
    return run_search(db, query, qoff, 1, matrix, gap_open, gap_extend, scores_out, nullptr, nullptr);
  });
}

SW_API int sw_search_async(const sw_db *db, const uint8_t *query, int32_t query_len,
                           const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                           int32_t *scores_dev, void *hip_stream) {
  return abi_guard([&]() -> int {
    int rc = validate_search(db, matrix, gap_open, gap_extend);
    if (rc) return rc;
    if (!scores_dev && db->n_seqs > 0) return SW_EINVAL;
    if ((rc = validate_query(db, query, query_len))) return rc;
    if (db->n_seqs == 0) return SW_OK;
    const int64_t qoff[2] = {0, query_len};
    return run_search(db, query, qoff, 1, matrix, gap_open, gap_extend, nullptr, scores_dev,
                      (hipStream_t)hip_stream);
  });
}

SW_API int sw_search_batch(const sw_db *db, const uint8_t *queries, const int64_t *query_offsets,
                           int64_t n_queries, const int32_t *matrix, int32_t gap_open,
                           int32_t gap_extend, int32_t *scores_out) {
  return abi_guard([&]() -> int {
    int rc = validate_search(db, matrix, gap_open, gap_extend);
    if (rc) return rc;
    if (n_queries < 0 || !query_offsets || query_offsets[0] != 0) return SW_EINVAL;
    if (n_queries > 0 && db->n_seqs > 0 && !scores_out) return SW_EINVAL;
    if ((double)n_queries * (double)db->n_seqs > 2.0e9) return SW_EINVAL;
    for (int64_t q = 0; q < n_queries; ++q) {
      if (query_offsets[q + 1] < query_offsets[q]) return SW_EINVAL;
      const int64_t m = query_offsets[q + 1] - query_offsets[q];
      if ((rc = validate_query(db, queries ? queries + query_offsets[q] : nullptr, m))) return rc;
    }
    return run_search(db, queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                      scores_out, nullptr, nullptr);
  });
}

SW_API int sw_timing_enable(sw_db *db, int32_t enable) {
  return abi_guard([&]() -> int {
    if (!db) return SW_ENODB;
    std::lock_guard<std::mutex> lk(db->mu);
    db->timing = enable != 0;
    for (int k = 0; k < 3; ++k) {
      db->timing_launches[k] = 0;
      db->timing_ms[k] = 0.0;
    }
    // events for the searches to come, created here rather than inside a timed region
    // (a first hipEventCreate took about 0.1 ms; a search of the plain workload 0.3)
    if (db->timing) {
      hip_check(hipSetDevice(db->device));
      while (db->spare_events.size() < kTimingSpares) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        db->spare_events.push_back(e);
      }
    }
    for (auto &e : db->timing_events) {  // recorded, possibly unfinished: not reused
      (void)hipEventDestroy(e.e0);
      (void)hipEventDestroy(e.e1);
    }
    db->timing_events.clear();
    return SW_OK;
  });
}

SW_API int sw_timing_read_kernel(const sw_db *cdb, int32_t kernel, int64_t *launches,
                                 double *total_ms) {
  return abi_guard([&]() -> int {
    if (!cdb) return SW_ENODB;
    if (!launches || !total_ms || kernel < 0 || kernel > 2) return SW_EINVAL;
    sw_db *db = const_cast<sw_db *>(cdb);
    std::lock_guard<std::mutex> lk(db->mu);
    for (auto &e : db->timing_events) {
      float ms = 0.f;
      if (hipEventSynchronize(e.e1) != hipSuccess) return SW_EDEVICE;
      if (hipEventElapsedTime(&ms, e.e0, e.e1) != hipSuccess) return SW_EDEVICE;
      db->timing_launches[e.kind] += 1;
      db->timing_ms[e.kind] += ms;
      db->spare_events.push_back(e.e0);
      db->spare_events.push_back(e.e1);
    }
    db->timing_events.clear();
    *launches = db->timing_launches[kernel];
    *total_ms = db->timing_ms[kernel];
    return SW_OK;
  });
}

SW_API int sw_search_stats(const sw_db *cdb, int64_t *values, int32_t n) {
  return abi_guard([&]() -> int {
    if (!cdb) return SW_ENODB;
    if (!values || n < 0) return SW_EINVAL;
    sw_db *db = const_cast<sw_db *>(cdb);
    std::lock_guard<std::mutex> lk(db->mu);
    for (int32_t k = 0; k < n && k < SW_SEARCH_NSTATS; ++k) values[k] = db->last_stats[k];
    return SW_OK;
  });
}

SW_API int sw_timing_read(const sw_db *db, int64_t *launches, double *total_ms) {
  return abi_guard([&]() -> int {
    return sw_timing_read_kernel(db, SW_KERNEL_INTER16, launches, total_ms);
  });
}

// ------------------------------------------------------------------------ plans
// A plan owns a dedicated workspace and an instantiated hipGraph of one (batched)
// search, so replays cost one graph launch.  The graph is captured after an eager run
// has sized every buffer (no allocation happens while capturing), and it contains no
// memset nodes: the counters are cleared by the profile kernel.
struct sw_plan {
  sw_db *db = nullptr;
  Workspace *w = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

SW_API int sw_plan_create(const sw_db *cdb, const uint8_t *queries, const int64_t *query_offsets,
                          int64_t n_queries, const int32_t *matrix, int32_t gap_open,
                          int32_t gap_extend, int32_t *scores_dev, sw_plan **out) {
  return abi_guard([&]() -> int {
    int rc = validate_search(cdb, matrix, gap_open, gap_extend);
    if (rc) return rc;
    if (!out || !query_offsets || n_queries < 1 || query_offsets[0] != 0) return SW_EINVAL;
    if (!scores_dev && cdb->n_seqs > 0) return SW_EINVAL;
    if ((double)n_queries * (double)cdb->n_seqs > 2.0e9) return SW_EINVAL;
    for (int64_t q = 0; q < n_queries; ++q) {
      if (query_offsets[q + 1] < query_offsets[q]) return SW_EINVAL;
      const int64_t m = query_offsets[q + 1] - query_offsets[q];
      if ((rc = validate_query(cdb, queries ? queries + query_offsets[q] : nullptr, m))) return rc;
    }
    sw_db *db = const_cast<sw_db *>(cdb);
    sw_plan *plan = new (std::nothrow) sw_plan();
    if (!plan) return SW_ENOMEM;
    plan->db = db;
    hipStream_t cap = nullptr;
    try {
      hip_check(hipSetDevice(db->device));
      plan->w = new_workspace();
      Workspace *w = plan->w;
      if (db->n_seqs > 0) {
        // eager run: allocates and fills every buffer
        enqueue_search(db, w, queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                       scores_dev, w->own, false);
        hip_check(hipStreamSynchronize(w->own));
        hip_check(hipStreamSynchronize(w->aux));
        hip_check(hipStreamSynchronize(w->crit));
        // capture the same launch sequence
        hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
          enqueue_search(db, w, queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                         scores_dev, cap, false);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cap, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        hip_check(hipStreamEndCapture(cap, &plan->graph));
        hip_check(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
        hip_check(hipStreamDestroy(cap));
        cap = nullptr;
      }
    } catch (const HipFail &f) {
      if (cap) (void)hipStreamDestroy(cap);
      if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
      if (plan->graph) (void)hipGraphDestroy(plan->graph);
      if (plan->w) destroy_workspace(plan->w);
      delete plan;
      return map_hip(f.err);
    } catch (const std::bad_alloc &) {
      if (cap) (void)hipStreamDestroy(cap);
      if (plan->w) destroy_workspace(plan->w);
      delete plan;
      return SW_ENOMEM;
    }
    *out = plan;
    return SW_OK;
  });
}

SW_API int sw_plan_launch(sw_plan *plan, void *hip_stream) {
  return abi_guard([&]() -> int {
    if (!plan) return SW_EINVAL;
    if (!plan->exec) return SW_OK;  // empty database: nothing to do
    if (hipSetDevice(plan->db->device) != hipSuccess) return SW_EDEVICE;
    const hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? SW_OK : map_hip(e);
  });
}

SW_API void sw_plan_free(sw_plan *plan) {
  abi_guard_void([&]() {
    if (!plan) return;
    (void)hipSetDevice(plan->db->device);
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->w) destroy_workspace(plan->w);
    delete plan;
  });
}

// ------------------------------------------------------------------------ serving
// Continuous batching over a resident database.  Two modes, chosen at creation:
//
// Session mode (a database that fills the device several times over, with no sequence
// long enough for the intra-task kernel): one persistent launch of k_serve serves every
// query admitted while it runs.  The worker thread turns queued requests into records
// (one query, or two of similar length sharing the lanes), writes them into host memory
// and raises the doorbell; the running kernel's work list grows by the record's groups,
// so a query that arrives while others are on the device joins the same launch right
// behind them.  The kernel reports each completed record through host memory; scores are
// already in host memory and are copied into the caller's buffer.  The session is closed
// once the server is idle, or before a query that must take the standard path (one longer
// than the session's query cache, or one with a score at the int16 ceiling, which is
// searched again exactly).
//
// Batch mode (small databases, or long sequences): every queued request the budget
// admits is launched as one batched search on a free stream slot; batches in flight on
// different slots overlap on the device.
namespace {

struct ServerRequest {
  uint64_t ticket = 0;
  std::vector<uint8_t> query;
  int32_t *scores_out = nullptr;  // caller's host buffer (n_seqs)
  int status = 1;                 // 1 = pending, 0 = done, < 0 = error
  bool exact = false;             // must run (again) through the standard search path
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct ServerSlot {
  Workspace *w = nullptr;
  hipEvent_t finished = nullptr;
  bool busy = false;
  size_t mem = 0;                       // admitted bytes of the batch in flight
  int64_t items = 0;                    // inter-task work items of the batch
  std::vector<ServerRequest *> batch;
  DevBuf scores;
  HostBuf host_scores;
  HostBuf host_error;                   // Counters::error of the batch, copied after it
};

// A record of the running session: its number, slot, queries and score rows.
struct SessionRecord {
  int32_t r = 0;
  int32_t slot = 0;
  ServerRequest *qa = nullptr, *qb = nullptr;
  int32_t row_a = -1, row_b = -1;
  int32_t bits = 0;       // saturation bits, once complete
  bool copying = false;   // complete on the device, rows being copied to the host
  hipEvent_t copied = nullptr;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Host memory the device reads and writes while a session runs (coherent, mapped).
struct CoherentBuf {
  void *ptr = nullptr;  // host address
  void *dev = nullptr;  // the same memory as the device addresses it
  size_t bytes = 0;
  void alloc(size_t n) {
    hip_check(hipHostMalloc(&ptr, std::max<size_t>(n, 64), hipHostMallocMapped | hipHostMallocCoherent));
    bytes = n;
    std::memset(ptr, 0, bytes);
    hip_check(hipHostGetDevicePointer(&dev, ptr, 0));
  }
  void release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = dev = nullptr;
    bytes = 0;
  }
};

template <class T> T *dev_of(const CoherentBuf &b, const T *host) {
  return (T *)((uint8_t *)b.dev + ((const uint8_t *)host - (const uint8_t *)b.ptr));
}

constexpr int kServeMaxQuery = 16384;  // longest query a session takes
// bytes per query in a record slot: the strips of the longest query, padded to 64
constexpr int kServeQcap = ((kServeMaxQuery + 2 * kServeT1 + 63) / 64) * 64 + 64;
constexpr double kServeLinger = 0.002;  // idle seconds before a session is closed
constexpr double kServePairSpeed = 1.10;  // two-query strips vs one-query strips, per row
constexpr int64_t kServeTimeoutS = 30;   // a session wave waits at most this long for work
constexpr size_t kServePairQueue = 4;    // queued requests from which records take pairs

}  // namespace

struct sw_server {
  sw_db *db = nullptr;
  std::vector<int32_t> matrix;
  int32_t gap_open = 0, gap_extend = 0;
  int32_t max_batch = 1;
  int64_t mem_budget = 0;
  std::mutex mu;
  std::condition_variable cv;       // wakes the worker
  std::condition_variable done_cv;  // wakes waiters
  std::deque<ServerRequest *> queue;
  std::unordered_map<uint64_t, ServerRequest *> requests;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  int64_t launches = 0, max_in_flight = 0, refused = 0;
  int64_t records = 0, paired = 0, exact_runs = 0;
  double copy_s = 0;  // host time spent copying session scores to the callers

  // batch mode
  int64_t fill_items = 0;  // inter-task work items that keep every wave slot busy
  std::vector<ServerSlot> slots;

  // session mode
  bool session_mode = false;
  int32_t max_records = 2;  // records in flight at once
  int32_t nrec = 0, nrows = 0, grid = 0;
  hipStream_t sstream = nullptr;
  hipEvent_t sended = nullptr;
  bool open = false;        // a session launch is running
  bool closing = false;     // its doorbell carries the closed bit
  int32_t published = 0;    // records published in the running launch
  double idle_since = 0;
  int64_t timeout_ticks = 0;
  CoherentBuf hrec, hq, hbell;  // records, query staging, doorbell + flags
  DevBuf dmatrix, dctr, qcache, bnd, dscores;
  HostBuf hscores;               // pinned rows the scores are copied into
  hipStream_t cstream = nullptr; // copies of complete records' rows
  std::vector<hipEvent_t> free_events;
  std::vector<int32_t> free_rows;
  std::deque<SessionRecord> inflight;
  std::vector<ServerRequest *> exact_queue;  // requests waiting for the standard path
};

namespace {

// Device bytes one batch of queries needs beyond the slot's boundary scratch: profiles
// (two int16 layouts, <= 128 bytes per query row plus padding), scores, recompute list.
size_t batch_bytes(const sw_db *db, const std::vector<ServerRequest *> &batch) {
  size_t b = 0;
  for (const ServerRequest *r : batch)
    b += (r->query.size() + 64 * kIntraR) * 2 * kCodes * 2 + (size_t)db->n_seqs * 4 +
         (size_t)db->n_short * sizeof(PairItem);
  return b;
}

// Free device memory, or SIZE_MAX if it cannot be read.
size_t device_free_bytes() {
  size_t fr = 0, tot = 0;
  return hipMemGetInfo(&fr, &tot) == hipSuccess ? fr : SIZE_MAX;
}

void finish_request(sw_server *sv, ServerRequest *r, int status) {
  r->status = status;
  r->t_done = now_s();
  sv->done_cv.notify_all();
}

// ---- batch mode

void server_finish_slot(sw_server *sv, ServerSlot &sl) {
  // called with sv->mu held, after sl.finished has completed
  const size_t n = (size_t)sv->db->n_seqs;
  // a bounded wait between the segments of a split pair that gave up leaves some scores
  // unwritten: the whole batch fails
  const int32_t err = *(const int32_t *)sl.host_error.ptr;
  for (size_t k = 0; k < sl.batch.size(); ++k) {
    ServerRequest *r = sl.batch[k];
    if (!err && n && r->scores_out)
      std::memcpy(r->scores_out, (const int32_t *)sl.host_scores.ptr + k * n, n * 4);
    finish_request(sv, r, err ? SW_EDEVICE : SW_OK);
  }
  sl.batch.clear();
  sl.busy = false;
  sl.mem = 0;
}

// One pass of the batch-mode worker; returns false when the worker should wait.
bool batch_step(sw_server *sv, int in_flight, size_t mem_in_flight, int64_t items_in_flight) {
  // Admit queued requests into a free slot, but only while the batches in flight leave
  // wave slots idle, and stop growing a batch once it alone fills them: a second batch
  // running beside a device-filling one only halves the speed of both.
  ServerSlot *free_slot = nullptr;
  for (ServerSlot &sl : sv->slots)
    if (!sl.busy) { free_slot = &sl; break; }
  const int64_t per_query = std::max<int64_t>(1, sv->db->ngroups);
  if (!free_slot || sv->queue.empty() || items_in_flight >= sv->fill_items) return false;
  const size_t dev_free = device_free_bytes();
  std::vector<ServerRequest *> batch;
  while (!sv->queue.empty() && (int)batch.size() < sv->max_batch &&
         (int64_t)batch.size() * per_query < sv->fill_items) {
    batch.push_back(sv->queue.front());
    const size_t need = batch_bytes(sv->db, batch);
    if ((sv->mem_budget > 0 && (int64_t)(mem_in_flight + need) > sv->mem_budget) ||
        need > dev_free) {
      batch.pop_back();
      break;
    }
    sv->queue.pop_front();
  }
  if (batch.empty()) {
    if (in_flight > 0) return false;  // wait for memory to free up
    // a single request larger than the budget (or the free memory) can never be admitted
    ServerRequest *r = sv->queue.front();
    sv->queue.pop_front();
    ++sv->refused;
    finish_request(sv, r, SW_ENOMEM);
    return true;
  }
  ServerSlot &sl = *free_slot;
  std::vector<uint8_t> cat;
  std::vector<int64_t> offs(1, 0);
  for (ServerRequest *r : batch) {
    cat.insert(cat.end(), r->query.begin(), r->query.end());
    offs.push_back((int64_t)cat.size());
  }
  if (cat.empty()) cat.push_back(0);
  const size_t n = (size_t)sv->db->n_seqs * batch.size();
  int rc = SW_OK;
  try {
    grow(sl.scores, std::max<size_t>(1, n) * 4);
    grow_host(sl.host_scores, std::max<size_t>(1, n) * 4);
    grow_host(sl.host_error, 4);
    *(int32_t *)sl.host_error.ptr = 0;
    const double t = now_s();
    for (ServerRequest *r : batch) r->t_start = t;
    if (n > 0) {
      enqueue_search(sv->db, sl.w, cat.data(), offs.data(), (int64_t)batch.size(),
                     sv->matrix.data(), sv->gap_open, sv->gap_extend, (int32_t *)sl.scores.ptr,
                     sl.w->own, false);
      hip_check(hipMemcpyAsync(sl.host_scores.ptr, sl.scores.ptr, n * 4, hipMemcpyDeviceToHost,
                               sl.w->own));
      hip_check(hipMemcpyAsync(sl.host_error.ptr, &((Counters *)sl.w->ctr.ptr)->error, 4,
                               hipMemcpyDeviceToHost, sl.w->own));
    }
    hip_check(hipEventRecord(sl.finished, sl.w->own));
  } catch (const HipFail &f) {
    rc = map_hip(f.err);
  } catch (const std::bad_alloc &) {
    rc = SW_ENOMEM;
  }
  if (rc != SW_OK) {
    (void)hipStreamSynchronize(sl.w->own);
    for (ServerRequest *r : batch) finish_request(sv, r, rc);
  } else {
    sl.batch = std::move(batch);
    sl.busy = true;
    sl.mem = batch_bytes(sv->db, sl.batch);
    sl.items = (int64_t)sl.batch.size() * per_query;
    ++sv->launches;
    sv->max_in_flight = std::max<int64_t>(sv->max_in_flight, in_flight + 1);
  }
  return true;
}

// ---- session mode

constexpr int kServePollers = 8;  // session workgroups that read the doorbell

int32_t *bell(sw_server *sv) { return (int32_t *)sv->hbell.ptr; }
int32_t *progress(sw_server *sv) { return (int32_t *)sv->hbell.ptr + 16; }  // kServePollers
int32_t *complete_flags(sw_server *sv) { return (int32_t *)sv->hbell.ptr + 64; }
int32_t *sat_flags(sw_server *sv) { return (int32_t *)sv->hbell.ptr + 64 + sv->nrec; }

// Items claimed so far in the running launch, as last reported by the polling waves.
int64_t claimed_items(sw_server *sv) {
  int64_t c = 0;
  for (int k = 0; k < kServePollers; ++k)
    c = std::max<int64_t>(c, __atomic_load_n(progress(sv) + k, __ATOMIC_RELAXED));
  return c;
}

size_t session_device_bytes(const sw_db *db, int grid, int nrec, int nrows) {
  return (size_t)grid * db->max_ncols * 128 * 4 + (size_t)grid * 2 * kServeQcap +
         (size_t)(64 + 2 * nrec) * 4 + (size_t)kCodes * kCodes * 4 +
         (size_t)nrows * db->n_seqs * 4;
}

// Allocate the session's buffers (device scratch, coherent host memory for records,
// queries, scores and flags).  Throws HipFail.
void session_setup(sw_server *sv) {
  sw_db *db = sv->db;
  sv->nrec = std::max(4, 2 * sv->max_records);
  sv->hrec.alloc((size_t)sv->nrec * sizeof(ServeRecord));
  sv->hq.alloc((size_t)sv->nrec * 2 * kServeQcap);
  grow_host(sv->hscores, (size_t)sv->nrows * db->n_seqs * 4);
  grow(sv->dscores, (size_t)sv->nrows * db->n_seqs * 4);
  sv->hbell.alloc((size_t)(64 + 2 * sv->nrec) * 4);
  grow(sv->dmatrix, (size_t)db->alphabet * db->alphabet * 4);
  hip_check(hipMemcpy(sv->dmatrix.ptr, sv->matrix.data(), sv->matrix.size() * 4,
                      hipMemcpyHostToDevice));
  grow(sv->dctr, (size_t)(64 + 2 * sv->nrec) * 4);
  grow(sv->qcache, (size_t)sv->grid * 2 * kServeQcap);
  grow(sv->bnd, (size_t)sv->grid * db->max_ncols * 128 * 4);
  hip_check(hipStreamCreateWithFlags(&sv->sstream, hipStreamNonBlocking));
  hip_check(hipStreamCreateWithFlags(&sv->cstream, hipStreamNonBlocking));
  hip_check(hipEventCreateWithFlags(&sv->sended, hipEventDisableTiming));
  for (int32_t k = 0; k < sv->nrec; ++k) {
    hipEvent_t e = nullptr;
    hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    sv->free_events.push_back(e);
  }
  int khz = 0;
  hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, db->device));
  sv->timeout_ticks = (int64_t)std::max(khz, 1) * 1000 * kServeTimeoutS;
  for (int32_t k = sv->nrows - 1; k >= 0; --k) sv->free_rows.push_back(k);
}

void session_release(sw_server *sv) {
  if (sv->sstream) (void)hipStreamSynchronize(sv->sstream);
  if (sv->cstream) (void)hipStreamSynchronize(sv->cstream);
  if (sv->sended) (void)hipEventDestroy(sv->sended);
  for (SessionRecord &sr : sv->inflight)
    if (sr.copied) sv->free_events.push_back(sr.copied);
  for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
  sv->free_events.clear();
  if (sv->sstream) (void)hipStreamDestroy(sv->sstream);
  if (sv->cstream) (void)hipStreamDestroy(sv->cstream);
  sv->sended = nullptr;
  sv->sstream = sv->cstream = nullptr;
  for (DevBuf *b : {&sv->dmatrix, &sv->dctr, &sv->qcache, &sv->bnd, &sv->dscores}) b->release();
  for (CoherentBuf *b : {&sv->hrec, &sv->hq, &sv->hbell}) b->release();
  sv->hscores.release();
}

// Start a session launch (the previous one has ended).  Throws HipFail.
void session_open(sw_server *sv) {
  sw_db *db = sv->db;
  std::memset(complete_flags(sv), 0, (size_t)sv->nrec * 4);
  std::memset(sat_flags(sv), 0, (size_t)sv->nrec * 4);
  std::memset(progress(sv), 0, (size_t)kServePollers * 4);
  __atomic_store_n(bell(sv), 0, __ATOMIC_RELEASE);
  hip_check(hipMemsetAsync(sv->dctr.ptr, 0, sv->dctr.bytes, sv->sstream));
  int32_t *c = (int32_t *)sv->dctr.ptr;
  ServeArgs a;
  a.packed = (const uint8_t *)db->packed.ptr;
  a.groups = (const GroupDesc *)db->groups.ptr;
  a.ngroups = db->ngroups;
  a.perm = (const int32_t *)db->perm.ptr;
  a.goe = sv->gap_open + sv->gap_extend;
  a.ge = sv->gap_extend;
  a.matrix = (const int32_t *)sv->dmatrix.ptr;
  a.alphabet = db->alphabet;
  a.nrec = sv->nrec;
  a.qcap = kServeQcap;
  a.records = (const ServeRecord *)sv->hrec.dev;
  a.qstage = (const uint8_t *)sv->hq.dev;
  a.scores = (int32_t *)sv->dscores.ptr;
  a.doorbell = dev_of(sv->hbell, bell(sv));
  a.complete = dev_of(sv->hbell, complete_flags(sv));
  a.hsat = dev_of(sv->hbell, sat_flags(sv));
  a.hprog = dev_of(sv->hbell, progress(sv));
  a.mirror = c + 0;
  a.claim = c + 1;
  a.error = c + 2;
  a.done = c + 64;
  a.satf = c + 64 + sv->nrec;
  a.qcache = (uint8_t *)sv->qcache.ptr;
  a.bnd = (uint32_t *)sv->bnd.ptr;
  a.bnd_slot_words = (int64_t)db->max_ncols * 128;
  a.npoll = std::min(sv->grid, kServePollers);
  a.prio_cols = prio_cols_for(db->short_residues, sv->grid);
  a.timeout_ticks = sv->timeout_ticks;
  hip_check(launch_serve(a, sv->grid, sv->sstream));
  hip_check(hipEventRecord(sv->sended, sv->sstream));
  sv->open = true;
  sv->closing = false;
  sv->published = 0;
  ++sv->launches;
}

void session_close(sw_server *sv) {
  if (!sv->open || sv->closing) return;
  __atomic_store_n(bell(sv), 2 * sv->published + 1, __ATOMIC_RELEASE);
  sv->closing = true;
}

// Rows a record of queries (ma, mb) costs in the pair kernel vs as two one-query records.
bool worth_pairing(int64_t ma, int64_t mb) {
  auto single = [](int64_t m) { return (double)((m + 2 * kServeT1 - 1) / (2 * kServeT1)) * 2 * kServeT1; };
  const int64_t mx = std::max(ma, mb);
  const double paired = 2.0 * (double)((mx + kServeT2 - 1) / kServeT2) * kServeT2 / kServePairSpeed;
  return paired < single(ma) + single(mb);
}

// Write a record for `qa` (and `qb`) into its slot and raise the doorbell.  Opens a
// session if none is running.  Throws HipFail.
void session_publish(sw_server *sv, ServerRequest *qa, ServerRequest *qb) {
  if (!sv->open) session_open(sv);
  const int32_t r = sv->published;
  const int32_t slot = r % sv->nrec;
  SessionRecord sr;
  sr.r = r;
  sr.slot = slot;
  sr.qa = qa;
  sr.qb = qb;
  sr.row_a = sv->free_rows.back();
  sv->free_rows.pop_back();
  if (qb) {
    sr.row_b = sv->free_rows.back();
    sv->free_rows.pop_back();
  }
  const int64_t ma = (int64_t)qa->query.size(), mb = qb ? (int64_t)qb->query.size() : 0;
  uint8_t *stage = (uint8_t *)sv->hq.ptr + (size_t)slot * 2 * kServeQcap;
  std::memset(stage, kPadCode, (size_t)2 * kServeQcap);
  std::memcpy(stage, qa->query.data(), (size_t)ma);
  if (qb) std::memcpy(stage + kServeQcap, qb->query.data(), (size_t)mb);
  ServeRecord rec;
  rec.out_a = (int64_t)sr.row_a * sv->db->n_seqs;
  rec.out_b = qb ? (int64_t)sr.row_b * sv->db->n_seqs : -1;
  rec.ma = (int32_t)ma;
  rec.mb = (int32_t)mb;
  rec.kind = qb ? 2 : 1;
  rec.nstrips = qb ? (int32_t)((std::max(ma, mb) + kServeT2 - 1) / kServeT2)
                   : (int32_t)((ma + 2 * kServeT1 - 1) / (2 * kServeT1));
  ((ServeRecord *)sv->hrec.ptr)[slot] = rec;
  const double t = now_s();
  qa->t_start = t;
  if (qb) qb->t_start = t;
  sv->published = r + 1;
  __atomic_store_n(bell(sv), 2 * sv->published, __ATOMIC_RELEASE);
  sv->inflight.push_back(sr);
  ++sv->records;
  if (qb) ++sv->paired;
  sv->max_in_flight = std::max<int64_t>(sv->max_in_flight, (int64_t)sv->inflight.size());
}

// Completed records: copy their rows to pinned host memory (a DMA copy beside the
// running kernel), then to the callers.  Records may complete out of order.  Throws
// HipFail.
void session_collect(sw_server *sv) {
  const size_t n = (size_t)sv->db->n_seqs;
  for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
    SessionRecord &sr = *it;
    ServerRequest *qs[2] = {sr.qa, sr.qb};
    const int32_t row[2] = {sr.row_a, sr.row_b};
    if (!sr.copying) {
      if (__atomic_load_n(complete_flags(sv) + sr.slot, __ATOMIC_ACQUIRE) != sr.r + 1) {
        ++it;
        continue;
      }
      sr.bits = __atomic_load_n(sat_flags(sv) + sr.slot, __ATOMIC_ACQUIRE);
      for (int h = 0; h < 2; ++h)
        if (qs[h] && !(sr.bits & (1 << h)))
          hip_check(hipMemcpyAsync((int32_t *)sv->hscores.ptr + (size_t)row[h] * n,
                                   (const int32_t *)sv->dscores.ptr + (size_t)row[h] * n, n * 4,
                                   hipMemcpyDeviceToHost, sv->cstream));
      sr.copied = sv->free_events.back();
      sv->free_events.pop_back();
      hip_check(hipEventRecord(sr.copied, sv->cstream));
      sr.copying = true;
    }
    if (hipEventQuery(sr.copied) != hipSuccess) {
      ++it;
      continue;
    }
    const int32_t *rows = (const int32_t *)sv->hscores.ptr;
    for (int h = 0; h < 2; ++h) {
      if (!qs[h]) continue;
      if (sr.bits & (1 << h)) {
        // a score at the int16 ceiling: the whole query is searched again exactly
        qs[h]->exact = true;
        sv->exact_queue.push_back(qs[h]);
        continue;
      }
      const double t0 = now_s();
      if (n && qs[h]->scores_out) std::memcpy(qs[h]->scores_out, rows + (size_t)row[h] * n, n * 4);
      sv->copy_s += now_s() - t0;
      finish_request(sv, qs[h], SW_OK);
    }
    sv->free_events.push_back(sr.copied);
    sv->free_rows.push_back(sr.row_a);
    if (sr.row_b >= 0) sv->free_rows.push_back(sr.row_b);
    it = sv->inflight.erase(it);
  }
}

// Fail every record in flight with `status` (after the copy stream has drained).
void session_fail(sw_server *sv, int status) {
  if (sv->inflight.empty()) return;
  (void)hipStreamSynchronize(sv->cstream);
  for (SessionRecord &sr : sv->inflight) {
    if (sr.qa) finish_request(sv, sr.qa, status);
    if (sr.qb) finish_request(sv, sr.qb, status);
    if (sr.copied) sv->free_events.push_back(sr.copied);
    sv->free_rows.push_back(sr.row_a);
    if (sr.row_b >= 0) sv->free_rows.push_back(sr.row_b);
  }
  sv->inflight.clear();
}

// The standard search of one request, blocking, with the server lock released.
void run_exact(sw_server *sv, std::unique_lock<std::mutex> &lk, ServerRequest *r) {
  const int64_t qoff[2] = {0, (int64_t)r->query.size()};
  const uint8_t z = 0;
  lk.unlock();
  const int rc = run_search(sv->db, r->query.empty() ? &z : r->query.data(), qoff, 1,
                            sv->matrix.data(), sv->gap_open, sv->gap_extend, r->scores_out,
                            nullptr, nullptr);
  lk.lock();
  ++sv->exact_runs;
  finish_request(sv, r, rc);
}

// One pass of the session-mode worker (lock held); returns false when it should wait.
bool session_step(sw_server *sv, std::unique_lock<std::mutex> &lk) {
  try {
    session_collect(sv);
  } catch (const HipFail &f) {
    session_fail(sv, map_hip(f.err));
    return true;
  }
  // A launch that has ended: every record it took is complete (its rows copied once the
  // copy stream is done) unless a wait timed out.
  if (sv->open && hipEventQuery(sv->sended) == hipSuccess) {
    (void)hipStreamSynchronize(sv->cstream);
    try {
      session_collect(sv);
    } catch (const HipFail &f) {
      session_fail(sv, map_hip(f.err));
    }
    session_fail(sv, SW_EDEVICE);  // records that never completed
    sv->open = false;
    sv->closing = false;
    return true;
  }
  // requests for the standard path run once the session has drained
  if (!sv->exact_queue.empty()) {
    if (sv->open) {
      session_close(sv);
      return false;
    }
    ServerRequest *r = sv->exact_queue.front();
    sv->exact_queue.erase(sv->exact_queue.begin());
    run_exact(sv, lk, r);
    return true;
  }
  if (sv->closing) return false;  // wait for the closed launch to end
  // the launch's int32 item counter stays far from overflow: a long-running session is
  // closed (its records still complete) and the next record opens a new one
  if (sv->open && (int64_t)(sv->published + 1) * sv->db->ngroups + sv->grid >= ((int64_t)1 << 30)) {
    session_close(sv);
    return false;
  }
  // Admit: publish a record only when the device is about to run out of published work
  // (fewer than half a record's items left unclaimed), so that requests wait here, where
  // two of similar length can still share a record, rather than on the device.  A
  // record's longest groups can keep it on the device well after its items are all
  // claimed, so several records may be in flight (at most max_records).
  bool did = false;
  while (!sv->queue.empty() && (int32_t)sv->inflight.size() < sv->max_records &&
         sv->free_rows.size() >= 1 &&
         (!sv->open || sv->inflight.empty() ||
          (int64_t)sv->published * sv->db->ngroups - claimed_items(sv) < sv->db->ngroups / 2)) {
    ServerRequest *qa = sv->queue.front();
    if (qa->query.empty()) {
      sv->queue.pop_front();
      if (sv->db->n_seqs && qa->scores_out) std::memset(qa->scores_out, 0, (size_t)sv->db->n_seqs * 4);
      qa->t_start = now_s();
      finish_request(sv, qa, SW_OK);
      did = true;
      continue;
    }
    if ((int64_t)qa->query.size() > kServeMaxQuery) {
      sv->queue.pop_front();
      qa->exact = true;
      sv->exact_queue.push_back(qa);
      return true;
    }
    // The queued request of the most similar length, if sharing lanes pays.  A pair takes
    // about 1.8 times as long as one of its queries, so queries are paired only when
    // requests are piling up (several waiting besides this one): under light load each
    // runs alone, at its lowest latency.
    ServerRequest *qb = nullptr;
    size_t qb_at = 0;
    if (sv->max_batch >= 2 && sv->free_rows.size() >= 2 && sv->queue.size() >= kServePairQueue) {
      const size_t look = std::min<size_t>(sv->queue.size(), 64);
      int64_t best = -1;
      for (size_t k = 1; k < look; ++k) {
        ServerRequest *c = sv->queue[k];
        if (c->query.empty() || (int64_t)c->query.size() > kServeMaxQuery) continue;
        const int64_t d = std::llabs((int64_t)c->query.size() - (int64_t)qa->query.size());
        if (worth_pairing((int64_t)qa->query.size(), (int64_t)c->query.size()) &&
            (best < 0 || d < best)) {
          best = d;
          qb = c;
          qb_at = k;
        }
      }
    }
    if (qb) sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)qb_at);
    sv->queue.pop_front();
    try {
      session_publish(sv, qa, qb);
    } catch (const HipFail &f) {
      finish_request(sv, qa, map_hip(f.err));
      if (qb) finish_request(sv, qb, map_hip(f.err));
    }
    did = true;
  }
  // close an idle session after a short linger
  const double t = now_s();
  if (sv->open && sv->inflight.empty() && sv->queue.empty()) {
    if (sv->idle_since == 0) sv->idle_since = t;
    if (t - sv->idle_since >= kServeLinger || sv->stop) session_close(sv);
  } else {
    sv->idle_since = 0;
  }
  return did;
}

void server_loop(sw_server *sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  (void)hipSetDevice(sv->db->device);
  for (;;) {
    bool busy;
    if (sv->session_mode) {
      const bool progressed = session_step(sv, lk);
      busy = sv->open || !sv->exact_queue.empty();
      if (sv->stop && sv->queue.empty() && !busy) break;
      if (progressed) continue;
    } else {
      // retire finished batches
      int in_flight = 0;
      size_t mem_in_flight = 0;
      int64_t items_in_flight = 0;
      for (ServerSlot &sl : sv->slots) {
        if (sl.busy && hipEventQuery(sl.finished) == hipSuccess) server_finish_slot(sv, sl);
        if (sl.busy) {
          ++in_flight;
          mem_in_flight += sl.mem;
          items_in_flight += sl.items;
        }
      }
      if (sv->stop && sv->queue.empty() && in_flight == 0) break;
      if (batch_step(sv, in_flight, mem_in_flight, items_in_flight)) continue;
      busy = in_flight > 0;
    }
    // wait for new work, or poll the work in flight
    if (busy)
      sv->cv.wait_for(lk, std::chrono::microseconds(50));
    else
      sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
  }
}

void server_destroy(sw_server *sv) {
  for (ServerSlot &sl : sv->slots) {
    if (sl.w) destroy_workspace(sl.w);
    if (sl.finished) (void)hipEventDestroy(sl.finished);
    sl.scores.release();
    sl.host_scores.release();
    sl.host_error.release();
  }
  session_release(sv);
  for (auto &kv : sv->requests) delete kv.second;
  delete sv;
}

}  // namespace

SW_API int sw_server_create(sw_db *db, const int32_t *matrix, int32_t gap_open,
                            int32_t gap_extend, int32_t slots, int32_t max_batch,
                            int64_t mem_budget_bytes, sw_server **out) {
  return abi_guard([&]() -> int {
    int rc = validate_search(db, matrix, gap_open, gap_extend);
    if (rc) return rc;
    if (!out || slots < 1 || slots > 16 || max_batch < 1 || max_batch > 4096 ||
        mem_budget_bytes < 0)
      return SW_EINVAL;
    sw_server *sv = new (std::nothrow) sw_server();
    if (!sv) return SW_ENOMEM;
    try {
      sv->db = db;
      sv->matrix.assign(matrix, matrix + (size_t)db->alphabet * db->alphabet);
      sv->gap_open = gap_open;
      sv->gap_extend = gap_extend;
      sv->max_batch = max_batch;
      sv->mem_budget = mem_budget_bytes;
      hip_check(hipSetDevice(db->device));
      const int per_cu = std::max(1, inter16_max_blocks_per_cu(24));
      sv->fill_items = 4LL * per_cu * std::max(1, db->num_cu);
      // Session mode when every record fills the device four times over and no sequence
      // needs the intra-task kernel; its device scratch must fit the free memory and the
      // budget, which also bounds the score rows.
      sv->grid = std::max(1, serve_max_blocks_per_cu()) * std::max(1, db->num_cu);
      sv->max_records = std::max(4, 4 * (int)slots);
      sv->nrows = 2 * sv->max_records;
      // score rows: two per record in flight, fewer if the budget says so (at least two)
      const size_t row_bytes = (size_t)db->n_seqs * 4;
      const int nrec = std::max(4, 2 * sv->max_records);
      const size_t fixed = session_device_bytes(db, sv->grid, nrec, 0);
      if (mem_budget_bytes > 0 && (int64_t)fixed < mem_budget_bytes)
        sv->nrows = (int32_t)std::max<int64_t>(
            2, std::min<int64_t>(sv->nrows, (mem_budget_bytes - (int64_t)fixed) / (int64_t)row_bytes));
      const size_t dev_bytes = fixed + (size_t)sv->nrows * row_bytes;
      const bool fits = dev_bytes + ((size_t)1 << 30) < device_free_bytes() &&
                        (mem_budget_bytes == 0 || (int64_t)dev_bytes <= mem_budget_bytes);
      sv->session_mode = db->longs.empty() && db->n_seqs > 0 &&
                         (int64_t)db->ngroups >= 4LL * sv->grid && fits;
      if (sv->session_mode) {
        session_setup(sv);
      } else {
        sv->slots.resize((size_t)slots);
        for (ServerSlot &sl : sv->slots) {
          sl.w = new_workspace();
          hip_check(hipEventCreateWithFlags(&sl.finished, hipEventDisableTiming));
        }
      }
      sv->worker = std::thread(server_loop, sv);
    } catch (const HipFail &f) {
      server_destroy(sv);
      return map_hip(f.err);
    } catch (const std::bad_alloc &) {
      server_destroy(sv);
      return SW_ENOMEM;
    } catch (...) {  // std::system_error from the worker thread
      server_destroy(sv);
      return SW_EDEVICE;
    }
    *out = sv;
    return SW_OK;
  });
}

SW_API int sw_server_submit(sw_server *sv, const uint8_t *query, int32_t query_len,
                            int32_t *scores_out, uint64_t *ticket) {
  return abi_guard([&]() -> int {
    if (!sv || !ticket) return SW_EINVAL;
    if (!scores_out && sv->db->n_seqs > 0) return SW_EINVAL;
    int rc = validate_query(sv->db, query, query_len);
    if (rc) return rc;
    ServerRequest *r = new (std::nothrow) ServerRequest();
    if (!r) return SW_ENOMEM;
    try {
      r->query.assign(query, query + query_len);
      r->scores_out = scores_out;
      r->t_submit = now_s();
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->stop) {
        delete r;
        return SW_EINVAL;
      }
      r->ticket = sv->next_ticket++;
      sv->requests[r->ticket] = r;
      sv->queue.push_back(r);
      *ticket = r->ticket;
    } catch (...) {  // std::bad_alloc
      delete r;
      return SW_ENOMEM;
    }
    sv->cv.notify_one();
    return SW_OK;
  });
}

SW_API int sw_server_wait(sw_server *sv, uint64_t ticket, double *latency_ms,
                          double *queue_ms) {
  return abi_guard([&]() -> int {
    if (!sv) return SW_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return SW_EINVAL;
    ServerRequest *r = it->second;
    sv->done_cv.wait(lk, [&] { return r->status != 1; });
    const int status = r->status;
    if (latency_ms) *latency_ms = (r->t_done - r->t_submit) * 1e3;
    if (queue_ms) *queue_ms = (r->t_start > 0 ? r->t_start - r->t_submit : 0.0) * 1e3;
    sv->requests.erase(it);
    delete r;
    return status;
  });
}

SW_API int sw_server_stats(sw_server *sv, int64_t *launches, int64_t *max_in_flight,
                           int64_t *refused) {
  return abi_guard([&]() -> int {
    if (!sv) return SW_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (launches) *launches = sv->launches;
    if (max_in_flight) *max_in_flight = sv->max_in_flight;
    if (refused) *refused = sv->refused;
    return SW_OK;
  });
}

SW_API int sw_server_counters(sw_server *sv, int64_t *values, int32_t n) {
  return abi_guard([&]() -> int {
    if (!sv || !values || n < 0) return SW_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    const int64_t v[SW_SERVER_NCOUNTERS] = {sv->launches, sv->max_in_flight, sv->refused,
                                            sv->session_mode ? 1 : 0, sv->records, sv->paired,
                                            sv->exact_runs, sv->session_mode ? sv->grid : 0,
                                            (int64_t)(sv->copy_s * 1e6)};
    for (int32_t k = 0; k < n && k < SW_SERVER_NCOUNTERS; ++k) values[k] = v[k];
    return SW_OK;
  });
}

SW_API void sw_server_free(sw_server *sv) {
  abi_guard_void([&]() {
    if (!sv) return;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipSetDevice(sv->db->device);
    server_destroy(sv);
  });
}

// ------------------------------------------------------------------------ sorting stage
SW_API int sw_topk(const sw_db *cdb, const int32_t *scores_dev, int32_t k, int32_t *hit_index,
                   int32_t *hit_score, int32_t *n_hits, void *hip_stream) {
  return abi_guard([&]() -> int {
    if (!cdb) return SW_ENODB;
    if (k < 1 || k > kTopkMax || !n_hits || !hit_index || !hit_score) return SW_EINVAL;
    sw_db *db = const_cast<sw_db *>(cdb);
    const int64_t n = db->n_seqs;
    if (n > 0 && !scores_dev) return SW_EINVAL;
    const int32_t kk = (int32_t)std::min<int64_t>(k, n);
    *n_hits = 0;
    if (kk == 0) return SW_OK;
    std::lock_guard<std::mutex> lk(db->topk_mu);
    try {
      hip_check(hipSetDevice(db->device));
      const size_t off_hist = 64, off_list = off_hist + 256 * 4, off_idx = off_list + kTopkMax * 8,
                   off_sc = off_idx + kTopkMax * 4, total = off_sc + kTopkMax * 4;
      grow(db->topk_scratch, total);
      uint8_t *base = (uint8_t *)db->topk_scratch.ptr;
      TopkArgs a;
      a.scores = scores_dev;
      a.n = n;
      a.k = kk;
      a.state = (TopkState *)base;
      a.hist = (uint32_t *)(base + off_hist);
      a.list = (uint64_t *)(base + off_list);
      a.hit_index = (int32_t *)(base + off_idx);
      a.hit_score = (int32_t *)(base + off_sc);
      hipStream_t s = (hipStream_t)hip_stream;
      hip_check(launch_topk(a, s));
      hip_check(hipMemcpyAsync(hit_index, a.hit_index, (size_t)kk * 4, hipMemcpyDeviceToHost, s));
      hip_check(hipMemcpyAsync(hit_score, a.hit_score, (size_t)kk * 4, hipMemcpyDeviceToHost, s));
      hip_check(hipStreamSynchronize(s));
    } catch (const HipFail &f) {
      return map_hip(f.err);
    } catch (const std::bad_alloc &) {
      return SW_ENOMEM;
    }
    *n_hits = kk;
    return SW_OK;
  });
}
