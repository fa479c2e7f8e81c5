// Host side of the C ABI declared in include/swmi.h: argument checks, database
// pre-processing (Section 4: sort by length, group by lane count, pad), device
// workspaces, and the launch sequence of one search.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/swmi.h"
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
  hipEvent_t done = nullptr, fork = nullptr, join = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;  // inter-task kernel timing
  bool timed = false;
  bool busy = false;
  DevBuf queries, qoff, qdesc, matrix, qp16, qp32, ctr, flagged, longitems, bnd16, bnd32,
      scores;
  HostBuf staging;
  size_t total_bytes() const {
    return queries.bytes + qoff.bytes + qdesc.bytes + matrix.bytes + qp16.bytes + qp32.bytes +
           ctr.bytes + flagged.bytes + longitems.bytes + bnd16.bytes + bnd32.bytes + scores.bytes;
  }
};

}  // namespace

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
  DevBuf packed, groups, perm, lens;
  struct LongSeq {
    int64_t base;
    int32_t len;
    int32_t orig;
  };
  std::vector<LongSeq> longs;  // sorted by decreasing length
  std::vector<GroupDesc> hgroups;   // host copy of the group table
  std::vector<int32_t> hperm;       // host copy: sorted position -> caller index
  std::vector<int32_t> hlens;       // host copy: sorted position -> length
  int64_t short_residues = 0;       // residues in groups
  std::mutex mu;
  std::vector<Workspace *> pool;
  std::atomic<bool> timing{false};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_events;
  int64_t timing_launches = 0;
  double timing_ms = 0.0;
};

namespace {

int map_hip(hipError_t e) {
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SW_ENOMEM : SW_EDEVICE;
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
  for (DevBuf *b : {&w->queries, &w->qoff, &w->qdesc, &w->matrix, &w->qp16, &w->qp32, &w->ctr,
                    &w->flagged, &w->longitems, &w->bnd16, &w->bnd32, &w->scores})
    b->release();
  w->staging.release();
  for (hipEvent_t e : {w->done, w->fork, w->join, w->t0, w->t1})
    if (e) (void)hipEventDestroy(e);
  if (w->own) (void)hipStreamDestroy(w->own);
  if (w->aux) (void)hipStreamDestroy(w->aux);
  delete w;
}

Workspace *acquire(sw_db *db) {
  std::lock_guard<std::mutex> lk(db->mu);
  for (Workspace *w : db->pool) {
    if (!w->busy && hipEventQuery(w->done) == hipSuccess) {
      w->busy = true;
      return w;
    }
  }
  // at most 8 workspaces; beyond that wait for the oldest idle one
  if (db->pool.size() >= 8) {
    for (Workspace *w : db->pool) {
      if (!w->busy) {
        hip_check(hipEventSynchronize(w->done));
        w->busy = true;
        return w;
      }
    }
  }
  Workspace *w = new Workspace();
  try {
    hip_check(hipStreamCreateWithFlags(&w->own, hipStreamNonBlocking));
    hip_check(hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking));
    hip_check(hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
    hip_check(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
    hip_check(hipEventCreateWithFlags(&w->join, hipEventDisableTiming));
    hip_check(hipEventCreate(&w->t0));
    hip_check(hipEventCreate(&w->t1));
    hip_check(hipEventRecord(w->done, w->own));
  } catch (...) {
    destroy_workspace(w);
    throw;
  }
  w->busy = true;
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

// Strip half-height T for the inter-task kernel: the fewest padded query rows, weighted
// by the measured relative per-cell speed of each compiled height on gfx950 (T = 24 runs
// at three waves per SIMD and was fastest on the full-scale search).
int choose_T(const std::vector<int64_t> &lens) {
  const int64_t forced = g_knob_strip_rows.load();
  if (forced > 0 && inter16_supported((int)forced)) return (int)forced;
  struct Cand { int T; double speed; };
  const Cand cands[] = {{24, 1.0}, {40, 0.985}, {32, 0.968}, {16, 0.89}};
  int best = 24;
  double best_cost = 1e300;
  for (const Cand &c : cands) {
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

struct Plan {
  int T = 32;
  int32_t ngroups_inter = 0;
  int32_t n_wide = 0;
  int grid16 = 0;
  int grid_long = 0;
  int grid_re = 0;
  std::vector<QueryDesc> qd;
  std::vector<PairItem> longitems;
  int64_t qp16_elems = 0, qp32_elems = 0;
};

// Enqueue one (possibly batched) search on `s`.  Queries are host memory; scores go to
// `scores_dev` (n_queries x n_seqs).  The caller owns `w` until `done` is recorded.
void enqueue_search(sw_db *db, Workspace *w, const uint8_t *queries, const int64_t *qoff,
                    int64_t nq, const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t *scores_dev, hipStream_t s) {
  hip_check(hipSetDevice(db->device));
  const int A = db->alphabet;
  Plan p;
  std::vector<int64_t> lens((size_t)nq);
  for (int64_t q = 0; q < nq; ++q) lens[q] = qoff[q + 1] - qoff[q];
  p.T = choose_T(lens);
  const int band = 64 * kIntraR;
  p.qd.resize((size_t)nq);
  for (int64_t q = 0; q < nq; ++q) {
    QueryDesc &d = p.qd[q];
    d.m = (int32_t)lens[q];
    d.nstrips = (int32_t)((lens[q] + 2 * p.T - 1) / (2 * p.T));
    d.nbands = (int32_t)((lens[q] + band - 1) / band);
    d.mpad32 = d.nbands * band;
    d.qp16 = p.qp16_elems;
    d.qp32 = p.qp32_elems;
    d.out = q * db->n_seqs;
    p.qp16_elems += (int64_t)d.nstrips * kCodes * 2 * p.T;
    p.qp32_elems += (int64_t)kCodes * d.mpad32;
  }
  // launch geometry of the inter-task kernel
  int per_cu = (int)g_knob_grid_waves.load();
  if (per_cu <= 0) per_cu = std::max(1, inter16_max_blocks_per_cu(p.T));
  const int64_t lanes = (int64_t)per_cu * db->num_cu * 64;

  // Route the longest groups to the intra-task kernel.  One lane runs a whole alignment
  // in the inter-task kernel, so a group of length L costs about L * m on one wave; keep
  // L below twice the average number of residues per lane (weighted by the number of
  // equally long queries), else that wave becomes the critical path.
  int64_t sum_m = 0, max_m = 1;
  for (int64_t q = 0; q < nq; ++q) { sum_m += lens[q]; max_m = std::max(max_m, lens[q]); }
  const double weight = (double)sum_m / (double)max_m;
  int64_t route = (int64_t)(2.0 * (double)db->short_residues * weight / (double)lanes);
  route = std::max<int64_t>(route, 64);
  const int64_t forced_route = g_knob_route_len.load();
  if (forced_route > 0) route = forced_route;
  int32_t ninter = db->ngroups;
  while (ninter > 0 && db->hgroups[ninter - 1].maxlen > route) --ninter;
  p.ngroups_inter = ninter;

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
    const double cost = (double)len * (double)lens[q];
    const bool is_wide = len >= 64 * 6 * kIntraLag && p.qd[q].nbands >= 2;
    (is_wide ? wide : narrow).emplace_back(cost, it);
  };
  for (int64_t q = 0; q < nq; ++q) {
    if (lens[q] == 0) continue;
    for (const auto &L : db->longs) add_item(L.base, 4, L.len, L.orig, q);
    for (int32_t g = ninter; g < db->ngroups; ++g) {
      const GroupDesc &gd = db->hgroups[g];
      for (int32_t l = 0; l < gd.count; ++l)
        add_item(gd.base + 4 * l, 256, db->hlens[gd.first + l], db->hperm[gd.first + l], q);
    }
  }
  auto by_cost = [](const std::pair<double, PairItem> &x, const std::pair<double, PairItem> &y) {
    return x.first > y.first;
  };
  std::stable_sort(wide.begin(), wide.end(), by_cost);
  std::stable_sort(narrow.begin(), narrow.end(), by_cost);
  p.n_wide = (int32_t)wide.size();
  for (auto &x : wide) p.longitems.push_back(x.second);
  for (auto &x : narrow) p.longitems.push_back(x.second);

  const int64_t nitems16 = (int64_t)ninter * nq;
  p.grid16 = (int)std::min<int64_t>(nitems16, (int64_t)per_cu * db->num_cu);
  p.grid_long = (int)std::min<int64_t>((int64_t)wide.size() + ((int64_t)narrow.size() + kIntraWaves - 1) / kIntraWaves,
                                       4LL * db->num_cu);
  p.grid_re = (db->n_short > 0 && nq > 0) ? db->num_cu : 0;
  const int grid32 = p.grid_long + p.grid_re;

  // workspace sizes
  const int64_t qbytes = qoff[nq];
  const size_t bnd16_slot = (size_t)db->max_ncols * 64;  // dwords
  const int bnd32_stride = ((db->max_len + 128 + 63) / 64) * 64;
  const size_t bnd32_slot = (size_t)std::max(kIntraWaves + 1, 2 * kIntraWaves) * bnd32_stride;
  const size_t need_flagged = (size_t)std::max<int64_t>(1, db->n_short * nq);
  const int64_t cap_mb = g_knob_mem_cap_mb.load();
  {
    size_t need = (size_t)qbytes + 64 + (nq + 1) * 8 + nq * sizeof(QueryDesc) + A * A * 4 +
                  (size_t)p.qp16_elems * 2 + (size_t)p.qp32_elems * 2 + sizeof(Counters) +
                  need_flagged * sizeof(PairItem) + p.longitems.size() * sizeof(PairItem) +
                  (size_t)p.grid16 * bnd16_slot * 4 + (size_t)grid32 * bnd32_slot * 8;
    if (cap_mb > 0 && (int64_t)(std::max(need, w->total_bytes()) >> 20) > cap_mb)
      throw HipFail{hipErrorOutOfMemory};
  }
  grow(w->queries, (size_t)qbytes + 64);
  grow(w->qoff, (size_t)(nq + 1) * 8);
  grow(w->qdesc, std::max<size_t>(1, nq) * sizeof(QueryDesc));
  grow(w->matrix, (size_t)A * A * 4);
  grow(w->qp16, (size_t)std::max<int64_t>(8, p.qp16_elems) * 2);
  grow(w->qp32, (size_t)std::max<int64_t>(8, p.qp32_elems) * 2);
  grow(w->ctr, sizeof(Counters));
  grow(w->flagged, need_flagged * sizeof(PairItem));
  grow(w->longitems, std::max<size_t>(1, p.longitems.size()) * sizeof(PairItem));
  grow(w->bnd16, std::max<size_t>(1, (size_t)p.grid16 * bnd16_slot) * 4);
  grow(w->bnd32, std::max<size_t>(1, (size_t)grid32 * bnd32_slot) * 8);

  // stage small inputs through pinned memory (reused only after `done`)
  const size_t off_qoff = ((size_t)qbytes + 63) & ~size_t(63);
  const size_t off_qd = off_qoff + (((size_t)(nq + 1) * 8 + 63) & ~size_t(63));
  const size_t off_mx = off_qd + ((nq * sizeof(QueryDesc) + 63) & ~size_t(63));
  const size_t off_li = off_mx + (((size_t)A * A * 4 + 63) & ~size_t(63));
  const size_t stage_bytes = off_li + p.longitems.size() * sizeof(PairItem) + 64;
  grow_host(w->staging, stage_bytes);
  uint8_t *st = (uint8_t *)w->staging.ptr;
  if (qbytes) std::memcpy(st, queries, (size_t)qbytes);
  std::memcpy(st + off_qoff, qoff, (size_t)(nq + 1) * 8);
  if (nq) std::memcpy(st + off_qd, p.qd.data(), nq * sizeof(QueryDesc));
  std::memcpy(st + off_mx, matrix, (size_t)A * A * 4);
  if (!p.longitems.empty())
    std::memcpy(st + off_li, p.longitems.data(), p.longitems.size() * sizeof(PairItem));
  if (qbytes) hip_check(hipMemcpyAsync(w->queries.ptr, st, (size_t)qbytes, hipMemcpyHostToDevice, s));
  hip_check(hipMemcpyAsync(w->qoff.ptr, st + off_qoff, (size_t)(nq + 1) * 8, hipMemcpyHostToDevice, s));
  if (nq) hip_check(hipMemcpyAsync(w->qdesc.ptr, st + off_qd, nq * sizeof(QueryDesc), hipMemcpyHostToDevice, s));
  hip_check(hipMemcpyAsync(w->matrix.ptr, st + off_mx, (size_t)A * A * 4, hipMemcpyHostToDevice, s));
  if (!p.longitems.empty())
    hip_check(hipMemcpyAsync(w->longitems.ptr, st + off_li, p.longitems.size() * sizeof(PairItem),
                             hipMemcpyHostToDevice, s));

  Counters *ctr = (Counters *)w->ctr.ptr;
  ProfileArgs pa;
  pa.query = (const uint8_t *)w->queries.ptr;
  pa.qoff = (const int64_t *)w->qoff.ptr;
  pa.queries = (const QueryDesc *)w->qdesc.ptr;
  pa.nqueries = (int32_t)nq;
  pa.matrix = (const int32_t *)w->matrix.ptr;
  pa.alphabet = A;
  pa.T = p.T;
  pa.qp16 = (int16_t *)w->qp16.ptr;
  pa.qp32 = (int16_t *)w->qp32.ptr;
  pa.ctr = ctr;
  if (nq > 0) hip_check(launch_profile(pa, s));

  // long sequences: intra-task kernel on the auxiliary stream, concurrent with the sweep
  if (p.grid_long > 0) {
    hip_check(hipEventRecord(w->fork, s));
    hip_check(hipStreamWaitEvent(w->aux, w->fork, 0));
    IntraArgs ia;
    ia.packed = (const uint8_t *)db->packed.ptr;
    ia.items = (const PairItem *)w->longitems.ptr;
    ia.count_dev = nullptr;
    ia.count = (int32_t)p.longitems.size();
    ia.next = &ctr->intra_next;
    ia.next_narrow = &ctr->intra_narrow;
    ia.n_wide = p.n_wide;
    ia.queries = (const QueryDesc *)w->qdesc.ptr;
    ia.qp32 = (const int16_t *)w->qp32.ptr;
    ia.goe = gap_open + gap_extend;
    ia.ge = gap_extend;
    ia.scores = scores_dev;
    ia.bnd = (int2 *)w->bnd32.ptr;
    ia.bnd_slot_elems = (int64_t)bnd32_slot;
    ia.bnd_stride = bnd32_stride;
    hip_check(launch_intra32(ia, kIntraR, kIntraWaves, p.grid_long, w->aux));
    hip_check(hipEventRecord(w->join, w->aux));
  }

  if (nq > 0) {
    InterArgs ia;
    ia.packed = (const uint8_t *)db->packed.ptr;
    ia.groups = (const GroupDesc *)db->groups.ptr;
    ia.ngroups = p.ngroups_inter;
    ia.nqueries = (int32_t)nq;
    ia.queries = (const QueryDesc *)w->qdesc.ptr;
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
    ia.recompute_all = g_knob_recompute_all.load() ? 1 : 0;
    ia.nitems = (int32_t)nitems16;
    const bool timed = db->timing.load();
    if (timed) hip_check(hipEventRecord(w->t0, s));
    hip_check(launch_inter16(ia, p.T, p.grid16, s));
    if (timed) {
      hip_check(hipEventRecord(w->t1, s));
      w->timed = true;
    }
    // exact int32 recompute of the saturated alignments (count read on the device);
    // it uses the boundary slots after the long-sequence kernel's, so both may overlap
    IntraArgs ra;
    ra.packed = (const uint8_t *)db->packed.ptr;
    ra.items = (const PairItem *)w->flagged.ptr;
    ra.count_dev = &ctr->flagged;
    ra.count = 0;
    ra.next = &ctr->recompute_next;
    ra.next_narrow = &ctr->recompute_narrow;
    ra.n_wide = 0;
    ra.queries = (const QueryDesc *)w->qdesc.ptr;
    ra.qp32 = (const int16_t *)w->qp32.ptr;
    ra.goe = gap_open + gap_extend;
    ra.ge = gap_extend;
    ra.scores = scores_dev;
    ra.bnd = (int2 *)w->bnd32.ptr + (size_t)p.grid_long * bnd32_slot;
    ra.bnd_slot_elems = (int64_t)bnd32_slot;
    ra.bnd_stride = bnd32_stride;
    hip_check(launch_intra32(ra, kIntraR, kIntraWaves, p.grid_re, s));
  }
  if (p.grid_long > 0) hip_check(hipStreamWaitEvent(s, w->join, 0));
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
      if (value != 0 && !inter16_supported((int)value)) return SW_EINVAL;
      g_knob_strip_rows = value; return SW_OK;
    case SW_KNOB_GRID_WAVES: if (value < 0 || value > 64) return SW_EINVAL; g_knob_grid_waves = value; return SW_OK;
    case SW_KNOB_MEM_CAP_MB: if (value < 0) return SW_EINVAL; g_knob_mem_cap_mb = value; return SW_OK;
    case SW_KNOB_ROUTE_LEN: if (value < 0) return SW_EINVAL; g_knob_route_len = value; return SW_OK;
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
    default: return SW_EINVAL;
  }
}

SW_API int sw_db_load(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs,
                      int32_t alphabet, sw_db **out) {
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
    std::vector<int32_t> lens((size_t)std::max<int64_t>(1, n_short));
    for (int64_t p = 0; p < n_short; ++p) lens[p] = (int32_t)len_of(order[p]);
    for (int64_t p = n_seqs - 1; p >= n_short; --p) {  // longest first
      sw_db::LongSeq L;
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
    delete db;
    return f.err == hipErrorNoDevice || f.err == hipErrorNoBinaryForGpu ? SW_EDEVICE
                                                                      : map_hip(f.err);
  } catch (const std::bad_alloc &) {
    if (d_raw) (void)hipFree(d_raw);
    if (d_off) (void)hipFree(d_off);
    db->packed.release(); db->groups.release(); db->perm.release(); db->lens.release();
    delete db;
    return SW_ENOMEM;
  }
  *out = db;
  return SW_OK;
}

SW_API int64_t sw_db_size(const sw_db *db) { return db ? db->n_seqs : SW_ENODB; }

SW_API void sw_db_free(sw_db *db) {
  if (!db) return;
  (void)hipSetDevice(db->device);
  for (Workspace *w : db->pool) destroy_workspace(w);
  for (auto &e : db->timing_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  db->packed.release(); db->groups.release(); db->perm.release(); db->lens.release();
  delete db;
}

namespace {

void collect_timing(sw_db *db, Workspace *w) {
  if (!w->timed) return;
  w->timed = false;
  float ms = 0.f;
  hip_check(hipEventSynchronize(w->t1));
  hip_check(hipEventElapsedTime(&ms, w->t0, w->t1));
  std::lock_guard<std::mutex> lk(db->mu);
  db->timing_launches += 1;
  db->timing_ms += ms;
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
    hip_check(hipEventRecord(w->done, s));
    if (host_out) {
      if (nscores > 0)
        hip_check(hipMemcpyAsync(host_out, scores, nscores * 4, hipMemcpyDeviceToHost, s));
      hip_check(hipStreamSynchronize(s));
    }
    if (db->timing.load() && host_out) collect_timing(db, w);
    if (db->timing.load() && !host_out && w->timed) {
      // keep the event pair for sw_timing_read; replace the workspace's own pair
      std::lock_guard<std::mutex> lk(db->mu);
      db->timing_events.emplace_back(w->t0, w->t1);
      w->timed = false;
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        w->t0 = a;
        w->t1 = b;
      }
    }
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
  int rc = validate_search(db, matrix, gap_open, gap_extend);
  if (rc) return rc;
  if (!scores_out && db->n_seqs > 0) return SW_EINVAL;
  if ((rc = validate_query(db, query, query_len))) return rc;
  const int64_t qoff[2] = {0, query_len};
  return run_search(db, query, qoff, 1, matrix, gap_open, gap_extend, scores_out, nullptr, nullptr);
}

SW_API int sw_search_async(const sw_db *db, const uint8_t *query, int32_t query_len,
                           const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                           int32_t *scores_dev, void *hip_stream) {
  int rc = validate_search(db, matrix, gap_open, gap_extend);
  if (rc) return rc;
  if (!scores_dev && db->n_seqs > 0) return SW_EINVAL;
  if ((rc = validate_query(db, query, query_len))) return rc;
  if (db->n_seqs == 0) return SW_OK;
  const int64_t qoff[2] = {0, query_len};
  return run_search(db, query, qoff, 1, matrix, gap_open, gap_extend, nullptr, scores_dev,
                    (hipStream_t)hip_stream);
}

SW_API int sw_search_batch(const sw_db *db, const uint8_t *queries, const int64_t *query_offsets,
                           int64_t n_queries, const int32_t *matrix, int32_t gap_open,
                           int32_t gap_extend, int32_t *scores_out) {
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
}

SW_API int sw_timing_enable(sw_db *db, int32_t enable) {
  if (!db) return SW_ENODB;
  std::lock_guard<std::mutex> lk(db->mu);
  db->timing = enable != 0;
  db->timing_launches = 0;
  db->timing_ms = 0.0;
  for (auto &e : db->timing_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  db->timing_events.clear();
  return SW_OK;
}

SW_API int sw_timing_read(const sw_db *cdb, int64_t *launches, double *total_ms) {
  if (!cdb) return SW_ENODB;
  if (!launches || !total_ms) return SW_EINVAL;
  sw_db *db = const_cast<sw_db *>(cdb);
  std::lock_guard<std::mutex> lk(db->mu);
  for (auto &e : db->timing_events) {
    float ms = 0.f;
    if (hipEventSynchronize(e.second) != hipSuccess) return SW_EDEVICE;
    if (hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess) return SW_EDEVICE;
    db->timing_launches += 1;
    db->timing_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  db->timing_events.clear();
  *launches = db->timing_launches;
  *total_ms = db->timing_ms;
  return SW_OK;
}
