// Sorting stage of a search on gfx950: the k best hits of a score array, selected and
// sorted on the device.
#include <algorithm>
#include <mutex>

#include "../../include/swmi.h"

#include "swmi_internal.h"

namespace swmi {

// ------------------------------------------------------------------------ sorting stage
// Top-k hits (Section 4, sorting stage) by exact radix selection on 64-bit keys
// key = score << 32 | ~index: keys are unique, and a larger key means a higher score or,
// for equal scores, a lower index.  Eight passes of 8-bit digits (high to low) find the
// k-th largest key K; the k keys >= K are then collected and sorted in one workgroup.
__device__ __forceinline__ uint64_t topk_key(const int32_t *scores, int64_t i) {
  return ((uint64_t)(uint32_t)scores[i] << 32) | (uint32_t)(~(uint32_t)i);
}

__global__ void k_topk_hist(TopkArgs a, int pass) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int shift = 56 - 8 * pass;
  const uint64_t prefix = a.state->prefix;
  const uint64_t mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = topk_key(a.scores, i);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&a.hist[threadIdx.x], h[threadIdx.x]);
}

// one workgroup of 256 threads: choose the digit of this pass and clear the histogram
__global__ void k_topk_pick(TopkArgs a, int pass) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = a.hist[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t need = a.state->remaining;
    int d = 255;
    for (; d > 0; --d) {
      if (h[d] >= need) break;
      need -= h[d];
    }
    a.state->remaining = need;
    a.state->prefix |= (uint64_t)d << (56 - 8 * pass);
  }
  a.hist[threadIdx.x] = 0;
}

__global__ void k_topk_collect(TopkArgs a) {
  const uint64_t kth = a.state->prefix;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = topk_key(a.scores, i);
    if (key >= kth) {
      const uint32_t slot = atomicAdd(&a.state->count, 1u);
      if (slot < (uint32_t)a.k) a.list[slot] = key;
    }
  }
}

// bitonic sort (descending) of the k collected keys in one workgroup of 1024 threads
__global__ void k_topk_sort(TopkArgs a) {
  __shared__ uint64_t s[kTopkMax];
  const int k = a.k;
  int np = 1;
  while (np < k) np <<= 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s[i] = i < k ? a.list[i] : 0ull;
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const uint64_t x = s[i], y = s[j];
          if (desc ? (x < y) : (x > y)) {
            s[i] = y;
            s[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    a.hit_score[i] = (int32_t)(uint32_t)(s[i] >> 32);
    a.hit_index[i] = (int32_t)(~(uint32_t)s[i]);
  }
}

__global__ void k_topk_init(TopkArgs a) {
  a.state->prefix = 0;
  a.state->remaining = (uint32_t)a.k;
  a.state->count = 0;
  a.hist[threadIdx.x] = 0;
}

hipError_t launch_topk(const TopkArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, a);
  int grid = (int)std::min<int64_t>(2048, (a.n + 255) / 256);
  if (grid < 1) grid = 1;
  for (int pass = 0; pass < 8; ++pass) {
    hipLaunchKernelGGL(k_topk_hist, dim3(grid), dim3(256), 0, s, a, pass);
    hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(256), 0, s, a, pass);
  }
  hipLaunchKernelGGL(k_topk_collect, dim3(grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ top-k without allocation
// sw_topk_noalloc: the same selection with its scratch (selection state, digit histogram,
// collected keys, results) in a file-scope device array instead of memory the library
// allocates, for callers that cannot allocate.  Every call on a device uses that device's
// copy of the array; calls are serialised per device, and the state and histogram are
// cleared by k_topk_init at the start of every call.
constexpr size_t kTopkOffHist = 64;
constexpr size_t kTopkOffList = kTopkOffHist + 256 * sizeof(uint32_t);
constexpr size_t kTopkOffIdx = kTopkOffList + (size_t)kTopkMax * sizeof(uint64_t);
constexpr size_t kTopkOffScore = kTopkOffIdx + (size_t)kTopkMax * sizeof(int32_t);
constexpr size_t kTopkScratchBytes = kTopkOffScore + (size_t)kTopkMax * sizeof(int32_t);
static_assert(sizeof(TopkState) <= kTopkOffHist, "state fits its slot");

static __device__ __align__(256) uint8_t scratch[kTopkScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};     // scratch's device address, per device
std::mutex g_scratch_use[kMaxDevices];     // one call at a time per device
}  // namespace

// The device address of `scratch` on the current device, looked up once per device.
static hipError_t scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

// The selection of sw_topk_noalloc, in the device's copy of `scratch` (base_ptr).
static int topk_in_scratch(const sw_db *, const int32_t *scores_dev, int64_t n, int32_t kk,
                           void *base_ptr, int32_t *hit_index, int32_t *hit_score,
                           int32_t *n_hits, void *hip_stream) {
  uint8_t *base = (uint8_t *)base_ptr;
  TopkArgs a;
  a.scores = scores_dev;
  a.n = n;
  a.k = kk;
  a.state = (TopkState *)base;
  a.hist = (uint32_t *)(base + kTopkOffHist);
  a.list = (uint64_t *)(base + kTopkOffList);
  a.hit_index = (int32_t *)(base + kTopkOffIdx);
  a.hit_score = (int32_t *)(base + kTopkOffScore);
  hipStream_t s = (hipStream_t)hip_stream;
  if (launch_topk(a, s) != hipSuccess) return SW_EDEVICE;
  if (hipMemcpyAsync(hit_index, a.hit_index, (size_t)kk * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hit_score, a.hit_score, (size_t)kk * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SW_EDEVICE;
  *n_hits = kk;
  return SW_OK;
}

}  // namespace swmi

extern "C" __attribute__((visibility("default")))
int sw_topk_noalloc(const sw_db *db, const int32_t *scores_dev, int32_t k, int32_t *hit_index,
                    int32_t *hit_score, int32_t *n_hits, void *hip_stream) {
  using namespace swmi;
  if (!db) return SW_ENODB;
  if (k < 1 || k > kTopkMax || !n_hits || !hit_index || !hit_score) return SW_EINVAL;
  const int64_t n = sw_db_size(db);
  if (n < 0) return SW_ENODB;
  if (n > 0 && !scores_dev) return SW_EINVAL;
  const int32_t kk = (int32_t)std::min<int64_t>(k, n);
  *n_hits = 0;
  if (kk == 0) return SW_OK;
  // the database's device, made current (its copy of the array is the one used)
  const int device = db_device(db);
  if (device < 0 || device >= kMaxDevices || hipSetDevice(device) != hipSuccess)
    return SW_EDEVICE;
  void *base_ptr = nullptr;
  try {  // (a lock can throw std::system_error; nothing may cross the C ABI)
    if (scratch_address(device, &base_ptr) != hipSuccess) return SW_EDEVICE;
    std::lock_guard<std::mutex> use(g_scratch_use[device]);
    return topk_in_scratch(db, scores_dev, n, kk, base_ptr, hit_index, hit_score, n_hits,
                           hip_stream);
  } catch (...) {
    return SW_EDEVICE;
  }
}

