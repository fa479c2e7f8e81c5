// Sorting stage of a search on gfx950: the k best hits of a score array, selected and
// sorted on the device.
#include <algorithm>

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

}  // namespace swmi
