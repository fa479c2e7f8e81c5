// VALU calibration kernels (libswmi_calib.so): register-only copies of the DP cell at
// three integer widths, to measure on the device what each arithmetic tier can sustain
// without memory traffic.
//
//   kind 0: packed int16, two alignments per 32-bit lane (the inter-task cell: saturating
//           add, three maxima for H and the running maximum, three saturating subtracts
//           and two maxima for E and F, one v_perm_b32 to pack the two profile values);
//   kind 1: int32, one alignment per lane (the intra-task cell);
//   kind 2: SWAR int8, four alignments per lane in unsigned biased bytes, every byte
//           operation built from 32-bit logic (CDNA4 has no packed 8-bit add, subtract
//           or maximum).
//
// Each lane runs two independent chains (as the inter-task kernel's lead and lag columns)
// over kRows rows and `ncols` columns.  The result is folded into one word per lane so
// the work cannot be removed.  Recurrences follow Section 2, Eqs. 1-3 (E and F clamped at
// zero, which leaves H unchanged).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "swmi_calib.h"

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_adds(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(s16x2, a),
                                                                    __builtin_bit_cast(s16x2, b)));
}
__device__ __forceinline__ uint32_t pk_subu(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                    __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, a),
                                                                __builtin_bit_cast(s16x2, b)));
}
__device__ __forceinline__ int32_t subu32(int32_t a, int32_t b) {
  return (int32_t)__builtin_elementwise_sub_sat((uint32_t)a, (uint32_t)b);
}

// Byte-wise unsigned arithmetic on four lanes of a 32-bit word (no carries between bytes).
// bytemask turns bit 7 of each byte into a full byte: (x << 1) - (x >> 7) is
// sum(0x100 << 8k) - sum(1 << 8k) = sum(0xff << 8k), modulo 2^32.
__device__ __forceinline__ uint32_t bytemask(uint32_t top_bits) {
  return (top_bits << 1) - (top_bits >> 7);
}
__device__ __forceinline__ uint32_t addus8(uint32_t a, uint32_t b) {
  const uint32_t sum = ((a & 0x7f7f7f7fu) + (b & 0x7f7f7f7fu)) ^ ((a ^ b) & 0x80808080u);
  const uint32_t carry = ((a & b) | ((a | b) & ~sum)) & 0x80808080u;  // byte overflowed
  return sum | bytemask(carry);
}
__device__ __forceinline__ uint32_t subus8(uint32_t a, uint32_t b) {
  const uint32_t d = ((a | 0x80808080u) - (b & 0x7f7f7f7fu)) ^ ((a ^ ~b) & 0x80808080u);
  const uint32_t borrow = ((~a & b) | (~(a ^ b) & d)) & 0x80808080u;  // a < b in that byte
  return d & ~bytemask(borrow);
}
__device__ __forceinline__ uint32_t maxu8(uint32_t a, uint32_t b) { return b + subus8(a, b); }

struct Cell16 {
  static constexpr int kCellsPerLane = 2;
  uint32_t goe, ge;
  __device__ uint32_t operator()(uint32_t hd, uint32_t p0, uint32_t p1, uint32_t &E, uint32_t &f,
                                 uint32_t &vmax) const {
    const uint32_t sm = __builtin_amdgcn_perm(p1, p0, 0x05040100u);
    const uint32_t h = pk_max(pk_max(pk_adds(hd, sm), E), f);
    vmax = pk_max(vmax, h);
    const uint32_t t = pk_subu(h, goe);
    E = pk_max(pk_subu(E, ge), t);
    f = pk_max(pk_subu(f, ge), t);
    return h;
  }
};

struct Cell32 {
  static constexpr int kCellsPerLane = 1;
  uint32_t goe, ge;
  __device__ uint32_t operator()(uint32_t hd, uint32_t p0, uint32_t, uint32_t &E, uint32_t &f,
                                 uint32_t &vmax) const {
    const int32_t h = max(max((int32_t)hd + (int32_t)(int8_t)p0, (int32_t)E), (int32_t)f);
    vmax = (uint32_t)max((int32_t)vmax, h);
    const int32_t t = subu32(h, (int32_t)goe);
    E = (uint32_t)max(subu32((int32_t)E, (int32_t)ge), t);
    f = (uint32_t)max(subu32((int32_t)f, (int32_t)ge), t);
    return (uint32_t)h;
  }
};

struct Cell8 {
  static constexpr int kCellsPerLane = 4;
  uint32_t goe, ge;  // replicated in every byte; profile bytes carry score + bias
  __device__ uint32_t operator()(uint32_t hd, uint32_t p0, uint32_t, uint32_t &E, uint32_t &f,
                                 uint32_t &vmax) const {
    const uint32_t bias = 0x40404040u;
    const uint32_t h = maxu8(maxu8(subus8(addus8(hd, p0), bias), E), f);
    vmax = maxu8(vmax, h);
    const uint32_t t = subus8(h, goe);
    E = maxu8(subus8(E, ge), t);
    f = maxu8(subus8(f, ge), t);
    return h;
  }
};

template <typename Cell, int ROWS>
__global__ __launch_bounds__(64) void k_cellmix(uint32_t *out, int ncols, uint32_t seed,
                                                Cell cell) {
  uint32_t Ha[ROWS], Ea[ROWS], Hb[ROWS], Eb[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) { Ha[r] = 0; Ea[r] = 0; Hb[r] = 0; Eb[r] = 0; }
  uint32_t va = 0, vb = 0;
  uint32_t prof[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) prof[i] = (seed * (threadIdx.x + 2 * i + 1)) & 0x07070707u;
  for (int c = 0; c < ncols; ++c) {
    uint32_t fa = 0, fb = 0, da = (uint32_t)c, db = (uint32_t)c ^ 5u;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const uint32_t pa = prof[r & 7] ^ (uint32_t)c, pb = prof[(r + 3) & 7] ^ (uint32_t)c;
      const uint32_t ha = cell(da, pa, pb, Ea[r], fa, va);
      const uint32_t hb = cell(db, pb, pa, Eb[r], fb, vb);
      da = Ha[r]; Ha[r] = ha;
      db = Hb[r]; Hb[r] = hb;
    }
  }
  out[blockIdx.x * 64 + threadIdx.x] = va ^ vb;
}

constexpr int kRows = 16;

}  // namespace

extern "C" __attribute__((visibility("default")))
int swcal_cellmix(int32_t kind, int32_t waves_per_cu, int32_t ncols, double *ms, double *cells) {
  if (!ms || !cells || kind < 0 || kind > 2 || waves_per_cu < 1 || waves_per_cu > 32 ||
      ncols < 1 || ncols > (1 << 20))
    return -1;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -3;
  const int grid = ncu * waves_per_cu;
  uint32_t *out = nullptr;
  if (hipMalloc(&out, (size_t)grid * 64 * sizeof(uint32_t)) != hipSuccess) return -2;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  int per_lane = 0;
  float t = 0.f;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = -3;
  for (int rep = 0; rc == 0 && rep < 2; ++rep) {  // the first launch warms up
    if (hipEventRecord(a, 0) != hipSuccess) { rc = -3; break; }
    if (kind == 0) {
      hipLaunchKernelGGL((k_cellmix<Cell16, kRows>), dim3(grid), dim3(64), 0, 0, out, ncols, 12345u,
                         Cell16{0x000c000cu, 0x00020002u});
      per_lane = Cell16::kCellsPerLane;
    } else if (kind == 1) {
      hipLaunchKernelGGL((k_cellmix<Cell32, kRows>), dim3(grid), dim3(64), 0, 0, out, ncols, 12345u,
                         Cell32{12u, 2u});
      per_lane = Cell32::kCellsPerLane;
    } else {
      hipLaunchKernelGGL((k_cellmix<Cell8, kRows>), dim3(grid), dim3(64), 0, 0, out, ncols, 12345u,
                         Cell8{0x0c0c0c0cu, 0x02020202u});
      per_lane = Cell8::kCellsPerLane;
    }
    if (hipGetLastError() != hipSuccess || hipEventRecord(b, 0) != hipSuccess ||
        hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess)
      rc = -3;
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(out);
  if (rc) return rc;
  *ms = t;
  *cells = (double)grid * 64 * per_lane * 2 /* chains */ * kRows * (double)ncols;
  return 0;
}
