// HIP kernels for Smith-Waterman database search on gfx950 (CDNA4).
//
// Recurrences (Section 2, Eqs. 1-3), Goe = gap_open + gap_extend, Ge = gap_extend:
//   H[i][j] = max{0, H[i-1][j-1] + SM(q_i, d_j), E[i][j], F[i][j]}
//   E[i][j] = max{H[i][j-1] - Goe, E[i][j-1] - Ge}
//   F[i][j] = max{H[i-1][j] - Goe, F[i-1][j] - Ge}
//
// All kernels keep E and F clamped at zero (E' = max(E, 0), F' = max(F, 0)), computed
// with unsigned saturating subtraction.  Because H >= 0, max(0, x, E, F) equals
// max(x, E', F'), and E'/F' obey the same recurrences with every intermediate clamped,
// so H (and the score) is unchanged while the explicit "max with 0" disappears.
//
// Kernels:
//   k_profile   query profiles (Section 4.3, QP): P[d][i] = SM(q_i, d), plus counters.
//   k_pack      length-sorted groups of 64 sequences, interleaved and padded (Section 4,
//               pre-processing: sort by length, group by lane count, pad with dummies).
//   k_inter16   inter-task DP (Sections 1 and 4.1) in packed int16 with saturation
//               (Section 4.2): one sequence per lane, two DP cells per 32-bit lane.
//   k_intra32   intra-task DP (Section 1), anti-diagonal, for very long sequences, for
//               every pair of a database too small to fill the GPU, and for the exact
//               recompute of saturated alignments (Section 4.2): int32, or two pairs
//               per wave in packed int16 with the same saturation rule.
#include "swmi_internal.h"

namespace swmi {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// v_pk_add_i16 with clamp: per-half signed saturating add.
__device__ __forceinline__ uint32_t pk_adds(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(
      __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}
// v_pk_sub_u16 with clamp: per-half unsigned saturating subtract (floors at 0).
__device__ __forceinline__ uint32_t pk_subu(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
      __builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}
// v_pk_max_i16: per-half signed max.
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(
      __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}
// v_sub_u32 with clamp.
__device__ __forceinline__ int32_t subu(int32_t a, int32_t b) {
  return (int32_t)__builtin_elementwise_sub_sat((uint32_t)a, (uint32_t)b);
}

// ------------------------------------------------------------------------ profiles
// Inter-task profile of query q: [nstrips][32 codes][2T rows] int16, so one strip's
// slice is a contiguous block.  Intra-task profile: [32 codes][mrows rows] int8 (every
// matrix entry and kPadScore fit: the boundary rejects |entries| > 127).
// Rows past the query end and codes outside the alphabet (including the padding code)
// score kPadScore.
__global__ void k_profile(ProfileArgs a) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < sizeof(Counters) / 4)
    reinterpret_cast<int32_t *>(a.ctr)[threadIdx.x] = 0;
  if (blockIdx.y == 0)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.nzero;
         e += (int64_t)gridDim.x * blockDim.x)
      a.zero[e] = 0;
  const int q = blockIdx.y;
  const QueryDesc d = a.queries[q];
  const uint8_t *qs = a.query + a.qoff[q];
  const int twoT = 2 * a.T;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // An empty query scores 0 against every sequence.  No DP kernel gets an item of it
  // (the intra-task lists skip it), so its whole row is written here, before any of them
  // runs on the stream.
  if (d.m == 0)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_seqs; e += stride)
      a.scores[d.out + e] = 0;
  const int64_t n16 = (int64_t)d.nstrips * kCodes * twoT;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n16; e += stride) {
    const int r = (int)(e % twoT);
    const int code = (int)((e / twoT) % kCodes);
    const int64_t i = (e / ((int64_t)twoT * kCodes)) * twoT + r;
    int v = kPadScore;
    if (i < d.m && code < a.alphabet) v = a.matrix[qs[i] * a.alphabet + code];
    a.qp16[d.qp16 + e] = (int16_t)v;
  }
  const int64_t n8 = (int64_t)kCodes * d.mrows;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n8; e += stride) {
    const int64_t i = e % d.mrows;
    const int code = (int)(e / d.mrows);
    int v = kPadScore;
    if (i < d.m && code < a.alphabet) v = a.matrix[qs[i] * a.alphabet + code];
    a.qp8[d.qp8 + e] = (int8_t)v;
  }
}

hipError_t launch_profile(const ProfileArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_profile, dim3(64, a.nqueries), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ packing
// One block per group.  Output dword (chunk c, lane l) holds residues 4c..4c+3 of the
// group's sequence l; columns past a sequence's end hold kPadCode.
__global__ void k_pack(PackArgs a) {
  const GroupDesc d = a.groups[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int sub = threadIdx.x >> 6;
  int64_t src = 0;
  int64_t len = 0;
  if (lane < d.count) {
    const int orig = a.perm[d.first + lane];
    src = a.offsets[orig];
    len = a.offsets[orig + 1] - src;
  }
  uint32_t *out = reinterpret_cast<uint32_t *>(a.packed + d.base);
  const int nchunks = d.ncols >> 2;
  for (int c = sub; c < nchunks; c += blockDim.x >> 6) {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t col = 4 * (int64_t)c + k;
      const uint32_t r = col < len ? a.raw[src + col] : (uint32_t)kPadCode;
      w |= r << (8 * k);
    }
    out[(int64_t)c * 64 + lane] = w;
  }
}

hipError_t launch_pack(const PackArgs &a, hipStream_t s) {
  if (a.ngroups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3(a.ngroups), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ inter-task
// Persistent kernel, one wave per workgroup.  A work item is (query, group); each lane
// aligns the query against one sequence of the group.  The query is cut into strips of
// 2T rows.  In every 32-bit register the low int16 half holds strip rows [0, T) at
// DB column c and the high half holds rows [T, 2T) of the same alignment at column
// c - 2, so the hand-off from the low rows to the high rows stays in the lane.  Columns
// are processed two at a time ("lead" c and "lag" c + 1, the lag one row behind the
// lead), which gives every wave two independent dependency chains.  Per strip, the
// bottom row's (H, F) of each column goes to a per-wave boundary buffer that the next
// strip reads back (layout [column][64 lanes] dwords: H low half, F high half).
//
// Saturation (Section 4.2): only H[i-1][j-1] + SM can exceed the int16 range, and the
// clamped add then pins H at 32767, so the running maximum equals 32767 exactly when
// the true score may be >= 32767.  Those alignments are appended to a list and
// recomputed in int32; every other int16 score is exact.

// (lo16 of a) | (lo16 of b) << 16
__device__ __forceinline__ uint32_t pack_lo(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x05040100u);
}
// (hi16 of a) | (hi16 of b) << 16
__device__ __forceinline__ uint32_t pack_hi(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x07060302u);
}
// (hi16 of a) | (lo16 of b) << 16
__device__ __forceinline__ uint32_t pack_hl(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x05040302u);
}

// One DP cell pair (both int16 halves) of Eqs. 1-3 with E and F clamped at zero:
// returns H; E becomes E of the next column and f becomes F of the next row.
__device__ __forceinline__ uint32_t cell16(uint32_t hd, uint32_t sm, uint32_t &E, uint32_t &f,
                                           uint32_t &vmax, uint32_t goe2, uint32_t ge2) {
  const uint32_t h = pk_max(pk_max(pk_adds(hd, sm), E), f);
  vmax = pk_max(vmax, h);
  const uint32_t t = pk_subu(h, goe2);
  E = pk_max(pk_subu(E, ge2), t);
  f = pk_max(pk_subu(f, ge2), t);
  return h;
}

// The strip loop of one (query, group) item of the one-query inter-task kernel (see
// k_inter16).  The caller fills the LDS profile slice of strip s (32 codes x 2T rows,
// code rows Inter16Lds<T>::RS bytes apart, low rows [0, T) then high rows [T, 2T)) in
// `stage(s)`, which runs between two barriers of the single-wave workgroup.  `res`
// points at the lane's first packed residue dword, `bnd` at its strip-boundary column 0.
// Returns the packed running maximum of H.
template <int T> struct Inter16Lds {
  static constexpr int RS = 4 * T + 16;  // LDS bytes per code row; RS/16 is odd (fewer conflicts)
  static constexpr int bytes = kCodes * RS;
};

template <int T, class Stage>
__device__ __forceinline__ uint32_t inter16_strips(uint8_t *lds, const uint32_t *res, int ncols,
                                                   uint32_t *bnd, int nstrips, uint32_t goe2,
                                                   uint32_t ge2, Stage &&stage) {
  static_assert(T % 8 == 0, "strip half-height must be a multiple of 8");
  constexpr int RS = Inter16Lds<T>::RS;
  const int nchunks = ncols >> 2;
  uint32_t vmaxA = 0, vmaxB = 0;
  for (int s = 0; s < nstrips; ++s) {
    __syncthreads();
    stage(s);
    __syncthreads();

    const bool first = (s == 0);
    const bool last = (s == nstrips - 1);
    uint32_t Hs[T], Es[T];
#pragma unroll
    for (int r = 0; r < T; ++r) { Hs[r] = 0; Es[r] = 0; }
    // low-half outputs of earlier columns, handed to the high half two columns later
    uint32_t hA = 0, fA = 0;   // lead of the previous pair (column c - 2)
    uint32_t hB = 0, fB = 0;   // lag of the previous pair (column c - 1)
    uint32_t hBB = 0;          // lag of the pair before (column c - 3)
    uint32_t hbnd_prev = 0;    // boundary H of column c - 1
    uint32_t rwp = 0x1f1f1f1fu;  // codes of the previous 4 columns (all padding)

    uint32_t rw = res[0];
    uint32_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    if (!first) { b0 = bnd[0]; b1 = bnd[64]; b2 = bnd[128]; b3 = bnd[192]; }

    for (int c = 0; c < nchunks; ++c) {
      uint32_t rwn = 0, n0 = 0, n1 = 0, n2 = 0, n3 = 0;
      if (c + 1 < nchunks) {
        rwn = res[(int64_t)(c + 1) * 64];
        if (!first) {
          const uint32_t *bp = bnd + (int64_t)(c + 1) * 256;
          n0 = bp[0]; n1 = bp[64]; n2 = bp[128]; n3 = bp[192];
        }
      }
      // the pair's codes (J, J + 1) are the low two bytes of cw, those of (J - 2, J - 1)
      // the low two bytes of pw; boundary words of (J, J + 1) are bJ, bJ1
      uint32_t cw = rw, pw = rwp >> 16;
      uint32_t bJ = b0, bJ1 = b1;
#pragma unroll 1
      for (int p = 0; p < 2; ++p) {
        const int J = c * 4 + 2 * p;  // lead column (low half); lag is J + 1
        const uint32_t dJ = cw & 0xffu;
        const uint32_t dJ1 = (cw >> 8) & 0xffu;
        const uint32_t dJm2 = pw & 0xffu;
        const uint32_t dJm1 = (pw >> 8) & 0xffu;
        const uint8_t *plA = lds + dJ * RS;               // lead low rows, column J
        const uint8_t *phA = lds + dJm2 * RS + 2 * T;     // lead high rows, column J - 2
        const uint8_t *plB = lds + dJ1 * RS;              // lag low rows, column J + 1
        const uint8_t *phB = lds + dJm1 * RS + 2 * T;     // lag high rows, column J - 1
        // row-0 inputs: low half from the boundary row, high half from the low rows
        uint32_t hdA = pack_lo(hbnd_prev, hBB);  // H(row-1, col-1)
        uint32_t fa = pack_hl(bJ, fA);           // F entering row 0
        uint32_t hdB = pack_lo(bJ, hA);
        uint32_t fb = pack_hl(bJ1, fB);
        // Row r of the lead column runs next to row r - 1 of the lag column: the lead
        // reads Hs[r-1] (H of column J - 1) just before the lag overwrites it with
        // column J + 1, so every row keeps one H and one E register.
        uint32_t ha = 0, hb = 0;
        uint32_t dA1 = hdB, dA2 = 0;  // lead H of rows r-1 and r-2 (lag diagonals)
        uint32_t smB_prev = 0;
#pragma unroll
        for (int r8 = 0; r8 < T; r8 += 8) {
          // 8 profile rows per stream: one 16-byte LDS read each
          const uint4 A1 = *reinterpret_cast<const uint4 *>(plA + 2 * r8);
          const uint4 A2 = *reinterpret_cast<const uint4 *>(phA + 2 * r8);
          const uint4 B1 = *reinterpret_cast<const uint4 *>(plB + 2 * r8);
          const uint4 B2 = *reinterpret_cast<const uint4 *>(phB + 2 * r8);
          const uint32_t a1[4] = {A1.x, A1.y, A1.z, A1.w}, a2[4] = {A2.x, A2.y, A2.z, A2.w};
          const uint32_t b1v[4] = {B1.x, B1.y, B1.z, B1.w}, b2v[4] = {B2.x, B2.y, B2.z, B2.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int r = r8 + q;
            const uint32_t smA = (q & 1) ? pack_hi(a1[q >> 1], a2[q >> 1])
                                         : pack_lo(a1[q >> 1], a2[q >> 1]);
            const uint32_t smB = (q & 1) ? pack_hi(b1v[q >> 1], b2v[q >> 1])
                                         : pack_lo(b1v[q >> 1], b2v[q >> 1]);
            // lead, row r
            const uint32_t h = cell16(r == 0 ? hdA : Hs[r - 1], smA, Es[r], fa, vmaxA,
                                      goe2, ge2);
            // lag, row r - 1 (its diagonal is the lead's H of row r - 2)
            if (r >= 1) Hs[r - 1] = cell16(dA2, smB_prev, Es[r - 1], fb, vmaxB, goe2, ge2);
            dA2 = dA1;
            dA1 = h;
            smB_prev = smB;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        ha = dA1;
        hb = cell16(dA2, smB_prev, Es[T - 1], fb, vmaxB, goe2, ge2);
        Hs[T - 1] = hb;
        // high halves finished columns J - 2 (lead) and J - 1 (lag): hand them down
        if (!last) {
          if (J >= 2) bnd[(int64_t)(J - 2) * 64] = pack_hi(ha, fa);
          if (J >= 1) bnd[(int64_t)(J - 1) * 64] = pack_hi(hb, fb);
        }
        hBB = hB;
        hA = ha; fA = fa;
        hB = hb; fB = fb;
        hbnd_prev = bJ1;
        pw = cw;
        cw >>= 16;
        bJ = b2;
        bJ1 = b3;
      }
      rwp = rw;
      rw = rwn; b0 = n0; b1 = n1; b2 = n2; b3 = n3;
    }
    // the last two columns are padding that the high half never reaches
    if (!last) {
      bnd[(int64_t)(ncols - 2) * 64] = 0u;
      bnd[(int64_t)(ncols - 1) * 64] = 0u;
    }
  }
  return pk_max(vmaxA, vmaxB);
}

template <int T, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_inter16(InterArgs a) {
  constexpr int RS = Inter16Lds<T>::RS;
  __shared__ __attribute__((aligned(16))) uint8_t lds[Inter16Lds<T>::bytes];
  const int lane = threadIdx.x;
  // The first big_waves waves have full-width boundary slots and take the widest items
  // [0, wide_items) first; every wave then takes the others in order from wide_items.
  const int wave = (int)blockIdx.x;
  const bool big = wave < a.big_waves;
  uint32_t *bnd = a.bnd + lane +
                  (big ? (int64_t)wave * a.bnd_slot_words
                       : (int64_t)a.big_waves * a.bnd_slot_words +
                             (int64_t)(wave - a.big_waves) * a.small_slot_words);
  const uint32_t goe2 = (uint32_t)a.goe * 0x10001u;
  const uint32_t ge2 = (uint32_t)a.ge * 0x10001u;
  __shared__ int s_item;
  bool wide_left = big && a.wide_items > 0;

  for (;;) {
    // claim the next item: lane 0 takes it, the (single-wave) workgroup barrier makes the
    // value visible to every lane and keeps the wave converged around the claim
    __syncthreads();
    if (lane == 0) {
      int it = -1;
      if (wide_left) {
        it = atomicAdd(&a.ctr->inter_wide, 1);
        if (it >= a.wide_items) it = -1;
      }
      if (it < 0) it = a.wide_items + atomicAdd(&a.ctr->inter_next, 1);
      s_item = it;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= a.nitems) break;
    wide_left = wide_left && item < a.wide_items;
    const int g = a.ngroups - 1 - item / a.nqueries;  // longest groups first
    const int qi = a.qorder[item % a.nqueries];       // then longest queries first
    const GroupDesc gd = a.groups[g];
    const QueryDesc qd = a.queries[qi];
    const int16_t *qp = a.qp16 + qd.qp16;
    const uint32_t *res = reinterpret_cast<const uint32_t *>(a.packed + gd.base) + lane;
    // each strip's profile slice (32 codes x 2T rows) is copied into LDS
    auto stage = [&](int s) {
      const uint4 *src = reinterpret_cast<const uint4 *>(qp + (int64_t)s * kCodes * 2 * T);
      constexpr int PER_CODE = T / 4;  // 16-byte pieces per code row
      constexpr int PIECES = kCodes * PER_CODE;
#pragma unroll
      for (int c = lane; c < PIECES; c += 64) {
        const int code = c / PER_CODE, k = c - code * PER_CODE;
        *reinterpret_cast<uint4 *>(lds + code * RS + k * 16) = src[c];
      }
    };
    // the widest groups are claimed first and each is one wave's work for most of the
    // launch: they run at raised priority on their SIMDs, so they end with the rest
    const bool prio = gd.ncols >= a.prio_cols;
    if (prio) __builtin_amdgcn_s_setprio(2);
    const uint32_t vmax = inter16_strips<T>(lds, res, gd.ncols, bnd, qd.nstrips, goe2, ge2, stage);
    if (prio) __builtin_amdgcn_s_setprio(0);
    const int lo = (int)(int16_t)(vmax & 0xffffu);
    const int hi = (int)(int16_t)(vmax >> 16);
    const int sc = lo > hi ? lo : hi;
    if (lane < gd.count) {
      const int p = gd.first + lane;
      const int orig = a.perm[p];
      if (sc >= kSat16 || a.recompute_all) {
        const int k = atomicAdd(&a.ctr->flagged, 1);
        if (k < a.flag_cap) {
          PairItem it;
          it.base = gd.base + 4 * lane;
          it.cstride = 256;
          it.len = a.lens[p];
          it.out = orig;
          it.query = qi;
          it.band0 = 0;
          it.band1 = qd.nbands;
          it.xin = it.xout = -1;
          it.prog_in = it.prog_out = -1;
          it.segment = 0;
          it.nsegments = 1;
          a.flagged[k] = it;
        } else {
          a.scores[qd.out + orig] = kSat16;  // the list is full: k_rescan finds the mark
        }
      } else {
        a.scores[qd.out + orig] = sc;
      }
    }
  }
}

// Minimum waves per SIMD requested from the register allocator for each strip height.
template <int T> struct Inter16Occ { static constexpr int wpe = T <= 8 ? 6 : (T <= 16 ? 4 : (T <= 24 ? 3 : 2)); };

template <int T>
static hipError_t launch_inter16_t(const InterArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_inter16<T, Inter16Occ<T>::wpe>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

bool inter16_supported(int T) { return T == 8 || T == 16 || T == 24 || T == 32 || T == 40; }

int inter16_max_blocks_per_cu(int T) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (T) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16<8, Inter16Occ<8>::wpe>, 64, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16<16, Inter16Occ<16>::wpe>, 64, 0); break;
    case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16<24, Inter16Occ<24>::wpe>, 64, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16<32, Inter16Occ<32>::wpe>, 64, 0); break;
    case 40: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16<40, Inter16Occ<40>::wpe>, 64, 0); break;
    default: break;
  }
  return e == hipSuccess ? n : 0;
}

hipError_t launch_inter16(const InterArgs &a, int T, int grid, hipStream_t s) {
  if (a.nitems == 0 || grid == 0) return hipSuccess;
  switch (T) {
    case 8: return launch_inter16_t<8>(a, grid, s);
    case 16: return launch_inter16_t<16>(a, grid, s);
    case 24: return launch_inter16_t<24>(a, grid, s);
    case 32: return launch_inter16_t<32>(a, grid, s);
    case 40: return launch_inter16_t<40>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------ intra-task
// One (query, sequence) pair is swept by NW cooperating waves, int32.  The query is cut
// into bands of 64*R rows; lane l of the wave that owns band b holds rows
// b*64R + l*R .. + R-1 and, at step s, works on DB column s - l (an anti-diagonal
// sweep).  After every step the bottom row's H and the F entering the next lane's
// first row move one lane down with a DPP wave shift; lane 0 takes them from the
// boundary row of the band above instead, and lane 63 writes its bottom row for the
// band below.  Bands go to the NW waves round-robin and run as a pipeline: band b starts
// kIntraLag chunks (of 64 steps) after band b-1, with a workgroup barrier after every
// chunk, so every boundary value a band reads was written at least one barrier earlier.
// With NW = 1 a single wave runs the bands in order and needs no barrier.  Columns
// outside [0, n) carry the padding code and a zero boundary, which leaves every
// in-range cell unchanged and never raises the maximum.
__device__ __forceinline__ int wave_shr1(int src, int lane0_value) {
  // lanes 1..63 receive src from lane - 1; lane 0 keeps lane0_value
  return __builtin_amdgcn_update_dpp(lane0_value, src, 0x138, 0xf, 0xf, false);
}

// What one lane carries while its wave sweeps a band: its R rows of H and E, the bottom
// row's H and F (passed one lane down after every step), the H that becomes the next
// step's diagonal for its first row, the band-top values and residues of the current
// 64-column chunk (lane l holds column 64k + l), and the profile rows of the next
// IntraBuf<R>::n steps, already requested (cfar is the residue code of the last of them).
// One lane's R int8 profile rows for one code (R = 2, 4, 8 or 16: one 2-, 4-, 8- or
// 16-byte load).
// Profile-row buffers per lane (prefetch distance + 1): 8 (for the latency-bound long
// pairs of the 8-row launch the deeper prefetch was about 5% faster than 4); the two-pair
// path at R = 16, which holds two sets, keeps kIntraBuf (8 measured no faster there).
template <int R> struct IntraBuf { static constexpr int n = 8; };
template <int R> struct IntraBuf16 { static constexpr int n = R <= 8 ? 8 : kIntraBuf; };

template <int R> struct RowBuf;
template <> struct RowBuf<2> {
  uint16_t v;
  __device__ uint32_t word(int) const { return v; }
};
template <> struct RowBuf<4> {
  uint32_t v;
  __device__ uint32_t word(int) const { return v; }
};
template <> struct RowBuf<8> {
  uint2 v;
  __device__ uint32_t word(int i) const { return i == 0 ? v.x : v.y; }
};
template <> struct RowBuf<16> {
  uint4 v;
  __device__ uint32_t word(int i) const {
    return i < 2 ? (i == 0 ? v.x : v.y) : (i == 2 ? v.z : v.w);
  }
};

template <int R>
struct BandLane {
  int32_t H[R], E[R];
  int32_t hbot, fbot, hdiag, cfar;
  int2 tq;
  int rq;
  RowBuf<R> P[IntraBuf<R>::n];
};

// Profile rows (int8) of one lane.  The band's profile starts at `pbase` (the same for
// the whole wave), code c's rows of the band are c * pstride bytes further and lane l's R
// rows l * R bytes further still.  The code travels down the lanes already multiplied by
// pstride, so a request is one add and one load with a wave-uniform base.
template <int R>
__device__ __forceinline__ void load_rows(RowBuf<R> &dst, const uint8_t *pbase, uint32_t off) {
  dst.v = *reinterpret_cast<const decltype(dst.v) *>(pbase + off);
}

// A wave-uniform 64-bit value held in scalar registers (the profile loads take the band's
// profile address as their scalar base).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Residue code of column `col` of a sequence (kPadCode outside [0, n)), multiplied by
// the profile's code stride.
__device__ __forceinline__ int code_off(const uint8_t *resbase, int cs, int col, int n,
                                        uint32_t pstride) {
  const int c = col < n ? (int)resbase[(col >> 2) * (int64_t)cs + (col & 3)] : kPadCode;
  return c * (int)pstride;
}

// Start a band: zero state, load the first chunk's band-top values and residues, and
// request the profile rows of steps 0 .. IntraBuf<R>::n - 2.  The code lane l needs at step s
// is that of column s - l: its left neighbour's code of step s - 1 (lane 0 takes column
// s's residue), so codes run ahead as a chain of wave shifts (as offsets: code * pstride).
template <int R>
__device__ __forceinline__ void band_start(BandLane<R> &L, int lane, int n, const int2 *top,
                                           bool has_top, const uint8_t *resbase, int cs,
                                           const uint8_t *pbase, uint32_t lane_off,
                                           uint32_t pstride) {
#pragma unroll
  for (int r = 0; r < R; ++r) { L.H[r] = 0; L.E[r] = 0; }
  L.hbot = 0; L.fbot = 0; L.hdiag = 0; L.cfar = kPadCode * (int)pstride;
  L.tq = (has_top && lane < n) ? top[lane] : make_int2(0, 0);
  L.rq = code_off(resbase, cs, lane, n, pstride);
#pragma unroll
  for (int t = 0; t + 1 < IntraBuf<R>::n; ++t) {
    L.cfar = wave_shr1(L.cfar, __builtin_amdgcn_readlane(L.rq, t));
    load_rows(L.P[t], pbase, (uint32_t)L.cfar + lane_off);
  }
}

// Chunk k (steps 64k .. 64k + 63) of a band sweep.  Raises vmax to the largest H
// computed.  Step s computes with the rows in buffer s % NB (NB = IntraBuf<R>::n) and
// requests those of step s + NB - 1 into the buffer step s - 1 used, so each request has
// NB - 1 steps to arrive; steps go in groups of NB, so no buffer is ever
// copied.  The last group's requests reach into the next chunk's residues, so it is
// unrolled apart from the others and the loop over groups has no branch.  Each row's
// diagonal sum H(i-1, j-1) + SM is formed before the row above is overwritten, which
// lets H stay in place from step to step.  Lane 63 (when `store_bot`) stores the bottom
// row's (H, F) of column s - 63 at every step.
//
// The 64 steps themselves are sweep_chunk: `bchunk` is where lane 63 stores step i's
// bottom row (bchunk[i]), rq_next the next chunk's code offsets.  With WRAP (chained
// bands, below) the lane that enters a new band at step i (lane i - w0) first clears its
// rows' H and E and its diagonal: the band's left boundary.
template <int R, bool WRAP>
__device__ __forceinline__ void sweep_chunk(BandLane<R> &L, int32_t &vmax, const IntraArgs &a,
                                            int lane, int2 *bchunk, bool store_bot,
                                            int rq_next, const uint8_t *pbase,
                                            uint32_t lane_off, int w0) {
  constexpr int NB = IntraBuf<R>::n;
  constexpr int D = NB - 1;  // prefetch distance in steps
  static_assert(64 % NB == 0 && NB >= 2, "a chunk must hold whole groups of steps");

  auto step = [&](const int i, const int cin, const RowBuf<R> &P, RowBuf<R> &Pfar) {
    if (WRAP && (unsigned)(i - w0) < 64u) {  // (uniform)
      const int keep = lane == i - w0 ? 0 : -1;
#pragma unroll
      for (int r = 0; r < R; ++r) { L.H[r] &= keep; L.E[r] &= keep; }
      L.hdiag &= keep;
    }
    // request the rows of step s + D
    L.cfar = wave_shr1(L.cfar, cin);
    load_rows(Pfar, pbase, (uint32_t)L.cfar + lane_off);
    const int hup = wave_shr1(L.hbot, __builtin_amdgcn_readlane(L.tq.x, i));
    int f = wave_shr1(L.fbot, __builtin_amdgcn_readlane(L.tq.y, i));
    auto sm = [&](int r) {  // row r's score, sign-extended from its byte
      return (int32_t)(int8_t)(P.word(r >> 2) >> (8 * (r & 3)));
    };
    int x = L.hdiag + sm(0);
    L.hdiag = hup;
    int h = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int xn = r + 1 < R ? L.H[r] + sm(r + 1) : 0;
      h = max(max(x, L.E[r]), f);                   // Eq. 1 (E, F clamped >= 0)
      vmax = max(vmax, h);
      const int t = subu(h, a.goe);
      L.E[r] = max(subu(L.E[r], a.ge), t);          // Eq. 2
      f = max(subu(f, a.ge), t);                    // Eq. 3
      L.H[r] = h;
      x = xn;
    }
    L.hbot = h;
    L.fbot = f;
    if (store_bot) bchunk[i] = make_int2(h, f);
    // The running maximum is brought up to date at every step of a chained sweep and at
    // R = 16.  Left free, the compiler defers the maxima of a whole group of steps to the
    // group's end, which keeps every H of the group live (about 80 more VGPRs at R = 16)
    // and leaves no room to clear a lane's rows in place.  At R = 2 to 8 in a band sweep
    // the deferred form is kept: there the registers are not short, and pinning made the
    // latency-bound searches (a wave alone on its SIMD) 2-6% slower.  (An empty asm
    // statement without side effects: no instruction is emitted.)
    if (WRAP || R >= 16) asm("" : "+v"(vmax));
  };
#pragma unroll 1
  for (int i = 0; i < 64 - NB; i += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u)
      step(i + u, __builtin_amdgcn_readlane(L.rq, i + u + D), L.P[u], L.P[(u + NB - 1) % NB]);
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    step(64 - NB + u,
         u == 0 ? __builtin_amdgcn_readlane(L.rq, 63) : __builtin_amdgcn_readlane(rq_next, u - 1),
         L.P[u], L.P[(u + NB - 1) % NB]);
}

template <int R>
__device__ __forceinline__ void band_chunk(BandLane<R> &L, int32_t &vmax, const IntraArgs &a,
                                           int lane, int k, int n, const int2 *top,
                                           bool has_top, int2 *bot, bool store_bot,
                                           const uint8_t *resbase, int cs,
                                           const uint8_t *pbase, uint32_t lane_off,
                                           uint32_t pstride) {
  const int col_next = 64 * (k + 1) + lane;
  const int2 tq_next = (has_top && col_next < n) ? top[col_next] : make_int2(0, 0);
  const int rq_next = code_off(resbase, cs, col_next, n, pstride);
  sweep_chunk<R, false>(L, vmax, a, lane, bot + (64 * k - 63), store_bot, rq_next, pbase,
                        lane_off, 0);
  L.tq = tq_next;
  L.rq = rq_next;
}

// ---- Two pairs per wave in packed int16 (Section 4.2: narrow range first).  The low
// half of every register belongs to sequence A, the high half to sequence B; both run
// against the same query rows, so one packed instruction advances two cells.  Values
// stay in [0, 32767] exactly as in the inter-task kernel (saturating add, E and F
// clamped at zero by unsigned saturating subtraction), a half whose maximum reaches
// 32767 is recomputed in int32, and every other half is exact.
template <int R>
struct BandLane16 {
  uint32_t H[R], E[R];
  uint32_t hbot, fbot, hdiag;
  int cfarA, cfarB;
  int2 tq;  // band-top (H, F), both halves packed
  int rqA, rqB;
  RowBuf<R> PA[IntraBuf16<R>::n], PB[IntraBuf16<R>::n];
};

// Row r's scores for A (low half) and B (high half), sign-extended from their int8
// bytes by one byte permute: the permute can copy a sign only from bytes 1 and 3 of
// each word, so rows at even byte positions are first moved up by a byte.
template <int R>
__device__ __forceinline__ uint32_t pair_score(const RowBuf<R> &A, const RowBuf<R> &B, int r) {
  const int j = r & 3;
  uint32_t a = A.word(r >> 2), b = B.word(r >> 2);
  if ((j & 1) == 0) { a <<= 8; b <<= 8; }
  const uint32_t k = (uint32_t)(j | 1);  // byte of A (1 or 3); B's is k + 4
  const uint32_t sel = k | ((k == 1 ? 8u : 9u) << 8) | ((k + 4) << 16) | ((k == 1 ? 10u : 11u) << 24);
  return __builtin_amdgcn_perm(b, a, sel);
}

template <int R>
__device__ __forceinline__ void band_start16(BandLane16<R> &L, int lane, int nA, int nB,
                                             const int2 *top, bool has_top,
                                             const uint8_t *resA, int csA, const uint8_t *resB,
                                             int csB, const uint8_t *pbase, uint32_t lane_off,
                                             uint32_t pstride) {
#pragma unroll
  for (int r = 0; r < R; ++r) { L.H[r] = 0; L.E[r] = 0; }
  L.hbot = 0; L.fbot = 0; L.hdiag = 0;
  L.cfarA = L.cfarB = kPadCode * (int)pstride;
  L.tq = (has_top && lane < nA) ? top[lane] : make_int2(0, 0);
  L.rqA = code_off(resA, csA, lane, nA, pstride);
  L.rqB = code_off(resB, csB, lane, nB, pstride);
#pragma unroll
  for (int t = 0; t + 1 < IntraBuf16<R>::n; ++t) {
    L.cfarA = wave_shr1(L.cfarA, __builtin_amdgcn_readlane(L.rqA, t));
    L.cfarB = wave_shr1(L.cfarB, __builtin_amdgcn_readlane(L.rqB, t));
    load_rows(L.PA[t], pbase, (uint32_t)L.cfarA + lane_off);
    load_rows(L.PB[t], pbase, (uint32_t)L.cfarB + lane_off);
  }
}

// Chunk k of a band sweep for both pairs (nA >= nB; B's columns past nB carry the
// padding code).  Same schedule as band_chunk.
template <int R, bool WRAP>
__device__ __forceinline__ void sweep_chunk16(BandLane16<R> &L, uint32_t &vmax, uint32_t goe2,
                                              uint32_t ge2, int lane, int2 *bchunk,
                                              bool store_bot, int rqA_next, int rqB_next,
                                              const uint8_t *pbase, uint32_t lane_off,
                                              int w0) {
  constexpr int NB = IntraBuf16<R>::n;
  constexpr int D = NB - 1;
  static_assert(64 % NB == 0 && NB >= 2, "a chunk must hold whole groups of steps");

  auto step = [&](const int i, const int cinA, const int cinB, const RowBuf<R> &PA,
                  const RowBuf<R> &PB, RowBuf<R> &PAfar, RowBuf<R> &PBfar) {
    if (WRAP && (unsigned)(i - w0) < 64u) {  // (uniform)
      const int keep = lane == i - w0 ? 0 : -1;
#pragma unroll
      for (int r = 0; r < R; ++r) { L.H[r] &= keep; L.E[r] &= keep; }
      L.hdiag &= keep;
    }
    L.cfarA = wave_shr1(L.cfarA, cinA);
    L.cfarB = wave_shr1(L.cfarB, cinB);
    load_rows(PAfar, pbase, (uint32_t)L.cfarA + lane_off);
    load_rows(PBfar, pbase, (uint32_t)L.cfarB + lane_off);
    const uint32_t hup = (uint32_t)wave_shr1((int)L.hbot, __builtin_amdgcn_readlane(L.tq.x, i));
    uint32_t f = (uint32_t)wave_shr1((int)L.fbot, __builtin_amdgcn_readlane(L.tq.y, i));
    uint32_t x = pk_adds(L.hdiag, pair_score<R>(PA, PB, 0));
    L.hdiag = hup;
    uint32_t h = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t xn = r + 1 < R ? pk_adds(L.H[r], pair_score<R>(PA, PB, r + 1)) : 0u;
      h = pk_max(pk_max(x, L.E[r]), f);             // Eq. 1 (E, F clamped >= 0)
      vmax = pk_max(vmax, h);
      const uint32_t t = pk_subu(h, goe2);
      L.E[r] = pk_max(pk_subu(L.E[r], ge2), t);     // Eq. 2
      f = pk_max(pk_subu(f, ge2), t);               // Eq. 3
      L.H[r] = h;
      x = xn;
    }
    L.hbot = h;
    L.fbot = f;
    if (store_bot) bchunk[i] = make_int2((int)h, (int)f);
    asm("" : "+v"(vmax));  // (as in sweep_chunk)
  };
#pragma unroll 1
  for (int i = 0; i < 64 - NB; i += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u)
      step(i + u, __builtin_amdgcn_readlane(L.rqA, i + u + D),
           __builtin_amdgcn_readlane(L.rqB, i + u + D), L.PA[u], L.PB[u],
           L.PA[(u + NB - 1) % NB], L.PB[(u + NB - 1) % NB]);
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    step(64 - NB + u,
         u == 0 ? __builtin_amdgcn_readlane(L.rqA, 63) : __builtin_amdgcn_readlane(rqA_next, u - 1),
         u == 0 ? __builtin_amdgcn_readlane(L.rqB, 63) : __builtin_amdgcn_readlane(rqB_next, u - 1),
         L.PA[u], L.PB[u], L.PA[(u + NB - 1) % NB], L.PB[(u + NB - 1) % NB]);
}

template <int R>
__device__ __forceinline__ void band_chunk16(BandLane16<R> &L, uint32_t &vmax, uint32_t goe2,
                                             uint32_t ge2, int lane, int k, int nA, int nB,
                                             const int2 *top, bool has_top, int2 *bot,
                                             bool store_bot, const uint8_t *resA, int csA,
                                             const uint8_t *resB, int csB,
                                             const uint8_t *pbase, uint32_t lane_off,
                                             uint32_t pstride) {
  const int col_next = 64 * (k + 1) + lane;
  const int2 tq_next = (has_top && col_next < nA) ? top[col_next] : make_int2(0, 0);
  const int rqA_next = code_off(resA, csA, col_next, nA, pstride);
  const int rqB_next = code_off(resB, csB, col_next, nB, pstride);
  sweep_chunk16<R, false>(L, vmax, goe2, ge2, lane, bot + (64 * k - 63), store_bot, rqA_next,
                          rqB_next, pbase, lane_off, 0);
  L.tq = tq_next;
  L.rqA = rqA_next;
  L.rqB = rqB_next;
}

// ---- Chained bands.  Swept one after another, the bands of a pair each pay the wave's
// fill and drain: 63 steps in which some lanes lie outside [0, n), plus the rounding up
// to whole chunks; on sequences of a few hundred residues that is a fifth of the steps.
// A single wave (no segment boundary) can instead run a pair's nb bands back to back as
// one stream of nb * n steps: lane 0 takes column j of band b at step b * n + j and lane
// l the same column l steps later, so at a band boundary the upper lanes finish the old
// band while the lower ones start the new one.  A lane entering band b >= 1 clears its
// rows' H and E and its diagonal at that step (the band's left boundary); nothing else
// changes, since its first row's H and F from above come from the lane above, already in
// the new band, or (lane 0) from the band above's bottom row.  The code offsets carry the
// band (code * pstride + b * 64R), so every profile request follows the band of the step
// it is for.  Bottom rows go to one linear buffer, buf[b * n + j] for band b, column j,
// which lane 63 writes at step b * n + j + 63; band b + 1's lane 0 reads it a chunk
// ahead, at step (b + 1) * n + j - 127 or later, which comes after the write in program
// order when n >= 191 (kChainMinLen).  With n >= 64 at most one lane enters a band per
// step, and the 64 steps in which lanes do fall in one chunk or two consecutive ones.
constexpr int kChainMinLen = 192;

struct ChainPos {
  int b, j;  // band and column lane 0 works on at one of the chunk's steps
};

__device__ __forceinline__ ChainPos chain_next(ChainPos p, int n) {
  p.j += 64;
  if (p.j >= n) { p.j -= n; p.b += 1; }
  return p;
}

// Code offset of position p: the residue (padding past len, and past the last band) times
// pstride, plus the band's rows.
__device__ __forceinline__ int chain_code(const uint8_t *res, int cs, ChainPos p, int len,
                                          int nb, uint32_t pstride, int band_bytes) {
  if (p.b >= nb) return kPadCode * (int)pstride;
  return code_off(res, cs, p.j, len, pstride) + p.b * band_bytes;
}

// Top-row input of position p: the bottom row of the band above (zero for band 0 and
// past the last band).
__device__ __forceinline__ int2 chain_top(const int2 *buf, ChainPos p, int n, int nb) {
  return (p.b >= 1 && p.b < nb) ? buf[(p.b - 1) * n + p.j] : make_int2(0, 0);
}

// The step within chunk (lane 0 at position p0) at which lane 0 enters a band >= 1, so
// that lane l enters it at step w0 + l; 64 if no lane enters a band in this chunk.
__device__ __forceinline__ int chain_window(ChainPos p0, int n) {
  if (p0.b >= 1 && p0.j < 64) return -p0.j;
  if (n - p0.j < 64) return n - p0.j;
  return 64;
}

// Whether a narrow item runs as chained bands: no segment boundary, two bands or more,
// n >= kChainMinLen, and buf (kBndLead + nb * n + 63 entries) fits the wave's ring.
__device__ __forceinline__ bool chain_fits(const IntraArgs &a, const PairItem &pi) {
  const int nb = pi.band1 - pi.band0;
  return a.chain && pi.xin < 0 && pi.xout < 0 && nb >= 2 && pi.len >= kChainMinLen &&
         (int64_t)kBndLead + (int64_t)nb * pi.len + 64 <= 2 * (int64_t)a.bnd_stride;
}

template <int R>
__device__ int32_t intra_chain(const IntraArgs &a, const PairItem &pi, const QueryDesc &qd,
                               int2 *ring) {
  const int lane = threadIdx.x & 63;
  const int n = pi.len, nb = pi.band1 - pi.band0;
  const int nch = (nb * n + 63 + 63) / 64;
  int2 *buf = ring + kBndLead;
  const uint8_t *resbase = a.packed + pi.base;
  const int cs = pi.cstride;
  const uint32_t pstride = (uint32_t)qd.mrows;
  const uint32_t lane_off = (uint32_t)(lane * R);
  const uint8_t *pbase = reinterpret_cast<const uint8_t *>(a.qp8) +
                         uniform64(qd.qp8 + (int64_t)pi.band0 * 64 * R);
  int32_t vmax = 0;
  BandLane<R> L;
  band_start(L, lane, n, nullptr, false, resbase, cs, pbase, lane_off, pstride);
  ChainPos cp{0, lane};
  for (int k = 0; k < nch; ++k) {
    const ChainPos p0{__builtin_amdgcn_readfirstlane(cp.b), __builtin_amdgcn_readfirstlane(cp.j)};
    const int w0 = chain_window(p0, n);
    const ChainPos nx = chain_next(cp, n);
    const int2 tq_next = chain_top(buf, nx, n, nb);
    const int rq_next = chain_code(resbase, cs, nx, n, nb, pstride, 64 * R);
    int2 *bchunk = buf + (64 * k - 63);
    sweep_chunk<R, true>(L, vmax, a, lane, bchunk, lane == 63, rq_next, pbase, lane_off, w0);
    L.tq = tq_next;
    L.rq = rq_next;
    cp = nx;
  }
  return vmax;
}

// Chained bands of a two-pair item (nA >= nB: the stream's period is nA, B's columns
// past nB carry the padding code).
template <int R>
__device__ uint32_t intra_chain16(const IntraArgs &a, const PairItem &pa, const PairItem &pb,
                                  const QueryDesc &qd, int2 *ring) {
  const int lane = threadIdx.x & 63;
  const int nA = pa.len, nB = pb.len, nb = pa.band1 - pa.band0;
  const int nch = (nb * nA + 63 + 63) / 64;
  int2 *buf = ring + kBndLead;
  const uint8_t *resA = a.packed + pa.base, *resB = a.packed + pb.base;
  const int csA = pa.cstride, csB = pb.cstride;
  const uint32_t pstride = (uint32_t)qd.mrows;
  const uint32_t goe2 = (uint32_t)a.goe * 0x10001u, ge2 = (uint32_t)a.ge * 0x10001u;
  const uint32_t lane_off = (uint32_t)(lane * R);
  const uint8_t *pbase = reinterpret_cast<const uint8_t *>(a.qp8) +
                         uniform64(qd.qp8 + (int64_t)pa.band0 * 64 * R);
  uint32_t vmax = 0;
  BandLane16<R> L;
  band_start16(L, lane, nA, nB, nullptr, false, resA, csA, resB, csB, pbase, lane_off, pstride);
  ChainPos cp{0, lane};
  for (int k = 0; k < nch; ++k) {
    const ChainPos p0{__builtin_amdgcn_readfirstlane(cp.b), __builtin_amdgcn_readfirstlane(cp.j)};
    const int w0 = chain_window(p0, nA);
    const ChainPos nx = chain_next(cp, nA);
    const int2 tq_next = chain_top(buf, nx, nA, nb);
    const int rqA_next = chain_code(resA, csA, nx, nA, nb, pstride, 64 * R);
    const int rqB_next = chain_code(resB, csB, nx, nB, nb, pstride, 64 * R);
    int2 *bchunk = buf + (64 * k - 63);
    sweep_chunk16<R, true>(L, vmax, goe2, ge2, lane, bchunk, lane == 63, rqA_next, rqB_next,
                           pbase, lane_off, w0);
    L.tq = tq_next;
    L.rqA = rqA_next;
    L.rqB = rqB_next;
    cp = nx;
  }
  return vmax;
}

// Segments of a split pair hand the bottom row of their last band to the next segment
// through a global buffer, column by column, with a progress counter.  The waiting side
// polls relaxed and then takes one acquire fence (an acquire load per poll would
// invalidate the cache on every iteration); the wait is bounded: after a.spin_limit polls,
// or once any wait has given up, the error flag is set and the kernel runs to its end with
// whatever the buffer holds.
__device__ __forceinline__ void wait_columns(const IntraArgs &a, int prog, int need) {
  int polls = 0;
  while (__hip_atomic_load(a.xprog + prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    __builtin_amdgcn_s_sleep(4);
    if (++polls > a.spin_limit) {
      __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Columns 0 .. done - 1 of a segment's bottom row are written (every lane stores the same
// count, with release order).
__device__ __forceinline__ void publish_columns(const IntraArgs &a, int prog, int done) {
  __hip_atomic_store(a.xprog + prog, done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Segments of a split pair chain their maxima: each waits (bounded, as above) for the
// previous segment's "finished" flag and takes the maximum so far; the last segment writes
// the score.  Waits point only to earlier segments.  One thread of the workgroup.
__device__ __forceinline__ int32_t wait_max(const IntraArgs &a, int prog) {
  int polls = 0;
  while (__hip_atomic_load(a.xfin + prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    __builtin_amdgcn_s_sleep(4);
    if (++polls > a.spin_limit) {
      __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return __hip_atomic_load(a.xmax + prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void pass_max(const IntraArgs &a, int prog, int32_t m) {
  __hip_atomic_store(a.xmax + prog, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(a.xfin + prog, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Both pairs of a two-pair item swept by NW waves (the band pipeline of intra_pair),
// possibly one segment of a split item: the first band of a later segment reads the
// previous segment's bottom row (both halves packed) and the last band of an earlier one
// writes its own, as in intra_pair.  Returns this lane's packed running maximum.
template <int R, int NW>
__device__ uint32_t intra_pair16(const IntraArgs &a, const PairItem &pa, const PairItem &pb,
                                 const QueryDesc &qd, int w, int2 *ring) {
  const int lane = threadIdx.x & 63;
  const int nA = pa.len, nB = pb.len;  // nA >= nB
  const int nb = pa.band1 - pa.band0;
  uint32_t vmax = 0;
  if (nA <= 0 || nb <= 0) return 0;
  const int nc = (nA + 63 + 63) / 64;
  const int nce = nc > kIntraLag * NW ? nc : kIntraLag * NW;
  const int lastb = nb - 1;
  const int rounds = (lastb / NW) * nce + kIntraLag * (lastb % NW) + nc;
  const uint8_t *resA = a.packed + pa.base, *resB = a.packed + pb.base;
  const int csA = pa.cstride, csB = pb.cstride;
  const uint32_t pstride = (uint32_t)qd.mrows;
  const uint32_t goe2 = (uint32_t)a.goe * 0x10001u, ge2 = (uint32_t)a.ge * 0x10001u;
  const uint32_t lane_off = (uint32_t)(lane * R);

  int bl = w;
  BandLane16<R> L;
  for (int rd = 0; rd < rounds; ++rd) {
    if (bl < nb) {
      const int st = (bl / NW) * nce + kIntraLag * (bl % NW);
      if (rd >= st && rd < st + nc) {
        const int k = rd - st;
        const int b = pa.band0 + bl;
        const bool ext_top = bl == 0 && pa.xin >= 0;
        const bool ext_bot = bl == nb - 1 && pa.xout >= 0;
        const int2 *top = (ext_top ? a.xbnd + pa.xin
                                   : ring + (int64_t)((bl + NW) % (NW + 1)) * a.bnd_stride) +
                          kBndLead;
        int2 *bot = (ext_bot ? a.xbnd + pa.xout
                             : ring + (int64_t)(bl % (NW + 1)) * a.bnd_stride) + kBndLead;
        const bool has_top = bl > 0 || ext_top, has_bot = bl < nb - 1 || ext_bot;
        // the columns this chunk and the next read
        if (ext_top) wait_columns(a, pa.prog_in, min(nA, 64 * (k + 2)));
        const uint8_t *pbase = reinterpret_cast<const uint8_t *>(a.qp8) +
                               uniform64(qd.qp8 + (int64_t)b * 64 * R);
        if (k == 0)
          band_start16(L, lane, nA, nB, top, has_top, resA, csA, resB, csB, pbase, lane_off,
                       pstride);
        band_chunk16(L, vmax, goe2, ge2, lane, k, nA, nB, top, has_top, bot,
                     has_bot && lane == 63, resA, csA, resB, csB, pbase, lane_off, pstride);
        if (ext_bot) publish_columns(a, pa.prog_out, k == nc - 1 ? nA : min(nA, 64 * k + 1));
        if (k == nc - 1) bl += NW;
      }
    }
    if (NW > 1) __syncthreads();
  }
  return vmax;
}

// Score of one half of a two-pair item: written, or (if it may have saturated) the pair
// is appended to the int32 recompute list.  Called by all lanes of a wave with the same
// score (lane 0 claims the list slot, every lane stores the same item) or by lane 0 of a
// workgroup alone.
__device__ __forceinline__ void finish_half(const IntraArgs &a, const PairItem &p,
                                            const QueryDesc &qd, int score) {
  const int lane = threadIdx.x & 63;
  if (score >= kSat16) {
    PairItem it = p;
    it.band0 = 0;
    it.band1 = qd.nbands;  // the recompute runs with 16 rows per lane
    it.xin = it.xout = -1;
    it.prog_in = it.prog_out = -1;
    it.segment = 0;
    it.nsegments = 1;
    const int k = __builtin_amdgcn_readfirstlane(atomicAdd(a.flag_count, lane == 0 ? 1 : 0));
    if (k < a.flag_cap)
      a.flagged[k] = it;
    else
      a.scores[qd.out + p.out] = kSat16;  // the list is full: k_rescan finds the mark
  } else {
    a.scores[qd.out + p.out] = score;
  }
}

__device__ __forceinline__ uint32_t wave_pk_max(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = pk_max(v, (uint32_t)__shfl_xor((int)v, off));
  return v;
}

// Returns this lane's running maximum of H over the cells it computed.  `ring` holds
// NW + 1 band-boundary buffers of a.bnd_stride (H, F) pairs.
template <int R, int NW>
__device__ int32_t intra_pair(const IntraArgs &a, const PairItem &pi, const QueryDesc &qd,
                              int w, int2 *ring) {
  const int lane = threadIdx.x & 63;
  const int n = pi.len;
  const int b_lo = pi.band0;
  const int nb = pi.band1 - pi.band0;  // bands of this segment
  int32_t vmax = 0;
  if (n <= 0 || nb <= 0) return 0;
  const int nc = (n + 63 + 63) / 64;  // chunks covering n + 63 steps
  const int nce = nc > kIntraLag * NW ? nc : kIntraLag * NW;
  const int lastb = nb - 1;
  const int rounds = (lastb / NW) * nce + kIntraLag * (lastb % NW) + nc;
  const uint8_t *resbase = a.packed + pi.base;
  const int cs = pi.cstride;
  const uint32_t pstride = (uint32_t)qd.mrows;
  const uint32_t lane_off = (uint32_t)(lane * R);

  int bl = w;  // band of this segment that this wave works on
  BandLane<R> L;

  for (int rd = 0; rd < rounds; ++rd) {
    if (bl < nb) {
      const int st = (bl / NW) * nce + kIntraLag * (bl % NW);
      if (rd >= st && rd < st + nc) {
        const int k = rd - st;
        const int b = b_lo + bl;  // query band
        // the first band of a later segment reads the previous segment's bottom row,
        // the last band of an earlier segment writes its own for the next segment
        const bool ext_top = bl == 0 && pi.xin >= 0;
        const bool ext_bot = bl == nb - 1 && pi.xout >= 0;
        const int2 *top = (ext_top ? a.xbnd + pi.xin
                                   : ring + (int64_t)((bl + NW) % (NW + 1)) * a.bnd_stride) +
                          kBndLead;
        int2 *bot = (ext_bot ? a.xbnd + pi.xout
                             : ring + (int64_t)(bl % (NW + 1)) * a.bnd_stride) + kBndLead;
        const bool has_top = bl > 0 || ext_top;
        const bool has_bot = bl < nb - 1 || ext_bot;
        // wait until the columns this chunk and the next read are published
        if (ext_top) wait_columns(a, pi.prog_in, min(n, 64 * (k + 2)));
        // the profile rows of band b
        const uint8_t *pbase = reinterpret_cast<const uint8_t *>(a.qp8) +
                               uniform64(qd.qp8 + (int64_t)b * 64 * R);
        if (k == 0) band_start(L, lane, n, top, has_top, resbase, cs, pbase, lane_off, pstride);
        band_chunk(L, vmax, a, lane, k, n, top, has_top, bot, has_bot && lane == 63, resbase,
                   cs, pbase, lane_off, pstride);
        // columns 0 .. 64k of the bottom row are written (all of them after the last chunk)
        if (ext_bot) publish_columns(a, pi.prog_out, k == nc - 1 ? n : min(n, 64 * k + 1));
        if (k == nc - 1) bl += NW;
      }
    }
    if (NW > 1) __syncthreads();
  }
  return vmax;
}

// Items [0, n_wide) are swept by a whole workgroup each ("wide"); items [n_wide, count)
// by a single wave each ("narrow").  Each workgroup first takes wide items, then its waves
// take narrow items independently.  If a.second is given, an item whose second entry has
// a length >= 0 is a two-pair item (int16, recompute on saturation); the others run in
// int32.
template <int R, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2)))
void k_intra32(IntraArgs a) {
  __shared__ int s_item;
  __shared__ int s_max[W];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  int2 *slot = a.bnd + (int64_t)blockIdx.x * a.bnd_slot_elems;
  // (the recompute list: the kernels count every pair they tried to append, and only the
  // first flag_cap are in the list; the others are left to k_rescan)
  const int count = a.count_dev ? min(*a.count_dev, a.flag_cap) : a.count;
  const int n_wide = a.n_wide < count ? a.n_wide : count;

  // Wide items hold the longest pairs, whose band pipelines set the critical path: their
  // waves issue first on their SIMDs (critical-pair launch 3, main launch 2), and the
  // narrow phase below, which fills the remaining issue slots, runs at priority 0.
  if (a.wide_prio == 3) __builtin_amdgcn_s_setprio(3);
  else if (a.wide_prio == 2) __builtin_amdgcn_s_setprio(2);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const int it = atomicAdd(a.next, 1);
      s_item = it < n_wide ? it : -1;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it < 0) break;
    const PairItem pi = a.items[it];
    const QueryDesc qd = a.queries[pi.query];
    if (a.second && a.second[it].len >= 0) {
      const PairItem pb = a.second[it];
      const uint32_t v = wave_pk_max(intra_pair16<R, W>(a, pi, pb, qd, w, slot));
      if (lane == 0) s_max[w] = (int32_t)v;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int i = 0; i < W; ++i) m = pk_max(m, (uint32_t)s_max[i]);
        // the packed maxima of a split item's segments are chained like a single pair's
        if (pi.segment > 0) m = pk_max(m, (uint32_t)wait_max(a, pi.prog_in));
        if (pi.segment + 1 < pi.nsegments) {
          pass_max(a, pi.prog_out, (int32_t)m);
        } else {
          finish_half(a, pi, qd, (int)(int16_t)(m & 0xffffu));
          finish_half(a, pb, qd, (int)(int16_t)(m >> 16));
        }
      }
      continue;
    }
    int32_t vmax = intra_pair<R, W>(a, pi, qd, w, slot);
    for (int off = 32; off > 0; off >>= 1) vmax = max(vmax, __shfl_xor(vmax, off));
    if (lane == 0) s_max[w] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
      int m = 0;
      for (int i = 0; i < W; ++i) m = max(m, s_max[i]);
      // the segments of a split pair chain their maxima; the last one writes the score
      if (pi.segment > 0) m = max(m, wait_max(a, pi.prog_in));
      if (pi.segment + 1 < pi.nsegments) {
        pass_max(a, pi.prog_out, m);
      } else {
        a.scores[qd.out + pi.out] = m;
      }
    }
  }

  if (a.wide_prio) __builtin_amdgcn_s_setprio(0);
  int2 *ring = slot + (int64_t)w * 2 * a.bnd_stride;  // two band buffers per wave
  // Narrow phase.  The waves run independently, so the claim cannot go through LDS and a
  // barrier.  It must not sit in a lane-0-only branch either: the compiler may then split
  // the wave across the loop back-edge and let lanes 1..63 re-read a stale item forever.
  // Every lane therefore executes the atomic (adding 1 from lane 0, 0 elsewhere; lane 0
  // gets the old value), and every lane stores the same reduced score.
  // Narrow items come longest first (cost = residues x query rows).  With priorities on,
  // the items within 70% of the first one's cost run at wave priority 1, the rest at 0:
  // when the search is bound by its longest pairs' dependency chains, those waves then
  // issue first on the SIMDs they share (plain search, 2,000 sequences up to 2,000
  // residues against 144 rows: 0.45-0.47 -> 0.38-0.39 ms).
  int64_t hot_cost = 0;
  if (a.wide_prio && n_wide < count) {
    const PairItem p0 = a.items[n_wide];
    hot_cost = (int64_t)p0.len * a.queries[p0.query].m;
  }
  for (;;) {
    const int claimed = atomicAdd(a.next_narrow, lane == 0 ? 1 : 0);
    const int it = __builtin_amdgcn_readfirstlane(claimed) + n_wide;
    if (it >= count) break;
    const PairItem pi = a.items[it];
    const QueryDesc qd = a.queries[pi.query];
    if (a.wide_prio) {
      if ((int64_t)pi.len * qd.m * 10 >= hot_cost * 7)
        __builtin_amdgcn_s_setprio(1);
      else
        __builtin_amdgcn_s_setprio(0);
    }
    if (a.second && a.second[it].len >= 0) {
      const PairItem pb = a.second[it];
      const uint32_t v = wave_pk_max(chain_fits(a, pi) ? intra_chain16<R>(a, pi, pb, qd, ring)
                                                       : intra_pair16<R, 1>(a, pi, pb, qd, 0, ring));
      finish_half(a, pi, qd, (int)(int16_t)(v & 0xffffu));
      finish_half(a, pb, qd, (int)(int16_t)(v >> 16));
      continue;
    }
    int32_t vmax = chain_fits(a, pi) ? intra_chain<R>(a, pi, qd, ring)
                                     : intra_pair<R, 1>(a, pi, qd, 0, ring);
    for (int off = 32; off > 0; off >>= 1) vmax = max(vmax, __shfl_xor(vmax, off));
    a.scores[qd.out + pi.out] = vmax;
  }
}

// LDS that an intra-task workgroup reserves and does not use, so that at most per_cu
// workgroups of its launch share a CU (per_cu = 1: more than half the CU's LDS, which
// still leaves room for one four-wave workgroup of another launch at per_cu = 2).  With
// 85-146 VGPRs the registers alone would admit more than the launches are planned for;
// a third four-wave workgroup beside the critical pairs' waves slowed the 5478-residue
// query over the long-sequence mix by 10-15%.  Sized from the device's LDS per CU and
// per workgroup (read once per device).
static size_t intra_lds_reserve(int per_cu) {
  static std::atomic<int> lds_cu[64], lds_wg[64];  // 0 = not yet known
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int cu = lds_cu[dev].load(std::memory_order_relaxed);
  int wg = lds_wg[dev].load(std::memory_order_relaxed);
  if (cu <= 0 || wg <= 0) {
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        cu <= 0 || wg <= 0)
      return 0;
    lds_cu[dev].store(cu, std::memory_order_relaxed);
    lds_wg[dev].store(wg, std::memory_order_relaxed);
  }
  const int limit = std::max(0, wg - 4096);  // (the kernels' own LDS is under 2 KB)
  const int r = per_cu <= 1 ? cu / 2 + 1024 : cu / per_cu - 4096;
  return (size_t)std::max(0, std::min(limit, r));
}

// Workgroups of kIntraWaves (8) or 4 waves at R = 2, 4, 8 or 16.  Four-wave workgroups
// serve the critical-pair launch (one wave per SIMD, none idle) and throughput-bound
// main launches (two per CU beside a critical-pair workgroup, else three).
hipError_t launch_intra32(const IntraArgs &a, int R, int waves, int grid, hipStream_t s,
                          int per_cu) {
  if (grid == 0) return hipSuccess;
  static_assert(kCritWaves == 4 && kNarrowWaves == 4, "four-wave instances below");
  const size_t lds = intra_lds_reserve(per_cu);
  if (waves == 4) {
    switch (R) {
      case 2: hipLaunchKernelGGL((k_intra32<2, 4>), dim3(grid), dim3(256), lds, s, a); break;
      case 4: hipLaunchKernelGGL((k_intra32<4, 4>), dim3(grid), dim3(256), lds, s, a); break;
      case 8: hipLaunchKernelGGL((k_intra32<8, 4>), dim3(grid), dim3(256), lds, s, a); break;
      case 16: hipLaunchKernelGGL((k_intra32<16, 4>), dim3(grid), dim3(256), lds, s, a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (waves != kIntraWaves) return hipErrorInvalidValue;
  const dim3 blk(64 * kIntraWaves);
  switch (R) {
    case 2: hipLaunchKernelGGL((k_intra32<2, kIntraWaves>), dim3(grid), blk, lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_intra32<4, kIntraWaves>), dim3(grid), blk, lds, s, a); break;
    case 8: hipLaunchKernelGGL((k_intra32<8, kIntraWaves>), dim3(grid), blk, lds, s, a); break;
    case 16: hipLaunchKernelGGL((k_intra32<16, kIntraWaves>), dim3(grid), blk, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------ recompute-list overflow
// The recompute list holds a bounded number of pairs.  When more pairs saturate (or all
// are forced through the recompute), the kernels mark the pairs they could not append
// with the score kSat16, which no exact int16 result below the ceiling takes, and this
// pass finds and recomputes them in int32.  A wave claims 64 sequences of one query at a
// time (a group, or up to 64 long sequences), and sweeps each marked one alone, as a
// narrow pair of the intra-task kernel.  It returns at once when the list did not
// overflow.  Single-wave workgroups; wave b uses band ring b % 8 of slot b / 8.
__global__ __launch_bounds__(64) void k_rescan(RescanArgs a) {
  if (*a.count <= a.ia.flag_cap) return;
  const int lane = threadIdx.x;
  int2 *ring = a.ia.bnd + (int64_t)(blockIdx.x / kIntraWaves) * a.ia.bnd_slot_elems +
               (int64_t)(blockIdx.x % kIntraWaves) * 2 * a.ia.bnd_stride;
  const int per_query = a.ngroups + (a.nlongs + 63) / 64;
  const int total = per_query * a.nqueries;
  for (;;) {
    const int claimed = atomicAdd(a.next, lane == 0 ? 1 : 0);
    const int c = __builtin_amdgcn_readfirstlane(claimed);
    if (c >= total) break;
    const int q = c / per_query, j = c - q * per_query;
    const QueryDesc qd = a.ia.queries[q];
    PairItem it;
    it.cstride = 256;
    it.base = 0;
    it.len = 0;
    it.out = -1;
    if (j < a.ngroups) {
      const GroupDesc gd = a.groups[j];
      if (lane < gd.count) {
        const int p = gd.first + lane;
        it.base = gd.base + 4 * lane;
        it.len = a.lens[p];
        it.out = a.perm[p];
      }
    } else {
      const int li = (j - a.ngroups) * 64 + lane;
      if (li < a.nlongs) {
        const LongSeq L = a.longs[li];
        it.base = L.base;
        it.cstride = 4;
        it.len = L.len;
        it.out = L.orig;
      }
    }
    const bool marked = it.out >= 0 && qd.m > 0 && a.ia.scores[qd.out + it.out] == kSat16;
    uint64_t todo = __ballot(marked);
    while (todo) {
      const int src = __builtin_ffsll((long long)todo) - 1;
      todo &= todo - 1;
      PairItem pi;
      pi.base = (int64_t)(((uint64_t)(uint32_t)__shfl((int)((uint64_t)it.base >> 32), src) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)it.base, src));
      pi.cstride = __shfl(it.cstride, src);
      pi.len = __shfl(it.len, src);
      pi.out = __shfl(it.out, src);
      pi.query = q;
      pi.band0 = 0;
      pi.band1 = qd.nbands;
      pi.xin = pi.xout = -1;
      pi.prog_in = pi.prog_out = -1;
      pi.segment = 0;
      pi.nsegments = 1;
      int32_t vmax = intra_pair<kIntraR, 1>(a.ia, pi, qd, 0, ring);
      for (int off = 32; off > 0; off >>= 1) vmax = max(vmax, __shfl_xor(vmax, off));
      a.ia.scores[qd.out + pi.out] = vmax;
    }
  }
}

hipError_t launch_rescan(const RescanArgs &a, int grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rescan, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ inter-task, two queries
// Batched searches (several queries against the same database): the inter-task DP of
// k_inter16 with the two int16 halves of every register given to two different queries
// aligned against the same sequence, at the same DB column and the same strip row.  Both
// halves then read the substitution score of the same residue code, so the profile is
// stored pre-packed, one dword per (code, row) holding the scores of both queries
// (k_profile2), and a cell pair is nine VALU instructions instead of ten (no byte
// permute).  The two halves are independent alignments: each strip of T rows starts from
// the previous strip's bottom row of the same two alignments, kept per wave in a boundary
// buffer laid out [column][H plane, F plane][64 lanes] dwords (the H pair of the bottom
// row, and the F pair entering the next strip).  Pairs of queries are formed longest
// first; an odd query out gets an empty partner whose rows all score kPadScore, which
// keeps that half at zero.  Saturation is handled per half as in k_inter16.

// Pair profile of query pair p: [nstrips][32 codes][T rows] dwords, low half query qa,
// high half query qb; rows past a query's end, codes outside the alphabet and the whole
// high half of a pair without qb score kPadScore.
__global__ void k_profile2(Profile2Args a) {
  const QueryPair pr = a.pairs[blockIdx.y];
  const int64_t n = (int64_t)pr.nstrips * kCodes * a.T;
  const uint8_t *qa = a.query + a.qoff[pr.qa];
  const int64_t ma = a.qoff[pr.qa + 1] - a.qoff[pr.qa];
  const uint8_t *qb = pr.qb >= 0 ? a.query + a.qoff[pr.qb] : nullptr;
  const int64_t mb = pr.qb >= 0 ? a.qoff[pr.qb + 1] - a.qoff[pr.qb] : 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % a.T);
    const int code = (int)((e / a.T) % kCodes);
    const int64_t i = (e / ((int64_t)a.T * kCodes)) * a.T + r;
    int lo = kPadScore, hi = kPadScore;
    if (code < a.alphabet) {
      if (i < ma) lo = a.matrix[qa[i] * a.alphabet + code];
      if (i < mb) hi = a.matrix[qb[i] * a.alphabet + code];
    }
    a.qp2[pr.qp2 + e] = ((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16);
  }
}

hipError_t launch_profile2(const Profile2Args &a, hipStream_t s) {
  if (a.npairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_profile2, dim3(32, a.npairs), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Writes the score of one half, or appends the pair to the recompute list when the half
// may have saturated.
__device__ __forceinline__ void inter2_finish(const Inter2Args &a, int q, int sc, int p,
                                              int orig, const GroupDesc &gd, int lane) {
  const QueryDesc qd = a.queries[q];
  if (sc >= kSat16 || a.recompute_all) {
    const int k = atomicAdd(&a.ctr->flagged, 1);
    if (k >= a.flag_cap) {
      a.scores[qd.out + orig] = kSat16;  // the list is full: k_rescan finds the mark
      return;
    }
    PairItem it;
    it.base = gd.base + 4 * lane;
    it.cstride = 256;
    it.len = a.lens[p];
    it.out = orig;
    it.query = q;
    it.band0 = 0;
    it.band1 = qd.nbands;
    it.xin = it.xout = -1;
    it.prog_in = it.prog_out = -1;
    it.segment = 0;
    it.nsegments = 1;
    a.flagged[k] = it;
  } else {
    a.scores[qd.out + orig] = sc;
  }
}

// The strip loop of one (query pair, group) item of the two-query inter-task kernel (see
// k_inter16q2).  The caller fills the LDS slice of strip s (32 codes x T rows of packed
// dwords, code rows Inter16q2Lds<T>::RS bytes apart) in `stage(s)`, which runs between
// two barriers of the single-wave workgroup.  Returns the packed running maximum of H.
template <int T> struct Inter16q2Lds {
  // LDS bytes per code row: an odd number of 16-byte units (fewer bank conflicts)
  static constexpr int RS = (T / 4) % 2 == 1 ? 4 * T : 4 * T + 16;
  static constexpr int bytes = kCodes * RS;
};

template <int T, class Stage>
__device__ __forceinline__ uint32_t inter16q2_strips(uint8_t *lds, const uint32_t *res, int ncols,
                                                     uint32_t *bnd, int nstrips, uint32_t goe2,
                                                     uint32_t ge2, Stage &&stage) {
  static_assert(T % 4 == 0, "strip height must be a multiple of 4");
  constexpr int RS = Inter16q2Lds<T>::RS;
  const int nchunks = ncols >> 2;
  uint32_t vmaxA = 0, vmaxB = 0;
  for (int s = 0; s < nstrips; ++s) {
    __syncthreads();
    stage(s);
    __syncthreads();

    const bool first = (s == 0);
    const bool last = (s == nstrips - 1);
    uint32_t Hs[T], Es[T];
#pragma unroll
    for (int r = 0; r < T; ++r) { Hs[r] = 0; Es[r] = 0; }
    uint32_t hprev = 0;  // boundary H pair of the column before the lead
    uint32_t rw = res[0];
    uint32_t h0 = 0, h1 = 0, h2 = 0, h3 = 0, f0 = 0, f1 = 0, f2 = 0, f3 = 0;
    if (!first) {
      h0 = bnd[0]; h1 = bnd[128]; h2 = bnd[256]; h3 = bnd[384];
      f0 = bnd[64]; f1 = bnd[192]; f2 = bnd[320]; f3 = bnd[448];
    }

    for (int c = 0; c < nchunks; ++c) {
      uint32_t rwn = 0, nh0 = 0, nh1 = 0, nh2 = 0, nh3 = 0, nf0 = 0, nf1 = 0, nf2 = 0, nf3 = 0;
      if (c + 1 < nchunks) {
        rwn = res[(int64_t)(c + 1) * 64];
        if (!first) {
          const uint32_t *bp = bnd + (int64_t)(c + 1) * 512;
          nh0 = bp[0]; nh1 = bp[128]; nh2 = bp[256]; nh3 = bp[384];
          nf0 = bp[64]; nf1 = bp[192]; nf2 = bp[320]; nf3 = bp[448];
        }
      }
      // codes of the pair's columns (J, J + 1) in the low two bytes of cw; boundary
      // words of those columns in hJ, hJ1 (H pairs) and fJ, fJ1 (F pairs)
      uint32_t cw = rw;
      uint32_t hJ = h0, hJ1 = h1, fJ = f0, fJ1 = f1;
#pragma unroll 1
      for (int p = 0; p < 2; ++p) {
        const int J = c * 4 + 2 * p;  // lead column; the lag column is J + 1
        const uint8_t *plA = lds + (cw & 0xffu) * RS;
        const uint8_t *plB = lds + ((cw >> 8) & 0xffu) * RS;
        // row-0 inputs from the boundary row: diagonal H and the F entering row 0
        const uint32_t hdA = hprev;
        uint32_t fa = fJ;
        const uint32_t hdB = hJ;
        uint32_t fb = fJ1;
        // The lead runs row r next to the lag's row r - 1, as in k_inter16.
        uint32_t dA1 = hdB, dA2 = 0;
        uint32_t smB_prev = 0;
#pragma unroll
        for (int r8 = 0; r8 < T; r8 += 8) {
          // 8 rows per block; a height that is not a multiple of 8 ends with 4
          const bool full = r8 + 8 <= T;
          const uint4 A1 = *reinterpret_cast<const uint4 *>(plA + 4 * r8);
          const uint4 B1 = *reinterpret_cast<const uint4 *>(plB + 4 * r8);
          uint4 A2 = make_uint4(0, 0, 0, 0), B2 = make_uint4(0, 0, 0, 0);
          if (full) {
            A2 = *reinterpret_cast<const uint4 *>(plA + 4 * r8 + 16);
            B2 = *reinterpret_cast<const uint4 *>(plB + 4 * r8 + 16);
          }
          const uint32_t av[8] = {A1.x, A1.y, A1.z, A1.w, A2.x, A2.y, A2.z, A2.w};
          const uint32_t bw[8] = {B1.x, B1.y, B1.z, B1.w, B2.x, B2.y, B2.z, B2.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (!full && q >= 4) break;
            const int r = r8 + q;
            const uint32_t h = cell16(r == 0 ? hdA : Hs[r - 1], av[q], Es[r], fa, vmaxA,
                                      goe2, ge2);
            if (r >= 1) Hs[r - 1] = cell16(dA2, smB_prev, Es[r - 1], fb, vmaxB, goe2, ge2);
            dA2 = dA1;
            dA1 = h;
            smB_prev = bw[q];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        const uint32_t ha = dA1;
        const uint32_t hb = cell16(dA2, smB_prev, Es[T - 1], fb, vmaxB, goe2, ge2);
        Hs[T - 1] = hb;
        if (!last) {
          uint32_t *bp = bnd + (int64_t)J * 128;
          bp[0] = ha; bp[64] = fa;
          bp[128] = hb; bp[192] = fb;
        }
        hprev = hJ1;
        cw >>= 16;
        hJ = h2; hJ1 = h3;
        fJ = f2; fJ1 = f3;
      }
      rw = rwn;
      h0 = nh0; h1 = nh1; h2 = nh2; h3 = nh3;
      f0 = nf0; f1 = nf1; f2 = nf2; f3 = nf3;
    }
  }
  return pk_max(vmaxA, vmaxB);
}

template <int T, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_inter16q2(Inter2Args a) {
  constexpr int RS = Inter16q2Lds<T>::RS;
  __shared__ __attribute__((aligned(16))) uint8_t lds[Inter16q2Lds<T>::bytes];
  const int lane = threadIdx.x;
  // The first big_waves waves have full-width boundary slots and take the widest items
  // [0, wide_items) first; every wave then takes the others in order from wide_items.
  const int wave = (int)blockIdx.x;
  const bool big = wave < a.big_waves;
  uint32_t *bnd = a.bnd + lane +
                  (big ? (int64_t)wave * a.bnd_slot_words
                       : (int64_t)a.big_waves * a.bnd_slot_words +
                             (int64_t)(wave - a.big_waves) * a.small_slot_words);
  const uint32_t goe2 = (uint32_t)a.goe * 0x10001u;
  const uint32_t ge2 = (uint32_t)a.ge * 0x10001u;
  __shared__ int s_item;
  bool wide_left = big && a.wide_items > 0;

  for (;;) {
    __syncthreads();
    if (lane == 0) {
      int it = -1;
      if (wide_left) {
        it = atomicAdd(&a.ctr->inter_wide, 1);
        if (it >= a.wide_items) it = -1;
      }
      if (it < 0) it = a.wide_items + atomicAdd(&a.ctr->inter_next, 1);
      s_item = it;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= a.nitems) break;
    wide_left = wide_left && item < a.wide_items;
    const int g = a.ngroups - 1 - item / a.npairs;  // longest groups first
    const QueryPair pr = a.pairs[item % a.npairs];  // pairs are ordered longest first
    const GroupDesc gd = a.groups[g];
    const uint32_t *qp = a.qp2 + pr.qp2;
    const uint32_t *res = reinterpret_cast<const uint32_t *>(a.packed + gd.base) + lane;
    // each strip's pair-profile slice (32 codes x T rows) is copied into LDS
    auto stage = [&](int s) {
      const uint4 *src = reinterpret_cast<const uint4 *>(qp + (int64_t)s * kCodes * T);
      constexpr int PER_CODE = T / 4;  // 16-byte pieces per code row
      constexpr int PIECES = kCodes * PER_CODE;
#pragma unroll
      for (int c = lane; c < PIECES; c += 64) {
        const int code = c / PER_CODE, k = c - code * PER_CODE;
        *reinterpret_cast<uint4 *>(lds + code * RS + k * 16) = src[c];
      }
    };
    const bool prio = gd.ncols >= a.prio_cols;  // as in k_inter16
    if (prio) __builtin_amdgcn_s_setprio(2);
    const uint32_t vmax =
        inter16q2_strips<T>(lds, res, gd.ncols, bnd, pr.nstrips, goe2, ge2, stage);
    if (prio) __builtin_amdgcn_s_setprio(0);
    if (lane < gd.count) {
      const int p = gd.first + lane;
      const int orig = a.perm[p];
      inter2_finish(a, pr.qa, (int)(int16_t)(vmax & 0xffffu), p, orig, gd, lane);
      if (pr.qb >= 0) inter2_finish(a, pr.qb, (int)(int16_t)(vmax >> 16), p, orig, gd, lane);
    }
  }
}

// Minimum waves per SIMD requested for each strip height of the pair kernel (28 rows
// still fit three waves: it has no skew registers).
template <int T> struct Inter16q2Occ { static constexpr int wpe = T <= 8 ? 6 : (T <= 16 ? 4 : (T <= 28 ? 3 : 2)); };

template <int T>
static hipError_t launch_inter16q2_t(const Inter2Args &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_inter16q2<T, Inter16q2Occ<T>::wpe>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

bool inter16q2_supported(int T) { return T == 8 || T == 16 || T == 24 || T == 28 || T == 32 || T == 40; }

int inter16q2_max_blocks_per_cu(int T) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (T) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<8, Inter16q2Occ<8>::wpe>, 64, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<16, Inter16q2Occ<16>::wpe>, 64, 0); break;
    case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<24, Inter16q2Occ<24>::wpe>, 64, 0); break;
    case 28: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<28, Inter16q2Occ<28>::wpe>, 64, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<32, Inter16q2Occ<32>::wpe>, 64, 0); break;
    case 40: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_inter16q2<40, Inter16q2Occ<40>::wpe>, 64, 0); break;
    default: break;
  }
  return e == hipSuccess ? n : 0;
}

hipError_t launch_inter16q2(const Inter2Args &a, int T, int grid, hipStream_t s) {
  if (a.nitems == 0 || grid == 0) return hipSuccess;
  switch (T) {
    case 8: return launch_inter16q2_t<8>(a, grid, s);
    case 16: return launch_inter16q2_t<16>(a, grid, s);
    case 24: return launch_inter16q2_t<24>(a, grid, s);
    case 28: return launch_inter16q2_t<28>(a, grid, s);
    case 32: return launch_inter16q2_t<32>(a, grid, s);
    case 40: return launch_inter16q2_t<40>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------ serving session
// Continuous batching (not in the paper, whose queries run one after another): one
// persistent launch serves every query admitted while it runs.  Work item i belongs to
// record i / ngroups and is its group ngroups - 1 - i % ngroups (longest first), so the
// items of a record admitted while others are on the device queue up right behind them
// and the waves move on to it as they finish, with no launch in between.
//
// A record is one query (the one-query strip loop of k_inter16, strips of 2 * T1 rows) or
// two queries of similar length sharing the lanes (the strip loop of k_inter16q2, T2
// rows).  The host writes records and query residues into host memory and then raises a
// doorbell (2 * records published, plus 1 once no more will come).  A wave that claims
// an item of a record not yet published waits: workgroups [0, npoll) read the doorbell
// over the bus and raise a device-memory mirror of it, the others read the mirror, with
// a growing sleep between reads.  No other kernel can run beside the session's waves,
// so the waves build each strip's profile slice themselves, in LDS, from the query
// residues (copied once per record into a per-wave cache) and the substitution matrix
// (kept in LDS), and write scores through the caches into device memory.  The wave that
// finishes a record's last item publishes its completion (and whether any score reached
// the int16 ceiling, Section 4.2, in which case the host recomputes that query exactly)
// with a system-scope release; the host then copies the rows out (a DMA copy, which runs
// beside the kernel).

// Claim the next item and wait until its record is published.  Lane 0 only.  Returns
// the item, or -1 once the session is closed before the item's record came, or when the
// wait timed out (then the error flag is set).
__device__ int serve_claim(const ServeArgs &a) {
  const int item = atomicAdd(a.claim, 1);
  const int need = item / a.ngroups + 1;  // records that must be published
  const bool poller = (int)blockIdx.x < a.npoll;
  // the polling waves also tell the host how far the claims have got, which it uses to
  // publish a record only when the device is about to run out of published work
  if (poller)
    __hip_atomic_store(a.hprog + blockIdx.x, item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const int64_t t0 = wall_clock64();
  int backoff = 1;
  for (;;) {
    int v;
    if (poller) {
      v = __hip_atomic_load(a.doorbell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_fetch_max(a.mirror, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      v = __hip_atomic_load(a.mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if ((v >> 1) >= need) return item;
    if (v & 1) return -1;  // closed: this record will never be published
    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return -1;
    if (wall_clock64() - t0 > a.timeout_ticks) {
      __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return -1;
    }
    for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(127);
    if (backoff < 16) backoff += 1;
  }
}

template <int T1, int T2>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void k_serve(ServeArgs a) {
  constexpr int RS1 = Inter16Lds<T1>::RS, RS2 = Inter16q2Lds<T2>::RS;
  constexpr int LB = Inter16Lds<T1>::bytes > Inter16q2Lds<T2>::bytes ? Inter16Lds<T1>::bytes
                                                                     : Inter16q2Lds<T2>::bytes;
  static_assert(2 * T1 <= 64 && T2 <= 64, "a strip's residues fit one 64-byte row");
  __shared__ __attribute__((aligned(16))) uint8_t lds[LB];
  __shared__ int8_t smat[kCodes * kCodes];  // [query code][database code]; |entries| <= 127
  __shared__ __attribute__((aligned(16))) uint8_t sres[2][64];  // residues of one strip
  __shared__ int s_item;
  const int lane = threadIdx.x;
  for (int e = lane; e < kCodes * kCodes; e += 64) {
    const int d = e >> 5, c = e & 31;
    smat[e] = (int8_t)((d < a.alphabet && c < a.alphabet) ? a.matrix[d * a.alphabet + c]
                                                          : kPadScore);
  }
  uint32_t *bnd = a.bnd + (int64_t)blockIdx.x * a.bnd_slot_words + lane;
  uint8_t *qc = a.qcache + (int64_t)blockIdx.x * 2 * a.qcap;
  const uint32_t goe2 = (uint32_t)a.goe * 0x10001u;
  const uint32_t ge2 = (uint32_t)a.ge * 0x10001u;
  int cur = -1;  // record whose queries are in this wave's cache
  int64_t out_a = 0, out_b = -1;
  int ma = 0, mb = 0, kind = 1, nstrips = 0;

  for (;;) {
    __syncthreads();
    if (lane == 0) s_item = serve_claim(a);
    __syncthreads();
    const int item = s_item;
    if (item < 0) break;
    // (no cache maintenance per item: what the host wrote before the doorbell, the
    // record and its queries, is read below with loads that bypass the caches)
    const int r = item / a.ngroups;
    const int g = a.ngroups - 1 - (item - r * a.ngroups);
    const int slot = r % a.nrec;
    if (r != cur) {
      // a new record: its descriptor, then both queries into this wave's cache
      const int32_t *rw = reinterpret_cast<const int32_t *>(a.records + slot);
      constexpr int NW = (int)(sizeof(ServeRecord) / 4);
      const int v = lane < NW ? __hip_atomic_load(rw + lane, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM) : 0;
      const uint32_t oa_lo = (uint32_t)__builtin_amdgcn_readlane(v, 0);
      const uint32_t oa_hi = (uint32_t)__builtin_amdgcn_readlane(v, 1);
      const uint32_t ob_lo = (uint32_t)__builtin_amdgcn_readlane(v, 2);
      const uint32_t ob_hi = (uint32_t)__builtin_amdgcn_readlane(v, 3);
      out_a = (int64_t)(((uint64_t)oa_hi << 32) | oa_lo);
      out_b = (int64_t)(((uint64_t)ob_hi << 32) | ob_lo);
      ma = __builtin_amdgcn_readlane(v, 4);
      mb = __builtin_amdgcn_readlane(v, 5);
      kind = __builtin_amdgcn_readlane(v, 6);
      nstrips = __builtin_amdgcn_readlane(v, 7);
      const uint32_t *src = reinterpret_cast<const uint32_t *>(a.qstage + (int64_t)slot * 2 * a.qcap);
      uint32_t *dst = reinterpret_cast<uint32_t *>(qc);
      // every row the strips read, padding included (the staging is padded that far)
      const int nbytes = (nstrips * (kind == 1 ? 2 * T1 : T2) + 63) & ~63;
      const int na = nbytes >> 2, nbq = kind == 1 ? 0 : nbytes >> 2;
      const int qw = a.qcap >> 2;
      // (bus reads that bypass the caches: the slot held other queries before)
      for (int k = lane; k < na; k += 64)
        dst[k] = __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      for (int k = lane; k < nbq; k += 64)
        dst[qw + k] = __hip_atomic_load(src + qw + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      // the copy must be visible to every lane's later reads of the cache (one wave, one
      // compute unit: a workgroup-scope fence)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      cur = r;
    }
    const GroupDesc gd = a.groups[g];
    const uint32_t *res = reinterpret_cast<const uint32_t *>(a.packed + gd.base) + lane;
    // a record's widest groups, each one wave's work for much of the record's time, run at
    // raised priority on their SIMDs (as in k_inter16)
    const bool prio = gd.ncols >= a.prio_cols;
    if (prio) __builtin_amdgcn_s_setprio(2);
    uint32_t vmax;
    if (kind == 1) {
      // strip s: rows [s * 2T1, (s + 1) * 2T1) of query a, as int16 row pairs per code
      auto stage = [&](int s) {
        constexpr int ROWS = 2 * T1;
        if (lane < ROWS / 4)
          *reinterpret_cast<uint32_t *>(&sres[0][4 * lane]) =
              reinterpret_cast<const uint32_t *>(qc + (int64_t)s * ROWS)[lane];
        __syncthreads();
        constexpr int DW = kCodes * ROWS / 2;  // dwords of the slice
#pragma unroll
        for (int w = lane; w < DW; w += 64) {
          const int code = w / (ROWS / 2), rp = w - code * (ROWS / 2);
          const uint32_t lo = (uint16_t)(int16_t)smat[sres[0][2 * rp] * kCodes + code];
          const uint32_t hi = (uint16_t)(int16_t)smat[sres[0][2 * rp + 1] * kCodes + code];
          *reinterpret_cast<uint32_t *>(lds + code * RS1 + 4 * rp) = lo | (hi << 16);
        }
      };
      vmax = inter16_strips<T1>(lds, res, gd.ncols, bnd, nstrips, goe2, ge2, stage);
      const int lo = (int)(int16_t)(vmax & 0xffffu), hi = (int)(int16_t)(vmax >> 16);
      vmax = (uint32_t)(lo > hi ? lo : hi);
    } else {
      // strip s: rows [s * T2, (s + 1) * T2) of both queries, packed per code and row
      auto stage = [&](int s) {
        if (lane < 2 * (T2 / 4)) {
          const int q = lane >= T2 / 4, k = lane - q * (T2 / 4);
          *reinterpret_cast<uint32_t *>(&sres[q][4 * k]) =
              reinterpret_cast<const uint32_t *>(qc + q * a.qcap + (int64_t)s * T2)[k];
        }
        __syncthreads();
        constexpr int DW = kCodes * T2;
#pragma unroll
        for (int w = lane; w < DW; w += 64) {
          const int code = w / T2, rr = w - code * T2;
          const uint32_t lo = (uint16_t)(int16_t)smat[sres[0][rr] * kCodes + code];
          const uint32_t hi = (uint16_t)(int16_t)smat[sres[1][rr] * kCodes + code];
          *reinterpret_cast<uint32_t *>(lds + code * RS2 + 4 * rr) = lo | (hi << 16);
        }
      };
      vmax = inter16q2_strips<T2>(lds, res, gd.ncols, bnd, nstrips, goe2, ge2, stage);
    }
    if (prio) __builtin_amdgcn_s_setprio(0);
    // Scores go to device memory with stores that write through the caches; the wave waits
    // until they are done before it counts the item, so a release (which would write back
    // the whole L2 after every item) is needed only once per record, by the last wave.
    // (Scattered 4-byte stores straight into host memory cost about a tenth of the
    // throughput; the host copies a complete record's rows out instead.)
    int sat = 0;
    if (lane < gd.count) {
      const int orig = a.perm[gd.first + lane];
      int sa = (int)vmax, sb = 0;
      if (kind != 1) {
        sa = (int)(int16_t)(vmax & 0xffffu);
        sb = (int)(int16_t)(vmax >> 16);
      }
      __hip_atomic_store(a.scores + out_a + orig, sa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      sat = sa >= kSat16 ? 1 : 0;
      if (kind != 1 && out_b >= 0) {
        __hip_atomic_store(a.scores + out_b + orig, sb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        sat |= sb >= kSat16 ? 2 : 0;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    // saturation bits of the wave, then the item count of the record (each atomic
    // completes before the next is issued); the wave that finishes the record's last item
    // reports it to the host
    for (int off = 32; off > 0; off >>= 1) sat |= __shfl_xor(sat, off);
    if (lane == 0) {
      if (sat) {
        __hip_atomic_fetch_or(a.satf + slot, sat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
      }
      const int old = __hip_atomic_fetch_add(a.done + slot, 1, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      if (old == a.ngroups - 1) {
        const int bits = __hip_atomic_load(a.satf + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.satf + slot, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.done + slot, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.hsat + slot, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.complete + slot, r + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

int serve_max_blocks_per_cu() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, k_serve<kServeT1, kServeT2>, 64, 0);
  return e == hipSuccess ? n : 0;
}

hipError_t launch_serve(const ServeArgs &a, int grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_serve<kServeT1, kServeT2>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace swmi
