// Device-side building blocks shared by the binning, fitting and prediction
// kernels: the Philox4x64-10 generator, the packed row-entry and node formats,
// exact integer helpers and wave64 collectives for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aiwc {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each multiplies
// counter words 0 and 2 by the round multipliers, xors the high halves into the
// other two words with the key, and bumps the key by the Weyl increments.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return {{c0, c1, c2, c3}};
}

// Stream tags (counter word 1).
constexpr uint64_t kTagBootstrap = 0;
constexpr uint64_t kTagMtry = 1;

// Integer in [0, m) from a 64-bit draw: floor(r * m / 2^64).
__device__ __forceinline__ uint64_t scale_draw(uint64_t r, uint64_t m) { return __umul64hi(r, m); }

// ---------------------------------------------------------------------------
// Row entry: one 64-bit word per in-bag row of a tree, moved by the partition.
//   bits  0..17  row index (n <= 2^18)
//   bits 18..36  bootstrap multiplicity w (<= 2^18)
//   bits 37..63  fixed-point response y_fp, signed 27 bits (|y_fp| <= 2^22)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t entry_pack(uint32_t row, uint32_t w, int64_t y) {
  return (uint64_t)row | ((uint64_t)w << 18) | ((uint64_t)y << 37);
}
__device__ __forceinline__ uint32_t entry_row(uint64_t e) { return (uint32_t)(e & 0x3FFFFu); }
__device__ __forceinline__ uint32_t entry_w(uint64_t e) { return (uint32_t)((e >> 18) & 0x7FFFFu); }
__device__ __forceinline__ int64_t entry_y(uint64_t e) { return (int64_t)e >> 37; }

// ---------------------------------------------------------------------------
// Node word: one 64-bit word per tree node, the only thing traversal reads.
//   split: bits 0..7 column (< 255), 8..15 bin, 16..47 left child id
//   leaf:  bits 0..7 = 255, bits 8..63 leaf value q (signed, |q| <= 2^38)
// ---------------------------------------------------------------------------
constexpr uint32_t kLeafCol = 255;
__device__ __host__ __forceinline__ uint64_t node_split(uint32_t col, uint32_t bin, uint32_t left) {
  return (uint64_t)col | ((uint64_t)bin << 8) | ((uint64_t)left << 16);
}
__device__ __host__ __forceinline__ uint64_t node_leaf(int64_t q) { return (uint64_t)kLeafCol | ((uint64_t)q << 8); }
__device__ __host__ __forceinline__ uint32_t node_col(uint64_t v) { return (uint32_t)(v & 0xFF); }
__device__ __host__ __forceinline__ uint32_t node_bin(uint64_t v) { return (uint32_t)((v >> 8) & 0xFF); }
__device__ __host__ __forceinline__ uint32_t node_left(uint64_t v) { return (uint32_t)(v >> 16); }
__device__ __host__ __forceinline__ int64_t node_q(uint64_t v) { return (int64_t)v >> 8; }

// ---------------------------------------------------------------------------
// Exact integer helpers.
// ---------------------------------------------------------------------------
// Pure node: N * Q == S^2, compared as 128-bit products (N <= 2^18, Q <= 2^62).
__device__ __forceinline__ bool node_is_pure(uint64_t N, int64_t S, uint64_t Q) {
  const uint64_t a = S < 0 ? (uint64_t)(-S) : (uint64_t)S;
  return (N * Q == a * a) && (__umul64hi(N, Q) == __umul64hi(a, a));
}

// Leaf value: round-half-away(S * 2^16 / N) = sign(S) * floor((|S| 2^17 + N) / (2N)).
__device__ __forceinline__ int64_t leaf_value(uint64_t N, int64_t S) {
  const uint64_t a = S < 0 ? (uint64_t)(-S) : (uint64_t)S;
  const uint64_t m = (a * 131072ull + N) / (2ull * N);
  return S < 0 ? -(int64_t)m : (int64_t)m;
}

// Split score S_L^2/N_L + S_R^2/N_R: two products, two correctly rounded
// divisions and one sum in binary64, in this order (the library is compiled
// with -ffp-contract=off, so no fused multiply-add is formed).
__device__ __forceinline__ double split_score(int64_t SL, uint32_t NL, int64_t SR, uint32_t NR) {
  const double a = (double)SL, b = (double)SR;
  const double l = a * a / (double)NL;
  const double r = b * b / (double)NR;
  return l + r;
}
__device__ __forceinline__ double parent_score(int64_t S, uint64_t N) {
  const double a = (double)S;
  return a * a / (double)N;
}

// ---------------------------------------------------------------------------
// Wave64 collectives.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = (int)lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = (int)lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Arg-max of (score, key) over the wave: the largest score, then the smallest
// key.  Every lane returns the winner and the lane that holds it (lowest lane
// among equals).
struct ArgMax {
  double score;
  int32_t key;
  int32_t lane;
};
__device__ __forceinline__ bool argmax_better(double s1, int32_t k1, int32_t l1, double s2, int32_t k2, int32_t l2) {
  if (s1 != s2) return s1 > s2;
  if (k1 != k2) return k1 < k2;
  return l1 < l2;
}
__device__ __forceinline__ ArgMax wave_argmax(double score, int32_t key) {
  ArgMax m{score, key, (int32_t)lane_id()};
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const double s = __shfl_xor(m.score, d, kWave);
    const int32_t k = __shfl_xor(m.key, d, kWave);
    const int32_t l = __shfl_xor(m.lane, d, kWave);
    if (argmax_better(s, k, l, m.score, m.key, m.lane)) {
      m.score = s;
      m.key = k;
      m.lane = l;
    }
  }
  return m;
}

// Make this wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace aiwc
