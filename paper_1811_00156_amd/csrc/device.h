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

// The 128-bit product a * b from four 32 x 32 -> 64-bit multiply-adds (the
// schoolbook terms; no partial sum overflows 64 bits).
__device__ __forceinline__ void mul_64x64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t t = (uint64_t)a0 * b0;
  const uint64_t u = (uint64_t)a1 * b0 + (t >> 32);
  const uint64_t v = (uint64_t)a0 * b1 + (uint32_t)u;
  hi = (uint64_t)a1 * b1 + (u >> 32) + (v >> 32);
  lo = (v << 32) | (uint32_t)t;
}

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mul_64x64(c0, kM0, hi0, lo0);
    mul_64x64(c2, kM1, hi1, lo1);
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

// Integer in [0, m) from a 64-bit draw: floor(r * m / 2^64), for m < 2^32:
// floor((r1 m + floor(r0 m / 2^32)) / 2^32) with r = r1 2^32 + r0.
__device__ __forceinline__ uint64_t scale_draw(uint64_t r, uint32_t m) {
  const uint64_t t = (uint64_t)(uint32_t)r * m;
  return ((uint64_t)(uint32_t)(r >> 32) * m + (t >> 32)) >> 32;
}

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
// (double)x for a 64-bit integer: h 2^32 + l with both halves converted exactly
// and one rounding in the fused multiply-add, the correctly rounded value the
// plain conversion gives, in three instructions instead of four.
__device__ __forceinline__ double i64_to_f64(int64_t x) {
  return __builtin_fma((double)(int32_t)(x >> 32), 4294967296.0, (double)(uint32_t)x);
}

// a / b, correctly rounded, for a zero or in [1, 2^90] and b in [1, 2^20]: the
// divide sequence the compiler emits for IEEE division (reciprocal, two Newton
// steps, the quotient, one correction by fused multiply-add) without its
// operand scaling and special-value fixup, which leave operands in these
// ranges unchanged (no denormal, no overflow, no exponent gap near 768), so
// the quotient is the same; 8 instructions instead of 11.  aiwc_rf_probe_divide
// (libaiwc_rf_probe.so) checks it against IEEE division on that domain.
__device__ __forceinline__ double div_pos(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = a * r;
  const double rem = __builtin_fma(-b, q, a);
  return __builtin_fma(rem, r, q);
}

// (|S| < 2^41 and N < 2^19 by the fixed-point budget: S^2 < 2^82.)
__device__ __forceinline__ double split_score(int64_t SL, uint32_t NL, int64_t SR, uint32_t NR) {
  const double a = i64_to_f64(SL), b = i64_to_f64(SR);
  const double l = div_pos(a * a, (double)NL);
  const double r = div_pos(b * b, (double)NR);
  return l + r;
}
// The same score for a node that weighs below 512: |S_L|, |S_R| < 511 * 2^22 <
// 2^31, so each converts exactly from 32 bits (one conversion instead of
// i64_to_f64's three) to the same double.
__device__ __forceinline__ double split_score32(int32_t SL, uint32_t NL, int32_t SR, uint32_t NR) {
  const double a = (double)SL, b = (double)SR;
  const double l = div_pos(a * a, (double)NL);
  const double r = div_pos(b * b, (double)NR);
  return l + r;
}
__device__ __forceinline__ double parent_score(int64_t S, uint64_t N) {
  const double a = i64_to_f64(S);
  return div_pos(a * a, (double)N);
}

// ---------------------------------------------------------------------------
// Loads through global-address-space pointers.  Pointers the kernel carves
// out of its scratch area are generic, and a generic (flat) load counts
// against the LDS counter as well as the memory counter, so a wait for an LDS
// result also waits for it.  A 16-byte load goes through a native vector type
// (a copy of uint4 would read through a generic reference).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gload16(const void* p) {
  const u32x4_t v = *(const __attribute__((address_space(1))) u32x4_t*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------
// Wave64 collectives.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The collectives below move values between lanes with DPP row operations
// (GFX9 encoding) instead of LDS permutes, and must be called with every lane
// of the wave active.  A wave64 inclusive scan is a Kogge-Stone scan inside each
// row of 16 lanes (row_shr 1, 2, 4, 8), then row_bcast:15 adds row 0's total
// into row 1 and row 2's into row 3, and row_bcast:31 adds the first two rows'
// total into rows 2 and 3.  A lane whose source is outside its row, or in a
// row the row mask leaves out, receives the operation's identity.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t identity, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t identity, uint64_t v) {
  const uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)identity, (uint32_t)v);
  const uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(identity >> 32), (uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_move(T v) {
  if constexpr (sizeof(T) == 8)
    return (T)dpp64<CTRL, ROW_MASK>(0ull, (uint64_t)v);
  else
    return (T)dpp32<CTRL, ROW_MASK>(0u, (uint32_t)v);
}

// Inclusive prefix sum over the wave's lanes (integer T of 4 or 8 bytes).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  v += dpp_move<kDppRowShr1, 0xf>(v);
  v += dpp_move<kDppRowShr2, 0xf>(v);
  v += dpp_move<kDppRowShr4, 0xf>(v);
  v += dpp_move<kDppRowShr8, 0xf>(v);
  v += dpp_move<kDppRowBcast15, 0xa>(v);
  v += dpp_move<kDppRowBcast31, 0xc>(v);
  return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) { return wave_incl_scan<uint32_t>(v); }

// v of lane `src` (per lane) by two LDS-crossbar permutes; every lane active.
__device__ __forceinline__ uint64_t lane_pick64(uint64_t v, uint32_t src) {
  const int addr = (int)(src << 2);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T read_lane(T v, int l) {
  if constexpr (sizeof(T) == 8) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (T)(((uint64_t)hi << 32) | lo);
  } else {
    return (T)__builtin_amdgcn_readlane((int)v, l);
  }
}

// Sum over the wave (integer T), in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return read_lane(wave_incl_scan<T>(v), kWave - 1);
}

// Arg-max of (score, key) over the wave: the largest score, then the smallest
// key.  Every lane returns the winner and the lane that holds it (lowest lane
// among equals).  A prefix arg-max with the scan's DPP pattern leaves the
// wave's winner in the last lane.
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
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void argmax_step(ArgMax& m) {
  constexpr uint64_t kMinusInf = 0xFFF0000000000000ull;
  const double s = __builtin_bit_cast(double, dpp64<CTRL, ROW_MASK>(kMinusInf, __builtin_bit_cast(uint64_t, m.score)));
  const int32_t k = (int32_t)dpp32<CTRL, ROW_MASK>(0x7FFFFFFFu, (uint32_t)m.key);
  const int32_t l = (int32_t)dpp32<CTRL, ROW_MASK>(0x7FFFFFFFu, (uint32_t)m.lane);
  if (argmax_better(s, k, l, m.score, m.key, m.lane)) {
    m.score = s;
    m.key = k;
    m.lane = l;
  }
}
__device__ __forceinline__ ArgMax wave_argmax(double score, int32_t key) {
  ArgMax m{score, key, (int32_t)lane_id()};
  argmax_step<kDppRowShr1, 0xf>(m);
  argmax_step<kDppRowShr2, 0xf>(m);
  argmax_step<kDppRowShr4, 0xf>(m);
  argmax_step<kDppRowShr8, 0xf>(m);
  argmax_step<kDppRowBcast15, 0xa>(m);
  argmax_step<kDppRowBcast31, 0xc>(m);
  ArgMax r;
  r.score = __builtin_bit_cast(double, read_lane(__builtin_bit_cast(uint64_t, m.score), kWave - 1));
  r.key = read_lane(m.key, kWave - 1);
  r.lane = read_lane(m.lane, kWave - 1);
  return r;
}

// The same when lane order is key order (lane l's key below lane l+1's): a wave
// max of the scores with the scan's DPP pattern, then the lowest lane that holds
// it.  Scores must not be NaN.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double max_step(double m) {
  constexpr uint64_t kMinusInf = 0xFFF0000000000000ull;
  const double o = __builtin_bit_cast(double, dpp64<CTRL, ROW_MASK>(kMinusInf, __builtin_bit_cast(uint64_t, m)));
  return o > m ? o : m;
}
__device__ __forceinline__ ArgMax wave_argmax_lane_ordered(double score, int32_t key) {
  double m = score;
  m = max_step<kDppRowShr1, 0xf>(m);
  m = max_step<kDppRowShr2, 0xf>(m);
  m = max_step<kDppRowShr4, 0xf>(m);
  m = max_step<kDppRowShr8, 0xf>(m);
  m = max_step<kDppRowBcast15, 0xa>(m);
  m = max_step<kDppRowBcast31, 0xc>(m);
  ArgMax r;
  r.score = __builtin_bit_cast(double, read_lane(__builtin_bit_cast(uint64_t, m), kWave - 1));
  r.lane = __builtin_ctzll(__ballot(score == r.score));
  r.key = read_lane(key, r.lane);
  return r;
}

// All-reductions inside aligned segments of W = 4, 8, 16 or 32 lanes, for an
// operation that is associative and commutative.  Within a row of 16 the steps
// are DPP permutations (every source lane valid): a rotation by 8 pairs lanes
// i and i ^ 8, the half-row mirror pairs i and 7 - i of each group of 8, and
// two quad permutations pair i ^ 2 and i ^ 1; for any W the combined sets of
// each lane cover its segment exactly once.  The 16-lane step of W = 32 is one
// LDS permute.
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowRor8 = 0x128;

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_perm(T v) {
  return dpp_move<CTRL, 0xf>(v);
}
template <int W, typename T>
__device__ __forceinline__ T seg_sum(T v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32, "segment width");
  if constexpr (W == 32) v += __shfl_xor(v, 16, kWave);
  if constexpr (W >= 16) v += dpp_perm<kDppRowRor8>(v);
  if constexpr (W >= 8) v += dpp_perm<kDppHalfMirror>(v);
  v += dpp_perm<kDppQuadXor2>(v);
  v += dpp_perm<kDppQuadXor1>(v);
  return v;
}

// Segment arg-max of (score, key): the largest score, then the smallest key.
template <int CTRL>
__device__ __forceinline__ void seg_argmax_step(double& s, uint32_t& k) {
  const double os = __builtin_bit_cast(double, dpp_perm<CTRL>(__builtin_bit_cast(uint64_t, s)));
  const uint32_t ok = dpp_perm<CTRL>(k);
  if (os > s || (os == s && ok < k)) {
    s = os;
    k = ok;
  }
}
template <int W>
__device__ __forceinline__ void seg_argmax(double& s, uint32_t& k) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32, "segment width");
  if constexpr (W == 32) {
    const double os = __shfl_xor(s, 16, kWave);
    const uint32_t ok = (uint32_t)__shfl_xor((int)k, 16, kWave);
    if (os > s || (os == s && ok < k)) {
      s = os;
      k = ok;
    }
  }
  if constexpr (W >= 16) seg_argmax_step<kDppRowRor8>(s, k);
  if constexpr (W >= 8) seg_argmax_step<kDppHalfMirror>(s, k);
  seg_argmax_step<kDppQuadXor2>(s, k);
  seg_argmax_step<kDppQuadXor1>(s, k);
}

// Make this wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace aiwc
