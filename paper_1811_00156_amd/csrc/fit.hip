// Forest fitting on gfx950: one workgroup grows one tree at a time, level by
// level, pulling trees from a device-side queue until every tree of every
// forest in the launch is grown.
//
// Per tree (Sec. III-B: a random-forest regression tree with num.trees, mtry and
// min.node.size; the readings of the unspecified steps are listed in the public
// header):
//   1. bootstrap: n_train Philox draws -> multiplicity per training row, then the
//      in-bag rows are packed into 64-bit entries (row, weight, y_fp);
//   2. for each level, one thread per open node applies the leaf rules
//      (min.node.size, purity) and draws the node's mtry candidate columns; the
//      split search over every (candidate column, bin) is then tiered by the
//      node's number of in-bag rows:
//        - small (<= 64 rows): one row per lane in a segment of 4..64 lanes,
//          every candidate column's codes gathered at once, the left sums of
//          each lane's split found from the segment's rows staged in LDS;
//        - large (<= huge limit): one wave per (node, column), LDS histogram of
//          (N, S, Q) per bin and a wave prefix scan over bins;
//        - wide (above a tuned size): the whole workgroup takes a batch of such
//          nodes at once; each row's entry is read once and its codes in all
//          candidate columns are gathered by one thread, into packed (N, S)
//          LDS histograms of every node and candidate column of the batch;
//          one wave per (node, column) then scans;
//      every split maximises S_L^2/N_L + S_R^2/N_R; ties keep the lowest
//      (column, bin);
//   3. split nodes get breadth-first child ids from a workgroup scan, node words
//      are written, and the in-bag entries are partitioned into the children's
//      segments of the other entry buffer (wave-aggregated cursor atomics).
// All sums are integers and the only floating point is the binary64 score, so
// the order in which rows are visited never changes a result.
#include <limits.h>

#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "device.h"
#include "internal.h"

namespace aiwc {
namespace {

// kSplitDone: split and already partitioned by the wave that searched it (nodes
// of at most kSegMax rows); kSplit: a large or wide node decided to split in
// the child-id step, its rows still to be partitioned (never stored)
constexpr uint8_t kLeaf = 0, kSmall = 1, kBig = 2, kHuge = 3, kSplit = 4, kSplitDone = 5;
// Nodes with at most kSegMax in-bag rows are searched with their rows in a
// lane segment of width 4, 8, 16, 32 or 64 (the smallest that holds them).
constexpr uint32_t kSegMax = 64;
constexpr int kSegClasses = 5;
constexpr int kMaxBins = 256;

// A searched node as the split-search tasks see it (filled when the node is
// classified, so a task needs one dependent load to find its rows).
struct NodeDesc {
  uint32_t k;      // index of the node within its level
  uint32_t start;  // first entry of its segment
  uint32_t len;    // in-bag rows
  uint32_t N;      // bootstrap weight
  int64_t S;       // sum of weight * y_fp
};

struct Rec {
  double score;
  int64_t SL;
  uint32_t NL;
  uint32_t colbin;  // column << 8 | bin
};

// Per-workgroup global scratch.  The per-level arrays come in two copies (the
// level being grown and the next one), selected by the level parity without
// indexing, so that every pointer stays in scalar registers.
struct Level2 {
  uint64_t* buf;
  uint32_t* mstart;
  uint32_t* mend;
  uint32_t* mN;
  int64_t* mS;
  uint64_t* mQ;
};

// A node's candidate list takes mtry bytes rounded up to 16 (the padding
// repeats the last candidate), so that it can be read with 16-byte loads.
__host__ __device__ inline int cand_stride(int mtry) { return (mtry + 15) & ~15; }

// A split node's partition state, by its rank among the level's split nodes:
// the next free slots from the left and from the right of its entry range, and
// the left side's sum of w y^2.
struct Cursor {
  uint32_t L, R;
  uint64_t q;
};

struct Scratch {
  uint32_t* cnt;
  Level2 L0, L1;
  uint8_t* status;
  uint8_t* cand;     // level node k's candidate columns at k * cand_stride(mtry), ascending, padded
  uint32_t* btask;   // large node j's candidate i at j * mtry + i: column | bin count << 8
  uint8_t* dcol;  // small split node k's decision: column, bin, left weight and sum
  uint8_t* dbin;
  uint32_t* dNL;
  int64_t* dSL;
  uint32_t* ridx;  // large node k: its index among the level's large (or wide) nodes
  uint32_t* dcnt;  // small split node k: entries that went left
  uint64_t* dQL;   // small split node k: left side's sum of w y^2
  Cursor* cur;    // by split rank, when a level's do not fit the LDS
  uint4* chunks;  // partition work per 64-entry chunk: first entry, the node's end, split rank, column | bin << 8
  NodeDesc* seg[kSegClasses];  // small nodes by segment width 4 << class
  NodeDesc* big;
  NodeDesc* huge;
  Rec* recs;  // large node j's candidate i at j * mtry + i; wide node h's at (n_big + h) * mtry + i
  // entry p of a wide node: its row's codes in the node's candidate columns, at
  // p * cand_stride(mtry) + i (written by the wide batches, read by the partition
  // instead of the row's code line); null when the launch has no wide phase
  uint8_t* side;
  // the level at which the trees of a group of tasks part, as its split
  // searches left it (kept while each member grows on from it): this level's
  // entries and node sums, the next level's entries (the small nodes' rows,
  // placed by their searches), and the per-node search results and records;
  // null when the launch has no groups
  struct Parted {
    Level2 L;
    uint64_t* nbuf;
    uint8_t *status, *dcol, *dbin;
    uint32_t *ridx, *dNL, *dcnt;
    int64_t* dSL;
    uint64_t* dQL;
    Rec* recs;
    uint8_t* side;
  } SN;
};

__host__ __device__ inline size_t carve(Scratch* s, uintptr_t base, int64_t n_cap, int32_t mtry_max, bool wide,
                                        bool grouped) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> uintptr_t {
    const size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return base + o;
  };
  const size_t n = (size_t)n_cap;
  // large and huge nodes hold more than kSegMax rows each
  const size_t n_large = n / (kSegMax + 1) + 1;
  s->cnt = reinterpret_cast<uint32_t*>(take(4 * n));
  Level2* lv[2] = {&s->L0, &s->L1};
  for (int b = 0; b < 2; ++b) {
    lv[b]->buf = reinterpret_cast<uint64_t*>(take(8 * n));
    lv[b]->mstart = reinterpret_cast<uint32_t*>(take(4 * n));
    lv[b]->mend = reinterpret_cast<uint32_t*>(take(4 * n));
    lv[b]->mN = reinterpret_cast<uint32_t*>(take(4 * n));
    lv[b]->mS = reinterpret_cast<int64_t*>(take(8 * n));
    lv[b]->mQ = reinterpret_cast<uint64_t*>(take(8 * n));
  }
  s->status = reinterpret_cast<uint8_t*>(take(n));
  s->cand = reinterpret_cast<uint8_t*>(take(n * (size_t)cand_stride(mtry_max)));
  s->dcol = reinterpret_cast<uint8_t*>(take(n));
  s->dbin = reinterpret_cast<uint8_t*>(take(n));
  s->dNL = reinterpret_cast<uint32_t*>(take(4 * n));
  s->dSL = reinterpret_cast<int64_t*>(take(8 * n));
  // a split node holds at least two rows, so a level has at most n/2 of them
  // and at most n/64 + n/2 chunks
  s->cur = reinterpret_cast<Cursor*>(take(sizeof(Cursor) * (n / 2 + 1)));
  s->dcnt = reinterpret_cast<uint32_t*>(take(4 * n));
  s->ridx = reinterpret_cast<uint32_t*>(take(4 * n));
  s->dQL = reinterpret_cast<uint64_t*>(take(8 * n));
  s->chunks = reinterpret_cast<uint4*>(take(sizeof(uint4) * (n / 64 + n / 2 + 2)));
  // class c holds nodes of more than 2 << c rows (c >= 1)
  for (int c = 0; c < kSegClasses; ++c)
    s->seg[c] = reinterpret_cast<NodeDesc*>(take(sizeof(NodeDesc) * (n / (1 + (c ? (2u << c) : 0)) + 1)));
  s->big = reinterpret_cast<NodeDesc*>(take(sizeof(NodeDesc) * n_large));
  s->huge = reinterpret_cast<NodeDesc*>(take(sizeof(NodeDesc) * n_large));
  s->recs = reinterpret_cast<Rec*>(take(sizeof(Rec) * n_large * (size_t)mtry_max));
  s->btask = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * n_large * (size_t)mtry_max));
  s->side = wide ? reinterpret_cast<uint8_t*>(take(n * (size_t)cand_stride(mtry_max))) : nullptr;
  s->SN = Scratch::Parted{};
  if (grouped) {
    s->SN.L.buf = reinterpret_cast<uint64_t*>(take(8 * n));
    s->SN.L.mstart = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.L.mend = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.L.mN = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.L.mS = reinterpret_cast<int64_t*>(take(8 * n));
    s->SN.L.mQ = reinterpret_cast<uint64_t*>(take(8 * n));
    s->SN.nbuf = reinterpret_cast<uint64_t*>(take(8 * n));
    s->SN.status = reinterpret_cast<uint8_t*>(take(n));
    s->SN.dcol = reinterpret_cast<uint8_t*>(take(n));
    s->SN.dbin = reinterpret_cast<uint8_t*>(take(n));
    s->SN.ridx = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.dNL = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.dcnt = reinterpret_cast<uint32_t*>(take(4 * n));
    s->SN.dSL = reinterpret_cast<int64_t*>(take(8 * n));
    s->SN.dQL = reinterpret_cast<uint64_t*>(take(8 * n));
    s->SN.recs = reinterpret_cast<Rec*>(take(sizeof(Rec) * n_large * (size_t)mtry_max));
    s->SN.side = wide ? reinterpret_cast<uint8_t*>(take(n * (size_t)cand_stride(mtry_max))) : nullptr;
  }
  return off;
}

// Per-wave LDS: one histogram of packed (N, S) bins over at most 256 bins.
// The small-node methods reuse the area for their staged weights, sums and
// codes (up to 4864 bytes).
struct WaveHist {
  uint64_t hv[kMaxBins];
  uint8_t stage[4864 - 8 * kMaxBins];
};

struct GrowArgs {
  const uint8_t* codes;
  int32_t C;
  const uint8_t* codes_p;  // the same codes, rows padded to Cp bytes (one cache line holds whole rows)
  int32_t Cp;
  // the copy the searches and the partition gather codes from: the dense rows
  // while the training set's codes fit an L2 comfortably, else the padded ones
  const uint8_t* rcodes;
  int32_t rC;
  const int32_t* n_bins;
  const int64_t* y_fp;
  const int32_t* train_rows;
  const TreeTask* tasks;
  int32_t n_tasks;
  // groups of tasks that differ only in min.node.size: group g's members are
  // tasks group_task[group_first[g] .. group_first[g + 1]), by min.node.size
  // ascending; null: every task is a group of its own, in task order
  const int32_t* group_task;
  const int32_t* group_first;
  int32_t n_groups;
  uint64_t* nodes;
  uint32_t* node_N;
  int32_t* n_nodes;
  int64_t* work;  // per task (kWorkWords each): searched rows, searched nodes, partitioned rows, levels, LDS bin adds
  uint64_t* inbag;
  uint32_t* queue;
  uint32_t* status;
  uint8_t* scratch;
  int64_t n_cap;
  int32_t mtry_max;
  int32_t huge_min;  // nodes with more rows than this are searched in workgroup-wide batches
  int32_t wide_sums;  // 1: the small-node searches add 64-bit sums even when weights fit a byte
  int32_t bstride;   // bins per column histogram in the workgroup-wide layout
  int32_t big_cols;    // candidate columns per large-node task (1 .. 4)
  int32_t big_stride;  // bins per column histogram of a large-node task
  size_t scratch_stride;
  uint32_t union_bytes;  // dynamic LDS
  uint32_t wave_bytes;   // per-wave area of the split-search tasks
};

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup exclusive scan of one u32 per thread; `total` receives the sum.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* tmp, uint32_t& total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = (int)lane_id(), wid = threadIdx.x / kWave;
  const uint32_t incl = wave_incl_scan_u32(v);
  if (lane == kWave - 1) tmp[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    const uint32_t t = lane < NW ? tmp[lane] : 0u;
    const uint32_t ti = wave_incl_scan_u32(t);
    if (lane < NW) tmp[lane] = ti - t;
    if (lane == NW - 1) tmp[NW] = ti;
  }
  __syncthreads();
  const uint32_t res = tmp[wid] + incl - v;
  total = tmp[NW];
  __syncthreads();
  return res;
}

// The same for one u64 per thread (two counts packed in its halves).
template <int BLOCK>
__device__ __forceinline__ uint64_t block_exscan64(uint64_t v, uint64_t* tmp, uint64_t& total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = (int)lane_id(), wid = threadIdx.x / kWave;
  const uint64_t incl = wave_incl_scan<uint64_t>(v);
  if (lane == kWave - 1) tmp[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    const uint64_t t = lane < NW ? tmp[lane] : 0ull;
    const uint64_t ti = wave_incl_scan<uint64_t>(t);
    if (lane < NW) tmp[lane] = ti - t;
    if (lane == NW - 1) tmp[NW] = ti;
  }
  __syncthreads();
  const uint64_t res = tmp[wid] + incl - v;
  total = tmp[NW];
  __syncthreads();
  return res;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T* tmp) {
  constexpr int NW = BLOCK / kWave;
  const int lane = (int)lane_id(), wid = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) tmp[wid] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < NW; ++i) s += tmp[i];
  __syncthreads();
  return s;
}

// The mtry candidate columns of node `node` of tree `tree`, drawn by one
// thread: a partial Fisher-Yates shuffle of 0..C-1 driven by draws k = 0 ..
// mtry-1 of the stream (seed, tag 1, node, tree); position k swaps with
// k + floor(r_k (C-k) / 2^64).  `perm` is this thread's C-entry LDS row
// (stride `pst` bytes between entries).  The chosen columns are written
// ascending to `out`, and, when `bt` is given, column | bin count << 8 to
// bt[0 .. mtry) (`nb`: the bin counts, in LDS).
__device__ __forceinline__ void draw_candidates(uint8_t* perm, int pst, uint64_t seed, uint32_t node, uint32_t tree, int C, int mtry,
                                uint8_t* out, uint32_t* bt, const uint16_t* nb) {
  for (int c = 0; c < C; ++c) perm[c * pst] = (uint8_t)c;
  uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
  for (int b = 0; 4 * b < mtry; ++b) {
    const U64x4 r = philox4x64_10((uint64_t)b, kTagMtry, node, tree, seed, 0);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int k = 4 * b + w;
      if (k < mtry) {
        const int j = k + (int)scale_draw(r.w[w], (uint32_t)(C - k));
        const uint8_t vk = perm[k * pst], vj = perm[j * pst];
        perm[k * pst] = vj;
        perm[j * pst] = vk;
        const uint64_t bit = 1ull << (vj & 63);
        switch (vj >> 6) {
          case 0: m0 |= bit; break;
          case 1: m1 |= bit; break;
          case 2: m2 |= bit; break;
          default: m3 |= bit; break;
        }
      }
    }
  }
  int i = 0;
  uint32_t last = 0;
  auto put = [&](uint32_t c) {
    out[i] = (uint8_t)c;
    if (bt) bt[i] = c | ((uint32_t)nb[c] << 8);
    ++i;
    last = c;
  };
  for (uint64_t m = m0; m; m &= m - 1) put((uint32_t)__builtin_ctzll(m));
  for (uint64_t m = m1; m; m &= m - 1) put(64u + (uint32_t)__builtin_ctzll(m));
  for (uint64_t m = m2; m; m &= m - 1) put(128u + (uint32_t)__builtin_ctzll(m));
  for (uint64_t m = m3; m; m &= m - 1) put(192u + (uint32_t)__builtin_ctzll(m));
  for (; i < cand_stride(mtry); ++i) out[i] = (uint8_t)last;
}

struct Ctx {
  const GrowArgs* a;
  const TreeTask* T;
  Scratch sc;
  const uint64_t* buf;  // this level's entries
  uint64_t* nbuf;       // the next level's entries
  const uint32_t* mstart;
  const uint32_t* mend;
  const uint32_t* mN;
  const int64_t* mS;
  const uint64_t* mQ;
};

// Small nodes (at most kSegMax rows): a wave takes P = 64 / W nodes whose rows
// fit a segment of W lanes, one row per lane.  For each candidate position i
// (node k's i-th column, ascending) every lane takes the split at its own
// row's code: the left sums come from the W rows of its segment staged in
// LDS, the segment keeps the best (max score, then lowest bin), and across
// columns a strictly greater score is needed, so ties keep the lowest column.
// The segment's first lane then decides the node; the children's sums come
// from one more segment reduction over the winning column.
// Packed bin of the workgroup-wide and rank histograms: N * 2^45 + S in one unsigned
// 64-bit word.  With N <= 2^18 and |S| <= 2^40 (the fixed-point budget) a bin,
// and every prefix sum of bins, lies in [0, 2^64) and decodes exactly; a bin
// is empty iff its word is 0.  One LDS atomic adds a row to a bin.
__device__ __forceinline__ uint64_t pack_ns(uint32_t w, int64_t wy) { return ((uint64_t)w << 45) + (uint64_t)wy; }
__device__ __forceinline__ uint32_t packed_n(uint64_t v) { return (uint32_t)((v + (1ull << 44)) >> 45); }
__device__ __forceinline__ int64_t packed_s(uint64_t v, uint32_t n) { return (int64_t)(v - ((uint64_t)n << 45)); }

// Inclusive wave scan of packed bins of a node that weighs below 512: every
// prefix of its weights fits 9 bits and of its sums 32 bits (|y_fp| <= 2^22),
// so the two are scanned as 32-bit words (one DPP add a step) and packed again.
__device__ __forceinline__ uint64_t scan_packed_small(uint64_t h) {
  const uint32_t n = packed_n(h);
  const int32_t s = (int32_t)packed_s(h, n);
  const uint32_t pn = wave_incl_scan_u32(n);
  const int32_t ps = (int32_t)wave_incl_scan_u32((uint32_t)s);
  return pack_ns(pn, ps);
}

// The end of a small node's search, for the W lanes of its segment (one row
// each, lane `sbase + r`): the left child's weight, sum and sum of w y^2 from
// segment reductions, and the node's rows placed into its children's segments
// of the next level (left ones first, in lane order, then the right ones), so
// that the partition skips it; the segment's first lane writes the decision.
template <int W>
__device__ __forceinline__ void small_finish(const Ctx& x, uint32_t k, bool node_ok, int r, int sbase, bool split,
                                             uint32_t col, uint32_t bin, bool valid, bool left, uint64_t e,
                                             uint32_t start) {
  const uint32_t w = entry_w(e);
  const int64_t y = entry_y(e);
  const int64_t wy = (int64_t)w * y;
  uint64_t acc, QL;
  if constexpr (W == kWave) {
    acc = wave_sum(left ? pack_ns(w, wy) : 0ull);
    QL = wave_sum(left ? (uint64_t)(wy * y) : 0ull);
  } else {
    acc = seg_sum<W>(left ? pack_ns(w, wy) : 0ull);
    QL = seg_sum<W>(left ? (uint64_t)(wy * y) : 0ull);
  }
  const uint32_t NL = packed_n(acc);
  const int64_t SL = packed_s(acc, NL);
  const uint64_t seg = (W == kWave ? ~0ull : ((1ull << W) - 1ull)) << sbase;
  const uint64_t lm = __ballot(left) & seg, rm = __ballot(split && valid && !left) & seg;
  const uint64_t below = (1ull << lane_id()) - 1ull;
  const uint32_t nl = (uint32_t)__popcll(lm);
  if (split && valid)
    x.nbuf[start + (left ? (uint32_t)__popcll(lm & below) : nl + (uint32_t)__popcll(rm & below))] = e;
  if (node_ok && r == 0) {
    if (split) {
      x.sc.dcol[k] = (uint8_t)col;
      x.sc.dbin[k] = (uint8_t)bin;
      x.sc.dNL[k] = NL;
      x.sc.dSL[k] = SL;
      x.sc.dcnt[k] = nl;
      x.sc.dQL[k] = QL;
      x.sc.status[k] = kSplitDone;
    } else {
      x.sc.status[k] = kLeaf;
    }
  }
  wave_lds_sync();
}

// Left sums of the split at `code` over a segment of W rows staged as byte
// planes (the group of rows 4j..4j+3 takes 32 bytes: word 0 their weights,
// words 1..4 bytes 0..3 of their w y), four rows at a time: byte b of `ind`
// marks row b's code <= `code`, then dot products with the planes.  C7 (every
// code below 128): 128 + code - c stays in [1, 255] in each byte, so no borrow
// crosses the bytes and its bit 7 is the comparison; `ind` keeps that bit in
// place (byte 0x80: 128 unsigned, -128 signed), so the sums come out times 128
// (the signed top plane's times -128) and one exact shift at the end divides it
// out.  Otherwise per 16-bit half 256 + code - c stays in [1, 511] and its high
// byte (0 or 1) is the comparison: bytes 0 and 2 of the codes are compared in
// place, bytes 1 and 3 moved down by a byte permute, and a second permute
// gathers the four high bytes.
template <int W, bool C7, bool B3>
__device__ __forceinline__ void byte_plane_sums(uint32_t code, const uint32_t* seg_codes, const uint8_t* seg_planes,
                                                uint32_t& NL, int64_t& SL) {
  const uint32_t kk = C7 ? (code + 0x80u) * 0x01010101u : code * 0x00010001u + 0x01000100u;
  uint32_t aN = 0, a0 = 0, a1 = 0;
  int32_t a2 = 0, a3 = 0;
#pragma unroll 4
  for (int b4 = 0; b4 < W / 4; ++b4) {
    const uint32_t c4 = seg_codes[b4];
    uint32_t ind;
    if constexpr (C7) {
      ind = (kk - c4) & 0x80808080u;
    } else {
      const uint32_t d02 = kk - (c4 & 0x00FF00FFu);
      const uint32_t d13 = kk - __builtin_amdgcn_perm(0u, c4, 0x0c030c01u);  // bytes 1, 3 of c4 to 0, 2
      ind = __builtin_amdgcn_perm(d02, d13, 0x03070105u);  // bytes 1, 3 of each difference, interleaved
    }
    const uint4 pl = *reinterpret_cast<const uint4*>(seg_planes + b4 * 32);
    aN = __builtin_amdgcn_udot4(ind, pl.x, aN, false);
    a0 = __builtin_amdgcn_udot4(ind, pl.y, a0, false);
    a1 = __builtin_amdgcn_udot4(ind, pl.z, a1, false);
    if constexpr (B3) {
      // w y in 24 bits: byte 2 is its signed top byte
      a2 = __builtin_amdgcn_sdot4((int32_t)ind, (int32_t)pl.w, a2, false);
    } else {
      const uint32_t p3 = *reinterpret_cast<const uint32_t*>(seg_planes + b4 * 32 + 16);
      a2 = (int32_t)__builtin_amdgcn_udot4(ind, pl.w, (uint32_t)a2, false);
      a3 = __builtin_amdgcn_sdot4((int32_t)ind, (int32_t)p3, a3, false);
    }
  }
  if constexpr (C7) {
    // every accumulator is a multiple of 128 (at most 128 * 255 * 32): byte
    // plane j's sum times 2^(8 j) is a_j / 128 * 2^(8 j), the signed top
    // plane's negated
    NL = aN >> 7;
    if constexpr (B3)
      SL = (int64_t)(a0 >> 7) + ((int64_t)a1 << 1) - ((int64_t)a2 << 9);
    else
      SL = (int64_t)(a0 >> 7) + ((int64_t)a1 << 1) + ((int64_t)(uint32_t)a2 << 9) - ((int64_t)a3 << 17);
  } else {
    NL = aN;
    if constexpr (B3)
      SL = (int64_t)a0 + ((int64_t)a1 << 8) + ((int64_t)a2 << 16);
    else
      SL = (int64_t)a0 + ((int64_t)a1 << 8) + ((int64_t)(uint32_t)a2 << 16) + ((int64_t)a3 << 24);
  }
}

template <int W>
__device__ __forceinline__ void small_task(const Ctx& x, const NodeDesc* list, uint32_t t, uint32_t n_list, WaveHist& wl) {
  const GrowArgs& a = *x.a;
  const int mtry = x.T->mtry;
  const int lane = (int)lane_id();
  constexpr int P = kWave / W;
  const int g = lane / W, r = lane % W, sbase = g * W;
  const uint32_t idx = t * (uint32_t)P + (uint32_t)g;
  const bool node_ok = idx < n_list;
  NodeDesc d{0u, 0u, 0u, 0u, 0};
  if (node_ok) d = list[idx];
  const uint32_t k = d.k, start = d.start, len = d.len, N = d.N;
  const int64_t S = d.S;
  const bool valid = (uint32_t)r < len;
  const uint64_t e = valid ? x.buf[start + r] : 0ull;
  const uint32_t row = entry_row(e);
  const uint32_t w = valid ? entry_w(e) : 0u;
  const int64_t y = entry_y(e);
  const int64_t wy = (int64_t)w * y;
  uint8_t* area = reinterpret_cast<uint8_t*>(&wl);
  uint8_t* s_codes = area + 512;  // [64 columns][64 lanes]
  // The rows' weights and w y, staged in the first 512 bytes.  When every weight
  // of the wave fits a byte (bootstrap multiplicities nearly always do), as byte
  // planes: the group of rows 4j..4j+3 takes 32 bytes, word 0 their weights and
  // words 1..4 bytes 0..3 of their w y (|w y| < 2^30: two's complement, the top
  // byte signed), so that four rows' left sums are five 4-byte dot products
  // (four when every w y fits 24 bits).  Otherwise packed (w, w y) words, one
  // per row.
  const bool bytes_ok = !a.wide_sums && __ballot(w > 255u) == 0ull;
  // every w y of the wave fits 24 bits: its top byte is a sign extension, and
  // three byte planes of w y carry it
  const bool b3 = __ballot(wy < -(int64_t)(1 << 23) || wy >= (int64_t)(1 << 23)) == 0ull;
  // every column's codes fit 7 bits (at most 128 bins)
  const bool codes7 = a.bstride <= 128;
  // every node of the wave weighs below 512: its sums fit 32 bits
  const bool light = __ballot(N >= 512u) == 0ull;
  uint8_t* planes = area;
  uint64_t* s_pv = reinterpret_cast<uint64_t*>(area);
  if (bytes_ok) {
    const uint32_t wy32 = (uint32_t)(int32_t)wy;
    uint8_t* gp = planes + (lane >> 2) * 32 + (lane & 3);
    gp[0] = (uint8_t)w;
    gp[4] = (uint8_t)wy32;
    gp[8] = (uint8_t)(wy32 >> 8);
    gp[12] = (uint8_t)(wy32 >> 16);
    gp[16] = (uint8_t)(wy32 >> 24);
  } else {
    s_pv[lane] = pack_ns(w, wy);
  }
  const uint8_t* rowp = a.rcodes + (size_t)row * a.rC;
  const uint8_t* cand = x.sc.cand + (size_t)k * cand_stride(mtry);

  // each lane keeps its own best split (score, candidate index, bin) over the
  // candidates in order; one segment arg-max at the end picks the node's
  double best = -1.0;
  uint32_t best_ib = 0xFFFFFFFFu;  // candidate index << 8 | bin
  const uint64_t* seg_pv = s_pv + sbase;
  const uint8_t* seg_planes = planes + (sbase >> 2) * 32;
  for (int i0 = 0; i0 < mtry; i0 += kWave) {
    const int nc = min(kWave, mtry - i0);
    // gather the row's codes in every candidate column of this chunk at once:
    // sixteen candidates per 16-byte load, sixteen gathers in flight.  Every
    // lane loads and stores without a branch: a lane without a row reads row 0
    // (entry 0), whose codes no sum uses (its weight and w y are zero), and a
    // position past the chunk reads column 0 into a slot no candidate reads
    // (g0 + u < 64: inside the 64-column staging area).
    for (int g0 = 0; g0 < nc; g0 += 16) {
      const uint4 c16 = gload16(cand + i0 + g0);
      const uint32_t cw[4] = {c16.x, c16.y, c16.z, c16.w};
      uint32_t cd[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint32_t c = g0 + u < nc ? (cw[u >> 2] >> (8 * (u & 3))) & 0xFFu : 0u;
        cd[u] = gload(rowp + c);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s_codes[(g0 + u) * kWave + lane] = (uint8_t)cd[u];
    }
    wave_lds_sync();
    for (int i = 0; i < nc; ++i) {
      const uint8_t* col_codes = s_codes + i * kWave;
      const uint32_t code = col_codes[lane];
      const uint32_t* seg_codes = reinterpret_cast<const uint32_t*>(col_codes + sbase);
      // left sums of the split at this lane's code: the segment's rows with a code <= it
      uint32_t NL;
      int64_t SL;
      if (bytes_ok) {
        if (codes7)
          b3 ? byte_plane_sums<W, true, true>(code, seg_codes, seg_planes, NL, SL)
             : byte_plane_sums<W, true, false>(code, seg_codes, seg_planes, NL, SL);
        else
          b3 ? byte_plane_sums<W, false, true>(code, seg_codes, seg_planes, NL, SL)
             : byte_plane_sums<W, false, false>(code, seg_codes, seg_planes, NL, SL);
      } else {
        uint64_t acc = 0;  // packed left sums
#pragma unroll 2
        for (int b4 = 0; b4 < W / 4; ++b4) {
          const uint32_t c4 = seg_codes[b4];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc += ((c4 >> (8 * u)) & 0xFFu) <= code ? seg_pv[4 * b4 + u] : 0ull;
        }
        NL = packed_n(acc);
        SL = packed_s(acc, NL);
      }
      if (valid && NL < N) {
        const double sc = light ? split_score32((int32_t)SL, NL, (int32_t)S - (int32_t)SL, N - NL)
                                : split_score(SL, NL, S - SL, N - NL);
        if (sc > best) {
          best = sc;
          best_ib = ((uint32_t)(i0 + i) << 8) | code;
        }
      }
    }
    wave_lds_sync();
  }
  // segment arg-max: the largest score, then the lowest candidate, then the lowest bin
  seg_argmax<W>(best, best_ib);
  const bool split = node_ok && best >= 0.0 && best - parent_score(S, N) > 0.0;
  const uint32_t col = split ? cand[best_ib >> 8] : 0u, bin = best_ib & 0xFF;
  const bool left = split && valid && rowp[col] <= bin;
  small_finish<W>(x, k, node_ok, r, sbase, split, col, bin, valid, left, e, start);
}

// Nodes of 33..64 rows: one node per wave, one row per lane.  Per candidate
// column the rows' packed (w, w y) are added into the column's LDS bins, a wave
// prefix scan over the bins (ceil(B / 64) per lane) turns them into left sums,
// and every lane scores the split at its own row's code (rows with the largest
// code leave the right side empty and are skipped; lanes sharing a code score
// the same split).  A column of at most 64 bins keeps its prefix sums in
// registers (one bin per lane, read and cleared by its lane) and each lane
// takes the one at its own code by a cross-lane read; a wider column writes
// them back to LDS.  Two bin buffers alternate between candidates, so that a
// wider column's bins are cleared while the next candidate is scanned.
__device__ __forceinline__ void rank_task(const Ctx& x, const NodeDesc* list, uint32_t t, uint32_t n_list, WaveHist& wl) {
  const GrowArgs& a = *x.a;
  const int mtry = x.T->mtry;
  const int lane = (int)lane_id();
  if (t >= n_list) return;
  const NodeDesc d = list[t];
  const uint32_t k = rfl(d.k), start = rfl(d.start), len = rfl(d.len), N = rfl(d.N);
  const int64_t S = d.S;
  const bool valid = (uint32_t)lane < len;
  const uint64_t e = valid ? x.buf[start + lane] : 0ull;
  const uint32_t w = valid ? entry_w(e) : 0u;
  const int64_t y = entry_y(e);
  const int64_t wy = (int64_t)w * y;
  const uint64_t pv = pack_ns(w, wy);
  const uint8_t* rowp = a.rcodes + (size_t)entry_row(e) * a.rC;
  const uint8_t* cand = x.sc.cand + (size_t)k * cand_stride(mtry);
  uint8_t* area = reinterpret_cast<uint8_t*>(&wl);
  uint64_t* hb = reinterpret_cast<uint64_t*>(area);  // [2][256] packed bins, then prefix sums
  uint8_t* s_cand = area + 4096;                     // [mtry]
  uint8_t* s_bm1 = area + 4352;                      // [mtry]: each candidate's bin count - 1
  for (int i = lane; i < mtry; i += kWave) {
    const uint32_t c = gload(cand + i);
    s_cand[i] = (uint8_t)c;
    s_bm1[i] = (uint8_t)(gload(a.n_bins + c) - 1);
  }
  // both buffers start zeroed: four bins per lane each
  *reinterpret_cast<uint4*>(hb + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
  *reinterpret_cast<uint4*>(hb + 4 * lane + 2) = make_uint4(0u, 0u, 0u, 0u);
  *reinterpret_cast<uint4*>(hb + 256 + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
  *reinterpret_cast<uint4*>(hb + 256 + 4 * lane + 2) = make_uint4(0u, 0u, 0u, 0u);
  wave_lds_sync();

  // each lane keeps the best of the splits it scores (the one at its own code,
  // for every candidate) as (score, candidate index << 8 | bin); one arg-max at
  // the end
  double best = -1.0;
  int32_t best_ib = INT_MAX;
  // every lane fetches its code (a lane without a row reads row 0, entry 0, and
  // adds nothing), so that the fetch is not a branch the memory wait must close
  uint32_t c_next = rfl(s_cand[0]);
  uint32_t code_next = gload(rowp + c_next);
  bool prev_in_lds = false;  // the previous candidate left prefix sums in its buffer
  for (int i = 0; i < mtry; ++i) {
    const uint32_t code = code_next;
    const uint32_t B = rfl(s_bm1[i]) + 1u;  // this candidate column's bins
    if (i + 1 < mtry) {  // fetch the next column's codes while this one is scanned
      c_next = rfl(s_cand[i + 1]);
      code_next = gload(rowp + c_next);
    }
    uint64_t* hv = hb + (i & 1) * 256;
    if (valid) atomicAdd((unsigned long long*)&hv[code], (unsigned long long)pv);
    wave_lds_sync();
    // a previous candidate whose prefix sums went to LDS left its buffer dirty;
    // every lane read its left sums before these adds: clear it while this one
    // is scanned
    if (prev_in_lds) {
      uint64_t* ho = hb + ((i - 1) & 1) * 256;
      *reinterpret_cast<uint4*>(ho + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(ho + 4 * lane + 2) = make_uint4(0u, 0u, 0u, 0u);
    }
    uint64_t V;  // left sums (packed) of the split at this lane's code
    if (B <= (uint32_t)kWave) {
      // one bin per lane: the lane owning bin b reads and clears it (the buffer
      // is zero again for its next use), the prefix sums stay in registers,
      // and each lane takes the one at its own code by a cross-lane read
      const uint64_t h = lane < (int)B ? hv[lane] : 0ull;
      if (lane < (int)B) hv[lane] = 0ull;
      const uint64_t v = N < 512u ? scan_packed_small(h) : wave_incl_scan<uint64_t>(h);
      V = lane_pick64(v, code);
      prev_in_lds = false;
    } else {
      // inclusive prefix sums of the B bins, ceil(B / 64) consecutive bins per lane
      const int q = ((int)B + kWave - 1) / kWave;
      const int b0 = lane * q;
      uint64_t h[4];
      uint64_t loc = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        h[u] = u < q && b0 + u < (int)B ? hv[b0 + u] : 0ull;
        loc += h[u];
      }
      uint64_t v = wave_incl_scan<uint64_t>(loc) - loc;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v += h[u];
        if (u < q && b0 + u < (int)B) hv[b0 + u] = v;
      }
      wave_lds_sync();
      V = hv[code];  // code < B for every lane (a lane without a row has row 0's)
      prev_in_lds = true;
    }
    if (valid) {
      const uint32_t NL = packed_n(V);
      if (NL < N) {
        const int64_t SL = packed_s(V, NL);
        const double sc = N < 512u ? split_score32((int32_t)SL, NL, (int32_t)S - (int32_t)SL, N - NL)
                                   : split_score(SL, NL, S - SL, N - NL);
        if (sc > best) {
          best = sc;
          best_ib = (i << 8) | (int32_t)code;
        }
      }
    }
  }
  const ArgMax am = wave_argmax(best, best_ib);
  const bool split = am.score >= 0.0 && am.score - parent_score(S, N) > 0.0;
  const uint32_t col = split ? (uint32_t)s_cand[am.key >> 8] : 0u, bin = (uint32_t)am.key & 0xFF;
  const bool left = split && valid && rowp[col] <= bin;
  small_finish<kWave>(x, k, true, lane, 0, split, col, bin, valid, left, e, start);
}

// Scan one column's histogram of packed bins (B <= 256 bins) with a wave: lane
// l owns bins [l q, l q + q) with q = ceil(B / 64) (so a 64-bin column takes one
// bin per lane); prefix sums give the left side of every split b <= B-2.
// Returns the wave's best (max score, lowest bin) in every lane; the left sums
// oNL, oSL of that split are valid in lane `am.lane`.
__device__ __forceinline__ ArgMax scan_packed(const uint64_t* hv, int B, uint32_t N, int64_t S, uint32_t& oNL,
                                              int64_t& oSL) {
  const int lane = (int)lane_id();
  if (B <= kWave) {  // one bin per lane
    const uint64_t h = lane < B ? hv[lane] : 0ull;
    const uint64_t v = N < 512u ? scan_packed_small(h) : wave_incl_scan<uint64_t>(h);
    double lbest = -1.0;
    oNL = 0;
    oSL = 0;
    // an empty bin repeats the previous split, which already won any tie
    if (h != 0 && lane <= B - 2) {
      const uint32_t NL = packed_n(v);
      if (NL < N) {
        const int64_t SL = packed_s(v, NL);
        lbest = N < 512u ? split_score32((int32_t)SL, NL, (int32_t)S - (int32_t)SL, N - NL)
                         : split_score(SL, NL, S - SL, N - NL);
        oNL = NL;
        oSL = SL;
      }
    }
    return wave_argmax_lane_ordered(lbest, lbest >= 0.0 ? lane : INT_MAX);
  }
  const int q = (B + kWave - 1) / kWave;
  const int b0 = lane * q;
  uint64_t h[4];
  uint64_t loc = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    h[u] = u < q && b0 + u < B ? hv[b0 + u] : 0ull;
    loc += h[u];
  }
  uint64_t v = (N < 512u ? scan_packed_small(loc) : wave_incl_scan<uint64_t>(loc)) - loc;
  double lbest = -1.0;
  int32_t lbin = INT_MAX;
  oNL = 0;
  oSL = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int b = b0 + u;
    // an empty bin repeats the previous split, which already won any tie
    if (u >= q || h[u] == 0) continue;
    v += h[u];
    const uint32_t NL = packed_n(v);
    if (b <= B - 2 && NL < N) {
      const int64_t SL = packed_s(v, NL);
      const double s = N < 512u ? split_score32((int32_t)SL, NL, (int32_t)S - (int32_t)SL, N - NL)
                                : split_score(SL, NL, S - SL, N - NL);
      if (s > lbest) {
        lbest = s;
        lbin = b;
        oNL = NL;
        oSL = SL;
      }
    }
  }
  // lane l's bins precede lane l+1's: the lowest lane with the best score holds
  // the lowest best bin
  return wave_argmax_lane_ordered(lbest, lbin);
}

// Large nodes: one wave per (node, up to four consecutive candidate columns),
// one LDS histogram per column: the node's entries are read once for all of
// them and the columns' code gathers overlap.
__device__ __forceinline__ void big_task(const Ctx& x, uint32_t j, int ci0, WaveHist& L) {
  constexpr int G = 4;
  const GrowArgs& a = *x.a;
  const int lane = (int)lane_id();
  const int mtry = x.T->mtry;
  const int gn = min(a.big_cols, mtry - ci0);  // columns of this task
  const int gs = a.big_stride;
  const NodeDesc d = x.sc.big[j];
  const uint32_t start = rfl(d.start);
  const uint32_t end = start + rfl(d.len);
  const uint32_t N = rfl(d.N);
  const int64_t S = d.S;
  const uint32_t* bt = x.sc.btask + (size_t)j * mtry + ci0;
  int c[G];
#pragma unroll
  for (int g = 0; g < G; ++g) c[g] = g < gn ? (int)(rfl(bt[g]) & 0xFFu) : 0;
  uint64_t* hv = L.hv;
  for (int b = lane; b < gn * gs; b += kWave) hv[b] = 0;
  wave_lds_sync();
  // two rows per lane in flight: entries, then their codes in every column,
  // then the atomics
  constexpr int U = 2;
  for (uint32_t p0 = start + lane; p0 < end; p0 += U * kWave) {
    uint64_t e[U];
    uint32_t code[U][G];
#pragma unroll
    for (int u = 0; u < U; ++u) e[u] = p0 + u * kWave < end ? x.buf[p0 + u * kWave] : 0ull;
    // every lane loads the task's gn codes under a wave-uniform condition only:
    // past the node's end the entry is 0 (row 0), whose codes are not added
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint8_t* rp = a.rcodes + (size_t)entry_row(e[u]) * a.rC;
#pragma unroll
      for (int g = 0; g < G; ++g) code[u][g] = g < gn ? gload(rp + c[g]) : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + u * kWave < end) {
        const uint32_t w = entry_w(e[u]);
        const uint64_t v = pack_ns(w, (int64_t)w * entry_y(e[u]));
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (g < gn) atomicAdd((unsigned long long*)&hv[g * gs + (int)code[u][g]], (unsigned long long)v);
      }
    }
  }
  wave_lds_sync();
#pragma unroll 1
  for (int g = 0; g < gn; ++g) {
    const uint32_t t = rfl(bt[g]);
    uint32_t NL;
    int64_t SL;
    const ArgMax am = scan_packed(hv + g * gs, (int)(t >> 8), N, S, NL, SL);
    if (lane == am.lane) {
      Rec r;
      r.score = am.score;
      r.SL = SL;
      r.NL = NL;
      r.colbin = ((t & 0xFFu) << 8) | (uint32_t)(am.score >= 0.0 ? am.key : 0);
      x.sc.recs[(size_t)j * mtry + ci0 + g] = r;
    }
  }
  wave_lds_sync();
}

// A split decision: the column and bin, and the left child's weight and sum.
struct Decision {
  bool split;
  uint32_t col, bin, NL;
  int64_t SL;
  uint32_t cand;  // the split column's position among the node's candidates
};

// Decide a large or wide node from its per-column records (columns ascending:
// keep the first strictly greater score).
__device__ __forceinline__ Decision decide_from_recs(const Rec* recs, int mtry, int64_t S, uint32_t N) {
  double best = -1.0;
  int bi = -1;
  for (int i = 0; i < mtry; ++i) {
    const double s = recs[i].score;
    if (s > best) {
      best = s;
      bi = i;
    }
  }
  Decision d{false, 0u, 0u, 0u, 0, 0u};
  if (bi >= 0 && best - parent_score(S, N) > 0.0) {
    const Rec r = recs[bi];
    d = Decision{true, r.colbin >> 8, r.colbin & 0xFFu, r.NL, r.SL, (uint32_t)bi};
  }
  return d;
}

constexpr int kWideMax = 8;  // nodes per workgroup-wide batch

struct Shared {
  uint16_t nbins[256];  // bin count of every column
  uint32_t tmp[17];
  uint64_t tmp64[17];
  uint64_t red[16];
  uint32_t cnt[3 + kSegClasses];  // [1] large, [2] wide, [3..] small nodes per segment width
  uint32_t task;
  uint32_t next_task;  // the split-search tasks' queue head
  // two wide batches (the one being searched and the next): node j's first
  // entry, rows, first chunk, weight, sum, and its candidates at
  // j * round_up(mtry, 8) + i
  uint32_t wstart[2][kWideMax], wlen[2][kWideMax], wcpre[2][kWideMax], wN[2][kWideMax];
  int64_t wS[2][kWideMax];
  alignas(8) uint8_t cand[2][256];
  // the group being grown: its members' task indices, min.node.size, node
  // slots and in-bag bitmaps, and the level at which their trees part (first
  // node id, node count, next free id, entry buffer, levels grown, large and
  // wide nodes)
  int32_t gk, vi;  // members; the member being grown, -1 while their trees agree
  int64_t vmin, vbase;  // its min.node.size and node slot
  int32_t gtask[kGroupMax];
  int32_t gmin[kGroupMax];
  int64_t gbase[kGroupMax];
  int64_t ginbag[kGroupMax];
  uint32_t n_inbag;
  uint32_t f_lo, f_cnt, f_next, f_cur, f_levels, f_big, f_huge;
  uint32_t part;    // this level holds a node that is a leaf for some members only
  uint32_t resume;  // the member grows on from the decisions of the parting level
};

// Metadata of wide batch `bi` (nodes list[0 .. nb)) into buffer bi & 1.
template <int BLOCK>
__device__ __forceinline__ void wide_setup(const Ctx& x, const NodeDesc* list, int nb, int bi, Shared& sh) {
  const int mtry = x.T->mtry, tid = threadIdx.x, q = bi & 1;
  if (tid < nb) {
    const NodeDesc d = list[tid];
    uint32_t first = 0;
    for (int j = 0; j < tid; ++j) first += (list[j].len + kWave - 1) / kWave;
    sh.wstart[q][tid] = d.start;
    sh.wlen[q][tid] = d.len;
    sh.wcpre[q][tid] = first;
    sh.wN[q][tid] = d.N;
    sh.wS[q][tid] = d.S;
  }
  // candidates padded to 8 per node (with the node's last one), read 8 at a time
  const int cst = (mtry + 7) & ~7;
  for (int i = tid; i < nb * cst; i += BLOCK)
    sh.cand[q][i] = x.sc.cand[(size_t)list[i / cst].k * cand_stride(mtry) + min(i % cst, mtry - 1)];
}

// The wide nodes of a level, nb at a time.  Node j of a batch has its rows cut
// into chunks of 64, one wave per chunk, so the candidate columns are uniform
// across a wave.  Each lane reads its row's entry once and, when a row has at
// most 80 codes, the first 80 bytes of its padded code row with five 16-byte
// loads; the
// candidate codes are picked from registers and each is added to the packed
// bin of its (node, column) histogram (hc columns at a time when they do not
// all fit the LDS).  One wave per (node, column) then scans, writes the
// column's record (decided with the other nodes' after the phase) and zeroes
// the bins it read, while the next batch's metadata is staged.
template <int BLOCK>
__device__ __forceinline__ void wide_phase(const Ctx& x, const NodeDesc* list, uint32_t n_wide, int nb_max, int hc, uint32_t rec_base,
                           uint8_t* lds, Shared& sh) {
  constexpr int NW = BLOCK / kWave;
  const GrowArgs& a = *x.a;
  const int mtry = x.T->mtry;
  const int bs = a.bstride;
  const int cst = (mtry + 7) & ~7;
  const size_t sst = (size_t)cand_stride(mtry);
  const int tid = threadIdx.x, wid = tid / kWave, lane = (int)lane_id();
  uint64_t* H = reinterpret_cast<uint64_t*>(lds);
  const bool row_regs = a.C <= 80;
  // the histograms start zeroed; each scan zeroes what it read
  for (uint32_t i = 2 * tid; i < a.union_bytes / 8; i += 2 * BLOCK)
    *reinterpret_cast<uint4*>(H + i) = make_uint4(0u, 0u, 0u, 0u);
  wide_setup<BLOCK>(x, list, (int)min((uint32_t)nb_max, n_wide), 0, sh);
  __syncthreads();
  int bi = 0;
  for (uint32_t h0 = 0; h0 < n_wide; h0 += (uint32_t)nb_max, ++bi) {
    const int nb = (int)min((uint32_t)nb_max, n_wide - h0);
    const NodeDesc* bl = list + h0;
    const int q = bi & 1;
    uint32_t cpre[kWideMax];  // first chunk of node j (uniform)
    uint32_t n_chunks = 0;
#pragma unroll
    for (int j = 0; j < kWideMax; ++j) {
      cpre[j] = n_chunks;
      n_chunks += j < nb ? (bl[j].len + kWave - 1) / kWave : 0u;
    }
    // node of chunk ch: the number of later nodes' first chunks <= ch
    auto node_of = [&](uint32_t ch) {
      int j = 0;
#pragma unroll
      for (int jj = 1; jj < kWideMax; ++jj) j += (jj < nb && ch >= cpre[jj]) ? 1 : 0;
      return j;
    };
    for (int c0 = 0; c0 < mtry; c0 += hc) {
      const int nc = min(hc, mtry - c0);
      for (uint32_t ch = (uint32_t)wid; ch < n_chunks; ch += NW) {
        const int j = node_of(ch);
        const uint32_t r = (ch - sh.wcpre[q][j]) * kWave + (uint32_t)lane;
        const bool valid = r < sh.wlen[q][j];
        uint64_t v = 0;
        uint32_t row = 0;
        // this entry's slot of the candidate codes the partition reads back
        uint8_t* side_row = x.sc.side + (size_t)(sh.wstart[q][j] + r) * sst;
        if (valid) {
          const uint64_t e = x.buf[sh.wstart[q][j] + r];
          const uint32_t w = entry_w(e);
          v = pack_ns(w, (int64_t)w * entry_y(e));
          row = entry_row(e);
        }
        const uint8_t* cj = sh.cand[q] + j * cst + c0;
        uint64_t* Hj = H + (size_t)j * nc * bs;
        if (row_regs) {
          // five unconditional loads: the padded copy has 64 bytes of slack after
          // its last row, and a lane without a row reads row 0
          uint32_t rw[20];
          const uint4* rp = reinterpret_cast<const uint4*>(a.codes_p + (size_t)row * a.Cp);
#pragma unroll
          for (int u = 0; u < 5; ++u) {
            const uint4 t = rp[u];
            rw[4 * u] = t.x;
            rw[4 * u + 1] = t.y;
            rw[4 * u + 2] = t.z;
            rw[4 * u + 3] = t.w;
          }
          for (int i0 = 0; i0 < nc; i0 += 8) {
            const uint64_t c8 = *reinterpret_cast<const uint64_t*>(cj + i0);
            const uint32_t lo = rfl((uint32_t)c8), hi = rfl((uint32_t)(c8 >> 32));
            uint32_t sv0 = 0, sv1 = 0;  // the eight codes, for the partition
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const uint32_t col = ((u < 4 ? lo : hi) >> (8 * (u & 3))) & 0xFFu;
              const uint32_t code = (rw[col >> 2] >> (8 * (col & 3))) & 0xFFu;
              if (u < 4)
                sv0 |= code << (8 * u);
              else
                sv1 |= code << (8 * (u - 4));
              if (valid && i0 + u < nc)
                atomicAdd((unsigned long long*)&Hj[(i0 + u) * bs + (int)code], (unsigned long long)v);
            }
            if (valid) *reinterpret_cast<uint2*>(side_row + c0 + i0) = make_uint2(sv0, sv1);
          }
        } else {
          const uint8_t* rp = a.rcodes + (size_t)row * a.rC;
          for (int i0 = 0; i0 < nc; i0 += 8) {
            const uint64_t c8 = *reinterpret_cast<const uint64_t*>(cj + i0);
            uint32_t cd[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) cd[u] = valid ? rp[(uint32_t)(c8 >> (8 * u)) & 0xFFu] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (valid && i0 + u < nc)
                atomicAdd((unsigned long long*)&Hj[(i0 + u) * bs + (int)cd[u]], (unsigned long long)v);
            if (valid)
              *reinterpret_cast<uint2*>(side_row + c0 + i0) =
                  make_uint2(cd[0] | cd[1] << 8 | cd[2] << 16 | cd[3] << 24, cd[4] | cd[5] << 8 | cd[6] << 16 | cd[7] << 24);
          }
        }
      }
      __syncthreads();
      for (int t = wid; t < nb * nc; t += NW) {
        const int j = t / nc, i = t % nc;
        const int c = sh.cand[q][j * cst + c0 + i];
        const int B = a.n_bins[c];
        uint64_t* hv = H + (size_t)t * bs;
        uint32_t NL;
        int64_t SL;
        const ArgMax am = scan_packed(hv, B, sh.wN[q][j], sh.wS[q][j], NL, SL);
        if (lane == am.lane) {
          Rec rc;
          rc.score = am.score;
          rc.SL = SL;
          rc.NL = NL;
          rc.colbin = ((uint32_t)c << 8) | (uint32_t)(am.score >= 0.0 ? am.key : 0);
          x.sc.recs[(size_t)(rec_base + h0 + j) * mtry + c0 + i] = rc;
        }
        // zero the column's bins, four per lane (the scan's reads are done)
        if (4 * lane < B) *reinterpret_cast<uint4*>(hv + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
        if (4 * lane + 2 < B) *reinterpret_cast<uint4*>(hv + 4 * lane + 2) = make_uint4(0u, 0u, 0u, 0u);
      }
      // the next batch's metadata goes to the other buffer meanwhile
      if (c0 + hc >= mtry && h0 + (uint32_t)nb_max < n_wide)
        wide_setup<BLOCK>(x, list + h0 + nb_max, (int)min((uint32_t)nb_max, n_wide - h0 - nb_max), bi + 1, sh);
      __syncthreads();
    }
  }
}

// One wave per chunk of 64 entries of a split node: the lanes that go left take
// consecutive slots from the left cursor in lane order, the others from the
// right cursor, one atomic each; the left side's sum of w y^2 is added up on
// the way.  Rows of leaves are not touched again.  Four chunks per wave are in
// flight at a time, so that their dependent loads (chunk, entry, code)
// overlap.  `cur` is in LDS or in global memory (inlined once for each).
template <int BLOCK, bool WIDE>
__device__ __forceinline__ void partition_level(const Ctx& x, uint64_t* __restrict__ out, Cursor* cur,
                                                uint32_t n_chunks) {
  constexpr int NW = BLOCK / kWave;
  constexpr int UP = 4;
  const GrowArgs& a = *x.a;
  const int lane = (int)lane_id();
  const size_t sst = (size_t)cand_stride(x.T->mtry);
  for (uint32_t c0 = threadIdx.x / kWave; c0 < n_chunks; c0 += UP * NW) {
    uint32_t rk[UP], col[UP], bin[UP], sci[UP], pos[UP];
    uint64_t e[UP];
    bool mv[UP], go_left[UP];
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      const uint32_t ch = c0 + (uint32_t)(u * NW);
      const uint4 cw = ch < n_chunks ? x.sc.chunks[ch] : make_uint4(0u, 0u, 0u, 0u);
      const uint32_t p0 = rfl(cw.x), en = rfl(cw.y), cb = rfl(cw.w);
      rk[u] = rfl(cw.z);
      col[u] = cb & 0xFFu;
      bin[u] = (cb >> 8) & 0xFFu;
      sci[u] = cb >> 16;
      pos[u] = p0 + (uint32_t)lane;
      mv[u] = pos[u] < en;
      e[u] = mv[u] ? x.buf[pos[u]] : 0ull;
    }
    // the split column's code: beside the entry when a wide batch searched the
    // node (candidate index + 1 in the chunk word), else from the row's codes
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      uint32_t code = 0;
      if (mv[u]) {
        if constexpr (WIDE)
          code = sci[u] ? x.sc.side[(size_t)pos[u] * sst + (sci[u] - 1u)]
                        : a.rcodes[(size_t)entry_row(e[u]) * a.rC + col[u]];
        else
          code = a.rcodes[(size_t)entry_row(e[u]) * a.rC + col[u]];
      }
      go_left[u] = mv[u] && code <= bin[u];
    }
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      if (c0 + (uint32_t)(u * NW) >= n_chunks) break;
      const uint64_t lm = __ballot(go_left[u]), rm = __ballot(mv[u] && !go_left[u]);
      const uint64_t below = (1ull << lane) - 1ull;
      uint32_t bl = 0, br = 0;
      if (lane == 0) {
        const uint32_t nl = (uint32_t)__popcll(lm), nr = (uint32_t)__popcll(rm);
        if (nl) bl = atomicAdd(&cur[rk[u]].L, nl);
        if (nr) br = atomicSub(&cur[rk[u]].R, nr) - nr;
      }
      bl = read_lane(bl, 0);
      br = read_lane(br, 0);
      if (mv[u]) out[go_left[u] ? bl + (uint32_t)__popcll(lm & below) : br + (uint32_t)__popcll(rm & below)] = e[u];
      const int64_t y = entry_y(e[u]);
      const uint64_t q = wave_sum(go_left[u] ? (uint64_t)((int64_t)entry_w(e[u]) * y * y) : 0ull);
      if (lane == 0 && q != 0) atomicAdd((unsigned long long*)&cur[rk[u]].q, (unsigned long long)q);
    }
  }
}

// Bootstrap multiplicities of a tree's n training rows into cnt[0 .. n): n
// draws with replacement, draw i = floor(r_i n / 2^64) for the words r_i of
// the Philox stream (seed, tag 0, 0, tree) (every row once without
// bootstrap).  `cnt` is in LDS or in global memory (inlined once for each).
template <int BLOCK>
__device__ __forceinline__ void bootstrap_counts(const TreeTask& T, int64_t n, uint32_t* cnt) {
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < n; i += BLOCK) cnt[i] = T.bootstrap ? 0u : 1u;
  __syncthreads();
  if (T.bootstrap) {
    const int64_t nblk = (n + 3) / 4;
    for (int64_t b = tid; b < nblk; b += BLOCK) {
      const U64x4 r = philox4x64_10((uint64_t)b, kTagBootstrap, 0, (uint64_t)T.tree, T.seed, 0);
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (4 * b + w < n) atomicAdd(&cnt[scale_draw(r.w[w], (uint32_t)n)], 1u);
    }
    __syncthreads();
  }
}

// The trees of one group: K tasks that differ only in min.node.size (sh.gtask,
// by min.node.size ascending; a lone task is a group of one), T being the
// first.  Their trees agree node for node down to the first level holding an
// open node whose leaf rule depends on min.node.size (more weight than the
// smallest value, at most the largest, and not pure), since every other step
// (bootstrap, candidate draws by node id, searches, child ids) is the same.
// Those levels, and the split searches of the parting level itself, are done
// once, with the smallest value (every node open for some member is searched,
// and a search does not depend on min.node.size).  The parting level's state
// is then put aside as the searches left it, and each member in turn grows its
// own tree on from its decisions: the nodes of at most its min.node.size are
// made leaves, the shared levels' node words are copied into its slot.  The
// work counters count the work done: the shared levels, searches included,
// count for the group's first member.
// WIDE: the launch may hold nodes above the wide limit (the kernel without
// the wide-batch phase is compiled separately, so that small training sets
// keep its leaner register allocation).  GROUPED: the launch has groups (the
// kernels of launches without compile the group logic out, which keeps their
// register allocation as it was).
template <int BLOCK, bool WIDE, bool GROUPED>
__device__ __forceinline__ void grow_group(const GrowArgs& a, const TreeTask& T, const Scratch& sc, uint8_t* lds, Shared& sh) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, wid = tid / kWave, lane = (int)lane_id();
  const int64_t n = T.n_train;
  const int32_t* train = T.train_off >= 0 ? a.train_rows + T.train_off : nullptr;
  const int mtry = T.mtry;

  // 1. bootstrap multiplicities, counted in the LDS union area (free until the
  // first level) when the training set fits it, else in scratch
  const bool lds_cnt = n <= (int64_t)(a.union_bytes / 4u);
  uint32_t* const cnt_lds = reinterpret_cast<uint32_t*>(lds);
  if (lds_cnt)
    bootstrap_counts<BLOCK>(T, n, cnt_lds);
  else
    bootstrap_counts<BLOCK>(T, n, sc.cnt);
  // in-bag entries and root sums; each thread takes eight rows per pass,
  // strided by the block, so a pass costs one workgroup scan (the order of the
  // entries is free: every later sum over them is exact)
  uint32_t n_inbag = 0;
  uint64_t N0 = 0, Q0 = 0;
  int64_t S0 = 0;
  constexpr int R = 8;
  for (int64_t base = 0; base < n; base += (int64_t)R * BLOCK) {
    uint32_t c[R];
    uint32_t mine = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + (int64_t)r * BLOCK + tid;
      c[r] = i < n ? (lds_cnt ? cnt_lds[i] : sc.cnt[i]) : 0u;
      mine += c[r] > 0 ? 1u : 0u;
      // in-bag bitmap: this wave's 64 consecutive rows form one word
      const uint64_t bits = __ballot(c[r] > 0);
      const int64_t wbase = base + (int64_t)r * BLOCK + (int64_t)(tid / kWave) * kWave;
      if (lane_id() == 0 && T.inbag_off >= 0 && wbase < n) {
        if (GROUPED)
          for (int v = 0; v < sh.gk; ++v) a.inbag[sh.ginbag[v] + wbase / kWave] = bits;
        else
          a.inbag[T.inbag_off + wbase / kWave] = bits;
      }
    }
    uint32_t total;
    uint32_t pos = block_exscan<BLOCK>(mine, sh.tmp, total) + n_inbag;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (c[r] > 0) {
        const int64_t i = base + (int64_t)r * BLOCK + tid;
        const uint32_t row = train ? (uint32_t)train[i] : (uint32_t)i;
        const int64_t y = a.y_fp[row];
        sc.L0.buf[pos++] = entry_pack(row, c[r], y);
        N0 += c[r];
        S0 += (int64_t)c[r] * y;
        Q0 += (uint64_t)((int64_t)c[r] * y * y);
      }
    }
    n_inbag += total;
  }
  N0 = block_sum<BLOCK, uint64_t>(N0, sh.red);
  S0 = (int64_t)block_sum<BLOCK, uint64_t>((uint64_t)S0, sh.red);
  Q0 = block_sum<BLOCK, uint64_t>(Q0, sh.red);
  if (tid == 0) {
    sc.L0.mstart[0] = 0;
    sc.L0.mend[0] = n_inbag;
    sc.L0.mN[0] = (uint32_t)N0;
    sc.L0.mS[0] = S0;
    sc.L0.mQ[0] = Q0;
  }
  if (tid < 3 + kSegClasses) sh.cnt[tid] = 0;
  if (tid == 0) {
    sh.next_task = NW;
    sh.n_inbag = n_inbag;
    sh.vi = sh.gk > 1 ? -1 : 0;
    sh.vmin = sh.gmin[0];
    sh.vbase = sh.gbase[0];
    sh.part = 0;
    sh.resume = 0;
  }
  __syncthreads();

  // threads that draw candidates each own a C-byte row of the LDS union area
  const int n_draw = min(BLOCK, (int)(a.union_bytes / (uint32_t)a.C));
  const uint32_t draw_q = ((uint32_t)n_draw * (uint32_t)a.C + 15u) & ~15u;  // the draw queue, after the rows
  // (the member being grown, its min.node.size and node slot are kept in the
  // LDS, which spares registers across the level loop)
  uint32_t level_lo = 0, level_cnt = 1, next_id = 1;
  int cur = 0;
  uint64_t work_rows = 0, work_nodes = 0, work_part = 0, levels = 0, work_hist = 0;
  for (;;) {
    while (level_cnt > 0) {
      const Level2 C = cur ? sc.L1 : sc.L0;  // this level
      const Level2 X = cur ? sc.L0 : sc.L1;  // the next level
      const Ctx x{&a, &T, sc, C.buf, X.buf, C.mstart, C.mend, C.mN, C.mS, C.mQ};
      // (a) - (c) are skipped by a member that grows on from the parting level
      if (!GROUPED || !sh.resume) {
        ++levels;
        // (a) leaf rules, candidate draws, tiers (the tier counts and the task
        // queue head were reset before the level began).  A one-wave workgroup
        // queues its open nodes in the LDS after the draw rows (node and large-node
        // index, 128 entries) and draws them 64 at a time, so that a level whose
        // open nodes are sparse among its nodes runs the draws fewer times.
        const bool queue_draws = BLOCK == kWave && n_draw == kWave && draw_q + 1024u <= a.union_bytes;
        if (tid < n_draw) {
          const int64_t min_node = GROUPED ? sh.vmin : (int64_t)T.min_node;
          // while the members' trees agree: an open node of at most the largest
          // member's min.node.size is a leaf for some members only
          const int64_t m_part = GROUPED && sh.vi < 0 ? (int64_t)sh.gmin[sh.gk - 1] : -1;
          uint32_t* const qk = reinterpret_cast<uint32_t*>(lds + draw_q);
          uint32_t* const qj = qk + 128;
          uint32_t q_head = 0, q_tail = 0;
          auto draw_queued = [&](uint32_t n_q) {
            if ((uint32_t)tid < n_q) {
              const uint32_t e = (q_head + (uint32_t)tid) & 127u;
              const uint32_t k = qk[e], j1 = qj[e];
              draw_candidates(lds + tid, n_draw, T.seed, level_lo + k, (uint32_t)T.tree, a.C, mtry,
                              sc.cand + (size_t)k * cand_stride(mtry), j1 ? sc.btask + (size_t)(j1 - 1) * mtry : nullptr,
                              sh.nbins);
            }
            q_head += n_q;
          };
          const uint32_t k_end = queue_draws ? (level_cnt + kWave - 1) / kWave * kWave : level_cnt;
          for (uint32_t k = tid; k < k_end; k += n_draw) {
            bool open = false;
            uint32_t j1 = 0;  // large node j: j + 1
            uint32_t* bt = nullptr;
            if (k < level_cnt) {
              const uint32_t N = x.mN[k];
              const int64_t S = x.mS[k];
              const uint64_t Q = x.mQ[k];
              const uint32_t st = x.mstart[k];
              const uint32_t len = x.mend[k] - st;
              if ((int64_t)N <= min_node || node_is_pure(N, S, Q)) {
                sc.status[k] = kLeaf;
              } else {
                open = true;
                if (GROUPED && (int64_t)N <= m_part) sh.part = 1u;
                work_rows += len;
                ++work_nodes;
                // nodes above 32 rows add each row to an LDS bin per candidate column
                if (len > 32) work_hist += (uint64_t)len * (uint64_t)mtry;
                if (len <= kSegMax) {
                  const int cls = len <= 4 ? 0 : len <= 8 ? 1 : len <= 16 ? 2 : len <= 32 ? 3 : 4;
                  sc.status[k] = kSmall;
                  NodeDesc* list = cls == 0   ? sc.seg[0]
                                   : cls == 1 ? sc.seg[1]
                                   : cls == 2 ? sc.seg[2]
                                   : cls == 3 ? sc.seg[3]
                                              : sc.seg[4];
                  list[atomicAdd(&sh.cnt[3 + cls], 1u)] = NodeDesc{k, st, len, N, S};
                } else if (!WIDE || (int32_t)len <= a.huge_min) {
                  sc.status[k] = kBig;
                  const uint32_t j = atomicAdd(&sh.cnt[1], 1u);
                  sc.big[j] = NodeDesc{k, st, len, N, S};
                  sc.ridx[k] = j;
                  j1 = j + 1;
                  bt = sc.btask + (size_t)j * mtry;  // each (node, column) task's column and bin count
                } else {
                  sc.status[k] = kHuge;
                  const uint32_t h = atomicAdd(&sh.cnt[2], 1u);
                  sc.huge[h] = NodeDesc{k, st, len, N, S};
                  sc.ridx[k] = h;
                }
              }
            }
            if (queue_draws) {
              const uint64_t om = __ballot(open);
              if (open) {
                const uint32_t e = (q_tail + (uint32_t)__popcll(om & ((1ull << lane) - 1ull))) & 127u;
                qk[e] = k;
                qj[e] = j1;
              }
              q_tail += (uint32_t)__popcll(om);
              wave_lds_sync();
              if (q_tail - q_head >= (uint32_t)kWave) {
                draw_queued(kWave);
                wave_lds_sync();
              }
            } else if (open) {
              draw_candidates(lds + tid, n_draw, T.seed, level_lo + k, (uint32_t)T.tree, a.C, mtry,
                              sc.cand + (size_t)k * cand_stride(mtry), bt, sh.nbins);
            }
          }
          if (queue_draws && q_tail > q_head) draw_queued(q_tail - q_head);
        }
        __syncthreads();
        const uint32_t n_big = sh.cnt[1], n_huge = sh.cnt[2];
        // (b) wide nodes, in batches, with the whole workgroup
        if (WIDE && n_huge > 0) {
          const int per_node = mtry * a.bstride * 8;
          int nb = 1, hc = mtry;
          if (per_node <= (int)a.union_bytes)
            nb = min(min(kWideMax, 256 / ((mtry + 7) & ~7)), (int)a.union_bytes / per_node);
          // (records of wide node j go after the large nodes', at n_big + j)
          else  // column chunks of a multiple of 8 (the LDS holds at least 8 columns)
            hc = max(8, (int)a.union_bytes / (a.bstride * 8) / 8 * 8);
          wide_phase<BLOCK>(x, sc.huge, n_huge, nb, hc, n_big, lds, sh);
        }
        // (c) large-node columns and small-node segments, one wave each; a wave
        // takes its next task from the queue head when it starts one (their costs
        // differ widely, so a fixed deal would leave waves idle at the barrier)
        {
          const uint32_t per_big = (uint32_t)((mtry + a.big_cols - 1) / a.big_cols);
          const uint32_t n_big_tasks = n_big * per_big;
          uint32_t first[kSegClasses + 1];
          first[0] = n_big_tasks;
          for (int c = 0; c < kSegClasses; ++c) {
            const uint32_t per_wave = (uint32_t)(kWave >> (2 + c));
            first[c + 1] = first[c] + (sh.cnt[3 + c] + per_wave - 1) / per_wave;
          }
          WaveHist& wl = *reinterpret_cast<WaveHist*>(lds + (size_t)wid * a.wave_bytes);
          for (uint32_t t = wid; t < first[kSegClasses];) {
            uint32_t t_next = 0;
            if (lane == 0) t_next = atomicAdd(&sh.next_task, 1u);
            if (t < n_big_tasks)
              big_task(x, t / per_big, (int)(t % per_big) * a.big_cols, wl);
            else if (t < first[1])
              small_task<4>(x, sc.seg[0], t - first[0], sh.cnt[3], wl);
            else if (t < first[2])
              small_task<8>(x, sc.seg[1], t - first[1], sh.cnt[4], wl);
            else if (t < first[3])
              small_task<16>(x, sc.seg[2], t - first[2], sh.cnt[5], wl);
            else if (t < first[4])
              small_task<32>(x, sc.seg[3], t - first[3], sh.cnt[6], wl);
            else
              rank_task(x, sc.seg[4], t - first[4], sh.cnt[7], wl);
            t = read_lane(t_next, 0);
          }
        }
        __syncthreads();
        if (GROUPED && sh.part) {
          // the members' trees part at this level: put its searched state aside
          // (the open nodes' entries lie in [0, n_inbag)); the first member goes on
          const uint32_t ni = sh.n_inbag;
          for (uint32_t i = tid; i < ni; i += BLOCK) {
            sc.SN.L.buf[i] = C.buf[i];
            sc.SN.nbuf[i] = X.buf[i];
          }
          for (uint32_t k = tid; k < level_cnt; k += BLOCK) {
            sc.SN.L.mstart[k] = C.mstart[k];
            sc.SN.L.mend[k] = C.mend[k];
            sc.SN.L.mN[k] = C.mN[k];
            sc.SN.L.mS[k] = C.mS[k];
            sc.SN.L.mQ[k] = C.mQ[k];
            sc.SN.status[k] = sc.status[k];
            sc.SN.ridx[k] = sc.ridx[k];
            sc.SN.dcol[k] = sc.dcol[k];
            sc.SN.dbin[k] = sc.dbin[k];
            sc.SN.dNL[k] = sc.dNL[k];
            sc.SN.dSL[k] = sc.dSL[k];
            sc.SN.dcnt[k] = sc.dcnt[k];
            sc.SN.dQL[k] = sc.dQL[k];
          }
          for (uint32_t i = tid; i < (n_big + n_huge) * (uint32_t)mtry; i += BLOCK) sc.SN.recs[i] = sc.recs[i];
          if (WIDE && n_huge > 0) {
            const uint4* src = reinterpret_cast<const uint4*>(sc.side);
            uint4* dst = reinterpret_cast<uint4*>(sc.SN.side);
            for (uint32_t i = tid; i < ni * (uint32_t)cand_stride(mtry) / 16u; i += BLOCK) dst[i] = src[i];
          }
          __syncthreads();  // (every thread has read the flag)
          if (tid == 0) {
            sh.part = 0;
            sh.vi = 0;
            sh.f_lo = level_lo;
            sh.f_cnt = level_cnt;
            sh.f_next = next_id;
            sh.f_cur = (uint32_t)cur;
            sh.f_levels = (uint32_t)levels;
            sh.f_big = n_big;
            sh.f_huge = n_huge;
          }
        }
      }
      const uint32_t n_big = sh.cnt[1];
      // (d) the large and wide nodes' decisions from their records (the wide
      // nodes' records follow the large nodes'), then (e) breadth-first child
      // ids, node words, children's sums and cursors, and the partition's chunks
      // of 64 entries of every split node that is not placed yet.  The cursors
      // live in the LDS union area (free until the next level) when the level's
      // nodes fit it, else in scratch.
      const bool lds_cur = level_cnt <= a.union_bytes / (uint32_t)sizeof(Cursor);
      const int64_t base_node = GROUPED ? sh.vbase : T.node_base;
      Cursor* lcur = reinterpret_cast<Cursor*>(lds);
      uint32_t n_split = 0, n_chunks = 0;
      for (uint32_t b0 = 0; b0 < level_cnt; b0 += BLOCK) {
        const uint32_t k = b0 + tid;
        const bool in = k < level_cnt;
        uint8_t stk = in ? sc.status[k] : kLeaf;
        Decision dc{false, 0u, 0u, 0u, 0, 0u};
        // a wide node's rows carry their candidate codes (candidate index + 1 in
        // the partition's chunk word; 0 = read the row's code)
        uint32_t side_ci = 0;
        if (stk == kBig || stk == kHuge) {
          const uint32_t ri = sc.ridx[k] + (stk == kHuge ? n_big : 0u);
          dc = decide_from_recs(sc.recs + (size_t)ri * mtry, mtry, x.mS[k], x.mN[k]);
          if (WIDE && stk == kHuge) side_ci = dc.cand + 1u;
          stk = dc.split ? kSplit : kLeaf;
        } else if (stk == kSplitDone) {
          dc = Decision{true, sc.dcol[k], sc.dbin[k], sc.dNL[k], sc.dSL[k], 0u};
        }
        const bool split = stk == kSplit || stk == kSplitDone;
        // (the small nodes' rows were placed by their searches)
        const uint32_t nch = stk == kSplit ? (x.mend[k] - x.mstart[k] + kWave - 1) / kWave : 0u;
        // split ranks in the low half, chunk offsets in the high half
        uint64_t tot;
        const uint64_t ex = block_exscan64<BLOCK>((split ? 1ull : 0ull) | ((uint64_t)nch << 32), sh.tmp64, tot);
        const uint32_t total = (uint32_t)tot, ctotal = (uint32_t)(tot >> 32);
        const uint32_t r = (uint32_t)ex + n_split;
        const uint32_t cfirst = (uint32_t)(ex >> 32) + n_chunks;
        // (the bounds below hold by construction; the guards keep a broken
        // invariant from writing outside the scratch arrays)
        if (nch > 0 && (uint64_t)cfirst + nch <= (uint64_t)(a.n_cap / 64 + a.n_cap / 2 + 2)) {
          const uint32_t st = x.mstart[k], en = x.mend[k], cb = dc.col | (dc.bin << 8) | (side_ci << 16);
          for (uint32_t c = 0; c < nch; ++c) sc.chunks[cfirst + c] = make_uint4(st + c * kWave, en, r, cb);
        }
        if (in) {
          const uint32_t node = level_lo + k;
          const uint32_t N = x.mN[k];
          const int64_t S = x.mS[k];
          if (split && (int64_t)2 * r + 1 >= a.n_cap) {
            atomicOr(a.status, kStatusCapacity);
          } else if (split) {
            const uint32_t left = next_id + 2 * r;
            if ((int64_t)left + 1 < T.capacity) {
              a.nodes[base_node + node] = node_split(dc.col, dc.bin, left);
            } else {
              atomicOr(a.status, kStatusCapacity);
            }
            const uint32_t st = x.mstart[k], en = x.mend[k];
            work_part += en - st;
            // a placed node's boundary is known; its cursor is marked done
            const bool done = stk == kSplitDone;
            const Cursor c0{done ? 0xFFFFFFFFu : st, en, 0ull};
            if (lds_cur)
              lcur[r] = c0;
            else
              sc.cur[r] = c0;
            if (done) {
              const uint32_t b = st + sc.dcnt[k];
              const uint64_t QL = sc.dQL[k];
              X.mend[2 * r] = b;
              X.mstart[2 * r + 1] = b;
              X.mQ[2 * r] = QL;
            }
            const uint32_t NL = dc.NL;
            const int64_t SL = dc.SL;
            X.mstart[2 * r] = st;
            X.mN[2 * r] = NL;
            X.mS[2 * r] = SL;
            X.mend[2 * r + 1] = en;
            X.mN[2 * r + 1] = N - NL;
            X.mS[2 * r + 1] = S - SL;
            // the right side's: the parent's, less the left side's when known
            X.mQ[2 * r + 1] = x.mQ[k] - (done ? sc.dQL[k] : 0ull);
          } else {
            a.nodes[base_node + node] = node_leaf(leaf_value(N, S));
          }
          a.node_N[base_node + node] = N;
        }
        n_split += total;
        n_chunks += ctotal;
      }
      __syncthreads();
      if ((int64_t)next_id + 2 * (int64_t)n_split > T.capacity ||
          (int64_t)n_chunks > a.n_cap / 64 + a.n_cap / 2 + 2) {
        // cannot happen for consistent inputs: every child holds an in-bag row
        if (tid == 0) atomicOr(a.status, kStatusCapacity);
        next_id = (uint32_t)T.capacity;
        break;
      }
      // (f) partition the entries of split nodes into their children's segments
      if (lds_cur)
        partition_level<BLOCK, WIDE>(x, X.buf, lcur, n_chunks);
      else
        partition_level<BLOCK, WIDE>(x, X.buf, sc.cur, n_chunks);
      __syncthreads();
      // (g) the boundary between each pair of children, and their sums of w y^2
      for (uint32_t r = tid; r < n_split; r += BLOCK) {
        const Cursor c = lds_cur ? lcur[r] : sc.cur[r];
        if (c.L == 0xFFFFFFFFu) continue;  // placed by its search
        X.mend[2 * r] = c.L;
        X.mstart[2 * r + 1] = c.L;
        X.mQ[2 * r] = c.q;
        X.mQ[2 * r + 1] -= c.q;
      }
      // the next level's tier counts and task queue head
      if (tid < 3 + kSegClasses) sh.cnt[tid] = 0;
      if (tid == 0) {
        sh.next_task = NW;
        if (GROUPED) sh.resume = 0;
      }
      __syncthreads();
      level_lo = next_id;
      level_cnt = 2 * n_split;
      next_id += 2 * n_split;
      cur ^= 1;
    }
    // the tree of member max(vi, 0) is complete
    work_rows = block_sum<BLOCK, uint64_t>(work_rows, sh.red);
    work_nodes = block_sum<BLOCK, uint64_t>(work_nodes, sh.red);
    work_part = block_sum<BLOCK, uint64_t>(work_part, sh.red);
    work_hist = block_sum<BLOCK, uint64_t>(work_hist, sh.red);
    const int vi = GROUPED ? sh.vi : 0, K = GROUPED ? sh.gk : 1;
    const int64_t base_node = GROUPED ? sh.vbase : T.node_base;
    const int v0 = vi < 0 ? 0 : vi;
    // without a parting level every member's tree is the first one's
    const int v1 = vi < 0 ? K : vi + 1;
    for (int v = v0; v < v1; ++v) {
      if (v > v0) {
        const int64_t b = sh.gbase[v];
        for (uint32_t i = tid; i < next_id; i += BLOCK) {
          a.nodes[b + i] = a.nodes[base_node + i];
          a.node_N[b + i] = a.node_N[base_node + i];
        }
      }
      if (tid == 0) {
        const int64_t ti = GROUPED ? sh.gtask[v] : sh.gtask[0];
        a.n_nodes[ti] = (int32_t)next_id;
        int64_t* wk = a.work + kWorkWords * ti;
        const bool first = v == v0;
        wk[0] = first ? (int64_t)work_rows : 0;
        wk[1] = first ? (int64_t)work_nodes : 0;
        wk[2] = first ? (int64_t)work_part : 0;
        wk[3] = (int64_t)levels;
        wk[4] = first ? (int64_t)work_hist : 0;
      }
    }
    if (vi < 0 || vi + 1 == K) break;
    // member vi + 1 grows on from the parting level's decisions: its searched
    // state restored, the nodes of at most its min.node.size made leaves, the
    // shared levels' node words copied into its slot
    const int64_t nbase = sh.gbase[vi + 1], m_v = sh.gmin[vi + 1];
    level_lo = sh.f_lo;
    level_cnt = sh.f_cnt;
    next_id = sh.f_next;
    cur = (int)sh.f_cur;
    levels = sh.f_levels;
    work_rows = work_nodes = work_part = work_hist = 0;
    {
      const uint32_t f_big = sh.f_big, f_huge = sh.f_huge;
      const int64_t b0 = sh.gbase[0];
      for (uint32_t i = tid; i < level_lo; i += BLOCK) {
        a.nodes[nbase + i] = a.nodes[b0 + i];
        a.node_N[nbase + i] = a.node_N[b0 + i];
      }
      const Level2 C = cur ? sc.L1 : sc.L0;
      const Level2 X = cur ? sc.L0 : sc.L1;
      const uint32_t ni = sh.n_inbag;
      for (uint32_t i = tid; i < ni; i += BLOCK) {
        C.buf[i] = sc.SN.L.buf[i];
        X.buf[i] = sc.SN.nbuf[i];
      }
      for (uint32_t k = tid; k < level_cnt; k += BLOCK) {
        const uint32_t N = sc.SN.L.mN[k];
        C.mstart[k] = sc.SN.L.mstart[k];
        C.mend[k] = sc.SN.L.mend[k];
        C.mN[k] = N;
        C.mS[k] = sc.SN.L.mS[k];
        C.mQ[k] = sc.SN.L.mQ[k];
        const uint8_t st = sc.SN.status[k];
        sc.status[k] = (int64_t)N <= m_v ? kLeaf : st;
        sc.ridx[k] = sc.SN.ridx[k];
        sc.dcol[k] = sc.SN.dcol[k];
        sc.dbin[k] = sc.SN.dbin[k];
        sc.dNL[k] = sc.SN.dNL[k];
        sc.dSL[k] = sc.SN.dSL[k];
        sc.dcnt[k] = sc.SN.dcnt[k];
        sc.dQL[k] = sc.SN.dQL[k];
      }
      for (uint32_t i = tid; i < (f_big + f_huge) * (uint32_t)mtry; i += BLOCK) sc.recs[i] = sc.SN.recs[i];
      if (WIDE && f_huge > 0) {
        const uint4* src = reinterpret_cast<const uint4*>(sc.SN.side);
        uint4* dst = reinterpret_cast<uint4*>(sc.side);
        for (uint32_t i = tid; i < ni * (uint32_t)cand_stride(mtry) / 16u; i += BLOCK) dst[i] = src[i];
      }
      __syncthreads();  // (every thread has read the member index)
      if (tid < 3 + kSegClasses) sh.cnt[tid] = tid == 1 ? f_big : tid == 2 ? f_huge : 0u;
    }
    if (tid == 0) {
      sh.next_task = NW;
      sh.vi = vi + 1;
      sh.vmin = m_v;
      sh.vbase = nbase;
      sh.resume = 1;
    }
    __syncthreads();
  }
  (void)wid;
}

// OCC waves per SIMD (at most 512 / OCC VGPRs): the persistent kernel is bound
// by latency, so resident waves can matter more than the registers it spills;
// the kernel with the wide phase keeps four, the other is built for 4, 5 and 6.
template <int BLOCK, bool WIDE, int OCC, bool GROUPED>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(OCC))) void k_grow(GrowArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ Shared sh;
  // a code at or above its column's bin count (flagged by the prepare kernel,
  // which ran before on this stream) would index past a histogram: grow nothing
  // and let the fit report EINVAL
  if (__atomic_load_n(a.status, __ATOMIC_RELAXED) & kStatusBadCode) return;
  Scratch sc;
  carve(&sc, reinterpret_cast<uintptr_t>(a.scratch) + a.scratch_stride * blockIdx.x, a.n_cap, a.mtry_max, WIDE,
        GROUPED);
  for (int c = threadIdx.x; c < a.C; c += BLOCK) sh.nbins[c] = (uint16_t)a.n_bins[c];
  for (;;) {
    if (threadIdx.x == 0) sh.task = atomicAdd(a.queue, 1u);
    __syncthreads();
    const uint32_t g = sh.task;
    if (g >= (uint32_t)a.n_groups) return;
    // the group's members (the host keeps a group within kGroupMax tasks)
    const int32_t gf = GROUPED ? a.group_first[g] : (int32_t)g;
    const int K = GROUPED ? min(a.group_first[g + 1] - gf, kGroupMax) : 1;
    if (threadIdx.x == 0) sh.gk = K;
    if (threadIdx.x < K) {
      const int32_t ti = GROUPED ? a.group_task[gf + threadIdx.x] : (int32_t)g;
      sh.gtask[threadIdx.x] = ti;
      sh.gmin[threadIdx.x] = a.tasks[ti].min_node;
      sh.gbase[threadIdx.x] = a.tasks[ti].node_base;
      sh.ginbag[threadIdx.x] = a.tasks[ti].inbag_off;
    }
    __syncthreads();
    const TreeTask T = a.tasks[rfl((uint32_t)sh.gtask[0])];
    grow_group<BLOCK, WIDE, GROUPED>(a, T, sc, lds, sh);
    __syncthreads();
  }
}

// The grow kernel of this translation unit for a launch shape (block, wide
// phase, waves per SIMD): the kernels for launches with task groups are built
// in a unit of their own (which includes this file with AIWC_GROW_GROUPED set),
// so that the two sets compile in parallel.
#ifndef AIWC_GROW_GROUPED
#define AIWC_GROW_GROUPED 0
#endif
template <int BLOCK>
const void* grow_kernel(bool wide, int occ) {
  constexpr bool G = AIWC_GROW_GROUPED != 0;
  if constexpr (BLOCK < 192) {
    // one- and two-wave workgroups serve deep queues of small trees only
    if (wide) fail(AIWC_RF_EINVAL, "the workgroup-wide phase needs at least 192 threads per workgroup");
  } else {
    if (wide) return reinterpret_cast<const void*>(k_grow<BLOCK, true, 4, G>);
  }
  switch (occ) {
    case 5: return reinterpret_cast<const void*>(k_grow<BLOCK, false, 5, G>);
    case 6: return reinterpret_cast<const void*>(k_grow<BLOCK, false, 6, G>);
    default: return reinterpret_cast<const void*>(k_grow<BLOCK, false, 4, G>);
  }
}

const void* grow_kernel_block(int block, bool wide, int occ) {
  switch (block) {
    case 64: return grow_kernel<64>(wide, occ);
    case 128: return grow_kernel<128>(wide, occ);
    case 192: return grow_kernel<192>(wide, occ);
    case 256: return grow_kernel<256>(wide, occ);
    case 512: return grow_kernel<512>(wide, occ);
    case 1024: return grow_kernel<1024>(wide, occ);
    default: fail(AIWC_RF_EINVAL, "unsupported grow block size");
  }
}

#if AIWC_GROW_GROUPED
}  // namespace

const void* grow_kernel_grouped(int block, bool wide, int occ) { return grow_kernel_block(block, wide, occ); }

}  // namespace aiwc
#else

__global__ void k_init(uint32_t* status, uint32_t* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (status) *status = 0;
    if (queue) *queue = 0;
  }
}

// y -> y_fp = rint(y * 2^16) with range check, and every code < its column's bin count.
__global__ void k_prepare(const uint8_t* codes, int64_t n, int32_t C, const int32_t* n_bins, const double* y,
                          int64_t* y_fp, uint8_t* codes_p, int32_t Cp, uint32_t* status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t bad = 0;
  for (int64_t i = g; i < n; i += stride) {
    const double v = y[i];
    if (!(fabs(v) <= 64.0)) {
      bad |= kStatusBadY;
      y_fp[i] = 0;
    } else {
      y_fp[i] = (int64_t)rint(v * 65536.0);
    }
  }
  const int64_t total = n * C;
  for (int64_t i = g; i < total; i += stride)
    if ((int32_t)codes[i] >= n_bins[i % C]) bad |= kStatusBadCode;
  // the padded copy: row i at i * Cp, zeros after column C - 1
  const int64_t total_p = n * Cp;
  for (int64_t i = g; i < total_p; i += stride) {
    const int64_t row = i / Cp;
    const int32_t c = (int32_t)(i - row * Cp);
    codes_p[i] = c < C ? codes[row * C + c] : 0u;
  }
  if (bad) atomicOr(status, bad);
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Dynamic LDS of the grow kernel: the per-wave histograms, or the packed
// histograms of a batch of wide nodes, or the candidate-draw rows, whichever is
// largest (the three are used in different phases of a level).
struct Layout {
  uint32_t union_bytes;
  uint32_t wave_bytes;
  int32_t bstride;
  int32_t big_stride;  // bins per large-node column histogram (a multiple of 4)
  int32_t big_cols;    // large-node columns per wave task (the wave area holds that many histograms)
};

Layout grow_layout(const GrowConfig& cfg, int32_t mtry_max, int32_t C) {
  Layout L;
  L.bstride = (std::max(cfg.bins_max, 1) + 63) / 64 * 64;
  L.big_stride = (std::max(cfg.bins_max, 1) + 3) / 4 * 4;
  // a wave's histogram, or the staging of its small-node task (the rank task's
  // two bin buffers and candidates take 4096 + mtry bytes)
  const size_t wb = std::max(sizeof(WaveHist), (size_t)4096 + (size_t)mtry_max);
  L.wave_bytes = (uint32_t)((wb + 255) / 256 * 256);
  L.big_cols = (int32_t)std::min<size_t>(4, L.wave_bytes / (8 * (size_t)L.big_stride));
  const size_t waves = (size_t)(cfg.block / kWave) * L.wave_bytes;
  const size_t draw = (size_t)std::min(cfg.block, 256) * (size_t)C;
  size_t wide = 0;
  if (grow_has_wide_phase(cfg)) {
    // by default a quarter of the 128 KiB per 256 threads, so that the
    // workgroups that fit a CU still do
    const size_t want = cfg.wide_bytes > 0 ? (size_t)cfg.wide_bytes : (size_t)cfg.block * 128;
    wide = std::max(std::max(waves, want), (size_t)8 * L.bstride * 8);
  }
  L.union_bytes = (uint32_t)std::max(std::max(waves, wide), draw);
  return L;
}

const void* grow_kernel_for(const GrowConfig& cfg, bool wide, bool grouped) {
  return grouped ? grow_kernel_grouped(cfg.block, wide, cfg.occupancy)
                 : grow_kernel_block(cfg.block, wide, cfg.occupancy);
}

int occupancy(const void* kernel, int block, uint32_t lds) {
  int nb = 0;
  AIWC_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  AIWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, lds));
  return nb;
}

}  // namespace

void launch_init(uint32_t* d_status, uint32_t* d_queue, hipStream_t s) {
  k_init<<<1, 64, 0, s>>>(d_status, d_queue);
  AIWC_HIP(hipGetLastError());
}

void launch_set_i32(int32_t* p, int32_t v, hipStream_t s) {
  k_set_i32<<<1, 64, 0, s>>>(p, v);
  AIWC_HIP(hipGetLastError());
}

size_t grow_scratch_bytes(int64_t n_cap, int32_t mtry_max, bool wide, bool grouped) {
  Scratch s;
  return carve(&s, 0, n_cap, mtry_max, wide, grouped);
}

void launch_prepare(const uint8_t* codes, int64_t n, int32_t C, const int32_t* d_n_bins, const double* y,
                    int64_t* y_fp, uint8_t* codes_p, uint32_t* d_status, hipStream_t s) {
  const int64_t work = n * padded_cols(C);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (work + 255) / 256));
  k_prepare<<<blocks, 256, 0, s>>>(codes, n, C, d_n_bins, y, y_fp, codes_p, padded_cols(C), d_status);
  AIWC_HIP(hipGetLastError());
}

int grow_grid_size(const GrowConfig& cfg, int64_t n_tasks, int32_t mtry_max, int32_t C, bool grouped) {
  const uint32_t lds = grow_layout(cfg, mtry_max, C).union_bytes;
  if (lds > device_info().lds_per_block) fail(AIWC_RF_EINVAL, "grow kernel LDS exceeds the device limit");
  int per_cu = occupancy(grow_kernel_for(cfg, grow_has_wide_phase(cfg), grouped), cfg.block, lds);
  if (per_cu < 1) fail(AIWC_RF_ENOMEM, "grow kernel does not fit the device (LDS or registers)");
  if (cfg.wg_per_cu > 0) per_cu = std::min(per_cu, cfg.wg_per_cu);
  const int64_t slots = (int64_t)device_info().cus * per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(slots, n_tasks));
}

namespace {

GrowArgs grow_args(const GrowConfig& cfg, const GrowLaunch& g, int32_t C, const int32_t* d_n_bins, const int64_t* y_fp,
                   uint32_t* d_status, int32_t mtry_max) {
  GrowArgs a;
  a.codes = g.codes;
  a.C = C;
  a.codes_p = g.codes_p;
  a.Cp = padded_cols(C);
  const bool dense = g.n_cap * (int64_t)C <= (int64_t)1 << 20;
  a.rcodes = dense ? g.codes : g.codes_p;
  a.rC = dense ? C : a.Cp;
  a.n_bins = d_n_bins;
  a.y_fp = y_fp;
  a.train_rows = g.train_rows;
  a.tasks = g.tasks;
  a.n_tasks = g.n_tasks;
  a.group_task = g.group_task;
  a.group_first = g.group_first;
  a.n_groups = g.group_first ? g.n_groups : g.n_tasks;
  a.nodes = g.nodes;
  a.node_N = g.node_N;
  a.n_nodes = g.n_nodes;
  a.work = g.work;
  a.inbag = g.inbag;
  a.queue = g.queue;
  a.status = d_status;
  a.scratch = g.scratch;
  a.n_cap = g.n_cap;
  a.mtry_max = mtry_max;
  a.huge_min = cfg.huge_min;
  a.wide_sums = cfg.wide_sums ? 1 : 0;
  a.scratch_stride = grow_scratch_bytes(g.n_cap, mtry_max, grow_has_wide_phase(cfg), g.group_first != nullptr);
  const Layout L = grow_layout(cfg, mtry_max, C);
  a.union_bytes = L.union_bytes;
  a.wave_bytes = L.wave_bytes;
  a.bstride = L.bstride;
  a.big_stride = L.big_stride;
  a.big_cols = cfg.big_cols > 0 ? std::min(cfg.big_cols, L.big_cols) : L.big_cols;
  return a;
}

int prepare_blocks(int64_t n, int32_t C) {
  const int64_t work = n * padded_cols(C);
  return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (work + 255) / 256));
}

// Executable graphs of fused fits, one per launch shape: the status and queue
// reset, the prepare kernel and the grow launch as three kernel nodes.  A later
// fit of the same shape only replaces the nodes' arguments, once the graph's
// previous launch has finished.
struct GraphKey {
  int device;
  const void* kernel;
  int block, grid, prep_blocks;
  uint32_t lds;
  bool operator<(const GraphKey& o) const {
    return std::tie(device, kernel, block, grid, prep_blocks, lds) <
           std::tie(o.device, o.kernel, o.block, o.grid, o.prep_blocks, o.lds);
  }
};
struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t init = nullptr, prep = nullptr, grow = nullptr;
  hipEvent_t last = nullptr;  // recorded after the latest launch
  uint64_t used = 0;
};
constexpr size_t kMaxGraphs = 16;

std::mutex& graph_mu() {
  static std::mutex* m = new std::mutex();
  return *m;
}
std::map<GraphKey, GraphEntry>& graph_cache() {
  static auto* c = new std::map<GraphKey, GraphEntry>();  // kept until exit
  return *c;
}

hipKernelNodeParams node_params(const void* fn, int grid, int block, uint32_t lds, void** args) {
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof(p));
  p.func = const_cast<void*>(fn);
  p.gridDim = dim3((unsigned)grid);
  p.blockDim = dim3((unsigned)block);
  p.sharedMemBytes = lds;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}

}  // namespace

int effective_big_cols(const GrowConfig& cfg, int32_t mtry_max, int32_t C) {
  const Layout L = grow_layout(cfg, mtry_max, C);
  return cfg.big_cols > 0 ? std::min(cfg.big_cols, L.big_cols) : L.big_cols;
}

void launch_grow(const GrowConfig& cfg, const GrowLaunch& g, int32_t C, const int32_t* d_n_bins, const int64_t* y_fp,
                 uint32_t* d_status, int32_t mtry_max, int grid, hipStream_t s) {
  GrowArgs a = grow_args(cfg, g, C, d_n_bins, y_fp, d_status, mtry_max);
  const void* kernel = grow_kernel_for(cfg, grow_has_wide_phase(cfg), g.group_first != nullptr);
  void* args[] = {&a};
  AIWC_HIP(hipLaunchKernel(kernel, dim3((unsigned)grid), dim3((unsigned)cfg.block), args, a.union_bytes, s));
  AIWC_HIP(hipGetLastError());
}

bool launch_fit_graph(const GrowConfig& cfg, const GrowLaunch& g, const uint8_t* codes, int64_t n, int32_t C,
                      const int32_t* d_n_bins, const double* y, int64_t* y_fp, uint32_t* d_status, int32_t mtry_max,
                      int grid, hipStream_t s) {
  GrowArgs a = grow_args(cfg, g, C, d_n_bins, y_fp, d_status, mtry_max);
  const void* kernel = grow_kernel_for(cfg, grow_has_wide_phase(cfg), g.group_first != nullptr);
  const int pb = prepare_blocks(n, C);
  int32_t Cp = padded_cols(C);
  uint32_t* queue = g.queue;
  uint8_t* codes_p = g.codes_p;
  void* init_args[] = {&d_status, &queue};
  void* prep_args[] = {const_cast<uint8_t**>(&codes), &n, &C, const_cast<int32_t**>(&d_n_bins),
                       const_cast<double**>(&y), &y_fp, &codes_p, &Cp, &d_status};
  void* grow_args_v[] = {&a};
  const hipKernelNodeParams p_init = node_params(reinterpret_cast<const void*>(k_init), 1, 64, 0, init_args);
  const hipKernelNodeParams p_prep = node_params(reinterpret_cast<const void*>(k_prepare), pb, 256, 0, prep_args);
  const hipKernelNodeParams p_grow = node_params(kernel, grid, cfg.block, a.union_bytes, grow_args_v);
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  const GraphKey key{dev, kernel, cfg.block, grid, pb, a.union_bytes};
  static uint64_t clock = 0;
  std::lock_guard<std::mutex> lk(graph_mu());
  auto& cache = graph_cache();
  auto it = cache.find(key);
  const bool reused = it != cache.end();
  if (reused) {
    GraphEntry& e = it->second;
    AIWC_HIP(hipEventSynchronize(e.last));  // its previous launch read the old arguments
    AIWC_HIP(hipGraphExecKernelNodeSetParams(e.exec, e.init, &p_init));
    AIWC_HIP(hipGraphExecKernelNodeSetParams(e.exec, e.prep, &p_prep));
    AIWC_HIP(hipGraphExecKernelNodeSetParams(e.exec, e.grow, &p_grow));
  } else {
    if (cache.size() >= kMaxGraphs) {  // drop the least recently used shape
      auto old = cache.begin();
      for (auto j = cache.begin(); j != cache.end(); ++j)
        if (j->second.used < old->second.used) old = j;
      (void)hipEventSynchronize(old->second.last);
      (void)hipGraphExecDestroy(old->second.exec);
      (void)hipGraphDestroy(old->second.graph);
      (void)hipEventDestroy(old->second.last);
      cache.erase(old);
    }
    GraphEntry e;
    try {
      AIWC_HIP(hipGraphCreate(&e.graph, 0));
      AIWC_HIP(hipGraphAddKernelNode(&e.init, e.graph, nullptr, 0, &p_init));
      AIWC_HIP(hipGraphAddKernelNode(&e.prep, e.graph, &e.init, 1, &p_prep));
      AIWC_HIP(hipGraphAddKernelNode(&e.grow, e.graph, &e.prep, 1, &p_grow));
      AIWC_HIP(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
      AIWC_HIP(hipEventCreateWithFlags(&e.last, hipEventDisableTiming));
    } catch (...) {
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
      if (e.graph) (void)hipGraphDestroy(e.graph);
      throw;
    }
    it = cache.emplace(key, e).first;
  }
  GraphEntry& e = it->second;
  e.used = ++clock;
  AIWC_HIP(hipGraphLaunch(e.exec, s));
  AIWC_HIP(hipEventRecord(e.last, s));
  return reused;
}

}  // namespace aiwc
#endif
