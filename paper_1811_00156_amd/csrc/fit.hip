// Forest fitting on gfx950: one workgroup grows one tree at a time, level by
// level, pulling trees from a device-side queue until every tree of every
// forest in the launch is grown.
//
// Per tree (Sec. III-B: a random-forest regression tree with num.trees, mtry and
// min.node.size; the readings of the unspecified steps are listed in the public
// header):
//   1. bootstrap: n_train Philox draws -> multiplicity per training row, then the
//      in-bag rows are packed into 64-bit entries (row, weight, y_fp);
//   2. for each level, every open node is classified (leaf by min.node.size or
//      purity, or a split candidate); split candidates draw their mtry columns
//      and search every (column, bin) for the largest S_L^2/N_L + S_R^2/N_R:
//        - nodes with <= 64 in-bag rows: one wave per node, rows in lanes, the
//          left sums of every lane's bin obtained by broadcasting each row;
//        - larger nodes: one wave per (node, column) with a wave-private LDS
//          histogram of (N, S, Q) per bin, then a wave prefix scan over bins;
//   3. split nodes get breadth-first child ids from a workgroup scan, node words
//      are written, and the in-bag entries are partitioned into the children's
//      segments of the other entry buffer.
// All sums are integers, the only floating point is the binary64 score, so the
// order in which rows are visited never changes a result.
#include <limits.h>

#include "device.h"
#include "internal.h"

namespace aiwc {
namespace {

constexpr uint8_t kLeaf = 0, kSmall = 1, kBig = 2, kSplit = 3;
constexpr uint32_t kSmallMax = 64;  // rows per node handled by the register method

struct Rec {
  double score;
  int64_t SL;
  uint64_t QL;
  uint32_t NL;
  uint32_t colbin;  // column << 16 | bin
};

struct Scratch {
  uint32_t* cnt;
  uint64_t* buf[2];
  int32_t* slot[2];
  uint32_t* mstart[2];
  uint32_t* mend[2];
  uint32_t* mN[2];
  int64_t* mS[2];
  uint64_t* mQ[2];
  uint8_t* status;
  uint8_t* dcol;
  uint8_t* dbin;
  uint32_t* dNL;
  int64_t* dSL;
  uint64_t* dQL;
  uint32_t* rank;
  uint32_t* curL;
  uint32_t* curR;
  uint32_t* small;
  uint32_t* big;
  Rec* recs;
};

__host__ __device__ inline size_t carve(Scratch* s, uintptr_t base, int64_t n_cap, int32_t mtry_max) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> uintptr_t {
    const size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return base + o;
  };
  const size_t n = (size_t)n_cap;
  s->cnt = reinterpret_cast<uint32_t*>(take(4 * n));
  for (int b = 0; b < 2; ++b) {
    s->buf[b] = reinterpret_cast<uint64_t*>(take(8 * n));
    s->slot[b] = reinterpret_cast<int32_t*>(take(4 * n));
    s->mstart[b] = reinterpret_cast<uint32_t*>(take(4 * n));
    s->mend[b] = reinterpret_cast<uint32_t*>(take(4 * n));
    s->mN[b] = reinterpret_cast<uint32_t*>(take(4 * n));
    s->mS[b] = reinterpret_cast<int64_t*>(take(8 * n));
    s->mQ[b] = reinterpret_cast<uint64_t*>(take(8 * n));
  }
  s->status = reinterpret_cast<uint8_t*>(take(n));
  s->dcol = reinterpret_cast<uint8_t*>(take(n));
  s->dbin = reinterpret_cast<uint8_t*>(take(n));
  s->dNL = reinterpret_cast<uint32_t*>(take(4 * n));
  s->dSL = reinterpret_cast<int64_t*>(take(8 * n));
  s->dQL = reinterpret_cast<uint64_t*>(take(8 * n));
  s->rank = reinterpret_cast<uint32_t*>(take(4 * n));
  s->curL = reinterpret_cast<uint32_t*>(take(4 * n));
  s->curR = reinterpret_cast<uint32_t*>(take(4 * n));
  s->small = reinterpret_cast<uint32_t*>(take(4 * n));
  s->big = reinterpret_cast<uint32_t*>(take(4 * n));
  s->recs = reinterpret_cast<Rec*>(take(sizeof(Rec) * (n / kSmallMax + 1) * (size_t)mtry_max));
  return off;
}

// Per-wave LDS: one histogram of (N, S, Q) over at most 256 bins and the
// scratch of the mtry draw.
struct WaveLds {
  uint32_t hN[256];
  uint64_t hS[256];
  uint64_t hQ[256];
  uint8_t perm[256];
  uint8_t jidx[256];
  uint32_t mask[8];
};

struct GrowArgs {
  const uint8_t* codes;
  int32_t C;
  const int32_t* n_bins;
  const int64_t* y_fp;
  const int32_t* train_rows;
  const TreeTask* tasks;
  int32_t n_tasks;
  uint64_t* nodes;
  uint32_t* node_N;
  int32_t* n_nodes;
  int64_t* work;  // per task: searched rows, searched nodes, partitioned rows, levels
  uint32_t* queue;
  uint32_t* status;
  uint8_t* scratch;
  int64_t n_cap;
  int32_t mtry_max;
  size_t scratch_stride;
};

// Everything a wave task needs about the level being grown.
struct Level {
  const uint64_t* buf;
  const uint32_t* mstart;
  const uint32_t* mend;
  const uint32_t* mN;
  const int64_t* mS;
  uint32_t level_lo;
};

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t readlane64(int64_t v, uint32_t j) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, j);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), j);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The mtry candidate columns of node `node` of tree `tree`: a partial
// Fisher-Yates shuffle of 0..C-1 driven by draws k = 0..mtry-1 of the stream
// (seed, tag 1, node, tree); position k swaps with k + floor(r_k (C-k) / 2^64).
// The chosen set is left in L.mask (bit c = column c chosen).
__device__ void draw_candidates(WaveLds& L, uint64_t seed, uint32_t node, uint32_t tree, int C, int mtry) {
  const int lane = (int)lane_id();
  const int nblk = (mtry + 3) >> 2;
  for (int b = lane; b < nblk; b += kWave) {
    const U64x4 r = philox4x64_10((uint64_t)b, kTagMtry, node, tree, seed, 0);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int k = 4 * b + w;
      if (k < mtry) L.jidx[k] = (uint8_t)(k + (int)scale_draw(r.w[w], (uint64_t)(C - k)));
    }
  }
  for (int c = lane; c < C; c += kWave) L.perm[c] = (uint8_t)c;
  if (lane < 8) L.mask[lane] = 0;
  wave_lds_sync();
  if (lane == 0) {
    for (int k = 0; k < mtry; ++k) {
      const int j = L.jidx[k];
      const uint8_t t = L.perm[k];
      L.perm[k] = L.perm[j];
      L.perm[j] = t;
    }
  }
  wave_lds_sync();
  for (int k = lane; k < mtry; k += kWave) {
    const uint32_t c = L.perm[k];
    atomicOr(&L.mask[c >> 5], 1u << (c & 31));
  }
  wave_lds_sync();
}

// Split search of a node with at most 64 in-bag rows, whole node in one wave.
__device__ void small_node(const GrowArgs& a, const TreeTask& T, const Scratch& sc, const Level& lv, WaveLds& L,
                           uint32_t k) {
  const int lane = (int)lane_id();
  const uint32_t start = rfl(lv.mstart[k]);
  const uint32_t len = rfl(lv.mend[k]) - start;
  const uint32_t N = rfl(lv.mN[k]);
  const int64_t S = lv.mS[k];
  draw_candidates(L, T.seed, lv.level_lo + k, (uint32_t)T.tree, a.C, T.mtry);

  const bool valid = (uint32_t)lane < len;
  const uint64_t e = valid ? lv.buf[start + lane] : 0;
  const uint32_t w = valid ? entry_w(e) : 0;
  const int64_t y = entry_y(e);
  const int64_t wy = (int64_t)w * y;
  const uint8_t* rowp = a.codes + (size_t)entry_row(e) * a.C;

  double best = -1.0;
  int32_t best_col = -1, best_bin = 0;
  uint32_t best_NL = 0, best_code = 0;
  int64_t best_SL = 0;
  for (int mw = 0; mw < 8; ++mw) {
    uint32_t m = rfl(L.mask[mw]);
    while (m) {
      const int c = mw * 32 + __builtin_ctz(m);
      m &= m - 1;
      const uint32_t code = valid ? rowp[c] : 0u;
      uint32_t NL = 0;
      int64_t SL = 0;
      for (uint32_t j = 0; j < len; ++j) {
        const uint32_t cj = __builtin_amdgcn_readlane(code, j);
        const uint32_t wj = __builtin_amdgcn_readlane(w, j);
        const int64_t sj = readlane64(wy, j);
        if (cj <= code) {
          NL += wj;
          SL += sj;
        }
      }
      double s = -1.0;
      if (valid && NL < N) s = split_score(SL, NL, S - SL, N - NL);
      const ArgMax am = wave_argmax(s, (int32_t)code);
      if (am.score > best) {
        best = am.score;
        best_col = c;
        best_bin = am.key;
        best_NL = __shfl(NL, am.lane, kWave);
        best_SL = __shfl(SL, am.lane, kWave);
        best_code = code;
      }
    }
  }
  if (best_col >= 0 && best - parent_score(S, N) > 0.0) {
    uint64_t ql = (valid && best_code <= (uint32_t)best_bin) ? (uint64_t)(wy * y) : 0ull;
    ql = wave_sum(ql);
    if (lane == 0) {
      sc.dcol[k] = (uint8_t)best_col;
      sc.dbin[k] = (uint8_t)best_bin;
      sc.dNL[k] = best_NL;
      sc.dSL[k] = best_SL;
      sc.dQL[k] = ql;
      sc.status[k] = kSplit;
    }
  } else if (lane == 0) {
    sc.status[k] = kLeaf;
  }
}

// Best bin of candidate column number `ci` of a node with more than 64 in-bag
// rows: LDS histogram of (N, S, Q), wave prefix scan over bins, binary64 score.
__device__ void big_column(const GrowArgs& a, const TreeTask& T, const Scratch& sc, const Level& lv, WaveLds& L,
                           uint32_t j, int ci) {
  const int lane = (int)lane_id();
  const uint32_t k = rfl(sc.big[j]);
  const uint32_t start = rfl(lv.mstart[k]);
  const uint32_t end = rfl(lv.mend[k]);
  const uint32_t N = rfl(lv.mN[k]);
  draw_candidates(L, T.seed, lv.level_lo + k, (uint32_t)T.tree, a.C, T.mtry);
  int c = -1;
  {
    int seen = 0;
    for (int mw = 0; mw < 8 && c < 0; ++mw) {
      uint32_t m = rfl(L.mask[mw]);
      while (m) {
        const int cc = mw * 32 + __builtin_ctz(m);
        m &= m - 1;
        if (seen++ == ci) {
          c = cc;
          break;
        }
      }
    }
  }
  const int B = a.n_bins[c];
  for (int b = lane; b < B; b += kWave) {
    L.hN[b] = 0;
    L.hS[b] = 0;
    L.hQ[b] = 0;
  }
  wave_lds_sync();
  for (uint32_t p = start + lane; p < end; p += kWave) {
    const uint64_t e = lv.buf[p];
    const uint32_t w = entry_w(e);
    const int64_t y = entry_y(e);
    const uint32_t code = a.codes[(size_t)entry_row(e) * a.C + c];
    const int64_t wy = (int64_t)w * y;
    atomicAdd(&L.hN[code], w);
    atomicAdd((unsigned long long*)&L.hS[code], (unsigned long long)wy);
    atomicAdd((unsigned long long*)&L.hQ[code], (unsigned long long)(wy * y));
  }
  wave_lds_sync();
  const int R = (B + kWave - 1) / kWave;
  const int b0 = lane * R;
  const int b1 = min(b0 + R, B);
  uint32_t n_loc = 0;
  int64_t s_loc = 0;
  uint64_t q_loc = 0;
  for (int b = b0; b < b1; ++b) {
    n_loc += L.hN[b];
    s_loc += (int64_t)L.hS[b];
    q_loc += L.hQ[b];
  }
  uint32_t NL = wave_incl_scan_u32(n_loc) - n_loc;
  int64_t SL = wave_incl_scan<int64_t>(s_loc) - s_loc;
  uint64_t QL = wave_incl_scan<uint64_t>(q_loc) - q_loc;
  const int64_t S = lv.mS[k];
  double lbest = -1.0;
  int32_t lbin = INT_MAX;
  uint32_t lNL = 0;
  int64_t lSL = 0;
  uint64_t lQL = 0;
  for (int b = b0; b < b1; ++b) {
    NL += L.hN[b];
    SL += (int64_t)L.hS[b];
    QL += L.hQ[b];
    if (b <= B - 2 && NL > 0 && NL < N) {
      const double s = split_score(SL, NL, S - SL, N - NL);
      if (s > lbest) {
        lbest = s;
        lbin = b;
        lNL = NL;
        lSL = SL;
        lQL = QL;
      }
    }
  }
  const ArgMax am = wave_argmax(lbest, lbin);
  if (lane == am.lane) {
    Rec r;
    r.score = am.score;
    r.SL = lSL;
    r.QL = lQL;
    r.NL = lNL;
    r.colbin = ((uint32_t)c << 16) | (uint32_t)(am.score >= 0.0 ? lbin : 0);
    sc.recs[(size_t)j * T.mtry + ci] = r;
  }
}

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

template <int BLOCK>
__device__ void grow_tree(const GrowArgs& a, const TreeTask& T, int32_t task_index, const Scratch& sc, WaveLds* wl,
                          uint32_t* s_tmp, uint64_t* s_red, uint32_t* s_cnt) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, wid = tid / kWave;
  const int64_t n = T.n_train;
  const int32_t* train = T.train_off >= 0 ? a.train_rows + T.train_off : nullptr;

  // 1. bootstrap multiplicities
  for (int64_t i = tid; i < n; i += BLOCK) sc.cnt[i] = T.bootstrap ? 0u : 1u;
  __syncthreads();
  if (T.bootstrap) {
    const int64_t nblk = (n + 3) / 4;
    for (int64_t b = tid; b < nblk; b += BLOCK) {
      const U64x4 r = philox4x64_10((uint64_t)b, kTagBootstrap, 0, (uint64_t)T.tree, T.seed, 0);
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (4 * b + w < n) atomicAdd(&sc.cnt[scale_draw(r.w[w], (uint64_t)n)], 1u);
    }
    __syncthreads();
  }
  // in-bag entries, ascending local row order; root sums
  uint32_t n_inbag = 0;
  uint64_t N0 = 0, Q0 = 0;
  int64_t S0 = 0;
  for (int64_t base = 0; base < n; base += BLOCK) {
    const int64_t i = base + tid;
    const uint32_t c = i < n ? sc.cnt[i] : 0u;
    uint32_t total;
    const uint32_t pos = block_exscan<BLOCK>(c > 0 ? 1u : 0u, s_tmp, total) + n_inbag;
    if (c > 0) {
      const uint32_t row = train ? (uint32_t)train[i] : (uint32_t)i;
      const int64_t y = a.y_fp[row];
      sc.buf[0][pos] = entry_pack(row, c, y);
      sc.slot[0][pos] = 0;
      N0 += c;
      S0 += (int64_t)c * y;
      Q0 += (uint64_t)((int64_t)c * y * y);
    }
    n_inbag += total;
  }
  N0 = block_sum<BLOCK, uint64_t>(N0, s_red);
  S0 = (int64_t)block_sum<BLOCK, uint64_t>((uint64_t)S0, s_red);
  Q0 = block_sum<BLOCK, uint64_t>(Q0, s_red);
  if (tid == 0) {
    sc.mstart[0][0] = 0;
    sc.mend[0][0] = n_inbag;
    sc.mN[0][0] = (uint32_t)N0;
    sc.mS[0][0] = S0;
    sc.mQ[0][0] = Q0;
  }
  __syncthreads();

  const int64_t base_node = T.node_base;
  uint32_t level_lo = 0, level_cnt = 1, next_id = 1;
  int cur = 0;
  uint64_t work_rows = 0, work_nodes = 0, work_part = 0, levels = 0;
  while (level_cnt > 0) {
    ++levels;
    const int nxt = cur ^ 1;
    // (a) classify the level's nodes
    if (tid == 0) {
      s_cnt[0] = 0;
      s_cnt[1] = 0;
    }
    __syncthreads();
    for (uint32_t k = tid; k < level_cnt; k += BLOCK) {
      const uint32_t N = sc.mN[cur][k];
      const int64_t S = sc.mS[cur][k];
      const uint64_t Q = sc.mQ[cur][k];
      const uint32_t len = sc.mend[cur][k] - sc.mstart[cur][k];
      if ((int64_t)N <= T.min_node || node_is_pure(N, S, Q)) {
        sc.status[k] = kLeaf;
      } else if (len <= kSmallMax) {
        sc.status[k] = kSmall;
        sc.small[atomicAdd(&s_cnt[0], 1u)] = k;
        work_rows += len;
        ++work_nodes;
      } else {
        sc.status[k] = kBig;
        sc.big[atomicAdd(&s_cnt[1], 1u)] = k;
        work_rows += len;
        ++work_nodes;
      }
    }
    __syncthreads();
    const uint32_t n_small = s_cnt[0], n_big = s_cnt[1];
    const Level lv{sc.buf[cur], sc.mstart[cur], sc.mend[cur], sc.mN[cur], sc.mS[cur], level_lo};
    // (b) split search
    const uint32_t n_big_tasks = n_big * (uint32_t)T.mtry;
    const uint32_t n_tasks = n_big_tasks + n_small;
    for (uint32_t t = wid; t < n_tasks; t += NW) {
      if (t < n_big_tasks)
        big_column(a, T, sc, lv, wl[wid], t / T.mtry, (int)(t % T.mtry));
      else
        small_node(a, T, sc, lv, wl[wid], sc.small[t - n_big_tasks]);
    }
    __syncthreads();
    // (c) decisions of the large nodes
    for (uint32_t j = tid; j < n_big; j += BLOCK) {
      const uint32_t k = sc.big[j];
      double best = -1.0;
      int bi = -1;
      for (int i = 0; i < T.mtry; ++i) {
        const double s = sc.recs[(size_t)j * T.mtry + i].score;
        if (s > best) {
          best = s;
          bi = i;
        }
      }
      const int64_t S = sc.mS[cur][k];
      const uint32_t N = sc.mN[cur][k];
      if (bi >= 0 && best - parent_score(S, N) > 0.0) {
        const Rec r = sc.recs[(size_t)j * T.mtry + bi];
        sc.dcol[k] = (uint8_t)(r.colbin >> 16);
        sc.dbin[k] = (uint8_t)(r.colbin & 0xFFFF);
        sc.dNL[k] = r.NL;
        sc.dSL[k] = r.SL;
        sc.dQL[k] = r.QL;
        sc.status[k] = kSplit;
      } else {
        sc.status[k] = kLeaf;
      }
    }
    __syncthreads();
    // (d) breadth-first child ids, node words, children's sums and cursors
    uint32_t n_split = 0;
    for (uint32_t b0 = 0; b0 < level_cnt; b0 += BLOCK) {
      const uint32_t k = b0 + tid;
      const bool in = k < level_cnt;
      const bool split = in && sc.status[k] == kSplit;
      uint32_t total;
      const uint32_t r = block_exscan<BLOCK>(split ? 1u : 0u, s_tmp, total) + n_split;
      if (in) {
        const uint32_t node = level_lo + k;
        const uint32_t N = sc.mN[cur][k];
        const int64_t S = sc.mS[cur][k];
        if (split) {
          const uint32_t left = next_id + 2 * r;
          if ((int64_t)left + 1 < T.capacity) {
            a.nodes[base_node + node] = node_split(sc.dcol[k], sc.dbin[k], left);
          } else {
            atomicOr(a.status, kStatusCapacity);
          }
          sc.rank[k] = r;
          work_part += sc.mend[cur][k] - sc.mstart[cur][k];
          sc.curL[k] = sc.mstart[cur][k];
          sc.curR[k] = sc.mend[cur][k];
          const uint32_t NL = sc.dNL[k];
          const int64_t SL = sc.dSL[k];
          const uint64_t QL = sc.dQL[k];
          sc.mstart[nxt][2 * r] = sc.mstart[cur][k];
          sc.mN[nxt][2 * r] = NL;
          sc.mS[nxt][2 * r] = SL;
          sc.mQ[nxt][2 * r] = QL;
          sc.mend[nxt][2 * r + 1] = sc.mend[cur][k];
          sc.mN[nxt][2 * r + 1] = N - NL;
          sc.mS[nxt][2 * r + 1] = S - SL;
          sc.mQ[nxt][2 * r + 1] = sc.mQ[cur][k] - QL;
        } else {
          a.nodes[base_node + node] = node_leaf(leaf_value(N, S));
        }
        a.node_N[base_node + node] = N;
      }
      n_split += total;
    }
    __syncthreads();
    if ((int64_t)next_id + 2 * (int64_t)n_split > T.capacity) {
      // cannot happen for consistent inputs: every child holds an in-bag row
      next_id = (uint32_t)T.capacity;
      break;
    }
    // (e) partition the entries of split nodes into their children's segments
    for (uint32_t p = tid; p < n_inbag; p += BLOCK) {
      const int32_t k = sc.slot[cur][p];
      if (k >= 0 && sc.status[k] == kSplit) {
        const uint64_t e = sc.buf[cur][p];
        const uint32_t code = a.codes[(size_t)entry_row(e) * a.C + sc.dcol[k]];
        uint32_t dst;
        int32_t child;
        if (code <= sc.dbin[k]) {
          dst = atomicAdd(&sc.curL[k], 1u);
          child = (int32_t)(2 * sc.rank[k]);
        } else {
          dst = atomicSub(&sc.curR[k], 1u) - 1u;
          child = (int32_t)(2 * sc.rank[k] + 1);
        }
        sc.buf[nxt][dst] = e;
        sc.slot[nxt][dst] = child;
      } else {
        sc.slot[nxt][p] = -1;
      }
    }
    __syncthreads();
    // (f) the boundary between each pair of children
    for (uint32_t k = tid; k < level_cnt; k += BLOCK) {
      if (sc.status[k] == kSplit) {
        const uint32_t r = sc.rank[k];
        sc.mend[nxt][2 * r] = sc.curL[k];
        sc.mstart[nxt][2 * r + 1] = sc.curL[k];
      }
    }
    __syncthreads();
    level_lo = next_id;
    level_cnt = 2 * n_split;
    next_id += 2 * n_split;
    cur = nxt;
  }
  work_rows = block_sum<BLOCK, uint64_t>(work_rows, s_red);
  work_nodes = block_sum<BLOCK, uint64_t>(work_nodes, s_red);
  work_part = block_sum<BLOCK, uint64_t>(work_part, s_red);
  if (tid == 0) {
    a.n_nodes[task_index] = (int32_t)next_id;
    int64_t* wk = a.work + 4 * (int64_t)task_index;
    wk[0] = (int64_t)work_rows;
    wk[1] = (int64_t)work_nodes;
    wk[2] = (int64_t)work_part;
    wk[3] = (int64_t)levels;
  }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_grow(GrowArgs a) {
  constexpr int NW = BLOCK / kWave;
  __shared__ WaveLds wl[NW];
  __shared__ uint32_t s_tmp[NW + 1];
  __shared__ uint64_t s_red[NW];
  __shared__ uint32_t s_cnt[2];
  __shared__ uint32_t s_task;
  Scratch sc;
  carve(&sc, reinterpret_cast<uintptr_t>(a.scratch) + a.scratch_stride * blockIdx.x, a.n_cap, a.mtry_max);
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(a.queue, 1u);
    __syncthreads();
    const uint32_t t = s_task;
    __syncthreads();
    if (t >= (uint32_t)a.n_tasks) return;
    const TreeTask T = a.tasks[t];
    grow_tree<BLOCK>(a, T, (int32_t)t, sc, wl, s_tmp, s_red, s_cnt);
    __syncthreads();
  }
}

__global__ void k_init(uint32_t* status, uint32_t* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (status) *status = 0;
    if (queue) *queue = 0;
  }
}

// y -> y_fp = rint(y * 2^16) with range check, and every code < its column's bin count.
__global__ void k_prepare(const uint8_t* codes, int64_t n, int32_t C, const int32_t* n_bins, const double* y,
                          int64_t* y_fp, uint32_t* status) {
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
  if (bad) atomicOr(status, bad);
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
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

size_t grow_scratch_bytes(int64_t n_cap, int32_t mtry_max) {
  Scratch s;
  return carve(&s, 0, n_cap, mtry_max);
}

void launch_prepare(const uint8_t* codes, int64_t n, int32_t C, const int32_t* d_n_bins, const double* y,
                    int64_t* y_fp, uint32_t* d_status, hipStream_t s) {
  const int64_t work = n * C;
  const int blocks = (int)std::min<int64_t>(2048, (work + 255) / 256);
  k_prepare<<<std::max(blocks, 1), 256, 0, s>>>(codes, n, C, d_n_bins, y, y_fp, d_status);
  AIWC_HIP(hipGetLastError());
}

template <int BLOCK>
static int occupancy() {
  int nb = 0;
  AIWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grow<BLOCK>, BLOCK, 0));
  return std::max(nb, 1);
}

int grow_grid_size(const GrowConfig& cfg, int64_t n_tasks) {
  int per_cu = 1;
  switch (cfg.block) {
    case 256: per_cu = occupancy<256>(); break;
    case 512: per_cu = occupancy<512>(); break;
    case 1024: per_cu = occupancy<1024>(); break;
    default: fail(AIWC_RF_EINVAL, "unsupported grow block size");
  }
  if (cfg.wg_per_cu > 0) per_cu = std::min(per_cu, cfg.wg_per_cu);
  const int64_t slots = (int64_t)device_info().cus * per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(slots, n_tasks));
}

void launch_grow(const GrowConfig& cfg, const uint8_t* codes, int32_t C, const int32_t* d_n_bins,
                 const int64_t* y_fp, const int32_t* train_rows, const TreeTask* d_tasks, int32_t n_tasks,
                 uint64_t* nodes, uint32_t* node_N, int32_t* n_nodes, int64_t* work, uint32_t* d_queue,
                 uint32_t* d_status, uint8_t* scratch, int64_t n_cap, int32_t mtry_max, int grid, hipStream_t s) {
  GrowArgs a;
  a.codes = codes;
  a.C = C;
  a.n_bins = d_n_bins;
  a.y_fp = y_fp;
  a.train_rows = train_rows;
  a.tasks = d_tasks;
  a.n_tasks = n_tasks;
  a.nodes = nodes;
  a.node_N = node_N;
  a.n_nodes = n_nodes;
  a.work = work;
  a.queue = d_queue;
  a.status = d_status;
  a.scratch = scratch;
  a.n_cap = n_cap;
  a.mtry_max = mtry_max;
  a.scratch_stride = grow_scratch_bytes(n_cap, mtry_max);
  switch (cfg.block) {
    case 256: k_grow<256><<<grid, 256, 0, s>>>(a); break;
    case 512: k_grow<512><<<grid, 512, 0, s>>>(a); break;
    case 1024: k_grow<1024><<<grid, 1024, 0, s>>>(a); break;
    default: fail(AIWC_RF_EINVAL, "unsupported grow block size");
  }
  AIWC_HIP(hipGetLastError());
}

}  // namespace aiwc
