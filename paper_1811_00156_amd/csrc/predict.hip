// Batched prediction by tree traversal on gfx950.
//
// A thread follows one row down a chunk of trees (left when the row's code in
// the node's column is <= the node's bin, else right) and adds the leaf values
// as exact int64.  The grid is (row block x tree chunk); with the chunk index
// fastest and a multiple of 8 chunks, consecutive workgroups land on different
// XCDs while each XCD keeps working on the same trees, so the upper levels of
// those trees stay in that XCD's L2.  Partial sums of different chunks meet in
// a 64-bit integer atomic add, which is exact in any order.
#include <mutex>

#include "device.h"
#include "internal.h"

namespace aiwc {
namespace {

// The per-row int64 sums of the allocation-free prediction entry point live in
// this fixed array, one copy per GPU, held until the process ends.  Host code
// never uses its name as an address: the address of each device's copy comes
// from hipGetSymbolAddress (noalloc_predict_scratch).
__device__ __align__(256) unsigned long long scratch[kNoAllocPredictRows];

constexpr int kPredBlock = 256;
constexpr int kInterleave = 4;  // trees traversed together per thread to overlap load latency

__global__ __launch_bounds__(kPredBlock) void k_traverse(const uint64_t* __restrict__ nodes,
                                                         const int64_t* __restrict__ node_base, int32_t tree_begin,
                                                         int32_t tree_end, int32_t chunk, int32_t n_chunks,
                                                         const uint8_t* __restrict__ codes, int64_t n, int32_t C,
                                                         unsigned long long* __restrict__ sum, int accumulate) {
  const int32_t ci = (int32_t)(blockIdx.x % (unsigned)n_chunks);
  const int64_t rb = blockIdx.x / (unsigned)n_chunks;
  const int64_t r = rb * kPredBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t t0 = tree_begin + ci * chunk;
  const int32_t t1 = min(tree_end, t0 + chunk);
  if (t0 >= t1) return;
  const uint8_t* rp = codes + r * C;
  int64_t acc = 0;
  int32_t t = t0;
  for (; t + kInterleave <= t1; t += kInterleave) {
    const uint64_t* tn[kInterleave];
    uint64_t v[kInterleave];
#pragma unroll
    for (int u = 0; u < kInterleave; ++u) {
      tn[u] = nodes + node_base[t + u];
      v[u] = tn[u][0];
    }
    bool open = true;
    while (open) {
      open = false;
#pragma unroll
      for (int u = 0; u < kInterleave; ++u) {
        if (node_col(v[u]) != kLeafCol) {
          const uint32_t c = node_col(v[u]);
          const uint32_t next = node_left(v[u]) + (rp[c] > node_bin(v[u]) ? 1u : 0u);
          v[u] = tn[u][next];
          open = true;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kInterleave; ++u) acc += node_q(v[u]);
  }
  for (; t < t1; ++t) {
    const uint64_t* tn = nodes + node_base[t];
    uint64_t v = tn[0];
    while (node_col(v) != kLeafCol) v = tn[node_left(v) + (rp[node_col(v)] > node_bin(v) ? 1u : 0u)];
    acc += node_q(v);
  }
  if (accumulate)
    atomicAdd(&sum[r], (unsigned long long)acc);
  else
    sum[r] = (unsigned long long)acc;
}

__global__ void k_zero_i64(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// yhat = (P * 2^-32) / num.trees: an exact scaling then one rounded division.
__global__ void k_finalize(const int64_t* sum, int64_t n, double trees, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = ((double)sum[i] * 0x1p-32) / trees;
}

// Row i * D + d of the expanded matrix = kernel i's feature codes + device d.
__global__ void k_expand_devices(const uint8_t* feat, int64_t m, int32_t C, int32_t D, uint8_t* out) {
  const int64_t total = m * D * C;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / C;
    const int32_t j = (int32_t)(g % C);
    const int64_t i = row / D;
    out[g] = j < C - 1 ? feat[i * (C - 1) + j] : (uint8_t)(row % D);
  }
}

// Fastest device per kernel: the smallest predicted time, the lowest id on ties.
__global__ void k_argmin_devices(const double* times, int64_t m, int32_t D, int32_t* best) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const double* t = times + i * D;
    int32_t b = 0;
    for (int32_t d = 1; d < D; ++d)
      if (t[d] < t[b]) b = d;
    best[i] = b;
  }
}

// Sec. VI's scheduler criterion, one thread per kernel: for every device pair
// i < j the predicted choice is i when times[i] <= times[j] (lowest id on a
// tie), else j; it is right when the chosen device's true time is strictly the
// smaller.  Pairs with equal true times are not counted.  The fastest device is
// hit when the predicted best (smallest prediction, lowest id on ties) has the
// smallest true time.  Only comparisons: exact.
__global__ void k_rank_accuracy(const double* times, const double* truth, int64_t m, int32_t D, int32_t* correct,
                                int32_t* counted, int32_t* hit) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const double* p = times + k * D;
    const double* t = truth + k * D;
    int32_t c = 0, n = 0, best = 0;
    double tmin = t[0];
    for (int32_t i = 0; i < D; ++i) {
      const double pi = p[i], ti = t[i];
      if (pi < p[best]) best = i;
      tmin = ti < tmin ? ti : tmin;
      for (int32_t j = i + 1; j < D; ++j) {
        const double tj = t[j];
        if (ti == tj) continue;
        ++n;
        const bool pick_i = pi <= p[j];
        c += (pick_i ? ti < tj : tj < ti) ? 1 : 0;
      }
    }
    if (correct) correct[k] = c;
    if (counted) counted[k] = n;
    if (hit) hit[k] = t[best] == tmin ? 1 : 0;
  }
}

}  // namespace

void launch_rank_accuracy(const double* times, const double* truth, int64_t m, int32_t D, int32_t* correct,
                          int32_t* counted, int32_t* hit, hipStream_t s) {
  if (m <= 0) return;
  const int b = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (m + 255) / 256));
  k_rank_accuracy<<<b, 256, 0, s>>>(times, truth, m, D, correct, counted, hit);
  AIWC_HIP(hipGetLastError());
}

void launch_select_device(const uint64_t* nodes, const int64_t* node_base, int32_t tree_begin, int32_t tree_end,
                          const uint8_t* feature_codes, int64_t m, int32_t C, int32_t n_devices, int32_t num_trees,
                          uint8_t* expanded, int64_t* sum, double* times, int32_t* best, hipStream_t s) {
  const int64_t rows = m * n_devices;
  const int eb = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (rows * C + 255) / 256));
  k_expand_devices<<<eb, 256, 0, s>>>(feature_codes, m, C, n_devices, expanded);
  AIWC_HIP(hipGetLastError());
  launch_predict(nodes, node_base, tree_begin, tree_end, expanded, rows, C, sum, times, num_trees, s);
  const int ab = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (m + 255) / 256));
  k_argmin_devices<<<ab, 256, 0, s>>>(times, m, n_devices, best);
  AIWC_HIP(hipGetLastError());
}

int64_t* noalloc_predict_scratch() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(AIWC_RF_EINVAL, "device ordinal beyond the allocation-free table");
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    // this device is current: its own copy of the array, at its own address
    void* p = nullptr;
    AIWC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  return static_cast<int64_t*>(addr[dev]);
}

void launch_predict(const uint64_t* nodes, const int64_t* node_base, int32_t tree_begin, int32_t tree_end,
                    const uint8_t* codes, int64_t n, int32_t C, int64_t* sum, double* y, int32_t num_trees,
                    hipStream_t s) {
  if (n <= 0) return;
  const int32_t n_trees = tree_end - tree_begin;
  const int64_t row_blocks = (n + kPredBlock - 1) / kPredBlock;
  const int64_t target = 4LL * device_info().cus;
  int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(n_trees, (target + row_blocks - 1) / row_blocks));
  if (n_chunks > 1) n_chunks = std::min<int64_t>(n_trees, (n_chunks + 7) / 8 * 8);
  const int32_t chunk = (int32_t)((n_trees + n_chunks - 1) / n_chunks);
  n_chunks = (n_trees + chunk - 1) / chunk;
  const int accumulate = n_chunks > 1 ? 1 : 0;
  if (accumulate) {
    const int zb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    k_zero_i64<<<zb, 256, 0, s>>>(reinterpret_cast<unsigned long long*>(sum), n);
    AIWC_HIP(hipGetLastError());
  }
  const int64_t blocks = row_blocks * n_chunks;
  k_traverse<<<(unsigned)blocks, kPredBlock, 0, s>>>(nodes, node_base, tree_begin, tree_end, chunk, (int32_t)n_chunks,
                                                      codes, n, C, reinterpret_cast<unsigned long long*>(sum),
                                                      accumulate);
  AIWC_HIP(hipGetLastError());
  if (y) {
    const int fb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    k_finalize<<<fb, 256, 0, s>>>(sum, n, (double)num_trees, y);
    AIWC_HIP(hipGetLastError());
  }
}

}  // namespace aiwc
