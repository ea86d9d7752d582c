// Out-of-bag error on gfx950 (the tuning objective of Sec. III-B and Sec. III-C).
//
// Every training row of a forest is predicted by the trees whose bootstrap
// sample left it out (the in-bag bitmaps written by the fit), as an exact int64
// sum of leaf values and a tree count; its out-of-bag prediction is then
// (sum * 2^-32) / count, like the forest mean.  The squared and absolute errors
// are reduced per forest in a fixed order (wave butterflies, then workgroups in
// index order), so the result does not depend on scheduling.
#include "device.h"
#include "internal.h"

namespace aiwc {
namespace {

constexpr int kOobBlock = 256;

__global__ __launch_bounds__(kOobBlock) void k_oob_sums(const uint64_t* __restrict__ nodes,
                                                        const TreeTask* __restrict__ tasks,
                                                        const int64_t* __restrict__ node_base,
                                                        const uint64_t* __restrict__ inbag,
                                                        const int32_t* __restrict__ train_rows,
                                                        const OobForest* __restrict__ forests,
                                                        const uint8_t* __restrict__ codes, int32_t C,
                                                        int64_t* __restrict__ sum, int32_t* __restrict__ count) {
  const OobForest F = forests[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * kOobBlock + threadIdx.x;
  if (i >= F.n_train) return;
  const int64_t row = F.train_off >= 0 ? train_rows[F.train_off + i] : i;
  const uint8_t* rp = codes + row * C;
  int64_t P = 0;
  int32_t cnt = 0;
  for (int32_t t = 0; t < F.num_trees; ++t) {
    const int64_t off = tasks[F.first_task + t].inbag_off;
    if (off < 0) continue;  // no bootstrap: every row is in bag
    if ((inbag[off + i / kWave] >> (i % kWave)) & 1ull) continue;
    const uint64_t* tn = nodes + node_base[F.first_task + t];
    uint64_t v = tn[0];
    while (node_col(v) != kLeafCol) v = tn[node_left(v) + (rp[node_col(v)] > node_bin(v) ? 1u : 0u)];
    P += node_q(v);
    ++cnt;
  }
  sum[F.row_off + i] = P;
  count[F.row_off + i] = cnt;
}

// Held-out rows: every tree of the forest predicts; count = num.trees, so the
// prediction formed below is the forest mean of the prediction entry points.
__global__ __launch_bounds__(kOobBlock) void k_heldout_sums(const uint64_t* __restrict__ nodes,
                                                            const int64_t* __restrict__ node_base,
                                                            const int32_t* __restrict__ test_rows,
                                                            const OobForest* __restrict__ forests,
                                                            const uint8_t* __restrict__ codes, int32_t C,
                                                            int64_t* __restrict__ sum, int32_t* __restrict__ count) {
  const OobForest F = forests[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * kOobBlock + threadIdx.x;
  if (i >= F.n_train) return;
  const uint8_t* rp = codes + (int64_t)test_rows[F.train_off + i] * C;
  int64_t P = 0;
  for (int32_t t = 0; t < F.num_trees; ++t) {
    const uint64_t* tn = nodes + node_base[F.first_task + t];
    uint64_t v = tn[0];
    while (node_col(v) != kLeafCol) v = tn[node_left(v) + (rp[node_col(v)] > node_bin(v) ? 1u : 0u)];
    P += node_q(v);
  }
  sum[F.row_off + i] = P;
  count[F.row_off + i] = F.num_trees;
}

// Per workgroup: sums of squared error, absolute error and rows with a
// prediction (count > 0).
__global__ __launch_bounds__(kOobBlock) void k_oob_partial(const int64_t* __restrict__ sum,
                                                           const int32_t* __restrict__ count,
                                                           const int32_t* __restrict__ train_rows,
                                                           const OobForest* __restrict__ forests,
                                                           const double* __restrict__ y, double* __restrict__ partial) {
  __shared__ double s_sq[kOobBlock / kWave], s_ab[kOobBlock / kWave], s_m[kOobBlock / kWave];
  const OobForest F = forests[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * kOobBlock + threadIdx.x;
  double sq = 0.0, ab = 0.0, m = 0.0;
  if (i < F.n_train) {
    const int32_t c = count[F.row_off + i];
    if (c > 0) {
      const int64_t row = F.train_off >= 0 ? train_rows[F.train_off + i] : i;
      const double pred = ((double)sum[F.row_off + i] * 0x1p-32) / (double)c;
      const double e = pred - y[row];
      sq = e * e;
      ab = fabs(e);
      m = 1.0;
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    sq += __shfl_xor(sq, d, kWave);
    ab += __shfl_xor(ab, d, kWave);
    m += __shfl_xor(m, d, kWave);
  }
  const int wid = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_sq[wid] = sq;
    s_ab[wid] = ab;
    s_m[wid] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int w = 0; w < kOobBlock / kWave; ++w) {
      a += s_sq[w];
      b += s_ab[w];
      c += s_m[w];
    }
    double* out = partial + 3 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
    out[0] = a;
    out[1] = b;
    out[2] = c;
  }
}

// Per forest: mean squared error, mean absolute error, rows counted.
__global__ void k_oob_final(const double* partial, int32_t n_forests, int32_t blocks, double* result) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_forests) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int32_t k = 0; k < blocks; ++k) {
    const double* p = partial + 3 * ((int64_t)f * blocks + k);
    a += p[0];
    b += p[1];
    c += p[2];
  }
  result[3 * f + 0] = c > 0.0 ? a / c : 0.0;
  result[3 * f + 1] = c > 0.0 ? b / c : 0.0;
  result[3 * f + 2] = c;
}

}  // namespace

void launch_oob(const uint64_t* nodes, const TreeTask* tasks, const int64_t* node_base, const uint64_t* inbag,
                const int32_t* train_rows, const OobForest* forests, int32_t n_forests, int32_t max_n_train,
                const uint8_t* codes, int32_t C, const double* y, int64_t* sum, int32_t* count, double* partial,
                double* result, hipStream_t s) {
  const int32_t blocks = (max_n_train + kOobBlock - 1) / kOobBlock;
  const dim3 grid((unsigned)blocks, (unsigned)n_forests);
  k_oob_sums<<<grid, kOobBlock, 0, s>>>(nodes, tasks, node_base, inbag, train_rows, forests, codes, C, sum, count);
  AIWC_HIP(hipGetLastError());
  k_oob_partial<<<grid, kOobBlock, 0, s>>>(sum, count, train_rows, forests, y, partial);
  AIWC_HIP(hipGetLastError());
  k_oob_final<<<(n_forests + 255) / 256, 256, 0, s>>>(partial, n_forests, blocks, result);
  AIWC_HIP(hipGetLastError());
}

void launch_heldout(const uint64_t* nodes, const int64_t* node_base, const int32_t* test_rows,
                    const OobForest* forests, int32_t n_forests, int32_t max_n_test, const uint8_t* codes, int32_t C,
                    const double* y, int64_t* sum, int32_t* count, double* partial, double* result, hipStream_t s) {
  const int32_t blocks = std::max(1, (max_n_test + kOobBlock - 1) / kOobBlock);
  const dim3 grid((unsigned)blocks, (unsigned)n_forests);
  k_heldout_sums<<<grid, kOobBlock, 0, s>>>(nodes, node_base, test_rows, forests, codes, C, sum, count);
  AIWC_HIP(hipGetLastError());
  k_oob_partial<<<grid, kOobBlock, 0, s>>>(sum, count, test_rows, forests, y, partial);
  AIWC_HIP(hipGetLastError());
  k_oob_final<<<(n_forests + 255) / 256, 256, 0, s>>>(partial, n_forests, blocks, result);
  AIWC_HIP(hipGetLastError());
}

}  // namespace aiwc
