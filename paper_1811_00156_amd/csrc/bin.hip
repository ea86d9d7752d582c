// Quantile binning of the AIWC feature matrix on gfx950.
//
// Each feature column is turned into order-preserving u32 keys and sorted with
// a bitonic network (in LDS for short columns; LDS-local stages plus global
// merge passes for long ones).  From the sorted column the thresholds are the
// distinct values (when there are at most max_bins of them) or the order
// statistics s[floor(k n / B) - 1]; a feature's code is then the number of its
// column's thresholds strictly below it, found by binary search.  The device
// id is its own code column.
#include "device.h"
#include "internal.h"

namespace aiwc {
namespace {

constexpr int kChunk = 8192;  // keys sorted per workgroup in LDS (32 KiB)
constexpr int kSortBlock = 1024;

// Order-preserving key of a float (-0.0 folded onto +0.0).
__device__ __forceinline__ uint32_t float_key(float f) {
  if (f == 0.0f) f = 0.0f;
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

// keys[j][i] for i < n_pad; padding sorts last.
__global__ void k_make_keys(const float* X, int64_t n, int32_t p, int64_t n_pad, uint32_t* keys, uint32_t* status) {
  const int64_t total = n_pad * p;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t j = g / n_pad, i = g % n_pad;
    uint32_t k = 0xFFFFFFFFu;
    if (i < n) {
      const float x = X[i * p + j];
      if (isnan(x)) bad |= kStatusBadFeature;
      k = float_key(x);
    }
    keys[g] = k;
  }
  if (bad) atomicOr(status, bad);
}

__device__ __forceinline__ void cmp_swap(uint32_t& a, uint32_t& b, bool asc) {
  if ((a > b) == asc) {
    const uint32_t t = a;
    a = b;
    b = t;
  }
}

// Bitonic stages (k, j) with j < chunk inside LDS.  When `full`, runs every
// stage k = 2 .. min(chunk, n_pad); otherwise only stage k_outer's strides
// j = chunk/2 .. 1.  Directions use the global index, so chunks compose into
// the network over the whole column.
__global__ __launch_bounds__(kSortBlock) void k_sort_local(uint32_t* keys, int64_t n_pad, int64_t k_outer, int full) {
  __shared__ uint32_t s[kChunk];
  const int64_t L = n_pad < kChunk ? n_pad : kChunk;
  uint32_t* col = keys + (int64_t)blockIdx.y * n_pad;
  const int64_t base = (int64_t)blockIdx.x * L;
  for (int64_t i = threadIdx.x; i < L; i += kSortBlock) s[i] = col[base + i];
  __syncthreads();
  const int64_t k_lo = full ? 2 : k_outer;
  const int64_t k_hi = full ? L : k_outer;
  for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
    for (int64_t j = (full ? k : L) >> 1; j > 0; j >>= 1) {
      for (int64_t i = threadIdx.x; i < L; i += kSortBlock) {
        const int64_t l = i ^ j;
        if (l > i) {
          const bool asc = ((base + i) & k) == 0;
          cmp_swap(s[i], s[l], asc);
        }
      }
      __syncthreads();
    }
  }
  for (int64_t i = threadIdx.x; i < L; i += kSortBlock) col[base + i] = s[i];
}

// One global bitonic stride j >= chunk of stage k.
__global__ void k_sort_global(uint32_t* keys, int64_t n_pad, int64_t k, int64_t j) {
  uint32_t* col = keys + (int64_t)blockIdx.y * n_pad;
  const int64_t half = n_pad / 2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < half; t += (int64_t)gridDim.x * blockDim.x) {
    // t-th pair: i has bit j clear
    const int64_t i = ((t / j) * 2 * j) + (t % j);
    const int64_t l = i + j;
    uint32_t a = col[i], b = col[l];
    cmp_swap(a, b, (i & k) == 0);
    col[i] = a;
    col[l] = b;
  }
}

// Thresholds of one column from its sorted keys (one workgroup per column).
__global__ __launch_bounds__(256) void k_thresholds(const uint32_t* keys, int64_t n, int64_t n_pad, int32_t max_bins,
                                                    int32_t* n_bins, float* thresholds) {
  __shared__ uint32_t s_tmp[5];
  __shared__ uint32_t s_m;
  const int j = blockIdx.x;
  const uint32_t* s = keys + (int64_t)j * n_pad;
  float* t = thresholds + (int64_t)j * 255;
  const int tid = threadIdx.x, lane = (int)lane_id(), wid = tid / kWave;
  // distinct count m
  uint32_t m_loc = 0;
  for (int64_t i = tid; i < n; i += 256) m_loc += (i == 0 || s[i] != s[i - 1]) ? 1u : 0u;
  m_loc = wave_sum(m_loc);
  if (tid == 0) s_m = 0;
  __syncthreads();
  if (lane == 0) atomicAdd(&s_m, m_loc);
  __syncthreads();
  const uint32_t m = s_m;
  const uint32_t vmax = s[n - 1];
  for (int i = tid; i < 255; i += 256) t[i] = 0.0f;
  __syncthreads();
  if (m <= (uint32_t)max_bins) {
    // every distinct value except the largest, in order
    uint32_t run = 0;
    for (int64_t b0 = 0; b0 < n; b0 += 256) {
      const int64_t i = b0 + tid;
      const bool head = i < n && (i == 0 || s[i] != s[i - 1]) && s[i] != vmax;
      const uint32_t f = head ? 1u : 0u;
      const uint32_t incl = wave_incl_scan_u32(f);
      if (lane == kWave - 1) s_tmp[wid] = incl;
      __syncthreads();
      uint32_t off = 0, tot = 0;
      for (int w = 0; w < 4; ++w) {
        if (w < wid) off += s_tmp[w];
        tot += s_tmp[w];
      }
      if (head) t[run + off + incl - f] = key_float(s[i]);
      run += tot;
      __syncthreads();
    }
    if (tid == 0) n_bins[j] = (int32_t)m;
  } else if (tid == 0) {
    int n_t = 0;
    uint32_t last = 0;
    for (int k = 1; k < max_bins; ++k) {
      const int64_t idx = ((int64_t)k * n) / max_bins - 1;
      const uint32_t v = s[idx];
      if (v < vmax && (n_t == 0 || v > last)) {
        t[n_t++] = key_float(v);
        last = v;
      }
    }
    n_bins[j] = n_t + 1;
  }
}

// code(x) = #{thresholds < x}; column p = device id.
__global__ void k_encode(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                         const int32_t* n_bins, const float* thresholds, uint8_t* codes, uint32_t* status) {
  const int32_t C = p + 1;
  const int64_t total = n * C;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t i = g / C;
    const int32_t j = (int32_t)(g % C);
    uint32_t code;
    if (j == p) {
      const int32_t d = dev[i];
      if (d < 0 || d >= n_devices) {
        bad |= kStatusBadDevice;
        code = 0;
      } else {
        code = (uint32_t)d;
      }
    } else {
      const float x = X[i * p + j];
      if (isnan(x)) bad |= kStatusBadFeature;
      const float* t = thresholds + (int64_t)j * 255;
      int lo = 0, hi = n_bins[j] - 1;  // count of thresholds below x lies in [lo, hi]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] < x)
          lo = mid + 1;
        else
          hi = mid;
      }
      code = (uint32_t)lo;
    }
    codes[g] = (uint8_t)code;
  }
  if (bad) atomicOr(status, bad);
}

}  // namespace

void launch_bin_fit(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices, int32_t max_bins,
                    int32_t* d_n_bins, float* d_thresholds, uint32_t* d_status, hipStream_t s) {
  (void)dev;
  int64_t n_pad = 64;
  while (n_pad < n) n_pad <<= 1;
  DevBuf<uint32_t> keys((size_t)n_pad * p, s);
  {
    const int64_t work = n_pad * p;
    const int blocks = (int)std::min<int64_t>(4096, (work + 255) / 256);
    k_make_keys<<<blocks, 256, 0, s>>>(X, n, p, n_pad, keys.p, d_status);
    AIWC_HIP(hipGetLastError());
  }
  const int64_t L = std::min<int64_t>(n_pad, kChunk);
  const dim3 grid_local((unsigned)(n_pad / L), (unsigned)p);
  k_sort_local<<<grid_local, kSortBlock, 0, s>>>(keys.p, n_pad, 0, 1);
  AIWC_HIP(hipGetLastError());
  for (int64_t k = 2 * L; k <= n_pad; k <<= 1) {
    for (int64_t j = k >> 1; j >= L; j >>= 1) {
      const int64_t pairs = n_pad / 2;
      const dim3 grid((unsigned)std::min<int64_t>(1024, (pairs + 255) / 256), (unsigned)p);
      k_sort_global<<<grid, 256, 0, s>>>(keys.p, n_pad, k, j);
      AIWC_HIP(hipGetLastError());
    }
    k_sort_local<<<grid_local, kSortBlock, 0, s>>>(keys.p, n_pad, k, 0);
    AIWC_HIP(hipGetLastError());
  }
  k_thresholds<<<p, 256, 0, s>>>(keys.p, n, n_pad, max_bins, d_n_bins, d_thresholds);
  AIWC_HIP(hipGetLastError());
}

void launch_bin_encode(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                       const int32_t* d_n_bins, const float* d_thresholds, uint8_t* codes, uint32_t* d_status,
                       hipStream_t s) {
  const int64_t work = n * (p + 1);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (work + 255) / 256));
  k_encode<<<blocks, 256, 0, s>>>(X, dev, n, p, n_devices, d_n_bins, d_thresholds, codes, d_status);
  AIWC_HIP(hipGetLastError());
}

}  // namespace aiwc
