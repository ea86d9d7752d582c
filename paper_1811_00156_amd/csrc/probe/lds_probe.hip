// Measurement probes (declared in include/aiwc_rf_probe.h): the LDS atomic
// throughput that the tree-growing kernel's histogram adds are set against,
// and a check of the kernel's split-score division against IEEE division.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../device.h"
#include "aiwc_rf.h"
#include "aiwc_rf_probe.h"

namespace {

constexpr int kBlock = 256;
constexpr int kBins = 256;
constexpr int kUnroll = 8;
constexpr int kWaves = kBlock / 64;

thread_local std::string g_err;

// Every lane adds 1 to bins b[0..7] of its wave's histogram, iters times each.
// PATTERN 0: bin (lane + 64 u) mod 256, so the 64 lanes of one instruction hit
// 64 consecutive words; PATTERN 1: bins from a per-lane xorshift, drawn once
// before the loop, so that the loop holds only the atomics.
template <typename T, int PATTERN>
__global__ __launch_bounds__(kBlock) void k_lds_add(int iters, unsigned long long* sums) {
  __shared__ T h[kWaves][kBins];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kWaves * kBins; i += kBlock) (&h[0][0])[i] = 0;
  __syncthreads();
  T* hw = h[w];
  uint32_t b[kUnroll];
  uint32_t x = 0x9E3779B9u * (uint32_t)(blockIdx.x * kBlock + threadIdx.x + 1);
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (PATTERN == 0) {
      b[u] = (uint32_t)(lane + 64 * (u & 3));
    } else {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      b[u] = x & (kBins - 1);
    }
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) atomicAdd(&hw[b[u]], (T)1);
  }
  __syncthreads();
  // every bin of every wave into one per-block sum (read back and checked)
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < kWaves * kBins; i += kBlock) s += (unsigned long long)(&h[0][0])[i];
  atomicAdd(&sums[blockIdx.x], s);
}

template <typename T, int PATTERN>
void launch(int blocks, int iters, unsigned long long* sums, hipStream_t s) {
  k_lds_add<T, PATTERN><<<blocks, kBlock, 0, s>>>(iters, sums);
}

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

// A 64-bit finalizer (counter -> well-spread bits) for the check's operands.
__host__ __device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Quotient i of the split score's domain: the square of an integer of a random
// bit length up to 41 (zero included) over an integer weight in [1, 2^18] (odd
// lengths) or in [1, 64] (even lengths), by the kernel's division and by IEEE
// division; differing bit patterns are counted.
__global__ __launch_bounds__(256) void k_divide_check(uint64_t base, uint64_t seed, unsigned long long* bad) {
  const uint64_t i = base + (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const uint64_t h1 = mix64(seed ^ (2 * i + 1)), h2 = mix64(seed ^ (2 * i + 2));
  const int bits = (int)(h1 % 42u);
  const int64_t a = bits == 0 ? 0 : (int64_t)((h1 >> 8) & ((1ull << bits) - 1u));
  const uint32_t range = (bits & 1) ? 262144u : 64u;
  const uint32_t n = 1u + (uint32_t)((h2 >> 5) % range);
  const double ad = (double)a, num = ad * ad, den = (double)n;
  const double q_ieee = num / den, q = aiwc::div_pos(num, den);
  if (__double_as_longlong(q_ieee) != __double_as_longlong(q)) atomicAdd(bad, 1ull);
}

}  // namespace

extern "C" int aiwc_rf_probe_divide(int64_t samples, uint64_t seed, uint64_t* mismatches_host, void* stream) {
  if (!mismatches_host) return fail(AIWC_RF_EINVAL, "null pointer argument");
  if (samples < 1 || samples > ((int64_t)1 << 40)) return fail(AIWC_RF_EINVAL, "samples must be in [1, 2^40]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned long long* bad = nullptr;
  hipError_t e = hipMalloc((void**)&bad, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), s);
  // launches of up to 2^28 quotients, rounded up to whole workgroups
  const uint64_t mix = mix64((uint64_t)seed);
  for (int64_t b = 0; e == hipSuccess && b < samples; b += (int64_t)1 << 28) {
    const int64_t n = samples - b < ((int64_t)1 << 28) ? samples - b : ((int64_t)1 << 28);
    k_divide_check<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((uint64_t)b, mix, bad);
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (bad) (void)hipFree(bad);
  if (e != hipSuccess) return fail(AIWC_RF_EHIP, std::string("HIP error: ") + hipGetErrorString(e));
  *mismatches_host = h;
  g_err.clear();
  return AIWC_RF_OK;
}

extern "C" int aiwc_rf_probe_lds_add(int32_t width_bits, int32_t pattern, int32_t blocks, int32_t iters,
                                     double* adds_per_s_host, double* elapsed_ms_host, void* stream) {
  if (!adds_per_s_host || !elapsed_ms_host) return fail(AIWC_RF_EINVAL, "null pointer argument");
  if (blocks < 1 || iters < 1) return fail(AIWC_RF_EINVAL, "blocks and iters must be >= 1");
  if (width_bits != 32 && width_bits != 64) return fail(AIWC_RF_EINVAL, "width_bits must be 32 or 64");
  if (pattern != 0 && pattern != 1) return fail(AIWC_RF_EINVAL, "pattern must be 0 or 1");
  // one lane adds 1 iters x 8 times to a 32-bit bin: keep every bin below 2^32
  if ((int64_t)iters * kUnroll * 64 >= (int64_t)1 << 31) return fail(AIWC_RF_EINVAL, "iters too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned long long* sums = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&sums, sizeof(unsigned long long) * (size_t)blocks);
  auto run = [&]() {
    if (width_bits == 64)
      pattern ? launch<unsigned long long, 1>(blocks, iters, sums, s)
              : launch<unsigned long long, 0>(blocks, iters, sums, s);
    else
      pattern ? launch<unsigned int, 1>(blocks, iters, sums, s) : launch<unsigned int, 0>(blocks, iters, sums, s);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(sums, 0, sizeof(unsigned long long) * (size_t)blocks, s);
  if (e == hipSuccess) e = run();  // warm-up
  if (e == hipSuccess) e = hipMemsetAsync(sums, 0, sizeof(unsigned long long) * (size_t)blocks, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = run();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  unsigned long long total = 0;
  if (e == hipSuccess) {
    unsigned long long* h = new unsigned long long[(size_t)blocks];
    e = hipMemcpy(h, sums, sizeof(unsigned long long) * (size_t)blocks, hipMemcpyDeviceToHost);
    for (int i = 0; i < blocks; ++i) total += h[i];
    delete[] h;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sums) (void)hipFree(sums);
  if (e != hipSuccess) return fail(AIWC_RF_EHIP, std::string("HIP error: ") + hipGetErrorString(e));
  const unsigned long long want = (unsigned long long)blocks * kBlock * (unsigned long long)iters * kUnroll;
  if (total != want) return fail(AIWC_RF_ERANGE, "histogram sum differs from the number of adds");
  *elapsed_ms_host = ms;
  *adds_per_s_host = (double)want / (ms / 1000.0);
  g_err.clear();
  return AIWC_RF_OK;
}

extern "C" const char* aiwc_rf_probe_last_error(void) { return g_err.c_str(); }
