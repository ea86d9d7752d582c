// Host runtime of libaiwc_rf: errors, device properties and the device memory
// cache that every allocation of the library goes through.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace aiwc {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    fail(AIWC_RF_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
  }
  fail(AIWC_RF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

const DeviceInfo& device_info() {
  static std::mutex mu;
  static std::map<int, DeviceInfo> cache;
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  DeviceInfo d;
  d.device = dev;
  AIWC_HIP(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
  int lds = 0;
  AIWC_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  d.lds_per_block = (size_t)lds;
  return cache.emplace(dev, d).first->second;
}

namespace {

struct Block {
  void* p;
  size_t bytes;
  int device;
  hipStream_t stream;  // stream of the last release
  hipEvent_t ready;    // recorded on `stream` at release
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Block> free_blocks;  // by rounded size
  std::unordered_map<void*, Block> live;
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: releases may run during exit
  return *c;
}

size_t round_size(size_t b) {
  if (b == 0) return 256;
  if (b < (1u << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t mib = size_t(1) << 20;
  return (b + mib - 1) / mib * mib;
}

void free_all_cached_locked(Cache& c) {
  for (auto& kv : c.free_blocks) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(kv.second.device);
    (void)hipEventSynchronize(kv.second.ready);
    (void)hipEventDestroy(kv.second.ready);
    (void)hipFree(kv.second.p);
    (void)hipSetDevice(prev);
  }
  c.free_blocks.clear();
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t stream) {
  Cache& c = cache();
  const size_t r = round_size(bytes);
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(c.mu);
  for (auto it = c.free_blocks.lower_bound(r); it != c.free_blocks.end() && it->first == r; ++it) {
    if (it->second.device != dev) continue;
    Block b = it->second;
    c.free_blocks.erase(it);
    if (b.stream != stream) AIWC_HIP(hipStreamWaitEvent(stream, b.ready, 0));
    c.live.emplace(b.p, b);
    return b.p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    free_all_cached_locked(c);
    e = hipMalloc(&p, r);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(AIWC_RF_ENOMEM, "device allocation of " + std::to_string(r) + " bytes failed: " + hipGetErrorString(e));
  }
  Block b{p, r, dev, stream, nullptr};
  AIWC_HIP(hipEventCreateWithFlags(&b.ready, hipEventDisableTiming));
  c.live.emplace(p, b);
  return p;
}

void dev_release(void* p, hipStream_t stream) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  Block b = it->second;
  c.live.erase(it);
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != b.device) (void)hipSetDevice(b.device);
  b.stream = stream;
  (void)hipEventRecord(b.ready, stream);
  if (prev != b.device) (void)hipSetDevice(prev);
  c.free_blocks.emplace(b.bytes, b);
}

namespace {

struct Staging {
  std::mutex mu;
  uint8_t* p = nullptr;
  size_t cap = 0;
  hipEvent_t last = nullptr;  // the last copies out of the buffer
};

Staging& staging(int dev, bool down = false) {
  static std::mutex mu;
  static std::map<int, Staging> per_device, per_device_down;
  std::lock_guard<std::mutex> g(mu);
  return down ? per_device_down[dev] : per_device[dev];
}

// Makes st.p hold at least `total` bytes (the caller holds st.mu and no copy
// into or out of the buffer is pending).
void staging_reserve(Staging& st, size_t total) {
  if (total <= st.cap) return;
  if (st.p) AIWC_HIP(hipHostFree(st.p));
  st.p = nullptr;
  st.cap = 0;
  const size_t cap = std::max(total, (size_t)1 << 20);
  AIWC_HIP(hipHostMalloc((void**)&st.p, cap, hipHostMallocDefault));
  st.cap = cap;
}

struct WordPool {
  std::mutex mu;
  uint32_t* block = nullptr;
  std::vector<uint32_t*> free_words;
};

WordPool& word_pool() {
  static WordPool w;
  return w;
}

constexpr int kPinnedWords = 4096;

}  // namespace

void upload_staged(hipStream_t stream, const HostPart* parts, int n_parts) {
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  Staging& st = staging(dev);
  std::lock_guard<std::mutex> g(st.mu);
  size_t total = 0;
  for (int i = 0; i < n_parts; ++i) total += (parts[i].bytes + 255) / 256 * 256;
  if (total == 0) return;
  if (st.last) AIWC_HIP(hipEventSynchronize(st.last));  // the buffer's previous copies are done
  staging_reserve(st, total);
  if (!st.last) AIWC_HIP(hipEventCreateWithFlags(&st.last, hipEventDisableTiming));
  size_t off = 0;
  for (int i = 0; i < n_parts; ++i) {
    if (parts[i].bytes == 0) continue;
    std::memcpy(st.p + off, parts[i].src, parts[i].bytes);
    AIWC_HIP(hipMemcpyAsync(parts[i].dst, st.p + off, parts[i].bytes, hipMemcpyHostToDevice, stream));
    off += (parts[i].bytes + 255) / 256 * 256;
  }
  AIWC_HIP(hipEventRecord(st.last, stream));
}

void download_staged(hipStream_t stream, const DevicePart* parts, int n_parts) {
  int dev = 0;
  AIWC_HIP(hipGetDevice(&dev));
  Staging& st = staging(dev, true);
  std::lock_guard<std::mutex> g(st.mu);
  size_t total = 0;
  for (int i = 0; i < n_parts; ++i) total += (parts[i].bytes + 255) / 256 * 256;
  if (total == 0) return;
  staging_reserve(st, total);
  size_t off = 0;
  for (int i = 0; i < n_parts; ++i) {
    if (parts[i].bytes) AIWC_HIP(hipMemcpyAsync(st.p + off, parts[i].src, parts[i].bytes, hipMemcpyDeviceToHost, stream));
    off += (parts[i].bytes + 255) / 256 * 256;
  }
  AIWC_HIP(hipStreamSynchronize(stream));
  off = 0;
  for (int i = 0; i < n_parts; ++i) {
    if (parts[i].bytes) std::memcpy(parts[i].dst, st.p + off, parts[i].bytes);
    off += (parts[i].bytes + 255) / 256 * 256;
  }
}

uint32_t* pinned_word_acquire() {
  WordPool& w = word_pool();
  {
    std::lock_guard<std::mutex> g(w.mu);
    if (!w.block) {
      if (hipHostMalloc((void**)&w.block, sizeof(uint32_t) * kPinnedWords, hipHostMallocPortable) == hipSuccess) {
        for (int i = kPinnedWords - 1; i >= 0; --i) w.free_words.push_back(w.block + i);
      } else {
        (void)hipGetLastError();
        w.block = nullptr;
      }
    }
    if (!w.free_words.empty()) {
      uint32_t* p = w.free_words.back();
      w.free_words.pop_back();
      return p;
    }
  }
  uint32_t* p = nullptr;
  AIWC_HIP(hipHostMalloc((void**)&p, sizeof(uint32_t), hipHostMallocDefault));
  return p;
}

void pinned_word_release(uint32_t* p) {
  if (!p) return;
  WordPool& w = word_pool();
  std::lock_guard<std::mutex> g(w.mu);
  if (w.block && p >= w.block && p < w.block + kPinnedWords) {
    w.free_words.push_back(p);
    return;
  }
  (void)hipHostFree(p);
}

void dev_cache_trim() {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  free_all_cached_locked(c);
}

}  // namespace aiwc

// ---------------------------------------------------------------------------
// Launch-shape cache of the autotuner.
// ---------------------------------------------------------------------------
namespace aiwc {
namespace {

std::string key_text(const TuneKey& k) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "cus=%d n=2^%d cols=%d bins=%d mtry=%d tasks=2^%d", k.cus, k.n_cap_log2, k.cols,
                k.bins_max, k.mtry_max, k.tasks_log2);
  return buf;
}

struct TuneCache {
  std::mutex mu;
  bool loaded = false;
  std::map<std::string, std::array<int, 4>> entries;  // key -> (block, huge_min, occupancy, big_cols)
};

TuneCache& tune_cache() {
  static TuneCache* c = new TuneCache();
  return *c;
}

void load_file_locked(TuneCache& c) {
  if (c.loaded) return;
  c.loaded = true;
  const char* path = std::getenv("AIWC_RF_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    // "<key> | block=<b> huge_min=<h> occupancy=<o> big_cols=<c>"
    char* bar = std::strchr(line, '|');
    if (!bar) continue;
    std::string key(line, bar - line);
    while (!key.empty() && key.back() == ' ') key.pop_back();
    int b = 0, h = 0, o = 0, g = 0;
    if (std::sscanf(bar + 1, " block=%d huge_min=%d occupancy=%d big_cols=%d", &b, &h, &o, &g) == 4)
      c.entries[key] = {b, h, o, g};
  }
  std::fclose(f);
}

}  // namespace

bool tune_lookup(const TuneKey& key, GrowConfig* cfg) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  load_file_locked(c);
  auto it = c.entries.find(key_text(key));
  if (it == c.entries.end()) return false;
  cfg->block = it->second[0];
  cfg->huge_min = it->second[1];
  cfg->occupancy = it->second[2];
  cfg->big_cols = it->second[3];
  return true;
}

void tune_store(const TuneKey& key, const GrowConfig& cfg) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  load_file_locked(c);
  const std::string k = key_text(key);
  c.entries[k] = {cfg.block, cfg.huge_min, cfg.occupancy, cfg.big_cols};
  if (const char* path = std::getenv("AIWC_RF_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s | block=%d huge_min=%d occupancy=%d big_cols=%d\n", k.c_str(), cfg.block, cfg.huge_min,
                   cfg.occupancy, cfg.big_cols);
      std::fclose(f);
    }
  }
}

std::vector<GrowConfig> tune_candidates(const GrowConfig& base) {
  // workgroup size x wide-node limit; a limit at or above the largest training
  // set means no wide nodes, timed once per workgroup size at 4, 5 and 6 waves
  // per SIMD.  Where large-node tasks exist (limit above 64 rows) each shape is
  // timed with two and with four candidate columns per task.
  // One- and two-wave workgroups are timed without wide nodes only.
  std::vector<GrowConfig> out;
  for (int block : {64, 128, 192, 256, 512, 1024}) {
    bool narrow_done = false;
    for (int h : {64, 512, 4096}) {
      const bool narrow = base.n_cap <= h;
      if (narrow && narrow_done) continue;
      if (!narrow && block < 192) continue;
      narrow_done = narrow_done || narrow;
      for (int occ : {4, 5, 6}) {
        if (!narrow && occ != 4) continue;
        for (int bc : {2, 4}) {
          if (h <= 64 && bc != 2) continue;  // no large-node tasks: one timing suffices
          GrowConfig c = base;
          c.block = block;
          c.huge_min = h;
          c.occupancy = occ;
          c.big_cols = bc;
          out.push_back(c);
        }
      }
    }
  }
  return out;
}

}  // namespace aiwc

extern "C" const char* aiwc_rf_last_error(void) { return aiwc::g_last_error.c_str(); }
