// Host-side internals of libaiwc_rf: error plumbing, the device memory cache,
// handle layouts and the kernel launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "aiwc_rf.h"

namespace aiwc {

// ---------------------------------------------------------------------------
// Errors: internal code throws Error; the C ABI converts it to a return code
// and a thread-local message.
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define AIWC_HIP(call) ::aiwc::hip_check((call), #call)

// The calling thread's last error message (what aiwc_rf_last_error returns).
void set_last_error(const std::string& msg);

// Runs f, converting what it throws into a return code and the thread's
// message; a call that succeeds clears the message.
template <typename F>
int guard(F&& f) {
  try {
    f();
    set_last_error(std::string());
    return AIWC_RF_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return AIWC_RF_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return AIWC_RF_EINVAL;
  }
}

// ---------------------------------------------------------------------------
// Device memory cache.  Blocks are rounded up to 1 MiB multiples (small blocks
// to 256 B) and kept for reuse after release; a block released from one stream
// and reused on another waits on an event recorded at release time.
// ---------------------------------------------------------------------------
void* dev_alloc(size_t bytes, hipStream_t stream);
void dev_release(void* p, hipStream_t stream);
void dev_cache_trim();  // hand every cached block back to HIP

// Host-to-device copies of host buffers through one pinned staging buffer per
// device: the sources are copied into it on the host, its copies to `dst` are
// enqueued on `stream`, and the call returns without waiting for them (a later
// call waits for them before it reuses the buffer).
struct HostPart {
  void* dst;
  const void* src;
  size_t bytes;
};
void upload_staged(hipStream_t stream, const HostPart* parts, int n_parts);

// Device-to-host copies through a second pinned staging buffer per device:
// enqueued on `stream`, then the stream is synchronized and the results are
// copied to their host destinations.
struct DevicePart {
  void* dst;
  const void* src;
  size_t bytes;
};
void download_staged(hipStream_t stream, const DevicePart* parts, int n_parts);

// A pinned host word for a forest's status, from a process-wide pool (or its
// own pinned allocation when the pool is exhausted); release hands it back.
uint32_t* pinned_word_acquire();
void pinned_word_release(uint32_t* p);

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(size_t count, hipStream_t stream) { reset(count, stream); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; s = o.s;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  void reset(size_t count, hipStream_t stream) {
    release();
    s = stream;
    n = count;
    p = count ? static_cast<T*>(dev_alloc(count * sizeof(T), stream)) : nullptr;
  }
  void release() {
    if (p) dev_release(p, s);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { release(); }
};

// ---------------------------------------------------------------------------
// Handles.
// ---------------------------------------------------------------------------
}  // namespace aiwc

struct aiwc_rf_binner {
  int device = 0;
  int32_t p = 0;          // feature columns
  int32_t n_devices = 0;  // bins of the device column
  int32_t max_bins = 0;
  bool has_thresholds = false;
  std::vector<int32_t> n_bins;     // p + 1
  std::vector<float> thresholds;   // p * 255
  aiwc::DevBuf<int32_t> d_n_bins;  // p + 1
  aiwc::DevBuf<float> d_thresholds;
};

namespace aiwc {

// One tree to grow: which forest, which Philox tree index, its parameters and
// where its rows and nodes live.
struct TreeTask {
  int32_t forest;
  int32_t tree;
  int32_t n_train;
  int32_t mtry;
  int32_t min_node;
  int32_t bootstrap;
  uint64_t seed;
  int64_t train_off;  // offset into the training-row lists, -1 = rows 0..n_train-1
  int64_t node_base;  // first node of the tree's slot in the node pool
  int64_t capacity;   // node slots reserved for the tree (2 n_train - 1)
  int64_t inbag_off;  // first 64-bit word of the tree's in-bag bitmap over its training rows, -1 = none
};

// Work counters a fit writes per tree: searched rows, searched nodes,
// partitioned rows, levels, and rows added to LDS histogram bins (one per
// candidate column of every node above 32 rows).
constexpr int kWorkWords = 5;

// Most tasks in a group of a fused fit: trees that differ only in
// min.node.size, grown together up to the level where they part.
constexpr int kGroupMax = 8;

// Status bits a fit raises on the device.
constexpr uint32_t kStatusBadY = 1u;
constexpr uint32_t kStatusBadCode = 2u;
constexpr uint32_t kStatusCapacity = 4u;
constexpr uint32_t kStatusBadFeature = 8u;
constexpr uint32_t kStatusBadDevice = 16u;

}  // namespace aiwc

struct aiwc_rf_forest {
  int device = 0;
  int32_t n_cols = 0;
  std::vector<aiwc_rf_params> params;      // per forest
  std::vector<int64_t> first_task;         // per forest, index of tree 0 in the task list
  std::vector<aiwc::TreeTask> tasks;       // host copy
  aiwc::DevBuf<aiwc::TreeTask> d_tasks;
  aiwc::DevBuf<uint64_t> nodes;            // node words, all slots
  aiwc::DevBuf<uint32_t> node_N;           // bootstrap weight per node
  aiwc::DevBuf<int32_t> n_nodes;           // per task
  aiwc::DevBuf<int64_t> work;              // per task: kWorkWords counters
  aiwc::DevBuf<int64_t> node_base;         // per task, device copy for traversal
  aiwc::DevBuf<int32_t> group_task;        // task groups of a fused fit (members, by group)
  aiwc::DevBuf<int32_t> group_first;       // first member of every group, and the member count
  aiwc::DevBuf<uint32_t> status;           // device status word
  uint32_t* status_host = nullptr;         // pinned
  hipEvent_t done = nullptr;
  hipEvent_t grow_begin = nullptr;         // timing events around the tree-growing launch(es)
  hipEvent_t grow_end = nullptr;
  int32_t fit_status = 0;                  // resolved status after wait
  bool waited = false;
  int64_t pool_nodes = 0;
  aiwc_rf_launch_info launch{};            // the launch shape the fit used
  std::vector<int32_t> n_bins;             // bin count of every code column (device column last)
  aiwc::DevBuf<int32_t> train_rows;        // training-row lists of the forests that hold out a fold
  aiwc::DevBuf<uint64_t> inbag;            // per tree: bit i set if training row i is in its bootstrap sample
  std::vector<int32_t> n_train;            // per forest
  std::vector<int64_t> train_off;          // per forest, -1 = rows 0 .. n_train-1
  aiwc::DevBuf<int32_t> test_rows;         // held-out row lists (rows of a held-out fold or outside a mask)
  std::vector<int32_t> n_test;             // per forest
  std::vector<int64_t> test_off;           // per forest
};

namespace aiwc {

// ---------------------------------------------------------------------------
// Launchers (implemented in the .hip translation units).
// ---------------------------------------------------------------------------
// bin.hip
void launch_bin_fit(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices, int32_t max_bins,
                    int32_t* d_n_bins, float* d_thresholds, uint32_t* d_status, hipStream_t s);
void launch_bin_encode(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                       const int32_t* d_n_bins, const float* d_thresholds, uint8_t* codes, uint32_t* d_status,
                       hipStream_t s);

// fit.hip
struct GrowConfig {
  int block = 512;       // threads per workgroup
  int wg_per_cu = 0;     // 0 = as many as occupancy allows
  int occupancy = 4;     // waves per SIMD the kernel without the wide phase is built for (4, 5 or 6)
  int big_cols = 0;      // candidate columns per large-node task, at most what the wave area holds (0 = all it holds)
  int huge_min = 4096;   // nodes with more in-bag rows are searched in workgroup-wide batches
  bool wide_sums = false;  // small-node searches always add 64-bit sums (no byte-plane dot products)
  int wide_bytes = 0;    // LDS of a wide batch's histograms (0: 128 bytes per thread)
  int bins_max = 256;    // largest bin count of any column
  int64_t n_cap = 0;     // largest training set of any tree
};
// Autotuning of the grow kernel's launch shape.  A shape is keyed by the
// device, the training-set size class, the columns, the largest bin count,
// the largest mtry and the task-count class; the tuned config is cached in
// memory and, when AIWC_RF_TUNE_CACHE names a file, on disk.
struct TuneKey {
  int cus;
  int n_cap_log2;
  int cols;
  int bins_max;
  int mtry_max;
  int tasks_log2;
};
// A launch needs the kernel with the workgroup-wide phase iff a tree's
// training set exceeds the wide limit.
inline bool grow_has_wide_phase(const GrowConfig& cfg) { return cfg.n_cap > cfg.huge_min; }

bool tune_lookup(const TuneKey& key, GrowConfig* cfg);
void tune_store(const TuneKey& key, const GrowConfig& cfg);
std::vector<GrowConfig> tune_candidates(const GrowConfig& base);

void launch_init(uint32_t* d_status, uint32_t* d_queue, hipStream_t s);  // either may be null
void launch_set_i32(int32_t* p, int32_t v, hipStream_t s);
// Validates y and the codes, writes y_fp and a copy of the codes whose rows are
// padded to padded_cols(C) bytes (16-byte aligned rows); the copy's buffer must
// hold 64 bytes more than n * padded_cols(C), read but never used.
// Row stride of the padded code copy: a divisor of the 128-byte cache line
// (16, 32, 64 or 128 bytes) or a multiple of it, so that no row straddles two
// lines and a row's codes arrive with one line fetch.
inline int32_t padded_cols(int32_t C) {
  if (C <= 128) {
    int32_t p = 16;
    while (p < C) p *= 2;
    return p;
  }
  return (C + 127) / 128 * 128;
}
void launch_prepare(const uint8_t* codes, int64_t n, int32_t C, const int32_t* d_n_bins, const double* y,
                    int64_t* y_fp, uint8_t* codes_p, uint32_t* d_status, hipStream_t s);
// Scratch of one grow workgroup (wide: the launch has the wide phase, whose
// rows also keep their candidate codes for the partition; grouped: it grows
// groups of tasks, which put aside the level where their trees part).
size_t grow_scratch_bytes(int64_t n_cap, int32_t mtry_max, bool wide, bool grouped);
// Workgroups of a persistent grow launch over n_tasks work items (grouped: the
// kernel for launches with task groups).
int grow_grid_size(const GrowConfig& cfg, int64_t n_tasks, int32_t mtry_max, int32_t C, bool grouped = false);
// The grow kernels for launches with task groups (fit_grouped.hip).
const void* grow_kernel_grouped(int block, bool wide, int occ);
// The buffers of one grow launch: the codes (dense and row-padded), the
// training-row lists, the tasks and everything the trees write.
struct GrowLaunch {
  const uint8_t* codes;
  uint8_t* codes_p;
  const int32_t* train_rows;
  const TreeTask* tasks;
  int32_t n_tasks;
  uint64_t* nodes;
  uint32_t* node_N;
  int32_t* n_nodes;
  int64_t* work;
  uint64_t* inbag;
  uint32_t* queue;
  uint8_t* scratch;
  int64_t n_cap;
  // groups of tasks grown together (null: each task alone)
  const int32_t* group_task = nullptr;
  const int32_t* group_first = nullptr;
  int32_t n_groups = 0;
};
void launch_grow(const GrowConfig& cfg, const GrowLaunch& g, int32_t C, const int32_t* d_n_bins, const int64_t* y_fp,
                 uint32_t* d_status, int32_t mtry_max, int grid, hipStream_t s);
// Columns per large-node task that a launch shape actually uses.
int effective_big_cols(const GrowConfig& cfg, int32_t mtry_max, int32_t C);
// A fused fit as one executable graph launch (status and queue reset, prepare,
// grow), cached per launch shape: returns true when the graph of an earlier
// call was re-launched with this call's arguments instead of being built.
bool launch_fit_graph(const GrowConfig& cfg, const GrowLaunch& g, const uint8_t* codes, int64_t n, int32_t C,
                      const int32_t* d_n_bins, const double* y, int64_t* y_fp, uint32_t* d_status, int32_t mtry_max,
                      int grid, hipStream_t s);

// oob.hip: out-of-bag sums of every training row of forests [f0, f1), then
// the squared and absolute errors of the out-of-bag predictions per forest.
struct OobForest {
  int64_t first_task;
  int32_t num_trees;
  int32_t n_train;
  int64_t train_off;  // -1 = rows 0 .. n_train-1
  int64_t row_off;    // first slot of this forest's rows in the per-row outputs
};
void launch_oob(const uint64_t* nodes, const TreeTask* tasks, const int64_t* node_base, const uint64_t* inbag,
                const int32_t* train_rows, const OobForest* forests, int32_t n_forests, int32_t max_n_train,
                const uint8_t* codes, int32_t C, const double* y, int64_t* sum, int32_t* count, double* partial,
                double* result, hipStream_t s);
// Held-out error: the same per-forest reduction over each forest's held-out
// rows (OobForest.train_off / n_train name the held-out list in test_rows),
// every row predicted by all of the forest's trees.
void launch_heldout(const uint64_t* nodes, const int64_t* node_base, const int32_t* test_rows,
                    const OobForest* forests, int32_t n_forests, int32_t max_n_test, const uint8_t* codes, int32_t C,
                    const double* y, int64_t* sum, int32_t* count, double* partial, double* result, hipStream_t s);

// tune.cpp: the annealing search of aiwc_rf_tune_sa (arguments checked there).
void anneal(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner, const double* y_dev,
            const aiwc_rf_sa_config& cfg, int32_t* best_params, double* best_objective, aiwc_rf_sa_step* trace,
            hipStream_t s);

// predict.hip
// Rows of one allocation-free prediction (aiwc_rf_predict_noalloc): its int64
// row sums use a fixed device array of this many entries (8 MiB per GPU).
constexpr int64_t kNoAllocPredictRows = int64_t(1) << 20;
// That array's address on the current device (looked up once per device with
// hipGetSymbolAddress, then cached); allocates nothing.
int64_t* noalloc_predict_scratch();
void launch_predict(const uint64_t* nodes, const int64_t* node_base, int32_t tree_begin, int32_t tree_end,
                    const uint8_t* codes, int64_t n, int32_t C, int64_t* sum, double* y, int32_t num_trees,
                    hipStream_t s);

void launch_rank_accuracy(const double* times, const double* truth, int64_t m, int32_t D, int32_t* correct,
                          int32_t* counted, int32_t* hit, hipStream_t s);

void launch_select_device(const uint64_t* nodes, const int64_t* node_base, int32_t tree_begin, int32_t tree_end,
                          const uint8_t* feature_codes, int64_t m, int32_t C, int32_t n_devices, int32_t num_trees,
                          uint8_t* expanded, int64_t* sum, double* times, int32_t* best, hipStream_t s);

// Device properties of the current device (cached).
struct DeviceInfo {
  int device;
  int cus;
  size_t lds_per_block;
};
const DeviceInfo& device_info();

}  // namespace aiwc
