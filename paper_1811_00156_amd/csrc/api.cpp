// The C ABI of libaiwc_rf (declared in include/aiwc_rf.h): argument checks,
// handle management and the orchestration of the binning, fitting and
// prediction kernels.  Nothing here computes a result on the host.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <tuple>

#include "device.h"
#include "internal.h"

using namespace aiwc;

namespace {

void require(bool ok, const char* what) {
  if (!ok) fail(AIWC_RF_EINVAL, what);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int32_t status_to_code(uint32_t st, std::string& msg) {
  if (st & kStatusBadY) {
    msg = "response is non-finite or outside [-64, 64] (log10 seconds)";
    return AIWC_RF_ERANGE;
  }
  if (st & kStatusBadCode) {
    msg = "a code is not below its column's bin count";
    return AIWC_RF_EINVAL;
  }
  if (st & kStatusBadFeature) {
    msg = "a feature value is NaN";
    return AIWC_RF_EINVAL;
  }
  if (st & kStatusBadDevice) {
    msg = "a device id is outside [0, n_devices)";
    return AIWC_RF_EINVAL;
  }
  if (st & kStatusCapacity) {
    msg = "tree node capacity exceeded";
    return AIWC_RF_ERANGE;
  }
  return AIWC_RF_OK;
}

GrowConfig grow_config(int64_t n_cap, int64_t n_items, const std::vector<int32_t>& n_bins) {
  GrowConfig cfg;
  // n_items: the launch's work items (trees, or task groups of a fused fit).
  // Large training sets: 1024 threads per tree, nodes above 512 rows in
  // workgroup-wide batches (the autotuner's choice on 200000 rows, 2 % ahead
  // of 512 threads with every node above 64 rows in batches).  Small ones, by
  // work items per CU: below 4, 512 threads per tree; from 4, 192 threads at 6
  // waves per SIMD (eight resident trees per CU); from 16, 128 threads at 6
  // waves (twelve); from 64, 64 threads at 5 waves (twenty): a tree's levels
  // get fewer waves, which pays once the queue is deep enough that the CUs
  // stay full to the end (the tuning grid, 340 groups per CU: 380 ms against
  // 395 and 417; one fold of it, 34 per CU: 45 ms against 42 and 43).  A
  // large-node task takes two candidate columns while trees are few (more
  // tasks per node for the tree's waves), up to four once the CUs are full.
  cfg.big_cols = 2;
  const int64_t cus = device_info().cus;
  if (n_cap > 16384) {
    cfg.block = 1024;
    cfg.huge_min = 512;
  } else if (n_items >= 64 * cus) {
    cfg.block = 64;
    cfg.occupancy = 5;
    cfg.big_cols = 4;
  } else if (n_items >= 16 * cus) {
    cfg.block = 128;
    cfg.occupancy = 6;
    cfg.big_cols = 4;
  } else if (n_items >= 4 * cus) {
    cfg.block = 192;
    cfg.occupancy = 6;
    cfg.big_cols = 4;
  } else {
    cfg.block = 512;
  }
  cfg.n_cap = n_cap;
  cfg.bins_max = 1;
  for (int32_t b : n_bins) cfg.bins_max = std::max(cfg.bins_max, b);
  if (const char* e = std::getenv("AIWC_RF_GROW_BLOCK")) cfg.block = std::atoi(e);
  if (const char* e = std::getenv("AIWC_RF_GROW_WG_PER_CU")) cfg.wg_per_cu = std::atoi(e);
  if (const char* e = std::getenv("AIWC_RF_HUGE_MIN")) cfg.huge_min = std::atoi(e);
  if (const char* e = std::getenv("AIWC_RF_GROW_OCC")) cfg.occupancy = std::atoi(e);
  if (const char* e = std::getenv("AIWC_RF_BIG_COLS")) cfg.big_cols = std::atoi(e);
  if (const char* e = std::getenv("AIWC_RF_WIDE_SUMS")) cfg.wide_sums = std::atoi(e) != 0;
  return cfg;
}

// Node arrays of one tree, unpacked from the node words.
void unpack_nodes(const std::vector<uint64_t>& words, const std::vector<uint32_t>& N, size_t count, uint8_t* col,
                  uint8_t* bin, int32_t* left, int64_t* q, int32_t* Nout) {
  for (size_t i = 0; i < count; ++i) {
    const uint64_t v = words[i];
    const bool leaf = node_col(v) == kLeafCol;
    if (col) col[i] = (uint8_t)node_col(v);
    if (bin) bin[i] = leaf ? 0 : (uint8_t)node_bin(v);
    if (left) left[i] = leaf ? -1 : (int32_t)node_left(v);
    if (q) q[i] = leaf ? node_q(v) : 0;
    if (Nout) Nout[i] = (int32_t)N[i];
  }
}

void check_forest(const aiwc_rf_forest* f, int32_t forest_index) {
  require(f != nullptr, "forest is NULL");
  require(forest_index >= 0 && forest_index < (int32_t)f->params.size(), "forest_index out of range");
}

int32_t resolve_status(const aiwc_rf_forest* fc, std::string& msg) {
  aiwc_rf_forest* f = const_cast<aiwc_rf_forest*>(fc);
  if (!f->waited) {
    AIWC_HIP(hipEventSynchronize(f->done));
    f->fit_status = status_to_code(*f->status_host, msg);
    f->waited = true;
    return f->fit_status;
  }
  status_to_code(*f->status_host, msg);
  return f->fit_status;
}

int ilog2_ceil(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// The autotuner: time every candidate launch shape on the call's first trees
// (they are grown again by the real launch, with identical results) and keep
// the fastest for this problem shape.
GrowConfig tune_grow(const GrowConfig& base, int64_t n_items, int32_t n_cols, int32_t mtry_max, aiwc_rf_forest* F,
                     const uint8_t* codes, int64_t n, const aiwc_rf_binner* binner, const double* y, int64_t* y_fp,
                     uint8_t* codes_p,
                     const int32_t* d_train, uint32_t* queue, hipStream_t s) {
  const int64_t n_tasks = (int64_t)F->tasks.size();
  TuneKey key{device_info().cus, ilog2_ceil(base.n_cap), n_cols, base.bins_max, mtry_max, ilog2_ceil(n_items)};
  GrowConfig best = base;
  if (tune_lookup(key, &best)) return best;
  const int64_t trial = std::min<int64_t>(n_tasks, 64LL * device_info().cus);
  // the trial grows an evenly strided sample of the launch's trees, so that a
  // grid of forests is timed on all of its parameter triples and not only on
  // its first forests (each sampled tree writes its own slots, which the fit
  // overwrites)
  const TreeTask* d_trial = F->d_tasks.p;
  DevBuf<TreeTask> sample;
  std::vector<TreeTask> h_sample;
  if (trial < n_tasks) {
    h_sample.resize((size_t)trial);
    for (int64_t i = 0; i < trial; ++i) h_sample[(size_t)i] = F->tasks[(size_t)(i * n_tasks / trial)];
    sample.reset((size_t)trial, s);
    AIWC_HIP(hipMemcpyAsync(sample.p, h_sample.data(), sizeof(TreeTask) * (size_t)trial, hipMemcpyHostToDevice, s));
    d_trial = sample.p;
  }
  launch_init(F->status.p, nullptr, s);
  launch_prepare(codes, n, n_cols, binner->d_n_bins.p, y, y_fp, codes_p, F->status.p, s);
  // (sized for the wide phase, which any candidate shape may have)
  const size_t per_wg = grow_scratch_bytes(base.n_cap, mtry_max, true, false);
  hipEvent_t e0, e1;
  AIWC_HIP(hipEventCreate(&e0));
  AIWC_HIP(hipEventCreate(&e1));
  float best_ms = -1.0f;
  for (const GrowConfig& c : tune_candidates(base)) {
    int grid = 0;
    try {
      grid = grow_grid_size(c, trial, mtry_max, n_cols);
    } catch (const Error&) {
      continue;  // the shape does not fit this device
    }
    DevBuf<uint8_t> scratch(per_wg * (size_t)grid, s);
    // each shape is timed twice and keeps its faster run
    float ms = -1.0f;
    for (int rep = 0; rep < 2; ++rep) {
      launch_init(nullptr, queue, s);
      AIWC_HIP(hipEventRecord(e0, s));
      const GrowLaunch g{codes, codes_p, d_train, d_trial, (int32_t)trial, F->nodes.p, F->node_N.p,
                         F->n_nodes.p, F->work.p, F->inbag.p, queue, scratch.p, base.n_cap};
      launch_grow(c, g, n_cols, binner->d_n_bins.p, y_fp, F->status.p, mtry_max, grid, s);
      AIWC_HIP(hipEventRecord(e1, s));
      AIWC_HIP(hipEventSynchronize(e1));
      float m = 0.0f;
      AIWC_HIP(hipEventElapsedTime(&m, e0, e1));
      if (ms < 0.0f || m < ms) ms = m;
    }
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  AIWC_HIP(hipStreamSynchronize(s));  // the sample's host copy is released here
  tune_store(key, best);
  return best;
}

// Traversal trusts the node words, so it only runs on a forest whose fit
// finished without error (waits for an asynchronous fit).
void require_fitted(const aiwc_rf_forest* f) {
  std::string msg;
  if (resolve_status(f, msg) != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "forest fit failed: " + msg);
}

}  // namespace

extern "C" {

int aiwc_rf_bin(const float* X, const int32_t* device_id, int64_t n, int32_t p, int32_t n_devices, int32_t max_bins,
                aiwc_rf_binner** binner, uint8_t* codes, void* stream) {
  return guard([&] {
    require(X && device_id && codes && binner, "null pointer argument");
    require(n >= 1 && n <= AIWC_RF_MAX_ROWS, "n must be in [1, 2^18]");
    require(p >= 1 && p <= AIWC_RF_MAX_FEATURES, "p must be in [1, 254]");
    require(n_devices >= 1 && n_devices <= 256, "n_devices must be in [1, 256]");
    hipStream_t s = as_stream(stream);
    const bool fit = *binner == nullptr;
    std::unique_ptr<aiwc_rf_binner> fresh;
    aiwc_rf_binner* b = *binner;
    if (fit) {
      require(max_bins >= 2 && max_bins <= AIWC_RF_MAX_BINS, "max_bins must be in [2, 256]");
      fresh.reset(new aiwc_rf_binner());
      b = fresh.get();
      AIWC_HIP(hipGetDevice(&b->device));
      b->p = p;
      b->n_devices = n_devices;
      b->max_bins = max_bins;
      b->has_thresholds = true;
      b->n_bins.assign(p + 1, 0);
      b->thresholds.assign((size_t)p * 255, 0.0f);
      b->d_n_bins.reset(p + 1, s);
      b->d_thresholds.reset((size_t)p * 255, s);
    } else {
      require(b->has_thresholds, "binner carries no thresholds");
      require(b->p == p, "binner was fitted on another number of features");
      require(b->n_devices == n_devices, "binner was fitted with another number of devices");
    }
    DevBuf<uint32_t> status(1, s);
    launch_init(status.p, nullptr, s);
    if (fit) {
      launch_bin_fit(X, device_id, n, p, n_devices, max_bins, b->d_n_bins.p, b->d_thresholds.p, status.p, s);
      launch_set_i32(b->d_n_bins.p + p, n_devices, s);
    }
    launch_bin_encode(X, device_id, n, p, n_devices, b->d_n_bins.p, b->d_thresholds.p, codes, status.p, s);
    uint32_t st = 0;
    const DevicePart parts[3] = {{&st, status.p, sizeof(uint32_t)},
                                 {b->n_bins.data(), b->d_n_bins.p, fit ? sizeof(int32_t) * (size_t)(p + 1) : 0},
                                 {b->thresholds.data(), b->d_thresholds.p, fit ? sizeof(float) * (size_t)p * 255 : 0}};
    download_staged(s, parts, 3);
    std::string msg;
    const int32_t code = status_to_code(st, msg);
    if (code != AIWC_RF_OK) fail(code, msg);
    if (fit) *binner = fresh.release();
  });
}

int aiwc_rf_binner_from_counts(const int32_t* n_bins_host, int32_t n_cols, aiwc_rf_binner** binner) {
  return guard([&] {
    require(n_bins_host && binner, "null pointer argument");
    require(n_cols >= 1 && n_cols <= AIWC_RF_MAX_COLS, "n_cols must be in [1, 255]");
    for (int32_t c = 0; c < n_cols; ++c) require(n_bins_host[c] >= 1 && n_bins_host[c] <= 256, "bin count outside [1, 256]");
    std::unique_ptr<aiwc_rf_binner> b(new aiwc_rf_binner());
    AIWC_HIP(hipGetDevice(&b->device));
    b->p = n_cols - 1;
    b->n_devices = n_bins_host[n_cols - 1];
    b->has_thresholds = false;
    b->n_bins.assign(n_bins_host, n_bins_host + n_cols);
    b->d_n_bins.reset(n_cols, nullptr);
    AIWC_HIP(hipMemcpy(b->d_n_bins.p, n_bins_host, sizeof(int32_t) * n_cols, hipMemcpyHostToDevice));
    *binner = b.release();
  });
}

int aiwc_rf_binner_export_host(const aiwc_rf_binner* b, int32_t* p_host, int32_t* n_devices_host, int32_t* n_bins_host,
                               float* thresholds_host) {
  return guard([&] {
    require(b != nullptr, "binner is NULL");
    if (p_host) *p_host = b->p;
    if (n_devices_host) *n_devices_host = b->n_devices;
    if (n_bins_host) std::memcpy(n_bins_host, b->n_bins.data(), sizeof(int32_t) * b->n_bins.size());
    if (thresholds_host) {
      require(b->has_thresholds, "binner carries no thresholds");
      std::memcpy(thresholds_host, b->thresholds.data(), sizeof(float) * b->thresholds.size());
    }
  });
}

void aiwc_rf_binner_free(aiwc_rf_binner* b) {
  // every call that fills a binner's arrays has completed when it returns;
  // its device arrays go back to the cache behind the streams that used them
  delete b;
}

}  // extern "C"

namespace {

// Training and held-out row lists of a fit: forest k trains on rows
// train[k] = (offset into rows, count), offset -1 meaning rows 0 .. count-1, and
// holds out test[k] = (offset into test_rows, count).
struct RowLists {
  std::vector<int32_t> rows, test_rows;
  std::vector<std::pair<int64_t, int32_t>> train, test;
  template <class Pred>
  std::pair<int64_t, int32_t> add_train(Pred in, int64_t n) {
    const int64_t off = (int64_t)rows.size();
    for (int64_t i = 0; i < n; ++i)
      if (in(i)) rows.push_back((int32_t)i);
    const int64_t cnt = (int64_t)rows.size() - off;
    require(cnt >= 1, "a held-out fold or mask leaves no training rows");
    return {off, (int32_t)cnt};
  }
  template <class Pred>
  std::pair<int64_t, int32_t> add_test(Pred in, int64_t n) {
    const int64_t off = (int64_t)test_rows.size();
    for (int64_t i = 0; i < n; ++i)
      if (in(i)) test_rows.push_back((int32_t)i);
    return {off, (int32_t)((int64_t)test_rows.size() - off)};
  }
};

void check_fit_args(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                    const double* y_log10, const aiwc_rf_params* params_host, int32_t n_forests, uint32_t flags,
                    aiwc_rf_forest** forest) {
  require(codes && binner && y_log10 && params_host && forest, "null pointer argument");
  require(n >= 1 && n <= AIWC_RF_MAX_ROWS, "n must be in [1, 2^18]");
  require(n_cols >= 1 && n_cols <= AIWC_RF_MAX_COLS && (size_t)n_cols == binner->n_bins.size(),
          "n_cols must equal the binner's column count");
  require(n_forests >= 1, "n_forests must be >= 1");
  require((flags & ~(AIWC_RF_FIT_PLAIN | AIWC_RF_FIT_ASYNC | AIWC_RF_FIT_TUNE)) == 0, "unknown flag");
  int64_t total_trees = 0;
  for (int32_t f = 0; f < n_forests; ++f) {
    const aiwc_rf_params& P = params_host[f];
    require(P.num_trees >= 1 && P.num_trees <= AIWC_RF_MAX_TREES, "num_trees must be in [1, 2^14]");
    require(P.mtry >= 1 && P.mtry <= n_cols, "mtry must be in [1, n_cols]");
    require(P.min_node_size >= 1, "min_node_size must be >= 1");
    require(P.bootstrap == 0 || P.bootstrap == 1, "bootstrap must be 0 or 1");
    total_trees += P.num_trees;
  }
  require(total_trees <= (int64_t)INT32_MAX, "too many trees in one call");
}

// Task groups of a fused fit: tree t of every forest that differs from others
// only in min.node.size (same training rows, mtry, bootstrap, seed and tree
// count), by min.node.size ascending, at most kGroupMax to a group; the grow
// kernel grows a group's trees once down to the level where they part.  The
// groups of the costliest forests (training rows x mtry) come first in the
// queue, so that the cheapest ones fill the launch's tail.
void make_task_groups(const aiwc_rf_params* P, int32_t n_forests, const RowLists& L,
                      const std::vector<int64_t>& first_task, std::vector<int32_t>& member,
                      std::vector<int32_t>& first) {
  using Key = std::tuple<int64_t, int32_t, int32_t, int32_t, uint64_t, int32_t>;
  std::map<Key, std::vector<int32_t>> sets;
  std::vector<Key> order;
  for (int32_t f = 0; f < n_forests; ++f) {
    const Key k{L.train[f].first, L.train[f].second, P[f].mtry, P[f].bootstrap, P[f].seed, P[f].num_trees};
    auto it = sets.find(k);
    if (it == sets.end()) {
      order.push_back(k);
      it = sets.emplace(k, std::vector<int32_t>()).first;
    }
    it->second.push_back(f);
  }
  const auto cost = [](const Key& k) { return (int64_t)std::get<1>(k) * std::get<2>(k); };
  std::stable_sort(order.begin(), order.end(), [&](const Key& x, const Key& y) { return cost(x) > cost(y); });
  for (const Key& k : order) {
    std::vector<int32_t>& fs = sets[k];
    std::stable_sort(fs.begin(), fs.end(),
                     [&](int32_t x, int32_t y) { return P[x].min_node_size < P[y].min_node_size; });
    const int32_t nt = std::get<5>(k);
    for (size_t c = 0; c < fs.size(); c += kGroupMax) {
      const size_t e = std::min(fs.size(), c + (size_t)kGroupMax);
      for (int32_t t = 0; t < nt; ++t) {
        first.push_back((int32_t)member.size());
        for (size_t j = c; j < e; ++j) member.push_back((int32_t)(first_task[(size_t)fs[j]] + t));
      }
    }
  }
  first.push_back((int32_t)member.size());
}

// The fit of n_forests forests whose training (and held-out) rows are given
// by L; validation of the arguments is done by the caller.
void fit_common(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner, const double* y_log10,
                const aiwc_rf_params* params_host, int32_t n_forests, uint32_t flags, const RowLists& L,
                aiwc_rf_forest** forest, hipStream_t s) {
  int64_t total_trees = 0;
  int32_t mtry_max = 1;
  for (int32_t f = 0; f < n_forests; ++f) {
    total_trees += params_host[f].num_trees;
    mtry_max = std::max(mtry_max, params_host[f].mtry);
  }
  const std::vector<int32_t>& train_rows = L.rows;
  std::unique_ptr<aiwc_rf_forest> F(new aiwc_rf_forest());
  AIWC_HIP(hipGetDevice(&F->device));
  F->n_cols = n_cols;
  F->n_bins = binner->n_bins;
  F->params.assign(params_host, params_host + n_forests);
  F->tasks.reserve((size_t)total_trees);
  int64_t pool = 0, n_cap = 1, inbag_words = 0;
  for (int32_t f = 0; f < n_forests; ++f) {
    const aiwc_rf_params& P = params_host[f];
    const auto& Lf = L.train[f];
    F->first_task.push_back((int64_t)F->tasks.size());
    F->n_train.push_back(Lf.second);
    F->train_off.push_back(Lf.first);
    F->n_test.push_back(L.test[f].second);
    F->test_off.push_back(L.test[f].first);
    const int64_t cap = 2 * (int64_t)Lf.second - 1;
    n_cap = std::max<int64_t>(n_cap, Lf.second);
    for (int32_t t = 0; t < P.num_trees; ++t) {
      TreeTask T;
      T.forest = f;
      T.tree = t;
      T.n_train = Lf.second;
      T.mtry = P.mtry;
      T.min_node = P.min_node_size;
      T.bootstrap = P.bootstrap;
      T.seed = P.seed;
      T.train_off = Lf.first;
      T.node_base = pool;
      T.capacity = cap;
      T.inbag_off = P.bootstrap ? inbag_words : -1;
      if (P.bootstrap) inbag_words += (Lf.second + 63) / 64;
      pool += cap;
      F->tasks.push_back(T);
    }
  }
  F->pool_nodes = pool;
  const int64_t n_tasks = (int64_t)F->tasks.size();
  const bool plain = n_forests > 1 && (flags & AIWC_RF_FIT_PLAIN);
  // a fused fit of several forests grows its trees in task groups
  std::vector<int32_t> group_task, group_first;
  if (n_forests > 1 && !plain) make_task_groups(params_host, n_forests, L, F->first_task, group_task, group_first);
  const bool grouped = !group_first.empty();
  const int64_t n_groups = grouped ? (int64_t)group_first.size() - 1 : n_tasks;

  F->d_tasks.reset((size_t)n_tasks, s);
  F->nodes.reset((size_t)pool, s);
  F->node_N.reset((size_t)pool, s);
  F->n_nodes.reset((size_t)n_tasks, s);
  F->work.reset((size_t)n_tasks * kWorkWords, s);
  F->node_base.reset((size_t)n_tasks, s);
  F->status.reset(1, s);
  F->status_host = pinned_word_acquire();
  *F->status_host = 0;
  AIWC_HIP(hipEventCreateWithFlags(&F->done, hipEventDisableTiming));
  AIWC_HIP(hipEventCreate(&F->grow_begin));
  AIWC_HIP(hipEventCreate(&F->grow_end));
  {
    std::vector<int64_t> bases((size_t)n_tasks);
    for (int64_t i = 0; i < n_tasks; ++i) bases[i] = F->tasks[i].node_base;
    F->group_task.reset(group_task.size(), s);
    F->group_first.reset(group_first.size(), s);
    const HostPart parts[4] = {{F->d_tasks.p, F->tasks.data(), sizeof(TreeTask) * (size_t)n_tasks},
                               {F->node_base.p, bases.data(), sizeof(int64_t) * (size_t)n_tasks},
                               {F->group_task.p, group_task.data(), sizeof(int32_t) * group_task.size()},
                               {F->group_first.p, group_first.data(), sizeof(int32_t) * group_first.size()}};
    upload_staged(s, parts, grouped ? 4 : 2);
  }
  F->train_rows.reset(train_rows.size(), s);
  DevBuf<int32_t>& d_train = F->train_rows;
  if (!train_rows.empty())
    AIWC_HIP(hipMemcpyAsync(d_train.p, train_rows.data(), sizeof(int32_t) * train_rows.size(), hipMemcpyHostToDevice, s));
  F->inbag.reset((size_t)inbag_words, s);
  F->test_rows.reset(L.test_rows.size(), s);
  if (!L.test_rows.empty())
    AIWC_HIP(hipMemcpyAsync(F->test_rows.p, L.test_rows.data(), sizeof(int32_t) * L.test_rows.size(),
                            hipMemcpyHostToDevice, s));
  DevBuf<int64_t> y_fp((size_t)n, s);
  DevBuf<uint8_t> codes_p((size_t)n * padded_cols(n_cols) + 64, s);  // slack for 80-byte reads of the last row
  DevBuf<uint32_t> queue(1, s);

  // the work items of the (largest) launch: the task groups of a fused fit,
  // a forest's trees when every forest is launched on its own, as separate
  // fits would be
  int64_t n_items = n_groups;
  if (plain) {
    n_items = 0;
    for (int32_t f = 0; f < n_forests; ++f) n_items = std::max<int64_t>(n_items, params_host[f].num_trees);
  }
  GrowConfig cfg = grow_config(n_cap, n_items, binner->n_bins);
  bool tuned = false;
  if (flags & AIWC_RF_FIT_TUNE) {
    cfg = tune_grow(cfg, n_items, n_cols, mtry_max, F.get(), codes, n, binner, y_log10, y_fp.p, codes_p.p, d_train.p,
                    queue.p, s);
    tuned = true;
  }
  const size_t per_wg = grow_scratch_bytes(n_cap, mtry_max, grow_has_wide_phase(cfg), grouped);
  aiwc_rf_launch_info& LI = F->launch;
  LI.block = cfg.block;
  LI.waves_per_simd = grow_has_wide_phase(cfg) ? 4 : cfg.occupancy;
  LI.wide_limit = cfg.huge_min;
  LI.big_cols = effective_big_cols(cfg, mtry_max, n_cols);
  LI.wide_phase = grow_has_wide_phase(cfg) ? 1 : 0;
  LI.tuned = tuned ? 1 : 0;
  LI.task_groups = (int32_t)n_groups;

  if (plain) {
    // one launch sequence per forest, as separate fits would issue them
    const int grid_max = grow_grid_size(cfg, n_tasks, mtry_max, n_cols);
    DevBuf<uint8_t> scratch(per_wg * (size_t)grid_max, s);
    launch_init(F->status.p, nullptr, s);
    AIWC_HIP(hipEventRecord(F->grow_begin, s));
    int grid_used = 0;
    for (int32_t f = 0; f < n_forests; ++f) {
      const int64_t t0 = F->first_task[f];
      const int32_t nt = params_host[f].num_trees;
      const int grid = grow_grid_size(cfg, nt, mtry_max, n_cols);
      grid_used = std::max(grid_used, grid);
      launch_init(nullptr, queue.p, s);
      launch_prepare(codes, n, n_cols, binner->d_n_bins.p, y_log10, y_fp.p, codes_p.p, F->status.p, s);
      const GrowLaunch g{codes, codes_p.p, d_train.p, F->d_tasks.p + t0, nt, F->nodes.p, F->node_N.p,
                         F->n_nodes.p + t0, F->work.p + kWorkWords * t0, F->inbag.p, queue.p, scratch.p, n_cap};
      launch_grow(cfg, g, n_cols, binner->d_n_bins.p, y_fp.p, F->status.p, mtry_max, grid, s);
    }
    AIWC_HIP(hipEventRecord(F->grow_end, s));
    LI.grid = grid_used;
  } else {
    const int grid = grow_grid_size(cfg, n_groups, mtry_max, n_cols, grouped);
    LI.grid = grid;
    DevBuf<uint8_t> scratch(per_wg * (size_t)grid, s);
    const GrowLaunch g{codes,     codes_p.p, d_train.p,
                       F->d_tasks.p, (int32_t)n_tasks, F->nodes.p,
                       F->node_N.p, F->n_nodes.p, F->work.p,
                       F->inbag.p, queue.p,   scratch.p,
                       n_cap,     grouped ? F->group_task.p : nullptr, grouped ? F->group_first.p : nullptr,
                       (int32_t)n_groups};
    if (n_forests > 1) {
      // fused grid: the whole fit as one executable-graph launch (timing events
      // bracket the whole graph: reset, prepare, grow)
      AIWC_HIP(hipEventRecord(F->grow_begin, s));
      const bool reused = launch_fit_graph(cfg, g, codes, n, n_cols, binner->d_n_bins.p, y_log10, y_fp.p, F->status.p,
                                           mtry_max, grid, s);
      AIWC_HIP(hipEventRecord(F->grow_end, s));
      LI.graph = 1;
      LI.graph_reused = reused ? 1 : 0;
    } else {
      launch_init(F->status.p, queue.p, s);
      launch_prepare(codes, n, n_cols, binner->d_n_bins.p, y_log10, y_fp.p, codes_p.p, F->status.p, s);
      AIWC_HIP(hipEventRecord(F->grow_begin, s));
      launch_grow(cfg, g, n_cols, binner->d_n_bins.p, y_fp.p, F->status.p, mtry_max, grid, s);
      AIWC_HIP(hipEventRecord(F->grow_end, s));
    }
  }
  AIWC_HIP(hipMemcpyAsync(F->status_host, F->status.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  AIWC_HIP(hipEventRecord(F->done, s));
  if (!(flags & AIWC_RF_FIT_ASYNC)) {
    std::string msg;
    const int32_t code = resolve_status(F.get(), msg);
    if (code != AIWC_RF_OK) fail(code, msg);
  }
  *forest = F.release();
}

}  // namespace

extern "C" {

int aiwc_rf_fit(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner, const double* y_log10,
                const int8_t* fold_id, const aiwc_rf_params* params_host, const int32_t* heldout_fold_host,
                int32_t n_forests, uint32_t flags, aiwc_rf_forest** forest, void* stream) {
  return guard([&] {
    check_fit_args(codes, n, n_cols, binner, y_log10, params_host, n_forests, flags, forest);
    hipStream_t s = as_stream(stream);
    bool need_folds = false;
    for (int32_t f = 0; f < n_forests; ++f) {
      const int32_t h = heldout_fold_host ? heldout_fold_host[f] : -1;
      require(h >= -1 && h <= 127, "heldout fold must be in [-1, 127]");
      need_folds |= h >= 0;
    }
    require(!need_folds || fold_id != nullptr, "fold_id is NULL but a forest holds out a fold");
    // training and held-out row lists, one pair per distinct held-out fold
    RowLists L;
    L.train.assign((size_t)n_forests, {-1, (int32_t)n});
    L.test.assign((size_t)n_forests, {0, 0});
    if (need_folds) {
      std::vector<int8_t> folds((size_t)n);
      AIWC_HIP(hipMemcpyAsync(folds.data(), fold_id, (size_t)n, hipMemcpyDeviceToHost, s));
      AIWC_HIP(hipStreamSynchronize(s));
      std::map<int32_t, std::pair<std::pair<int64_t, int32_t>, std::pair<int64_t, int32_t>>> made;
      for (int32_t f = 0; f < n_forests; ++f) {
        const int32_t h = heldout_fold_host[f];
        if (h < 0) continue;
        auto it = made.find(h);
        if (it == made.end()) {
          const auto tr = L.add_train([&](int64_t i) { return folds[i] != h; }, n);
          const auto te = L.add_test([&](int64_t i) { return folds[i] == h; }, n);
          it = made.emplace(h, std::make_pair(tr, te)).first;
        }
        L.train[f] = it->second.first;
        L.test[f] = it->second.second;
      }
    }
    fit_common(codes, n, n_cols, binner, y_log10, params_host, n_forests, flags, L, forest, s);
  });
}

int aiwc_rf_fit_groups(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                       const double* y_log10, const int8_t* group_id, const uint64_t* train_mask_host,
                       const aiwc_rf_params* params_host, int32_t n_forests, uint32_t flags, aiwc_rf_forest** forest,
                       void* stream) {
  return guard([&] {
    check_fit_args(codes, n, n_cols, binner, y_log10, params_host, n_forests, flags, forest);
    require(group_id && train_mask_host, "null pointer argument");
    hipStream_t s = as_stream(stream);
    std::vector<int8_t> groups((size_t)n);
    AIWC_HIP(hipMemcpyAsync(groups.data(), group_id, (size_t)n, hipMemcpyDeviceToHost, s));
    AIWC_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) require(groups[i] >= -1 && groups[i] <= 63, "group_id must be in [-1, 63]");
    RowLists L;
    L.train.resize((size_t)n_forests);
    L.test.resize((size_t)n_forests);
    std::map<uint64_t, std::pair<std::pair<int64_t, int32_t>, std::pair<int64_t, int32_t>>> made;
    for (int32_t f = 0; f < n_forests; ++f) {
      const uint64_t m = train_mask_host[f];
      auto it = made.find(m);
      if (it == made.end()) {
        const auto in = [&](int64_t i) { return groups[i] < 0 || ((m >> groups[i]) & 1ull) != 0; };
        const auto tr = L.add_train(in, n);
        require(tr.second >= 1, "a training mask selects no rows");
        const auto te = L.add_test([&](int64_t i) { return !in(i); }, n);
        it = made.emplace(m, std::make_pair(tr, te)).first;
      }
      L.train[f] = it->second.first;
      L.test[f] = it->second.second;
    }
    fit_common(codes, n, n_cols, binner, y_log10, params_host, n_forests, flags, L, forest, s);
  });
}

int aiwc_rf_forest_wait(const aiwc_rf_forest* f) {
  int32_t code = AIWC_RF_OK;
  std::string msg;
  const int rc = guard([&] {
    require(f != nullptr, "forest is NULL");
    code = resolve_status(f, msg);
  });
  if (rc != AIWC_RF_OK) return rc;
  if (code != AIWC_RF_OK) set_last_error(msg);
  return code;
}

int aiwc_rf_forest_info(const aiwc_rf_forest* f, int32_t forest_index, int32_t* n_forests_host, int32_t* n_cols_host,
                        int32_t* num_trees_host, int64_t* total_nodes_host) {
  return guard([&] {
    check_forest(f, forest_index);
    if (n_forests_host) *n_forests_host = (int32_t)f->params.size();
    if (n_cols_host) *n_cols_host = f->n_cols;
    if (num_trees_host) *num_trees_host = f->params[forest_index].num_trees;
    if (total_nodes_host) {
      std::string msg;
      const int32_t code = resolve_status(f, msg);
      if (code != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "fit failed: " + msg);
      const int32_t nt = f->params[forest_index].num_trees;
      std::vector<int32_t> nn((size_t)nt);
      AIWC_HIP(hipMemcpy(nn.data(), f->n_nodes.p + f->first_task[forest_index], sizeof(int32_t) * nt,
                         hipMemcpyDeviceToHost));
      int64_t tot = 0;
      for (int32_t v : nn) tot += v;
      *total_nodes_host = tot;
    }
  });
}

int aiwc_rf_forest_stats(const aiwc_rf_forest* f, int32_t forest_index, int64_t* work_host, float* grow_ms_host) {
  return guard([&] {
    check_forest(f, forest_index);
    std::string msg;
    const int32_t code = resolve_status(f, msg);
    if (code != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "fit failed: " + msg);
    if (work_host) {
      const int32_t nt = f->params[forest_index].num_trees;
      std::vector<int64_t> w((size_t)nt * kWorkWords);
      AIWC_HIP(hipMemcpy(w.data(), f->work.p + kWorkWords * f->first_task[forest_index], sizeof(int64_t) * w.size(),
                         hipMemcpyDeviceToHost));
      for (int i = 0; i < kWorkWords; ++i) work_host[i] = 0;
      for (int32_t t = 0; t < nt; ++t) {
        for (int i = 0; i < kWorkWords; ++i)
          work_host[i] = i == 3 ? std::max(work_host[i], w[kWorkWords * t + i]) : work_host[i] + w[kWorkWords * t + i];
      }
    }
    if (grow_ms_host) AIWC_HIP(hipEventElapsedTime(grow_ms_host, f->grow_begin, f->grow_end));
  });
}

int aiwc_rf_forest_launch(const aiwc_rf_forest* f, aiwc_rf_launch_info* info_host) {
  return guard([&] {
    require(f != nullptr && info_host != nullptr, "null pointer argument");
    *info_host = f->launch;
  });
}

int aiwc_rf_forest_tree_sizes(const aiwc_rf_forest* f, int32_t forest_index, int32_t tree_begin, int32_t tree_end,
                              int64_t* n_nodes_host) {
  return guard([&] {
    check_forest(f, forest_index);
    require(n_nodes_host != nullptr, "null pointer argument");
    const int32_t nt = f->params[forest_index].num_trees;
    require(tree_begin >= 0 && tree_begin < tree_end && tree_end <= nt, "tree range out of bounds");
    std::string msg;
    const int32_t code = resolve_status(f, msg);
    if (code != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "fit failed: " + msg);
    std::vector<int32_t> nn((size_t)(tree_end - tree_begin));
    AIWC_HIP(hipMemcpy(nn.data(), f->n_nodes.p + f->first_task[forest_index] + tree_begin,
                       sizeof(int32_t) * nn.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < nn.size(); ++i) n_nodes_host[i] = nn[i];
  });
}

int aiwc_rf_forest_export_host(const aiwc_rf_forest* f, int32_t forest_index, int32_t tree_begin, int32_t tree_end,
                               uint8_t* col_host, uint8_t* bin_host, int32_t* left_host, int64_t* q_host,
                               int32_t* N_host) {
  return guard([&] {
    check_forest(f, forest_index);
    const int32_t nt = f->params[forest_index].num_trees;
    require(tree_begin >= 0 && tree_begin < tree_end && tree_end <= nt, "tree range out of bounds");
    std::string msg;
    const int32_t code = resolve_status(f, msg);
    if (code != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "fit failed: " + msg);
    const int64_t t0 = f->first_task[forest_index];
    std::vector<int32_t> nn((size_t)(tree_end - tree_begin));
    AIWC_HIP(hipMemcpy(nn.data(), f->n_nodes.p + t0 + tree_begin, sizeof(int32_t) * nn.size(), hipMemcpyDeviceToHost));
    size_t out = 0;
    std::vector<uint64_t> words;
    std::vector<uint32_t> N;
    for (int32_t t = tree_begin; t < tree_end; ++t) {
      const size_t cnt = (size_t)nn[t - tree_begin];
      const int64_t base = f->tasks[t0 + t].node_base;
      words.resize(cnt);
      N.resize(cnt);
      AIWC_HIP(hipMemcpy(words.data(), f->nodes.p + base, sizeof(uint64_t) * cnt, hipMemcpyDeviceToHost));
      AIWC_HIP(hipMemcpy(N.data(), f->node_N.p + base, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost));
      unpack_nodes(words, N, cnt, col_host ? col_host + out : nullptr, bin_host ? bin_host + out : nullptr,
                   left_host ? left_host + out : nullptr, q_host ? q_host + out : nullptr,
                   N_host ? N_host + out : nullptr);
      out += cnt;
    }
  });
}

void aiwc_rf_forest_free(aiwc_rf_forest* f) {
  if (!f) return;
  // only the fit's own stream is waited for (its status word is copied there);
  // work the caller enqueued on other streams must be complete (header)
  if (f->done) (void)hipEventSynchronize(f->done);
  if (f->done) (void)hipEventDestroy(f->done);
  if (f->grow_begin) (void)hipEventDestroy(f->grow_begin);
  if (f->grow_end) (void)hipEventDestroy(f->grow_end);
  pinned_word_release(f->status_host);
  delete f;
}

int aiwc_rf_predict(const aiwc_rf_forest* f, int32_t forest_index, const uint8_t* codes, int64_t n, double* y_log10_out,
                    void* stream) {
  return guard([&] {
    check_forest(f, forest_index);
    require(n >= 0, "n must be >= 0");
    if (n == 0) return;
    require(codes && y_log10_out, "null pointer argument");
    hipStream_t s = as_stream(stream);
    const int32_t nt = f->params[forest_index].num_trees;
    const int64_t t0 = f->first_task[forest_index];
    require_fitted(f);
    DevBuf<int64_t> sum((size_t)n, s);
    launch_predict(f->nodes.p, f->node_base.p, (int32_t)t0, (int32_t)(t0 + nt), codes, n, f->n_cols, sum.p,
                   y_log10_out, nt, s);
  });
}

int aiwc_rf_predict_noalloc(const aiwc_rf_forest* f, int32_t forest_index, const uint8_t* codes, int64_t n,
                            double* y_log10_out, void* stream) {
  return guard([&] {
    check_forest(f, forest_index);
    require(n >= 0, "n must be >= 0");
    if (n == 0) return;
    require(codes && y_log10_out, "null pointer argument");
    require(n <= kNoAllocPredictRows, "n exceeds the allocation-free limit of 2^20 rows per call");
    int dev = 0;
    AIWC_HIP(hipGetDevice(&dev));
    require(dev == f->device, "the current device is not the forest's device");
    hipStream_t s = as_stream(stream);
    const int32_t nt = f->params[forest_index].num_trees;
    const int64_t t0 = f->first_task[forest_index];
    require_fitted(f);
    // the same kernels as aiwc_rf_predict, with the row sums in the fixed array
    launch_predict(f->nodes.p, f->node_base.p, (int32_t)t0, (int32_t)(t0 + nt), codes, n, f->n_cols,
                   noalloc_predict_scratch(), y_log10_out, nt, s);
  });
}

int aiwc_rf_predict_sum(const aiwc_rf_forest* f, int32_t forest_index, int32_t tree_begin, int32_t tree_end,
                        const uint8_t* codes, int64_t n, int64_t* sum_out, void* stream) {
  return guard([&] {
    check_forest(f, forest_index);
    const int32_t nt = f->params[forest_index].num_trees;
    require(tree_begin >= 0 && tree_begin < tree_end && tree_end <= nt, "tree range out of bounds");
    require(n >= 0, "n must be >= 0");
    if (n == 0) return;
    require(codes && sum_out, "null pointer argument");
    hipStream_t s = as_stream(stream);
    const int64_t t0 = f->first_task[forest_index];
    require_fitted(f);
    launch_predict(f->nodes.p, f->node_base.p, (int32_t)(t0 + tree_begin), (int32_t)(t0 + tree_end), codes, n,
                   f->n_cols, sum_out, nullptr, nt, s);
  });
}

int aiwc_rf_oob_error(const aiwc_rf_forest* f, int32_t forest_begin, int32_t forest_end, const uint8_t* codes,
                      const double* y_log10, int64_t* oob_sum_out, int32_t* oob_count_out, double* mse_host,
                      double* mae_host, int64_t* rows_host, void* stream) {
  return guard([&] {
    require(f != nullptr, "forest is NULL");
    require(forest_begin >= 0 && forest_begin < forest_end && forest_end <= (int32_t)f->params.size(),
            "forest range out of bounds");
    require(codes && y_log10, "null pointer argument");
    hipStream_t s = as_stream(stream);
    require_fitted(f);
    const int32_t nf = forest_end - forest_begin;
    std::vector<OobForest> fr((size_t)nf);
    int64_t rows = 0;
    int32_t max_n = 1;
    for (int32_t k = 0; k < nf; ++k) {
      const int32_t fi = forest_begin + k;
      fr[k].first_task = f->first_task[fi];
      fr[k].num_trees = f->params[fi].num_trees;
      fr[k].n_train = f->n_train[fi];
      fr[k].train_off = f->train_off[fi];
      fr[k].row_off = rows;
      rows += f->n_train[fi];
      max_n = std::max(max_n, f->n_train[fi]);
    }
    DevBuf<OobForest> d_fr((size_t)nf, s);
    AIWC_HIP(hipMemcpyAsync(d_fr.p, fr.data(), sizeof(OobForest) * nf, hipMemcpyHostToDevice, s));
    DevBuf<int64_t> sum_tmp(oob_sum_out ? 0 : (size_t)rows, s);
    DevBuf<int32_t> cnt_tmp(oob_count_out ? 0 : (size_t)rows, s);
    const int32_t blocks = (max_n + 255) / 256;
    DevBuf<double> partial((size_t)3 * nf * blocks, s);
    DevBuf<double> result((size_t)3 * nf, s);
    launch_oob(f->nodes.p, f->d_tasks.p, f->node_base.p, f->inbag.p, f->train_rows.p, d_fr.p, nf, max_n, codes,
               f->n_cols, y_log10, oob_sum_out ? oob_sum_out : sum_tmp.p, oob_count_out ? oob_count_out : cnt_tmp.p,
               partial.p, result.p, s);
    std::vector<double> res((size_t)3 * nf);
    AIWC_HIP(hipMemcpyAsync(res.data(), result.p, sizeof(double) * res.size(), hipMemcpyDeviceToHost, s));
    AIWC_HIP(hipStreamSynchronize(s));
    for (int32_t k = 0; k < nf; ++k) {
      if (mse_host) mse_host[k] = res[3 * k];
      if (mae_host) mae_host[k] = res[3 * k + 1];
      if (rows_host) rows_host[k] = (int64_t)res[3 * k + 2];
    }
  });
}

int aiwc_rf_heldout_error(const aiwc_rf_forest* f, int32_t forest_begin, int32_t forest_end, const uint8_t* codes,
                          const double* y_log10, int64_t* pred_sum_out, double* mse_host, double* mae_host,
                          int64_t* rows_host, void* stream) {
  return guard([&] {
    require(f != nullptr, "forest is NULL");
    require(forest_begin >= 0 && forest_begin < forest_end && forest_end <= (int32_t)f->params.size(),
            "forest range out of bounds");
    require(codes && y_log10, "null pointer argument");
    hipStream_t s = as_stream(stream);
    require_fitted(f);
    const int32_t nf = forest_end - forest_begin;
    std::vector<OobForest> fr((size_t)nf);
    int64_t rows = 0;
    int32_t max_n = 0;
    for (int32_t k = 0; k < nf; ++k) {
      const int32_t fi = forest_begin + k;
      fr[k].first_task = f->first_task[fi];
      fr[k].num_trees = f->params[fi].num_trees;
      fr[k].n_train = f->n_test[fi];
      fr[k].train_off = f->test_off[fi];
      fr[k].row_off = rows;
      rows += f->n_test[fi];
      max_n = std::max(max_n, f->n_test[fi]);
    }
    std::vector<double> res((size_t)3 * nf, 0.0);
    if (rows > 0) {
      DevBuf<OobForest> d_fr((size_t)nf, s);
      AIWC_HIP(hipMemcpyAsync(d_fr.p, fr.data(), sizeof(OobForest) * nf, hipMemcpyHostToDevice, s));
      DevBuf<int64_t> sum_tmp(pred_sum_out ? 0 : (size_t)rows, s);
      DevBuf<int32_t> cnt((size_t)rows, s);
      const int32_t blocks = std::max(1, (max_n + 255) / 256);
      DevBuf<double> partial((size_t)3 * nf * blocks, s);
      DevBuf<double> result((size_t)3 * nf, s);
      launch_heldout(f->nodes.p, f->node_base.p, f->test_rows.p, d_fr.p, nf, max_n, codes, f->n_cols, y_log10,
                     pred_sum_out ? pred_sum_out : sum_tmp.p, cnt.p, partial.p, result.p, s);
      AIWC_HIP(hipMemcpyAsync(res.data(), result.p, sizeof(double) * res.size(), hipMemcpyDeviceToHost, s));
    }
    AIWC_HIP(hipStreamSynchronize(s));
    for (int32_t k = 0; k < nf; ++k) {
      if (mse_host) mse_host[k] = res[3 * k];
      if (mae_host) mae_host[k] = res[3 * k + 1];
      if (rows_host) rows_host[k] = (int64_t)res[3 * k + 2];
    }
  });
}

int aiwc_rf_tune_sa(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                    const double* y_log10, const aiwc_rf_sa_config* cfg, int32_t* best_params_host,
                    double* best_objective_host, aiwc_rf_sa_step* trace_host, void* stream) {
  return guard([&] {
    require(codes && binner && y_log10 && cfg && best_params_host && best_objective_host, "null pointer argument");
    require(n >= 1 && n <= AIWC_RF_MAX_ROWS, "n must be in [1, 2^18]");
    require(n_cols >= 1 && n_cols <= AIWC_RF_MAX_COLS && (size_t)n_cols == binner->n_bins.size(),
            "n_cols must equal the binner's column count");
    anneal(codes, n, n_cols, binner, y_log10, *cfg, best_params_host, best_objective_host, trace_host,
           as_stream(stream));
  });
}

int aiwc_rf_heldout_rows(const aiwc_rf_forest* f, int32_t forest_index, int32_t* rows_out_host, int32_t* n_host) {
  return guard([&] {
    check_forest(f, forest_index);
    require(n_host != nullptr, "null pointer argument");
    const int32_t cnt = f->n_test[forest_index];
    *n_host = cnt;
    if (rows_out_host && cnt > 0)
      AIWC_HIP(hipMemcpy(rows_out_host, f->test_rows.p + f->test_off[forest_index], sizeof(int32_t) * cnt,
                         hipMemcpyDeviceToHost));
  });
}

int aiwc_rf_select_device(const aiwc_rf_forest* f, int32_t forest_index, const uint8_t* feature_codes, int64_t m,
                          double* times_out, int32_t* best_out, void* stream) {
  return guard([&] {
    check_forest(f, forest_index);
    require(m >= 0, "m must be >= 0");
    if (m == 0) return;
    require(feature_codes && best_out, "null pointer argument");
    require(f->n_cols >= 2, "the forest has no feature column besides the device");
    hipStream_t s = as_stream(stream);
    const int32_t D = f->n_bins.back();
    const int32_t nt = f->params[forest_index].num_trees;
    const int64_t t0 = f->first_task[forest_index];
    require_fitted(f);
    const int64_t rows = m * D;
    DevBuf<uint8_t> expanded((size_t)(rows * f->n_cols), s);
    DevBuf<int64_t> sum((size_t)rows, s);
    DevBuf<double> times_tmp(times_out ? 0 : (size_t)rows, s);
    launch_select_device(f->nodes.p, f->node_base.p, (int32_t)t0, (int32_t)(t0 + nt), feature_codes, m, f->n_cols, D,
                         nt, expanded.p, sum.p, times_out ? times_out : times_tmp.p, best_out, s);
  });
}

int aiwc_rf_rank_accuracy(const double* times, const double* truth, int64_t m, int32_t n_devices,
                          int32_t* correct_out, int32_t* counted_out, int32_t* hit_out, void* stream) {
  return guard([&] {
    require(m >= 0, "m must be >= 0");
    require(n_devices >= 1 && n_devices <= 256, "n_devices must be in [1, 256]");
    if (m == 0) return;
    require(times && truth, "null pointer argument");
    launch_rank_accuracy(times, truth, m, n_devices, correct_out, counted_out, hit_out, as_stream(stream));
  });
}

}  // extern "C"
