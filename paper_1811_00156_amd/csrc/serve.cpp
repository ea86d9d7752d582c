// Prediction server: a resident forest answering a stream of requests of
// different sizes (the scheduler-facing query of Sec. I and Sec. VI).
//
// Memory.  At creation the server takes one device arena and one pinned host
// arena whose sizes add up to at most the memory budget.  Both are cut into the
// same K row slots (a row costs n_cols + 16 device bytes: codes, the int64 sum
// and the float64 answer; and n_cols + 8 pinned bytes: staged codes and the
// answer), so a batch of R rows is one contiguous range of R slots, taken from a
// first-fit free list and handed back when the batch retires.  A request is
// admitted only when its batch gets a range: requests that arrive while the
// arenas are full wait in FIFO order until a retiring batch frees slots, and no
// more than the budget is ever held.
//
// Batching.  One dispatcher thread owns n_streams HIP streams.  Whenever a
// stream is free it packs the oldest waiting requests into one batch for as long
// as they fit max_batch_rows and the largest free range; copies in, traversal
// and copies out of the batch are enqueued on that stream, so batches on
// different streams overlap on the device while new requests keep arriving.
// Finished batches are scattered back to the callers' output arrays.  Each row
// is traversed exactly as by aiwc_rf_predict, so an answer never depends on
// what it was batched with.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"

using namespace aiwc;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket;
  const uint8_t* codes;
  int64_t n;
  double* out;
  Clock::time_point submitted;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Request> reqs;
  int64_t first = 0;  // first row slot of the batch's range
  int64_t rows = 0;
  bool busy = false;
};

// First-fit allocator of contiguous ranges of row slots [0, capacity).
class RangePool {
 public:
  void reset(int64_t capacity) {
    free_.clear();
    if (capacity > 0) free_[0] = capacity;
    used_ = 0;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  // First slot of a range of `len` slots, or -1 if no free range is that long.
  int64_t take(int64_t len) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      const int64_t at = it->first, rest = it->second - len;
      free_.erase(it);
      if (rest > 0) free_[at + len] = rest;
      used_ += len;
      return at;
    }
    return -1;
  }
  void give(int64_t at, int64_t len) {
    used_ -= len;
    auto it = free_.emplace(at, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t used() const { return used_; }

 private:
  std::map<int64_t, int64_t> free_;  // first slot -> length
  int64_t used_ = 0;
};

}  // namespace

struct aiwc_rf_server {
  const aiwc_rf_forest* forest = nullptr;
  int32_t forest_index = 0;
  int32_t n_cols = 0;
  int32_t num_trees = 0;
  int64_t t0 = 0;
  int64_t budget = 0;
  int64_t max_rows = 0;
  int64_t capacity = 0;  // row slots of the arenas
  int64_t row_bytes = 0;  // device + pinned bytes of one row slot
  int device = 0;

  // arenas: device codes | int64 sums | float64 answers; pinned codes | answers
  uint8_t* d_arena = nullptr;
  uint8_t* h_arena = nullptr;
  uint8_t* d_codes = nullptr;
  int64_t* d_sum = nullptr;
  double* d_out = nullptr;
  uint8_t* h_codes = nullptr;
  double* h_out = nullptr;

  std::mutex mu;
  std::condition_variable cv_work;  // dispatcher waits for requests
  std::condition_variable cv_idle;  // drain waits for completion
  std::deque<Request> pending;
  std::deque<std::pair<int64_t, double>> completed;
  std::vector<Slot> slots;
  RangePool pool;
  int64_t next_ticket = 0;
  int64_t rows_served = 0;
  int64_t batches = 0;
  int64_t peak_bytes = 0;
  int64_t memory_waits = 0;  // times the oldest request waited for arena slots
  int busy_slots = 0;
  bool stop = false;
  std::string error;
  std::thread dispatcher;

  void run();
  void launch(Slot& s, std::vector<Request>&& batch, int64_t first, int64_t rows);
  void retire(Slot& s);
  void release_resources();
};

void aiwc_rf_server::launch(Slot& s, std::vector<Request>&& batch, int64_t first, int64_t rows) {
  uint8_t* hc = h_codes + first * n_cols;
  int64_t off = 0;
  for (const Request& r : batch) {
    std::memcpy(hc + off * n_cols, r.codes, (size_t)(r.n * n_cols));
    off += r.n;
  }
  s.first = first;
  s.rows = rows;
  s.reqs = std::move(batch);
  uint8_t* dc = d_codes + first * n_cols;
  AIWC_HIP(hipMemcpyAsync(dc, hc, (size_t)(rows * n_cols), hipMemcpyHostToDevice, s.stream));
  launch_predict(forest->nodes.p, forest->node_base.p, (int32_t)t0, (int32_t)(t0 + num_trees), dc, rows, n_cols,
                 d_sum + first, d_out + first, num_trees, s.stream);
  AIWC_HIP(hipMemcpyAsync(h_out + first, d_out + first, sizeof(double) * (size_t)rows, hipMemcpyDeviceToHost,
                          s.stream));
  AIWC_HIP(hipEventRecord(s.done, s.stream));
  s.busy = true;
}

void aiwc_rf_server::retire(Slot& s) {
  int64_t off = 0;
  const Clock::time_point now = Clock::now();
  std::vector<std::pair<int64_t, double>> done;
  for (const Request& r : s.reqs) {
    std::memcpy(r.out, h_out + s.first + off, sizeof(double) * (size_t)r.n);
    off += r.n;
    done.emplace_back(r.ticket, std::chrono::duration<double>(now - r.submitted).count());
  }
  std::lock_guard<std::mutex> g(mu);
  pool.give(s.first, s.rows);
  rows_served += s.rows;
  for (auto& d : done) completed.push_back(d);
  s.reqs.clear();
  s.busy = false;
  --busy_slots;
  cv_idle.notify_all();
}

void aiwc_rf_server::run() {
  try {
    AIWC_HIP(hipSetDevice(device));
    bool head_waited = false;  // the current head request already counted a wait
    for (;;) {
      // retire finished batches; any status but "done" or "not ready" is an error
      for (Slot& s : slots) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipSuccess)
          retire(s);
        else if (q != hipErrorNotReady)
          AIWC_HIP(q);
      }
      // pack a batch for a free stream from the oldest requests that fit
      std::vector<Request> batch;
      Slot* free_slot = nullptr;
      int64_t first = -1, rows = 0;
      {
        std::unique_lock<std::mutex> g(mu);
        for (Slot& s : slots)
          if (!s.busy) {
            free_slot = &s;
            break;
          }
        if (free_slot && !pending.empty()) {
          const int64_t room = std::min(max_rows, pool.largest());
          size_t k = 0;
          while (k < pending.size() && rows + pending[k].n <= room) rows += pending[k++].n;
          if (k > 0) {
            first = pool.take(rows);
            for (size_t i = 0; i < k; ++i) {
              batch.push_back(pending.front());
              pending.pop_front();
            }
            peak_bytes = std::max(peak_bytes, pool.used() * row_bytes);
            ++busy_slots;
            ++batches;
            head_waited = false;
          } else if (!head_waited) {
            ++memory_waits;  // the head request must wait for a batch to retire
            head_waited = true;
          }
        }
        if (batch.empty() && busy_slots == 0) {
          if (stop && pending.empty()) return;
          cv_work.wait_for(g, std::chrono::milliseconds(2), [&] { return stop || !pending.empty(); });
          continue;
        }
      }
      if (!batch.empty())
        launch(*free_slot, std::move(batch), first, rows);
      else  // every stream busy or the head request does not fit yet
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(mu);
    error = e.msg;
    stop = true;
    cv_idle.notify_all();
  }
}

void aiwc_rf_server::release_resources() {
  for (Slot& s : slots) {
    if (s.stream) {
      (void)hipStreamSynchronize(s.stream);
      (void)hipStreamDestroy(s.stream);
    }
    if (s.done) (void)hipEventDestroy(s.done);
  }
  slots.clear();
  if (d_arena) (void)hipFree(d_arena);
  if (h_arena) (void)hipHostFree(h_arena);
  d_arena = h_arena = nullptr;
}

extern "C" {

int aiwc_rf_server_create(const aiwc_rf_forest* forest, int32_t forest_index, int64_t memory_budget_bytes,
                          int32_t max_batch_rows, int32_t n_streams, aiwc_rf_server** server) {
  std::unique_ptr<aiwc_rf_server> S;
  const int rc = guard([&] {
    if (!forest || !server) fail(AIWC_RF_EINVAL, "null pointer argument");
    if (forest_index < 0 || forest_index >= (int32_t)forest->params.size())
      fail(AIWC_RF_EINVAL, "forest_index out of range");
    if (max_batch_rows < 1 || n_streams < 1 || n_streams > 8)
      fail(AIWC_RF_EINVAL, "max_batch_rows must be >= 1 and n_streams in [1, 8]");
    if (aiwc_rf_forest_wait(forest) != AIWC_RF_OK) fail(AIWC_RF_ESTATE, "forest fit failed");
    S.reset(new aiwc_rf_server());
    S->forest = forest;
    S->forest_index = forest_index;
    S->n_cols = forest->n_cols;
    S->num_trees = forest->params[forest_index].num_trees;
    S->t0 = forest->first_task[forest_index];
    S->budget = memory_budget_bytes;
    S->max_rows = max_batch_rows;
    S->device = forest->device;
    const int64_t dev_row = (int64_t)S->n_cols + 16, host_row = (int64_t)S->n_cols + 8;
    S->row_bytes = dev_row + host_row;
    // each arena region starts 256-byte aligned; the slack is charged to the budget
    const int64_t slack = 3 * 256 + 2 * 256;
    S->capacity = (memory_budget_bytes - slack) / S->row_bytes;
    if (S->capacity < 1) fail(AIWC_RF_EINVAL, "memory budget too small for one row");
    const int64_t K = S->capacity;
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t d_codes = up(K * S->n_cols), d_sum = up(8 * K), d_out = up(8 * K);
    const int64_t h_codes = up(K * S->n_cols), h_out = up(8 * K);
    AIWC_HIP(hipSetDevice(S->device));
    AIWC_HIP(hipMalloc((void**)&S->d_arena, (size_t)(d_codes + d_sum + d_out)));
    AIWC_HIP(hipHostMalloc((void**)&S->h_arena, (size_t)(h_codes + h_out), hipHostMallocDefault));
    S->d_codes = S->d_arena;
    S->d_sum = reinterpret_cast<int64_t*>(S->d_arena + d_codes);
    S->d_out = reinterpret_cast<double*>(S->d_arena + d_codes + d_sum);
    S->h_codes = S->h_arena;
    S->h_out = reinterpret_cast<double*>(S->h_arena + h_codes);
    S->pool.reset(K);
    S->slots.resize((size_t)n_streams);
    for (Slot& s : S->slots) {
      AIWC_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
      AIWC_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    }
    aiwc_rf_server* raw = S.get();
    S->dispatcher = std::thread([raw] { raw->run(); });
    *server = S.release();
  });
  if (rc != AIWC_RF_OK && S) S->release_resources();
  return rc;
}

int aiwc_rf_server_submit(aiwc_rf_server* S, const uint8_t* codes_host, int64_t n, double* out_host,
                          int64_t* ticket_host) {
  return guard([&] {
    if (!S || !codes_host || !out_host || !ticket_host) fail(AIWC_RF_EINVAL, "null pointer argument");
    if (n < 1) fail(AIWC_RF_EINVAL, "n must be >= 1");
    if (n > S->max_rows) fail(AIWC_RF_ENOMEM, "request exceeds max_batch_rows");
    if (n > S->capacity) fail(AIWC_RF_ENOMEM, "request exceeds the memory budget");
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) fail(AIWC_RF_ESTATE, S->error.empty() ? "server is stopping" : "server failed: " + S->error);
    Request r{S->next_ticket++, codes_host, n, out_host, Clock::now()};
    *ticket_host = r.ticket;
    S->pending.push_back(r);
    S->cv_work.notify_one();
  });
}

int aiwc_rf_server_poll(aiwc_rf_server* S, int64_t* tickets_host, double* latency_s_host, int32_t max_tickets,
                        int32_t* n_done_host) {
  return guard([&] {
    if (!S || !n_done_host || max_tickets < 0) fail(AIWC_RF_EINVAL, "bad poll arguments");
    std::lock_guard<std::mutex> g(S->mu);
    int32_t k = 0;
    while (k < max_tickets && !S->completed.empty()) {
      if (tickets_host) tickets_host[k] = S->completed.front().first;
      if (latency_s_host) latency_s_host[k] = S->completed.front().second;
      S->completed.pop_front();
      ++k;
    }
    *n_done_host = k;
    if (!S->error.empty()) fail(AIWC_RF_EHIP, "server failed: " + S->error);
  });
}

int aiwc_rf_server_drain(aiwc_rf_server* S) {
  return guard([&] {
    if (!S) fail(AIWC_RF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> g(S->mu);
    S->cv_idle.wait(g, [&] { return !S->error.empty() || (S->pending.empty() && S->busy_slots == 0); });
    if (!S->error.empty()) fail(AIWC_RF_EHIP, "server failed: " + S->error);
  });
}

int aiwc_rf_server_stats(const aiwc_rf_server* S, int64_t* rows_host, int64_t* batches_host, int64_t* peak_bytes_host,
                         int64_t* memory_waits_host) {
  return guard([&] {
    if (!S) fail(AIWC_RF_EINVAL, "server is NULL");
    aiwc_rf_server* s = const_cast<aiwc_rf_server*>(S);
    std::lock_guard<std::mutex> g(s->mu);
    if (rows_host) *rows_host = s->rows_served;
    if (batches_host) *batches_host = s->batches;
    if (peak_bytes_host) *peak_bytes_host = s->peak_bytes;
    if (memory_waits_host) *memory_waits_host = s->memory_waits;
  });
}

void aiwc_rf_server_free(aiwc_rf_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->dispatcher.joinable()) S->dispatcher.join();
  S->release_resources();
  delete S;
}

}  // extern "C"
