// Prediction server: a resident forest answering a stream of requests of
// different sizes (the scheduler-facing query of Sec. I and Sec. VI).
//
// One dispatcher thread owns a ring of n_streams slots, each with its own HIP
// stream, pinned host staging and device buffers sized for max_batch_rows.
// Requests wait in FIFO order until a slot is free; a batch is then packed from
// the oldest waiting requests for as long as they fit both the slot's row
// capacity and the memory budget (rows * (n_cols + 8) bytes of every request
// in flight).  Copies in, traversal and copies out of one batch are enqueued
// on its slot's stream, so batches on different slots overlap on the device
// while new requests keep arriving; finished batches are scattered back to the
// callers' output arrays.  Each row is traversed exactly as by aiwc_rf_predict,
// so an answer never depends on what it was batched with.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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
  int64_t bytes;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* h_codes = nullptr;
  double* h_out = nullptr;
  uint8_t* d_codes = nullptr;
  double* d_out = nullptr;
  int64_t* d_sum = nullptr;
  std::vector<Request> reqs;
  int64_t rows = 0;
  bool busy = false;
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
  int device = 0;

  std::mutex mu;
  std::condition_variable cv_work;  // dispatcher waits for requests
  std::condition_variable cv_idle;  // drain waits for completion
  std::deque<Request> pending;
  std::deque<std::pair<int64_t, double>> completed;
  std::vector<Slot> slots;
  int64_t in_flight_bytes = 0;
  int64_t next_ticket = 0;
  int64_t rows_served = 0;
  int64_t batches = 0;
  int64_t peak_bytes = 0;
  int busy_slots = 0;
  bool stop = false;
  std::string error;
  std::thread dispatcher;

  void run();
  void launch(Slot& s, std::vector<Request>&& batch);
  void retire(Slot& s);
};

void aiwc_rf_server::launch(Slot& s, std::vector<Request>&& batch) {
  int64_t off = 0;
  for (const Request& r : batch) {
    std::memcpy(s.h_codes + off * n_cols, r.codes, (size_t)(r.n * n_cols));
    off += r.n;
  }
  s.rows = off;
  s.reqs = std::move(batch);
  AIWC_HIP(hipMemcpyAsync(s.d_codes, s.h_codes, (size_t)(off * n_cols), hipMemcpyHostToDevice, s.stream));
  launch_predict(forest->nodes.p, forest->node_base.p, (int32_t)t0, (int32_t)(t0 + num_trees), s.d_codes, off, n_cols,
                 s.d_sum, s.d_out, num_trees, s.stream);
  AIWC_HIP(hipMemcpyAsync(s.h_out, s.d_out, sizeof(double) * off, hipMemcpyDeviceToHost, s.stream));
  AIWC_HIP(hipEventRecord(s.done, s.stream));
  s.busy = true;
}

void aiwc_rf_server::retire(Slot& s) {
  int64_t off = 0;
  const Clock::time_point now = Clock::now();
  std::vector<std::pair<int64_t, double>> done;
  for (const Request& r : s.reqs) {
    std::memcpy(r.out, s.h_out + off, sizeof(double) * (size_t)r.n);
    off += r.n;
    done.emplace_back(r.ticket, std::chrono::duration<double>(now - r.submitted).count());
  }
  std::lock_guard<std::mutex> g(mu);
  for (const Request& r : s.reqs) in_flight_bytes -= r.bytes;
  rows_served += s.rows;
  for (auto& d : done) completed.push_back(d);
  s.reqs.clear();
  s.busy = false;
  --busy_slots;
  cv_idle.notify_all();
}

void aiwc_rf_server::run() {
  (void)hipSetDevice(device);
  try {
    for (;;) {
      // retire finished batches
      for (Slot& s : slots)
        if (s.busy && hipEventQuery(s.done) == hipSuccess) retire(s);
      // pack a batch for a free slot
      std::vector<Request> batch;
      Slot* free_slot = nullptr;
      bool idle;
      {
        std::unique_lock<std::mutex> g(mu);
        for (Slot& s : slots)
          if (!s.busy) {
            free_slot = &s;
            break;
          }
        if (free_slot) {
          int64_t rows = 0;
          while (!pending.empty()) {
            const Request& r = pending.front();
            if (rows + r.n > max_rows || in_flight_bytes + r.bytes > budget) break;
            rows += r.n;
            in_flight_bytes += r.bytes;
            batch.push_back(r);
            pending.pop_front();
          }
          peak_bytes = std::max(peak_bytes, in_flight_bytes);
          if (!batch.empty()) {
            ++busy_slots;
            ++batches;
          }
        }
        idle = batch.empty() && busy_slots == 0;
        if (idle) {
          if (stop && pending.empty()) return;
          cv_work.wait_for(g, std::chrono::milliseconds(2),
                           [&] { return stop || !pending.empty(); });
          continue;
        }
      }
      if (!batch.empty()) {
        launch(*free_slot, std::move(batch));
      } else {
        // every slot busy or the head request does not fit yet: wait a little
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(mu);
    error = e.msg;
    stop = true;
    cv_idle.notify_all();
  }
}

extern "C" {

int aiwc_rf_server_create(const aiwc_rf_forest* forest, int32_t forest_index, int64_t memory_budget_bytes,
                          int32_t max_batch_rows, int32_t n_streams, aiwc_rf_server** server) {
  std::unique_ptr<aiwc_rf_server> S;
  try {
    if (!forest || !server || forest_index < 0 || forest_index >= (int32_t)forest->params.size() ||
        memory_budget_bytes <= 0 || max_batch_rows < 1 || n_streams < 1 || n_streams > 8)
      fail(AIWC_RF_EINVAL, "bad server arguments");
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
    AIWC_HIP(hipSetDevice(S->device));
    S->slots.resize((size_t)n_streams);
    for (Slot& s : S->slots) {
      AIWC_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
      AIWC_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
      AIWC_HIP(hipHostMalloc((void**)&s.h_codes, (size_t)max_batch_rows * S->n_cols, hipHostMallocDefault));
      AIWC_HIP(hipHostMalloc((void**)&s.h_out, sizeof(double) * (size_t)max_batch_rows, hipHostMallocDefault));
      AIWC_HIP(hipMalloc((void**)&s.d_codes, (size_t)max_batch_rows * S->n_cols));
      AIWC_HIP(hipMalloc((void**)&s.d_out, sizeof(double) * (size_t)max_batch_rows));
      AIWC_HIP(hipMalloc((void**)&s.d_sum, sizeof(int64_t) * (size_t)max_batch_rows));
    }
    aiwc_rf_server* raw = S.get();
    S->dispatcher = std::thread([raw] { raw->run(); });
    *server = S.release();
    return AIWC_RF_OK;
  } catch (const Error& e) {
    if (S) {
      for (Slot& s : S->slots) {
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.h_codes) (void)hipHostFree(s.h_codes);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.d_codes) (void)hipFree(s.d_codes);
        if (s.d_out) (void)hipFree(s.d_out);
        if (s.d_sum) (void)hipFree(s.d_sum);
      }
    }
    return e.code;
  }
}

int aiwc_rf_server_submit(aiwc_rf_server* S, const uint8_t* codes_host, int64_t n, double* out_host,
                          int64_t* ticket_host) {
  if (!S || !codes_host || !out_host || !ticket_host || n < 1) return AIWC_RF_EINVAL;
  const int64_t bytes = n * ((int64_t)S->n_cols + 8);
  if (n > S->max_rows || bytes > S->budget) return AIWC_RF_ENOMEM;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return AIWC_RF_ESTATE;
  Request r{S->next_ticket++, codes_host, n, out_host, Clock::now(), bytes};
  *ticket_host = r.ticket;
  S->pending.push_back(r);
  S->cv_work.notify_one();
  return AIWC_RF_OK;
}

int aiwc_rf_server_poll(aiwc_rf_server* S, int64_t* tickets_host, double* latency_s_host, int32_t max_tickets,
                        int32_t* n_done_host) {
  if (!S || !n_done_host || max_tickets < 0) return AIWC_RF_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  int32_t k = 0;
  while (k < max_tickets && !S->completed.empty()) {
    if (tickets_host) tickets_host[k] = S->completed.front().first;
    if (latency_s_host) latency_s_host[k] = S->completed.front().second;
    S->completed.pop_front();
    ++k;
  }
  *n_done_host = k;
  return S->error.empty() ? AIWC_RF_OK : AIWC_RF_EHIP;
}

int aiwc_rf_server_drain(aiwc_rf_server* S) {
  if (!S) return AIWC_RF_EINVAL;
  std::unique_lock<std::mutex> g(S->mu);
  S->cv_idle.wait(g, [&] { return !S->error.empty() || (S->pending.empty() && S->busy_slots == 0); });
  return S->error.empty() ? AIWC_RF_OK : AIWC_RF_EHIP;
}

int aiwc_rf_server_stats(const aiwc_rf_server* S, int64_t* rows_host, int64_t* batches_host, int64_t* peak_bytes_host) {
  if (!S) return AIWC_RF_EINVAL;
  aiwc_rf_server* s = const_cast<aiwc_rf_server*>(S);
  std::lock_guard<std::mutex> g(s->mu);
  if (rows_host) *rows_host = s->rows_served;
  if (batches_host) *batches_host = s->batches;
  if (peak_bytes_host) *peak_bytes_host = s->peak_bytes;
  return AIWC_RF_OK;
}

void aiwc_rf_server_free(aiwc_rf_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->dispatcher.joinable()) S->dispatcher.join();
  for (Slot& s : S->slots) {
    (void)hipStreamSynchronize(s.stream);
    (void)hipStreamDestroy(s.stream);
    (void)hipEventDestroy(s.done);
    (void)hipHostFree(s.h_codes);
    (void)hipHostFree(s.h_out);
    (void)hipFree(s.d_codes);
    (void)hipFree(s.d_out);
    (void)hipFree(s.d_sum);
  }
  delete S;
}

}  // extern "C"
