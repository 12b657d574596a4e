// server.hip -- continuous-batching GEMM serving loop (native).
//
// Requests (one C <- alpha*A*B + beta*C each, operands on the host) enter a
// FIFO.  A scheduler thread admits the head of the queue whenever a slot and
// room in the caller's HBM arena are free (first-fit allocator), copies the
// operands into the arena, and groups everything admitted since the last
// launch into one step: one grouped persistent launch on the next idle stream.
// Steps on different streams overlap on the device, so requests that arrive
// while others run are admitted and computed without waiting for them -- the
// concurrency of independent connected components on separate streams that
// the paper describes for GPUs (Sec. 3.3, "Concurrency").  Each request's tile
// shape depends only on its (M, N), so its result is bitwise the same alone
// and in any mix.
//
// Latency of a request = time from its arrival stamp to the host observing
// the completion event of its step's kernel; the time until its result is in
// host memory is recorded beside it.
//
// Failures: every HIP call of a step is checked.  A step whose copies or
// launches cannot be enqueued fails its own requests (server_poll returns
// GEMM_STATUS_HIP_ERROR for them) after the stream has drained what was
// enqueued, so their arena ranges are never reused under an in-flight copy.
// An error reported asynchronously by a completion event also fails the
// step's requests and marks the server failed: later submits return the
// error.  Queued requests can be cancelled, and a queue timeout drops
// requests that waited longer than it without being admitted.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "grouped.hpp"
#include "kernels.hpp"

namespace mm {

// First-fit allocator over [0, size) with 256-byte granularity.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t &off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        high_ = std::max(high_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t size() const { return size_; }
  size_t high_water() const { return high_; }

 private:
  size_t size_, used_ = 0, high_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket;
  int64_t M, N, K;
  float alpha, beta;
  const float *hA, *hB, *hC0;
  float *hC;
  double t_arrival = 0, t_admit = 0, t_done = 0, t_result = 0;
  size_t off = 0, bytes = 0;
  // 0 queued, 1 admitted, 2 computed, 3 result in host memory,
  // 4 ended without a result (status and message below)
  int state = 0;
  gemm_status status = GEMM_STATUS_OK;
  std::string error;
};

struct Step {
  std::vector<uint64_t> tickets;
  bool computed = false;
};

struct StreamCtx {
  hipStream_t stream = nullptr;
  void *ws = nullptr;      // grouped workspace for this stream (inside the arena)
  void *pinned = nullptr;  // pinned staging of the descriptor table
  hipEvent_t kernel_done = nullptr, result_done = nullptr;  // reused by every step
  Step *busy = nullptr;
};

}  // namespace mm

struct gemm_server {
  int device = 0;
  int max_slots = 0;
  int path = GEMM_PATH_3XBF16;
  uint8_t *arena_base = nullptr;
  mm::Arena *arena = nullptr;
  std::vector<mm::StreamCtx> streams;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;                           // FIFO of queued tickets
  std::unordered_map<uint64_t, mm::Request> reqs;
  std::vector<uint64_t> pending_step;                   // admitted, not yet launched
  int in_flight = 0, max_in_flight = 0;
  int steps_busy = 0, max_steps_busy = 0;               // steps on the device at once
  uint64_t next_ticket = 1, completed = 0, rejected = 0, failed = 0;
  double queue_timeout_s = 0;                           // 0: queued requests wait forever
  int inject_step_failures = 0;                         // host-forced failures (tests)
  double flops_done = 0, first_arrival = -1, last_done = 0;
  std::vector<double> lat_ms, lat_result_ms;
  std::atomic<bool> stop{false};
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  std::string worker_error;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace mm {

static size_t request_bytes(int64_t M, int64_t N, int64_t K) {
  auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return r(4 * (size_t)(M * K)) + r(4 * (size_t)(K * N)) + r(4 * (size_t)(M * N));
}

// A request ends without a result: record why, give back its slot and arena
// range.  The caller guarantees nothing enqueued for it is still in flight.
static void end_request(gemm_server *s, Request &r, gemm_status status, const std::string &why) {
  const bool admitted = r.state >= 1 && r.state <= 2;
  r.state = 4;
  r.status = status;
  r.error = why;
  if (admitted) {
    s->arena->release(r.off, r.bytes);
    s->in_flight--;
  }
  if (status == GEMM_STATUS_HIP_ERROR) s->failed++;
}

static void fail_step(gemm_server *s, Step *st, const std::string &why) {
  for (uint64_t t : st->tickets) end_request(s, s->reqs[t], GEMM_STATUS_HIP_ERROR, why);
  delete st;
  s->cv.notify_all();
}

// Launch everything admitted since the last step on an idle stream.  Called
// with the lock held; every HIP call here is asynchronous (pinned staging for
// the descriptor table; operand copies are asynchronous when the caller's host
// buffers are pinned) and checked.  On a failure nothing more is enqueued,
// the stream is drained (so no copy still targets the step's arena ranges)
// and the step's requests end with GEMM_STATUS_HIP_ERROR.
static void launch_step(gemm_server *s, StreamCtx &sc) {
  Step *st = new Step();
  st->tickets.swap(s->pending_step);
  std::vector<gemm_problem> probs;
  probs.reserve(st->tickets.size());
  gemm_status status = GEMM_STATUS_OK;
  std::string why;
  auto hip = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && !status) {
      status = hip_fail(what, e);
      why = gemm_last_error();
    }
  };
  if (s->inject_step_failures > 0) {
    s->inject_step_failures--;
    status = GEMM_STATUS_HIP_ERROR;
    why = "server: injected step failure";
  }
  for (uint64_t t : st->tickets) {
    Request &r = s->reqs[t];
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    float *dA = reinterpret_cast<float *>(s->arena_base + r.off);
    float *dB = reinterpret_cast<float *>(s->arena_base + r.off + r256(4 * (size_t)(r.M * r.K)));
    float *dC = reinterpret_cast<float *>(s->arena_base + r.off + r256(4 * (size_t)(r.M * r.K)) +
                                          r256(4 * (size_t)(r.K * r.N)));
    if (!status && r.M * r.K)
      hip(hipMemcpyAsync(dA, r.hA, 4 * (size_t)(r.M * r.K), hipMemcpyHostToDevice, sc.stream),
          "server: copy of A");
    if (!status && r.K * r.N)
      hip(hipMemcpyAsync(dB, r.hB, 4 * (size_t)(r.K * r.N), hipMemcpyHostToDevice, sc.stream),
          "server: copy of B");
    if (!status && r.beta != 0.0f && r.M * r.N)
      hip(hipMemcpyAsync(dC, r.hC0, 4 * (size_t)(r.M * r.N), hipMemcpyHostToDevice, sc.stream),
          "server: copy of C");
    gemm_problem q;
    q.M = r.M; q.N = r.N; q.K = r.K;
    q.lda = std::max<int64_t>(1, r.K); q.ldb = std::max<int64_t>(1, r.N); q.ldc = std::max<int64_t>(1, r.N);
    q.A = dA; q.B = dB; q.C = dC; q.alpha = r.alpha; q.beta = r.beta;
    probs.push_back(q);
  }
  std::vector<Desc> descs;
  std::vector<int> starts;
  int total = 0;
  auto lib = [&](gemm_status e) {
    if (e && !status) {
      status = e;
      why = gemm_last_error();
    }
  };
  if (!status) lib(grouped_build(probs.data(), (int)probs.size(), nullptr, descs, starts, total));
  for (size_t i = 0; !status && i < probs.size(); ++i) {
    const gemm_problem &q = probs[i];
    if (q.M > 0 && q.N > 0 && (q.K == 0 || q.alpha == 0.0f))
      lib(scale_c(q.M, q.N, q.beta, q.C, q.ldc, sc.stream));
  }
  if (!status) lib(grouped_upload_pinned(sc.ws, sc.pinned, descs, starts, sc.stream));
  if (!status) lib(grouped_enqueue(sc.ws, (int)probs.size(), total, grouped_grid(total), sc.stream));
  if (!status) hip(hipEventRecord(sc.kernel_done, sc.stream), "server: record kernel event");
  for (size_t i = 0; !status && i < st->tickets.size(); ++i) {
    Request &r = s->reqs[st->tickets[i]];
    if (r.hC && r.M * r.N)
      hip(hipMemcpyAsync(r.hC, probs[i].C, 4 * (size_t)(r.M * r.N), hipMemcpyDeviceToHost,
                         sc.stream),
          "server: copy of the result");
  }
  if (!status) hip(hipEventRecord(sc.result_done, sc.stream), "server: record result event");
  if (status) {
    (void)hipStreamSynchronize(sc.stream);  // the step fails whatever this returns
    fail_step(s, st, why);
    return;
  }
  sc.busy = st;
  s->steps_busy++;
  s->max_steps_busy = std::max(s->max_steps_busy, s->steps_busy);
}

// Polls a completion event: 1 done, 0 not yet, -1 failed (why is set).
static int event_done(hipEvent_t ev, const char *what, std::string &why) {
  const hipError_t e = hipEventQuery(ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  hip_fail(what, e);
  why = gemm_last_error();
  return -1;
}

static void worker_loop(gemm_server *s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool progressed = false;
    // 1. completions
    for (StreamCtx &sc : s->streams) {
      Step *st = sc.busy;
      if (!st) continue;
      std::string why;
      int k = st->computed ? 1 : event_done(sc.kernel_done, "server: kernel event", why);
      if (k == 1 && !st->computed) {
        const double t = s->now();
        for (uint64_t tk : st->tickets) {
          Request &r = s->reqs[tk];
          r.t_done = t;
          r.state = 2;
        }
        st->computed = true;
        progressed = true;
      }
      if (k == 1) k = event_done(sc.result_done, "server: result event", why);
      if (k == 1) {
        const double t = s->now();
        for (uint64_t tk : st->tickets) {
          Request &r = s->reqs[tk];
          r.t_result = t;
          r.state = 3;
          s->arena->release(r.off, r.bytes);
          s->lat_ms.push_back(1e3 * (r.t_done - r.t_arrival));
          s->lat_result_ms.push_back(1e3 * (r.t_result - r.t_arrival));
          s->flops_done += 2.0 * (double)r.M * (double)r.N * (double)r.K;
          s->last_done = std::max(s->last_done, r.t_done);
          s->completed++;
          s->in_flight--;
        }
        delete st;
      } else if (k < 0) {
        // an asynchronous device error: the step's work may have stopped at
        // any point; drain the stream before its ranges are given back
        (void)hipStreamSynchronize(sc.stream);
        s->worker_error = why;
        fail_step(s, st, why);
      }
      if (k != 0) {
        sc.busy = nullptr;
        s->steps_busy--;
        progressed = true;
        s->cv.notify_all();
      }
    }
    // 2. queue timeout: requests that waited too long are dropped unadmitted
    if (s->queue_timeout_s > 0 && !s->queue.empty()) {
      const double t = s->now();
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request &r = s->reqs[*it];
        if (t - r.t_arrival > s->queue_timeout_s) {
          end_request(s, r, GEMM_STATUS_TIMED_OUT, "server: request timed out in the queue");
          it = s->queue.erase(it);
          progressed = true;
        } else {
          ++it;
        }
      }
      if (progressed) s->cv.notify_all();
    }
    // 3. FIFO admission: the head waits until it fits (no overtaking)
    while (!s->queue.empty() && s->in_flight < s->max_slots) {
      Request &r = s->reqs[s->queue.front()];
      size_t off = 0;
      if (!s->arena->alloc(r.bytes, off)) break;
      r.off = off;
      r.state = 1;
      r.t_admit = s->now();
      s->pending_step.push_back(r.ticket);
      s->queue.pop_front();
      s->in_flight++;
      s->max_in_flight = std::max(s->max_in_flight, s->in_flight);
      progressed = true;
    }
    // 4. launch the admitted requests as one step on an idle stream
    if (!s->pending_step.empty()) {
      for (StreamCtx &sc : s->streams) {
        if (!sc.busy) {
          launch_step(s, sc);
          progressed = true;
          break;
        }
      }
    }
    if (!progressed) {
      const bool busy = s->in_flight > 0;
      s->cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 500));
    }
  }
}

}  // namespace mm

using namespace mm;

extern "C" {

gemm_status server_create(void *arena, size_t arena_bytes, int max_slots, int path, int n_streams,
                          gemm_server **out) {
  clear_error();
  const char *fn = "server_create";
  if (!arena) return bad_arg(1, fn, "(arena) is NULL");
  if (((uintptr_t)arena & 255) != 0) return bad_arg(1, fn, "(arena) must be 256-byte aligned");
  if (max_slots < 1 || max_slots > 4096) return bad_arg(3, fn, "(max_slots) must be in [1, 4096]");
  if (path != GEMM_PATH_3XBF16) return bad_arg(4, fn, "(path) must be GEMM_PATH_3XBF16");
  if (n_streams < 1 || n_streams > 16) return bad_arg(5, fn, "(n_streams) must be in [1, 16]");
  if (!out) return bad_arg(6, fn, "(out) is NULL");
  const size_t ws_each = (grouped_ws_bytes(max_slots) + 255) & ~(size_t)255;
  if (arena_bytes <= ws_each * (size_t)n_streams + 4096)
    return bad_arg(2, fn, "(arena_bytes) too small for the per-stream workspaces");
  auto *s = new gemm_server();
  hipGetDevice(&s->device);
  s->max_slots = max_slots;
  s->path = path;
  s->t0 = std::chrono::steady_clock::now();
  uint8_t *base = static_cast<uint8_t *>(arena);
  s->streams.resize(n_streams);
  auto release_streams = [s]() {
    for (StreamCtx &sc : s->streams) {
      if (sc.kernel_done) hipEventDestroy(sc.kernel_done);
      if (sc.result_done) hipEventDestroy(sc.result_done);
      if (sc.pinned) hipHostFree(sc.pinned);
      if (sc.stream) hipStreamDestroy(sc.stream);
    }
  };
  for (int i = 0; i < n_streams; ++i) {
    StreamCtx &sc = s->streams[i];
    sc.ws = base + (size_t)i * ws_each;
    hipError_t e = hipStreamCreateWithFlags(&sc.stream, hipStreamNonBlocking);
    const char *what = "server_create: stream";
    if (e == hipSuccess) {
      e = hipHostMalloc(&sc.pinned, ws_each, hipHostMallocDefault);
      what = "server_create: pinned staging";
    }
    if (e == hipSuccess) {
      e = hipEventCreateWithFlags(&sc.kernel_done, hipEventDisableTiming);
      what = "server_create: event";
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sc.result_done, hipEventDisableTiming);
    if (e != hipSuccess) {
      release_streams();
      delete s;
      return hip_fail(what, e);
    }
  }
  // Host-forced failures for tests of the error path: the first n steps fail
  // before anything is enqueued, as if a copy could not be issued.
  if (const char *inj = getenv("GEMM_SERVER_INJECT_STEP_FAILURES"))
    s->inject_step_failures = std::max(0, atoi(inj));
  s->arena_base = base + ws_each * (size_t)n_streams;
  s->arena = new Arena(arena_bytes - ws_each * (size_t)n_streams);
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return GEMM_STATUS_OK;
}

double server_now(gemm_server *s) { return s ? s->now() : 0.0; }

gemm_status server_submit(gemm_server *s, int64_t M, int64_t N, int64_t K, float alpha,
                          const float *hA, const float *hB, float beta, const float *hC0,
                          float *hC_out, double arrival, uint64_t *ticket) {
  clear_error();
  const char *fn = "server_submit";
  if (!s) return bad_arg(1, fn, "(server) is NULL");
  if (M < 0) return bad_arg(2, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(3, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(4, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL) return bad_arg(2, fn, "size exceeds 2^31-1");
  // The grouped tile body addresses a 128-row panel of A (row stride K) and a
  // 32-row slab of B (row stride N) with 32-bit byte offsets.
  const bool fits32 = (128 * std::max<int64_t>(1, K) + K) * 4 < ((int64_t)1 << 31) &&
                      (32 * std::max<int64_t>(1, N) + N) * 4 < ((int64_t)1 << 31);
  if (M * K > 0 && !hA) return bad_arg(6, fn, "(hA) is NULL");
  if (K * N > 0 && !hB) return bad_arg(7, fn, "(hB) is NULL");
  if (beta != 0.0f && M * N > 0 && !hC0) return bad_arg(9, fn, "(hC0) is NULL");
  if (!ticket) return bad_arg(12, fn, "(ticket) is NULL");
  Request r;
  r.M = M; r.N = N; r.K = K; r.alpha = alpha; r.beta = beta;
  r.hA = hA; r.hB = hB; r.hC0 = hC0; r.hC = hC_out;
  r.bytes = request_bytes(M, N, K);
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->worker_error.empty()) {
    set_error("server: " + s->worker_error);
    return GEMM_STATUS_HIP_ERROR;
  }
  if (!fits32) {
    s->rejected++;
    set_error("server_submit: K or N too large for the 32-bit tile offsets of the grouped kernel");
    return GEMM_STATUS_UNSUPPORTED;
  }
  if (r.bytes > s->arena->size()) {
    s->rejected++;
    set_error("server_submit: request needs more memory than the whole arena");
    return GEMM_STATUS_REJECTED;
  }
  r.ticket = s->next_ticket++;
  r.t_arrival = arrival >= 0 ? arrival : s->now();
  if (s->first_arrival < 0 || r.t_arrival < s->first_arrival) s->first_arrival = r.t_arrival;
  *ticket = r.ticket;
  s->reqs.emplace(r.ticket, r);
  s->queue.push_back(r.ticket);
  s->cv.notify_all();
  return GEMM_STATUS_OK;
}

gemm_status server_poll(gemm_server *s, uint64_t ticket, double *latency_ms,
                        double *result_latency_ms) {
  clear_error();
  if (!s) return bad_arg(1, "server_poll", "(server) is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    set_error("server_poll: unknown ticket");
    return GEMM_STATUS_UNKNOWN;
  }
  if (it->second.state == 4) {
    const gemm_status st = it->second.status;
    set_error(it->second.error);
    s->reqs.erase(it);
    return st;
  }
  if (it->second.state < 3) return GEMM_STATUS_NOT_READY;
  if (latency_ms) *latency_ms = 1e3 * (it->second.t_done - it->second.t_arrival);
  if (result_latency_ms) *result_latency_ms = 1e3 * (it->second.t_result - it->second.t_arrival);
  s->reqs.erase(it);
  return GEMM_STATUS_OK;
}

gemm_status server_cancel(gemm_server *s, uint64_t ticket) {
  clear_error();
  if (!s) return bad_arg(1, "server_cancel", "(server) is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    set_error("server_cancel: unknown ticket");
    return GEMM_STATUS_UNKNOWN;
  }
  Request &r = it->second;
  if (r.state != 0) {
    set_error("server_cancel: request already admitted (it completes normally) or ended");
    return GEMM_STATUS_NOT_READY;
  }
  auto q = std::find(s->queue.begin(), s->queue.end(), ticket);
  if (q != s->queue.end()) s->queue.erase(q);
  end_request(s, r, GEMM_STATUS_CANCELLED, "server: request cancelled");
  s->cv.notify_all();
  return GEMM_STATUS_OK;
}

gemm_status server_set_queue_timeout(gemm_server *s, double seconds) {
  clear_error();
  if (!s) return bad_arg(1, "server_set_queue_timeout", "(server) is NULL");
  if (!(seconds >= 0)) return bad_arg(2, "server_set_queue_timeout", "(seconds) must be >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  s->queue_timeout_s = seconds;
  s->cv.notify_all();
  return GEMM_STATUS_OK;
}

gemm_status server_drain(gemm_server *s, double timeout_s) {
  clear_error();
  if (!s) return bad_arg(1, "server_drain", "(server) is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double>(timeout_s));
  while (!(s->queue.empty() && s->in_flight == 0)) {
    if (!s->worker_error.empty()) {
      set_error("server: " + s->worker_error);
      return GEMM_STATUS_HIP_ERROR;
    }
    if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
        !(s->queue.empty() && s->in_flight == 0)) {
      set_error("server_drain: timed out");
      return GEMM_STATUS_NOT_READY;
    }
  }
  return GEMM_STATUS_OK;
}

static double pct(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

gemm_status server_stats(gemm_server *s, double *p50_ms, double *p99_ms, double *tflops,
                         uint64_t *completed, double *result_p50_ms, double *result_p99_ms,
                         int *max_in_flight, size_t *arena_high_water, uint64_t *rejected,
                         uint64_t *failed, int *max_concurrent_steps) {
  clear_error();
  if (!s) return bad_arg(1, "server_stats", "(server) is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (p50_ms) *p50_ms = pct(s->lat_ms, 0.50);
  if (p99_ms) *p99_ms = pct(s->lat_ms, 0.99);
  if (result_p50_ms) *result_p50_ms = pct(s->lat_result_ms, 0.50);
  if (result_p99_ms) *result_p99_ms = pct(s->lat_result_ms, 0.99);
  if (tflops) {
    const double span = s->last_done - s->first_arrival;
    *tflops = span > 0 ? s->flops_done / span / 1e12 : 0.0;
  }
  if (completed) *completed = s->completed;
  if (max_in_flight) *max_in_flight = s->max_in_flight;
  if (arena_high_water) *arena_high_water = s->arena->high_water();
  if (rejected) *rejected = s->rejected;
  if (failed) *failed = s->failed;
  if (max_concurrent_steps) *max_concurrent_steps = s->max_steps_busy;
  return GEMM_STATUS_OK;
}

gemm_status server_destroy(gemm_server *s) {
  clear_error();
  if (!s) return GEMM_STATUS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop.store(true);
    s->cv.notify_all();
  }
  s->worker.join();
  for (StreamCtx &sc : s->streams) {
    hipStreamSynchronize(sc.stream);
    delete sc.busy;
    hipEventDestroy(sc.kernel_done);
    hipEventDestroy(sc.result_done);
    hipStreamDestroy(sc.stream);
    hipHostFree(sc.pinned);
  }
  delete s->arena;
  delete s;
  return GEMM_STATUS_OK;
}

}  // extern "C"
