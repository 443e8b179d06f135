// Served form: a request loop that runs k-bisimulation jobs of different
// sizes concurrently on one GPU.
//
// Requests enter a FIFO queue. A request is admitted when a slot is free and
// its estimated device footprint fits in what the HBM budget has left; the
// queue head waits for memory rather than being overtaken (no starvation).
// Every slot is a worker thread with its own stream, so the rounds of all
// admitted requests overlap on the device, and a request that arrives while
// others run starts as soon as a slot and memory free up. Each job keeps its
// partition state in device memory across its rounds; the ids are copied to
// host memory when it completes and its device memory is released.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "engine.h"

namespace kb {

// Small requests share launches: a worker that takes a small request from
// the queue head also takes the small requests queued right behind it (up to
// kServeGroupEdges edges and kServeGroupMax requests in all, within the
// budget) and refines them as one disjoint union (the batched form, each
// with its own k); every request's ids are those of a run on its own graph.
constexpr int64_t kServeSmallEdges = int64_t(1) << 21;
constexpr int64_t kServeGroupEdges = int64_t(1) << 24;
constexpr size_t kServeGroupMax = 256;

// Device bytes a job of n nodes and m edges may hold at its peak: inputs
// (12 m), the CSR sort's key and value buffers (16 m), the adjacency and the
// per-round keys (8 m), per-node state, the active set and the global
// ordering passes (~160 n), plus slack for the caching allocator's rounding.
inline uint64_t job_footprint(uint64_t n, uint64_t m) { return 36 * m + 160 * n + (uint64_t(64) << 20); }

struct Request {
  enum State { kQueued, kRunning, kDone, kFailed, kCancelled };
  uint64_t id = 0;
  int32_t k = 0;
  int64_t n = 0, m = 0;
  bool device_inputs = false;
  const int32_t* dev[4] = {nullptr, nullptr, nullptr, nullptr};  // caller-owned device arrays
  hipEvent_t ready = nullptr;  // device inputs: recorded on the caller's stream at submit
  std::vector<int32_t> host[4];                                   // copies of host arrays
  uint64_t footprint = 0;
  State state = kQueued;
  int status = 0;  // kbisim_status of a failed request
  std::string error;
  bool cancel = false;
  std::vector<int32_t> pid;
  std::vector<int64_t> counts;
  int32_t rounds = 0;
  std::chrono::steady_clock::time_point t_submit, t_start, t_end;
};

class Server {
 public:
  Server(uint64_t budget, int32_t slots, const Options& o);
  ~Server();
  // Returns the request id; throws InvalidInput / OutOfMemory (never fits).
  // Device inputs are read after the work enqueued on `caller` before the
  // call (an event recorded there at submit, waited for by the worker).
  uint64_t submit(const int32_t* label, const int32_t* src, const int32_t* lab, const int32_t* dst, int64_t n,
                  int64_t m, bool device_inputs, int32_t k, hipStream_t caller);
  // Waits up to timeout_s (< 0: forever). Returns 0 when done and fills the
  // outputs; otherwise a negative status (failed/cancelled/timed out).
  int wait(uint64_t id, int32_t* pid_out, bool to_device, int64_t* num_blocks, int32_t* rounds,
           double timeout_s, std::string* err);
  int cancel(uint64_t id);
  // Seconds from submit to start and to completion (done requests).
  bool timing(uint64_t id, double* queued_s, double* total_s);
  void release(uint64_t id);  // forget a finished request
  int state(uint64_t id, int32_t* st);  // KBISIM_EINVAL for an unknown id
  uint64_t in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return in_use_;
  }

 private:
  void worker(int slot);
  void run(Request& r, hipStream_t s);
  // several small requests as one union; false when the union was rejected
  // as invalid input (the requests are then run one by one)
  bool run_group(std::vector<std::shared_ptr<Request>>& group, hipStream_t s);
  void finish(Request& r, int status, const std::string& err, bool cancelled);

  uint64_t budget_;
  int32_t slots_;
  Options opt_;
  int device_ = 0;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::map<uint64_t, std::shared_ptr<Request>> all_;
  uint64_t next_id_ = 1;
  uint64_t in_use_ = 0;
  bool stop_ = false;
  std::vector<std::thread> threads_;
  std::vector<hipStream_t> streams_;
};

}  // namespace kb
