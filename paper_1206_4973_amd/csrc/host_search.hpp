// host_search.hpp -- CPU threads of the hybrid search (host_search.hip).
#pragma once
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include "fsp_internal.hpp"

namespace fspi {

// The two-machine bound on the host (same definition as the device kernels).
struct HostBound {
  struct Step {
    int32_t job, a, lag, b;
  };
  int n = 0, m = 0, P = 0;
  std::vector<int32_t> p, H, Q;  // [n][m]
  std::vector<int> pk, pl;       // machines of pair pi
  std::vector<Step> steps;       // [P][n]: pair pi's jobs in Johnson order
  void init(const std::vector<int32_t> &p, int n, int m);
  int32_t bound(const uint8_t *prefix, int d) const;
};

// Worker threads exploring the subtrees of the nodes they are given.
struct HostSearch {
  struct Node {
    int d = 0;
    int32_t lb = 0;
    uint8_t prefix[256];
  };
  struct Counters {
    int64_t bounded = 0, branched = 0, pruned = 0, leaves = 0;
  };
  HostBound hb;
  int n = 0, rule = 0;
  std::chrono::steady_clock::time_point t0;
  std::atomic<int32_t> ub_host{INT32_MAX};  // best makespan known to the host
  std::atomic<int32_t> left_lb{INT32_MAX};  // smallest bound left unexplored at a stop
  std::atomic<bool> quit{false};
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::vector<Node> queue;
  int busy = 0;
  std::vector<std::thread> workers;
  Counters total;  // summed when the threads stop
  std::mutex best_mu;
  int32_t best = INT32_MAX;  // best schedule found by the host
  uint8_t best_perm[256];
  double t_found = 0.0;

  ~HostSearch();
  void start(const fsp_instance *inst, int threads, int rule, int32_t ub,
             std::chrono::steady_clock::time_point t0);
  // Hands over `count` pending node records (stride bytes each) and bounds.
  void give(const uint8_t *recs, const int32_t *lbs, int count, int stride);
  bool idle();
  void wait_idle();
  void stop_threads();
  int32_t open_lb();
  void propose(int32_t makespan, const uint8_t *perm);
  void explore(const Node &root, Counters &c);
  void worker();
};

}  // namespace fspi
