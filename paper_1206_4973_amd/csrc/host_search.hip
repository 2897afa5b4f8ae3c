// host_search.hip -- the host half of the hybrid search: CPU threads that
// explore subtrees beside the device (the paper's future work, Sec. VI:
// host cores exploring the tree concurrently with the GPU's pool bounding).
//
// Host-only code.  The threads take pending nodes that the device search hands
// over (nodes near the leaves, taken from the deepest bucket between two
// batches of device iterations) and search each one's subtree depth-first,
// bounding every child with the same two-machine bound as the device: per
// machine pair, the jobs in the pair's Johnson order (one order per pair for
// the whole instance; restricting it to the unscheduled jobs keeps it a
// Johnson order), the scheduled jobs skipped; heads from the prefix's front,
// tails over the unscheduled jobs; the bound is the maximum over pairs, the
// makespan for a complete schedule.  UB is shared between the threads (an
// atomic) and exchanged with the device at every batch boundary.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "host_search.hpp"

namespace fspi {

void HostBound::init(const std::vector<int32_t> &p_in, int n_, int m_) {
  n = n_;
  m = m_;
  P = m * (m - 1) / 2;
  p = p_in;
  H.assign((size_t)n * m, 0);
  Q.assign((size_t)n * m, 0);
  for (int j = 0; j < n; ++j) {
    int32_t before = 0, row = 0;
    for (int k = 0; k < m; ++k) row += p[(size_t)j * m + k];
    for (int k = 0; k < m; ++k) {
      H[(size_t)j * m + k] = before;
      before += p[(size_t)j * m + k];
      Q[(size_t)j * m + k] = row - before;
    }
  }
  pk.resize(P);
  pl.resize(P);
  steps.resize((size_t)P * n);
  int pi = 0;
  for (int k = 0; k < m; ++k)
    for (int l = k + 1; l < m; ++l, ++pi) {
      pk[pi] = k;
      pl[pi] = l;
      // Johnson's rule on lag-shifted times: A = a + lag, B = b + lag; jobs
      // with A < B first by A ascending, then the rest by B descending;
      // equal keys by job id (the bound does not depend on the tie order)
      std::vector<int> ord(n);
      std::vector<int32_t> A(n), B(n), lag(n);
      for (int j = 0; j < n; ++j) {
        int32_t lg = 0;
        for (int h = k + 1; h < l; ++h) lg += p[(size_t)j * m + h];
        lag[j] = lg;
        A[j] = p[(size_t)j * m + k] + lg;
        B[j] = p[(size_t)j * m + l] + lg;
        ord[j] = j;
      }
      std::sort(ord.begin(), ord.end(), [&](int x, int y) {
        const bool fx = A[x] < B[x], fy = A[y] < B[y];
        if (fx != fy) return fx;
        if (fx) return A[x] != A[y] ? A[x] < A[y] : x < y;
        return B[x] != B[y] ? B[x] > B[y] : x < y;
      });
      for (int t = 0; t < n; ++t) {
        const int j = ord[t];
        Step &s = steps[(size_t)pi * n + t];
        s.job = j;
        s.a = p[(size_t)j * m + k];
        s.lag = lag[j];
        s.b = p[(size_t)j * m + l];
      }
    }
}

int32_t HostBound::bound(const uint8_t *prefix, int d) const {
  uint64_t U[4] = {0, 0, 0, 0};
  for (int j = 0; j < n; ++j) U[j >> 6] |= 1ull << (j & 63);
  int32_t F[kMaxMachines] = {0};
  for (int i = 0; i < d; ++i) {
    const int j = prefix[i];
    U[j >> 6] &= ~(1ull << (j & 63));
    const int32_t *row = &p[(size_t)j * m];
    F[0] += row[0];
    for (int k = 1; k < m; ++k) F[k] = std::max(F[k], F[k - 1]) + row[k];
  }
  if (d == n) return F[m - 1];
  int32_t hmin[kMaxMachines], qmin[kMaxMachines];
  for (int k = 0; k < m; ++k) hmin[k] = qmin[k] = INT32_MAX;
  for (int j = 0; j < n; ++j) {
    if (!((U[j >> 6] >> (j & 63)) & 1ull)) continue;
    for (int k = 0; k < m; ++k) {
      hmin[k] = std::min(hmin[k], H[(size_t)j * m + k]);
      qmin[k] = std::min(qmin[k], Q[(size_t)j * m + k]);
    }
  }
  int32_t r[kMaxMachines];
  for (int k = 0; k < m; ++k) r[k] = std::max(F[k], F[0] + hmin[k]);
  int32_t lb = 0;
  for (int pi = 0; pi < P; ++pi) {
    int32_t tk = r[pk[pi]], tl = r[pl[pi]];
    const Step *st = &steps[(size_t)pi * n];
    for (int t = 0; t < n; ++t) {
      const int j = st[t].job;
      if (!((U[j >> 6] >> (j & 63)) & 1ull)) continue;
      tk += st[t].a;
      tl = std::max(tl, tk + st[t].lag) + st[t].b;
    }
    lb = std::max(lb, tl + qmin[pl[pi]]);
  }
  return lb;
}

namespace {
bool keeps_host(int rule, int32_t lb, int32_t ub) {
  return rule == FSP_PRUNE_GT ? lb <= ub : lb < ub;
}
}  // namespace

HostSearch::~HostSearch() { stop_threads(); }

void HostSearch::start(const fsp_instance *inst, int threads, int rule_, int32_t ub,
                       std::chrono::steady_clock::time_point t0_) {
  hb.init(inst->p_host, inst->n, inst->m);
  n = inst->n;
  rule = rule_;
  t0 = t0_;
  ub_host.store(ub);
  quit.store(false);
  for (int i = 0; i < threads; ++i) workers.emplace_back([this] { worker(); });
}

void HostSearch::give(const uint8_t *recs, const int32_t *lbs, int count, int stride) {
  {
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < count; ++i) {
      Node v;
      const uint8_t *r = recs + (size_t)i * stride;
      v.d = r[0];
      std::memcpy(v.prefix, r + 1, (size_t)v.d);
      v.lb = lbs[i];
      queue.push_back(v);
    }
  }
  cv.notify_all();
}

bool HostSearch::idle() {
  std::lock_guard<std::mutex> lock(mu);
  return queue.empty() && busy == 0;
}

void HostSearch::wait_idle() {
  std::unique_lock<std::mutex> lock(mu);
  done_cv.wait(lock, [this] { return queue.empty() && busy == 0; });
}

void HostSearch::stop_threads() {
  {
    std::lock_guard<std::mutex> lock(mu);
    quit.store(true);
  }
  cv.notify_all();
  for (std::thread &t : workers) t.join();
  workers.clear();
}

// Smallest bound among the nodes still queued (after the threads stopped).
int32_t HostSearch::open_lb() {
  std::lock_guard<std::mutex> lock(mu);
  int32_t v = INT32_MAX;
  for (const Node &x : queue) v = std::min(v, x.lb);
  return std::min(v, left_lb.load());
}

void HostSearch::propose(int32_t mk, const uint8_t *perm) {
  int32_t cur = ub_host.load();
  while (mk < cur && !ub_host.compare_exchange_weak(cur, mk)) {
  }
  if (mk < cur) {
    std::lock_guard<std::mutex> lock(best_mu);
    if (mk < best) {
      best = mk;
      std::memcpy(best_perm, perm, (size_t)n);
      t_found = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
}

// Depth-first search of one node's subtree (the node itself was bounded and
// counted where it was created): a node that can no longer beat UB is
// eliminated; otherwise every child (unscheduled jobs in ascending id) is
// bounded, complete children propose themselves as the new best, the kept
// ones are searched, smallest job first.
void HostSearch::explore(const Node &root, Counters &c) {
  std::vector<Node> stack;
  stack.push_back(root);
  while (!stack.empty()) {
    if (quit.load()) {
      // time limit: what is left keeps its bound for the open bound
      int32_t v = INT32_MAX;
      for (const Node &x : stack) v = std::min(v, x.lb);
      int32_t cur = left_lb.load();
      while (v < cur && !left_lb.compare_exchange_weak(cur, v)) {
      }
      return;
    }
    const Node v = stack.back();
    stack.pop_back();
    if (!keeps_host(rule, v.lb, ub_host.load())) {
      c.pruned++;
      continue;
    }
    c.branched++;
    bool used[256] = {false};
    for (int i = 0; i < v.d; ++i) used[v.prefix[i]] = true;
    Node kids[256];
    int nk = 0;
    for (int j = 0; j < n; ++j) {
      if (used[j]) continue;
      Node ch;
      ch.d = v.d + 1;
      std::memcpy(ch.prefix, v.prefix, (size_t)v.d);
      ch.prefix[v.d] = (uint8_t)j;
      ch.lb = hb.bound(ch.prefix, ch.d);
      c.bounded++;
      const int32_t ub = ub_host.load();
      if (ch.d == n) {
        c.leaves++;
        if (ch.lb < ub)
          propose(ch.lb, ch.prefix);
        else
          c.pruned++;
      } else if (keeps_host(rule, ch.lb, ub)) {
        kids[nk++] = ch;
      } else {
        c.pruned++;
      }
    }
    for (int i = nk - 1; i >= 0; --i) stack.push_back(kids[i]);
  }
}

void HostSearch::worker() {
  Counters c;
  while (true) {
    Node v;
    {
      std::unique_lock<std::mutex> lock(mu);
      cv.wait(lock, [this] { return quit.load() || !queue.empty(); });
      if (quit.load()) break;
      v = queue.back();
      queue.pop_back();
      ++busy;
    }
    explore(v, c);
    {
      std::lock_guard<std::mutex> lock(mu);
      --busy;
      if (queue.empty() && busy == 0) done_cv.notify_all();
    }
  }
  std::lock_guard<std::mutex> lock(mu);
  total.bounded += c.bounded;
  total.branched += c.branched;
  total.pruned += c.pruned;
  total.leaves += c.leaves;
}

}  // namespace fspi
