// bnb.hpp -- device-resident branch-and-bound state (bnb.hip).
#pragma once
#include <vector>

#include "fsp_internal.hpp"

namespace fspi {

// Wave-level compaction: returns this lane's slot in an array whose length
// counter is *counter (one atomic per wave).  Only lanes with pred get a slot.
// Every lane of the wave must call it.
__device__ __forceinline__ int wave_slot(bool pred, int32_t *counter) {
  const uint64_t mask = __ballot(pred);
  const int lane = __lane_id();
  const uint64_t below = lane == 0 ? 0ull : (mask & ((~0ull) >> (64 - lane)));
  const int rank = __popcll(below);
  const uint64_t act = __ballot(1);
  const int leader = __ffsll((unsigned long long)act) - 1;
  int base = 0;
  if (lane == leader && mask) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + rank;
}

// Workgroup-level compaction: this lane's slot in an array whose length
// counter is *counter, with one atomic per workgroup.  s_cnt is an LDS array
// of blockDim.x / 64 + 1 ints.  Every thread of the workgroup must call it
// (it synchronises the workgroup).
__device__ __forceinline__ int block_slot(bool pred, int32_t *counter, int *s_cnt) {
  const uint64_t mask = __ballot(pred);
  const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int rank = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) s_cnt[w] = __popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < nw; ++i) {
      const int c = s_cnt[i];
      s_cnt[i] = tot;
      tot += c;
    }
    s_cnt[nw] = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  const int slot = s_cnt[nw] + s_cnt[w] + rank;
  __syncthreads();  // s_cnt is reused by the next call
  return slot;
}

// Adds the workgroup's sum of v to *counter (one atomic per workgroup).
// s_cnt as above.  Every thread of the workgroup must call it.
__device__ __forceinline__ void block_total(int64_t *counter, int v, int *s_cnt) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (__lane_id() == 0) s_cnt[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int i = 0; i < nw; ++i) tot += s_cnt[i];
    if (tot) atomicAdd(reinterpret_cast<unsigned long long *>(counter), (unsigned long long)tot);
  }
  __syncthreads();
}

// Adds the wave's sum of v to *counter (one atomic per wave).  Every active
// lane of the wave must call it.
__device__ __forceinline__ void wave_total(int64_t *counter, int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const uint64_t act = __ballot(1);
  const int leader = __ffsll((unsigned long long)act) - 1;
  if (__lane_id() == leader && v)
    atomicAdd(reinterpret_cast<unsigned long long *>(counter), (unsigned long long)v);
}

// Iteration descriptor and counters, in device memory; the host reads a copy
// once per batch of pools.
// bins of the histogram of scores that the best-K selection builds
constexpr int kSelBins = 4096;
// depths one pool may take parents from
constexpr int kMaxSeg = 8;

struct BnbDesc {
  int32_t active;       // the current iteration has parents
  // The pool's parents come from up to kMaxSeg depths, deepest first: every
  // depth but the last is taken whole; depth, parents, parent_base and
  // sel_count describe the last (shallowest) one, the only one a pool may
  // take in part (and so the one the learned ordering selects in).
  int32_t depth;        // parent depth of the last segment
  int32_t parents;      // parents taken from it
  int32_t parent_base;  // index of the first taken parent in its bucket
  int32_t children;     // children written by branch (pool size)
  int32_t ub;           // best makespan known (UB)
  int32_t done;         // no pending node left
  int32_t overflow;     // a bucket ran out of room (never expected)
  int32_t found;        // a schedule better than the initial UB was found
  int32_t improved;     // UB improved since the host last cleared this
  int32_t root_lb;
  int32_t sel_count;    // nodes of the parent depth before the plan took K
  int32_t sel_lo, sel_hi, sel_tie;  // best-K selection slot counters
  int32_t feat_count;   // nodes scored after the last prune
  int32_t log_count;    // training samples logged (may exceed the capacity)
  int32_t nseg;         // depth segments of the current pool
  int32_t seg_depth[kMaxSeg];  // parent depth of each segment, deepest first
  int32_t seg_base[kMaxSeg];   // first taken parent's index in its bucket
  int32_t seg_off[kMaxSeg + 1];  // child-slot offsets: sum of parents x (n - depth)
  int64_t nodes_bounded, nodes_branched, nodes_pruned, leaves, pools;
  uint64_t best_key;    // (makespan << 32) | pool index, best leaf of a pool
};

struct BnbState {
  const fsp_instance *inst = nullptr;
  int n = 0, stride = 0, rule = 0, cus = 0;
  int prefilter = 0;  // one-machine pre-filter in the bounding launches
  uint32_t *lb1_mask = nullptr;     // depths bounded by the one-machine bound (8 words)
  uint32_t *depth_stats = nullptr;  // measurement of the per-depth choice ([3][256])
  int multi = 0;      // pools take parents from several depths (deepest first)
  int64_t cap = 0;  // records per bucket and in the pool buffer
  uint8_t *bnodes = nullptr;   // [n][cap][stride]
  int32_t *blb = nullptr;      // [n][cap]
  int32_t *bcount = nullptr;   // [n]
  uint8_t *pool = nullptr;     // [cap][stride]
  int32_t *pool_lb = nullptr;  // [cap]
  void *slots = nullptr;       // job-mask scratch of the bounding launches
  BnbDesc *desc = nullptr;
  uint8_t *best_perm = nullptr;  // [256]
  int64_t *target_dev = nullptr;
  BnbDesc *host_desc = nullptr;  // pinned
  int64_t *host_target = nullptr;  // pinned
  hipStream_t stream = nullptr;
  int grid = 1;  // workgroups of the branch/prune/selection kernels

  // learned ordering (model != nullptr)
  const fsp_model *model = nullptr;
  float inv_scale = 0.f;
  float *bscore = nullptr;    // [n][cap] estimated completion / scale
  uint8_t *tnodes = nullptr;  // [cap][stride] selection scratch
  int32_t *tlb = nullptr;
  float *tscore = nullptr;
  int32_t *hist = nullptr;    // selection histogram (kept zeroed)
  void *X = nullptr;          // [cap][32] bf16 features
  int64_t *rowdst = nullptr;  // [cap] bucket slot (depth * cap + index) of feature row r

  // training samples (log_cap > 0)
  int64_t log_cap = 0;
  uint32_t log_threshold = 0;  // keep a survivor if hash < threshold
  uint32_t log_seed = 0;
  uint8_t *log_nodes = nullptr;  // [log_cap][stride]
  int32_t *log_lb = nullptr;

  // captured iterations (with the learned ordering: graph / exec include the
  // network's kernels, graph_plain / exec_plain do not)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr, graph_plain = nullptr;
  hipGraphExec_t exec = nullptr, exec_plain = nullptr;
  int32_t *min_est = nullptr;       // device: smallest pending estimate (float bits)
  int32_t *host_min_est = nullptr;  // pinned copy

  int init(const fsp_instance *inst, int64_t max_pool, int rule);
  int init_model(const fsp_model *model, float inv_scale);
  int init_log(int64_t cap, double prob, uint64_t seed);
  void release();
  int start(int32_t ub0, const std::vector<uint8_t> &perm0);
  int set_target(int64_t target);
  int enqueue_iteration(hipStream_t s, bool use_model = true);
  int enqueue_iteration_impl(hipStream_t s);
  int capture(int iters);
  int capture_plain(int iters);
  int replay(bool plain = false);
  int pending_min_estimate(float *out);
  int commit();
  int read_desc();
};

// learned ordering (policy.hip)
int policy_enqueue_select(BnbState &S, hipStream_t s, int grid);
int policy_enqueue_score(BnbState &S, hipStream_t s, int grid);
int policy_features(const fsp_instance *in, const uint8_t *nodes, const int32_t *lbs,
                    int64_t count, int stride, float inv_scale, void *X, hipStream_t s);
int policy_label(const fsp_instance *in, const uint8_t *nodes, const int32_t *lbs,
                 int64_t count, int stride, int32_t final_ub, float inv_scale, float *target,
                 hipStream_t s);
int policy_in_features(int m);

// network (mlp.hip)
int model_forward_dev(const fsp_model *m, const void *x, const int32_t *n_dev, int64_t max_n,
                      float *y, hipStream_t s);
// Forward pass whose epilogue writes the learned ordering's estimate instead
// of the outputs: row r is the node at bucket slot i = rowdst[r], and
// est[i] = lb[i] * inv_scale + y0.
struct ScoreEpilogue {
  const int64_t *rowdst;
  const int32_t *lb;
  float *est;
  float inv_scale;
};
int model_forward_score_dev(const fsp_model *m, const void *x, const int32_t *n_dev,
                            int64_t max_n, const ScoreEpilogue &sc, hipStream_t s);
int model_outputs(const fsp_model *m);
int model_in_features(const fsp_model *m);
int model_trained_jobs(const fsp_model *m);

struct AdaptivePolicy {
  int nb_threads = 256, nb_blocks = 0;
  int64_t max_nb_threads = 0;
  int phase = 0;  // 0 doubling, 1 search around the best, 2 frozen
  double best_eff = -1.0;
  int64_t best_size = 0, current = 0, lo = 0, hi = 0;
  int rounds = 0, trial = 0;
  void init(int threads_per_block, int cus, int64_t max_threads, int64_t max_pool);
  void observe(double efficiency);
  int64_t round_pool(double x) const;
};

int64_t neh_host(const std::vector<int32_t> &p, int n, int m,
                 std::vector<uint8_t> &perm);

}  // namespace fspi
