// bnb.hip -- device-resident branch-and-bound around the pool-bounding kernel.
//
// The paper's loop (Sec. III, Fig. 2): select a pool of pending nodes,
// deepest first; branch them; bound every child in one launch; eliminate the
// children that cannot beat the best known schedule; repeat until no node is
// pending.  Here every step stays on the device; the host only chooses the
// pool size and reads back a few counters once per batch of pools.
//
// Pending nodes live in one bucket per depth (records + their bounds), in
// HBM.  Selection takes the last K nodes of the deepest non-empty bucket
// (LIFO inside a bucket); the batched kinds then continue with the next
// shallower non-empty buckets, taking each whole until the pool is full
// (deepest pending nodes first, at most kMaxSeg depths, the last one in
// part).  The children of depth-d parents all go to bucket d+1, and a bucket
// receives children only when it is empty (every depth below the deepest
// taken one is empty, and every taken depth but the last is emptied), so a
// bucket never holds more than one pool of children, which bounds its size
// by the largest pool.
//
// One iteration = four launches, all sized from a device descriptor so that
// the sequence can be queued back-to-back (or captured once and replayed):
//   plan    1 wave: commit the best leaf of the previous pool, pick the
//           depths and the number of parents, or flag the search as done;
//   branch  one lane per (parent, child slot): a parent whose bound can no
//           longer beat UB is eliminated (lazy re-check, Sec. II.A); the others
//           append their unscheduled jobs in ascending id (Sec. II.B: one son
//           per unscheduled job); children are compacted with a wave ballot;
//           a record's bytes past its prefix are never read, so only the
//           16-byte chunks up to the prefix are moved;
//   bound   the pool-bounding kernel, count read from the descriptor;
//   prune   one lane per child: leaves propose themselves as the new best
//           (64-bit atomic min of (makespan, index)); other children that can
//           still beat UB are compacted into the next bucket.
// Elimination compares with the UB in force when the pool was selected (the
// paper eliminates after the whole pool has been bounded, Sec. III).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fsp_internal.hpp"
#include "bnb.hpp"
#include "host_search.hpp"

using namespace fspi;

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ bool keeps(int rule, int lb, int ub) {
  return rule == FSP_PRUNE_GT ? lb <= ub : lb < ub;
}

// ---- plan ------------------------------------------------------------------
// Plan the next pool, one wave: commit the best leaf of the previous pool,
// then take parents deepest first: from the deepest non-empty depth as many
// nodes (from the top) as make about `target` children (at least one); with
// `multi`, a depth taken whole is followed by the next shallower non-empty
// depth, and so on (at most kMaxSeg depths), until the target is reached.
// The wave reads 64 bucket counts per load; every lane then walks the
// counts in step (uniform values).  Every bucket that receives children is
// empty when the pool is planned: a depth taken whole is emptied, and the
// depth below the deepest taken one was empty.
__global__ __launch_bounds__(64) void plan_kernel(BnbDesc *D, int32_t *bcount,
                                                  const uint8_t *pool, uint8_t *best_perm,
                                                  int n, int stride,
                                                  const int64_t *target_dev,
                                                  int commit_only, int multi) {
  const int lane = (int)threadIdx.x;
  int done = 0;
  if (lane == 0) {
    const uint64_t key = D->best_key;
    if (key != ~0ull) {
      const int mk = (int)(key >> 32);
      const uint32_t idx = (uint32_t)(key & 0xffffffffu);
      if (mk < D->ub) {
        D->ub = mk;
        const uint8_t *rec = pool + (size_t)idx * stride;
        for (int i = 0; i < n; ++i) best_perm[i] = rec[1 + i];
        D->found = 1;
        D->improved = 1;
      }
      D->best_key = ~0ull;
    }
    D->children = 0;
    D->active = 0;
    D->parents = 0;
    if (D->overflow) D->done = 1;
    done = D->done;
  }
  done = __shfl(done, 0);
  if (commit_only || done) return;
  const int64_t target = *target_dev;
  int nseg = 0, last_d = -1, last_k = 0, last_c = 0;
  int64_t children = 0;
  bool stop = false;
  for (int base = ((n - 1) / 64) * 64; base >= 0 && !stop; base -= 64) {
    const int idx = base + lane;
    const int cnt = idx < n ? bcount[idx] : 0;
    uint64_t mask = __ballot(cnt > 0);
    while (mask && !stop) {
      const int hi = 63 - __builtin_clzll(mask);
      mask &= ~(1ull << hi);
      const int d = base + hi, c = __shfl(cnt, hi), u = n - d;
      int64_t k = (target - children) / u;
      if (nseg == 0 && k < 1) k = 1;
      if (k < 1) {
        stop = true;
        break;
      }
      if (k > c) k = c;
      if (lane == 0) {
        D->seg_depth[nseg] = d;
        D->seg_base[nseg] = c - (int)k;
        D->seg_off[nseg] = (int)children;
        bcount[d] = c - (int)k;
      }
      children += k * u;
      ++nseg;
      last_d = d;
      last_k = (int)k;
      last_c = c;
      if (!multi || k < c || nseg == kMaxSeg) stop = true;
    }
  }
  if (lane != 0) return;
  if (nseg == 0) {
    D->done = 1;
    return;
  }
  D->nseg = nseg;
  D->seg_off[nseg] = (int)children;
  D->depth = last_d;
  D->parents = last_k;
  D->sel_count = last_c;
  D->parent_base = last_c - last_k;
  D->active = 1;
  D->pools += 1;
}

// ---- branch ----------------------------------------------------------------
// The parent record is read as 16-byte chunks (records are 16-byte aligned):
// the chunks up to the one holding byte 1 + d are decoded for the scheduled
// set and written back, patched, as the child; later bytes of a record are
// never read at depth d + 1.
//
// With the learned ordering, a pool that takes only part of its depth was
// partitioned into the scratch buffers (tnodes, tlb, tscore: the nodes that
// stay first, the K taken ones on top).  The parents are then read from the
// scratch, and this kernel also writes the nodes that stay back into the
// bucket and clears the selection's histogram and counters for its next use.
__global__ __launch_bounds__(kThreads) void branch_kernel(
    BnbDesc *D, uint8_t *__restrict__ bnodes, int32_t *__restrict__ blb,
    uint8_t *__restrict__ pool, int n, int stride, int64_t cap, int rule,
    const uint8_t *__restrict__ tnodes, const int32_t *__restrict__ tlb,
    const float *__restrict__ tscore, float *__restrict__ bscore,
    int32_t *__restrict__ hist, int learned) {
  if (!D->active) return;
  const int K = D->parents, base = D->parent_base, nseg = D->nseg;
  const int ub = D->ub;
  // the last segment is read from the selection scratch when the learned
  // ordering took part of its depth
  const bool sel = learned && K < D->sel_count;
  const int total = D->seg_off[nseg];  // <= target + n: fits 32 bits
  const int gsz = gridDim.x * blockDim.x;
  __shared__ int s_cnt[kThreads / 64 + 1];
  int branched = 0, pruned = 0;
  // iterate so that every thread of the grid takes part in each round
  for (int r0 = blockIdx.x * blockDim.x; r0 < total; r0 += gsz) {
    const int slot = r0 + threadIdx.x;
    const bool in = slot < total;
    int p = 0, c = 0, d = 0;
    bool live = false, from_sel = false;
    if (in) {
      int s = 0;
#pragma unroll
      for (int t = 1; t < kMaxSeg; ++t)
        if (t < nseg && slot >= D->seg_off[t]) s = t;
      d = D->seg_depth[s];
      const int u = n - d, r = slot - D->seg_off[s];
      const int q = r / u;
      c = r - q * u;
      p = D->seg_base[s] + q;
      from_sel = sel && s == nseg - 1;
      const int32_t *par_lb = from_sel ? tlb : blb + (int64_t)d * cap;
      live = keeps(rule, par_lb[p], ub);
      if (c == 0) {
        branched += live ? 1 : 0;
        pruned += live ? 0 : 1;
      }
    }
    const int pos = block_slot(live, &D->children, s_cnt);
    if (!live) continue;
    const int dd = d, lc = (1 + d) >> 4;  // chunk holding the new job's byte
    const uint8_t *par_nodes = from_sel ? tnodes : bnodes + (int64_t)d * cap * stride;
    const uint4 *src = reinterpret_cast<const uint4 *>(par_nodes + (int64_t)p * stride);
    uint4 *dst = reinterpret_cast<uint4 *>(pool + (size_t)pos * stride);
    if (n <= 32) {
      // scheduled set in one register; byte 1 + d <= 32 lies in chunk 0..2
      uint32_t used = 0;
      uint4 ch[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k > lc) break;
        const uint4 v = src[k];
        ch[k] = v;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          const int at = 16 * k + b;
          if (at >= 1 && at <= dd) used |= 1u << ((w[b >> 2] >> (8 * (b & 3))) & 31u);
        }
      }
      // c-th unscheduled job in ascending id
      uint32_t freew = ~used & (n == 32 ? 0xffffffffu : ((1u << n) - 1u));
      for (int t = 0; t < c; ++t) freew &= freew - 1u;
      const uint32_t job = (uint32_t)(__ffs(freew) - 1);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k > lc) break;
        const uint4 v = ch[k];
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
        if (k == 0) w[0] = (w[0] & ~0xffu) | (uint32_t)(d + 1);
        if (k == lc) {
          const int b = (1 + d) & 15, sh = 8 * (b & 3);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q == (b >> 2)) w[q] = (w[q] & ~(0xffu << sh)) | (job << sh);
        }
        dst[k] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    } else {
      uint32_t used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int k = 0; 16 * k <= dd; ++k) {
        const uint4 v = src[k];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          const int at = 16 * k + b;
          if (at >= 1 && at <= dd) {
            const uint32_t j = (w[b >> 2] >> (8 * (b & 3))) & 0xffu;
            used[j >> 5] |= 1u << (j & 31u);
          }
        }
      }
      int job = -1, left = c;
      for (int w = 0; w < 8 && job < 0; ++w) {
        const int lo = w * 32;
        if (lo >= n) break;
        uint32_t freew = ~used[w];
        if (n - lo < 32) freew &= (1u << (n - lo)) - 1u;
        const int cnt = __popc(freew);
        if (left < cnt) {
          for (int t = 0; t < left; ++t) freew &= freew - 1u;
          job = lo + __ffs(freew) - 1;
        } else {
          left -= cnt;
        }
      }
      for (int k = 0; k <= lc; ++k) dst[k] = src[k];
      uint8_t *crec = reinterpret_cast<uint8_t *>(dst);
      crec[0] = (uint8_t)(d + 1);
      crec[1 + d] = (uint8_t)job;
    }
  }
  block_total(&D->nodes_branched, branched, s_cnt);
  block_total(&D->nodes_pruned, pruned, s_cnt);
  if (!sel) return;
  const int64_t at0 = (int64_t)D->depth * cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < base; i += gsz) {
    const uint4 *src = reinterpret_cast<const uint4 *>(tnodes + (int64_t)i * stride);
    uint4 *dst = reinterpret_cast<uint4 *>(bnodes + (at0 + i) * stride);
    for (int q = 0; q < stride / 16; ++q) dst[q] = src[q];
    blb[at0 + i] = tlb[i];
    bscore[at0 + i] = tscore[i];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSelBins; i += gsz) hist[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) D->sel_lo = D->sel_hi = D->sel_tie = 0;
}

// ---- prune + compaction ----------------------------------------------------
// 32-bit mix of (pool counter, index, seed): the training-sample lottery
__device__ __forceinline__ uint32_t sample_hash(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return (uint32_t)x;
}

__global__ __launch_bounds__(kThreads) void prune_kernel(
    BnbDesc *D, const uint8_t *__restrict__ pool,
    const int32_t *__restrict__ pool_lb, uint8_t *__restrict__ bnodes,
    int32_t *__restrict__ blb, int32_t *__restrict__ bcount, int n, int stride,
    int64_t cap, int rule, int64_t log_cap, uint32_t log_threshold, uint32_t log_seed,
    uint8_t *__restrict__ log_nodes, int32_t *__restrict__ log_lb) {
  if (!D->active) return;
  const int total = D->children;
  const int nseg = D->nseg;
  // only the deepest segment's children can be complete schedules
  const bool complete = D->seg_depth[0] + 1 == n;
  const int ub = D->ub;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(&D->nodes_bounded),
              (unsigned long long)total);
  const int gsz = gridDim.x * blockDim.x;
  __shared__ int s_cnt[kThreads / 64 + 1];
  int leaves = 0, pruned = 0;
  for (int r0 = blockIdx.x * blockDim.x; r0 < total; r0 += gsz) {
    const int i = r0 + threadIdx.x;
    const bool in = i < total;
    const int lb = in ? pool_lb[i] : 0;
    const int d1 = in ? (int)pool[(size_t)i * stride] : 0;  // the child's depth
    const bool leaf = in && d1 == n;
    const bool keep = in && !leaf && keeps(rule, lb, ub);
    leaves += leaf ? 1 : 0;
    pruned += (in && !keep && !(leaf && lb < ub)) ? 1 : 0;
    if (complete) {
      // the wave's smallest (makespan, index) key, then one atomic per wave
      uint64_t key = (leaf && lb < ub) ? (((uint64_t)(uint32_t)lb << 32) | (uint64_t)i)
                                       : ~0ull;
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(key, off);
        key = o < key ? o : key;
      }
      if (__lane_id() == 0 && key != ~0ull)
        atomicMin(reinterpret_cast<unsigned long long *>(&D->best_key),
                  (unsigned long long)key);
    }
    // compaction into the bucket of each segment's children (uniform loop)
    int pos = 0;
    for (int sg = 0; sg < nseg; ++sg) {
      const int ds1 = D->seg_depth[sg] + 1;
      if (ds1 >= n) continue;
      const bool mine = keep && d1 == ds1;
      const int ps = block_slot(mine, &bcount[ds1], s_cnt);
      if (mine) pos = ps;
    }
    if (!keep) continue;
    if (log_cap > 0 &&
        sample_hash(((uint64_t)D->pools << 32) ^ (uint64_t)i ^ ((uint64_t)log_seed << 16)) <
            log_threshold) {
      const int slot = atomicAdd(&D->log_count, 1);
      if (slot < log_cap) {
        const uint4 *src = reinterpret_cast<const uint4 *>(pool + (size_t)i * stride);
        uint4 *dst = reinterpret_cast<uint4 *>(log_nodes + (size_t)slot * stride);
        for (int q = 0; q < stride / 16; ++q) dst[q] = src[q];
        log_lb[slot] = lb;
      }
    }
    if (pos >= cap) {
      D->overflow = 1;
      continue;
    }
    const int64_t at = (int64_t)d1 * cap + pos;
    const uint4 *src = reinterpret_cast<const uint4 *>(pool + (size_t)i * stride);
    uint4 *dst = reinterpret_cast<uint4 *>(bnodes + at * stride);
    // bytes past the prefix are never read
    for (int q = 0; q <= (d1 >> 4); ++q) dst[q] = src[q];
    blb[at] = lb;
  }
  block_total(&D->leaves, leaves, s_cnt);
  block_total(&D->nodes_pruned, pruned, s_cnt);
}

// smallest bound among the pending nodes (for the optimality gap after a
// time limit): an atomic min over every bucket entry
__global__ void open_lb_kernel(const int32_t *__restrict__ blb,
                               const int32_t *__restrict__ bcount, int n, int64_t cap,
                               int32_t *__restrict__ out) {
  for (int d = 0; d < n; ++d) {
    const int c = bcount[d];
    int best = 0x7fffffff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
      best = min(best, blb[(int64_t)d * cap + i]);
    for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_down(best, off));
    if ((threadIdx.x & 63) == 0 && best != 0x7fffffff) atomicMin(out, best);
  }
}

// smallest estimate (est = bound / scale + predicted gap, >= 0) among the
// pending nodes, as float bits: for non-negative floats the bit patterns
// order like the values, so an integer atomic min serves
__global__ void min_est_kernel(const float *__restrict__ bscore,
                               const int32_t *__restrict__ bcount, int n, int64_t cap,
                               int32_t *__restrict__ out) {
  for (int d = 0; d < n; ++d) {
    const int c = bcount[d];
    int best = 0x7fffffff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
      best = min(best, __float_as_int(fmaxf(bscore[(int64_t)d * cap + i], 0.f)));
    for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_down(best, off));
    if ((threadIdx.x & 63) == 0 && best != 0x7fffffff) atomicMin(out, best);
  }
}

// seed: place the root in bucket 0 if it can beat UB; count its bound
__global__ void seed_kernel(BnbDesc *D, const int32_t *root_lb,
                            uint8_t *bnodes, int32_t *blb, int32_t *bcount,
                            int stride, int rule) {
  if (threadIdx.x != 0) return;
  D->nodes_bounded += 1;
  D->root_lb = *root_lb;
  if (keeps(rule, *root_lb, D->ub)) {
    for (int i = 0; i < stride; ++i) bnodes[i] = 0;
    blb[0] = *root_lb;
    bcount[0] = 1;
  } else {
    D->nodes_pruned += 1;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace fspi {

int64_t neh_host(const std::vector<int32_t> &p, int n, int m,
                 std::vector<uint8_t> &perm) {
  // NEH insertion: jobs by total work (descending, ties by id), each inserted
  // at the position giving the smallest partial makespan (earliest on ties).
  std::vector<int> order(n);
  std::vector<int64_t> tot(n, 0);
  for (int j = 0; j < n; ++j) {
    order[j] = j;
    for (int k = 0; k < m; ++k) tot[j] += p[(size_t)j * m + k];
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return tot[a] > tot[b]; });
  std::vector<int> seq;
  std::vector<int64_t> c(m);
  auto span = [&](const std::vector<int> &s) {
    std::fill(c.begin(), c.end(), 0);
    for (int x : s) {
      c[0] += p[(size_t)x * m];
      for (int k = 1; k < m; ++k) c[k] = std::max(c[k], c[k - 1]) + p[(size_t)x * m + k];
    }
    return c[m - 1];
  };
  seq.push_back(order[0]);
  std::vector<int> trial;
  for (int a = 1; a < n; ++a) {
    int best_pos = 0;
    int64_t best = -1;
    for (int pos = 0; pos <= (int)seq.size(); ++pos) {
      trial = seq;
      trial.insert(trial.begin() + pos, order[a]);
      const int64_t v = span(trial);
      if (best < 0 || v < best) {
        best = v;
        best_pos = pos;
      }
    }
    seq.insert(seq.begin() + best_pos, order[a]);
  }
  perm.assign(seq.begin(), seq.end());
  return span(seq);
}

int BnbState::init(const fsp_instance *inst_, int64_t max_pool, int rule_) {
  inst = inst_;
  n = inst->n;
  stride = round_up(n + 1, 16);
  rule = rule_;
  cap = max_pool + n;
  const size_t bbytes = (size_t)n * cap * stride;
  if (hipMalloc(&bnodes, bbytes) != hipSuccess ||
      hipMalloc(&blb, (size_t)n * cap * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&bcount, (size_t)n * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&pool, (size_t)cap * stride) != hipSuccess ||
      hipMalloc(&pool_lb, (size_t)cap * sizeof(int32_t)) != hipSuccess ||
      (walk_scratch_bytes(inst, cap) > 0 &&
       hipMalloc(&slots, walk_scratch_bytes(inst, cap)) != hipSuccess) ||
      hipMalloc(&desc, sizeof(BnbDesc)) != hipSuccess ||
      hipMalloc(&best_perm, 256) != hipSuccess ||
      hipMalloc(&target_dev, sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&min_est, sizeof(int32_t)) != hipSuccess ||
      hipHostMalloc(&host_min_est, sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&host_desc, sizeof(BnbDesc), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(&host_target, sizeof(int64_t), hipHostMallocDefault) !=
          hipSuccess)
    return FSP_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FSP_EDEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
      hipSuccess)
    return FSP_EDEVICE;
  grid = std::max(1, std::min<int>(cus * 4, (int)((cap + kThreads - 1) / kThreads)));
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
    return FSP_EDEVICE;
  return FSP_OK;
}

int BnbState::init_model(const fsp_model *model_, float inv_scale_) {
  model = model_;
  inv_scale = inv_scale_;
  if (hipMalloc(&bscore, (size_t)n * cap * sizeof(float)) != hipSuccess ||
      hipMalloc(&tnodes, (size_t)cap * stride) != hipSuccess ||
      hipMalloc(&tlb, (size_t)cap * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&tscore, (size_t)cap * sizeof(float)) != hipSuccess ||
      hipMalloc(&hist, 4096 * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&X, (size_t)cap * 32 * 2) != hipSuccess ||
      hipMalloc(&rowdst, (size_t)cap * sizeof(int64_t)) != hipSuccess)
    return FSP_ENOMEM;
  FSP_HIP_TRY(hipMemsetAsync(hist, 0, 4096 * sizeof(int32_t), stream));
  // the root (bucket 0) is alone: any score will do
  FSP_HIP_TRY(hipMemsetAsync(bscore, 0, sizeof(float), stream));
  return FSP_OK;
}

int BnbState::init_log(int64_t lcap, double prob, uint64_t seed) {
  log_cap = lcap;
  const double t = prob <= 0 ? 0.0 : (prob >= 1 ? 4294967295.0 : prob * 4294967296.0);
  log_threshold = (uint32_t)t;
  log_seed = (uint32_t)(seed ^ (seed >> 32));
  if (hipMalloc(&log_nodes, (size_t)lcap * stride) != hipSuccess ||
      hipMalloc(&log_lb, (size_t)lcap * sizeof(int32_t)) != hipSuccess)
    return FSP_ENOMEM;
  return FSP_OK;
}

void BnbState::release() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (exec_plain) (void)hipGraphExecDestroy(exec_plain);
  if (graph_plain) (void)hipGraphDestroy(graph_plain);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (void *p : {(void *)bnodes, (void *)blb, (void *)bcount, (void *)pool, (void *)pool_lb, slots,
                  (void *)desc, (void *)best_perm, (void *)target_dev, (void *)bscore,
                  (void *)tnodes, (void *)tlb, (void *)tscore, (void *)hist, X,
                  (void *)rowdst,
                  (void *)log_nodes, (void *)log_lb, (void *)min_est, (void *)lb1_mask,
                  (void *)depth_stats})
    if (p) (void)hipFree(p);
  if (host_min_est) (void)hipHostFree(host_min_est);
  if (host_desc) (void)hipHostFree(host_desc);
  if (host_target) (void)hipHostFree(host_target);
  if (stream) (void)hipStreamDestroy(stream);
  *this = BnbState();
}

int BnbState::start(int32_t ub0, const std::vector<uint8_t> &perm0) {
  BnbDesc h{};
  h.ub = ub0;
  h.best_key = ~0ull;
  FSP_HIP_TRY(hipMemcpyAsync(desc, &h, sizeof(h), hipMemcpyHostToDevice, stream));
  FSP_HIP_TRY(hipMemsetAsync(bcount, 0, (size_t)n * sizeof(int32_t), stream));
  std::vector<uint8_t> bp(256, 0);
  std::copy(perm0.begin(), perm0.end(), bp.begin());
  FSP_HIP_TRY(hipMemcpyAsync(best_perm, bp.data(), 256, hipMemcpyHostToDevice, stream));
  // bound the root: an all-zero record in the pool buffer
  FSP_HIP_TRY(hipMemsetAsync(pool, 0, stride, stream));
  int rc = launch_bound(inst, pool, stride, 1, pool_lb, stream, nullptr, slots);
  if (rc != FSP_OK) return rc;
  hipLaunchKernelGGL(seed_kernel, dim3(1), dim3(64), 0, stream, desc, pool_lb,
                     bnodes, blb, bcount, stride, rule);
  FSP_HIP_TRY(hipGetLastError());
  FSP_HIP_TRY(hipStreamSynchronize(stream));
  return FSP_OK;
}

int BnbState::set_target(int64_t target) {
  *host_target = target;
  FSP_HIP_TRY(hipMemcpyAsync(target_dev, host_target, sizeof(int64_t),
                             hipMemcpyHostToDevice, stream));
  return FSP_OK;
}

// One iteration; use_model = false leaves out the learned ordering's
// kernels (the branch kernel then takes the top of the depth, LIFO).
int BnbState::enqueue_iteration(hipStream_t s, bool use_model) {
  const fsp_model *saved = model;
  if (!use_model) model = nullptr;
  const int rc = enqueue_iteration_impl(s);
  model = saved;
  return rc;
}

int BnbState::enqueue_iteration_impl(hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(64), 0, s, desc, bcount,
                     pool, best_perm, n, stride, target_dev, 0, multi);
  FSP_HIP_TRY(hipGetLastError());
  int rc;
  if (model && (rc = policy_enqueue_select(*this, s, grid)) != FSP_OK) return rc;
  hipLaunchKernelGGL(branch_kernel, dim3(grid), dim3(kThreads), 0, s, desc,
                     bnodes, blb, pool, n, stride, cap, rule, tnodes, tlb, tscore, bscore,
                     hist, model ? 1 : 0);
  FSP_HIP_TRY(hipGetLastError());
  Prefilter pf;
  if (prefilter || depth_stats) {
    pf.ub = &desc->ub;  // constant from this iteration's plan to the next
    pf.rule = rule;
  }
  pf.lb1_depths = lb1_mask;
  pf.depth_stats = depth_stats;
  rc = launch_bound(inst, pool, stride, cap, pool_lb, s, &desc->children, slots, pf);
  if (rc != FSP_OK) return rc;
  hipLaunchKernelGGL(prune_kernel, dim3(grid), dim3(kThreads), 0, s, desc,
                     pool, pool_lb, bnodes, blb, bcount, n, stride, cap, rule, log_cap,
                     log_threshold, log_seed, log_nodes, log_lb);
  FSP_HIP_TRY(hipGetLastError());
  if (model && (rc = policy_enqueue_score(*this, s, grid)) != FSP_OK) return rc;
  return FSP_OK;
}

// Capture `iters` iterations once; every replay then costs one graph launch.
// The kernels read their sizes and the pool target from device memory, so
// one graph serves every pool size.
int BnbState::capture(int iters) {
  FSP_HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  FSP_HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = FSP_OK;
  for (int i = 0; i < iters && rc == FSP_OK; ++i) rc = enqueue_iteration(cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cap_stream, &g);
  if (rc != FSP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return FSP_EDEVICE;
  graph = g;
  FSP_HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  return FSP_OK;
}

// The same iterations without the learned ordering's kernels (captured on
// first use).
int BnbState::capture_plain(int iters) {
  if (exec_plain) return FSP_OK;
  if (!cap_stream)
    FSP_HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  FSP_HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = FSP_OK;
  for (int i = 0; i < iters && rc == FSP_OK; ++i) rc = enqueue_iteration(cap_stream, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cap_stream, &g);
  if (rc != FSP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return FSP_EDEVICE;
  graph_plain = g;
  FSP_HIP_TRY(hipGraphInstantiate(&exec_plain, graph_plain, nullptr, nullptr, 0));
  return FSP_OK;
}

int BnbState::replay(bool plain) {
  FSP_HIP_TRY(hipGraphLaunch(plain ? exec_plain : exec, stream));
  return FSP_OK;
}

// Smallest estimate among the pending nodes (learned ordering only);
// synchronises the stream.
int BnbState::pending_min_estimate(float *out) {
  *host_min_est = 0x7fffffff;
  FSP_HIP_TRY(hipMemcpyAsync(min_est, host_min_est, sizeof(int32_t), hipMemcpyHostToDevice,
                             stream));
  hipLaunchKernelGGL(min_est_kernel, dim3(grid), dim3(256), 0, stream, bscore, bcount, n, cap,
                     min_est);
  FSP_HIP_TRY(hipGetLastError());
  FSP_HIP_TRY(hipMemcpyAsync(host_min_est, min_est, sizeof(int32_t), hipMemcpyDeviceToHost,
                             stream));
  FSP_HIP_TRY(hipStreamSynchronize(stream));
  const int32_t bits = *host_min_est;
  *out = bits == 0x7fffffff ? INFINITY : __builtin_bit_cast(float, bits);
  return FSP_OK;
}

int BnbState::commit() {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(64), 0, stream, desc, bcount,
                     pool, best_perm, n, stride, target_dev, 1, multi);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int BnbState::read_desc() {
  FSP_HIP_TRY(hipMemcpyAsync(host_desc, desc, sizeof(BnbDesc),
                             hipMemcpyDeviceToHost, stream));
  FSP_HIP_TRY(hipStreamSynchronize(stream));
  return FSP_OK;
}

// ---- pool-size policies (host) ---------------------------------------------

// The paper's dynamic parameter tuning (Algorithm 1, Sec. III): start with
// threads-per-block x #multiprocessors; every nb_iterations pools measure the
// efficiency (nodes bounded per second of the batch) and double the number of
// blocks while threads x blocks stays within the device's resident-thread
// maximum; then search around the best size (lower and upper midpoints of
// [best/2, 2 best], two rounds) and keep the best for the rest of the run.
void AdaptivePolicy::init(int threads_per_block, int cus, int64_t max_threads,
                          int64_t max_pool) {
  nb_threads = threads_per_block;
  nb_blocks = cus;
  max_nb_threads = std::min<int64_t>(max_threads, max_pool);
  phase = 0;
  best_eff = -1.0;
  best_size = (int64_t)nb_threads * nb_blocks;
  current = best_size;
  if (current > max_nb_threads) current = max_nb_threads;
  lo = hi = 0;
  rounds = 0;
  trial = 0;
}

int64_t AdaptivePolicy::round_pool(double x) const {
  int64_t v = (int64_t)std::llround(x / nb_threads) * nb_threads;
  if (v < nb_threads) v = nb_threads;
  if (v > max_nb_threads) v = max_nb_threads;
  return v;
}

void AdaptivePolicy::observe(double efficiency) {
  if (phase == 2) return;  // frozen
  const bool improved = efficiency > best_eff;
  if (improved) {
    best_eff = efficiency;
    best_size = current;
  }
  if (phase == 0) {
    const int64_t next = (int64_t)nb_threads * nb_blocks * 2;
    if (next <= max_nb_threads) {
      nb_blocks *= 2;
      current = next;
      return;
    }
    // doubling reached the device maximum: search around the best size
    phase = 1;
    lo = best_size / 2;
    hi = best_size * 2;
    rounds = 0;
    trial = 0;
  }
  if (phase == 1) {
    // trials alternate: lower midpoint, upper midpoint; after both, narrow
    // the interval around the best and start a new round
    if (trial == 2) {
      lo = std::max<int64_t>(lo, (lo + best_size) / 2);
      hi = std::min<int64_t>(hi, (best_size + hi) / 2);
      trial = 0;
      ++rounds;
    }
    if (rounds >= 2) {
      phase = 2;
      current = best_size;
      return;
    }
    const double mid = trial == 0 ? 0.5 * (double)(lo + best_size)
                                  : 0.5 * (double)(best_size + hi);
    current = round_pool(mid);
    ++trial;
  }
}

}  // namespace fspi

// ---------------------------------------------------------------------------
namespace {

struct SampleSpec {
  int64_t cap;      // samples to keep at most
  double prob;      // probability that a surviving child is logged
  uint64_t seed;
  void *x;          // device bf16 [cap][32]
  float *target;    // device fp32 [cap][2]
  int64_t *n_out;   // host
};

// Search throughput over the batches that start after the first `skip`
// fraction of the search loop's share of the time limit (the first batches of
// a search from the root hold few nodes, the more so the larger the pool
// target, and would bias a short measurement toward small pools).  The time
// limit is stretched, up to max_s, until min_batches batches were counted, so
// that shapes whose batches are long are rated on as many batches as cheap
// ones.
struct RateWindow {
  double skip;
  int min_batches;
  double max_s;
  int64_t nodes = 0;
  double secs = 0.0;
  int batches = 0;
};

struct TuneEntry {
  int dev, n, m;
  int64_t pool;
  double rate;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
// depths bounded by the one-machine bound, per (device, n, m)
struct BoundTuneEntry {
  int dev, n, m;
  uint32_t mask[8];
};
std::vector<BoundTuneEntry> g_bound_tune;

int run_bnb(const fsp_instance *inst, const fsp_pool_policy *policy, int32_t ub_in,
            fsp_result *out, const SampleSpec *samples, RateWindow *window = nullptr,
            std::vector<uint32_t> *depth_stats = nullptr);

int tuned_pool(const fsp_instance *inst, int64_t *pool) {
  int64_t p = 0;
  double r = 0;
  const int rc = fsp_autotune_pool(inst, 0.0, &p, &r);
  if (rc == FSP_OK) *pool = p;
  return rc;
}

// One exchange of the hybrid search, between two batches of device pools
// (the device stream is idle): UB both ways, then, if the host threads are
// idle, hand them nodes with at most `left` unscheduled jobs from the top of
// the deepest non-empty bucket.
int hybrid_exchange(BnbState &S, HostSearch &hs, const BnbDesc &h, int threads, int left,
                    int chunk, std::vector<int32_t> &hcount, std::vector<uint8_t> &hrec,
                    std::vector<int32_t> &hlb) {
  const int n = S.n;
  const int32_t hub = hs.ub_host.load();
  if (hub < h.ub) {
    FSP_HIP_TRY(hipMemcpy(&S.desc->ub, &hub, sizeof(int32_t), hipMemcpyHostToDevice));
  } else {
    int32_t cur = hub;
    while (h.ub < cur && !hs.ub_host.compare_exchange_weak(cur, h.ub)) {
    }
  }
  if (h.done || !hs.idle()) return FSP_OK;
  FSP_HIP_TRY(hipMemcpy(hcount.data(), S.bcount, (size_t)n * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
  int d = n - 1;
  while (d >= 0 && hcount[d] == 0) --d;
  if (d < 0 || n - d > left) return FSP_OK;
  const int c = (int)std::min<int64_t>(hcount[d], S.cap);
  const int k = std::min(c, chunk * threads);
  hrec.resize((size_t)k * S.stride);
  hlb.resize(k);
  const int64_t at = (int64_t)d * S.cap + (c - k);
  FSP_HIP_TRY(hipMemcpy(hrec.data(), S.bnodes + at * S.stride, (size_t)k * S.stride,
                        hipMemcpyDeviceToHost));
  FSP_HIP_TRY(hipMemcpy(hlb.data(), S.blb + at, (size_t)k * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
  const int32_t rest = c - k;
  FSP_HIP_TRY(hipMemcpy(S.bcount + d, &rest, sizeof(int32_t), hipMemcpyHostToDevice));
  hs.give(hrec.data(), hlb.data(), k, S.stride);
  return FSP_OK;
}

int run_bnb(const fsp_instance *inst, const fsp_pool_policy *policy, int32_t ub_in,
            fsp_result *out, const SampleSpec *samples, RateWindow *window,
            std::vector<uint32_t> *depth_stats) {
  if (!inst || !policy || !out) return FSP_EINVAL;
  if (policy->bound_choice < 0 || policy->bound_choice > 2) return FSP_EINVAL;
  // the per-depth choice of bound (Sec. VI: other lower bounds): the depths
  // whose nodes take the one-machine bound, from the autotuner or the caller
  uint32_t lb1_mask[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (policy->bound_choice == 1) {
    const int rc = fsp_autotune_bounds(inst, 0.0, lb1_mask);
    if (rc != FSP_OK) return rc;
  } else if (policy->bound_choice == 2) {
    std::copy(policy->lb1_depths, policy->lb1_depths + 8, lb1_mask);
  }
  if (policy->prune_rule != FSP_PRUNE_GE && policy->prune_rule != FSP_PRUNE_GT)
    return FSP_EINVAL;
  if (policy->host_threads < 0 || policy->host_threads > 256) return FSP_EINVAL;
  const int kind = policy->kind;
  if (kind < FSP_POOL_FIXED || kind > FSP_POOL_LEARNED) return FSP_EINVAL;
  if (kind == FSP_POOL_FIXED && policy->fixed_pool < 1) return FSP_EINVAL;
  const fsp_model *model = nullptr;
  if (kind == FSP_POOL_LEARNED) {
    model = reinterpret_cast<const fsp_model *>(policy->model);
    if (!model) return FSP_EINVAL;
    if (model_in_features(model) != policy_in_features(inst->m)) return FSP_EINVAL;
  }
  uint8_t *user_perm = out->perm;
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed = [&] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start)
        .count();
  };
  const int n = inst->n;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  int cus = 0, max_tpm = 0;
  FSP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  FSP_HIP_TRY(hipDeviceGetAttribute(&max_tpm, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev));
  const int64_t device_threads = (int64_t)cus * max_tpm;
  int64_t fixed = 0;
  if (kind == FSP_POOL_FIXED) fixed = policy->fixed_pool;
  if (kind == FSP_POOL_AUTOTUNED || kind == FSP_POOL_LEARNED) {
    fixed = policy->fixed_pool;
    if (fixed < 1) {
      const int rc = tuned_pool(inst, &fixed);
      if (rc != FSP_OK) return rc;
    }
  }
  int64_t max_pool = policy->max_pool > 0 ? policy->max_pool : device_threads;
  if (fixed > 0) max_pool = std::max(max_pool, fixed);
  if (max_pool > (int64_t(1) << 26)) return FSP_EUNSUPPORTED;

  // initial upper bound; the learned features are scaled by the NEH makespan
  std::vector<uint8_t> perm_neh(n);
  const int32_t neh = (int32_t)neh_host(inst->p_host, n, inst->m, perm_neh);
  std::vector<uint8_t> perm0(n);
  int32_t ub0;
  if (ub_in > 0) {
    ub0 = ub_in;
    for (int j = 0; j < n; ++j) perm0[j] = (uint8_t)j;
  } else {
    ub0 = neh;
    perm0 = perm_neh;
  }

  BnbState S;
  int rc = S.init(inst, max_pool, policy->prune_rule);
  S.prefilter = policy->prefilter == 1 ? 1 : 0;
  if (rc == FSP_OK && policy->bound_choice != 0) {
    if (hipMalloc(&S.lb1_mask, sizeof(lb1_mask)) != hipSuccess ||
        hipMemcpy(S.lb1_mask, lb1_mask, sizeof(lb1_mask), hipMemcpyHostToDevice) != hipSuccess)
      rc = FSP_ENOMEM;
  }
  if (rc == FSP_OK && depth_stats) {
    if (hipMalloc(&S.depth_stats, 768 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(S.depth_stats, 0, 768 * sizeof(uint32_t)) != hipSuccess)
      rc = FSP_ENOMEM;
  }
  // the batched kinds fill each pool from several depths, deepest first; the
  // paper's adaptive kind and fixed pools take one depth per pool
  S.multi = kind == FSP_POOL_AUTOTUNED || kind == FSP_POOL_LEARNED ? 1 : 0;
  if (rc == FSP_OK && model) rc = S.init_model(model, 1.0f / (float)neh);
  if (rc == FSP_OK && samples) rc = S.init_log(samples->cap, samples->prob, samples->seed);
  if (rc == FSP_OK) rc = S.start(ub0, perm0);
  const int nb_iter = policy->nb_iterations > 0 ? policy->nb_iterations : 10;
  const bool graphed = kind == FSP_POOL_AUTOTUNED || kind == FSP_POOL_LEARNED;
  if (rc == FSP_OK && graphed) rc = S.capture(nb_iter);
  if (rc != FSP_OK) {
    S.release();
    return rc;
  }

  AdaptivePolicy ap;
  ap.init(256, cus, device_threads, max_pool);
  // hybrid: host threads take nodes with at most kHostLeft unscheduled jobs
  // from the deepest bucket whenever they are idle (between two batches),
  // kHostChunk per thread, and search their subtrees on the CPU
  constexpr int kHostLeft = 6, kHostChunk = 64;
  const int host_threads = policy->host_threads;
  HostSearch hs;
  std::vector<int32_t> hcount(n);
  std::vector<uint8_t> hrec;
  std::vector<int32_t> hlb;
  if (host_threads > 0) hs.start(inst, host_threads, policy->prune_rule, ub0, t_start);
  FILE *log = policy->log_path ? std::fopen(policy->log_path, "w") : nullptr;

  int status = 0;
  double t_found = 0.0;
  int64_t last_bounded = 1;
  int64_t target = 0;
  // The learned kind's pool size: while the network estimates that some
  // pending node may still complete below UB, the search dives with small
  // pools of the best-estimated nodes (a sixteenth of the tuned size: on the
  // held-out 20x10 instances a quarter, a sixteenth and a sixty-fourth gave
  // 0.022, 0.020 and 0.021 s geometric-mean proof times, the tuned size
  // 0.031 s); once its smallest pending estimate reaches UB, the search is a
  // proof, where order does not matter: pools of the largest size the
  // buffers hold, without the network.  A batch that does not improve UB
  // doubles the dive pool (up to that largest size; an improvement resets
  // it), so a network whose estimates stay below UB still reaches large
  // pools.
  //
  // The switch to proof pools trusts the network's estimates only on
  // instances of at most as many jobs as it was trained on: beyond them its
  // estimates are extrapolations (on 200-job instances, with a network
  // trained on 50-job ones, they never fell below UB, so the search proved
  // from the start and never dived), and the search keeps diving.
  const int64_t dive_pool = std::max<int64_t>(1, fixed / 16);
  int64_t dive = dive_pool;
  bool proof = false;
  const bool trust_estimates =
      model && (model_trained_jobs(model) == 0 || inst->n <= model_trained_jobs(model));
  const double t_loop0 = elapsed();
  while (true) {
    target = kind == FSP_POOL_ADAPTIVE ? ap.current
             : !model                    ? fixed
             : proof                     ? max_pool
                                         : dive;
    if ((rc = S.set_target(target)) != FSP_OK) break;
    const double t0 = elapsed();
    if (graphed) {
      rc = S.replay(proof);
    } else {
      for (int it = 0; it < nb_iter && rc == FSP_OK; ++it) rc = S.enqueue_iteration(S.stream);
    }
    if (rc != FSP_OK) break;
    if ((rc = S.read_desc()) != FSP_OK) break;
    const double t1 = elapsed();
    const BnbDesc &h = *S.host_desc;
    const int64_t batch_nodes = h.nodes_bounded - last_bounded;
    last_bounded = h.nodes_bounded;
    if (window && t0 >= t_loop0 + window->skip * (policy->time_limit_s - t_loop0)) {
      window->nodes += batch_nodes;
      window->secs += t1 - t0;
      window->batches += 1;
    }
    if (h.improved) t_found = t1;
    const double eff = t1 > t0 ? (double)batch_nodes / (t1 - t0) : 0.0;
    if (log)
      std::fprintf(log,
                   "{\"t\": %.6f, \"pool_target\": %lld, \"nodes_bounded\": %lld, "
                   "\"batch_nodes\": %lld, \"eff\": %.17g, \"ub\": %d, \"pools\": %lld, "
                   "\"done\": %d, \"proof\": %d}\n",
                   t1, (long long)target, (long long)h.nodes_bounded,
                   (long long)batch_nodes, eff, h.ub, (long long)h.pools, h.done,
                   proof ? 1 : 0);
    if (h.overflow) {
      rc = FSP_ENOMEM;
      break;
    }
    if (host_threads > 0 && (rc = hybrid_exchange(S, hs, h, host_threads, kHostLeft,
                                                   kHostChunk, hcount, hrec, hlb)) != FSP_OK)
      break;
    if (h.done) break;
    const bool stretch = window && window->batches < window->min_batches &&
                         t1 < window->max_s;
    if (policy->time_limit_s > 0 && t1 >= policy->time_limit_s && !stretch) {
      status = 1;
      break;
    }
    if (kind == FSP_POOL_ADAPTIVE && t1 > t0) ap.observe(eff);
    if (model && !proof) {
      if (trust_estimates) {
        // estimates are completions in units of the NEH makespan
        float me = 0.f;
        if ((rc = S.pending_min_estimate(&me)) != FSP_OK) break;
        if ((double)me * (double)neh >= (double)h.ub) {
          proof = true;
          if ((rc = S.capture_plain(nb_iter)) != FSP_OK) break;
        }
      }
      dive = h.improved ? dive_pool : std::min<int64_t>(max_pool, 2 * dive);
    }
    // clear the "improved" flag for the next batch
    if (h.improved &&
        hipMemsetAsync(&S.desc->improved, 0, sizeof(int32_t), S.stream) != hipSuccess) {
      rc = FSP_EDEVICE;
      break;
    }
  }
  if (host_threads > 0) {
    // the device is done (or out of time): let the host finish its subtrees
    // (each has at most kHostLeft unscheduled jobs), unless out of time
    if (rc == FSP_OK && status == 0) hs.wait_idle();
    hs.stop_threads();
  }
  const double t_loop = elapsed() - t_loop0;
  if (rc == FSP_OK) rc = S.commit();
  int32_t open_lb = -1;
  if (rc == FSP_OK && status == 1) {
    // smallest bound among the pending nodes (pool_lb[0] as the scratch cell)
    const int32_t big = 0x7fffffff;
    if (hipMemcpyAsync(S.pool_lb, &big, sizeof(int32_t), hipMemcpyHostToDevice, S.stream) !=
        hipSuccess)
      rc = FSP_EDEVICE;
    if (rc == FSP_OK) {
      hipLaunchKernelGGL(open_lb_kernel, dim3(S.grid), dim3(256), 0, S.stream, S.blb, S.bcount,
                         n, S.cap, S.pool_lb);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(&open_lb, S.pool_lb, sizeof(int32_t), hipMemcpyDeviceToHost,
                         S.stream) != hipSuccess)
        rc = FSP_EDEVICE;
    }
  }
  if (rc == FSP_OK) rc = S.read_desc();
  if (log) std::fclose(log);
  if (rc == FSP_OK && samples) {
    const BnbDesc &h = *S.host_desc;
    const int64_t got = std::min<int64_t>(h.log_count, samples->cap);
    rc = policy_features(inst, S.log_nodes, S.log_lb, got, S.stride, 1.0f / (float)neh,
                         samples->x, S.stream);
    if (rc == FSP_OK)
      rc = policy_label(inst, S.log_nodes, S.log_lb, got, S.stride, h.ub, 1.0f / (float)neh,
                        samples->target, S.stream);
    if (rc == FSP_OK && hipStreamSynchronize(S.stream) != hipSuccess) rc = FSP_EDEVICE;
    *samples->n_out = got;
  }
  if (rc != FSP_OK) {
    S.release();
    return rc;
  }
  const BnbDesc &h = *S.host_desc;
  if (h.improved) t_found = elapsed();
  std::vector<uint8_t> perm(256);
  if (hipMemcpy(perm.data(), S.best_perm, 256, hipMemcpyDeviceToHost) != hipSuccess) {
    S.release();
    return FSP_EDEVICE;
  }
  std::memset(out, 0, sizeof(*out));
  out->perm = user_perm;
  out->makespan = h.ub;
  out->found = h.found;
  if (user_perm) std::copy(perm.begin(), perm.begin() + n, user_perm);
  out->status = status;
  out->root_lb = h.root_lb;
  out->nodes_bounded = h.nodes_bounded;
  out->nodes_branched = h.nodes_branched;
  out->nodes_pruned = h.nodes_pruned;
  out->leaves = h.leaves;
  out->pools = h.pools;
  out->t_found_s = h.found ? t_found : 0.0;
  out->t_total_s = elapsed();
  out->final_pool = target;
  out->t_search_s = t_loop;
  // lower bound on the optimum: the smallest pending bound, or the UB when
  // nothing is pending (the tree is exhausted)
  out->open_lb = status == 1 && open_lb != 0x7fffffff && open_lb >= 0
                     ? std::min<int32_t>(open_lb, h.ub)
                     : h.ub;
  out->proof_pools = proof ? 1 : 0;
  if (host_threads > 0) {
    out->nodes_bounded += hs.total.bounded;
    out->nodes_branched += hs.total.branched;
    out->nodes_pruned += hs.total.pruned;
    out->leaves += hs.total.leaves;
    out->host_nodes = hs.total.bounded;
    if (hs.best < INT32_MAX && hs.best <= out->makespan) {
      // the best schedule was found by a host thread (a device leaf can only
      // replace UB when strictly better)
      out->makespan = hs.best;
      out->found = hs.best < ub0 ? 1 : out->found;
      if (user_perm) std::copy(hs.best_perm, hs.best_perm + n, user_perm);
      out->t_found_s = hs.t_found;
    }
    if (status == 1) out->open_lb = std::min(out->open_lb, std::min(hs.open_lb(), out->makespan));
  }
  if (depth_stats) {
    depth_stats->assign(768, 0u);
    if (hipMemcpy(depth_stats->data(), S.depth_stats, 768 * sizeof(uint32_t),
                  hipMemcpyDeviceToHost) != hipSuccess) {
      S.release();
      return FSP_EDEVICE;
    }
  }
  S.release();
  return FSP_OK;
}

}  // namespace

extern "C" {

int fsp_neh(const fsp_instance *inst, uint8_t *perm_out, int32_t *makespan_out) {
  if (!inst) return FSP_EINVAL;
  std::vector<uint8_t> perm;
  const int64_t c = neh_host(inst->p_host, inst->n, inst->m, perm);
  if (perm_out) std::copy(perm.begin(), perm.end(), perm_out);
  if (makespan_out) *makespan_out = (int32_t)c;
  return FSP_OK;
}

int fsp_adaptive_schedule(int32_t threads_per_block, int32_t cus, int64_t max_threads,
                          int64_t max_pool, const double *efficiency, int32_t batches,
                          int64_t *targets_out) {
  if (threads_per_block < 1 || cus < 1 || max_threads < 1 || batches < 0 ||
      (batches > 0 && (!efficiency || !targets_out)))
    return FSP_EINVAL;
  AdaptivePolicy ap;
  ap.init(threads_per_block, cus, max_threads, max_pool > 0 ? max_pool : max_threads);
  for (int32_t i = 0; i < batches; ++i) {
    targets_out[i] = ap.current;
    ap.observe(efficiency[i]);
  }
  return FSP_OK;
}

int fsp_branch_and_bound(const fsp_instance *inst, const fsp_pool_policy *policy,
                         int32_t ub_in, fsp_result *out) {
  return run_bnb(inst, policy, ub_in, out, nullptr);
}

int fsp_policy_samples(const fsp_instance *inst, const fsp_pool_policy *policy, int32_t ub_in,
                       int64_t max_samples, double sample_prob, uint64_t seed, void *x_out,
                       float *target_out, int64_t *n_out, fsp_result *result) {
  if (!inst || !policy || !x_out || !target_out || !n_out || !result || max_samples < 1)
    return FSP_EINVAL;
  if (policy->kind == FSP_POOL_LEARNED) return FSP_EINVAL;
  SampleSpec s{max_samples, sample_prob, seed, x_out, target_out, n_out};
  *n_out = 0;
  return run_bnb(inst, policy, ub_in, result, &s);
}

int fsp_bound_choice_rule(int32_t n, const uint32_t *total, const uint32_t *elim1,
                          const uint32_t *elim2, uint32_t *mask_out) {
  if (n < 1 || n > kMaxJobs || !total || !elim1 || !elim2 || !mask_out) return FSP_EINVAL;
  std::fill(mask_out, mask_out + 8, 0u);
  // deepest first: depth d takes the one-machine bound when the nodes that
  // only the pair bound eliminates there, each branched into n - d children
  // bounded at the next depth, cost at most half the pair walks it saves, and
  // the next depth keeps the pair bound (so those children are eliminated
  // there: the pair bound never decreases along a branch)
  bool next_lb1 = false;
  for (int d = n - 1; d >= 1; --d) {
    const double t = total[d];
    const double extra = elim2[d] > elim1[d] ? (double)(elim2[d] - elim1[d]) : 0.0;
    const bool lb1 = t > 0 && !next_lb1 && extra * (double)(n - d) <= 0.5 * t;
    if (lb1) mask_out[d >> 5] |= 1u << (d & 31);
    next_lb1 = lb1;
  }
  return FSP_OK;
}

int fsp_autotune_bounds(const fsp_instance *inst, double budget_s, uint32_t *mask_out) {
  if (!inst || !mask_out) return FSP_EINVAL;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const BoundTuneEntry &e : g_bound_tune)
      if (e.dev == dev && e.n == inst->n && e.m == inst->m) {
        std::copy(e.mask, e.mask + 8, mask_out);
        return FSP_OK;
      }
  }
  // a short search from NEH with the pair bound at every depth, counting per
  // depth how many bounded nodes each bound eliminates against the UB of
  // the moment
  fsp_pool_policy pol{};
  pol.kind = FSP_POOL_AUTOTUNED;
  pol.nb_iterations = 10;
  pol.time_limit_s = budget_s > 0 ? budget_s : 1.0;
  pol.prune_rule = FSP_PRUNE_GE;
  fsp_result r{};
  std::vector<uint32_t> st;
  int rc = run_bnb(inst, &pol, 0, &r, nullptr, nullptr, &st);
  if (rc != FSP_OK) return rc;
  uint32_t mask[8];
  rc = fsp_bound_choice_rule(inst->n, st.data(), st.data() + 256, st.data() + 512, mask);
  if (rc != FSP_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    BoundTuneEntry e{dev, inst->n, inst->m, {}};
    std::copy(mask, mask + 8, e.mask);
    g_bound_tune.push_back(e);
  }
  std::copy(mask, mask + 8, mask_out);
  return FSP_OK;
}

int fsp_depth_stats(const fsp_instance *inst, const fsp_pool_policy *policy, int32_t ub_in,
                    uint32_t *stats_out, fsp_result *result) {
  if (!inst || !policy || !stats_out || !result) return FSP_EINVAL;
  if (policy->bound_choice != 0) return FSP_EINVAL;  // counts need the pair bound everywhere
  std::vector<uint32_t> st;
  const int rc = run_bnb(inst, policy, ub_in, result, nullptr, nullptr, &st);
  if (rc != FSP_OK) return rc;
  std::copy(st.begin(), st.end(), stats_out);
  return FSP_OK;
}

int fsp_autotune_pool(const fsp_instance *inst, double budget_s, int64_t *pool_out,
                      double *rate_out) {
  if (!inst || !pool_out) return FSP_EINVAL;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry &e : g_tune)
      if (e.dev == dev && e.n == inst->n && e.m == inst->m) {
        *pool_out = e.pool;
        if (rate_out) *rate_out = e.rate;
        return FSP_OK;
      }
  }
  int cus = 0, max_tpm = 0;
  FSP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  FSP_HIP_TRY(hipDeviceGetAttribute(&max_tpm, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev));
  const int64_t top = std::min<int64_t>((int64_t)cus * max_tpm, int64_t(1) << 20);
  std::vector<int64_t> cand;
  for (int64_t c = int64_t(1) << 14; c <= top; c <<= 1) cand.push_back(c);
  if (budget_s <= 0) budget_s = 0.25 * (double)cand.size();
  const double slice = budget_s / (double)cand.size();
  int64_t best = cand.front();
  double best_rate = -1.0;
  for (int64_t c : cand) {
    fsp_pool_policy pol{};
    pol.kind = FSP_POOL_AUTOTUNED;
    pol.fixed_pool = c;
    pol.nb_iterations = 10;
    pol.max_pool = c;
    pol.time_limit_s = slice;
    pol.prune_rule = FSP_PRUNE_GE;
    fsp_result r{};
    RateWindow win{1.0 / 3.0, 6, 8.0 * slice};
    const int rc = run_bnb(inst, &pol, 0, &r, nullptr, &win);
    if (rc != FSP_OK) return rc;
    // steady-state rate; a search that ends before the window counts whole
    const double rate = win.secs > 0 ? (double)win.nodes / win.secs
                        : r.t_search_s > 0 ? (double)r.nodes_bounded / r.t_search_s
                                           : 0.0;
    // candidates come in increasing size; a larger pool is taken unless it
    // is more than 3 % slower (short searches from the root understate
    // large pools, whose first batches fill slowest).  The reported rate is
    // the best measured.
    if (rate >= best_rate * 0.97) {
      best = c;
      best_rate = std::max(best_rate, rate);
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.push_back({dev, inst->n, inst->m, best, best_rate});
  }
  *pool_out = best;
  if (rate_out) *rate_out = best_rate;
  return FSP_OK;
}

}  // extern "C"
