// policy.hip -- device side of the learned pool policy.
//
// The policy network (mlp.hip) scores pending nodes; the scores only decide
// which nodes of the deepest depth are branched first (and so how soon good
// schedules, hence a low UB, are found).  The exact integer bound still
// decides every elimination, so the optimum is untouched.
//
//   features   node record -> x in R^32 (bf16): depth / n, bound / scale,
//              and for up to 15 machines the prefix completion time and the
//              remaining work, / scale (scale = the initial UB).  2m+2
//              features for m <= 15 machines; above, 15 evenly spaced
//              machines.
//   score      est = bound / scale + y0 (y0: predicted completion gap): the
//              estimated best completion; smaller is more promising.
//   selection  when the plan takes K < count nodes of a depth, the K nodes
//              with the smallest est are moved to the top of the bucket
//              (histogram of est, threshold, partition through a scratch
//              buffer).  All sizes come from the device descriptor, so the
//              kernels are captured with the rest of the iteration.
//   samples    the prune step logs a deterministic pseudo-random sample of
//              the surviving children (training data); labels come from a
//              suffix-NEH completion of each logged node (y0 target) and
//              from whether its bound reaches the final UB (y1 target).
#include <hip/hip_runtime.h>

#include <utility>

#include "bnb.hpp"
#include "fsp_internal.hpp"

namespace fspi {

namespace {

constexpr int kFeat = 32;
constexpr int kMaxFeatMachines = 15;

__device__ __forceinline__ int feat_machine(int t, int m, int mm) {
  return mm == m ? t : (t * (m - 1) + (mm - 1) / 2) / (mm - 1);
}

}  // namespace

// ---- features --------------------------------------------------------------
// Features of one node record (16-byte aligned, prefix of depth d), written
// as 32 bf16 values.  M (the machine count) is a template parameter so that
// the per-machine values stay in registers.
template <int M>
__device__ __forceinline__ void node_features(const uint8_t *rec, int lb,
                                              const int32_t *__restrict__ p,
                                              const int32_t *__restrict__ tot, int n,
                                              int mp, float inv_scale, __bf16 *x) {
  constexpr int mm = M < kMaxFeatMachines ? M : kMaxFeatMachines;
  int F[M], S[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    F[k] = 0;
    S[k] = tot[k];
  }
  const uint4 *rc = reinterpret_cast<const uint4 *>(rec);
  const int d = rec[0];
  for (int c = 0; 16 * c <= d; ++c) {
    const uint4 v = rc[c];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int at = 16 * c + b;
      if (at >= 1 && at <= d) {
        const int j = (int)((w[b >> 2] >> (8 * (b & 3))) & 0xffu);
        const int32_t *row = p + j * mp;
        F[0] += row[0];
        S[0] -= row[0];
#pragma unroll
        for (int k = 1; k < M; ++k) {
          F[k] = max(F[k], F[k - 1]) + row[k];
          S[k] -= row[k];
        }
      }
    }
  }
  float f[kFeat];
#pragma unroll
  for (int t = 0; t < kFeat; ++t) f[t] = 0.f;
  f[0] = (float)d / (float)n;
  f[1] = (float)lb * inv_scale;
#pragma unroll
  for (int t = 0; t < mm; ++t) {
    const int k = feat_machine(t, M, mm);
    f[2 + t] = (float)F[k] * inv_scale;
    f[2 + mm + t] = (float)S[k] * inv_scale;
  }
  uint4 *xo = reinterpret_cast<uint4 *>(x);
#pragma unroll
  for (int q = 0; q < kFeat / 8; ++q) {
    uint32_t h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const __bf16 lo = (__bf16)f[8 * q + 2 * e], hi = (__bf16)f[8 * q + 2 * e + 1];
      h[e] = (uint32_t)__builtin_bit_cast(uint16_t, lo) |
             ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
    }
    xo[q] = make_uint4(h[0], h[1], h[2], h[3]);
  }
}

// features of the nodes that the last prune added: the buckets one below
// each depth segment of the pool (each was empty before that prune), rows
// in segment order; rowdst[r] is the bucket slot of row r
template <int M>
__global__ __launch_bounds__(256) void features_kernel(
    BnbDesc *D, const int32_t *__restrict__ bcount, const uint8_t *__restrict__ bnodes,
    const int32_t *__restrict__ blb, int64_t cap, int stride,
    const int32_t *__restrict__ p, const int32_t *__restrict__ tot, int n, int mp,
    float inv_scale, __bf16 *__restrict__ X, int64_t *__restrict__ rowdst) {
  const int nseg = D->active ? D->nseg : 0;
  int off[kMaxSeg + 1], dep[kMaxSeg];
  off[0] = 0;
#pragma unroll
  for (int s = 0; s < kMaxSeg; ++s) {
    const int d1 = s < nseg ? D->seg_depth[s] + 1 : n;
    dep[s] = d1;
    off[s + 1] = off[s] + (d1 < n ? bcount[d1] : 0);
  }
  const int count = off[kMaxSeg];
  if (blockIdx.x == 0 && threadIdx.x == 0) D->feat_count = count;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < count;
       r += gridDim.x * blockDim.x) {
    int s = 0;
#pragma unroll
    for (int t = 1; t < kMaxSeg; ++t)
      if (r >= off[t]) s = t;
    const int64_t at = (int64_t)dep[s] * cap + (r - off[s]);
    node_features<M>(bnodes + at * stride, blb[at], p, tot, n, mp, inv_scale,
                     X + (int64_t)r * kFeat);
    rowdst[r] = at;
  }
}

// features of an explicit list of nodes (training samples)
template <int M>
__global__ __launch_bounds__(256) void features_list_kernel(
    const uint8_t *__restrict__ nodes, const int32_t *__restrict__ lbs, int64_t count,
    int stride, const int32_t *__restrict__ p, const int32_t *__restrict__ tot, int n,
    int mp, float inv_scale, __bf16 *__restrict__ X) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    node_features<M>(nodes + i * stride, lbs[i], p, tot, n, mp, inv_scale, X + i * kFeat);
}

using FeatBucketFn = decltype(&features_kernel<2>);
using FeatListFn = decltype(&features_list_kernel<2>);

template <int... Ks>
FeatBucketFn bucket_fn(int m, std::integer_sequence<int, Ks...>) {
  constexpr FeatBucketFn table[] = {features_kernel<Ks + 2>...};
  return table[m - 2];
}

template <int... Ks>
FeatListFn list_fn(int m, std::integer_sequence<int, Ks...>) {
  constexpr FeatListFn table[] = {features_list_kernel<Ks + 2>...};
  return table[m - 2];
}

// ---- best-K selection ------------------------------------------------------
constexpr int kBins = kSelBins;
constexpr float kBinScale = 2048.f;  // est in [0, 2)

__device__ __forceinline__ int est_bin(float e) {
  const float b = e * kBinScale;
  return b <= 0.f ? 0 : (b >= (float)(kBins - 1) ? kBins - 1 : (int)b);
}

__device__ __forceinline__ bool sel_needed(const BnbDesc *D) {
  return D->active && D->parents < D->sel_count;
}

// Histogram of est over the bucket: each workgroup counts a block of at
// least kHistPerBlock entries in LDS, then adds its non-empty bins to the
// global histogram (scores crowd into few bins, which would serialise
// per-entry global atomics).
constexpr int kHistPerBlock = 4096;

__global__ __launch_bounds__(256) void sel_hist_kernel(const BnbDesc *D,
                                                       const float *__restrict__ bscore,
                                                       int64_t cap, int32_t *__restrict__ hist) {
  if (!sel_needed(D)) return;
  const int count = D->sel_count;
  const int nblk = min((int)gridDim.x, (count + kHistPerBlock - 1) / kHistPerBlock);
  if ((int)blockIdx.x >= nblk) return;
  __shared__ int sh[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) sh[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)D->depth * cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += nblk * blockDim.x)
    atomicAdd(&sh[est_bin(bscore[base + i])], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (sh[b]) atomicAdd(&hist[b], sh[b]);
}

// The bin T of the K-th smallest score and how many nodes of bin T the pool
// takes, from the histogram: each thread sums 16 bins, a block-wide scan of
// the sums finds the thread whose bins hold the K-th node, and that thread
// walks them.  Every workgroup of the partition computes it (same input, same
// result), which saves a launch.  Every thread of the workgroup calls it.
__device__ void sel_threshold(const int32_t *__restrict__ hist, int K, int &T, int &need) {
  __shared__ int part[256];
  __shared__ int s_T, s_need;
  constexpr int per = kBins / 256;
  const int t = threadIdx.x;
  int h[per];
  int sum = 0;
#pragma unroll
  for (int b = 0; b < per; ++b) {
    h[b] = hist[t * per + b];
    sum += h[b];
  }
  if (t == 0) {
    s_T = kBins - 1;
    s_need = K;
  }
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const int incl = part[t], excl = incl - sum;
  if (excl < K && incl >= K) {  // exactly one thread: the counts sum to >= K
    int cb = excl;
#pragma unroll
    for (int b = 0; b < per; ++b) {
      if (cb + h[b] >= K) {
        s_T = t * per + b;
        s_need = K - cb;
        break;
      }
      cb += h[b];
    }
  }
  __syncthreads();
  T = s_T;
  need = s_need;
}

// Partition of the depth by the threshold into the scratch buffers: the
// nodes that stay first, in slot order, then the K taken ones on top (the
// positions the plan gave to the pool).  The branch kernel reads the taken
// ones from there and writes the others back.
__global__ __launch_bounds__(256) void sel_partition_kernel(
    BnbDesc *D, const int32_t *__restrict__ hist, const uint8_t *__restrict__ bnodes,
    const int32_t *__restrict__ blb, const float *__restrict__ bscore, int64_t cap, int stride,
    uint8_t *__restrict__ tnodes, int32_t *__restrict__ tlb, float *__restrict__ tscore) {
  if (!sel_needed(D)) return;
  const int count = D->sel_count, K = D->parents;
  int T, need;
  sel_threshold(hist, K, T, need);
  const int64_t base = (int64_t)D->depth * cap;
  __shared__ int s_cnt[256 / 64 + 1];
  // uniform rounds: every thread takes part in the workgroup-level slots
  for (int r0 = blockIdx.x * blockDim.x; r0 < count; r0 += gridDim.x * blockDim.x) {
    const int i = r0 + threadIdx.x;
    const bool in = i < count;
    const float e = in ? bscore[base + i] : 0.f;
    const int b = est_bin(e);
    const bool tie = in && b == T;
    const int trank = block_slot(tie, &D->sel_tie, s_cnt);
    const bool take = in && (b < T || (tie && trank < need));
    const int hi = block_slot(take, &D->sel_hi, s_cnt);
    const int lo = block_slot(in && !take, &D->sel_lo, s_cnt);
    if (!in) continue;
    const int pos = take ? count - K + hi : lo;
    const uint4 *src = reinterpret_cast<const uint4 *>(bnodes + (base + i) * stride);
    uint4 *dst = reinterpret_cast<uint4 *>(tnodes + (int64_t)pos * stride);
    for (int q = 0; q < stride / 16; ++q) dst[q] = src[q];
    tlb[pos] = blb[base + i];
    tscore[pos] = e;
  }
}

// ---- training samples --------------------------------------------------------

// suffix-NEH completion of a node: the unscheduled jobs, by total work
// descending (ties by id), are inserted one by one at the position of the
// suffix giving the smallest makespan (earliest on ties); the prefix stays.
__global__ void label_kernel(const uint8_t *__restrict__ nodes, const int32_t *__restrict__ lbs,
                             int64_t count, int stride, const int32_t *__restrict__ p, int n,
                             int m, int mp, int32_t final_ub, float inv_scale,
                             float *__restrict__ target) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint8_t *rec = nodes + i * stride;
  const int d = rec[0];
  uint32_t used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int F[kMaxMachines];
  for (int k = 0; k < m; ++k) F[k] = 0;
  for (int q = 0; q < d; ++q) {
    const int j = rec[1 + q];
    used[j >> 5] |= 1u << (j & 31);
    const int32_t *row = p + j * mp;
    F[0] += row[0];
    for (int k = 1; k < m; ++k) F[k] = max(F[k], F[k - 1]) + row[k];
  }
  uint8_t seq[256];  // the suffix being built
  int len = 0;
  uint32_t taken[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int step = 0; step < n - d; ++step) {
    // next job: largest total work among the unscheduled, smallest id on ties
    int best_j = -1, best_w = -1;
    for (int j = 0; j < n; ++j) {
      if ((used[j >> 5] >> (j & 31)) & 1u) continue;
      if ((taken[j >> 5] >> (j & 31)) & 1u) continue;
      int w = 0;
      for (int k = 0; k < m; ++k) w += p[j * mp + k];
      if (w > best_w) {
        best_w = w;
        best_j = j;
      }
    }
    taken[best_j >> 5] |= 1u << (best_j & 31);
    int best_pos = 0, best_c = 0x7fffffff;
    for (int pos = 0; pos <= len; ++pos) {
      int c[kMaxMachines];
      for (int k = 0; k < m; ++k) c[k] = F[k];
      for (int q = 0; q <= len; ++q) {
        const int j = q < pos ? seq[q] : (q == pos ? best_j : seq[q - 1]);
        const int32_t *row = p + j * mp;
        c[0] += row[0];
        for (int k = 1; k < m; ++k) c[k] = max(c[k], c[k - 1]) + row[k];
      }
      if (c[m - 1] < best_c) {
        best_c = c[m - 1];
        best_pos = pos;
      }
    }
    for (int q = len; q > best_pos; --q) seq[q] = seq[q - 1];
    seq[best_pos] = (uint8_t)best_j;
    ++len;
  }
  int c_final;
  if (len == 0) {
    c_final = F[m - 1];
  } else {
    int c[kMaxMachines];
    for (int k = 0; k < m; ++k) c[k] = F[k];
    for (int q = 0; q < len; ++q) {
      const int32_t *row = p + seq[q] * mp;
      c[0] += row[0];
      for (int k = 1; k < m; ++k) c[k] = max(c[k], c[k - 1]) + row[k];
    }
    c_final = c[m - 1];
  }
  target[i * 2 + 0] = (float)(c_final - lbs[i]) * inv_scale;
  target[i * 2 + 1] = lbs[i] >= final_ub ? 1.f : 0.f;
}

// ---- host helpers ------------------------------------------------------------
int policy_enqueue_select(BnbState &S, hipStream_t s, int grid) {
  // the branch kernel that follows reads the taken nodes from the scratch,
  // writes the others back and clears the histogram and the slot counters
  hipLaunchKernelGGL(sel_hist_kernel, dim3(grid), dim3(256), 0, s, S.desc, S.bscore, S.cap,
                     S.hist);
  hipLaunchKernelGGL(sel_partition_kernel, dim3(grid), dim3(256), 0, s, S.desc, S.hist,
                     S.bnodes, S.blb, S.bscore, S.cap, S.stride, S.tnodes, S.tlb, S.tscore);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int policy_enqueue_score(BnbState &S, hipStream_t s, int grid) {
  const fsp_instance *in = S.inst;
  FeatBucketFn fn = bucket_fn(in->m, std::make_integer_sequence<int, kMaxMachines - 1>());
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, S.desc, S.bcount, S.bnodes, S.blb, S.cap,
                     S.stride, in->d_p, in->d_tot, in->n, in->mp, S.inv_scale,
                     reinterpret_cast<__bf16 *>(S.X), S.rowdst);
  FSP_HIP_TRY(hipGetLastError());
  // the forward pass writes est = bound / s + predicted gap itself
  const ScoreEpilogue sc{S.rowdst, S.blb, S.bscore, S.inv_scale};
  return model_forward_score_dev(S.model, S.X, &S.desc->feat_count, S.cap, sc, s);
}

int policy_features(const fsp_instance *in, const uint8_t *nodes, const int32_t *lbs,
                    int64_t count, int stride, float inv_scale, void *X, hipStream_t s);

int policy_label(const fsp_instance *in, const uint8_t *nodes, const int32_t *lbs,
                 int64_t count, int stride, int32_t final_ub, float inv_scale, float *target,
                 hipStream_t s) {
  if (count == 0) return FSP_OK;
  hipLaunchKernelGGL(label_kernel, dim3((unsigned)((count + 127) / 128)), dim3(128), 0, s,
                     nodes, lbs, count, stride, in->d_p, in->n, in->m, in->mp, final_ub,
                     inv_scale, target);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int policy_features(const fsp_instance *in, const uint8_t *nodes, const int32_t *lbs,
                    int64_t count, int stride, float inv_scale, void *X, hipStream_t s) {
  if (count == 0) return FSP_OK;
  FeatListFn fn = list_fn(in->m, std::make_integer_sequence<int, kMaxMachines - 1>());
  hipLaunchKernelGGL(fn, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, nodes, lbs,
                     count, stride, in->d_p, in->d_tot, in->n, in->mp, inv_scale,
                     reinterpret_cast<__bf16 *>(X));
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int policy_in_features(int m) {
  const int mm = m < kMaxFeatMachines ? m : kMaxFeatMachines;
  return 2 + 2 * mm;
}

}  // namespace fspi
