// fsp_internal.hpp -- internal declarations shared by the libfsp sources.
//
// Device data of an instance (all int32, row = job, padded machine stride MP):
//   p   [n][MP]  processing times
//   H   [n][MP]  H[j][k] = sum_{h<k} p[j][h]    (work before machine k)
//   Q   [n][MP]  Q[j][k] = sum_{h>k} p[j][h]    (work after machine k)
//   Hp, Qp [n][MP/2]  H and Q as 16-bit pairs (machines 2t, 2t+1)
//   tot [MP]     tot[k]  = sum_j p[j][k]
//   rec [P][npad] per machine pair (lexicographic k<l), the jobs in Johnson
//                 order with lags, one record per position, padded to npad
//                 positions with neutral records (see bound.hip for the
//                 record encoding and why padding is neutral).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fsp.h"

namespace fspi {

constexpr int kMaxJobs = 255;   // a job id is one byte
constexpr int kMaxMachines = 20;  // largest instantiated machine count
constexpr int kBlock = 256;       // threads per workgroup of the pool kernels
constexpr int kLogBlock = 8;

// Table records, one per (machine pair, position in the pair's Johnson order):
//   x = 256 * (b - a)            (signed, |.| < 2^23)
//   y = ((lag + b) << 8) | job   (unsigned, < 2^24; job < 256)
// with a = p[job][k], b = p[job][l], lag = sum_{k<h<l} p[job][h].  A second
// table [P][npad] holds 8 * job of every position (the byte offset of the
// job's mask in a wave's mask slot); padding positions have x = y = 0 and
// offset 8 * n.
using Rec = int2;

// Bytes of one wave's job-mask slot in the bounding scratch (n > 64): one
// 64-bit lane mask per job id 0..n (n = the padding id), rounded up to 256
// bytes so that no two slots share a cache line.
inline int mask_slot_bytes(int n) { return ((n + 1) * 8 + 255) / 256 * 256; }

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

// Bytes of the mask-offset table: [P][npad] plus one group of four entries
// that the walk may request (and not use) past the last pair.
inline size_t joff_bytes(int P, int npad) { return ((size_t)P * npad + 4) * sizeof(uint32_t); }
// Entries of the bytes walk's tables: [P][npad8] plus two groups of eight
// past the last pair that the walk may request (and not use).
inline size_t bytes_entries(int P, int npad8) { return (size_t)P * npad8 + 16; }
inline int npairs(int m) { return m * (m - 1) / 2; }
// Words of the packed job table: [P][npad] plus one group of eight that the
// walk may request (and not use) past the last pair.
inline size_t p16_job_words(int P, int npad) { return (size_t)P * npad + 8; }

}  // namespace fspi

struct fsp_instance {
  int n = 0, m = 0, mp = 0, P = 0, npad = 0;
  int wide = 0;    // 1 when n > 32 (job sets of more than one word)
  int device = 0;
  int32_t *d_p = nullptr, *d_H = nullptr, *d_Q = nullptr, *d_tot = nullptr;
  uint32_t *d_Hp = nullptr, *d_Qp = nullptr;  // H, Q as packed 16-bit pairs
  fspi::Rec *d_rec = nullptr;  // [P][npad]
  // Packed 16-bit tables for two nodes per lane (p16 = 1: n <= 32 and total
  // work <= 32767, so every quantity of the bound fits in 16 bits), one
  // 32-bit word per table position, couples of pairs interleaved:
  //   xy16  x | y << 16 with x = b - a, y = lag + b   (staged in LDS)
  //   job16 the position's job id                    (read by scalar loads;
  //         p16_job_words(P, npad) words: one spare group past the end)
  int p16 = 0;
  uint32_t *d_xy16 = nullptr;
  uint32_t *d_job16 = nullptr;
  uint32_t *d_joff = nullptr;  // [P][npad] 8 * job id per table position
  // n > 64: 1 when loaded with FSP_LOAD_JOB_MASKS (the job-mask walk, with
  // its per-wave scratch), 0 for the bytes walk
  int masks_walk = 0;
  // The bytes walk's tables (n > 64), [P][npad8] with npad8 = n rounded up
  // to 8, read by scalar loads (bytes_entries(P, npad8) entries each):
  //   bxy   x | y << 16 with x = b - a (two's complement), y = lag + b; both
  //         fit in 16 bits because p <= 32767 and every job total <= 65535
  //   bjob  the position's job id (padding: n)
  int npad8 = 0;
  uint32_t *d_bxy = nullptr;
  uint8_t *d_bjob = nullptr;
  std::vector<int32_t> p_host;  // [n][m], for host-side set-up work (NEH)
};


// Status helpers
#define FSP_HIP_TRY(expr)                          \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return FSP_EDEVICE;      \
  } while (0)

namespace fspi {
// Device scratch that one bounding launch of `count` nodes of an n-job
// instance needs: for n > 64 (the job-mask walk), one mask slot per wave of
// every tile; none up to 64 jobs (the job set of a node is a register there).
inline bool uses_job_masks(int n) { return n > 64; }
inline size_t bound_scratch_bytes(int n, int64_t count) {
  if (!uses_job_masks(n)) return 0;
  const int64_t tiles = (count + kBlock - 1) / kBlock;
  return (size_t)tiles * (kBlock / 64) * (size_t)mask_slot_bytes(n);
}
// Whether bounding this instance takes the job-mask walk, and the scratch
// that walk needs for a pool of `count` nodes (0 for every other walk).
inline bool takes_mask_walk(const fsp_instance *in) {
  return uses_job_masks(in->n) && in->masks_walk != 0;
}
inline size_t walk_scratch_bytes(const fsp_instance *in, int64_t count) {
  return takes_mask_walk(in) ? bound_scratch_bytes(in->n, count) : 0;
}

// Launches the pool-bounding kernel (bound.hip).  Validates nothing: the
// caller has checked every argument.  With count_dev set, the kernel reads
// the node count from device memory when it starts (at most `count`, which
// sizes the grid).  scratch holds at least bound_scratch_bytes(n, count)
// bytes and is used by no other work running at the same time; null takes
// the workspace that the library keeps for the stream (allocated or grown on
// first need, which synchronises the stream).
// One-machine pre-filter of a bounding launch.  With ub set, a wave whose
// live nodes all have a one-machine bound that the rule eliminates against
// *ub skips the pair walks and reports those bounds (the eliminations are
// the same: the pair bound is never smaller).  lb1_only: every node gets
// its one-machine bound.  lb1_depths (device, 8 words): a node whose depth's
// bit is set gets its one-machine bound (the other bound of the choice per
// depth); a wave whose nodes all have it skips the pair walks.
// depth_stats (device, [3][256] words, measurement): per depth of the
// bounded nodes with jobs left, the count of such nodes, of those the
// one-machine bound eliminates against *ub, and of those the pair bound
// eliminates; the pre-filter's skipping is off while measuring.
struct Prefilter {
  const int32_t *ub = nullptr;  // device pointer, read when the kernel starts
  int rule = 0;                 // FSP_PRUNE_GE or FSP_PRUNE_GT
  int lb1_only = 0;
  const uint32_t *lb1_depths = nullptr;
  uint32_t *depth_stats = nullptr;
};

int launch_bound(const fsp_instance *inst, const uint8_t *nodes, int stride,
                 int64_t count, int32_t *lb_out, hipStream_t stream,
                 const int32_t *count_dev, void *scratch,
                 const Prefilter &pf = Prefilter());

// The library's per-stream bounding workspace of at least `bytes` bytes.
int stream_scratch(hipStream_t stream, size_t bytes, void **out);
}  // namespace fspi
