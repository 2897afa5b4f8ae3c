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

// Narrow records (n <= 32: one 32-bit job mask per node):
//   x = 256 * (b - a)            (signed, |.| < 2^23)
//   y = ((lag + b) << 8) | job   (unsigned, < 2^24)
// Wide records (n > 32) add the byte offset, in the kernels' [word][lane]
// LDS layout of the unscheduled-job masks, of the job's 32-job word:
//   {x, y, (job / 32) * 256 lanes * 4 bytes, 0}
// with a = p[job][k], b = p[job][l], lag = sum_{k<h<l} p[job][h].
using NarrowRec = int2;
using WideRec = int4;

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }
inline int npairs(int m) { return m * (m - 1) / 2; }

}  // namespace fspi

struct fsp_instance {
  int n = 0, m = 0, mp = 0, P = 0, npad = 0;
  int wide = 0;    // 1 when n > 32 (records carry the job id separately)
  int device = 0;
  int32_t *d_p = nullptr, *d_H = nullptr, *d_Q = nullptr, *d_tot = nullptr;
  uint32_t *d_Hp = nullptr, *d_Qp = nullptr;  // H, Q as packed 16-bit pairs
  void *d_rec = nullptr;    // NarrowRec or WideRec [P][npad]
  size_t rec_bytes = 0;
  std::vector<int32_t> p_host;  // [n][m], for host-side set-up work (NEH)
};

// Status helpers
#define FSP_HIP_TRY(expr)                          \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return FSP_EDEVICE;      \
  } while (0)

namespace fspi {
// Launches the pool-bounding kernel (bound.hip).  Validates nothing: the
// caller has checked every argument.  With count_dev set, the kernel reads
// the node count from device memory when it starts (at most `count`, which
// sizes the grid).
int launch_bound(const fsp_instance *inst, const uint8_t *nodes, int stride,
                 int64_t count, int32_t *lb_out, hipStream_t stream,
                 const int32_t *count_dev);
}  // namespace fspi
