/*
 * fsp.h -- C ABI of libfsp: parallel bounding for permutation flow-shop
 * branch-and-bound on AMD Instinct MI355X (gfx950).
 *
 * Problem (Chakroun & Melab, Sec. II.B): n jobs, m machines, every job visits
 * machines 0..m-1 in order, p[j][k] is the processing time of job j on
 * machine k, each machine runs one job at a time, and every machine processes
 * the jobs in the same order (a permutation schedule).  The objective is the
 * makespan.  A search-tree node is a scheduled prefix (Sec. II.B: node i
 * schedules job i first; its sons append one more job).
 *
 * The bound (Sec. V.D gives only its cost, O(m^2 n log n)): for every machine
 * pair (k,l), k<l, the two-machine relaxation in which the machines between k
 * and l become per-job delays (lags) is solved exactly by Johnson's rule on
 * the lag-shifted times; each pair starts from the earliest availability of
 * its machines (heads) and adds the least work any unscheduled job still has
 * after machine l (tail).  The bound is the maximum over pairs.  A node with
 * no unscheduled job bounds to its makespan.
 *
 * Conventions for every function:
 *   - return FSP_OK (0) or a negative status; nothing throws;
 *   - argument errors are detected before any device work is queued;
 *   - "device pointer" means memory of the device that was current when the
 *     instance was loaded (e.g. a torch CUDA tensor's data_ptr());
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream);
 *     asynchronous calls return once the work is queued, the caller keeps the
 *     buffers alive until the stream has finished it, and a device fault
 *     surfaces at the caller's next synchronisation;
 *   - an fsp_instance is immutable after loading and may be used from several
 *     streams at once; distinct objects may be used from distinct threads.
 */
#ifndef FSP_H
#define FSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define FSP_OK 0
#define FSP_EINVAL (-1)       /* bad argument (null pointer, size, range)   */
#define FSP_ENOMEM (-2)       /* device or host allocation failed           */
#define FSP_EDEVICE (-3)      /* a HIP call failed                          */
#define FSP_EUNSUPPORTED (-4) /* valid input outside what this build serves */

/* Bound written for a malformed node: depth > n, a job id >= n, or a job
 * scheduled twice. */
#define FSP_LB_INVALID (-1)

/* Human-readable text for a status code (static storage). */
const char *fsp_status_string(int32_t status);

/* ---- instances --------------------------------------------------------- */
typedef struct fsp_instance fsp_instance;

/*
 * fsp_load_instance -- copy an instance to the current device and build its
 * per-instance tables there (Sec. II.B problem data; the tables are the
 * per-pair Johnson orders with lags, the head/tail sums and the column
 * totals the bound needs).  Synchronous.
 *   p_host : HOST int32 [n][m], row-major (row = job); copied, the caller may
 *            free it on return.
 *   n      : 1 <= n <= 255 jobs (a job id is one byte).
 *   m      : 2 <= m <= 20 machines (a pair needs two machines; 20 is the
 *            largest machine count this build instantiates: FSP_EUNSUPPORTED
 *            above it).
 *   out    : receives the handle; release it with fsp_free_instance.
 * Limits (FSP_EUNSUPPORTED otherwise): every p[j][k] in [0, 32767], every
 * job's total time <= 65535, the sum of all times < 2^22.  Negative times are
 * FSP_EINVAL.
 */
int fsp_load_instance(const int32_t *p_host, int32_t n, int32_t m,
                      fsp_instance **out);

/* Release the instance and its device tables (NULL is a no-op).  The caller
 * must have finished all stream work that uses it. */
int fsp_free_instance(fsp_instance *inst);

/* n, m and the device the instance lives on (any pointer may be NULL). */
int fsp_instance_info(const fsp_instance *inst, int32_t *n, int32_t *m,
                      int32_t *device);

/* ---- pool bounding (Sec. III: one launch bounds a whole pool) --------- */

/* A pool of nodes in device memory.  Record i starts at data + i*stride:
 * byte 0 = depth d (number of scheduled jobs), bytes 1..d = the prefix (job
 * ids in schedule order), remaining bytes ignored.  stride >= n+1.  Records
 * 16-byte aligned (data and stride multiples of 16) take the fast load path;
 * any other layout is accepted and read byte by byte. */
typedef struct {
  const fsp_instance *inst;
  const uint8_t *data; /* device pointer */
  int32_t stride;
} fsp_nodes;

/*
 * fsp_bound_pool -- lb_out[i] = bound of record i, for i in [0, count)
 * (Sec. III: every sub-problem of the off-loaded pool is bounded
 * independently; Sec. V.D bound).  lb_out is a device int32[count].  Malformed
 * records get FSP_LB_INVALID.  count == 0 queues nothing.  Asynchronous on
 * `stream`.
 */
int fsp_bound_pool(const fsp_nodes *nodes, int64_t count, int32_t *lb_out,
                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FSP_H */
