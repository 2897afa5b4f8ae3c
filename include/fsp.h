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
#define FSP_EUNSUPPORTED (-4) /* valid input outside what this library serves */
#define FSP_ESCRATCH (-5)     /* pool beyond the fixed scratch of
                                 fsp_bound_pool_noalloc                     */

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
 *            largest machine count this library instantiates: FSP_EUNSUPPORTED
 *            above it).
 *   out    : receives the handle; release it with fsp_free_instance.
 * Limits (FSP_EUNSUPPORTED otherwise): every p[j][k] in [0, 32767], every
 * job's total time <= 65535, the sum of all times < 2^22.  Negative times are
 * FSP_EINVAL.
 */
int fsp_load_instance(const int32_t *p_host, int32_t n, int32_t m,
                      fsp_instance **out);

/* Load flags of fsp_load_instance_ex.  FSP_LOAD_ONE_NODE_PER_LANE keeps an
 * instance that would take the packed two-nodes-per-lane form (see
 * fsp_instance_path) on the one-node-per-lane 32-bit register form; the
 * bounds are identical, only the arithmetic differs (for comparing the two
 * forms on one pool).  FSP_LOAD_JOB_MASKS puts an instance of more than 64
 * jobs on the job-mask walk instead of the bytes walk (same bounds; the
 * job-mask walk needs per-wave scratch, see fsp_bound_pool_noalloc). */
#define FSP_LOAD_ONE_NODE_PER_LANE 1
#define FSP_LOAD_JOB_MASKS 2

/* fsp_load_instance with load flags (0 or FSP_LOAD_* or-ed together; any
 * other bit is FSP_EINVAL).  fsp_load_instance(p, n, m, out) is
 * fsp_load_instance_ex(p, n, m, 0, out). */
int fsp_load_instance_ex(const int32_t *p_host, int32_t n, int32_t m,
                         int32_t flags, fsp_instance **out);

/* Release the instance and its device tables (NULL is a no-op).  The caller
 * must have finished all stream work that uses it. */
int fsp_free_instance(fsp_instance *inst);

/* n, m and the device the instance lives on (any pointer may be NULL). */
int fsp_instance_info(const fsp_instance *inst, int32_t *n, int32_t *m,
                      int32_t *device);

/* Which form of the pool-bounding walk (Sec. V.D's bound; the forms give
 * identical bounds) fsp_bound_pool uses for this instance:
 *   FSP_PATH_REGISTER    n <= 32: one node per lane, the unscheduled set in a
 *                        register;
 *   FSP_PATH_PACKED      n <= 32 and total work <= 32767: two nodes per lane
 *                        in packed 16-bit arithmetic (every value of the bound
 *                        then fits in 16 bits);
 *   FSP_PATH_BYTES       n > 64: one node per lane, each lane's unscheduled
 *                        flags as bytes in LDS, the table by scalar loads;
 *   FSP_PATH_MASKS       n > 64 when loaded with FSP_LOAD_JOB_MASKS: one node
 *                        per lane, per-wave job masks read by scalar loads;
 *   FSP_PATH_REGISTER64  32 < n <= 64: one node per lane, the unscheduled set
 *                        in a 64-bit register pair.
 * A batch may take another allowed form per shape (fsp_batch_paths). */
enum { FSP_PATH_REGISTER = 0, FSP_PATH_PACKED = 1, FSP_PATH_MASKS = 2,
       FSP_PATH_REGISTER64 = 3, FSP_PATH_BYTES = 4 };
int fsp_instance_path(const fsp_instance *inst, int32_t *path);


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
 * For n > 64 the walk needs device scratch (about n/8 + 1 bytes per node):
 * the library keeps one workspace per (device, stream), and a call that needs
 * more than the stream's workspace holds first synchronizes the stream, then
 * replaces it (so such a call cannot be captured in a graph; a smaller or
 * equal pool on the same stream can).  Calls on one stream are ordered, so
 * they share the workspace safely; the workspace lives until the process
 * ends.
 */
int fsp_bound_pool(const fsp_nodes *nodes, int64_t count, int32_t *lb_out,
                   void *stream);

/*
 * fsp_bound_pool_noalloc -- fsp_bound_pool for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same bounds, but it never calls
 * hipMalloc, hipFree or any other allocating routine.  The job-mask walk
 * (instances with n > 64 loaded with FSP_LOAD_JOB_MASKS) takes its scratch
 * from a fixed device array of 32 MiB that the library holds on every device
 * it runs on until the process ends (found with hipGetSymbolAddress on the
 * first call per device); every other walk needs no scratch and any count is
 * served.  On the job-mask walk, a pool of more than
 * fsp_noalloc_max_count(n) nodes returns FSP_ESCRATCH before any device work
 * is queued.  All calls on one device share the array: calls that overlap on
 * one device (different streams, or host threads, without ordering between
 * them) race on it and give undefined bounds; calls ordered on one stream are
 * safe.  Nothing in the array needs clearing between calls (every slot is
 * written before it is read).
 */
int fsp_bound_pool_noalloc(const fsp_nodes *nodes, int64_t count, int32_t *lb_out,
                           void *stream);

/* Largest pool fsp_bound_pool_noalloc serves for an instance of n jobs on
 * the job-mask walk (INT64_MAX for n <= 64, where that walk is never taken;
 * 0 for n outside 1..255).  Instances on the other walks take any count. */
int64_t fsp_noalloc_max_count(int32_t n);

/*
 * fsp_bound_pool_one_machine -- lb_out[i] = the one-machine bound of record
 * i: the largest over machines k of head r[k] + remaining work of the
 * unscheduled jobs on k + their smallest tail after k (heads and tails as for
 * the pair bound; Sec. VI names other bounds as future work).  Never larger
 * than fsp_bound_pool's bound; the makespan for a complete record;
 * FSP_LB_INVALID for a malformed one.  Same arguments and behaviour as
 * fsp_bound_pool.
 */
int fsp_bound_pool_one_machine(const fsp_nodes *nodes, int64_t count,
                               int32_t *lb_out, void *stream);

/* ---- batched bounding: many instances in one launch ------------------- */

/* One pool of one instance.  data/lb_out: device pointers as in
 * fsp_bound_pool; stride >= inst's n + 1; count may be 0. */
typedef struct {
  const fsp_instance *inst;
  const uint8_t *data;
  int32_t stride;
  int64_t count;
  int32_t *lb_out;
} fsp_segment;

/* Launch shape of a batch (a NULL config, or all fields 0: the defaults).
 *   blocks_per_cu     workgroups per compute unit; 0: as many as fit (or the
 *                     autotuner's pick).
 *   autotune          1: before planning, time the candidate walk forms of
 *                     each (n, m) shape on the batch's own segments of that
 *                     shape (packed or 32-bit for n <= 32, 64-bit register or
 *                     job masks for 33..64 jobs, job masks or bytes above),
 *                     then the workgroups per CU
 *                     on the whole batch, and keep the fastest; the picks
 *                     are cached per device and shape (forms) and per batch
 *                     signature (workgroups per CU), so later batches of the
 *                     same shapes plan without timing.  Timing launches the
 *                     batch: its lb_out buffers are written.  0: every
 *                     segment takes its shape's default form (the fastest in
 *                     single-pool measurements, as fsp_instance_path).
 *   one_node_per_lane 1: never the packed two-nodes-per-lane form.
 *   job_masks         1: segments of more than 64 jobs take the job masks
 *                     by default instead of the bytes walk (instances loaded
 *                     with FSP_LOAD_JOB_MASKS always take them).
 * Other values are FSP_EINVAL. */
typedef struct {
  int32_t blocks_per_cu;
  int32_t autotune;
  int32_t one_node_per_lane;
  int32_t job_masks;
} fsp_batch_config;

typedef struct fsp_batch fsp_batch;

/*
 * fsp_batch_create -- plan one persistent launch that bounds every segment
 * (the parallel bounding of Sec. III over a batch of pools).  The segment
 * table (instances, device pointers, counts) is copied to the device; the
 * node buffers themselves are read at launch time, so their contents may
 * change between launches.  Segments of 5, 10 or 20 machines share the one
 * persistent kernel, each in its walk form (two nodes per lane for n <= 32
 * with small times, see fsp_instance_path); any other machine count is
 * bounded by single-pool launches queued right after it.  Synchronous.
 * Release with fsp_batch_free once no queued launch uses it.
 */
int fsp_batch_create(const fsp_segment *segs, int32_t nsegs,
                     const fsp_batch_config *cfg, fsp_batch **out);

/* Queue the batch on `stream` (a counter reset and the persistent kernel). */
int fsp_batch_launch(fsp_batch *b, void *stream);

/* Same work as fsp_batch_launch, through a hipGraph captured on the first
 * call and replayed on every call (on `stream`). */
int fsp_batch_replay(fsp_batch *b, void *stream);

/* Tiles (256 nodes, or 512 in the packed form), the largest persistent
 * grid, segments in the batch kernels (one-node forms, packed form) and
 * segments bounded by single-pool launches (any pointer may be NULL). */
int fsp_batch_info(const fsp_batch *b, int64_t *tiles, int32_t *grid,
                   int32_t *kernel_segments, int32_t *fallback_segments);

/* The walk form (FSP_PATH_*) each of the nsegs segments given to
 * fsp_batch_create takes (-1: empty segment, or bounded by a single-pool
 * launch, which takes fsp_instance_path), and the workgroups per CU of the
 * batch kernel.  nsegs must equal the count given at creation. */
int fsp_batch_paths(const fsp_batch *b, int32_t *paths, int32_t nsegs,
                    int32_t *blocks_per_cu);

int fsp_batch_free(fsp_batch *b);

/* One-shot: create, queue on `stream`, wait for the stream, free. */
int fsp_bound_batch(const fsp_segment *segs, int32_t nsegs, void *stream);

/* ---- branch-and-bound (Sec. II.A operators, Sec. III pool loop) --------- */

/* Pool-size policies.  FSP_POOL_FIXED: every pool has fixed_pool children.
 * FSP_POOL_ADAPTIVE: the paper's dynamic parameter tuning (Algorithm 1): start
 * at 256 threads x #compute units, double every nb_iterations pools while the
 * size stays within the device's resident-thread maximum, keeping the size
 * with the best measured efficiency (nodes bounded per second), then try the
 * midpoints around the best size for nb_iterations pools each and keep the
 * best for the rest of the run. */
#define FSP_POOL_FIXED 0
#define FSP_POOL_ADAPTIVE 1
#define FSP_POOL_AUTOTUNED 2
#define FSP_POOL_LEARNED 3

/* Elimination rule (Sec. II.A eliminates a node whose bound is greater than
 * the best makespan known).  FSP_PRUNE_GE (default) also eliminates a bound
 * equal to it, since such a node cannot hold a strictly better schedule;
 * FSP_PRUNE_GT keeps it, as the paper's wording does.  The optimum is the same
 * under both; the number of nodes explored differs. */
#define FSP_PRUNE_GE 0
#define FSP_PRUNE_GT 1

typedef struct {
  int32_t kind;           /* FSP_POOL_*                                      */
  int32_t nb_iterations;  /* pools per measurement/batch; <= 0: 10          */
  int64_t fixed_pool;     /* FSP_POOL_FIXED: children per pool (>= 1)      */
  int64_t max_pool;       /* largest pool; <= 0: resident threads of the
                             device.  Sizes the device buffers: about
                             n * (max_pool + n) * stride bytes of HBM.     */
  double time_limit_s;    /* stop after this wall time; <= 0: no limit     */
  int32_t prune_rule;     /* FSP_PRUNE_GE or FSP_PRUNE_GT                  */
  int32_t prefilter;      /* 1: one-machine pre-filter in every bounding
                             launch (a wave whose nodes that bound already
                             eliminates skips the pair walks; same
                             eliminations, same optimum); 0: none          */
  const void *model;      /* FSP_POOL_LEARNED: the policy network          */
  const char *log_path;   /* one JSON line per batch of pools; NULL: none  */
  int32_t host_threads;   /* hybrid search (Sec. VI, future work): CPU
                             threads that explore, beside the device, the
                             subtrees of nodes with at most six unscheduled
                             jobs taken from the deepest bucket whenever
                             they are idle, sharing UB with the device at
                             every batch of pools; 0: none                 */
  int32_t bound_choice;   /* the bound per depth (Sec. VI: other lower
                             bounds): 0: the two-machine bound at every
                             depth; 1: the depths chosen by
                             fsp_autotune_bounds (cached per shape) take
                             the one-machine bound, the others the
                             two-machine bound; 2: the depths whose bit is
                             set in lb1_depths take the one-machine bound.
                             Exact in every case (both are lower bounds);
                             host threads of the hybrid always take the
                             two-machine bound.                            */
  uint32_t lb1_depths[8]; /* bound_choice 2: bit d of word d / 32 set for
                             every depth d bounded by the one-machine bound */
} fsp_pool_policy;

typedef struct {
  int32_t makespan;   /* min(initial UB, best schedule found)               */
  int32_t found;      /* 1 if a schedule better than the initial UB was found */
  uint8_t *perm;      /* caller's HOST buffer of n bytes (may be NULL): the
                         best schedule when found == 1, or the NEH schedule
                         when ub_in <= 0; untouched meaning otherwise       */
  int32_t status;     /* 0: optimum proven (tree exhausted); 1: time limit */
  int32_t root_lb;    /* bound of the root                                  */
  int64_t nodes_bounded;   /* bound evaluations, root included             */
  int64_t nodes_branched;  /* nodes whose children were generated           */
  int64_t nodes_pruned;    /* nodes eliminated (children and stale parents) */
  int64_t leaves;          /* complete schedules bounded                    */
  int64_t pools;           /* pools bounded                                 */
  double t_found_s;   /* wall time when the final UB was found (0 if none) */
  double t_total_s;   /* wall time of the whole call                        */
  int64_t final_pool; /* pool size in force at the end                      */
  double t_search_s;  /* wall time of the search loop (set-up excluded)     */
  int32_t open_lb;    /* a lower bound on the optimum: the smallest bound of
                         the nodes still pending after a time limit (status
                         1), else the makespan; gap = (makespan - open_lb) /
                         makespan                                           */
  int32_t proof_pools; /* FSP_POOL_LEARNED: 1 if the network's estimates
                         switched the search to proof pools (see below)    */
  int64_t host_nodes;  /* of nodes_bounded, those bounded by host threads
                         (policy->host_threads > 0)                         */
} fsp_result;

/*
 * fsp_branch_and_bound -- exact minimum makespan of the instance (Sec. II:
 * branching appends one unscheduled job, bounding is the pool kernel,
 * selection takes the deepest pending nodes, elimination drops nodes that
 * cannot beat UB; Sec. III: pools are bounded in one launch each).
 *   ub_in > 0 : initial UB (e.g. a known optimum: then only the nodes whose
 *               bound is below it are explored, whatever the order);
 *   ub_in <= 0: initial UB from the NEH insertion heuristic.
 * Synchronous; allocates and frees its own device memory and stream.  With
 * status 0 the returned makespan is optimal.
 * FSP_POOL_AUTOTUNED: pools of policy->fixed_pool children, or (when <= 0)
 * of the size fsp_autotune_pool picks for this shape; the nb_iterations
 * iterations of a batch are captured once in a hipGraph and replayed.
 * FSP_POOL_LEARNED: as FSP_POOL_AUTOTUNED, and policy->model (an fsp_model
 * with 2 + 2 min(m, 15) inputs) orders the pools and sets their size.  While
 * the smallest estimated completion (bound + predicted gap) among the pending
 * nodes is below UB, the search dives: pools of a sixteenth of the autotuned
 * (or fixed_pool) number of children, doubled after every batch of
 * nb_iterations pools that does not improve UB (reset by an improvement),
 * and a pool that takes only part of a depth takes its nodes with the
 * smallest estimates; once that smallest
 * estimate reaches UB (the network expects no pending node to beat UB: what
 * is left is a proof, in which order does not matter), pools take the
 * largest size the buffers hold (policy->max_pool, or the device's resident
 * threads) and the network is no longer run (proof_pools = 1); on an
 * instance of more jobs than the network was trained on
 * (fsp_model_set_trained_jobs) the search does not switch and keeps diving,
 * its dive pools doubling up to that largest size.  The exact
 * bound still decides every elimination, so the optimum does not depend on
 * the model.
 * FSP_POOL_AUTOTUNED and FSP_POOL_LEARNED fill a pool from several depths,
 * deepest first (a depth taken whole is followed by the next shallower one,
 * at most eight); FSP_POOL_FIXED and FSP_POOL_ADAPTIVE take one depth per
 * pool.
 */
int fsp_branch_and_bound(const fsp_instance *inst,
                         const fsp_pool_policy *policy, int32_t ub_in,
                         fsp_result *out);

/*
 * fsp_adaptive_schedule -- the pool sizes that FSP_POOL_ADAPTIVE (the paper's
 * dynamic parameter tuning, Sec. III, Algorithm 1) sets, as a function of the
 * efficiencies it measures; host only, no device work.  Batch i (of
 * nb_iterations pools) runs with targets_out[i] children per pool and then
 * reports efficiency[i] (nodes bounded per second of that batch; the search
 * logs both per batch, see log_path).  The schedule starts at
 * threads_per_block x cus, doubles after every batch while the size stays
 * within min(max_threads, max_pool) (max_pool <= 0: max_threads), then
 * tries the midpoints between the best size and the ends of [best/2,
 * 2 best] (two rounds, the interval narrowed around the best after each),
 * sizes rounded to multiples of threads_per_block, and keeps the size of
 * the best efficiency from then on (a strictly higher efficiency replaces
 * the best).  efficiency, targets_out: host arrays of `batches` entries.
 */
int fsp_adaptive_schedule(int32_t threads_per_block, int32_t cus, int64_t max_threads,
                          int64_t max_pool, const double *efficiency, int32_t batches,
                          int64_t *targets_out);

/* The per-depth choice of bound (bound_choice 1; Sec. VI names other lower
 * bounds as future work).  A short search from NEH (budget_s seconds, <= 0:
 * 1 s; autotuned pool, the two-machine bound everywhere) counts per depth d
 * the bounded nodes with jobs left, those the one-machine bound eliminates
 * against the UB of the moment, and those the two-machine bound eliminates;
 * fsp_bound_choice_rule turns the counts into the mask (8 words, bit d of
 * word d / 32).  Cached per (device, n, m): later calls return the first
 * result. */
int fsp_autotune_bounds(const fsp_instance *inst, double budget_s, uint32_t *mask_out);

/* The rule of fsp_autotune_bounds (host only): from the deepest depth up,
 * depth d (1 .. n-1) takes the one-machine bound when it had nodes, the
 * next depth keeps the two-machine bound, and (elim2[d] - elim1[d]) *
 * (n - d) <= total[d] / 2 -- the nodes only the two-machine bound would have
 * eliminated, branched into n - d children that the next depth's
 * two-machine bound eliminates, cost at most half of the two-machine
 * walks saved.  total, elim1, elim2: 256 counts each, indexed by depth. */
int fsp_bound_choice_rule(int32_t n, const uint32_t *total, const uint32_t *elim1,
                          const uint32_t *elim2, uint32_t *mask_out);

/* fsp_branch_and_bound that also returns the per-depth counts of the bound
 * choice (stats_out: [3][256] words: bounded nodes with jobs left, those
 * the one-machine bound eliminates, those the two-machine bound eliminates,
 * against the UB of the moment).  While counting, the pre-filter skips no
 * walk; policy->bound_choice must be 0 (FSP_EINVAL otherwise). */
int fsp_depth_stats(const fsp_instance *inst, const fsp_pool_policy *policy, int32_t ub_in,
                    uint32_t *stats_out, fsp_result *result);

/*
 * fsp_autotune_pool -- the pool size (children per pool) that maximises
 * nodes bounded per second of search for this instance's shape: FSP_POOL_
 * AUTOTUNED searches of budget_s / #candidates seconds each (budget_s <= 0:
 * 0.25 s per candidate) over 2^14 .. min(resident threads, 2^20), each rated
 * on the batches after the first third of its search time, stretched up to
 * 8x until six batches were rated (a search that ends sooner is rated
 * whole); a larger pool is taken unless it is more than 3 % slower than the
 * best so far.
 * Cached per (device, n, m) for the life of
 * the process.  rate_out (may be NULL): the best rate measured (nodes per
 * second).
 */
int fsp_autotune_pool(const fsp_instance *inst, double budget_s,
                      int64_t *pool_out, double *rate_out);

/*
 * fsp_policy_samples -- training data for the pool-policy network, logged by
 * the search itself: runs fsp_branch_and_bound (any kind but LEARNED) and
 * logs each child that survives elimination with probability sample_prob
 * (deterministic in seed), at most max_samples.  For every logged node it
 * writes the network input (x_out, device bf16 [max_samples][32]) and two
 * targets (target_out, device fp32 [max_samples][2]): the gap between a
 * suffix-NEH completion of the node and its bound, over the NEH makespan;
 * and 1 if the node's bound reaches the final UB (it would be eliminated
 * with that UB), else 0.  *n_out: samples written; result: the search.
 */
int fsp_policy_samples(const fsp_instance *inst, const fsp_pool_policy *policy,
                       int32_t ub_in, int64_t max_samples, double sample_prob,
                       uint64_t seed, void *x_out, float *target_out,
                       int64_t *n_out, fsp_result *result);

/* NEH insertion heuristic (host): jobs by total time descending (ties by
 * id), each inserted where the partial makespan is smallest (earliest
 * position on ties).  perm_out: host buffer of n bytes (may be NULL). */
int fsp_neh(const fsp_instance *inst, uint8_t *perm_out, int32_t *makespan_out);

/* ---- the pool-policy network (learned pool policy) ---------------------- */

/* A 3-layer perceptron y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 over node
 * features x (in_features <= 32, zero-padded to 32), 128 hidden units per
 * layer, outputs <= 16.  bf16 matrix-core products with fp32 accumulation;
 * fp32 master weights.  Parameter vector (fp32, fsp_model_param_count()
 * entries): W1[32][128] b1[128] W2[128][128] b2[128] W3[128][16] b3[16],
 * rows/columns beyond in_features/outputs are zero and stay zero.  The
 * network only orders pools and sizes them; it never decides an elimination. */
typedef struct fsp_model fsp_model;

int fsp_model_create(int32_t in_features, int32_t hidden, int32_t outputs,
                     uint64_t seed, fsp_model **out); /* hidden must be 128 */
int fsp_model_free(fsp_model *m);
int64_t fsp_model_param_count(void);
/* The job count of the instances the network was trained on (0, the value
 * at creation: unknown).  The learned search (FSP_POOL_LEARNED) switches to
 * proof pools on the network's estimates only for instances of at most that
 * many jobs; on larger ones the estimates are extrapolations and the search
 * keeps diving (see fsp_branch_and_bound).  n < 0 or a NULL model:
 * FSP_EINVAL. */
int fsp_model_set_trained_jobs(fsp_model *m, int32_t n);
int fsp_model_set_params(fsp_model *m, const float *host, int64_t n);
int fsp_model_get_params(const fsp_model *m, float *host, int64_t n);
int fsp_model_get_grads(const fsp_model *m, float *host, int64_t n);

/* y[N][outputs] (device fp32) = network(x), x device bf16 [N][32].  Async. */
int fsp_model_forward(const fsp_model *m, const void *x, int64_t n, float *y,
                      void *stream);

/* Gradients of sum(dy . y) w.r.t. the parameters (stored in the model,
 * added to the previous ones when accumulate != 0) and, if dx is not NULL,
 * w.r.t. x (device fp32 [N][32]).  dy: device fp32 [N][outputs].  Async. */
int fsp_model_backward(fsp_model *m, const void *x, int64_t n, const float *dy,
                       float *dx, int32_t accumulate, void *stream);

/* Adam update of the parameters from the stored gradients.  Async. */
int fsp_model_adam_step(fsp_model *m, float lr, float beta1, float beta2,
                        float eps, float weight_decay, void *stream);

/* One training step on a batch: forward, loss (output 0: squared error
 * against target[r][0]; output 1, if present: logistic loss against
 * target[r][1] in {0,1}), backward, Adam (lr, 0.9, 0.999, 1e-8).  target:
 * device fp32 [N][2].  Writes the batch loss to *loss_out (host) if not NULL
 * (then synchronises the stream). */
int fsp_model_train_step(fsp_model *m, const void *x, const float *target,
                         int64_t n, float lr, float *loss_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FSP_H */
