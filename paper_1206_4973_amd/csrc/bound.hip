// bound.hip -- the pool-bounding kernel: one launch bounds every node of a
// pool (the parallel bounding model of Sec. III), one lane per node.
//
// Per node (the bound whose cost Sec. V.D gives as O(m^2 n log n)):
//   1. decode the prefix, build the unscheduled-job mask U, and run the
//      makespan recurrence over the prefix: F[k] = completion on machine k
//      (Sec. II.B);
//   2. heads r[k] = max(F[k], F[0] + min_{j in U} H[j][k]), tails
//      q[l] = min_{j in U} Q[j][l], remaining work S[k] = sum_{j in U} p[j][k];
//   3. for every pair (k,l): walk the pair's Johnson order (the table built
//      at load time), taking the jobs of U; the bound of the pair is the
//      completion on l of the two-machine relaxation plus q[l];
//   4. bound = max over pairs (the makespan itself when U is empty).
//
// Step 3 is the hot loop.  The textbook form keeps two clocks,
//     tk += a;  tl = max(tl, tk + lag) + b,
// i.e. four operations per (pair, unscheduled job).  This kernel keeps only
// their difference z = tl - tk >= 0:
//     z' = max(z - a, lag) + b = max(z + (b - a), lag + b),
// and recovers tl at the end as r[k] + S[k] + z (tk ends at r[k] + S[k]
// whatever the order).  Every lane walks the same table position in
// lock-step; the record {x = 256 (b - a), y = 256 (lag + b) + job} is a
// wave-uniform LDS broadcast, and a lane whose node has the position's job
// already scheduled must keep its z.  Five forms of that choice:
//   register (n <= 32): the node's unscheduled set U is one register, and
//       alpha = bit job of U;  z = max(z + alpha*x, alpha*y)
//     (v_bfe_u32, v_mad_i32_i24, v_mul_u32_u24, v_max_i32); alpha = 0 gives
//     max(z, 0) = z.
//   packed (n <= 32 and total work <= 32767): the same step for two nodes
//     per lane in 16-bit halves, the per-job multipliers of both nodes in
//     registers picked by the VGPR index mode (v_pk_mad_u16,
//     v_pk_mul_lo_u16, v_pk_max_i16: three instructions for two nodes); see
//     bound_tile.hpp.
//   register64 (33..64 jobs): U in a 64-bit register pair, alpha taken with
//     v_lshrrev_b64 by the job in y's low bits and v_and_b32.
//   masks (n > 64): each wave first writes, once per tile, the 64-bit mask of
//     lanes that still have job j, for every j, into a scratch slot (one
//     ballot per job), and the walk reads the position's mask with a scalar
//     load (the job's slot offset comes from a second, scalar-read table):
//       t = max(z + x, y);  z = mask[job] ? t : z
//     (v_add_u32, v_max_i32, v_cndmask_b32 on the SGPR pair).  Up to 64 jobs
//     the register forms are faster: the scalar loads miss the scalar cache
//     more than the bit extract they save costs.  Taken by load flag.
//   bytes (n > 64, the default there): each lane keeps its unscheduled flags
//     as bytes in LDS ([job][lane] rows of its wave); the records, one word
//     x | y << 16 in plain units (b - a and lag + b fit in 16 bits under the
//     instance limits), and the job ids come from scalar loads of global
//     tables, so LDS returns only the flag bytes:
//       z = max(z + alpha*x, alpha*y)
//     (v_lshl_add_u32 for the flag address, v_mad_i32_i16 and v_mad_u32_u16
//     on the record's halves, v_max_i32).
// In the register and mask forms z is kept scaled by 256 with the job id
// riding in the low byte of y (so no extra instruction is needed to split
// the record): for integers the high part of max(256u + e, 256v + j) with
// 0 <= e, j < 256 is max(u, v), so z = Z >> 8 exactly.
//
// Data layout: in LDS (per workgroup) the pair records (whole table, or chunk
// by chunk when it does not fit; none in the bytes form), the padded p
// matrix for the prefix recurrence (packed machine pairs in the packed form)
// and, for n > 32, the unscheduled-job words of every lane (the flag bytes in
// the bytes form); in global memory the tables read by scalar loads (mask
// offsets; the bytes form's record words and job bytes) and, for the job-mask
// walk, the scratch of job-mask slots, one per wave of every tile, each
// written once per launch.
#include <algorithm>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "bound_tile.hpp"

using namespace fspi;

namespace {

struct BoundParams {
  InstView I;
  const uint8_t *nodes;
  int64_t count;
  int64_t ntiles;
  const int32_t *count_dev;  // when set, the node count is read from here
  int stride;
  int aligned;  // records 16-byte aligned: load them as uint4
  int32_t *lb;
  char *slots;  // bound_scratch_bytes(n, count) bytes of job-mask slots (n > 64)
  Prefilter pf;
};

template <int M, int FORM, bool CHUNKED>
__global__ __launch_bounds__(kBlock, 4) void bound_kernel(
    const BoundParams a) {
  constexpr bool WIDE = FORM == kFormMasks || FORM == kFormBytes;
  extern __shared__ __align__(16) char smem[];
  int64_t count = a.count, ntiles = a.ntiles;
  if (a.count_dev) {
    // never more than the capacity that sized the grid and the scratch
    count = min((int64_t)*a.count_dev, a.count);
    ntiles = (count + kBlock - 1) / kBlock;
  }
  // a workgroup without a tile leaves before staging the tables
  if ((int64_t)blockIdx.x >= ntiles) return;
  const LdsView L = carve<WIDE, FORM == kFormBytes>(smem, a.I);
  stage_instance<WIDE, FORM == kFormBytes>(a.I, L);
  __syncthreads();
  const size_t tile_bytes = (size_t)(kBlock / 64) * (size_t)a.I.slot_bytes;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    bound_nodes<M, FORM, CHUNKED>(a.I, L, a.nodes, a.stride, a.aligned != 0,
                                  tile * kBlock, count, a.lb,
                                  a.slots + (size_t)tile * tile_bytes, a.pf);
}

// Two nodes per lane in packed 16-bit arithmetic (n <= 32, total work <=
// 32767): tiles of 2 * kBlock nodes.  Both nodes are set up together in
// packed form, so the kernel fits four workgroups per CU (128 VGPRs).  PF:
// the launch carries a pre-filter, a per-depth bound choice or depth counts.
template <int M, bool PF>
__global__ __launch_bounds__(kBlock, 4) void bound_kernel_p16(const BoundParams a) {
  extern __shared__ __align__(16) char smem[];
  int64_t count = a.count, ntiles = a.ntiles;
  if (a.count_dev) {
    count = min((int64_t)*a.count_dev, a.count);
    ntiles = (count + 2 * kBlock - 1) / (2 * kBlock);
  }
  if ((int64_t)blockIdx.x >= ntiles) return;
  const LdsView L = carve_p16(smem, a.I);
  stage_p16_rows(a.I, L);
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    bound_nodes_p16<M, PF>(a.I, L, a.nodes, a.stride, a.aligned != 0,
                           tile * 2 * kBlock, count, a.lb, a.pf);
}

using BoundFn = void (*)(BoundParams);

template <int... Ks>
BoundFn p16_kernel(int m, bool pf, std::integer_sequence<int, Ks...>) {
  constexpr BoundFn plain[] = {bound_kernel_p16<Ks + 2, false>...};
  constexpr BoundFn filtered[] = {bound_kernel_p16<Ks + 2, true>...};
  return pf ? filtered[m - 2] : plain[m - 2];
}

template <int M>
BoundFn pick(int form, bool chunked) {
  // the 64-bit register form always takes the chunked body (it also serves a
  // table of one chunk)
  if (form == kFormReg64) return bound_kernel<M, kFormReg64, true>;
  if (form == kFormReg32) return bound_kernel<M, kFormReg32, false>;
  // the bytes walk stages no table, so it is never chunked
  if (form == kFormBytes) return bound_kernel<M, kFormBytes, false>;
  return chunked ? bound_kernel<M, kFormMasks, true> : bound_kernel<M, kFormMasks, false>;
}

BoundFn kernel_for(int m, int form, bool chunked) {
  switch (m) {
    case 2: return pick<2>(form, chunked);
    case 3: return pick<3>(form, chunked);
    case 4: return pick<4>(form, chunked);
    case 5: return pick<5>(form, chunked);
    case 6: return pick<6>(form, chunked);
    case 7: return pick<7>(form, chunked);
    case 8: return pick<8>(form, chunked);
    case 9: return pick<9>(form, chunked);
    case 10: return pick<10>(form, chunked);
    case 11: return pick<11>(form, chunked);
    case 12: return pick<12>(form, chunked);
    case 13: return pick<13>(form, chunked);
    case 14: return pick<14>(form, chunked);
    case 15: return pick<15>(form, chunked);
    case 16: return pick<16>(form, chunked);
    case 17: return pick<17>(form, chunked);
    case 18: return pick<18>(form, chunked);
    case 19: return pick<19>(form, chunked);
    case 20: return pick<20>(form, chunked);
    default: return nullptr;
  }
}

// LDS budget of one workgroup for the pair table: the whole table for
// n <= 32 (at most 48.6 KB); 32 KB chunks above, so that four workgroups fit
// on a compute unit next to the job words.
constexpr size_t kTableBudgetNarrow = 64 * 1024;
constexpr size_t kTableBudgetWide = 32 * 1024;


}  // namespace

namespace fspi {

InstView inst_view(const fsp_instance *inst, size_t table_budget) {
  InstView v{};
  v.p = inst->d_p;
  v.Hp = inst->d_Hp;
  v.Qp = inst->d_Qp;
  v.tot = inst->d_tot;
  v.rec = inst->d_rec;
  v.joff = inst->d_joff;
  v.xy16 = inst->d_xy16;
  v.job16 = inst->d_job16;
  v.bxy = inst->d_bxy;
  v.bjob = inst->d_bjob;
  v.npad8 = inst->npad8;
  v.slot_bytes = uses_job_masks(inst->n) ? mask_slot_bytes(inst->n) : 0;
  v.n = inst->n;
  v.mp = inst->mp;
  v.npad = inst->npad;
  v.P = inst->P;
  const size_t per_pair = (size_t)inst->npad * sizeof(Rec);
  int ppc = (int)(table_budget / per_pair);
  if (ppc < 1) ppc = 1;
  if (ppc > inst->P) ppc = inst->P;
  v.ppc = ppc;
  v.nchunks = (inst->P + ppc - 1) / ppc;
  return v;
}

int stream_scratch(hipStream_t stream, size_t bytes, void **out) {
  // one workspace per (device, stream); the per-thread default stream is a
  // different stream in every host thread, so it is also keyed by thread
  struct Ws {
    int dev;
    hipStream_t stream;
    std::thread::id thread;
    void *ptr;
    size_t bytes;
  };
  static std::mutex mu;
  static std::vector<Ws> spaces;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  const std::thread::id tid = stream == hipStreamPerThread
                                  ? std::this_thread::get_id()
                                  : std::thread::id();
  std::lock_guard<std::mutex> lock(mu);
  Ws *w = nullptr;
  for (Ws &s : spaces)
    if (s.dev == dev && s.stream == stream && s.thread == tid) w = &s;
  if (!w) {
    spaces.push_back({dev, stream, tid, nullptr, 0});
    w = &spaces.back();
  }
  if (w->bytes < bytes) {
    // the old workspace may still be in use by work queued on the stream
    if (w->ptr) {
      FSP_HIP_TRY(hipStreamSynchronize(stream));
      (void)hipFree(w->ptr);
      w->ptr = nullptr;
      w->bytes = 0;
    }
    const size_t grow = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&w->ptr, grow) != hipSuccess) {
      w->ptr = nullptr;
      return FSP_ENOMEM;
    }
    w->bytes = grow;
  }
  *out = w->ptr;
  return FSP_OK;
}

int launch_bound(const fsp_instance *inst, const uint8_t *nodes, int stride,
                 int64_t count, int32_t *lb_out, hipStream_t stream,
                 const int32_t *count_dev, void *scratch, const Prefilter &pf) {
  if (count == 0) return FSP_OK;
  const bool wide = inst->wide != 0;
  const size_t need = walk_scratch_bytes(inst, count);
  if (!scratch && need > 0) {
    const int rc = stream_scratch(stream, need, &scratch);
    if (rc != FSP_OK) return rc;
  }
  const bool p16 = inst->p16 != 0;
  const int64_t tile_nodes = p16 ? 2 * kBlock : kBlock;
  BoundParams a{};
  a.pf = pf;
  a.slots = static_cast<char *>(scratch);
  a.nodes = nodes;
  a.count = count;
  a.ntiles = (count + tile_nodes - 1) / tile_nodes;
  a.count_dev = count_dev;
  a.stride = stride;
  a.aligned = ((reinterpret_cast<uintptr_t>(nodes) & 15) == 0 &&
               (stride & 15) == 0)
                  ? 1
                  : 0;
  a.lb = lb_out;
  // n > 32: the 64-bit register form up to 64 jobs, the bytes walk above
  // (or the job masks, by load flag)
  const int form = !wide                        ? kFormReg32
                   : !uses_job_masks(inst->n)   ? kFormReg64
                   : takes_mask_walk(inst)      ? kFormMasks
                                                : kFormBytes;
  a.I = inst_view(inst, form == kFormBytes ? table_budget_bytes(inst->n)
                        : wide             ? kTableBudgetWide
                                           : kTableBudgetNarrow);
  if (form != kFormMasks) a.I.slot_bytes = 0;
  BoundFn fn;
  if (p16) {
    fn = inst->m >= 2 && inst->m <= kMaxMachines
             ? p16_kernel(inst->m, pf.ub || pf.lb1_only || pf.lb1_depths || pf.depth_stats,
                          std::make_integer_sequence<int, kMaxMachines - 1>())
             : nullptr;
  } else {
    fn = kernel_for(inst->m, form, a.I.nchunks > 1);
  }
  if (!fn) return FSP_EUNSUPPORTED;
  const size_t lds = p16 ? lds_bytes_p16(a.I.n, a.I.mp, a.I.npad, a.I.P)
                        : lds_bytes(a.I.n, a.I.mp, a.I.npad, a.I.ppc,
                                    form == kFormMasks || form == kFormBytes,
                                    form == kFormBytes);

  // device attributes and per-kernel occupancy are queried once per
  // (device, kernel, LDS size) and cached for this thread, in a fixed table
  // (no host allocation on the launch path; a full table is refilled from
  // its start)
  struct Occ {
    int dev;
    BoundFn fn;
    size_t lds;
    int per_cu;
  };
  constexpr int kOccSlots = 64;
  static thread_local Occ occ_cache[kOccSlots];
  static thread_local int occ_used = 0, occ_next = 0;
  static thread_local int cached_dev = -1, cached_cus = 0;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  if (dev != cached_dev) {
    FSP_HIP_TRY(hipDeviceGetAttribute(&cached_cus,
                                      hipDeviceAttributeMultiprocessorCount, dev));
    cached_dev = dev;
  }
  int per_cu = -1;
  for (int i = 0; i < occ_used; ++i) {
    const Occ &o = occ_cache[i];
    if (o.dev == dev && o.fn == fn && o.lds == lds) per_cu = o.per_cu;
  }
  if (per_cu < 0) {
    FSP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    FSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(fn), kBlock, lds));
    occ_cache[occ_next] = {dev, fn, lds, per_cu};
    occ_next = (occ_next + 1) % kOccSlots;
    if (occ_used < kOccSlots) ++occ_used;
  }
  if (per_cu < 1) return FSP_EUNSUPPORTED;
  int64_t grid = (int64_t)per_cu * cached_cus;
  if (grid > a.ntiles) grid = a.ntiles;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kBlock), lds, stream, a);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

}  // namespace fspi

// ---- bounding without allocation ------------------------------------------
// The job-mask walk (n > 64) needs scratch that grows with the pool.  For
// callers that cannot allocate, fsp_bound_pool_noalloc takes it from this
// fixed array instead: every device the library runs on holds one copy for
// the life of the process.  In host code `scratch` is only a stand-in for the
// symbol; its device address, per device, comes from hipGetSymbolAddress on
// the first call made with that device current.
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device.
int noalloc_scratch(void **out) {
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FSP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    FSP_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return FSP_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FSP_OK;
}

}  // namespace

extern "C" int64_t fsp_noalloc_max_count(int32_t n) {
  if (n < 1 || n > kMaxJobs) return 0;
  if (!uses_job_masks(n)) return INT64_MAX;
  // whole tiles of kBlock nodes, each kBlock / 64 wave slots
  const int64_t per_tile = (int64_t)(kBlock / 64) * mask_slot_bytes(n);
  return (int64_t)(kNoAllocScratchBytes / (size_t)per_tile) * kBlock;
}

extern "C" int fsp_bound_pool_noalloc(const fsp_nodes *nodes, int64_t count,
                                      int32_t *lb_out, void *stream) {
  if (!nodes || !nodes->inst || count < 0) return FSP_EINVAL;
  if (count == 0) return FSP_OK;
  if (!nodes->data || !lb_out) return FSP_EINVAL;
  if (nodes->stride < nodes->inst->n + 1) return FSP_EINVAL;
  const fsp_instance *inst = nodes->inst;
  void *ptr = nullptr;
  if (takes_mask_walk(inst)) {
    if (count > fsp_noalloc_max_count(inst->n) ||
        bound_scratch_bytes(inst->n, count) > kNoAllocScratchBytes)
      return FSP_ESCRATCH;
    const int rc = noalloc_scratch(&ptr);
    if (rc != FSP_OK) return rc;
  }
  // with scratch given (or none needed) the launch allocates nothing
  return fspi::launch_bound(inst, nodes->data, nodes->stride, count, lb_out,
                            reinterpret_cast<hipStream_t>(stream), nullptr, ptr);
}

extern "C" int fsp_bound_pool_one_machine(const fsp_nodes *nodes, int64_t count,
                                          int32_t *lb_out, void *stream) {
  if (!nodes || !nodes->inst || count < 0) return FSP_EINVAL;
  if (count == 0) return FSP_OK;
  if (!nodes->data || !lb_out) return FSP_EINVAL;
  if (nodes->stride < nodes->inst->n + 1) return FSP_EINVAL;
  Prefilter pf;
  pf.lb1_only = 1;
  return fspi::launch_bound(nodes->inst, nodes->data, nodes->stride, count,
                            lb_out, reinterpret_cast<hipStream_t>(stream),
                            nullptr, nullptr, pf);
}

extern "C" int fsp_bound_pool(const fsp_nodes *nodes, int64_t count,
                              int32_t *lb_out, void *stream) {
  if (!nodes || !nodes->inst || count < 0) return FSP_EINVAL;
  if (count == 0) return FSP_OK;
  if (!nodes->data || !lb_out) return FSP_EINVAL;
  if (nodes->stride < nodes->inst->n + 1) return FSP_EINVAL;
  return fspi::launch_bound(nodes->inst, nodes->data, nodes->stride, count,
                            lb_out, reinterpret_cast<hipStream_t>(stream),
                            nullptr, nullptr);
}
