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
// whatever the order).  The same algebra makes an absent job a no-op: with
// (b - a) and (lag + b) both replaced by 0, z' = max(z, 0) = z.  So every
// lane walks the same table position in lock-step, the table entry is a
// wave-uniform LDS broadcast, and the per-lane work is
//     alpha = bit job of U            (v_bfe_u32)
//     z     = max(z + alpha*x, alpha*y)   (v_mad_i32_i24, v_mul_u32_u24, v_max_i32)
// z is kept scaled by 256 with the job id riding in the low byte of y (so no
// extra instruction is needed to split the record): for integers the high
// part of max(256u + e, 256v + j) with 0 <= e, j < 256 is max(u, v), so
// z = Z >> 8 exactly.
//
// Data layout in LDS (per workgroup): the pair table (whole, or chunk by
// chunk when it does not fit), the padded p matrix for the prefix recurrence
// and, for n > 32, one membership byte per (job, lane).
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
};

template <int M, bool WIDE, bool CHUNKED>
__global__ __launch_bounds__(kBlock, 4) void bound_kernel(const BoundParams a) {
  extern __shared__ __align__(16) char smem[];
  const LdsView L = carve<WIDE>(smem, a.I);
  stage_instance<WIDE>(a.I, L);
  __syncthreads();
  int64_t count = a.count, ntiles = a.ntiles;
  if (a.count_dev) {
    count = *a.count_dev;
    ntiles = (count + kBlock - 1) / kBlock;
  }
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    bound_nodes<M, WIDE, CHUNKED>(a.I, L, a.nodes, a.stride, a.aligned != 0,
                                  tile * kBlock, count, a.lb);
}

using BoundFn = void (*)(BoundParams);

template <int M>
BoundFn pick(bool wide, bool chunked) {
  if (!wide) return bound_kernel<M, false, false>;
  return chunked ? bound_kernel<M, true, true> : bound_kernel<M, true, false>;
}

BoundFn kernel_for(int m, bool wide, bool chunked) {
  switch (m) {
    case 2: return pick<2>(wide, chunked);
    case 3: return pick<3>(wide, chunked);
    case 4: return pick<4>(wide, chunked);
    case 5: return pick<5>(wide, chunked);
    case 6: return pick<6>(wide, chunked);
    case 7: return pick<7>(wide, chunked);
    case 8: return pick<8>(wide, chunked);
    case 9: return pick<9>(wide, chunked);
    case 10: return pick<10>(wide, chunked);
    case 11: return pick<11>(wide, chunked);
    case 12: return pick<12>(wide, chunked);
    case 13: return pick<13>(wide, chunked);
    case 14: return pick<14>(wide, chunked);
    case 15: return pick<15>(wide, chunked);
    case 16: return pick<16>(wide, chunked);
    case 17: return pick<17>(wide, chunked);
    case 18: return pick<18>(wide, chunked);
    case 19: return pick<19>(wide, chunked);
    case 20: return pick<20>(wide, chunked);
    default: return nullptr;
  }
}

// LDS budget of one workgroup for the pair table: the whole table for
// n <= 32 (at most 48.6 KB); 32 KB chunks above, so that four workgroups fit
// on a compute unit.
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
  v.n = inst->n;
  v.mp = inst->mp;
  v.npad = inst->npad;
  v.P = inst->P;
  const size_t rsz = inst->wide ? sizeof(WideRec) : sizeof(NarrowRec);
  const size_t per_pair = (size_t)inst->npad * rsz;
  int ppc = (int)(table_budget / per_pair);
  if (ppc < 1) ppc = 1;
  if (ppc > inst->P) ppc = inst->P;
  v.ppc = ppc;
  v.nchunks = (inst->P + ppc - 1) / ppc;
  return v;
}

int launch_bound(const fsp_instance *inst, const uint8_t *nodes, int stride,
                 int64_t count, int32_t *lb_out, hipStream_t stream,
                 const int32_t *count_dev) {
  if (count == 0) return FSP_OK;
  const bool wide = inst->wide != 0;
  BoundParams a{};
  a.nodes = nodes;
  a.count = count;
  a.ntiles = (count + kBlock - 1) / kBlock;
  a.count_dev = count_dev;
  a.stride = stride;
  a.aligned = ((reinterpret_cast<uintptr_t>(nodes) & 15) == 0 &&
               (stride & 15) == 0)
                  ? 1
                  : 0;
  a.lb = lb_out;
  a.I = inst_view(inst, wide ? kTableBudgetWide : kTableBudgetNarrow);
  BoundFn fn = kernel_for(inst->m, wide, a.I.nchunks > 1);
  if (!fn) return FSP_EUNSUPPORTED;
  const size_t lds = lds_bytes(a.I.n, a.I.mp, a.I.npad, a.I.ppc, wide);

  // device attributes and per-kernel occupancy are queried once per
  // (device, kernel, LDS size) and cached for this thread
  struct Occ {
    int dev;
    BoundFn fn;
    size_t lds;
    int per_cu;
  };
  static thread_local std::vector<Occ> occ_cache;
  static thread_local int cached_dev = -1, cached_cus = 0;
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  if (dev != cached_dev) {
    FSP_HIP_TRY(hipDeviceGetAttribute(&cached_cus,
                                      hipDeviceAttributeMultiprocessorCount, dev));
    cached_dev = dev;
  }
  int per_cu = -1;
  for (const Occ &o : occ_cache)
    if (o.dev == dev && o.fn == fn && o.lds == lds) per_cu = o.per_cu;
  if (per_cu < 0) {
    FSP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    FSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(fn), kBlock, lds));
    occ_cache.push_back({dev, fn, lds, per_cu});
  }
  if (per_cu < 1) return FSP_EUNSUPPORTED;
  int64_t grid = (int64_t)per_cu * cached_cus;
  if (grid > a.ntiles) grid = a.ntiles;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kBlock), lds, stream, a);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

}  // namespace fspi

extern "C" int fsp_bound_pool(const fsp_nodes *nodes, int64_t count,
                              int32_t *lb_out, void *stream) {
  if (!nodes || !nodes->inst || count < 0) return FSP_EINVAL;
  if (count == 0) return FSP_OK;
  if (!nodes->data || !lb_out) return FSP_EINVAL;
  if (nodes->stride < nodes->inst->n + 1) return FSP_EINVAL;
  return fspi::launch_bound(nodes->inst, nodes->data, nodes->stride, count,
                            lb_out, reinterpret_cast<hipStream_t>(stream),
                            nullptr);
}
