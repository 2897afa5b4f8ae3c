// batch.hip -- many instances and uneven pools bounded in one persistent
// launch (the parallel bounding of Sec. III applied to a batch of pools).
//
// The host concatenates the pools into one tile space (256 nodes per tile),
// most expensive shape first (a node of shape n x m costs about m^2 n table
// steps), so that the cheap tiles fill the tail.  Workgroups take tiles from a
// device counter; when a workgroup moves on to another instance it restages
// that instance's LDS tables.  The kernel body is the same per-tile code as
// the single-pool kernel (bound_tile.hpp), specialised for 5, 10 and 20
// machines; segments with another machine count are bounded by single-pool
// launches queued right after the batch kernel.
//
// A batch object keeps the segment table and the counter on the device, so the
// pair of launches (counter reset, batch kernel) can be captured once in a
// hipGraph and replayed; replays see the current contents of the node buffers.
#include <algorithm>
#include <new>
#include <vector>

#include "bound_tile.hpp"

using namespace fspi;

namespace {

enum Variant : int {
  // per machine count: register (n <= 32), masks (one table chunk), masks
  // (chunked), 64-bit register (33..64 jobs, chunked body)
  V5N, V5W, V5C, V5R, V10N, V10W, V10C, V10R, V20N, V20W, V20C, V20R, VNONE
};

struct BatchSeg {
  InstView I;
  const uint8_t *nodes;
  int32_t *lb;
  int64_t count;
  int64_t tile_begin;  // first tile of this segment in the batch tile space
  int stride;
  int aligned;
  int variant;
  int pad;
};

constexpr size_t kWideBudget = 32 * 1024;
constexpr size_t kNarrowBudget = 64 * 1024;

__global__ void reset_counter(unsigned long long *c) {
  if (threadIdx.x == 0) *c = 0ull;
}

template <int M, int FORM, bool CHUNKED>
__device__ __forceinline__ void run_tile(const BatchSeg &S, char *smem,
                                         int64_t t, bool restage,
                                         char *tile_slots) {
  constexpr bool WIDE = FORM == kFormMasks;
  const InstView I = S.I;
  const LdsView L = carve<WIDE>(smem, I);
  if (restage) {
    stage_instance<WIDE>(I, L);
    __syncthreads();
  }
  bound_nodes<M, FORM, CHUNKED>(I, L, S.nodes, S.stride, S.aligned != 0,
                                (t - S.tile_begin) * kBlock, S.count, S.lb,
                                tile_slots);
}

__global__ __launch_bounds__(kBlock, 4) void batch_kernel(
    const BatchSeg *__restrict__ segs, int nsegs, int64_t total_tiles,
    unsigned long long *counter, char *slots, int64_t tile_bytes) {
  extern __shared__ __align__(16) char smem[];
  __shared__ long long s_tile;
  int cur = -1;
  while (true) {
    // every lane has finished the previous tile once it passes this barrier
    __syncthreads();
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= total_tiles) break;
    int lo = 0, hi = nsegs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile_begin <= t)
        lo = mid;
      else
        hi = mid - 1;
    }
    const BatchSeg &S = segs[lo];
    const bool restage = lo != cur;
    cur = lo;
    char *ts = slots + t * tile_bytes;  // this tile's job-mask slots
    switch (S.variant) {
      case V5N: run_tile<5, kFormReg32, false>(S, smem, t, restage, ts); break;
      case V5W: run_tile<5, kFormMasks, false>(S, smem, t, restage, ts); break;
      case V5C: run_tile<5, kFormMasks, true>(S, smem, t, restage, ts); break;
      case V5R: run_tile<5, kFormReg64, true>(S, smem, t, restage, ts); break;
      case V10N: run_tile<10, kFormReg32, false>(S, smem, t, restage, ts); break;
      case V10W: run_tile<10, kFormMasks, false>(S, smem, t, restage, ts); break;
      case V10C: run_tile<10, kFormMasks, true>(S, smem, t, restage, ts); break;
      case V10R: run_tile<10, kFormReg64, true>(S, smem, t, restage, ts); break;
      case V20N: run_tile<20, kFormReg32, false>(S, smem, t, restage, ts); break;
      case V20W: run_tile<20, kFormMasks, false>(S, smem, t, restage, ts); break;
      case V20C: run_tile<20, kFormMasks, true>(S, smem, t, restage, ts); break;
      case V20R: run_tile<20, kFormReg64, true>(S, smem, t, restage, ts); break;
      default: break;
    }
  }
}

int variant_of(const fsp_instance *inst, const InstView &v) {
  int base;
  switch (inst->m) {
    case 5: base = V5N; break;
    case 10: base = V10N; break;
    case 20: base = V20N; break;
    default: return VNONE;
  }
  if (!inst->wide) return base;
  if (!uses_job_masks(inst->n)) return base + 3;
  return v.nchunks > 1 ? base + 2 : base + 1;
}

}  // namespace

struct fsp_batch {
  int device = 0;
  int nsegs = 0;       // segments in the batch kernel
  int64_t total_tiles = 0;
  BatchSeg *d_segs = nullptr;
  unsigned long long *d_counter = nullptr;
  char *d_slots = nullptr;  // job-mask scratch of the batch kernel and fallbacks
  int64_t tile_bytes = 0;   // scratch bytes per tile of the batch kernel
  size_t lds = 0;
  int grid = 0;
  std::vector<fsp_segment> fallback;  // bounded by single-pool launches
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int enqueue(fsp_batch *b, hipStream_t s) {
  if (b->nsegs > 0) {
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, b->d_counter);
    hipLaunchKernelGGL(batch_kernel, dim3(b->grid), dim3(kBlock), b->lds, s,
                       b->d_segs, b->nsegs, b->total_tiles, b->d_counter,
                       b->d_slots, b->tile_bytes);
    FSP_HIP_TRY(hipGetLastError());
  }
  for (const fsp_segment &f : b->fallback) {
    // queued after the batch kernel on the same stream: the scratch is free
    const int rc = launch_bound(f.inst, f.data, f.stride, f.count, f.lb_out, s,
                                nullptr, b->d_slots);
    if (rc != FSP_OK) return rc;
  }
  return FSP_OK;
}

void destroy(fsp_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_segs) (void)hipFree(b->d_segs);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->d_slots) (void)hipFree(b->d_slots);
  delete b;
}

}  // namespace

extern "C" {

int fsp_batch_create(const fsp_segment *segs, int32_t nsegs,
                     const fsp_batch_config *cfg, fsp_batch **out) {
  if (!out) return FSP_EINVAL;
  *out = nullptr;
  if (nsegs < 0 || (nsegs > 0 && !segs)) return FSP_EINVAL;
  for (int i = 0; i < nsegs; ++i) {
    const fsp_segment &g = segs[i];
    if (!g.inst || g.count < 0) return FSP_EINVAL;
    if (g.count == 0) continue;  // nothing to read: pointers and stride unused
    if (!g.data || !g.lb_out) return FSP_EINVAL;
    if (g.stride < g.inst->n + 1) return FSP_EINVAL;
  }
  fsp_batch *b = new (std::nothrow) fsp_batch();
  if (!b) return FSP_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    destroy(b);
    return FSP_EDEVICE;
  }
  struct Item {
    BatchSeg s;
    double cost;
  };
  std::vector<Item> items;
  for (int i = 0; i < nsegs; ++i) {
    const fsp_segment &g = segs[i];
    if (g.count == 0) continue;
    const fsp_instance *in = g.inst;
    Item it{};
    it.s.I = inst_view(in, in->wide ? kWideBudget : kNarrowBudget);
    it.s.variant = variant_of(in, it.s.I);
    if (it.s.variant == VNONE) {
      b->fallback.push_back(g);
      continue;
    }
    it.s.nodes = g.data;
    it.s.lb = g.lb_out;
    it.s.count = g.count;
    it.s.stride = g.stride;
    it.s.aligned = ((reinterpret_cast<uintptr_t>(g.data) & 15) == 0 &&
                    (g.stride & 15) == 0)
                       ? 1
                       : 0;
    it.cost = (double)in->P * in->npad;
    items.push_back(it);
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const Item &a, const Item &c) { return a.cost > c.cost; });
  std::vector<BatchSeg> table;
  int64_t tiles = 0;
  size_t lds = 16;
  int slot_max = 0;
  for (const Item &it : items) slot_max = std::max(slot_max, it.s.I.slot_bytes);
  size_t scratch = 0;
  for (const fsp_segment &f : b->fallback)
    scratch = std::max(scratch, bound_scratch_bytes(f.inst->n, f.count));
  for (Item &it : items) {
    it.s.tile_begin = tiles;
    tiles += (it.s.count + kBlock - 1) / kBlock;
    const int form = it.s.variant % 4;  // 0 register, 1-2 masks, 3 register64
    const bool wide = form == 1 || form == 2;
    lds = std::max(lds, lds_bytes(it.s.I.n, it.s.I.mp, it.s.I.npad, it.s.I.ppc, wide));
    table.push_back(it.s);
  }
  b->nsegs = (int)table.size();
  b->total_tiles = tiles;
  b->lds = lds;
  b->tile_bytes = (int64_t)(kBlock / 64) * slot_max;
  scratch = std::max(scratch, (size_t)(tiles * b->tile_bytes));
  if (scratch > 0 && hipMalloc(&b->d_slots, scratch) != hipSuccess) {
    destroy(b);
    return FSP_ENOMEM;
  }
  if (b->nsegs > 0) {
    if (hipMalloc(&b->d_segs, table.size() * sizeof(BatchSeg)) != hipSuccess ||
        hipMalloc(&b->d_counter, sizeof(unsigned long long)) != hipSuccess) {
      destroy(b);
      return FSP_ENOMEM;
    }
    if (hipMemcpy(b->d_segs, table.data(), table.size() * sizeof(BatchSeg),
                  hipMemcpyHostToDevice) != hipSuccess) {
      destroy(b);
      return FSP_EDEVICE;
    }
    const void *fn = reinterpret_cast<const void *>(batch_kernel);
    int cus = 0, per_cu = 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              b->device) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds) !=
            hipSuccess) {
      destroy(b);
      return FSP_EDEVICE;
    }
    if (per_cu < 1) {
      destroy(b);
      return FSP_EUNSUPPORTED;
    }
    int want = per_cu;
    if (cfg && cfg->blocks_per_cu > 0) want = std::min(per_cu, cfg->blocks_per_cu);
    int64_t grid = (int64_t)want * cus;
    if (grid > tiles) grid = tiles;
    b->grid = (int)std::max<int64_t>(1, grid);
  }
  *out = b;
  return FSP_OK;
}

int fsp_batch_launch(fsp_batch *b, void *stream) {
  if (!b) return FSP_EINVAL;
  return enqueue(b, reinterpret_cast<hipStream_t>(stream));
}

int fsp_batch_replay(fsp_batch *b, void *stream) {
  if (!b) return FSP_EINVAL;
  if (!b->exec) {
    FSP_HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    FSP_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != FSP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return FSP_EDEVICE;
    b->graph = g;
    FSP_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  FSP_HIP_TRY(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
  return FSP_OK;
}

int fsp_batch_info(const fsp_batch *b, int64_t *tiles, int32_t *grid,
                   int32_t *kernel_segments, int32_t *fallback_segments) {
  if (!b) return FSP_EINVAL;
  if (tiles) *tiles = b->total_tiles;
  if (grid) *grid = b->grid;
  if (kernel_segments) *kernel_segments = b->nsegs;
  if (fallback_segments) *fallback_segments = (int32_t)b->fallback.size();
  return FSP_OK;
}

int fsp_batch_free(fsp_batch *b) {
  if (!b) return FSP_OK;
  destroy(b);
  return FSP_OK;
}

int fsp_bound_batch(const fsp_segment *segs, int32_t nsegs, void *stream) {
  fsp_batch *b = nullptr;
  int rc = fsp_batch_create(segs, nsegs, nullptr, &b);
  if (rc != FSP_OK) return rc;
  rc = enqueue(b, reinterpret_cast<hipStream_t>(stream));
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess &&
      rc == FSP_OK)
    rc = FSP_EDEVICE;
  destroy(b);
  return rc;
}

}  // extern "C"
