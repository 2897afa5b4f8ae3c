// batch.hip -- many instances and uneven pools bounded in one persistent
// launch (the parallel bounding of Sec. III applied to a batch of pools).
//
// The host concatenates the pools into one tile space, most expensive tile
// first (a node of shape n x m costs about m^2 n table steps, scaled by the
// walk form's instructions per step), so that the cheap tiles fill the tail.
// A tile is 256 nodes (one per lane) or, in the packed form, 512 (two per
// lane).  Workgroups take tiles from a device counter; when a workgroup moves
// on to another instance it restages that instance's LDS tables.  The kernel
// body is the same per-tile code as the single-pool kernels
// (bound_tile.hpp), specialised for 5, 10 and 20 machines and every walk
// form; segments with another machine count are bounded by single-pool
// launches queued right after the batch kernel.
//
// Launch shape: by default every segment takes the fastest form that its
// shape allows in single-pool measurements (packed for n <= 32 with small
// times, the 64-bit register form for 33..64 jobs, the bytes walk above) and
// the grid holds as many workgroups per CU as fit.  Two kernels: the packed
// segments, and every one-node form.  With autotuning, the planner
// times the candidate forms of each shape on the batch's own segments of that
// shape, then the number of workgroups per CU on the whole batch, and keeps
// the fastest (cached per device and shape, resp. per batch signature).
//
// A batch object keeps the segment table and the counter on the device, so the
// pair of launches (counter reset, batch kernel) can be captured once in a
// hipGraph and replayed; replays see the current contents of the node buffers.
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "bound_tile.hpp"

using namespace fspi;

namespace {

// Walk forms of a segment (see bound.hip).
enum SegForm : int {
  kSegReg32 = 0,   // n <= 32, one node per lane
  kSegMasks = 1,   // job masks, whole table in LDS
  kSegMasksC = 2,  // job masks, table streamed in chunks
  kSegReg64 = 3,   // 33..64 jobs, 64-bit register
  kSegPacked = 4,  // n <= 32 and total work <= 32767, two nodes per lane
  kSegBytes = 5,   // n > 64, flag bytes in LDS, table by scalar loads
  kSegForms = 6
};

// Kernel (part) of a form: the one-node forms (register, 64-bit register,
// job masks, bytes), the packed form (its pinned registers would cost the
// others occupancy).
constexpr int kParts = 2;
__host__ __device__ constexpr int part_of(int form) { return form == kSegPacked ? 1 : 0; }

// Variant = machine-count base (5, 10 or 20 machines) * kSegForms + form.
__host__ __device__ constexpr int variant(int mbase, int form) { return mbase * kSegForms + form; }

struct BatchSeg {
  InstView I;
  const uint8_t *nodes;
  int32_t *lb;
  int64_t count;
  int64_t tile_begin;  // first tile of this segment in the batch tile space
  int stride;
  int aligned;
  int variant;
  int tile_nodes;  // 256, or 512 in the packed form
};

constexpr size_t kWideBudget = 32 * 1024;
constexpr size_t kNarrowBudget = 64 * 1024;

__global__ void reset_counters(unsigned long long *c0, unsigned long long *c1) {
  if (threadIdx.x == 0 && c0) *c0 = 0ull;
  if (threadIdx.x == 1 && c1) *c1 = 0ull;
}

template <int M, int FORM, bool CHUNKED>
__device__ __forceinline__ void run_tile(const BatchSeg &S, char *smem,
                                         int64_t t, bool restage,
                                         char *tile_slots) {
  constexpr bool WIDE = FORM == kFormMasks || FORM == kFormBytes;
  constexpr bool BYTES = FORM == kFormBytes;
  const InstView I = S.I;
  const LdsView L = carve<WIDE, BYTES>(smem, I);
  if (restage) {
    stage_instance<WIDE, BYTES>(I, L);
    __syncthreads();
  }
  bound_nodes<M, FORM, CHUNKED>(I, L, S.nodes, S.stride, S.aligned != 0,
                                (t - S.tile_begin) * kBlock, S.count, S.lb,
                                tile_slots);
}

template <int M>
__device__ __forceinline__ void run_tile_p16(const BatchSeg &S, char *smem, int64_t t,
                                             bool restage) {
  const InstView I = S.I;
  const LdsView L = carve_p16(smem, I);
  if (restage) {
    stage_p16_rows(I, L);
    __syncthreads();
  }
  bound_nodes_p16<M, false>(I, L, S.nodes, S.stride, S.aligned != 0,
                            (t - S.tile_begin) * 2 * kBlock, S.count, S.lb);
}

template <int M, int KIND>
__device__ __forceinline__ void run_any(const BatchSeg &S, int form, char *smem, int64_t t,
                                        bool restage, char *ts) {
  if constexpr (KIND == 1) {
    run_tile_p16<M>(S, smem, t, restage);
  } else {
    switch (form) {
      case kSegReg32: run_tile<M, kFormReg32, false>(S, smem, t, restage, ts); break;
      case kSegMasks: run_tile<M, kFormMasks, false>(S, smem, t, restage, ts); break;
      case kSegMasksC: run_tile<M, kFormMasks, true>(S, smem, t, restage, ts); break;
      case kSegReg64: run_tile<M, kFormReg64, true>(S, smem, t, restage, ts); break;
      case kSegBytes: run_tile<M, kFormBytes, false>(S, smem, t, restage, ts); break;
      default: break;
    }
  }
}

// The packed segments run in a kernel of their own: the packed walk pins
// 48 VGPRs (its multipliers and load buffers), which in one kernel with the
// other forms cost those forms spills and a fifth of their speed.
// KIND: 0 the one-node forms, 1 packed.
template <int KIND>
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
    const int mbase = S.variant / kSegForms, form = S.variant - mbase * kSegForms;
    switch (mbase) {
      case 0: run_any<5, KIND>(S, form, smem, t, restage, ts); break;
      case 1: run_any<10, KIND>(S, form, smem, t, restage, ts); break;
      case 2: run_any<20, KIND>(S, form, smem, t, restage, ts); break;
      default: break;
    }
  }
}

int machine_base(int m) { return m == 5 ? 0 : m == 10 ? 1 : m == 20 ? 2 : -1; }

// The walk forms an instance's shape allows, the default (fastest in
// single-pool measurements) first.
std::vector<int> forms_for(const fsp_instance *inst, const InstView &v, bool allow_packed,
                           bool prefer_masks) {
  const int masks = v.nchunks > 1 ? kSegMasksC : kSegMasks;
  if (!inst->wide) {
    if (inst->p16 && allow_packed) return {kSegPacked, kSegReg32};
    return {kSegReg32};
  }
  if (!uses_job_masks(inst->n)) return {kSegReg64, masks};
  // the bytes walk by default; the job masks when the batch asks for them or
  // the instance was loaded for them
  if (prefer_masks || inst->masks_walk) return {masks, kSegBytes};
  return {kSegBytes, masks};
}

// Relative cost of one tile: table steps per node times nodes per tile times
// the walk's vector instructions per step (per node).
double tile_cost(const fsp_instance *in, int form) {
  static const double per_step[kSegForms] = {4.0, 3.0, 3.0, 5.0, 1.5, 4.0};
  const double nodes = form == kSegPacked ? 2.0 * kBlock : (double)kBlock;
  return (double)in->P * in->npad * nodes * per_step[form];
}

}  // namespace

// One persistent launch over a segment table: part 0 holds the one-node-per-
// lane forms, part 1 the packed form.
struct BatchPart {
  int nsegs = 0;
  int64_t total_tiles = 0;
  BatchSeg *d_segs = nullptr;
  unsigned long long *d_counter = nullptr;
  size_t lds = 0;
  int grid = 0;
};

struct fsp_batch {
  int device = 0;
  BatchPart part[kParts];
  char *d_slots = nullptr;  // job-mask scratch of part 0 and the fallbacks
  int64_t tile_bytes = 0;   // scratch bytes per tile of part 0
  std::vector<fsp_segment> fallback;  // bounded by single-pool launches
  std::vector<int32_t> path;  // per input segment: its FSP_PATH_* (-1: none)
  int blocks_per_cu = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int enqueue(fsp_batch *b, hipStream_t s) {
  const BatchPart &p0 = b->part[0], &p1 = b->part[1];
  if (p0.nsegs > 0 || p1.nsegs > 0) {
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, p0.d_counter, p1.d_counter);
    if (p0.nsegs > 0)
      hipLaunchKernelGGL(batch_kernel<0>, dim3(p0.grid), dim3(kBlock), p0.lds, s,
                         p0.d_segs, p0.nsegs, p0.total_tiles, p0.d_counter, b->d_slots,
                         b->tile_bytes);
    if (p1.nsegs > 0)
      hipLaunchKernelGGL(batch_kernel<1>, dim3(p1.grid), dim3(kBlock), p1.lds, s,
                         p1.d_segs, p1.nsegs, p1.total_tiles, p1.d_counter,
                         (char *)nullptr, (int64_t)0);
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
  for (BatchPart &p : b->part) {
    if (p.d_segs) (void)hipFree(p.d_segs);
    if (p.d_counter) (void)hipFree(p.d_counter);
  }
  if (b->d_slots) (void)hipFree(b->d_slots);
  delete b;
}

}  // namespace

namespace {

// Form choice per (n, m) shape: the form every segment of that shape takes.
using FormMap = std::map<std::pair<int, int>, int>;

int path_of_form(int form) {
  switch (form) {
    case kSegReg32: return FSP_PATH_REGISTER;
    case kSegPacked: return FSP_PATH_PACKED;
    case kSegReg64: return FSP_PATH_REGISTER64;
    case kSegBytes: return FSP_PATH_BYTES;
    default: return FSP_PATH_MASKS;
  }
}

// Plans a batch with the given form per shape (absent shapes: the default
// form) and workgroups per CU (<= 0: as many as fit).
int build(const fsp_segment *segs, int32_t nsegs, const FormMap &forms, int bpc,
          bool allow_packed, bool prefer_masks, fsp_batch **out) {
  *out = nullptr;
  fsp_batch *b = new (std::nothrow) fsp_batch();
  if (!b) return FSP_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    destroy(b);
    return FSP_EDEVICE;
  }
  b->path.assign(nsegs, -1);
  struct Item {
    BatchSeg s;
    double cost;
  };
  std::vector<Item> items;
  for (int i = 0; i < nsegs; ++i) {
    const fsp_segment &g = segs[i];
    if (g.count == 0) continue;
    const fsp_instance *in = g.inst;
    const int mb = machine_base(in->m);
    if (mb < 0) {
      b->fallback.push_back(g);
      continue;
    }
    Item it{};
    it.s.I = inst_view(in, in->wide ? kWideBudget : kNarrowBudget);
    const std::vector<int> allowed = forms_for(in, it.s.I, allow_packed, prefer_masks);
    int form = allowed[0];
    const auto f = forms.find({in->n, in->m});
    if (f != forms.end() &&
        std::find(allowed.begin(), allowed.end(), f->second) != allowed.end())
      form = f->second;
    b->path[i] = path_of_form(form);
    // the job-mask walk needs its per-wave slots also below 65 jobs (where
    // the instance's default form needs none); the bytes walk none, and its
    // own table budget
    if (form == kSegMasks || form == kSegMasksC) it.s.I.slot_bytes = mask_slot_bytes(in->n);
    if (part_of(form) == 2) {
      it.s.I = inst_view(in, table_budget_bytes(in->n));
      it.s.I.slot_bytes = 0;
    }
    it.s.variant = variant(mb, form);
    it.s.tile_nodes = form == kSegPacked ? 2 * kBlock : kBlock;
    it.s.nodes = g.data;
    it.s.lb = g.lb_out;
    it.s.count = g.count;
    it.s.stride = g.stride;
    it.s.aligned = ((reinterpret_cast<uintptr_t>(g.data) & 15) == 0 &&
                    (g.stride & 15) == 0)
                       ? 1
                       : 0;
    it.cost = tile_cost(in, form);
    items.push_back(it);
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const Item &a, const Item &c) { return a.cost > c.cost; });
  std::vector<BatchSeg> table[kParts];
  int64_t tiles[kParts] = {0, 0};
  size_t lds[kParts] = {16, 16};
  int slot_max = 0;
  for (const Item &it : items) slot_max = std::max(slot_max, it.s.I.slot_bytes);
  size_t scratch = 0;
  for (const fsp_segment &f : b->fallback)
    scratch = std::max(scratch, bound_scratch_bytes(f.inst->n, f.count));
  for (Item &it : items) {
    const int form = it.s.variant % kSegForms;
    const int k = part_of(form);
    it.s.tile_begin = tiles[k];
    tiles[k] += (it.s.count + it.s.tile_nodes - 1) / it.s.tile_nodes;
    const InstView &I = it.s.I;
    lds[k] = std::max(lds[k], k == 1 ? lds_bytes_p16(I.n, I.mp, I.npad, I.P)
                              : form == kSegBytes ? lds_bytes(I.n, I.mp, I.npad, I.ppc, true, true)
                                       : lds_bytes(I.n, I.mp, I.npad, I.ppc,
                                                   form == kSegMasks || form == kSegMasksC));
    table[k].push_back(it.s);
  }
  b->tile_bytes = (int64_t)(kBlock / 64) * slot_max;
  scratch = std::max(scratch, (size_t)(tiles[0] * b->tile_bytes));
  // every job-mask segment has slots of its size in every tile
  for (const BatchSeg &g : table[0]) {
    const int form = g.variant % kSegForms;
    if ((form == kSegMasks || form == kSegMasksC) &&
        (g.I.slot_bytes < mask_slot_bytes(g.I.n) ||
         b->tile_bytes < (kBlock / 64) * g.I.slot_bytes ||
         scratch < (size_t)(tiles[0] * b->tile_bytes))) {
      destroy(b);
      return FSP_EINVAL;
    }
  }
  if (scratch > 0 && hipMalloc(&b->d_slots, scratch) != hipSuccess) {
    destroy(b);
    return FSP_ENOMEM;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) !=
      hipSuccess) {
    destroy(b);
    return FSP_EDEVICE;
  }
  for (int k = 0; k < kParts; ++k) {
    BatchPart &p = b->part[k];
    p.nsegs = (int)table[k].size();
    p.total_tiles = tiles[k];
    p.lds = lds[k];
    if (p.nsegs == 0) continue;
    if (hipMalloc(&p.d_segs, table[k].size() * sizeof(BatchSeg)) != hipSuccess ||
        hipMalloc(&p.d_counter, sizeof(unsigned long long)) != hipSuccess) {
      destroy(b);
      return FSP_ENOMEM;
    }
    if (hipMemcpy(p.d_segs, table[k].data(), table[k].size() * sizeof(BatchSeg),
                  hipMemcpyHostToDevice) != hipSuccess) {
      destroy(b);
      return FSP_EDEVICE;
    }
    const void *fn = k == 0 ? reinterpret_cast<const void *>(batch_kernel<0>)
                            : reinterpret_cast<const void *>(batch_kernel<1>);
    int per_cu = 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, p.lds) !=
            hipSuccess) {
      destroy(b);
      return FSP_EDEVICE;
    }
    if (per_cu < 1) {
      destroy(b);
      return FSP_EUNSUPPORTED;
    }
    const int want = bpc > 0 ? std::min(per_cu, bpc) : per_cu;
    b->blocks_per_cu = std::max(b->blocks_per_cu, want);
    int64_t grid = (int64_t)want * cus;
    if (grid > tiles[k]) grid = tiles[k];
    p.grid = (int)std::max<int64_t>(1, grid);
  }
  *out = b;
  return FSP_OK;
}

// Seconds per launch of a planned batch (two warm-up launches, then five
// timed with HIP events on a private stream).
int time_batch(fsp_batch *b, double *secs) {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = FSP_OK;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = FSP_EDEVICE;
  for (int i = 0; i < 2 && rc == FSP_OK; ++i) rc = enqueue(b, s);
  if (rc == FSP_OK && hipEventRecord(e0, s) != hipSuccess) rc = FSP_EDEVICE;
  for (int i = 0; i < 5 && rc == FSP_OK; ++i) rc = enqueue(b, s);
  float ms = 0.f;
  if (rc == FSP_OK && (hipEventRecord(e1, s) != hipSuccess ||
                       hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = FSP_EDEVICE;
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *secs = ms * 1e-3 / 5;
  return rc;
}

// Autotuner caches: the form per (device, n, m, packed allowed), and the
// workgroups per CU per (device, batch signature).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_form_cache;
std::map<std::pair<int, std::vector<int64_t>>, int> g_bpc_cache;

int autotune(const fsp_segment *segs, int32_t nsegs, bool allow_packed, bool prefer_masks,
             FormMap *forms,
             int *bpc) {
  int dev = 0;
  FSP_HIP_TRY(hipGetDevice(&dev));
  // shapes and their segments
  std::map<std::pair<int, int>, std::vector<fsp_segment>> shapes;
  for (int i = 0; i < nsegs; ++i)
    if (segs[i].count > 0 && machine_base(segs[i].inst->m) >= 0)
      shapes[{segs[i].inst->n, segs[i].inst->m}].push_back(segs[i]);
  for (const auto &sh : shapes) {
    const fsp_instance *in = sh.second[0].inst;
    // the packed form also needs small times: decided per instance, so a
    // shape whose instances differ keeps the default
    bool mixed = false;
    for (const fsp_segment &g : sh.second) mixed = mixed || g.inst->p16 != in->p16;
    const InstView v = inst_view(in, in->wide ? kWideBudget : kNarrowBudget);
    const std::vector<int> allowed = forms_for(in, v, allow_packed, prefer_masks);
    if (allowed.size() < 2 || mixed) continue;
    const auto key = std::make_tuple(dev, sh.first.first, sh.first.second,
                                     (int)(allow_packed && in->p16));
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      const auto c = g_form_cache.find(key);
      if (c != g_form_cache.end()) {
        (*forms)[sh.first] = c->second;
        continue;
      }
    }
    int best = allowed[0];
    double best_t = 0.0;
    for (int form : allowed) {
      FormMap fm;
      fm[sh.first] = form;
      fsp_batch *b = nullptr;
      int rc = build(sh.second.data(), (int32_t)sh.second.size(), fm, 0, allow_packed,
                     prefer_masks, &b);
      double t = 0.0;
      if (rc == FSP_OK) rc = time_batch(b, &t);
      if (b) destroy(b);
      if (rc != FSP_OK) return rc;
      if (best_t == 0.0 || t < best_t) {
        best_t = t;
        best = form;
      }
    }
    (*forms)[sh.first] = best;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_form_cache[key] = best;
  }
  // signature of the batch under a form map: sorted (n, m, form, nodes
  // rounded up to a power of two) of its segments
  auto signature = [&](const FormMap &fm) {
    std::vector<int64_t> sig;
    for (int i = 0; i < nsegs; ++i) {
      if (segs[i].count == 0) continue;
      int64_t c = 1;
      while (c < segs[i].count) c <<= 1;
      const auto f = fm.find({segs[i].inst->n, segs[i].inst->m});
      sig.push_back(((int64_t)segs[i].inst->n << 48) | ((int64_t)segs[i].inst->m << 40) |
                    ((int64_t)(f == fm.end() ? 7 : f->second) << 36) | c);
    }
    std::sort(sig.begin(), sig.end());
    sig.push_back((int64_t)allow_packed << 1 | (int64_t)prefer_masks);
    return sig;
  };
  // workgroups per CU on the whole batch
  fsp_batch *probe = nullptr;
  int rc = build(segs, nsegs, *forms, 0, allow_packed, prefer_masks, &probe);
  if (rc != FSP_OK) return rc;
  const int max_bpc = probe->blocks_per_cu;
  destroy(probe);
  const auto bkey = std::make_pair(dev, signature(*forms));
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto c = g_bpc_cache.find(bkey);
    if (c != g_bpc_cache.end()) {
      *bpc = c->second;
      return FSP_OK;
    }
  }
  int best = max_bpc;
  double best_t = 0.0;
  for (int k = max_bpc; k >= 1; --k) {
    fsp_batch *b = nullptr;
    rc = build(segs, nsegs, *forms, k, allow_packed, prefer_masks, &b);
    double t = 0.0;
    if (rc == FSP_OK) rc = time_batch(b, &t);
    if (b) destroy(b);
    if (rc != FSP_OK) return rc;
    // a smaller grid is taken only when clearly faster
    if (best_t == 0.0 || t < 0.97 * best_t) {
      best_t = t;
      best = k;
    }
  }
  *bpc = best;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_bpc_cache[bkey] = best;
  return FSP_OK;
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
  if (cfg && (cfg->blocks_per_cu < 0 || (cfg->autotune != 0 && cfg->autotune != 1) ||
              (cfg->one_node_per_lane != 0 && cfg->one_node_per_lane != 1) ||
              (cfg->job_masks != 0 && cfg->job_masks != 1)))
    return FSP_EINVAL;
  const bool allow_packed = !(cfg && cfg->one_node_per_lane == 1);
  const bool prefer_masks = cfg && cfg->job_masks == 1;
  FormMap forms;
  int bpc = cfg ? cfg->blocks_per_cu : 0;
  if (cfg && cfg->autotune == 1) {
    int tuned = 0;
    const int rc = autotune(segs, nsegs, allow_packed, prefer_masks, &forms, &tuned);
    if (rc != FSP_OK) return rc;
    if (bpc <= 0) bpc = tuned;
  }
  return build(segs, nsegs, forms, bpc, allow_packed, prefer_masks, out);
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
  int64_t t = 0;
  int32_t g = 0, k = 0;
  for (const BatchPart &p : b->part) {
    t += p.total_tiles;
    g = std::max(g, (int32_t)p.grid);
    k += p.nsegs;
  }
  if (tiles) *tiles = t;
  if (grid) *grid = g;
  if (kernel_segments) *kernel_segments = k;
  if (fallback_segments) *fallback_segments = (int32_t)b->fallback.size();
  return FSP_OK;
}

int fsp_batch_paths(const fsp_batch *b, int32_t *paths, int32_t nsegs,
                    int32_t *blocks_per_cu) {
  if (!b || nsegs < 0 || (nsegs > 0 && !paths)) return FSP_EINVAL;
  if (nsegs != (int32_t)b->path.size()) return FSP_EINVAL;
  for (int i = 0; i < nsegs; ++i) paths[i] = b->path[i];
  if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu;
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
