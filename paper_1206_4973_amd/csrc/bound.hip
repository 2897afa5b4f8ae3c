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

#include "fsp_internal.hpp"

using namespace fspi;

namespace {

struct BoundParams {
  const uint8_t *nodes;
  int64_t count;
  int64_t ntiles;
  const int32_t *count_dev;  // when set, the node count is read from here
  int stride;
  int aligned;  // records 16-byte aligned: load them as uint4
  int32_t *lb;
  const int32_t *__restrict__ p;    // [n][mp] (global; staged to LDS)
  const int32_t *__restrict__ H;    // [n][mp]
  const int32_t *__restrict__ Q;    // [n][mp]
  const int32_t *__restrict__ tot;  // [mp]
  const void *__restrict__ rec;     // [P][npad]
  int n, mp, npad, P;
  int ppc;      // pairs per LDS chunk
  int nchunks;  // chunks of the pair table
};

constexpr int kBig = 1 << 20;  // > any head or tail sum (<= 65535)

template <int M>
__host__ __device__ constexpr int pair_index(int k, int l) {
  return k * (2 * M - k - 1) / 2 + (l - k - 1);
}

template <bool WIDE>
__device__ __forceinline__ void stage_chunk(const BoundParams &a, char *s_rec,
                                            int chunk) {
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  const int lo = chunk * a.ppc;
  const int hi = min(a.P, lo + a.ppc);
  const int total = (hi - lo) * a.npad;
  const Rec *src = reinterpret_cast<const Rec *>(a.rec) + (size_t)lo * a.npad;
  Rec *dst = reinterpret_cast<Rec *>(s_rec);
  for (int i = threadIdx.x; i < total; i += kBlock) dst[i] = src[i];
}

// One step of the two-machine walk (see the header comment):
//   z = max(z + alpha*x, alpha*y)
__device__ __forceinline__ int step(uint32_t al, int x, int y, int Z) {
  const int up = __mul24((int)al, x) + Z;
  const int lo = (int)__umul24(al, (uint32_t)y);
  return max(up, lo);
}

template <bool WIDE>
__device__ __forceinline__ uint32_t member(uint32_t U, const uint8_t *alpha_lane,
                                           int y, int job) {
  if constexpr (WIDE)
    return alpha_lane[(uint32_t)job << kLogBlock];
  else
    return __builtin_amdgcn_ubfe(U, (uint32_t)y, 1u);  // job = y & 31
}

// Walk of one pair over its Johnson order (npad records in LDS at rp).
template <bool WIDE>
__device__ __forceinline__ int walk1(const char *rp_raw, int npad, uint32_t U,
                                     const uint8_t *alpha_lane, int Z) {
  if constexpr (!WIDE) {
    const int4 *rp = reinterpret_cast<const int4 *>(rp_raw);  // 2 records
    for (int i = 0; i < npad / 2; i += 2) {
      const int4 r0 = rp[i], r1 = rp[i + 1];
      Z = step(member<false>(U, nullptr, r0.y, 0), r0.x, r0.y, Z);
      Z = step(member<false>(U, nullptr, r0.w, 0), r0.z, r0.w, Z);
      Z = step(member<false>(U, nullptr, r1.y, 0), r1.x, r1.y, Z);
      Z = step(member<false>(U, nullptr, r1.w, 0), r1.z, r1.w, Z);
    }
  } else {
    const int4 *rp = reinterpret_cast<const int4 *>(rp_raw);
    for (int i = 0; i < npad; i += 2) {
      const int4 r0 = rp[i], r1 = rp[i + 1];
      Z = step(member<true>(0, alpha_lane, r0.y, r0.z), r0.x, r0.y, Z);
      Z = step(member<true>(0, alpha_lane, r1.y, r1.z), r1.x, r1.y, Z);
    }
  }
  return Z;
}

// Two pairs walked together: two independent dependency chains per lane.
template <bool WIDE>
__device__ __forceinline__ void walk2(const char *ra_raw, const char *rb_raw,
                                      int npad, uint32_t U,
                                      const uint8_t *alpha_lane, int &ZA,
                                      int &ZB) {
  if constexpr (!WIDE) {
    const int4 *ra = reinterpret_cast<const int4 *>(ra_raw);
    const int4 *rb = reinterpret_cast<const int4 *>(rb_raw);
    for (int i = 0; i < npad / 2; i += 2) {
      const int4 a0 = ra[i], a1 = ra[i + 1];
      const int4 b0 = rb[i], b1 = rb[i + 1];
      ZA = step(member<false>(U, nullptr, a0.y, 0), a0.x, a0.y, ZA);
      ZB = step(member<false>(U, nullptr, b0.y, 0), b0.x, b0.y, ZB);
      ZA = step(member<false>(U, nullptr, a0.w, 0), a0.z, a0.w, ZA);
      ZB = step(member<false>(U, nullptr, b0.w, 0), b0.z, b0.w, ZB);
      ZA = step(member<false>(U, nullptr, a1.y, 0), a1.x, a1.y, ZA);
      ZB = step(member<false>(U, nullptr, b1.y, 0), b1.x, b1.y, ZB);
      ZA = step(member<false>(U, nullptr, a1.w, 0), a1.z, a1.w, ZA);
      ZB = step(member<false>(U, nullptr, b1.w, 0), b1.z, b1.w, ZB);
    }
  } else {
    const int4 *ra = reinterpret_cast<const int4 *>(ra_raw);
    const int4 *rb = reinterpret_cast<const int4 *>(rb_raw);
    for (int i = 0; i < npad; i += 2) {
      const int4 a0 = ra[i], a1 = ra[i + 1];
      const int4 b0 = rb[i], b1 = rb[i + 1];
      ZA = step(member<true>(0, alpha_lane, a0.y, a0.z), a0.x, a0.y, ZA);
      ZB = step(member<true>(0, alpha_lane, b0.y, b0.z), b0.x, b0.y, ZB);
      ZA = step(member<true>(0, alpha_lane, a1.y, a1.z), a1.x, a1.y, ZA);
      ZB = step(member<true>(0, alpha_lane, b1.y, b1.z), b1.x, b1.y, ZB);
    }
  }
}

// Every pair whose index lies in [lo, hi): pairs (k,l) and (k,l+1) are walked
// together.  Returns the max over those pairs of 256*(pair bound) + junk.
// The record pointer advances pair by pair (pair index order = table order)
// so that no per-pair address stays live.
template <int M, bool WIDE>
__device__ __forceinline__ int pair_sweep(const char *s_rec, int lo, int hi,
                                          int npad, uint32_t U,
                                          const uint8_t *alpha_lane,
                                          const int (&R256)[M],
                                          const int (&T256)[M],
                                          const int (&Q256)[M], int LB256) {
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  int pb = npad * (int)sizeof(Rec);
  // Opaque per call: otherwise every per-pair offset is loop-invariant in the
  // tile loop and gets hoisted, one scalar register per pair.
  asm volatile("" : "+s"(pb));
  uint32_t off = 0;  // byte offset of pair index `pa - lo` (wraps below lo)
  off -= (uint32_t)(lo * pb);
#pragma unroll
  for (int k = 0; k < M - 1; ++k) {
#pragma unroll
    for (int l = k + 1; l < M; l += 2) {
      const int pa = pair_index<M>(k, l);
      if (l + 1 < M) {
        const bool ina = pa >= lo && pa < hi, inb = pa + 1 >= lo && pa + 1 < hi;
        if (ina && inb) {
          int ZA = R256[l] - R256[k], ZB = R256[l + 1] - R256[k];
          walk2<WIDE>(s_rec + off, s_rec + off + pb, npad, U, alpha_lane, ZA,
                      ZB);
          LB256 = max(LB256, max(T256[k] + Q256[l] + ZA,
                                 T256[k] + Q256[l + 1] + ZB));
          // keep the max chain sequential (a reassociated max tree would hold
          // one partial result per pair)
          asm volatile("" : "+v"(LB256));
        } else {
          if (ina) {
            int Z = walk1<WIDE>(s_rec + off, npad, U, alpha_lane,
                                R256[l] - R256[k]);
            LB256 = max(LB256, T256[k] + Q256[l] + Z);
            asm volatile("" : "+v"(LB256));
          }
          if (inb) {
            int Z = walk1<WIDE>(s_rec + off + pb, npad, U, alpha_lane,
                                R256[l + 1] - R256[k]);
            LB256 = max(LB256, T256[k] + Q256[l + 1] + Z);
            asm volatile("" : "+v"(LB256));
          }
        }
        off += 2 * pb;
      } else {
        if (pa >= lo && pa < hi) {
          int Z = walk1<WIDE>(s_rec + off, npad, U, alpha_lane,
                              R256[l] - R256[k]);
          LB256 = max(LB256, T256[k] + Q256[l] + Z);
          asm volatile("" : "+v"(LB256));
        }
        off += pb;
      }
    }
  }
  return LB256;
}

template <int M, bool WIDE, bool CHUNKED>
__global__ __launch_bounds__(kBlock, 4) void bound_kernel(const BoundParams a) {
  extern __shared__ __align__(16) char smem[];
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  const int tid = threadIdx.x;
  const int n = a.n, mp = a.mp, npad = a.npad;
  char *s_rec = smem;
  const size_t rec_bytes = (size_t)a.ppc * npad * sizeof(Rec);
  int32_t *s_p = reinterpret_cast<int32_t *>(smem + rec_bytes);
  uint8_t *s_alpha =
      reinterpret_cast<uint8_t *>(s_p + (size_t)n * mp);  // [n][kBlock] (WIDE)
  uint8_t *alpha_lane = s_alpha + tid;

  for (int i = tid; i < n * mp; i += kBlock) s_p[i] = a.p[i];
  if (!CHUNKED) stage_chunk<WIDE>(a, s_rec, 0);
  __syncthreads();

  const uint32_t full = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
  int64_t count = a.count, ntiles = a.ntiles;
  if (a.count_dev) {
    count = *a.count_dev;
    ntiles = (count + kBlock - 1) / kBlock;
  }

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t idx = tile * kBlock + tid;
    const bool live = idx < count;

    // ---- 1. decode the prefix, front recurrence, prefix column sums ----
    int F[M], Pk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) F[k] = Pk[k] = 0;
    uint32_t U = full;
    if constexpr (WIDE)
      for (int j = 0; j < n; ++j) alpha_lane[j << kLogBlock] = 1;
    bool bad = false;
    int d = 0;
    if (live) {
      const uint8_t *rp = a.nodes + idx * (int64_t)a.stride;
      d = rp[0];
      if (d > n) {
        bad = true;
        d = 0;
      }
      for (int c = 0; c * 16 <= d; ++c) {
        uint32_t w[4];
        if (a.aligned) {
          const uint4 v = *reinterpret_cast<const uint4 *>(rp + c * 16);
          w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            uint32_t acc = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int o = c * 16 + q * 4 + b;
              const uint32_t v = o < a.stride ? rp[o] : 0u;
              acc |= v << (8 * b);
            }
            w[q] = acc;
          }
        }
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          const int pos = c * 16 + b;
          if (pos >= 1 && pos <= d) {
            const int j = (w[b >> 2] >> (8 * (b & 3))) & 0xff;
            if (j >= n) {
              bad = true;
              continue;
            }
            if constexpr (WIDE) {
              if (!alpha_lane[j << kLogBlock]) bad = true;
              alpha_lane[j << kLogBlock] = 0;
            } else {
              if (!((U >> j) & 1u)) bad = true;
              U &= ~(1u << j);
            }
            const int32_t *row = s_p + j * mp;
            F[0] += row[0];
            Pk[0] += row[0];
#pragma unroll
            for (int k = 1; k < M; ++k) {
              F[k] = max(F[k], F[k - 1]) + row[k];
              Pk[k] += row[k];
            }
          }
        }
      }
    }

    // ---- 2. heads, remaining work, tails (two passes over the jobs, so
    //         that only 60 per-node values are live at a time) ----
    int T256[M], R256[M], Q256[M];
    {
      int hm[M];
#pragma unroll
      for (int k = 0; k < M; ++k) hm[k] = kBig;
      for (int j = 0; j < n; ++j) {
        uint32_t gone;
        if constexpr (WIDE)
          gone = 1u - alpha_lane[j << kLogBlock];
        else
          gone = __builtin_amdgcn_ubfe(~U, (uint32_t)j, 1u);
        const int32_t *hr = a.H + j * mp;
#pragma unroll
        for (int k = 0; k < M; ++k)
          hm[k] = min(hm[k], (int)__umul24(gone, kBig) + hr[k]);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int r = max(F[k], F[0] + hm[k]);
        R256[k] = r << 8;
        T256[k] = (r + a.tot[k] - Pk[k]) << 8;
      }
    }
    const int last = F[M - 1];
    {
#pragma unroll
      for (int k = 0; k < M; ++k) Q256[k] = kBig;
      for (int j = 0; j < n; ++j) {
        uint32_t gone;
        if constexpr (WIDE)
          gone = 1u - alpha_lane[j << kLogBlock];
        else
          gone = __builtin_amdgcn_ubfe(~U, (uint32_t)j, 1u);
        const int32_t *qr = a.Q + j * mp;
#pragma unroll
        for (int k = 0; k < M; ++k)
          Q256[k] = min(Q256[k], (int)__umul24(gone, kBig) + qr[k]);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) Q256[k] <<= 8;
    }

    // ---- 3. every machine pair ----
    int LB256 = 0;
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int k = 0; k < M; ++k)
        asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
      LB256 = pair_sweep<M, WIDE>(s_rec, 0, M * (M - 1) / 2, npad, U,
                                  alpha_lane, R256, T256, Q256, LB256);
    } else {
      for (int chunk = 0; chunk < a.nchunks; ++chunk) {
        __syncthreads();
        stage_chunk<WIDE>(a, s_rec, chunk);
        __syncthreads();
        // keep the per-node values from being re-derived per pair outside
        // the chunk loop (which would cost a register per pair)
#pragma unroll
        for (int k = 0; k < M; ++k)
          asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
        int lo = chunk * a.ppc, hi = lo + a.ppc;
        asm volatile("" : "+s"(lo), "+s"(hi));
        LB256 = pair_sweep<M, WIDE>(s_rec, lo, hi, npad, U, alpha_lane, R256,
                                    T256, Q256, LB256);
      }
    }

    // ---- 4. result ----
    int u_left;
    if constexpr (WIDE) {
      u_left = n - d;
    } else {
      u_left = __builtin_popcount(U);
    }
    int lb = u_left == 0 ? last : (LB256 >> 8);
    if (bad) lb = FSP_LB_INVALID;
    if (live) a.lb[idx] = lb;
  }
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

// LDS budget of one workgroup for the pair table.
constexpr size_t kTableBudget = 64 * 1024;

}  // namespace

namespace fspi {

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
  a.p = inst->d_p;
  a.H = inst->d_H;
  a.Q = inst->d_Q;
  a.tot = inst->d_tot;
  a.rec = inst->d_rec;
  a.n = inst->n;
  a.mp = inst->mp;
  a.npad = inst->npad;
  a.P = inst->P;
  const size_t rsz = wide ? sizeof(WideRec) : sizeof(NarrowRec);
  const size_t per_pair = (size_t)inst->npad * rsz;
  int ppc = (int)(kTableBudget / per_pair);
  if (ppc < 1) ppc = 1;
  if (ppc > inst->P) ppc = inst->P;
  a.ppc = ppc;
  a.nchunks = (inst->P + ppc - 1) / ppc;
  BoundFn fn = kernel_for(inst->m, wide, a.nchunks > 1);
  if (!fn) return FSP_EUNSUPPORTED;
  size_t lds = (size_t)ppc * per_pair + (size_t)inst->n * inst->mp * 4;
  if (wide) lds += (size_t)inst->n * kBlock;
  lds = (lds + 15) & ~size_t(15);

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
