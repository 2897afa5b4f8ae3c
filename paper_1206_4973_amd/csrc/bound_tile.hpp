// bound_tile.hpp -- the per-tile body of the pool-bounding kernels, shared
// by the single-pool kernel (bound.hip) and the multi-instance batch kernel
// (batch.hip).  See bound.hip for the method and the encoding of the table.
#pragma once
#include <type_traits>

#include "fsp_internal.hpp"

namespace fspi {

// Everything the bound needs about one instance (device pointers).
struct InstView {
  const int32_t *__restrict__ p;    // [n][mp]
  const uint32_t *__restrict__ Hp;  // [n][mp/2] head sums, packed 16-bit pairs
  const uint32_t *__restrict__ Qp;  // [n][mp/2] tail sums, packed 16-bit pairs
  const int32_t *__restrict__ tot;  // [mp]
  const void *__restrict__ rec;     // [P][npad]
  int n, mp, npad, P;
  int ppc;      // pairs per LDS chunk
  int nchunks;  // chunks of the pair table
};

// LDS of one workgroup for one instance: the table chunk, then (n <= 32)
// the p matrix for the prefix recurrence, or (n > 32) the unscheduled-job
// mask of every lane as ceil(n/32) words laid out [word][lane].
struct LdsView {
  char *s_rec;
  int32_t *s_p;       // narrow only
  uint32_t *s_words;  // wide only
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <int M>
__host__ __device__ constexpr int pair_index(int k, int l) {
  return k * (2 * M - k - 1) / 2 + (l - k - 1);
}

__host__ __device__ inline size_t lds_bytes(int n, int mp, int npad, int ppc,
                                            bool wide) {
  const size_t rsz = wide ? sizeof(WideRec) : sizeof(NarrowRec);
  size_t b = (size_t)ppc * npad * rsz;
  if (wide)
    b += (size_t)((n + 31) / 32) * kBlock * 4;
  else
    b += (size_t)n * mp * 4;
  return (b + 15) & ~size_t(15);
}

template <bool WIDE>
__device__ __forceinline__ LdsView carve(char *smem, const InstView I) {
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  LdsView L;
  L.s_rec = smem;
  char *after = smem + (size_t)I.ppc * I.npad * sizeof(Rec);
  L.s_p = WIDE ? nullptr : reinterpret_cast<int32_t *>(after);
  L.s_words = WIDE ? reinterpret_cast<uint32_t *>(after) : nullptr;
  return L;
}

template <bool WIDE>
__device__ __forceinline__ void stage_chunk(const InstView I, char *s_rec,
                                            int chunk) {
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  const int lo = chunk * I.ppc;
  const int hi = min(I.P, lo + I.ppc);
  const int total = (hi - lo) * I.npad;
  const Rec *src = reinterpret_cast<const Rec *>(I.rec) + (size_t)lo * I.npad;
  Rec *dst = reinterpret_cast<Rec *>(s_rec);
  for (int i = threadIdx.x; i < total; i += kBlock) dst[i] = src[i];
}

// Stage what stays in LDS for the whole instance: p, and the whole pair table
// when it fits.  The caller synchronises the workgroup afterwards.
template <bool WIDE>
__device__ __forceinline__ void stage_instance(const InstView I,
                                               const LdsView &L) {
  if (!WIDE)
    for (int i = threadIdx.x; i < I.n * I.mp; i += kBlock) L.s_p[i] = I.p[i];
  if (I.nchunks == 1) stage_chunk<WIDE>(I, L.s_rec, 0);
}

// One step of the two-machine walk (see the header comment):
//   z = max(z + alpha*x, alpha*y)
__device__ __forceinline__ int step(uint32_t al, int x, int y, int Z) {
  const int up = __mul24((int)al, x) + Z;
  const int lo = (int)__umul24(al, (uint32_t)y);
  return max(up, lo);
}

// Membership bit of the record's job in this lane's unscheduled set.  The
// low 5 bits of y are the job's bit within its 32-job word; wide records
// carry the byte offset of the word (in the [word][lane] LDS layout).
template <bool WIDE>
__device__ __forceinline__ uint32_t member(uint32_t U, const char *words_lane,
                                           int y, int woff) {
  if constexpr (WIDE) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(words_lane + woff);
    return __builtin_amdgcn_ubfe(w, (uint32_t)y, 1u);
  } else {
    return __builtin_amdgcn_ubfe(U, (uint32_t)y, 1u);  // job = y & 31
  }
}

// Walk of one pair over its Johnson order (npad records in LDS at rp).
template <bool WIDE>
__device__ __forceinline__ int walk1(const char *rp_raw, int npad, uint32_t U,
                                     const char *alpha_lane, int Z) {
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
                                      const char *alpha_lane, int &ZA,
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
                                          const char *alpha_lane,
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
        // wide tables: one chain per pair (the membership bytes come from LDS
        // and two chains would not fit the register budget)
        if (!WIDE && ina && inb) {
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

// Bound the 256 nodes [base, base + 256) of a pool (one per lane), writing
// lb_out[idx] for idx < count.  Every lane of the workgroup must call it (the
// chunked form synchronises the workgroup).
template <int M, bool WIDE, bool CHUNKED>
__device__ __forceinline__ void bound_nodes(const InstView I, const LdsView &L,
                                            const uint8_t *nodes, int stride,
                                            bool aligned, int64_t base,
                                            int64_t count, int32_t *lb_out) {
  using Rec = typename std::conditional<WIDE, WideRec, NarrowRec>::type;
  const int tid = threadIdx.x;
  const int n = I.n, mp = I.mp, npad = I.npad;
  char *s_rec = L.s_rec;
  const int32_t *s_p = L.s_p;
  uint32_t *words_lane = WIDE ? L.s_words + tid : nullptr;
  const char *alpha_lane = reinterpret_cast<const char *>(words_lane);
  const uint32_t full = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
  const int64_t idx = base + tid;
  const bool live = idx < count;
  (void)sizeof(Rec);

  // ---- 1. decode the prefix, front recurrence, prefix column sums ----
  int F[M], Pk[M];
#pragma unroll
  for (int k = 0; k < M; ++k) F[k] = Pk[k] = 0;
  uint32_t U = full;
  if constexpr (WIDE)
    for (int w = 0; w * 32 < n; ++w)
      words_lane[w * kBlock] = n - w * 32 >= 32 ? 0xffffffffu
                                                 : ((1u << (n - w * 32)) - 1u);
  bool bad = false;
  int d = 0;
  if (live) {
    const uint8_t *rp = nodes + idx * (int64_t)stride;
    d = rp[0];
    if (d > n) {
      bad = true;
      d = 0;
    }
    for (int c = 0; c * 16 <= d; ++c) {
      uint32_t w[4];
      if (aligned) {
        const uint4 v = *reinterpret_cast<const uint4 *>(rp + c * 16);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t acc = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int o = c * 16 + q * 4 + b;
            const uint32_t v = o < stride ? rp[o] : 0u;
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
            uint32_t *wp = words_lane + (j >> 5) * kBlock;
            const uint32_t v = *wp, bit = 1u << (j & 31);
            if (!(v & bit)) bad = true;
            *wp = v & ~bit;
          } else {
            if (!((U >> j) & 1u)) bad = true;
            U &= ~(1u << j);
          }
          const int32_t *row = WIDE ? I.p + j * mp : s_p + j * mp;
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

  // ---- 2. heads, tails, remaining work.  Head and tail sums are at most
  //         65535 (instance limits), so the minima over the unscheduled jobs
  //         run on packed 16-bit pairs of machines: a scheduled job's pair is
  //         forced to 0xffff by an unsigned max with its all-ones sign mask,
  //         then one unsigned min per pair of machines. ----
  int T256[M], R256[M], Q256[M];
  {
    constexpr int M2 = (M + 1) / 2;
    u16x2 hm2[M2], qm2[M2];
#pragma unroll
    for (int t = 0; t < M2; ++t) hm2[t] = qm2[t] = (u16x2){0xffff, 0xffff};
    const int mp2 = mp / 2;
    for (int j = 0; j < n; ++j) {
      uint32_t g;
      if constexpr (WIDE)
        g = (uint32_t)__builtin_amdgcn_sbfe((int)~words_lane[(j >> 5) * kBlock], j & 31, 1);
      else
        g = (uint32_t)__builtin_amdgcn_sbfe((int)~U, j, 1);
      const u16x2 gv = __builtin_bit_cast(u16x2, g);
      const uint32_t *hr = I.Hp + j * mp2;
      const uint32_t *qr = I.Qp + j * mp2;
#pragma unroll
      for (int t = 0; t < M2; ++t) {
        hm2[t] = __builtin_elementwise_min(
            hm2[t], __builtin_elementwise_max(__builtin_bit_cast(u16x2, hr[t]), gv));
        qm2[t] = __builtin_elementwise_min(
            qm2[t], __builtin_elementwise_max(__builtin_bit_cast(u16x2, qr[t]), gv));
      }
    }
    // the column totals are loaded here, not hoisted above the loop
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int hmk = (k & 1) ? hm2[k >> 1].y : hm2[k >> 1].x;
      const int qmk = (k & 1) ? qm2[k >> 1].y : qm2[k >> 1].x;
      const int r = max(F[k], F[0] + hmk);
      R256[k] = r << 8;
      T256[k] = (r + I.tot[k] - Pk[k]) << 8;
      Q256[k] = qmk << 8;
    }
  }
  const int last = F[M - 1];

  // ---- 3. every machine pair ----
  int LB256 = 0;
  if constexpr (!CHUNKED) {
#pragma unroll
    for (int k = 0; k < M; ++k)
      asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
    LB256 = pair_sweep<M, WIDE>(s_rec, 0, M * (M - 1) / 2, npad, U,
                                alpha_lane, R256, T256, Q256, LB256);
  } else {
    for (int chunk = 0; chunk < I.nchunks; ++chunk) {
      __syncthreads();
      stage_chunk<WIDE>(I, s_rec, chunk);
      __syncthreads();
      // keep the per-node values from being re-derived per pair outside
      // the chunk loop (which would cost a register per pair)
#pragma unroll
      for (int k = 0; k < M; ++k)
        asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
      int lo = chunk * I.ppc, hi = lo + I.ppc;
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
  if (live) lb_out[idx] = lb;
}

// InstView of a loaded instance with the pair table split into LDS chunks of
// at most table_budget bytes (bound.hip).
InstView inst_view(const fsp_instance *inst, size_t table_budget);

}  // namespace fspi
