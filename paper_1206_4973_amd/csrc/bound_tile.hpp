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
  const Rec *__restrict__ rec;       // [P][npad] {x, y} per table position
  const uint32_t *__restrict__ joff; // [P][npad] 8 * job id per position
  const uint32_t *__restrict__ xy16;  // packed form: [P][npad] x | y << 16
  const uint32_t *__restrict__ job16; // packed form: [P][npad] job id
  const uint32_t *__restrict__ bxy;   // bytes form: [P][npad8] x | y << 16
  const uint8_t *__restrict__ bjob;   // bytes form: [P][npad8] job id
  int n, mp, npad, P;
  int npad8;       // bytes form: n rounded up to 8
  int ppc;         // pairs per LDS chunk
  int nchunks;     // chunks of the pair table
  int slot_bytes;  // bytes of one wave's mask slot (mask_slot_bytes(n))
};

// LDS of one workgroup for one instance: the table chunk, then (n <= 32)
// the p matrix for the prefix recurrence, or (n > 32) the unscheduled-job
// mask of every lane as ceil(n/32) words laid out [word][lane]; in the bytes
// form only the same flags as bytes, [wave][job 0 .. n][lane].
struct LdsView {
  char *s_rec;
  int32_t *s_p;       // narrow only
  uint32_t *s_words;  // wide only
  uint8_t *s_alpha;   // bytes form only
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Forms of the one-node-per-lane walk (see the header comment of bound.hip).
enum Form : int {
  kFormReg32 = 0,  // n <= 32: unscheduled set in one register
  kFormMasks = 1,  // n > 32: per-wave job masks read by scalar loads
  kFormReg64 = 2,  // 32 < n <= 64: unscheduled set in a 64-bit register pair
  kFormBytes = 3,  // n > 32: unscheduled flags of the lanes as bytes in LDS
};

// Read-only views through the constant address space: loads from these with
// a wave-uniform address are scalar loads whose result lands in SGPRs.
typedef const __attribute__((address_space(4))) char kchar;
typedef const __attribute__((address_space(4))) uint32_t ku32;
typedef const __attribute__((address_space(4))) uint64_t ku64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) u32x4 ku128;

template <int M>
__host__ __device__ constexpr int pair_index(int k, int l) {
  return k * (2 * M - k - 1) / 2 + (l - k - 1);
}

// Row pitch (32-bit words) of the packed rows of p in LDS: mp / 2 rounded
// up to 16 bytes, so that a row is read with 16-byte loads.
__host__ __device__ constexpr int p16_row_words(int mp) { return (mp / 2 + 3) & ~3; }

// Bytes of the bytes form's flag rows: one byte per lane for jobs 0 .. n.
__host__ __device__ inline size_t alpha_bytes(int n) { return (size_t)kBlock * (n + 1); }

// The bytes walk's table budget (inst_view's): its records and flag offsets
// are read from global memory, so the whole table is one chunk and none of
// it is staged in LDS.
inline size_t table_budget_bytes(int) { return (size_t)1 << 40; }

__host__ __device__ inline size_t lds_bytes(int n, int mp, int npad, int ppc,
                                            bool wide, bool bytes = false) {
  // the bytes walk stages no records
  size_t b = bytes ? 0 : (size_t)ppc * npad * sizeof(Rec);
  if (bytes)
    b += alpha_bytes(n);  // the flag bytes stand in for the job words
  else if (wide)
    b += (size_t)((n + 31) / 32) * kBlock * 4;
  else {  // 32-bit rows of p, or the packed rows plus a row of zeros
    const int rows32 = n * mp, rows16 = (n + 1) * p16_row_words(mp);
    b += (size_t)(rows32 > rows16 ? rows32 : rows16) * 4;
  }
  return (b + 15) & ~size_t(15);
}

template <bool WIDE, bool BYTES = false>
__device__ __forceinline__ LdsView carve(char *smem, const InstView I) {
  LdsView L;
  L.s_rec = BYTES ? nullptr : smem;
  char *after = BYTES ? smem : smem + (size_t)I.ppc * I.npad * sizeof(Rec);
  L.s_p = WIDE ? nullptr : reinterpret_cast<int32_t *>(after);
  L.s_words = WIDE && !BYTES ? reinterpret_cast<uint32_t *>(after) : nullptr;
  L.s_alpha = BYTES ? reinterpret_cast<uint8_t *>(after) : nullptr;
  return L;
}

__device__ __forceinline__ void stage_chunk(const InstView I, char *s_rec,
                                            int chunk) {
  const int lo = chunk * I.ppc;
  const int hi = min(I.P, lo + I.ppc);
  const int total = (hi - lo) * I.npad;
  const Rec *src = I.rec + (size_t)lo * I.npad;
  Rec *dst = reinterpret_cast<Rec *>(s_rec);
  for (int i = threadIdx.x; i < total; i += kBlock) dst[i] = src[i];
}

// Stage what stays in LDS for the whole instance: p, and the whole pair table
// when it fits.  The caller synchronises the workgroup afterwards.
template <bool WIDE, bool BYTES = false>
__device__ __forceinline__ void stage_instance(const InstView I,
                                               const LdsView &L) {
  if (!WIDE)
    for (int i = threadIdx.x; i < I.n * I.mp; i += kBlock) L.s_p[i] = I.p[i];
  if (!BYTES && I.nchunks == 1) stage_chunk(I, L.s_rec, 0);
}

// Write the wave's job masks: entry j of the slot is the 64-bit set of lanes
// whose node still has job j unscheduled; entries n .. end of slot are zero
// (the padding positions of the table point at entry n).  One ballot per job
// transposes the lanes' job sets; lane t then stores the mask of job 64c + t.
// Every lane of the wave calls it.
template <bool WIDE>
__device__ __forceinline__ void write_masks(uint64_t *slot, int n,
                                            int slot_bytes, uint32_t U,
                                            const uint32_t *words_lane) {
  const int lane = (int)__lane_id();
  const int entries = slot_bytes / 8;
  for (int c = 0; c * 64 < entries; ++c) {
    uint64_t mine = 0;
    const int jend = min(n, c * 64 + 64);
    for (int j = c * 64; j < jend; ++j) {
      uint32_t bit;
      if constexpr (WIDE)
        bit = (words_lane[(j >> 5) * kBlock] >> (j & 31)) & 1u;
      else
        bit = (U >> j) & 1u;
      const uint64_t mk = __ballot(bit);
      if (lane == j - c * 64) mine = mk;
    }
    if (c * 64 + lane < entries) slot[c * 64 + lane] = mine;
  }
}

// ---- n <= 32: the node's unscheduled jobs are one 32-bit register ----
// One position: alpha = bit `job` of U (job = low 5 bits of y), then
//   z = max(z + alpha*x, alpha*y)
// which leaves z unchanged for alpha = 0 because z >= 0.
__device__ __forceinline__ int step_u(uint32_t U, int x, int y, int Z) {
  const uint32_t al = __builtin_amdgcn_ubfe(U, (uint32_t)y, 1u);
  const int up = __mul24((int)al, x) + Z;
  const int lo = (int)__umul24(al, (uint32_t)y);
  return max(up, lo);
}

__device__ __forceinline__ int walk1_u(const char *rp_raw, int npad, uint32_t U,
                                       int Z) {
  const int4 *rp = reinterpret_cast<const int4 *>(rp_raw);  // 2 records
  for (int i = 0; i < npad / 4; ++i) {
    const int4 r0 = rp[2 * i], r1 = rp[2 * i + 1];
    Z = step_u(U, r0.x, r0.y, Z);
    Z = step_u(U, r0.z, r0.w, Z);
    Z = step_u(U, r1.x, r1.y, Z);
    Z = step_u(U, r1.z, r1.w, Z);
  }
  return Z;
}

__device__ __forceinline__ void walk2_u(const char *ra_raw, const char *rb_raw,
                                        int npad, uint32_t U, int &ZA,
                                        int &ZB) {
  const int4 *ra = reinterpret_cast<const int4 *>(ra_raw);
  const int4 *rb = reinterpret_cast<const int4 *>(rb_raw);
  for (int i = 0; i < npad / 4; ++i) {
    const int4 a0 = ra[2 * i], a1 = ra[2 * i + 1];
    const int4 b0 = rb[2 * i], b1 = rb[2 * i + 1];
    ZA = step_u(U, a0.x, a0.y, ZA);
    ZB = step_u(U, b0.x, b0.y, ZB);
    ZA = step_u(U, a0.z, a0.w, ZA);
    ZB = step_u(U, b0.z, b0.w, ZB);
    ZA = step_u(U, a1.x, a1.y, ZA);
    ZB = step_u(U, b1.x, b1.y, ZB);
    ZA = step_u(U, a1.z, a1.w, ZA);
    ZB = step_u(U, b1.z, b1.w, ZB);
  }
}

// ---- 32 < n <= 64: the node's unscheduled jobs are a 64-bit register pair ----
// alpha = bit `job` of U, taken by a 64-bit shift by y (the shift uses the low
// 6 bits of y, which hold the job id) and an and; then the same three
// operations as above: 5 VALU per position and no memory access besides the
// LDS record.
__device__ __forceinline__ int step_u64(uint64_t U, int x, int y, int Z) {
  uint64_t sh;
  asm("v_lshrrev_b64 %0, %1, %2" : "=v"(sh) : "v"(y), "v"(U));
  const uint32_t al = (uint32_t)sh & 1u;
  const int up = __mul24((int)al, x) + Z;
  const int lo = (int)__umul24(al, (uint32_t)y);
  return max(up, lo);
}

__device__ __forceinline__ int walk1_u64(const char *rp_raw, int npad, uint64_t U,
                                         int Z) {
  const int4 *rp = reinterpret_cast<const int4 *>(rp_raw);  // 2 records
  for (int i = 0; i < npad / 4; ++i) {
    const int4 r0 = rp[2 * i], r1 = rp[2 * i + 1];
    Z = step_u64(U, r0.x, r0.y, Z);
    Z = step_u64(U, r0.z, r0.w, Z);
    Z = step_u64(U, r1.x, r1.y, Z);
    Z = step_u64(U, r1.z, r1.w, Z);
  }
  return Z;
}

__device__ __forceinline__ void walk2_u64(const char *ra_raw, const char *rb_raw,
                                          int npad, uint64_t U, int &ZA, int &ZB) {
  const int4 *ra = reinterpret_cast<const int4 *>(ra_raw);
  const int4 *rb = reinterpret_cast<const int4 *>(rb_raw);
  for (int i = 0; i < npad / 4; ++i) {
    const int4 a0 = ra[2 * i], a1 = ra[2 * i + 1];
    const int4 b0 = rb[2 * i], b1 = rb[2 * i + 1];
    ZA = step_u64(U, a0.x, a0.y, ZA);
    ZB = step_u64(U, b0.x, b0.y, ZB);
    ZA = step_u64(U, a0.z, a0.w, ZA);
    ZB = step_u64(U, b0.z, b0.w, ZB);
    ZA = step_u64(U, a1.x, a1.y, ZA);
    ZB = step_u64(U, b1.x, b1.y, ZB);
    ZA = step_u64(U, a1.z, a1.w, ZA);
    ZB = step_u64(U, b1.z, b1.w, ZB);
  }
}

// ---- n > 32: the wave's job masks, read back as SGPR pairs ----
// One position of the two-machine walk (see the header comment of bound.hip):
// z = max(z + x, y) in the lanes whose node has the position's job
// unscheduled, z unchanged in the others.  off is the byte offset of the
// job's mask in the wave's slot; the mask comes from a scalar load, so the
// lane select is one v_cndmask on an SGPR pair.
__device__ __forceinline__ int step(kchar *ms, uint32_t off, int x, int y,
                                    int Z) {
  const uint64_t mk = *reinterpret_cast<ku64 *>(ms + off);
  const int up = max(Z + x, y);
  return __builtin_amdgcn_inverse_ballot_w64(mk) ? up : Z;
}

// Walk of one pair over its Johnson order: npad records in LDS at rp_raw,
// npad mask offsets at jp (npad is a multiple of 4).  The offsets of the next
// four positions are requested before the masks of the current four, so both
// scalar round trips overlap in one wait (the offset table is padded so that
// the request past the last pair stays inside it).
__device__ __forceinline__ int walk1(const char *rp_raw, kchar *jp, kchar *ms,
                                     int npad, int Z) {
  const int4 *rp = reinterpret_cast<const int4 *>(rp_raw);  // 2 records
  ku128 *jw = reinterpret_cast<ku128 *>(jp);                // 4 offsets
  u32x4 o = jw[0];
  asm volatile("" : "+s"(o));  // loaded before the loop, not waited for in it
  for (int i = 0; i < npad / 4; ++i) {
    const u32x4 nx = jw[i + 1];
    const int4 r0 = rp[2 * i], r1 = rp[2 * i + 1];
    Z = step(ms, o.x, r0.x, r0.y, Z);
    Z = step(ms, o.y, r0.z, r0.w, Z);
    Z = step(ms, o.z, r1.x, r1.y, Z);
    Z = step(ms, o.w, r1.z, r1.w, Z);
    // carried through an opaque copy: otherwise the two loads feeding the
    // loop-carried value are merged back into one load at the loop top
    o = nx;
    asm volatile("" : "+s"(o));
  }
  return Z;
}

// Two pairs walked together: two independent dependency chains per lane.
__device__ __forceinline__ void walk2(const char *ra_raw, const char *rb_raw,
                                      kchar *ja, kchar *jb, kchar *ms,
                                      int npad, int &ZA, int &ZB) {
  const int4 *ra = reinterpret_cast<const int4 *>(ra_raw);
  const int4 *rb = reinterpret_cast<const int4 *>(rb_raw);
  ku128 *wa = reinterpret_cast<ku128 *>(ja);
  ku128 *wb = reinterpret_cast<ku128 *>(jb);
  u32x4 oa = wa[0], ob = wb[0];
  asm volatile("" : "+s"(oa), "+s"(ob));  // loaded before the loop
  for (int i = 0; i < npad / 4; ++i) {
    const u32x4 na = wa[i + 1], nb = wb[i + 1];
    const int4 a0 = ra[2 * i], a1 = ra[2 * i + 1];
    const int4 b0 = rb[2 * i], b1 = rb[2 * i + 1];
    ZA = step(ms, oa.x, a0.x, a0.y, ZA);
    ZB = step(ms, ob.x, b0.x, b0.y, ZB);
    ZA = step(ms, oa.y, a0.z, a0.w, ZA);
    ZB = step(ms, ob.y, b0.z, b0.w, ZB);
    ZA = step(ms, oa.z, a1.x, a1.y, ZA);
    ZB = step(ms, ob.z, b1.x, b1.y, ZB);
    ZA = step(ms, oa.w, a1.z, a1.w, ZA);
    ZB = step(ms, ob.w, b1.z, b1.w, ZB);
    oa = na;
    ob = nb;
    asm volatile("" : "+s"(oa), "+s"(ob));
  }
}

// LDS byte offset of a pointer into the workgroup's LDS.
__device__ __forceinline__ uint32_t lds_offset(const char *p) {
  return (uint32_t)(uintptr_t)((__attribute__((address_space(3))) const char *)p);
}

// ---- the bytes walk's loop: records and job ids by scalar loads ----
//
// The records (x | y << 16, one word per position) and job ids (one byte per
// position) are read from the instance tables in global memory with scalar
// loads: every wave of the launch walks the same tables, so they are served
// by the scalar cache and the L2, and the arithmetic takes the record halves
// as scalar operands (op_sel picks the half):
//   t = z + al * x   (v_mad_i32_i16: x is signed)
//   u = al * y       (v_mad_u32_u16)
//   z = max(t, u)    (v_max_i32)
// with the lane's flag al = 0 or 1 read from its LDS byte row of the job,
// 64 * job bytes past its row 0 (v_lshl_add_u32 on the job id, which a
// scalar bit-field extract takes from the job bytes).  LDS returns only the
// lanes' flag bytes; a 16-byte record broadcast to a wave returns 1 KB
// through the LDS, which bounded the rate when the records were staged there.
// Groups of eight positions; two register sets take turns: records in
// s[64:79] (set X) and s[80:95] (set Y), pair A at +0 and pair B at +8; flags
// in v32..v47 (X) and v48..v63 (Y), A at +0 and B at +8; the job ids of a
// set's next group in s[48:51] (for X) and s[52:55] (for Y), A at +0, B at
// +2; s[56:63] hold the extracted ids.  A half waits for everything
// requested (scalar loads complete out of order, so the wait is for all),
// forms the other set's flag addresses from the job ids it holds, requests
// those flags, the other set's records and the job ids two groups ahead,
// then computes its own group.  The requests past a pair's end (one group of
// records, two of job ids) stay inside the tables, which carry two spare
// groups past the last pair; every request is waited for before the
// statement ends.
#define FSP_B8_STEP2(FA, RA, FB, RB)                                   \
  "v_mad_i32_i16 %[tA], " FA ", " RA ", %[zA]\n\t"                     \
  "v_mad_u32_u16 %[uA], " FA ", " RA ", 0 op_sel:[0,1,0,0]\n\t"        \
  "v_mad_i32_i16 %[tB], " FB ", " RB ", %[zB]\n\t"                     \
  "v_mad_u32_u16 %[uB], " FB ", " RB ", 0 op_sel:[0,1,0,0]\n\t"        \
  "v_max_i32 %[zA], %[tA], %[uA]\n\t"                                  \
  "v_max_i32 %[zB], %[tB], %[uB]\n\t"
#define FSP_B8_STEP1(FA, RA)                                           \
  "v_mad_i32_i16 %[tA], " FA ", " RA ", %[zA]\n\t"                     \
  "v_mad_u32_u16 %[uA], " FA ", " RA ", 0 op_sel:[0,1,0,0]\n\t"        \
  "v_max_i32 %[zA], %[tA], %[uA]\n\t"
// the eight job ids of two words into s56..s63
#define FSP_B8_IDS(W0, W1)                                             \
  "s_bfe_u32 s56, " W0 ", 0x80000\n\t"                                 \
  "s_bfe_u32 s57, " W0 ", 0x80008\n\t"                                 \
  "s_bfe_u32 s58, " W0 ", 0x80010\n\t"                                 \
  "s_lshr_b32 s59, " W0 ", 24\n\t"                                     \
  "s_bfe_u32 s60, " W1 ", 0x80000\n\t"                                 \
  "s_bfe_u32 s61, " W1 ", 0x80008\n\t"                                 \
  "s_bfe_u32 s62, " W1 ", 0x80010\n\t"                                 \
  "s_lshr_b32 s63, " W1 ", 24\n\t"
// flag address (lane's row-0 byte + 64 * job) and the byte load, in place
#define FSP_B8_FLAG(V, S)                                              \
  "v_lshl_add_u32 " V ", " S ", 6, %[lane]\n\t"                        \
  "ds_read_u8 " V ", " V "\n\t"
#define FSP_B8_FLAGS(V0, V1, V2, V3, V4, V5, V6, V7)                   \
  FSP_B8_FLAG(V0, "s56") FSP_B8_FLAG(V1, "s57")                        \
  FSP_B8_FLAG(V2, "s58") FSP_B8_FLAG(V3, "s59")                        \
  FSP_B8_FLAG(V4, "s60") FSP_B8_FLAG(V5, "s61")                        \
  FSP_B8_FLAG(V6, "s62") FSP_B8_FLAG(V7, "s63")

__device__ __forceinline__ void walk2_b8(uint64_t ra, uint64_t rb, uint64_t ja, uint64_t jb,
                                         uint32_t lane, int npad8, int &ZA, int &ZB) {
  int tA, uA, tB, uB;
  uint32_t cnt = (uint32_t)(npad8 / 8);  // groups
  uint32_t ro = 0, jo = 0;
  asm volatile(
      // group 0 into set X, the job ids of group 1 for set Y
      "s_load_dwordx2 s[48:49], %[ja], %[jo]\n\t"
      "s_load_dwordx2 s[50:51], %[jb], %[jo]\n\t"
      "s_load_dwordx8 s[64:71], %[ra], %[ro]\n\t"
      "s_load_dwordx8 s[72:79], %[rb], %[ro]\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx2 s[52:53], %[ja], %[jo]\n\t"
      "s_load_dwordx2 s[54:55], %[jb], %[jo]\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s48", "s49")
      FSP_B8_FLAGS("v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39")
      FSP_B8_IDS("s50", "s51")
      FSP_B8_FLAGS("v40", "v41", "v42", "v43", "v44", "v45", "v46", "v47")
      "1:\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s52", "s53")
      FSP_B8_FLAGS("v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55")
      FSP_B8_IDS("s54", "s55")
      FSP_B8_FLAGS("v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63")
      "s_add_u32 %[ro], %[ro], 32\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx8 s[80:87], %[ra], %[ro]\n\t"
      "s_load_dwordx8 s[88:95], %[rb], %[ro]\n\t"
      "s_load_dwordx2 s[48:49], %[ja], %[jo]\n\t"
      "s_load_dwordx2 s[50:51], %[jb], %[jo]\n\t"
      FSP_B8_STEP2("v32", "s64", "v40", "s72")
      FSP_B8_STEP2("v33", "s65", "v41", "s73")
      FSP_B8_STEP2("v34", "s66", "v42", "s74")
      FSP_B8_STEP2("v35", "s67", "v43", "s75")
      FSP_B8_STEP2("v36", "s68", "v44", "s76")
      FSP_B8_STEP2("v37", "s69", "v45", "s77")
      FSP_B8_STEP2("v38", "s70", "v46", "s78")
      FSP_B8_STEP2("v39", "s71", "v47", "s79")
      "s_sub_u32 %[cnt], %[cnt], 1\n\t"
      "s_cmp_eq_u32 %[cnt], 0\n\t"
      "s_cbranch_scc1 2f\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s48", "s49")
      FSP_B8_FLAGS("v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39")
      FSP_B8_IDS("s50", "s51")
      FSP_B8_FLAGS("v40", "v41", "v42", "v43", "v44", "v45", "v46", "v47")
      "s_add_u32 %[ro], %[ro], 32\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx8 s[64:71], %[ra], %[ro]\n\t"
      "s_load_dwordx8 s[72:79], %[rb], %[ro]\n\t"
      "s_load_dwordx2 s[52:53], %[ja], %[jo]\n\t"
      "s_load_dwordx2 s[54:55], %[jb], %[jo]\n\t"
      FSP_B8_STEP2("v48", "s80", "v56", "s88")
      FSP_B8_STEP2("v49", "s81", "v57", "s89")
      FSP_B8_STEP2("v50", "s82", "v58", "s90")
      FSP_B8_STEP2("v51", "s83", "v59", "s91")
      FSP_B8_STEP2("v52", "s84", "v60", "s92")
      FSP_B8_STEP2("v53", "s85", "v61", "s93")
      FSP_B8_STEP2("v54", "s86", "v62", "s94")
      FSP_B8_STEP2("v55", "s87", "v63", "s95")
      "s_sub_u32 %[cnt], %[cnt], 1\n\t"
      "s_cmp_eq_u32 %[cnt], 0\n\t"
      "s_cbranch_scc0 1b\n"
      "2:\n\t"
      "s_waitcnt lgkmcnt(0)"
      : [zA] "+v"(ZA), [zB] "+v"(ZB), [tA] "=&v"(tA), [uA] "=&v"(uA), [tB] "=&v"(tB),
        [uB] "=&v"(uB), [ro] "+s"(ro), [jo] "+s"(jo), [cnt] "+s"(cnt)
      : [ra] "s"(ra), [rb] "s"(rb), [ja] "s"(ja), [jb] "s"(jb), [lane] "v"(lane)
      : "v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39", "v40", "v41", "v42",
        "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53",
        "v54", "v55", "v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63",
        "s48", "s49", "s50", "s51", "s52", "s53", "s54", "s55", "s56", "s57", "s58",
        "s59", "s60", "s61", "s62", "s63", "s64", "s65", "s66", "s67", "s68", "s69",
        "s70", "s71", "s72", "s73", "s74", "s75", "s76", "s77", "s78", "s79", "s80",
        "s81", "s82", "s83", "s84", "s85", "s86", "s87", "s88", "s89", "s90", "s91",
        "s92", "s93", "s94", "s95", "scc", "memory");
}

// One pair, the same loop with pair A's registers only.
__device__ __forceinline__ int walk1_b8(uint64_t ra, uint64_t ja, uint32_t lane, int npad8,
                                        int Z) {
  int tA, uA;
  uint32_t cnt = (uint32_t)(npad8 / 8);
  uint32_t ro = 0, jo = 0;
  asm volatile(
      "s_load_dwordx2 s[48:49], %[ja], %[jo]\n\t"
      "s_load_dwordx8 s[64:71], %[ra], %[ro]\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx2 s[52:53], %[ja], %[jo]\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s48", "s49")
      FSP_B8_FLAGS("v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39")
      "1:\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s52", "s53")
      FSP_B8_FLAGS("v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55")
      "s_add_u32 %[ro], %[ro], 32\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx8 s[80:87], %[ra], %[ro]\n\t"
      "s_load_dwordx2 s[48:49], %[ja], %[jo]\n\t"
      FSP_B8_STEP1("v32", "s64") FSP_B8_STEP1("v33", "s65")
      FSP_B8_STEP1("v34", "s66") FSP_B8_STEP1("v35", "s67")
      FSP_B8_STEP1("v36", "s68") FSP_B8_STEP1("v37", "s69")
      FSP_B8_STEP1("v38", "s70") FSP_B8_STEP1("v39", "s71")
      "s_sub_u32 %[cnt], %[cnt], 1\n\t"
      "s_cmp_eq_u32 %[cnt], 0\n\t"
      "s_cbranch_scc1 2f\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      FSP_B8_IDS("s48", "s49")
      FSP_B8_FLAGS("v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39")
      "s_add_u32 %[ro], %[ro], 32\n\t"
      "s_add_u32 %[jo], %[jo], 8\n\t"
      "s_load_dwordx8 s[64:71], %[ra], %[ro]\n\t"
      "s_load_dwordx2 s[52:53], %[ja], %[jo]\n\t"
      FSP_B8_STEP1("v48", "s80") FSP_B8_STEP1("v49", "s81")
      FSP_B8_STEP1("v50", "s82") FSP_B8_STEP1("v51", "s83")
      FSP_B8_STEP1("v52", "s84") FSP_B8_STEP1("v53", "s85")
      FSP_B8_STEP1("v54", "s86") FSP_B8_STEP1("v55", "s87")
      "s_sub_u32 %[cnt], %[cnt], 1\n\t"
      "s_cmp_eq_u32 %[cnt], 0\n\t"
      "s_cbranch_scc0 1b\n"
      "2:\n\t"
      "s_waitcnt lgkmcnt(0)"
      : [zA] "+v"(Z), [tA] "=&v"(tA), [uA] "=&v"(uA), [ro] "+s"(ro), [jo] "+s"(jo),
        [cnt] "+s"(cnt)
      : [ra] "s"(ra), [ja] "s"(ja), [lane] "v"(lane)
      : "v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39", "v48", "v49", "v50",
        "v51", "v52", "v53", "v54", "v55", "s48", "s49", "s52", "s53", "s56", "s57",
        "s58", "s59", "s60", "s61", "s62", "s63", "s64", "s65", "s66", "s67", "s68",
        "s69", "s70", "s71", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87",
        "scc", "memory");
  return Z;
}

template <int FORM>
__device__ __forceinline__ int walk1_any(const char *rp, kchar *jp, kchar *ms,
                                         const uint8_t *al, int npad,
                                         uint64_t U, int Z) {
  if constexpr (FORM == kFormMasks) return walk1(rp, jp, ms, npad, Z);
  else if constexpr (FORM == kFormBytes)
    return walk1_b8(reinterpret_cast<uint64_t>(rp), reinterpret_cast<uint64_t>(jp),
                    lds_offset(reinterpret_cast<const char *>(al)), npad, Z);
  else if constexpr (FORM == kFormReg64) return walk1_u64(rp, npad, U, Z);
  else return walk1_u(rp, npad, (uint32_t)U, Z);
}

// Every pair whose index lies in [lo, hi): pairs (k,l) and (k,l+1) are walked
// together.  s_rec holds the records of pairs lo.. (LDS), jt the mask offsets
// of pair lo.  Returns the max over those pairs of 256*(pair bound) + junk.
// The bytes form walks the whole table from global memory (s_rec the record
// words, jt the job bytes, npad = npad8) and returns the plain maximum.
// The record and job pointers advance pair by pair (pair index order = table
// order) so that no per-pair address stays live.
template <int M, int FORM>
__device__ __forceinline__ int pair_sweep(const char *s_rec, kchar *jt, int lo,
                                          int hi, int npad, uint64_t U,
                                          kchar *ms, const uint8_t *al,
                                          const int (&R256)[M],
                                          const int (&T256)[M],
                                          const int (&Q256)[M], int LB256) {
  // per pair: npad records and mask offsets, or (bytes form, npad = npad8)
  // npad record words and job bytes
  int pb = npad * (FORM == kFormBytes ? 4 : (int)sizeof(Rec));
  int jb = npad * (FORM == kFormBytes ? 1 : (int)sizeof(uint32_t));
  // Opaque per call: otherwise every per-pair offset is loop-invariant in the
  // tile loop and gets hoisted, one scalar register per pair.
  asm volatile("" : "+s"(pb), "+s"(jb));
  // Byte offsets of pair index `pa - lo`, negative below lo.  Every offset is
  // formed in full before it is added to a pointer: the job table is a 64-bit
  // address, so a pointer stepped below its base and back would not wrap.
  int off = -lo * pb, joff = -lo * jb;
#pragma unroll
  for (int k = 0; k < M - 1; ++k) {
#pragma unroll
    for (int l = k + 1; l < M; l += 2) {
      const int pa = pair_index<M>(k, l);
      if (l + 1 < M) {
        const bool ina = pa >= lo && pa < hi, inb = pa + 1 >= lo && pa + 1 < hi;
        const int offb = off + pb, joffb = joff + jb;
        if (ina && inb) {
          int ZA = R256[l] - R256[k], ZB = R256[l + 1] - R256[k];
          if constexpr (FORM == kFormMasks)
            walk2(s_rec + off, s_rec + offb, jt + joff, jt + joffb, ms, npad,
                  ZA, ZB);
          else if constexpr (FORM == kFormBytes)
            walk2_b8(reinterpret_cast<uint64_t>(s_rec + off),
                     reinterpret_cast<uint64_t>(s_rec + offb),
                     reinterpret_cast<uint64_t>(jt + joff),
                     reinterpret_cast<uint64_t>(jt + joffb),
                     lds_offset(reinterpret_cast<const char *>(al)), npad, ZA, ZB);
          else if constexpr (FORM == kFormReg64)
            walk2_u64(s_rec + off, s_rec + offb, npad, U, ZA, ZB);
          else
            walk2_u(s_rec + off, s_rec + offb, npad, (uint32_t)U, ZA, ZB);
          LB256 = max(LB256, max(T256[k] + Q256[l] + ZA,
                                 T256[k] + Q256[l + 1] + ZB));
          // keep the max chain sequential (a reassociated max tree would hold
          // one partial result per pair)
          asm volatile("" : "+v"(LB256));
        } else {
          if (ina) {
            int Z = walk1_any<FORM>(s_rec + off, jt + joff, ms, al, npad, U,
                                    R256[l] - R256[k]);
            LB256 = max(LB256, T256[k] + Q256[l] + Z);
            asm volatile("" : "+v"(LB256));
          }
          if (inb) {
            int Z = walk1_any<FORM>(s_rec + offb, jt + joffb, ms, al, npad, U,
                                    R256[l + 1] - R256[k]);
            LB256 = max(LB256, T256[k] + Q256[l + 1] + Z);
            asm volatile("" : "+v"(LB256));
          }
        }
        off += 2 * pb;
        joff += 2 * jb;
      } else {
        if (pa >= lo && pa < hi) {
          int Z = walk1_any<FORM>(s_rec + off, jt + joff, ms, al, npad, U,
                                  R256[l] - R256[k]);
          LB256 = max(LB256, T256[k] + Q256[l] + Z);
          asm volatile("" : "+v"(LB256));
        }
        off += pb;
        joff += jb;
      }
    }
  }
  return LB256;
}

// Steps 1 and 2 for the node at idx (one per lane): decode the prefix (U,
// the front F, the prefix column sums), then heads r[k], tails q[k] and
// r[k] + S[k] (S = remaining work), each shifted left by SH into R, T, Q.
// last = F[m-1], the makespan of the prefix.  WIDE: the unscheduled set is
// kept in LDS, as the lane's words ([word][lane], words_lane), or with FLAGS
// as the lane's flag bytes (flags_lane[64 j] = job j unscheduled, for
// j < n; the byte of row n is zero).
template <int M, bool WIDE, int SH, typename SetT = uint32_t, bool FLAGS = false>
__device__ __forceinline__ void node_state(const InstView I, const int32_t *s_p,
                                           uint32_t *words_lane,
                                           const uint8_t *nodes, int stride,
                                           bool aligned, int64_t idx, bool live,
                                           SetT &U, int &d, bool &bad,
                                           int &last, int (&R)[M], int (&T)[M],
                                           int (&Q)[M], uint8_t *flags_lane = nullptr) {
  const int n = I.n, mp = I.mp;
  constexpr int kSetBits = 8 * (int)sizeof(SetT);
  const SetT full = n >= kSetBits ? ~SetT(0) : ((SetT(1) << n) - SetT(1));
  // ---- 1. decode the prefix, front recurrence, prefix column sums ----
  int F[M], Pk[M];
#pragma unroll
  for (int k = 0; k < M; ++k) F[k] = Pk[k] = 0;
  U = full;
  if constexpr (FLAGS) {
    for (int j = 0; j < n; ++j) flags_lane[j * 64] = 1;
    flags_lane[n * 64] = 0;
  } else if constexpr (WIDE)
    for (int w = 0; w * 32 < n; ++w)
      words_lane[w * kBlock] = n - w * 32 >= 32 ? 0xffffffffu
                                                 : ((1u << (n - w * 32)) - 1u);
  bad = false;
  d = 0;
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
          if constexpr (FLAGS) {
            if (flags_lane[j * 64] == 0) bad = true;
            flags_lane[j * 64] = 0;
          } else if constexpr (WIDE) {
            uint32_t *wp = words_lane + (j >> 5) * kBlock;
            const uint32_t v = *wp, bit = 1u << (j & 31);
            if (!(v & bit)) bad = true;
            *wp = v & ~bit;
          } else {
            if (!((U >> j) & 1u)) bad = true;
            U &= ~(SetT(1) << j);
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
  {
    constexpr int M2 = (M + 1) / 2;
    u16x2 hm2[M2], qm2[M2];
#pragma unroll
    for (int t = 0; t < M2; ++t) hm2[t] = qm2[t] = (u16x2){0xffff, 0xffff};
    const int mp2 = mp / 2;
    for (int j = 0; j < n; ++j) {
      uint32_t g;
      if constexpr (FLAGS)
        g = (uint32_t)flags_lane[j * 64] - 1u;
      else if constexpr (WIDE)
        g = (uint32_t)__builtin_amdgcn_sbfe((int)~words_lane[(j >> 5) * kBlock], j & 31, 1);
      else if constexpr (sizeof(SetT) == 8)
        g = 0u - (uint32_t)((~U >> j) & 1u);
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
      R[k] = r << SH;
      T[k] = (r + I.tot[k] - Pk[k]) << SH;
      Q[k] = qmk << SH;
    }
  }
  last = F[M - 1];
}

// Whether a node with bound lb is eliminated against ub (the B&B's rule).
__device__ __forceinline__ bool eliminated(int lb, int ub, int rule) {
  return rule == FSP_PRUNE_GT ? lb > ub : lb >= ub;
}

// Whether the per-depth choice gives a node of depth d the one-machine bound.
__device__ __forceinline__ bool lb1_at_depth(const uint32_t *mask, int d) {
  return mask && ((mask[d >> 5] >> (d & 31)) & 1u);
}

// Measurement of the per-depth choice: one count per node with jobs left
// (cnt), per depth d, of the node and of its eliminations by the one-machine
// (e1) and the pair bound (e2).  The lanes at the depth of the wave's first
// lane are counted with one atomic per counter, the others one by one.
// Every lane of the wave calls it.
__device__ __forceinline__ void count_depth_stats(uint32_t *stats, bool cnt, int d, bool e1,
                                                  bool e2) {
  const int d0 = __builtin_amdgcn_readfirstlane(d);
  const bool same = d == d0;
  const uint64_t b0 = __ballot(cnt && same), b1 = __ballot(cnt && same && e1),
                 b2 = __ballot(cnt && same && e2);
  if (__lane_id() == 0 && b0) {
    atomicAdd(&stats[d0], (uint32_t)__popcll(b0));
    if (b1) atomicAdd(&stats[256 + d0], (uint32_t)__popcll(b1));
    if (b2) atomicAdd(&stats[512 + d0], (uint32_t)__popcll(b2));
  }
  if (cnt && !same) {
    atomicAdd(&stats[d], 1u);
    if (e1) atomicAdd(&stats[256 + d], 1u);
    if (e2) atomicAdd(&stats[512 + d], 1u);
  }
}

// Bound the 256 nodes [base, base + 256) of a pool (one per lane), writing
// lb_out[idx] for idx < count.  For n > 32, tile_slots is this tile's part of
// the mask scratch: kBlock / 64 slots of I.slot_bytes, never used by another
// tile of the same launch (unused, may be null, for n <= 32).  Every lane of
// the workgroup must call it (the chunked form synchronises the workgroup).
template <int M, int FORM, bool CHUNKED>
__device__ __forceinline__ void bound_nodes(const InstView I, const LdsView &L,
                                            const uint8_t *nodes, int stride,
                                            bool aligned, int64_t base,
                                            int64_t count, int32_t *lb_out,
                                            char *tile_slots,
                                            const Prefilter pf = Prefilter()) {
  constexpr bool WIDE = FORM == kFormMasks || FORM == kFormBytes;
  const int tid = threadIdx.x;
  const int n = I.n, npad = I.npad;
  char *s_rec = L.s_rec;
  const int32_t *s_p = L.s_p;
  uint32_t *words_lane = WIDE && FORM != kFormBytes ? L.s_words + tid : nullptr;
  // the bytes form: the lane's flag bytes, rows [job 0 .. n] of its wave
  uint8_t *flags_lane =
      FORM == kFormBytes
          ? L.s_alpha + (size_t)(tid >> 6) * (size_t)(n + 1) * 64 + (tid & 63)
          : nullptr;
  const int64_t idx = base + tid;
  const bool live = idx < count;

  using SetT = typename std::conditional<FORM == kFormReg64, uint64_t, uint32_t>::type;
  SetT U;
  int d, last;
  bool bad;
  // values carry SH bits of fraction: 8 for the walks whose records carry
  // the job in y's low byte, none for the bytes walk
  constexpr int SH = FORM == kFormBytes ? 0 : 8;
  int T256[M], R256[M], Q256[M];
  node_state<M, WIDE, SH, SetT, FORM == kFormBytes>(I, s_p, words_lane, nodes, stride,
                                                   aligned, idx, live, U, d, bad, last,
                                                   R256, T256, Q256, flags_lane);
  int u_left;
  if constexpr (WIDE)
    u_left = n - d;
  else if constexpr (FORM == kFormReg64)
    u_left = __builtin_popcountll(U);
  else
    u_left = __builtin_popcount(U);

  // one-machine bound max_k r[k] + S[k] + q[k] (T and Q carry r + S and q);
  // the wave skips the pair walks when it decides every live node
  bool skip = false, only1 = false;
  int lb1 = 0;
  if (pf.lb1_only || pf.ub || pf.lb1_depths) {
    int m1 = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) m1 = max(m1, T256[k] + Q256[k]);
    lb1 = m1 >> SH;
    only1 = pf.lb1_only || (live && !bad && lb1_at_depth(pf.lb1_depths, d));
    bool decided = !live || bad || u_left == 0 || only1;
    if (pf.ub && !pf.lb1_only && !pf.depth_stats)
      decided = decided || eliminated(lb1, *pf.ub, pf.rule);
    skip = __ballot(!decided) == 0;
  }

  // ---- 3. (n > 32) the wave's job masks, then every machine pair.  The
  //         slot is written with vector stores and read back with scalar
  //         loads.  The vector L1 writes through, so once the wave's stores
  //         have completed (vmcnt 0) they are in the L2 that the scalar cache
  //         fills from; the slot address is fresh in this launch (the scalar
  //         cache starts every dispatch invalidated), so no scalar cache line
  //         can hold an older copy of it. ----
  kchar *ms = nullptr, *jt = nullptr;
  const uint8_t *al = nullptr;
  // only this lane reads its flag bytes, so no barrier is needed
  if constexpr (FORM == kFormBytes) al = flags_lane;
  if constexpr (FORM == kFormMasks) if (!skip) {
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint64_t *slot = reinterpret_cast<uint64_t *>(
        tile_slots + (size_t)wave * (size_t)I.slot_bytes);
    write_masks<WIDE>(slot, n, I.slot_bytes, U, words_lane);
    uint64_t slot_addr = reinterpret_cast<uint64_t>(slot);
    // wait for the stores; the address passes through the same statement so
    // that no load from the slot can be scheduled above the wait
    asm volatile("s_waitcnt vmcnt(0)" : "+s"(slot_addr)::"memory");
    ms = reinterpret_cast<kchar *>(slot_addr);
    jt = reinterpret_cast<kchar *>(reinterpret_cast<uint64_t>(I.joff));
  }

  int LB256 = 0;
  if constexpr (FORM == kFormBytes) {
    // the whole table, from global memory (one pass, no barriers)
#pragma unroll
    for (int k = 0; k < M; ++k)
      asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
    jt = reinterpret_cast<kchar *>(reinterpret_cast<uint64_t>(I.bjob));
    if (!skip)
      LB256 = pair_sweep<M, FORM>(reinterpret_cast<const char *>(I.bxy), jt, 0,
                                  M * (M - 1) / 2, I.npad8, U, ms, al, R256, T256,
                                  Q256, LB256);
  } else if constexpr (!CHUNKED) {
#pragma unroll
    for (int k = 0; k < M; ++k)
      asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
    if (!skip)
      LB256 = pair_sweep<M, FORM>(s_rec, jt, 0, M * (M - 1) / 2, npad, U, ms, al,
                                  R256, T256, Q256, LB256);
  } else {
    for (int chunk = 0; chunk < I.nchunks; ++chunk) {
      __syncthreads();
      stage_chunk(I, s_rec, chunk);
      __syncthreads();
      // keep the per-node values from being re-derived per pair outside
      // the chunk loop (which would cost a register per pair)
#pragma unroll
      for (int k = 0; k < M; ++k)
        asm volatile("" : "+v"(R256[k]), "+v"(T256[k]), "+v"(Q256[k]));
      int lo = chunk * I.ppc, hi = lo + I.ppc;
      asm volatile("" : "+s"(lo), "+s"(hi));
      // the barriers above are kept when the wave skips its walks
      if (!skip)
        LB256 = pair_sweep<M, FORM>(s_rec, jt + (size_t)lo * npad * 4, lo, hi,
                                    npad, U, ms, al, R256, T256, Q256, LB256);
    }
  }

  // ---- 4. result ----
  int lb = u_left == 0 ? last : ((skip || only1) ? lb1 : (LB256 >> SH));
  if (pf.depth_stats && pf.ub) {
    const int ub = *pf.ub;
    const bool cnt = live && !bad && u_left > 0;
    count_depth_stats(pf.depth_stats, cnt, d, cnt && eliminated(lb1, ub, pf.rule),
                      cnt && eliminated(LB256 >> SH, ub, pf.rule));
  }
  if (bad) lb = FSP_LB_INVALID;
  if (live) lb_out[idx] = lb;
}

// ---- two nodes per lane in packed 16-bit halves (instances whose total
//      work is at most 32767: every head, tail, clock difference and bound
//      of the method then lies in [0, 32767], and z + x in [-32767, 32767]) --
//
// The lane holds node A in the low and node B in the high 16 bits of every
// state value.  Before the walk, each lane builds one register per job,
//   al[j] = (job j unscheduled in A) | (job j unscheduled in B) << 16,
// in 32 VGPRs pinned at v96..v127.  The table position's job id is
// wave-uniform and comes from a scalar load; with the VGPR index mode on
// (s_set_gpr_idx_on), the job id is added to the register number of the
// first source operand, so the multiplier al[job] is read directly by the
// arithmetic.  One position then costs
//   t = z + al * x,  u = al * y       (v_pk_mad_u16, v_pk_mul_lo_u16; x and
//       y are the halves of one table word, broadcast by op_sel)
//   z = max(t, u)                     (v_pk_max_i16)
// i.e. 3 vector instructions for two nodes (plus scalar instructions that
// set the index, issued beside them).  al = 0 leaves z unchanged (z >= 0).
typedef unsigned int u32x32 __attribute__((ext_vector_type(32)));

// One position of two chains: pair A with the job in SGPR JA and the word in
// VGPR XA, pair B with JB and XB.  The caller saves M0 (the index) before and
// restores it after.
#define FSP_P16_STEP2(JA, XA, JB, XB)                                  \
  "s_set_gpr_idx_on " JA ", gpr_idx(SRC0)\n\t"                        \
  "v_pk_mad_u16 %[tA], v96, " XA ", %[zA] op_sel_hi:[1,0,1]\n\t"      \
  "v_pk_mul_lo_u16 %[uA], v96, " XA " op_sel:[0,1] op_sel_hi:[1,1]\n\t" \
  "s_set_gpr_idx_idx " JB "\n\t"                                      \
  "v_pk_mad_u16 %[tB], v96, " XB ", %[zB] op_sel_hi:[1,0,1]\n\t"      \
  "v_pk_mul_lo_u16 %[uB], v96, " XB " op_sel:[0,1] op_sel_hi:[1,1]\n\t" \
  "s_set_gpr_idx_off\n\t"                                             \
  "v_pk_max_i16 %[zA], %[tA], %[uA]\n\t"                              \
  "v_pk_max_i16 %[zB], %[tB], %[uB]\n\t"

#define FSP_P16_STEP1(JA, XA)                                          \
  "s_set_gpr_idx_on " JA ", gpr_idx(SRC0)\n\t"                        \
  "v_pk_mad_u16 %[tA], v96, " XA ", %[zA] op_sel_hi:[1,0,1]\n\t"      \
  "v_pk_mul_lo_u16 %[uA], v96, " XA " op_sel:[0,1] op_sel_hi:[1,1]\n\t" \
  "s_set_gpr_idx_off\n\t"                                             \
  "v_pk_max_i16 %[zA], %[tA], %[uA]\n\t"


// Two pairs walked together over `groups` groups of four positions.  Their
// tables are interleaved four positions at a time (four words of the first
// pair, then four of the second): the xy words in LDS at byte offset `lds`,
// the job ids in global memory at `jobs` (scalar loads).  The loop is double
// buffered: group g + 1 is requested (job ids into s[88:95], words into
// v[88:95], or s[80:87] / v[80:87]) before group g is computed, and waited for
// after it, so the loads of one group overlap the arithmetic of the other.
// The request one group past the end stays inside both tables (the job table
// has a spare group; in LDS the rows of p follow the xy table).  Every load
// is waited for inside the statement.
__device__ __forceinline__ void walk2_p16(uint32_t lds, const uint32_t *jobs, int groups,
                                          const u32x32 &AL, uint32_t &ZA,
                                          uint32_t &ZB) {
  uint32_t tA, uA, tB, uB, sv, soff, scnt;
  const uint64_t jp = reinterpret_cast<uint64_t>(jobs);
  asm volatile(
      "s_mov_b32 %[sv], m0\n\t"
      "s_mov_b32 %[soff], 0\n\t"
      "s_mov_b32 %[scnt], %[ng]\n\t"
      "s_load_dwordx8 s[80:87], %[jp], %[soff]\n\t"
      "ds_read_b128 v[80:83], %[va]\n\t"
      "ds_read_b128 v[84:87], %[va] offset:16\n\t"
      "s_waitcnt lgkmcnt(0)\n"
      "1:\n\t"
      "s_add_u32 %[soff], %[soff], 32\n\t"
      "s_load_dwordx8 s[88:95], %[jp], %[soff]\n\t"
      "ds_read_b128 v[88:91], %[va] offset:32\n\t"
      "ds_read_b128 v[92:95], %[va] offset:48\n\t"
      FSP_P16_STEP2("s80", "v80", "s84", "v84")
      FSP_P16_STEP2("s81", "v81", "s85", "v85")
      FSP_P16_STEP2("s82", "v82", "s86", "v86")
      FSP_P16_STEP2("s83", "v83", "s87", "v87")
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_sub_u32 %[scnt], %[scnt], 1\n\t"
      "s_cmp_eq_u32 %[scnt], 0\n\t"
      "s_cbranch_scc1 2f\n\t"
      "s_add_u32 %[soff], %[soff], 32\n\t"
      "s_load_dwordx8 s[80:87], %[jp], %[soff]\n\t"
      "ds_read_b128 v[80:83], %[va] offset:64\n\t"
      "ds_read_b128 v[84:87], %[va] offset:80\n\t"
      FSP_P16_STEP2("s88", "v88", "s92", "v92")
      FSP_P16_STEP2("s89", "v89", "s93", "v93")
      FSP_P16_STEP2("s90", "v90", "s94", "v94")
      FSP_P16_STEP2("s91", "v91", "s95", "v95")
      "s_waitcnt lgkmcnt(0)\n\t"
      "v_add_u32 %[va], 64, %[va]\n\t"
      "s_sub_u32 %[scnt], %[scnt], 1\n\t"
      "s_cmp_eq_u32 %[scnt], 0\n\t"
      "s_cbranch_scc0 1b\n"
      "2:\n\t"
      "s_mov_b32 m0, %[sv]"
      : [zA] "+v"(ZA), [zB] "+v"(ZB), [tA] "=&v"(tA), [uA] "=&v"(uA),
        [tB] "=&v"(tB), [uB] "=&v"(uB), [sv] "=&s"(sv), [soff] "=&s"(soff),
        [scnt] "=&s"(scnt), [va] "+v"(lds)
      : [jp] "s"(jp), [ng] "s"(groups), [al] "{v[96:127]}"(AL)
      : "v80", "v81", "v82", "v83", "v84", "v85", "v86", "v87", "v88", "v89", "v90",
        "v91", "v92", "v93", "v94", "v95", "s80", "s81", "s82", "s83", "s84", "s85",
        "s86", "s87", "s88", "s89", "s90", "s91", "s92", "s93", "s94", "s95", "scc",
        "memory");
}

// One pair alone (the last pair of a row with an odd number of pairs): four
// words and four job ids per group, double buffered as walk2_p16.
__device__ __forceinline__ uint32_t walk1_p16(uint32_t lds, const uint32_t *jobs, int groups,
                                              const u32x32 &AL, uint32_t Z) {
  uint32_t tA, uA, sv, soff, scnt;
  const uint64_t jp = reinterpret_cast<uint64_t>(jobs);
  asm volatile(
      "s_mov_b32 %[sv], m0\n\t"
      "s_mov_b32 %[soff], 0\n\t"
      "s_mov_b32 %[scnt], %[ng]\n\t"
      "s_load_dwordx4 s[80:83], %[jp], %[soff]\n\t"
      "ds_read_b128 v[80:83], %[va]\n\t"
      "s_waitcnt lgkmcnt(0)\n"
      "1:\n\t"
      "s_add_u32 %[soff], %[soff], 16\n\t"
      "s_load_dwordx4 s[88:91], %[jp], %[soff]\n\t"
      "ds_read_b128 v[88:91], %[va] offset:16\n\t"
      FSP_P16_STEP1("s80", "v80")
      FSP_P16_STEP1("s81", "v81")
      FSP_P16_STEP1("s82", "v82")
      FSP_P16_STEP1("s83", "v83")
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_sub_u32 %[scnt], %[scnt], 1\n\t"
      "s_cmp_eq_u32 %[scnt], 0\n\t"
      "s_cbranch_scc1 2f\n\t"
      "s_add_u32 %[soff], %[soff], 16\n\t"
      "s_load_dwordx4 s[80:83], %[jp], %[soff]\n\t"
      "ds_read_b128 v[80:83], %[va] offset:32\n\t"
      FSP_P16_STEP1("s88", "v88")
      FSP_P16_STEP1("s89", "v89")
      FSP_P16_STEP1("s90", "v90")
      FSP_P16_STEP1("s91", "v91")
      "s_waitcnt lgkmcnt(0)\n\t"
      "v_add_u32 %[va], 32, %[va]\n\t"
      "s_sub_u32 %[scnt], %[scnt], 1\n\t"
      "s_cmp_eq_u32 %[scnt], 0\n\t"
      "s_cbranch_scc0 1b\n"
      "2:\n\t"
      "s_mov_b32 m0, %[sv]"
      : [zA] "+v"(Z), [tA] "=&v"(tA), [uA] "=&v"(uA), [sv] "=&s"(sv),
        [soff] "=&s"(soff), [scnt] "=&s"(scnt), [va] "+v"(lds)
      : [jp] "s"(jp), [ng] "s"(groups), [al] "{v[96:127]}"(AL)
      : "v80", "v81", "v82", "v83", "v88", "v89", "v90", "v91", "s80", "s81", "s82",
        "s83", "s88", "s89", "s90", "s91", "scc", "memory");
  return Z;
}

__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) +
                                          __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) -
                                          __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                      __builtin_bit_cast(u16x2, b)));
}

// Every pair (the whole xy table is in LDS: n <= 32; the job table is read
// from global memory by scalar loads at the same offsets).  Returns the
// packed max over pairs of the pair bounds of nodes A and B.
template <int M>
__device__ __forceinline__ uint32_t pair_sweep_p16(const char *s_xy, const uint32_t *jt,
                                                   int npad, const u32x32 &AL,
                                                   const uint32_t (&R)[M],
                                                   const uint32_t (&T)[M],
                                                   const uint32_t (&Q)[M]) {
  // words of one pair, in both tables; groups of four positions per pair
  int pw = npad, groups = npad / 4;
  asm volatile("" : "+s"(pw), "+s"(groups));
  const uint32_t lds0 = lds_offset(s_xy);
  int off = 0;
  uint32_t LB = 0;
#pragma unroll
  for (int k = 0; k < M - 1; ++k) {
#pragma unroll
    for (int l = k + 1; l < M; l += 2) {
      if (l + 1 < M) {
        uint32_t ZA = pk_sub(R[l], R[k]), ZB = pk_sub(R[l + 1], R[k]);
        walk2_p16(lds0 + 4 * off, jt + off, groups, AL, ZA, ZB);
        // T + Q + z wraps in 16 bits only on the way: the sum is a bound of
        // the method, at most the total work
        LB = pk_max(LB, pk_max(pk_add(pk_add(T[k], Q[l]), ZA),
                               pk_add(pk_add(T[k], Q[l + 1]), ZB)));
        asm volatile("" : "+v"(LB));
        off += 2 * pw;
      } else {
        uint32_t Z = walk1_p16(lds0 + 4 * off, jt + off, groups, AL, pk_sub(R[l], R[k]));
        LB = pk_max(LB, pk_add(pk_add(T[k], Q[l]), Z));
        asm volatile("" : "+v"(LB));
        off += pw;
      }
    }
  }
  return LB;
}

// Lane view of one 16-byte chunk of a node record: chunk c of the record at
// rp (zeros when `take` is false).  Unaligned pools read byte by byte.
__device__ __forceinline__ void record_chunk(const uint8_t *rp, int c, bool take,
                                             bool aligned, int stride,
                                             uint32_t (&w)[4]) {
  w[0] = w[1] = w[2] = w[3] = 0u;
  if (!take) return;
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
}

// One prefix position of one node: job byte `j` at position `pos` of a node
// of depth d.  Returns the row of s_p16 to add (n, the row of zeros, past the
// node's depth or for an invalid job), clears the job in U and flags a job
// out of range or already scheduled.
__device__ __forceinline__ int prefix_job(uint32_t j, int pos, int d, int n,
                                          uint32_t &U, bool &bad) {
  const bool in = pos <= d;
  const bool ok = j < (uint32_t)n;
  const bool free = __builtin_amdgcn_ubfe(U, j, 1u) != 0u;
  bad = bad || (in && !(ok && free));
  const bool take = in && ok;
  U &= take ? ~(1u << (j & 31u)) : ~0u;
  return take ? (int)j : n;
}

// The state of both nodes of a lane at once, node A in the low and node B
// in the high 16 bits of every value (total work <= 32767, so every front,
// head, tail and column sum fits).  Step 1 walks the two prefixes together
// up to the deeper one; a position past a node's own depth adds the row of
// zeros (row n of s_p16), which leaves its front unchanged because a front
// is non-decreasing along the machines.  Step 2 takes the head and tail
// minima over each node's unscheduled jobs with the job's sums broadcast to
// both halves and a per-half all-ones mask for a scheduled job.
//   s_p16: [n + 1][p16_row_words(mp)] packed machine pairs of p, row n zero.
template <int M>
__device__ __forceinline__ void node_state_p16(
    const InstView I, const uint32_t *s_p16, const uint8_t *nodes, int stride,
    bool aligned, int64_t ia, int64_t ib, bool la, bool lbv, uint32_t &UA,
    uint32_t &UB, bool &badA, bool &badB, uint32_t &last, uint32_t (&R)[M],
    uint32_t (&T)[M], uint32_t (&Q)[M]) {
  const int n = I.n, h = p16_row_words(I.mp);
  const uint32_t full = n >= 32 ? ~0u : ((1u << n) - 1u);
  u16x2 F[M], Pk[M];
#pragma unroll
  for (int k = 0; k < M; ++k) F[k] = Pk[k] = (u16x2){0, 0};
  UA = UB = full;
  badA = badB = false;
  int dA = 0, dB = 0;
  const uint8_t *pa = nodes + ia * (int64_t)stride;
  const uint8_t *pb = nodes + ib * (int64_t)stride;
  if (la) dA = pa[0];
  if (lbv) dB = pb[0];
  if (dA > n) { badA = true; dA = 0; }
  if (dB > n) { badB = true; dB = 0; }
  const int dmax = max(dA, dB);
  // ---- 1. both prefixes: front recurrence and prefix column sums ----
  for (int c = 0; c * 16 <= dmax; ++c) {
    uint32_t wa[4], wb[4];
    // a lane past the end of the pool (la / lbv false) reads nothing
    record_chunk(pa, c, la && c * 16 <= dA, aligned, stride, wa);
    record_chunk(pb, c, lbv && c * 16 <= dB, aligned, stride, wb);
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int pos = c * 16 + b;
      if (pos >= 1 && pos <= dmax) {
        const int ja = prefix_job((wa[b >> 2] >> (8 * (b & 3))) & 0xffu, pos, dA, n, UA, badA);
        const int jb = prefix_job((wb[b >> 2] >> (8 * (b & 3))) & 0xffu, pos, dB, n, UB, badB);
        const uint32_t *ra = s_p16 + ja * h, *rb = s_p16 + jb * h;
#pragma unroll
        for (int t = 0; 2 * t < M; ++t) {
          const uint32_t xa = ra[t], xb = rb[t];
          // machine 2t of both nodes, then machine 2t + 1
          const u16x2 lo = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(xb, xa, 0x05040100u));
          const u16x2 hi = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(xb, xa, 0x07060302u));
          const int k = 2 * t;
          F[k] = (k == 0 ? F[0] : __builtin_elementwise_max(F[k], F[k - 1])) + lo;
          Pk[k] += lo;
          if (k + 1 < M) {
            F[k + 1] = __builtin_elementwise_max(F[k + 1], F[k]) + hi;
            Pk[k + 1] += hi;
          }
        }
      }
    }
  }
  // ---- 2. head and tail minima over the unscheduled jobs of each node ----
  const uint64_t W = (uint64_t)((UA & 0xffffu) | (UB << 16)) |
                     ((uint64_t)((UA >> 16) | (UB & 0xffff0000u)) << 32);
  u16x2 hm[M], qm[M];
#pragma unroll
  for (int k = 0; k < M; ++k) hm[k] = qm[k] = (u16x2){0xffff, 0xffff};
  const int mp2 = I.mp / 2;
  // the sums are the same for every lane: scalar loads
  ku32 *Hk = reinterpret_cast<ku32 *>(reinterpret_cast<uint64_t>(I.Hp));
  ku32 *Qk = reinterpret_cast<ku32 *>(reinterpret_cast<uint64_t>(I.Qp));
  for (int j = 0; j < n; ++j) {
    const uint32_t s = (uint32_t)((j & 15) + 32 * (j >> 4));
    // 1 in a half whose node has job j unscheduled; minus one: 0 or 0xffff
    const u16x2 al = __builtin_bit_cast(u16x2, (uint32_t)(W >> s) & 0x10001u);
    const u16x2 g = al - (u16x2){1, 1};
    ku32 *hr = Hk + j * mp2;
    ku32 *qr = Qk + j * mp2;
#pragma unroll
    for (int t = 0; 2 * t < M; ++t) {
      const uint32_t hw = hr[t], qw = qr[t];
      const u16x2 h0 = {(unsigned short)hw, (unsigned short)hw};
      const u16x2 q0 = {(unsigned short)qw, (unsigned short)qw};
      hm[2 * t] = __builtin_elementwise_min(hm[2 * t], __builtin_elementwise_max(h0, g));
      qm[2 * t] = __builtin_elementwise_min(qm[2 * t], __builtin_elementwise_max(q0, g));
      if (2 * t + 1 < M) {
        const u16x2 h1 = {(unsigned short)(hw >> 16), (unsigned short)(hw >> 16)};
        const u16x2 q1 = {(unsigned short)(qw >> 16), (unsigned short)(qw >> 16)};
        hm[2 * t + 1] =
            __builtin_elementwise_min(hm[2 * t + 1], __builtin_elementwise_max(h1, g));
        qm[2 * t + 1] =
            __builtin_elementwise_min(qm[2 * t + 1], __builtin_elementwise_max(q1, g));
      }
    }
  }
  // the column totals are loaded here, not hoisted above the loop
  asm volatile("" ::: "memory");
  ku32 *tot = reinterpret_cast<ku32 *>(reinterpret_cast<uint64_t>(I.tot));
  // ---- 3. heads r = max(F, F[0] + min H), r + remaining work, tails ----
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const u16x2 r = __builtin_elementwise_max(F[k], F[0] + hm[k]);
    const unsigned short tk = (unsigned short)tot[k];
    // r + tot - Pk may pass 65535 on the way; the result is at most the
    // total work, so the 16-bit wrap-around cancels
    R[k] = __builtin_bit_cast(uint32_t, r);
    T[k] = __builtin_bit_cast(uint32_t, r + (u16x2){tk, tk} - Pk[k]);
    Q[k] = __builtin_bit_cast(uint32_t, qm[k]);
  }
  last = __builtin_bit_cast(uint32_t, F[M - 1]);
}

// Bound the 512 nodes [base, base + 512) of a pool, nodes base + tid (low
// halves) and base + 256 + tid (high halves), writing lb_out[idx] for
// idx < count.  n <= 32 and the table is whole in LDS (I.rec is the packed
// table, L.s_p holds the packed rows of p).  Every lane of the workgroup must
// call it.  PF = false compiles the pre-filter, the per-depth choice and the
// depth counts out (pf is then ignored): their state, live across the walk,
// costs this form spills at 20 machines.
template <int M, bool PF>
__device__ __forceinline__ void bound_nodes_p16(const InstView I, const LdsView &L,
                                                const uint8_t *nodes, int stride,
                                                bool aligned, int64_t base,
                                                int64_t count, int32_t *lb_out,
                                                const Prefilter pf = Prefilter()) {
  const int tid = threadIdx.x;
  const int64_t ia = base + tid, ib = base + kBlock + tid;
  const bool la = ia < count, lbv = ib < count;
  uint32_t R[M], T[M], Q[M];
  uint32_t UA, UB, last;
  bool badA, badB;
  node_state_p16<M>(I, reinterpret_cast<const uint32_t *>(L.s_p), nodes, stride,
                    aligned, ia, ib, la, lbv, UA, UB, badA, badB, last, R, T, Q);
  // one-machine bounds of both nodes (see bound_nodes)
  bool skip = false, onlyA = false, onlyB = false;
  uint32_t LB1 = 0;
  const int dA = I.n - __builtin_popcount(UA), dB = I.n - __builtin_popcount(UB);
  if (PF && (pf.lb1_only || pf.ub || pf.lb1_depths)) {
#pragma unroll
    for (int k = 0; k < M; ++k) LB1 = pk_max(LB1, pk_add(T[k], Q[k]));
    onlyA = pf.lb1_only || (la && !badA && lb1_at_depth(pf.lb1_depths, dA));
    onlyB = pf.lb1_only || (lbv && !badB && lb1_at_depth(pf.lb1_depths, dB));
    bool da = !la || badA || UA == 0u || onlyA, db = !lbv || badB || UB == 0u || onlyB;
    if (pf.ub && !pf.lb1_only && !pf.depth_stats) {
      const int ub = *pf.ub;
      da = da || eliminated((int)(LB1 & 0xffffu), ub, pf.rule);
      db = db || eliminated((int)(LB1 >> 16), ub, pf.rule);
    }
    skip = __ballot(!(da && db)) == 0;
  }
#pragma unroll
  for (int k = 0; k < M; ++k) asm volatile("" : "+v"(R[k]), "+v"(T[k]), "+v"(Q[k]));
  uint32_t LB = LB1;
  if (!skip) {
    // the per-job multipliers of both nodes (jobs >= n are never named)
    u32x32 AL;
#pragma unroll
    for (int j = 0; j < 32; ++j)
      AL[j] = ((UA >> j) & 1u) | (((UB >> j) & 1u) << 16);
    LB = pair_sweep_p16<M>(L.s_rec, I.job16, I.npad, AL, R, T, Q);
  }
  if (PF && pf.depth_stats && pf.ub) {
    const int ub = *pf.ub;
    const bool ca = la && !badA && UA != 0u, cb = lbv && !badB && UB != 0u;
    count_depth_stats(pf.depth_stats, ca, dA, ca && eliminated((int)(LB1 & 0xffffu), ub, pf.rule),
                      ca && eliminated((int)(LB & 0xffffu), ub, pf.rule));
    count_depth_stats(pf.depth_stats, cb, dB, cb && eliminated((int)(LB1 >> 16), ub, pf.rule),
                      cb && eliminated((int)(LB >> 16), ub, pf.rule));
  }
  if (la) {
    int lb = UA == 0u ? (int)(last & 0xffffu) : (int)(((skip || onlyA) ? LB1 : LB) & 0xffffu);
    lb_out[ia] = badA ? FSP_LB_INVALID : lb;
  }
  if (lbv) {
    int lb = UB == 0u ? (int)(last >> 16) : (int)(((skip || onlyB) ? LB1 : LB) >> 16);
    lb_out[ib] = badB ? FSP_LB_INVALID : lb;
  }
}

// LDS of one workgroup of the packed kernel: the xy table (one word per
// position), then the packed rows of p plus a row of zeros.
__host__ __device__ inline size_t lds_bytes_p16(int n, int mp, int npad, int P) {
  const size_t b = (size_t)P * npad * 4 + (size_t)(n + 1) * p16_row_words(mp) * 4;
  return (b + 15) & ~size_t(15);
}

// LDS view of the packed kernel (see lds_bytes_p16).
__device__ __forceinline__ LdsView carve_p16(char *smem, const InstView I) {
  LdsView L;
  L.s_rec = smem;
  L.s_p = reinterpret_cast<int32_t *>(smem + (size_t)I.P * I.npad * 4);
  L.s_words = nullptr;
  return L;
}

// Stage the packed kernel's LDS: the xy table, and the packed rows of p for
// node_state_p16: s_p16[j][t] = p[j][2t] | p[j][2t + 1] << 16 for j < n and
// t < mp / 2; zeros elsewhere (row n and the pitch padding).
__device__ __forceinline__ void stage_p16_rows(const InstView I, const LdsView &L) {
  const int h = p16_row_words(I.mp);
  uint32_t *dst = reinterpret_cast<uint32_t *>(L.s_p);
  for (int i = threadIdx.x; i < (I.n + 1) * h; i += kBlock) {
    const int j = i / h, t = i - j * h;
    uint32_t v = 0;
    if (j < I.n && 2 * t < I.mp)
      v = ((uint32_t)I.p[j * I.mp + 2 * t] & 0xffffu) |
          ((uint32_t)I.p[j * I.mp + 2 * t + 1] << 16);
    dst[i] = v;
  }
  uint32_t *xy = reinterpret_cast<uint32_t *>(L.s_rec);
  for (int i = threadIdx.x; i < I.P * I.npad; i += kBlock) xy[i] = I.xy16[i];
}

// InstView of a loaded instance with the pair table split into LDS chunks of
// at most table_budget bytes (bound.hip).
InstView inst_view(const fsp_instance *inst, size_t table_budget);

}  // namespace fspi
