// instance.hip -- loading an instance and building its device tables.
//
// The tables are built on the device by three small kernels:
//   stage_rows   one thread per job: padded p, head sums H, tail sums Q
//   stage_totals one thread per machine: column totals
//   stage_pairs  one workgroup per machine pair: every job ranks itself in
//                Johnson's order for that pair (comparison counting, no sort)
//                and writes its record at its rank.
// Johnson's rule with Mitten's lags (the two-machine relaxation of the bound
// whose O(m^2 n log n) cost is quoted in Sec. V.D): with A = a + lag and
// B = b + lag, jobs with A < B come first by A ascending, then the others by
// B descending; equal keys by job id.  Restricting this order to any subset of
// jobs gives that subset's Johnson order, which is why one table per pair
// serves every node.
#include <cstring>
#include <new>

#include "fsp_internal.hpp"

using namespace fspi;

namespace {

__global__ void stage_rows(const int32_t *__restrict__ p_in, int n, int m,
                           int mp, int32_t *__restrict__ p,
                           int32_t *__restrict__ H, int32_t *__restrict__ Q,
                           uint32_t *__restrict__ Hp, uint32_t *__restrict__ Qp) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int row = 0;
  for (int k = 0; k < m; ++k) row += p_in[j * m + k];
  int before = 0;
  for (int k = 0; k < mp; ++k) {
    int v = k < m ? p_in[j * m + k] : 0;
    p[j * mp + k] = v;
    H[j * mp + k] = k < m ? before : 0;
    Q[j * mp + k] = k < m ? row - before - v : 0;
    before += v;
  }
  // sums are <= 65535 (a job's total time), so two fit in a word
  for (int t = 0; t < mp / 2; ++t) {
    Hp[j * (mp / 2) + t] =
        (uint32_t)H[j * mp + 2 * t] | ((uint32_t)H[j * mp + 2 * t + 1] << 16);
    Qp[j * (mp / 2) + t] =
        (uint32_t)Q[j * mp + 2 * t] | ((uint32_t)Q[j * mp + 2 * t + 1] << 16);
  }
}

__global__ void stage_totals(const int32_t *__restrict__ p, int n, int mp,
                             int32_t *__restrict__ tot) {
  int k = threadIdx.x;
  if (k >= mp) return;
  int s = 0;
  for (int j = 0; j < n; ++j) s += p[j * mp + k];
  tot[k] = s;
}

__global__ __launch_bounds__(256) void stage_pairs(
    const int32_t *__restrict__ p, int n, int m, int mp, int npad,
    Rec *__restrict__ rec_out, uint32_t *__restrict__ joff_out,
    uint32_t *__restrict__ xy16_out, uint32_t *__restrict__ job16_out, int npad8,
    uint32_t *__restrict__ bxy_out, uint8_t *__restrict__ bjob_out) {
  __shared__ int sA[256], sB[256];
  const int pi = blockIdx.x;
  // (k,l) of pair pi in lexicographic order
  int k = 0, rem = pi;
  while (rem >= m - 1 - k) {
    rem -= m - 1 - k;
    ++k;
  }
  const int l = k + 1 + rem;
  const int j = threadIdx.x;
  int a = 0, b = 0, lag = 0;
  if (j < n) {
    a = p[j * mp + k];
    b = p[j * mp + l];
    for (int h = k + 1; h < l; ++h) lag += p[j * mp + h];
    sA[j] = a + lag;
    sB[j] = b + lag;
  }
  __syncthreads();
  int pos = j;  // padding slots keep their own index
  if (j < n) {
    const int A = a + lag, B = b + lag;
    const bool first = A < B;
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      const int Ao = sA[o], Bo = sB[o];
      const bool ofirst = Ao < Bo;
      bool before;
      if (ofirst != first)
        before = ofirst;
      else if (first)
        before = Ao < A || (Ao == A && o < j);
      else
        before = Bo > B || (Bo == B && o < j);
      rank += before ? 1 : 0;
    }
    pos = rank;
  }
  if (bxy_out && j < npad8) {
    // the bytes walk's tables; padding: x = y = 0 and job n (a zero flag)
    const size_t slot8 = (size_t)pi * npad8 + pos;
    bxy_out[slot8] = j < n ? ((uint32_t)(b - a) & 0xffffu) | ((uint32_t)(lag + b) << 16) : 0u;
    bjob_out[slot8] = (uint8_t)(j < n ? j : n);
  }
  if (j >= npad) return;
  // Padding records are all-zero and point at job n's mask, which is empty:
  // the walk leaves the pair state unchanged there (see bound.hip).
  int x = 0, y = 0;
  if (j < n) {
    x = 256 * (b - a);
    y = ((lag + b) << 8) | j;
  }
  const size_t slot = (size_t)pi * npad + pos;
  rec_out[slot] = make_int2(x, y);
  joff_out[slot] = 8u * (uint32_t)(j < n ? j : n);
  if (xy16_out) {
    // padding: x = y = 0 leaves the packed state unchanged whatever job the
    // position names (job 0, a valid index)
    uint32_t xy = 0, job = 0;
    if (j < n) {
      xy = ((uint32_t)(b - a) & 0xffffu) | ((uint32_t)(lag + b) << 16);
      job = (uint32_t)j;
    }
    // The packed walk takes the pairs of a row two at a time, (k, k+1) with
    // (k, k+2), (k, k+3) with (k, k+4), ..., the last one alone when the row
    // has an odd count; the two tables of such a couple are interleaved four
    // positions at a time, so that one address serves both.
    const int i = l - k - 1, row = m - 1 - k;
    size_t slot16 = slot;
    if ((i | 1) < row) {
      const size_t base = (size_t)(pi - (i & 1)) * npad;
      slot16 = base + (size_t)(pos / 4) * 8 + (i & 1) * 4 + (pos & 3);
    }
    xy16_out[slot16] = xy;
    job16_out[slot16] = job;
  }
}

void free_device(fsp_instance *in) {
  if (in->d_p) (void)hipFree(in->d_p);
  if (in->d_H) (void)hipFree(in->d_H);
  if (in->d_Q) (void)hipFree(in->d_Q);
  if (in->d_tot) (void)hipFree(in->d_tot);
  if (in->d_rec) (void)hipFree(in->d_rec);
  if (in->d_joff) (void)hipFree(in->d_joff);
  if (in->d_bxy) (void)hipFree(in->d_bxy);
  if (in->d_bjob) (void)hipFree(in->d_bjob);
  if (in->d_xy16) (void)hipFree(in->d_xy16);
  if (in->d_job16) (void)hipFree(in->d_job16);
  if (in->d_Hp) (void)hipFree(in->d_Hp);
  if (in->d_Qp) (void)hipFree(in->d_Qp);
  in->d_Hp = in->d_Qp = nullptr;
  in->d_p = in->d_H = in->d_Q = in->d_tot = nullptr;
  in->d_rec = nullptr;
  in->d_joff = nullptr;
  in->d_bxy = nullptr;
  in->d_bjob = nullptr;
  in->d_xy16 = in->d_job16 = nullptr;
}

int build_tables(fsp_instance *in, const int32_t *p_host) {
  const int n = in->n, m = in->m, mp = in->mp;
  const size_t mat = (size_t)n * mp * sizeof(int32_t);
  if (hipMalloc(&in->d_p, mat) != hipSuccess ||
      hipMalloc(&in->d_H, mat) != hipSuccess ||
      hipMalloc(&in->d_Q, mat) != hipSuccess ||
      hipMalloc(&in->d_tot, mp * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&in->d_rec, (size_t)in->P * in->npad * sizeof(Rec)) != hipSuccess ||
      hipMalloc(&in->d_joff, joff_bytes(in->P, in->npad)) != hipSuccess ||
      (in->npad8 > 0 &&
       (hipMalloc(&in->d_bxy, bytes_entries(in->P, in->npad8) * 4) != hipSuccess ||
        hipMalloc(&in->d_bjob, bytes_entries(in->P, in->npad8)) != hipSuccess)) ||
      (in->p16 && (hipMalloc(&in->d_xy16, (size_t)in->P * in->npad * 4) != hipSuccess ||
                   hipMalloc(&in->d_job16, p16_job_words(in->P, in->npad) * 4) !=
                       hipSuccess)) ||
      hipMalloc(&in->d_Hp, mat / 2) != hipSuccess ||
      hipMalloc(&in->d_Qp, mat / 2) != hipSuccess)
    return FSP_ENOMEM;
  int32_t *d_in = nullptr;
  if (hipMalloc(&d_in, (size_t)n * m * sizeof(int32_t)) != hipSuccess)
    return FSP_ENOMEM;
  hipStream_t s = nullptr;
  int rc = FSP_OK;
  if (hipMemcpy(d_in, p_host, (size_t)n * m * sizeof(int32_t),
                hipMemcpyHostToDevice) != hipSuccess)
    rc = FSP_EDEVICE;
  // the tables' spare entries past the last pair are read, never used (the
  // bytes walk's job 0 names a valid flag row)
  if (rc == FSP_OK &&
      (hipMemset(in->d_joff, 0, joff_bytes(in->P, in->npad)) != hipSuccess ||
       (in->npad8 > 0 &&
        (hipMemset(in->d_bxy, 0, bytes_entries(in->P, in->npad8) * 4) != hipSuccess ||
         hipMemset(in->d_bjob, 0, bytes_entries(in->P, in->npad8)) != hipSuccess))))
    rc = FSP_EDEVICE;
  // likewise the packed job table's spare group (job 0: a valid index)
  if (rc == FSP_OK && in->p16 &&
      hipMemset(in->d_job16, 0, p16_job_words(in->P, in->npad) * 4) != hipSuccess)
    rc = FSP_EDEVICE;
  if (rc == FSP_OK) {
    hipLaunchKernelGGL(stage_rows, dim3((n + 63) / 64), dim3(64), 0, s, d_in,
                       n, m, mp, in->d_p, in->d_H, in->d_Q, in->d_Hp, in->d_Qp);
    hipLaunchKernelGGL(stage_totals, dim3(1), dim3(64), 0, s, in->d_p, n, mp,
                       in->d_tot);
    hipLaunchKernelGGL(stage_pairs, dim3(in->P), dim3(256), 0, s, in->d_p, n,
                       m, mp, in->npad, in->d_rec, in->d_joff,
                       in->d_xy16, in->d_job16, in->npad8, in->d_bxy, in->d_bjob);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
      rc = FSP_EDEVICE;
  }
  (void)hipFree(d_in);
  return rc;
}

}  // namespace

extern "C" {

const char *fsp_status_string(int32_t status) {
  switch (status) {
    case FSP_OK: return "ok";
    case FSP_EINVAL: return "invalid argument";
    case FSP_ENOMEM: return "out of memory";
    case FSP_EDEVICE: return "HIP device error";
    case FSP_EUNSUPPORTED: return "unsupported input for this library";
    case FSP_ESCRATCH:
      return "pool larger than the fixed scratch of the no-allocation entry point";
    default: return "unknown status";
  }
}

int fsp_load_instance(const int32_t *p_host, int32_t n, int32_t m,
                      fsp_instance **out) {
  return fsp_load_instance_ex(p_host, n, m, 0, out);
}

int fsp_load_instance_ex(const int32_t *p_host, int32_t n, int32_t m,
                         int32_t flags, fsp_instance **out) {
  if (!out) return FSP_EINVAL;
  *out = nullptr;
  if (!p_host || n < 1 || m < 2) return FSP_EINVAL;
  if (flags & ~(FSP_LOAD_ONE_NODE_PER_LANE | FSP_LOAD_JOB_MASKS)) return FSP_EINVAL;
  if (n > kMaxJobs || m > kMaxMachines) return FSP_EUNSUPPORTED;
  int64_t total = 0;
  for (int j = 0; j < n; ++j) {
    int64_t row = 0;
    for (int k = 0; k < m; ++k) {
      const int32_t v = p_host[(size_t)j * m + k];
      if (v < 0) return FSP_EINVAL;
      if (v > 32767) return FSP_EUNSUPPORTED;
      row += v;
    }
    if (row > 65535) return FSP_EUNSUPPORTED;
    total += row;
  }
  if (total >= (int64_t(1) << 22)) return FSP_EUNSUPPORTED;

  fsp_instance *in = new (std::nothrow) fsp_instance();
  if (!in) return FSP_ENOMEM;
  in->n = n;
  in->m = m;
  in->mp = round_up(m, 4);
  in->P = npairs(m);
  in->npad = round_up(n, 4);
  in->npad8 = uses_job_masks(n) ? round_up(n, 8) : 0;
  in->wide = n > 32 ? 1 : 0;
  in->p16 = (n <= 32 && total <= 32767 && !(flags & FSP_LOAD_ONE_NODE_PER_LANE)) ? 1 : 0;
  in->masks_walk = (flags & FSP_LOAD_JOB_MASKS) ? 1 : 0;
  in->p_host.assign(p_host, p_host + (size_t)n * m);
  if (hipGetDevice(&in->device) != hipSuccess) {
    delete in;
    return FSP_EDEVICE;
  }
  int rc = build_tables(in, p_host);
  if (rc != FSP_OK) {
    free_device(in);
    delete in;
    return rc;
  }
  *out = in;
  return FSP_OK;
}

int fsp_free_instance(fsp_instance *inst) {
  if (!inst) return FSP_OK;
  free_device(inst);
  delete inst;
  return FSP_OK;
}

int fsp_instance_info(const fsp_instance *inst, int32_t *n, int32_t *m,
                      int32_t *device) {
  if (!inst) return FSP_EINVAL;
  if (n) *n = inst->n;
  if (m) *m = inst->m;
  if (device) *device = inst->device;
  return FSP_OK;
}

int fsp_instance_path(const fsp_instance *inst, int32_t *path) {
  if (!inst || !path) return FSP_EINVAL;
  if (inst->wide)
    *path = !uses_job_masks(inst->n) ? FSP_PATH_REGISTER64
            : inst->masks_walk      ? FSP_PATH_MASKS
                                    : FSP_PATH_BYTES;
  else
    *path = inst->p16 ? FSP_PATH_PACKED : FSP_PATH_REGISTER;
  return FSP_OK;
}

}  // extern "C"
