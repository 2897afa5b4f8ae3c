// mlp.hip -- the pool-policy network: a 3-layer perceptron
//     h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3
// with x in R^32 (node features, zero padded), 128 hidden units per layer and
// up to 16 outputs.  Weights are kept in fp32 (master copy, Adam state) and
// exported to bf16 for the matrix cores; products run as bf16 MFMA
// (v_mfma_f32_16x16x32_bf16) with fp32 accumulation; activations and the
// gradients that feed a product are rounded to bf16 exactly where a product
// consumes them.
//
// Forward: layers computed transposed so that each result tile is already
// the next layer's operand (see forward_kernel); weights and biases stay in
// registers and each wave streams 16-row tiles.
// Backward: one workgroup per 64-row tile (4 waves); the forward is recomputed,
// then dW3, dH2, dW2 = H1^T dZ2, dH1 = dZ2 W2^T, dW1 = X^T dZ1 and dX = dZ1 W1^T
// are products on the matrix cores; each workgroup accumulates its weight
// gradients over its tiles and writes one partial; a second kernel sums the
// partials in a fixed order (deterministic).
//
// MFMA 16x16x32 bf16 fragments (lane l, g = l / 16, c = l % 16):
//   A (16 x 32): A[c][8g .. 8g+7]      B (32 x 16): B[8g .. 8g+7][c]
//   D (16 x 16): D[4g + i][c], i = 0..3
// so both operands are read as 8 consecutive bf16 along K; every operand is
// kept "K-contiguous" in memory (B as its transpose, N x K).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "fsp_internal.hpp"
#include "bnb.hpp"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32;    // padded input features
constexpr int kH = 128;    // hidden units
constexpr int kOut = 16;   // padded outputs
constexpr int kRows = 64;  // rows per backward tile

// parameter vector (fp32): W1[kIn][kH] b1[kH] W2[kH][kH] b2[kH] W3[kH][kOut] b3[kOut]
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kIn * kH;
constexpr int oW2 = oB1 + kH;
constexpr int oB2 = oW2 + kH * kH;
constexpr int oW3 = oB2 + kH;
constexpr int oB3 = oW3 + kH * kOut;
constexpr int kParams = oB3 + kOut;

// bf16 exports, all K-contiguous:
//   W1t [kH][kIn]  (forward layer 1: B = W1, N = hidden, K = input)
//   W1n [kIn][kH]  (dX = dZ1 W1^T: N = input, K = hidden)
//   W2t [kH][kH]   (forward layer 2: [out][in])
//   W2n [kH][kH]   (dH1 = dZ2 W2^T: [in][out])
//   W3t [kOut][kH] (forward layer 3: [out][in])
constexpr int eW1t = 0;
constexpr int eW1n = eW1t + kH * kIn;
constexpr int eW2t = eW1n + kIn * kH;
constexpr int eW2n = eW2t + kH * kH;
constexpr int eW3t = eW2n + kH * kH;
// Forward-kernel layouts of W2 and W3 (A operands of the transposed products,
// see forward_kernel): [out][kt][g][j] = W[32 kt + perm(g, j)][out] with
// perm(g, j) = 4g + j for j < 4 and 16 + 4g + (j - 4) for j >= 4.
constexpr int eW2p = eW3t + kOut * kH;
constexpr int eW3p = eW2p + kH * kH;
constexpr int kExport = eW3p + kOut * kH;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ bf16x8 frag(const bf16 *base, int ld, int r0, int k0) {
  const int l = lane_id();
  return *reinterpret_cast<const bf16x8 *>(base + (size_t)(r0 + (l & 15)) * ld + k0 +
                                           8 * (l >> 4));
}

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// D fragment coordinates of this lane: rows r0 + 4g + i, column c0 + c
__device__ __forceinline__ int drow(int i) { return 4 * (lane_id() >> 4) + i; }
__device__ __forceinline__ int dcol() { return lane_id() & 15; }

// ---------------------------------------------------------------------------
// export fp32 master weights to the bf16 operand layouts
__global__ void export_kernel(const float *__restrict__ P, bf16 *__restrict__ E) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kIn * kH) {
    const int k = t / kH, i = t % kH;  // W1[k][i]
    const bf16 v = (bf16)P[oW1 + t];
    E[eW1t + i * kIn + k] = v;
    E[eW1n + k * kH + i] = v;
  }
  if (t < kH * kH) {
    const int i = t / kH, o = t % kH;  // W2[i][o]
    const bf16 v = (bf16)P[oW2 + t];
    E[eW2t + o * kH + i] = v;
    E[eW2n + i * kH + o] = v;
  }
  if (t < kH * kOut) {
    const int c = t / kOut, o = t % kOut;  // W3[c][o]
    E[eW3t + o * kH + c] = (bf16)P[oW3 + t];
  }
  // permuted-K layouts, indexed by destination: t = ((out * 4 + kt) * 4 + g) * 8 + j
  {
    const int j = t & 7, g = (t >> 3) & 3, kt = (t >> 5) & 3, out = t >> 7;
    const int in = 32 * kt + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
    if (t < kH * kH) E[eW2p + t] = (bf16)P[oW2 + in * kH + out];
    if (t < kOut * kH) E[eW3p + t] = (bf16)P[oW3 + in * kOut + out];
  }
}

// ---------------------------------------------------------------------------
// forward: x [N][kIn] bf16 -> y [N][nout] fp32
//
// Every layer is computed transposed, Z^T = W^T A^T: the MFMA A operand is a
// 16-feature slice of W^T, the B operand 16 rows of the layer input.  The
// result tile holds, in lane (g, c), features 4g .. 4g+3 of row c, which is
// half of what lane (g, c) must supply as the next layer's B operand for a
// 32-feature K step.  Taking two consecutive result tiles gives the lane
// features {4g..4g+3} and {16+4g..16+4g+3} of the step: a fixed permutation
// of K, which the next layer's weights follow (the eW2p / eW3p exports), so
// no activation passes through LDS.  The bias is the accumulator's initial
// value.  All 44 weight fragments and the biases stay in registers for the
// whole kernel; each wave streams 16-row tiles.
__device__ __forceinline__ bf16x8 relu_pack(f32x4 a, f32x4 b) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = (bf16)fmaxf(a[i], 0.f);
    r[4 + i] = (bf16)fmaxf(b[i], 0.f);
  }
  return r;
}

__global__ __launch_bounds__(256) void forward_kernel(
    const bf16 *__restrict__ X, int64_t N, const int32_t *__restrict__ n_dev,
    const float *__restrict__ P, const bf16 *__restrict__ E, float *__restrict__ Y,
    int nout, const fspi::ScoreEpilogue sc) {
  if (n_dev) N = *n_dev;  // row count produced on the device
  if (N <= 0) return;
  const int l = lane_id(), g = l >> 4, c = l & 15;
  const int wave = threadIdx.x >> 6;
  // A operands: lane (g, c) holds out feature 16 mt + c, K elements 8g .. 8g+7
  // of the step (permuted for W2 and W3)
  bf16x8 w1[kH / 16], w2[kH / 16][kH / 32], w3[kH / 32];
  f32x4 b1[kH / 16], b2[kH / 16], b3;
#pragma unroll
  for (int mt = 0; mt < kH / 16; ++mt) {
    w1[mt] = *reinterpret_cast<const bf16x8 *>(E + eW1t + (mt * 16 + c) * kIn + 8 * g);
#pragma unroll
    for (int kt = 0; kt < kH / 32; ++kt)
      w2[mt][kt] = *reinterpret_cast<const bf16x8 *>(
          E + eW2p + ((mt * 16 + c) * 4 + kt) * 32 + 8 * g);
    b1[mt] = *reinterpret_cast<const f32x4 *>(P + oB1 + mt * 16 + 4 * g);
    b2[mt] = *reinterpret_cast<const f32x4 *>(P + oB2 + mt * 16 + 4 * g);
  }
#pragma unroll
  for (int kt = 0; kt < kH / 32; ++kt)
    w3[kt] = *reinterpret_cast<const bf16x8 *>(E + eW3p + (c * 4 + kt) * 32 + 8 * g);
  b3 = *reinterpret_cast<const f32x4 *>(P + oB3 + 4 * g);

  const int64_t tiles = (N + 15) / 16;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tiles;
       t += (int64_t)gridDim.x * 4) {
    const int64_t row = t * 16 + c;
    const int64_t rr = row < N ? row : N - 1;
    const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(X + rr * kIn + 8 * g);
    bf16x8 h1[kH / 32];
#pragma unroll
    for (int kt = 0; kt < kH / 32; ++kt) {
      const f32x4 a0 = mma(w1[2 * kt], xb, b1[2 * kt]);
      const f32x4 a1 = mma(w1[2 * kt + 1], xb, b1[2 * kt + 1]);
      h1[kt] = relu_pack(a0, a1);
    }
    bf16x8 h2[kH / 32];
#pragma unroll
    for (int ot = 0; ot < kH / 32; ++ot) {
      f32x4 a0 = b2[2 * ot], a1 = b2[2 * ot + 1];
#pragma unroll
      for (int kt = 0; kt < kH / 32; ++kt) {
        a0 = mma(w2[2 * ot][kt], h1[kt], a0);
        a1 = mma(w2[2 * ot + 1][kt], h1[kt], a1);
      }
      h2[ot] = relu_pack(a0, a1);
    }
    f32x4 y = b3;
#pragma unroll
    for (int kt = 0; kt < kH / 32; ++kt) y = mma(w3[kt], h2[kt], y);
    if (row < N) {
      if (sc.est) {
        if (g == 0) {
          const int64_t at = sc.rowdst[row];
          sc.est[at] = (float)sc.lb[at] * sc.inv_scale + y[0];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < nout) Y[row * nout + 4 * g + i] = y[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// backward: per 64-row tile, recompute the forward, then every gradient.
// dY [N][nout] fp32 is given.  Each workgroup writes one partial gradient
// vector (fp32, kParams) to partial[blockIdx.x]; dX (optional) [N][kIn] fp32.
// Every LDS row is padded by 16 bytes, so consecutive rows start 4 banks
// apart: the 16-byte fragment reads of 8 rows then cover all 32 banks once,
// and column-wise accesses conflict 8-way at most (64-way unpadded, where a
// row of 64 bf16 is exactly one pass over the banks).
constexpr int kPad = 8;
constexpr int kLdIn = kIn + kPad, kLdRows = kRows + kPad, kLdH = kH + kPad;
struct BwdLds {
  bf16 Xr[kRows][kLdIn];     // x, row-major
  bf16 Xt[kIn][kLdRows];     // x, transposed
  bf16 A1[kRows][kLdH];      // h1 row-major, then dZ1 row-major
  bf16 H1t[kH][kLdRows];     // h1 transposed
  bf16 H2t[kH][kLdRows];     // h2 transposed
  bf16 Z2r[kRows][kLdH];     // dZ2 row-major
  bf16 Z2t[kH][kLdRows];     // dZ2 transposed
  bf16 Z1t[kH][kLdRows];     // dZ1 transposed
  bf16 DYt[kOut][kLdRows];   // dY transposed (bf16, padded outputs)
  float dy[kRows][kOut + 1]; // dY fp32 (padded outputs, odd row stride)
};
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void backward_kernel(
    const bf16 *__restrict__ X, int64_t N, const float *__restrict__ P,
    const bf16 *__restrict__ E, const float *__restrict__ dY, int nout,
    float *__restrict__ dX, float *__restrict__ partial) {
  extern __shared__ __align__(16) char smem_raw[];
  BwdLds &S = *reinterpret_cast<BwdLds *>(smem_raw);
  const int tid = threadIdx.x, w = tid >> 6;
  // per-wave accumulators: dW2 tiles (wave w owns output rows i in [32w, 32w+32)),
  // dW1 tiles (wave w owns columns i in [32w, 32w+32)), dW3 (wave w rows c in [32w,32w+32))
  f32x4 gW2[2][8];
  f32x4 gW1[2][2];
  f32x4 gW3[2];
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 8; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < 2; ++b) gW1[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    gW3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;  // thread t < kH: column t

  const int64_t tiles = (N + kRows - 1) / kRows;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    // opaque per tile: otherwise every weight fragment is loop-invariant and
    // gets hoisted out of the tile loop into registers of its own
    asm volatile("" : "+s"(E), "+s"(P));
    const int64_t base = t * kRows;
    __syncthreads();
    // load x (rows past N are zero) and dY
    for (int e = tid; e < kRows * kIn; e += 256) {
      const int r = e / kIn, k = e % kIn;
      const bf16 v = base + r < N ? X[(base + r) * kIn + k] : (bf16)0.f;
      S.Xr[r][k] = v;
      S.Xt[k][r] = v;
    }
    for (int e = tid; e < kRows * kOut; e += 256) {
      const int r = e / kOut, o = e % kOut;
      const float v = (base + r < N && o < nout) ? dY[(base + r) * nout + o] : 0.f;
      S.dy[r][o] = v;
      S.DYt[o][r] = (bf16)v;
    }
    __syncthreads();
    // h1 = relu(x W1 + b1): wave w rows [16w, 16w+16)
    {
      const bf16x8 xa = frag(&S.Xr[0][0], kLdIn, 16 * w, 0);
      for (int nt = 0; nt < kH / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma(xa, frag(E + eW1t, kIn, nt * 16, 0), acc);
        const int col = nt * 16 + dcol();
        const float b = P[oB1 + col];
        bf16x4 t;
        for (int i = 0; i < 4; ++i) {
          const bf16 v = (bf16)fmaxf(acc[i] + b, 0.f);
          S.A1[16 * w + drow(i)][col] = v;
          t[i] = v;
        }
        // rows 16w + 4g .. +3 of the transposed copy in one 8-byte store
        *reinterpret_cast<bf16x4 *>(&S.H1t[col][16 * w + drow(0)]) = t;
      }
    }
    __syncthreads();
    // h2 = relu(h1 W2 + b2)
    for (int nt = 0; nt < kH / 16; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < kH / 32; ++kt)
        acc = mma(frag(&S.A1[0][0], kLdH, 16 * w, kt * 32),
                  frag(E + eW2t, kH, nt * 16, kt * 32), acc);
      const int col = nt * 16 + dcol();
      const float b = P[oB2 + col];
      bf16x4 t;
      for (int i = 0; i < 4; ++i) t[i] = (bf16)fmaxf(acc[i] + b, 0.f);
      *reinterpret_cast<bf16x4 *>(&S.H2t[col][16 * w + drow(0)]) = t;
    }
    __syncthreads();
    // dW3[c][o] += sum_r h2[r][c] dY[r][o]: wave w, c-tiles 2w, 2w+1; K = 64 rows
    for (int a = 0; a < 2; ++a)
      for (int kt = 0; kt < kRows / 32; ++kt)
        gW3[a] = mma(frag(&S.H2t[0][0], kLdRows, 32 * w + 16 * a, kt * 32),
                     frag(&S.DYt[0][0], kLdRows, 0, kt * 32), gW3[a]);
    // dZ2[r][c] = (sum_o dY[r][o] W3[c][o]) * (h2 > 0)   (VALU: K = nout)
    // consecutive lanes take consecutive rows of one column c: the transposed
    // accesses are then contiguous, and W3's row c is one broadcast
    for (int e = tid; e < kRows * kH; e += 256) {
      const int r = e % kRows, c = e / kRows;
      float s = 0.f;
      for (int o = 0; o < nout; ++o) s += S.dy[r][o] * (float)E[eW3t + o * kH + c];
      const float g = (float)S.H2t[c][r] > 0.f ? s : 0.f;
      const bf16 v = (bf16)g;
      S.Z2r[r][c] = v;
      S.Z2t[c][r] = v;
    }
    __syncthreads();
    // dW2[i][o] += sum_r h1[r][i] dZ2[r][o]: wave w owns i-tiles 2w, 2w+1
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 8; ++b)
        for (int kt = 0; kt < kRows / 32; ++kt)
          gW2[a][b] = mma(frag(&S.H1t[0][0], kLdRows, 32 * w + 16 * a, kt * 32),
                          frag(&S.Z2t[0][0], kLdRows, 16 * b, kt * 32), gW2[a][b]);
    // dZ1 = (dZ2 W2^T) * (h1 > 0): wave w rows [16w, 16w+16)
    {
      f32x4 acc[kH / 16];
      for (int nt = 0; nt < kH / 16; ++nt) {
        acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kH / 32; ++kt)
          acc[nt] = mma(frag(&S.Z2r[0][0], kLdH, 16 * w, kt * 32),
                        frag(E + eW2n, kH, nt * 16, kt * 32), acc[nt]);
      }
      __syncthreads();  // every wave is done reading A1 as h1 (layer 2) long ago;
                        // this barrier orders the masks below after all reads
      for (int nt = 0; nt < kH / 16; ++nt) {
        const int col = nt * 16 + dcol();
        const bf16x4 h = *reinterpret_cast<const bf16x4 *>(&S.H1t[col][16 * w + drow(0)]);
        bf16x4 t;
        for (int i = 0; i < 4; ++i) {
          const float g = (float)h[i] > 0.f ? acc[nt][i] : 0.f;
          const bf16 v = (bf16)g;
          S.A1[16 * w + drow(i)][col] = v;  // dZ1 row-major
          t[i] = v;
        }
        *reinterpret_cast<bf16x4 *>(&S.Z1t[col][16 * w + drow(0)]) = t;
      }
    }
    __syncthreads();
    // dW1[k][i] += sum_r x[r][k] dZ1[r][i]: k-tiles 0,1; wave w owns i-tiles 2w, 2w+1
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int kt = 0; kt < kRows / 32; ++kt)
          gW1[a][b] = mma(frag(&S.Xt[0][0], kLdRows, 16 * a, kt * 32),
                          frag(&S.Z1t[0][0], kLdRows, 32 * w + 16 * b, kt * 32), gW1[a][b]);
    // dX = dZ1 W1^T: wave w rows [16w, 16w+16), 2 column tiles, K = 128
    if (dX) {
      for (int nt = 0; nt < kIn / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kH / 32; ++kt)
          acc = mma(frag(&S.A1[0][0], kLdH, 16 * w, kt * 32),
                    frag(E + eW1n, kH, nt * 16, kt * 32), acc);
        const int col = nt * 16 + dcol();
        for (int i = 0; i < 4; ++i) {
          const int64_t r = base + 16 * w + drow(i);
          if (r < N) dX[r * kIn + col] = acc[i];
        }
      }
    }
    // bias gradients: column sums, from the row-major copies (consecutive
    // threads read consecutive columns)
    if (tid < kH) {
      float s1 = 0.f, s2 = 0.f;
      for (int r = 0; r < kRows; ++r) {
        s1 += (float)S.A1[r][tid];
        s2 += (float)S.Z2r[r][tid];
      }
      gb1 += s1;
      gb2 += s2;
    }
    if (tid < kOut) {
      float s3 = 0.f;
      for (int r = 0; r < kRows; ++r) s3 += S.dy[r][tid];
      gb3 += s3;
    }
  }
  // write this workgroup's partial gradient
  float *G = partial + (size_t)blockIdx.x * kParams;
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 8; ++b) {
      const int col = 16 * b + dcol();
      for (int i = 0; i < 4; ++i) {
        const int row = 32 * w + 16 * a + drow(i);
        G[oW2 + row * kH + col] = gW2[a][b][i];
      }
    }
    for (int b = 0; b < 2; ++b) {
      const int col = 32 * w + 16 * b + dcol();
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * a + drow(i);
        G[oW1 + row * kH + col] = gW1[a][b][i];
      }
    }
    {
      const int col = dcol();
      for (int i = 0; i < 4; ++i) {
        const int row = 32 * w + 16 * a + drow(i);
        G[oW3 + row * kOut + col] = gW3[a][i];
      }
    }
  }
  if (tid < kH) {
    G[oB1 + tid] = gb1;
    G[oB2 + tid] = gb2;
  }
  if (tid < kOut) G[oB3 + tid] = gb3;
}

// grad[j] (+)= sum over partials, in workgroup order
__global__ void reduce_kernel(const float *__restrict__ partial, int nparts,
                              float *__restrict__ grad, int accumulate) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kParams) return;
  float s = 0.f;
  for (int b = 0; b < nparts; ++b) s += partial[(size_t)b * kParams + j];
  grad[j] = accumulate ? grad[j] + s : s;
}

__global__ void adam_kernel(float *__restrict__ P, const float *__restrict__ G,
                            float *__restrict__ m1, float *__restrict__ m2,
                            const uint8_t *__restrict__ mask, float lr, float b1,
                            float b2, float eps, float wd, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kParams || !mask[j]) return;
  const float g = G[j] + wd * P[j];
  m1[j] = b1 * m1[j] + (1.f - b1) * g;
  m2[j] = b2 * m2[j] + (1.f - b2) * g * g;
  P[j] -= lr * (m1[j] / c1) / (sqrtf(m2[j] / c2) + eps);
}

// loss gradient for training: output 0 regression (squared error), output 1
// logistic (binary cross-entropy on the logit); weights per row (may be 0)
__global__ void loss_grad_kernel(const float *__restrict__ Y, const float *__restrict__ T,
                                 int64_t N, int nout, float inv_n, float *__restrict__ dY,
                                 float *__restrict__ loss) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (r < N) {
    const float y0 = Y[r * nout + 0], t0 = T[r * 2 + 0];
    const float d0 = y0 - t0;
    dY[r * nout + 0] = 2.f * d0 * inv_n;
    l += d0 * d0;
    if (nout > 1) {
      const float y1 = Y[r * nout + 1], t1 = T[r * 2 + 1];
      const float s = 1.f / (1.f + expf(-y1));
      dY[r * nout + 1] = (s - t1) * inv_n;
      l += fmaxf(y1, 0.f) - y1 * t1 + log1pf(expf(-fabsf(y1)));
    }
    for (int o = 2; o < nout; ++o) dY[r * nout + o] = 0.f;
  }
  // one atomic per wave
  for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l * inv_n);
}

}  // namespace

struct fsp_model {
  int device = 0;
  int in_features = 0, outputs = 0;
  float *P = nullptr, *G = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint8_t *mask = nullptr;  // 1 for parameters that exist at this size
  bf16 *E = nullptr;
  float *partial = nullptr;
  int nparts = 0;
  int64_t step = 0;
  // training scratch
  float *Y = nullptr, *dY = nullptr, *loss = nullptr;
  int64_t scratch_rows = 0;
  int cus = 0;
};

namespace {

void model_free(fsp_model *m) {
  for (void *p : {(void *)m->P, (void *)m->G, (void *)m->m1, (void *)m->m2, (void *)m->mask,
                  (void *)m->E, (void *)m->partial, (void *)m->Y, (void *)m->dY,
                  (void *)m->loss})
    if (p) (void)hipFree(p);
  delete m;
}

// splitmix64 (Steele, Lea, Flood 2014): deterministic initial weights
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

int export_weights(fsp_model *m, hipStream_t s) {
  hipLaunchKernelGGL(export_kernel, dim3((kH * kH + 255) / 256), dim3(256), 0, s, m->P, m->E);  // covers every layout
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int ensure_scratch(fsp_model *m, int64_t rows) {
  if (rows <= m->scratch_rows) return FSP_OK;
  if (m->Y) (void)hipFree(m->Y);
  if (m->dY) (void)hipFree(m->dY);
  m->Y = m->dY = nullptr;
  if (hipMalloc(&m->Y, (size_t)rows * m->outputs * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->dY, (size_t)rows * m->outputs * sizeof(float)) != hipSuccess)
    return FSP_ENOMEM;
  m->scratch_rows = rows;
  return FSP_OK;
}

}  // namespace

namespace fspi {
int forward_launch(const fsp_model *m, const void *x, const int32_t *n_dev, int64_t max_n,
                   float *y, const ScoreEpilogue &sc, hipStream_t s) {
  if (max_n <= 0) return FSP_OK;
  // one workgroup per CU: every wave keeps all weights in registers and
  // streams 16-row tiles
  const int64_t tiles = (max_n + 15) / 16;
  int64_t grid = (tiles + 3) / 4;
  if (grid > (int64_t)m->cus) grid = (int64_t)m->cus;
  hipLaunchKernelGGL(forward_kernel, dim3((unsigned)grid), dim3(256), 0, s,
                     reinterpret_cast<const bf16 *>(x), max_n, n_dev, m->P, m->E, y,
                     m->outputs, sc);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}
int model_forward_dev(const fsp_model *m, const void *x, const int32_t *n_dev, int64_t max_n,
                      float *y, hipStream_t s) {
  return forward_launch(m, x, n_dev, max_n, y, ScoreEpilogue{}, s);
}
int model_forward_score_dev(const fsp_model *m, const void *x, const int32_t *n_dev,
                            int64_t max_n, const ScoreEpilogue &sc, hipStream_t s) {
  return forward_launch(m, x, n_dev, max_n, nullptr, sc, s);
}
int model_forward(const fsp_model *m, const void *x, int64_t n, float *y, hipStream_t s) {
  return model_forward_dev(m, x, nullptr, n, y, s);
}
int model_outputs(const fsp_model *m) { return m->outputs; }
int model_in_features(const fsp_model *m) { return m->in_features; }
}  // namespace fspi

extern "C" {

int fsp_model_create(int32_t in_features, int32_t hidden, int32_t outputs, uint64_t seed,
                     fsp_model **out) {
  if (!out) return FSP_EINVAL;
  *out = nullptr;
  if (in_features < 1 || outputs < 1) return FSP_EINVAL;
  if (in_features > kIn || hidden != kH || outputs > kOut) return FSP_EUNSUPPORTED;
  fsp_model *m = new (std::nothrow) fsp_model();
  if (!m) return FSP_ENOMEM;
  m->in_features = in_features;
  m->outputs = outputs;
  if (hipGetDevice(&m->device) != hipSuccess ||
      hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, m->device) !=
          hipSuccess) {
    model_free(m);
    return FSP_EDEVICE;
  }
  m->nparts = m->cus;  // one backward workgroup per compute unit
  const size_t pb = kParams * sizeof(float);
  if (hipMalloc(&m->P, pb) != hipSuccess || hipMalloc(&m->G, pb) != hipSuccess ||
      hipMalloc(&m->m1, pb) != hipSuccess || hipMalloc(&m->m2, pb) != hipSuccess ||
      hipMalloc(&m->mask, kParams) != hipSuccess ||
      hipMalloc(&m->E, kExport * sizeof(bf16)) != hipSuccess ||
      hipMalloc(&m->partial, (size_t)m->nparts * pb) != hipSuccess ||
      hipMalloc(&m->loss, sizeof(float)) != hipSuccess) {
    model_free(m);
    return FSP_ENOMEM;
  }
  // He-uniform initial weights on the existing rows/columns, zero elsewhere
  std::vector<float> P(kParams, 0.f);
  std::vector<uint8_t> mask(kParams, 0);
  uint64_t s = seed;
  auto uni = [&](float a) {
    const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
    return (float)((2.0 * u - 1.0) * a);
  };
  const float a1 = std::sqrt(6.f / in_features), a2 = std::sqrt(6.f / kH),
              a3 = std::sqrt(6.f / kH);
  for (int k = 0; k < in_features; ++k)
    for (int i = 0; i < kH; ++i) {
      P[oW1 + k * kH + i] = uni(a1);
      mask[oW1 + k * kH + i] = 1;
    }
  for (int i = 0; i < kH; ++i) mask[oB1 + i] = mask[oB2 + i] = 1;
  for (int i = 0; i < kH * kH; ++i) {
    P[oW2 + i] = uni(a2);
    mask[oW2 + i] = 1;
  }
  for (int c = 0; c < kH; ++c)
    for (int o = 0; o < outputs; ++o) {
      P[oW3 + c * kOut + o] = uni(a3) * 0.1f;
      mask[oW3 + c * kOut + o] = 1;
    }
  for (int o = 0; o < outputs; ++o) mask[oB3 + o] = 1;
  if (hipMemcpy(m->P, P.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->mask, mask.data(), kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->G, 0, pb) != hipSuccess || hipMemset(m->m1, 0, pb) != hipSuccess ||
      hipMemset(m->m2, 0, pb) != hipSuccess || export_weights(m, nullptr) != FSP_OK ||
      hipDeviceSynchronize() != hipSuccess) {
    model_free(m);
    return FSP_EDEVICE;
  }
  *out = m;
  return FSP_OK;
}

int fsp_model_free(fsp_model *m) {
  if (m) model_free(m);
  return FSP_OK;
}

int64_t fsp_model_param_count(void) { return kParams; }

int fsp_model_set_params(fsp_model *m, const float *host, int64_t n) {
  if (!m || !host || n != kParams) return FSP_EINVAL;
  FSP_HIP_TRY(hipMemcpy(m->P, host, kParams * sizeof(float), hipMemcpyHostToDevice));
  int rc = export_weights(m, nullptr);
  if (rc != FSP_OK) return rc;
  FSP_HIP_TRY(hipDeviceSynchronize());
  return FSP_OK;
}

int fsp_model_get_params(const fsp_model *m, float *host, int64_t n) {
  if (!m || !host || n != kParams) return FSP_EINVAL;
  FSP_HIP_TRY(hipMemcpy(host, m->P, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return FSP_OK;
}

int fsp_model_get_grads(const fsp_model *m, float *host, int64_t n) {
  if (!m || !host || n != kParams) return FSP_EINVAL;
  FSP_HIP_TRY(hipMemcpy(host, m->G, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return FSP_OK;
}

int fsp_model_forward(const fsp_model *m, const void *x, int64_t n, float *y, void *stream) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return FSP_EINVAL;
  return fspi::model_forward(m, x, n, y, reinterpret_cast<hipStream_t>(stream));
}

int fsp_model_backward(fsp_model *m, const void *x, int64_t n, const float *dy, float *dx,
                       int32_t accumulate, void *stream) {
  if (!m || n < 0 || (n > 0 && (!x || !dy))) return FSP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t tiles = (n + kRows - 1) / kRows;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, m->nparts));
  const size_t lds = sizeof(BwdLds);
  static thread_local bool attr_set = false;
  if (!attr_set) {
    FSP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(backward_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  hipLaunchKernelGGL(backward_kernel, dim3(grid), dim3(256), lds, s,
                     reinterpret_cast<const bf16 *>(x), n, m->P, m->E, dy, m->outputs, dx,
                     m->partial);
  hipLaunchKernelGGL(reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, m->partial,
                     grid, m->G, accumulate ? 1 : 0);
  FSP_HIP_TRY(hipGetLastError());
  return FSP_OK;
}

int fsp_model_adam_step(fsp_model *m, float lr, float beta1, float beta2, float eps,
                        float weight_decay, void *stream) {
  if (!m) return FSP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  m->step += 1;
  const float c1 = 1.f - std::pow(beta1, (float)m->step);
  const float c2 = 1.f - std::pow(beta2, (float)m->step);
  hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, m->P, m->G,
                     m->m1, m->m2, m->mask, lr, beta1, beta2, eps, weight_decay, c1, c2);
  FSP_HIP_TRY(hipGetLastError());
  return export_weights(m, s);
}

int fsp_model_train_step(fsp_model *m, const void *x, const float *target, int64_t n, float lr,
                         float *loss_out, void *stream) {
  if (!m || n <= 0 || !x || !target) return FSP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = ensure_scratch(m, n);
  if (rc != FSP_OK) return rc;
  rc = fspi::model_forward(m, x, n, m->Y, s);
  if (rc != FSP_OK) return rc;
  FSP_HIP_TRY(hipMemsetAsync(m->loss, 0, sizeof(float), s));
  hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m->Y,
                     target, n, m->outputs, 1.f / (float)n, m->dY, m->loss);
  FSP_HIP_TRY(hipGetLastError());
  rc = fsp_model_backward(m, x, n, m->dY, nullptr, 0, stream);
  if (rc != FSP_OK) return rc;
  rc = fsp_model_adam_step(m, lr, 0.9f, 0.999f, 1e-8f, 0.f, stream);
  if (rc != FSP_OK) return rc;
  if (loss_out) {
    FSP_HIP_TRY(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    FSP_HIP_TRY(hipStreamSynchronize(s));
  }
  return FSP_OK;
}

}  // extern "C"
