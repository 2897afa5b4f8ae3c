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
// Backward: one workgroup per 64-row tile (8 waves, each owning a band of 16
// hidden units); the forward is recomputed, then dW3, dH2, dW2 = H1^T dZ2,
// dH1 = dZ2 W2^T, dW1 = X^T dZ1, the bias sums (products with a ones
// operand) and dX = dZ1 W1^T are products on the matrix cores; each
// workgroup accumulates its weight gradients over its tiles and writes one
// partial; a second kernel sums the partials in a fixed order
// (deterministic).
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
#include <utility>
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
  float w3[kOut][kH];        // W3 as exported (bf16 values), [output][hidden]
};
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Eight waves; wave w owns the band of hidden units [16w, 16w + 16) (column
// tile w) in every product whose output columns are hidden units: h1, h2,
// dZ2, dZ1, and the rows of dW2 / dW3, the columns of dW1.  Its weight
// fragments (W1, W2 and W2^T restricted to the band) are loaded once and
// stay in registers for the whole launch; only the products whose K runs
// over all hidden units (h2, dZ1, and dW2's right operand) read other
// waves' bands, after a barrier.  Two waves share each SIMD, so one issues
// while the other waits on LDS or on its matrix products.  The next tile's
// x and dY are loaded into registers while the current tile is computed.
constexpr int kBwdWaves = 8, kBwdThreads = 64 * kBwdWaves;
// NOUT: the network's outputs (1 .. kOut), a constant of the instantiation so
// that the products over outputs are unrolled to their real length.
template <int NOUT>
__global__ __launch_bounds__(kBwdThreads) void backward_kernel(
    const bf16 *__restrict__ X, int64_t N, const float *__restrict__ P,
    const bf16 *__restrict__ E, const float *__restrict__ dY,
    float *__restrict__ dX, float *__restrict__ partial) {
  constexpr int nout = NOUT;
  extern __shared__ __align__(16) char smem_raw[];
  BwdLds &S = *reinterpret_cast<BwdLds *>(smem_raw);
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  const int col = 16 * w + dcol();  // this lane's hidden unit in D fragments
  bf16x8 fW2t[kH / 32], fW2n[kH / 32];
  const bf16x8 fW1 = frag(E + eW1t, kIn, 16 * w, 0);
  for (int kt = 0; kt < kH / 32; ++kt) {
    fW2t[kt] = frag(E + eW2t, kH, 16 * w, kt * 32);
    fW2n[kt] = frag(E + eW2n, kH, 16 * w, kt * 32);
  }
  const float b1v = P[oB1 + col], b2v = P[oB2 + col];
  for (int e = tid; e < kOut * kH; e += kBwdThreads) S.w3[e / kH][e % kH] = (float)E[eW3t + e];
  // padded outputs of dY stay zero
  for (int e = tid; e < kRows * (kOut + 1); e += kBwdThreads) (&S.dy[0][0])[e] = 0.f;
  for (int e = tid; e < kOut * kLdRows; e += kBwdThreads) (&S.DYt[0][0])[e] = (bf16)0.f;

  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gW2[kH / 16], gW1[kIn / 16], gW3 = zero, gB1 = zero, gB2 = zero;
  for (int b = 0; b < kH / 16; ++b) gW2[b] = zero;
  for (int a = 0; a < kIn / 16; ++a) gW1[a] = zero;
  float gb3 = 0.f;  // threads < 256, (o, q): rows 4q .. 4q + 3 of output o, every tile
  bf16x8 ones;
  for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;

  // threads < 256 stage the tile: x, bf16 8*(t%4) .. +7 of row t/4; dY,
  // floats 4t .. 4t+3 of the tile's [kRows][nout] block (rows past N read as
  // zero)
  const bool stager = tid < 256;
  const bool x16 = (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  bf16x8 xv;
  float dyv[4];
  auto load_tile = [&](int64_t base) {
    const int r = tid >> 2, k0 = 8 * (tid & 3);
    if (base + r < N) {
      const bf16 *src = X + (base + r) * kIn + k0;
      if (x16)
        xv = *reinterpret_cast<const bf16x8 *>(src);
      else
        for (int j = 0; j < 8; ++j) xv[j] = src[j];
    } else {
      for (int j = 0; j < 8; ++j) xv[j] = (bf16)0.f;
    }
    const int64_t avail = (N - base < kRows ? N - base : kRows) * nout;
    for (int q = 0; q < 4; ++q) {
      const int e = 4 * tid + q;
      dyv[q] = e < avail ? dY[base * nout + e] : 0.f;
    }
  };

  const int64_t tiles = (N + kRows - 1) / kRows;
  if (stager && (int64_t)blockIdx.x < tiles) load_tile((int64_t)blockIdx.x * kRows);
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t base = t * kRows;
    __syncthreads();  // the previous tile's readers are done
    if (stager) {
      const int r = tid >> 2, k0 = 8 * (tid & 3);
      *reinterpret_cast<bf16x8 *>(&S.Xr[r][k0]) = xv;
      for (int j = 0; j < 8; ++j) S.Xt[k0 + j][r] = xv[j];
      for (int q = 0; q < 4; ++q) {
        const int e = 4 * tid + q;
        if (e < kRows * nout) {
          const int r2 = e / nout, o = e % nout;
          S.dy[r2][o] = dyv[q];
          S.DYt[o][r2] = (bf16)dyv[q];
        }
      }
    }
    __syncthreads();
    if (stager) {
      if (t + gridDim.x < tiles) load_tile(base + (int64_t)gridDim.x * kRows);
      // bias of layer 3: column sums of dY (fp32); thread (o, q) = (tid % 16,
      // tid / 16) adds rows 4q .. 4q + 3 of output o
      const int o = tid & 15, q = tid >> 4;
      float s3 = 0.f;
      for (int rr = 0; rr < 4; ++rr) s3 += S.dy[4 * q + rr][o];
      gb3 += s3;
    }

    // h1 = relu(x W1 + b1) on the band, every row
    {
      f32x4 acc[kRows / 16];
      for (int rt = 0; rt < kRows / 16; ++rt)
        acc[rt] = mma(frag(&S.Xr[0][0], kLdIn, 16 * rt, 0), fW1, zero);
      for (int rt = 0; rt < kRows / 16; ++rt) {
        bf16x4 v4;
        for (int i = 0; i < 4; ++i) {
          const bf16 v = (bf16)fmaxf(acc[rt][i] + b1v, 0.f);
          S.A1[16 * rt + drow(i)][col] = v;
          v4[i] = v;
        }
        *reinterpret_cast<bf16x4 *>(&S.H1t[col][16 * rt + drow(0)]) = v4;
      }
    }
    __syncthreads();  // h1 complete (h2 reads every band)
    // h2 = relu(h1 W2 + b2) on the band, and from the same registers
    // dZ2[r][c] = (sum_o dY[r][o] W3[c][o]) * (h2 > 0) (VALU, K = nout)
    {
      float w3v[nout];
#pragma unroll
      for (int o = 0; o < nout; ++o) w3v[o] = S.w3[o][col];
      for (int rt = 0; rt < kRows / 16; ++rt) {
        f32x4 acc = zero;
        for (int kt = 0; kt < kH / 32; ++kt)
          acc = mma(frag(&S.A1[0][0], kLdH, 16 * rt, kt * 32), fW2t[kt], acc);
        bf16x4 h4, z4;
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * rt + drow(i);
          const bf16 h = (bf16)fmaxf(acc[i] + b2v, 0.f);
          float sum = 0.f;
#pragma unroll
          for (int o = 0; o < nout; ++o) sum += S.dy[r][o] * w3v[o];
          const bf16 z = (bf16)((float)h > 0.f ? sum : 0.f);
          S.Z2r[r][col] = z;
          h4[i] = h;
          z4[i] = z;
        }
        *reinterpret_cast<bf16x4 *>(&S.H2t[col][16 * rt + drow(0)]) = h4;
        *reinterpret_cast<bf16x4 *>(&S.Z2t[col][16 * rt + drow(0)]) = z4;
      }
    }
    // dW3[c][o] += sum_r h2[r][c] dY[r][o] for the band's c, and the bias of
    // layer 2 as 1^T dZ2 (every row of the result holds the column sums);
    // K = rows
    for (int kt = 0; kt < kRows / 32; ++kt) {
      gW3 = mma(frag(&S.H2t[0][0], kLdRows, 16 * w, kt * 32),
                frag(&S.DYt[0][0], kLdRows, 0, kt * 32), gW3);
      gB2 = mma(ones, frag(&S.Z2t[0][0], kLdRows, 16 * w, kt * 32), gB2);
    }
    __syncthreads();  // dZ2 complete (dW2 and dZ1 read every band)
    // dW2[i][o] += sum_r h1[r][i] dZ2[r][o]: rows i of the band, every o
    for (int kt = 0; kt < kRows / 32; ++kt) {
      const bf16x8 ha = frag(&S.H1t[0][0], kLdRows, 16 * w, kt * 32);
      for (int b = 0; b < kH / 16; ++b)
        gW2[b] = mma(ha, frag(&S.Z2t[0][0], kLdRows, 16 * b, kt * 32), gW2[b]);
    }
    // dZ1 = (dZ2 W2^T) * (h1 > 0) on the band; h1 row-major (A1) is no longer
    // read by any wave (h2 is done everywhere), so dZ1 takes its place
    for (int rt = 0; rt < kRows / 16; ++rt) {
      f32x4 acc = zero;
      for (int kt = 0; kt < kH / 32; ++kt)
        acc = mma(frag(&S.Z2r[0][0], kLdH, 16 * rt, kt * 32), fW2n[kt], acc);
      const bf16x4 h = *reinterpret_cast<const bf16x4 *>(&S.H1t[col][16 * rt + drow(0)]);
      bf16x4 v4;
      for (int i = 0; i < 4; ++i) {
        const float g = (float)h[i] > 0.f ? acc[i] : 0.f;
        const bf16 v = (bf16)g;
        S.A1[16 * rt + drow(i)][col] = v;
        v4[i] = v;
      }
      *reinterpret_cast<bf16x4 *>(&S.Z1t[col][16 * rt + drow(0)]) = v4;
    }
    // dW1[k][i] += sum_r x[r][k] dZ1[r][i]: columns i of the band; bias of
    // layer 1 as 1^T dZ1
    for (int kt = 0; kt < kRows / 32; ++kt) {
      const bf16x8 zb = frag(&S.Z1t[0][0], kLdRows, 16 * w, kt * 32);
      for (int a = 0; a < kIn / 16; ++a)
        gW1[a] = mma(frag(&S.Xt[0][0], kLdRows, 16 * a, kt * 32), zb, gW1[a]);
      gB1 = mma(ones, zb, gB1);
    }
    // dX = dZ1 W1^T (optional): wave w takes row tile w / 2, column tile
    // w % 2; K = 128 over every band
    if (dX) {
      __syncthreads();
      const int rt = w >> 1, nt = w & 1;
      f32x4 acc = zero;
      for (int kt = 0; kt < kH / 32; ++kt)
        acc = mma(frag(&S.A1[0][0], kLdH, 16 * rt, kt * 32),
                  frag(E + eW1n, kH, nt * 16, kt * 32), acc);
      for (int i = 0; i < 4; ++i) {
        const int64_t r = base + 16 * rt + drow(i);
        if (r < N) dX[r * kIn + nt * 16 + dcol()] = acc[i];
      }
    }
  }
  // write this workgroup's partial gradient
  float *G = partial + (size_t)blockIdx.x * kParams;
  for (int b = 0; b < kH / 16; ++b)
    for (int i = 0; i < 4; ++i) G[oW2 + (16 * w + drow(i)) * kH + 16 * b + dcol()] = gW2[b][i];
  for (int a = 0; a < kIn / 16; ++a)
    for (int i = 0; i < 4; ++i) G[oW1 + (16 * a + drow(i)) * kH + col] = gW1[a][i];
  for (int i = 0; i < 4; ++i) G[oW3 + (16 * w + drow(i)) * kOut + dcol()] = gW3[i];
  if (l < 16) {
    G[oB1 + col] = gB1[0];
    G[oB2 + col] = gB2[0];
  }
  // the sixteen row groups of each output, added in a fixed order
  __syncthreads();
  if (stager) (&S.dy[0][0])[tid] = gb3;
  __syncthreads();
  if (tid < kOut) {
    float s3 = 0.f;
    for (int q = 0; q < 16; ++q) s3 += (&S.dy[0][0])[16 * q + tid];
    G[oB3 + tid] = s3;
  }
}

using BwdFn = void (*)(const bf16 *, int64_t, const float *, const bf16 *, const float *,
                      float *, float *);
template <int... Ks>
BwdFn backward_pick(int nout, std::integer_sequence<int, Ks...>) {
  constexpr BwdFn table[] = {backward_kernel<Ks + 1>...};
  return nout >= 1 && nout <= kOut ? table[nout - 1] : nullptr;
}
BwdFn backward_for(int nout) {
  return backward_pick(nout, std::make_integer_sequence<int, kOut>());
}

// grad[j] (+)= sum over partials, in a fixed order
// Workgroup of 256 threads per 64 parameters: wave q adds the partials of
// workgroups [q * chunk, (q + 1) * chunk) in order, then the four wave sums
// are added in the order q = 0 .. 3 (the same order on every run).
__global__ __launch_bounds__(256) void reduce_kernel(const float *__restrict__ partial,
                                                     int nparts, float *__restrict__ grad,
                                                     int accumulate) {
  __shared__ float red[4][64];
  const int jl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  const int chunk = (nparts + 3) / 4;
  const int b0 = q * chunk, b1 = min(nparts, b0 + chunk);
  float s = 0.f;
  if (j < kParams) {
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += partial[(size_t)b * kParams + j];
  }
  red[q][jl] = s;
  __syncthreads();
  if (q == 0 && j < kParams) {
    const float t = ((red[0][jl] + red[1][jl]) + red[2][jl]) + red[3][jl];
    grad[j] = accumulate ? grad[j] + t : t;
  }
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
  int trained_jobs = 0;  // job count of the training instances (0: unknown)
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
int model_trained_jobs(const fsp_model *m) { return m->trained_jobs; }
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

int fsp_model_set_trained_jobs(fsp_model *m, int32_t n) {
  if (!m || n < 0) return FSP_EINVAL;
  m->trained_jobs = n;
  return FSP_OK;
}

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
  const BwdFn fn = backward_for(m->outputs);
  if (!fn) return FSP_EUNSUPPORTED;
  static thread_local bool attr_set[kOut + 1] = {};
  if (!attr_set[m->outputs]) {
    FSP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set[m->outputs] = true;
  }
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBwdThreads), lds, s, reinterpret_cast<const bf16 *>(x), n,
                     m->P, m->E, dy, dx, m->partial);
  hipLaunchKernelGGL(reduce_kernel, dim3((kParams + 63) / 64), dim3(256), 0, s, m->partial,
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
