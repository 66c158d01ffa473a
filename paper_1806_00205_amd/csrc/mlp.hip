// Learned surrogate of the yield: an MLP from foam descriptors and (E, cos
// theta) to the RTMC yield, trained on yields the traversal path produces.
// Hidden layers are dense contractions, so they run on gfx950 matrix cores:
// BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16), with bias,
// GELU and its derivative fused into the GEMM epilogues.
//
// Training runs as three launches per step (k_mlp_train_rows: forward and
// backward signals of 32-row tiles with the activations in LDS;
// k_mlp_train_dw: the weight gradients as GEMMs over the batch's rows;
// k_mlp_train_update: AdamW and the BF16 weight copies); inference as one
// (k_mlp_infer: all layers of a 128-row tile).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "device_util.h"
#include "mlp_kernels.h"

namespace rtmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Upper tail of the standard normal for a >= 0, Q(a) = Phi(-a) = erfc(a /
// sqrt 2) / 2, with erfc from Abramowitz and Stegun 7.1.26 (absolute error
// <= 1.5e-7): Q = t R(t) g with t = 1 / (1 + p a / sqrt 2), R a quartic and
// g = exp(-a^2 / 2), which the derivative reuses (phi(a) = g / sqrt(2 pi)).
// One reciprocal and one exponential, all else explicit fused operations, so
// every kernel rounds it alike.
struct NormTail {
  float q, g;
};
__device__ inline NormTail norm_tail(float a) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.23164188826636f, a, 1.0f));
  float r = fmaf(t, 0.5307027145f, -0.7265760135f);
  r = fmaf(t, r, 0.7107068705f);
  r = fmaf(t, r, -0.142248368f);
  r = fmaf(t, r, 0.127414796f);
  const float g = __builtin_amdgcn_exp2f(a * (a * -0.72134752044448170f));  // 2^(-a^2 log2(e) / 2)
  return {(t * r) * g, g};
}

// GELU with the normal CDF, x Phi(x) = max(x, 0) - |x| Q(|x|) (no
// cancellation in the negative tail), and its derivative Phi(x) + x phi(x)
__device__ inline float gelu(float x) {
  const float a = fabsf(x);
  return fmaf(-a, norm_tail(a).q, fmaxf(x, 0.0f));
}
__device__ inline float gelu_d(float x) {
  const NormTail n = norm_tail(fabsf(x));
  return fmaf(x * 0.39894228040143268f, n.g, x >= 0.0f ? 1.0f - n.q : n.q);
}

// Fragment layout of the 16x16x32 BF16 MFMA (lane l):
//   A: row l % 16, k = 8 (l / 16) .. + 7;  B: column l % 16, same k;
//   C: column l % 16, rows 4 (l / 16) .. + 3.

__global__ void k_to_bf16(const float* __restrict__ W, int rows, int cols, __bf16* __restrict__ Wb,
                          __bf16* __restrict__ Wtb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i % cols;
  const __bf16 v = (__bf16)W[i];
  Wb[i] = v;
  if (Wtb) Wtb[(size_t)c * rows + r] = v;
}

// ---------------------------------------------------------------- fused training
// One workgroup (eight waves, two per SIMD) per tile of 32 batch rows; each
// wave owns 32 of the 256 columns of every [32 x 256] product (2 x 2 MFMA
// blocks).  The roundings are those of the layer-by-layer form: inputs,
// weights, hidden activations and hidden backward signals in BF16,
// pre-activations, sums and the output layer in FP32.
//   forward  Z_l = H_{l-1} W_l^T + b_l,  H_l = GELU(Z_l)    (A: H_{l-1} rows in LDS, B: W_l rows)
//   output   y = H_4 . w_out + b_out,  dy = 2 (y - t) / B,  G_4 = dy w_out GELU'(Z_4)
//   backward db_l += column sums of G_l
//            G_{l-1} = (G_l W_l) GELU'(Z_{l-1})   (A: G_l rows in LDS, B: W_l^T rows)
// H_{l-1}^T and G_l^T leave the workgroup (BF16) for the weight gradients
// dW_l = G_l^T H_{l-1}, which k_mlp_train_dw sums over all rows of the pass.
// LDS (bf16 elements; rows padded by 8 so that 16-byte fragment reads spread over the banks)
constexpr int kTrLdX = 32 + 8;    // [32][40]: the tile's inputs, and X^T
constexpr int kTrLdH = 256 + 8;   // [32][264]: activations or backward signal, row layout
constexpr int kTrLdT = 32 + 8;    // [256][40]: transposed tiles
constexpr int kTrOffX = 0;
constexpr int kTrOffXt = kTrOffX + kTrainRows * kTrLdX;
constexpr int kTrOffH = kTrOffXt + 32 * kTrLdT;
constexpr int kTrOffHt = kTrOffH + kTrainRows * kTrLdH;  // H_1^T, H_2^T, H_3^T
constexpr int kTrOffG = kTrOffHt + 3 * 256 * kTrLdT;
constexpr int kTrOffGt = kTrOffG + kTrainRows * kTrLdH;
constexpr int kTrBf16 = kTrOffGt + 256 * kTrLdT;
constexpr int kTrWaves = 8;                 // waves per workgroup: two per SIMD
constexpr int kTrThreads = 64 * kTrWaves;
constexpr int kTrCols = 256 / kTrWaves;     // columns of each product a wave owns
constexpr int kTrCB = kTrCols / 16;         // ... as 16-wide MFMA blocks
constexpr size_t kTrLdsBytes = (size_t)kTrBf16 * 2 + (size_t)(kTrWaves * kTrainRows + 2 * kTrainRows) * 4;
static_assert((kTrOffXt * 2) % 16 == 0 && (kTrOffH * 2) % 16 == 0 && (kTrOffHt * 2) % 16 == 0 &&
                  (kTrOffG * 2) % 16 == 0 && (kTrOffGt * 2) % 16 == 0 && (kTrBf16 * 2) % 16 == 0,
              "16-byte aligned LDS tiles");

typedef __attribute__((address_space(3))) __bf16 lbf16;
typedef __attribute__((address_space(3))) bf16x8 lbf16x8;
typedef __attribute__((address_space(3))) float lf32;

// out = v on a workgroup's first tile, out += v on its later ones
__device__ inline void accum(float* out, float v, bool first) {
  GAS float* o = (GAS float*)out;
  *o = first ? v : *o + v;
}

// A transposed [n][32] tile of the LDS (row stride kTrLdT) to rows of a
// global [.][ldk] array at column c0: 64 bytes per row, 16 per thread.
__device__ inline void tile_out(const lbf16* src, int n, __bf16* dst, int ldk, int c0) {
  for (int e = threadIdx.x; e < n * 4; e += kTrThreads) {
    const int row = e >> 2, seg = e & 3;
    *(GAS bf16x8*)(dst + (size_t)row * ldk + c0 + 8 * seg) = *(const lbf16x8*)(src + row * kTrLdT + 8 * seg);
  }
}

extern __shared__ __align__(16) unsigned char tr_smem[];

__global__ __launch_bounds__(kTrThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_train_rows(MlpTrain p) {
  lbf16* sb = (lbf16*)tr_smem;
  lf32* ypart = (lf32*)(tr_smem + (size_t)kTrBf16 * 2);  // [kTrWaves][32]
  lf32* sdy = ypart + kTrWaves * kTrainRows;               // [32]
  lf32* stg = sdy + kTrainRows;                            // [32] targets, then loss terms
  const int w = threadIdx.x >> 6;
  const uint32_t l = lane_id();
  const int r = l & 15, kg = (l >> 4) * 8, q4 = 4 * (l >> 4);
  const int n0 = w * kTrCols;  // the wave's columns of every [32 x 256] product
  const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
  float* part = p.part + (size_t)blockIdx.x * kTrainSmall;
  float* zb = p.zbuf + (size_t)blockIdx.x * 3 * kTrainRows * 256;
  const float* mst = p.master;
  const uint32_t step = p.state ? p.state[0] - p.state[1] : 0u;
  const int n_tiles = p.rows / kTrainRows;
  // this lane's columns of the biases and of the output weights, loaded once
  float bcol[4][kTrCB], wcol[kTrCB];
#pragma unroll
  for (int j = 0; j < kTrCB; ++j) {
    const int col = n0 + 16 * j + r;
#pragma unroll
    for (int L = 0; L < 4; ++L) bcol[L][j] = ((const GAS float*)(mst + p.off_b[L]))[col];
    wcol[j] = ((const GAS float*)(mst + p.off_wout))[col];
  }

  for (int tile = blockIdx.x, it = 0; tile < n_tiles; tile += gridDim.x, ++it) {
    const bool first = it == 0 && p.first_pass;  // the workgroup's first tile of the batch
    const int c0 = tile * kTrainRows;              // the tile's first column in gt / ht
    __syncthreads();  // the previous tile's readers of every LDS tile are done
    // ---- the tile's rows, given or drawn: eight threads per row, four inputs
    // each, loads independent of one another (clamped to the row, then masked)
    if (threadIdx.x < 8 * kTrainRows) {
      const int rr = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
      const int row = p.row0 + tile * kTrainRows + rr;
      const GAS float* xr;
      const GAS float* tr;
      if (p.src_x) {
        const U4 u = philox(p.seed, (uint32_t)row, step, 0u, 0u);
        const uint32_t i = __umulhi(u.x, p.n_src);
        xr = (const GAS float*)p.src_x + (size_t)i * p.n_in;
        tr = (const GAS float*)p.src_t + i;
      } else {
        xr = (const GAS float*)p.x + (size_t)row * p.n_in;
        tr = (const GAS float*)p.t + row;
      }
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = c0 + e;
        const float a = xr[k < p.n_in ? k : p.n_in - 1];
        v[e] = k < p.n_in ? a : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const __bf16 h = (__bf16)v[e];
        sb[kTrOffX + rr * kTrLdX + c0 + e] = h;
        sb[kTrOffXt + (c0 + e) * kTrLdT + rr] = h;
      }
      if ((threadIdx.x & 7) == 0) stg[rr] = *tr;
    }
    __syncthreads();
    tile_out(sb + kTrOffXt, 32, p.ht, p.ldk, c0);

    // ---- forward
    f32x4 acc[2][kTrCB];
#pragma unroll 1
    for (int layer = 1; layer <= 4; ++layer) {
      const int K = layer == 1 ? 32 : 256;
      const lbf16* A = sb + (layer == 1 ? kTrOffX : kTrOffH);
      const int lda = layer == 1 ? kTrLdX : kTrLdH;
      const __bf16* W = p.W[layer - 1];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kTrCB; ++j) acc[i][j] = zero4;
      for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 b[kTrCB];
#pragma unroll
        for (int j = 0; j < kTrCB; ++j) b[j] = *(const GAS bf16x8*)(W + (size_t)(n0 + 16 * j + r) * K + k0 + kg);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const bf16x8 a = *(const lbf16x8*)(A + (16 * i + r) * lda + k0 + kg);
#pragma unroll
          for (int j = 0; j < kTrCB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
        }
      }
      float bl[kTrCB];
#pragma unroll
      for (int j = 0; j < kTrCB; ++j) bl[j] = layer == 1 ? bcol[0][j] : (layer == 2 ? bcol[1][j] : (layer == 3 ? bcol[2][j] : bcol[3][j]));
      if (layer < 4) {
        __syncthreads();  // every wave has read the layer's input tile
#pragma unroll
        for (int j = 0; j < kTrCB; ++j) {
          const int col = n0 + 16 * j + r;
          const float bc = bl[j];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int m = 16 * i + q4 + q;
              const float z = acc[i][j][q] + bc;
              ((GAS float*)zb)[((layer - 1) * kTrainRows + m) * 256 + col] = z;
              const __bf16 h = (__bf16)gelu(z);
              sb[kTrOffH + m * kTrLdH + col] = h;
              sb[kTrOffHt + (layer - 1) * 256 * kTrLdT + col * kTrLdT + m] = h;
            }
        }
        __syncthreads();
        tile_out(sb + kTrOffHt + (layer - 1) * 256 * kTrLdT, 256, p.ht + (size_t)(32 + (layer - 1) * 256) * p.ldk,
                 p.ldk, c0);
      } else {
#pragma unroll
        for (int j = 0; j < kTrCB; ++j) {
          const float bc = bl[j];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] += bc;  // Z_4, kept in registers
        }
      }
    }

    // ---- output layer, loss, dy
    // H_4 (as BF16) and GELU'(Z_4) of this lane's elements, one normal tail each
    float h4[2][kTrCB][4], gd4[2][kTrCB][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < kTrCB; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float z = acc[i][j][q];
          const float a = fabsf(z);
          const NormTail n = norm_tail(a);  // gelu and gelu_d, term for term
          h4[i][j][q] = (float)(__bf16)fmaf(-a, n.q, fmaxf(z, 0.0f));
          gd4[i][j][q] = fmaf(z * 0.39894228040143268f, n.g, z >= 0.0f ? 1.0f - n.q : n.q);
        }
    {
      float py[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) py[i][q] = 0.f;
#pragma unroll
      for (int j = 0; j < kTrCB; ++j) {
        const float wc = wcol[j];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) py[i][q] += h4[i][j][q] * wc;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float v = py[i][q];
          v += __shfl_xor(v, 1, 64);
          v += __shfl_xor(v, 2, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 8, 64);
          if (r == 0) ypart[w * kTrainRows + 16 * i + q4 + q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kTrainRows) {
      const int m = threadIdx.x;
      float ys = 0.f;  // the waves' shares in wave order
#pragma unroll
      for (int q = 0; q < kTrWaves; ++q) ys += ypart[q * kTrainRows + m];
      const float y = mst[p.off_bout] + ys;
      const float d = y - stg[m];
      sdy[m] = 2.0f * d / (float)p.batch;
      stg[m] = d * d / (float)p.batch;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // the tile's loss and output-bias gradient, in row order
      float e = 0.f, gb = 0.f;
      for (int m = 0; m < kTrainRows; ++m) {
        e += stg[m];
        gb += sdy[m];
      }
      accum(p.loss_part + blockIdx.x, e, first);
      accum(part + 1280, gb, first);
    }
    // output weights: sum over the tile's rows of H_4 dy; and G_4
    {
      float dyv[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) dyv[i][q] = sdy[16 * i + q4 + q];
#pragma unroll
      for (int j = 0; j < kTrCB; ++j) {
        const int col = n0 + 16 * j + r;
        const float wc = wcol[j];
        float sw = 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = 16 * i + q4 + q;
            sw += h4[i][j][q] * dyv[i][q];
            const __bf16 g = (__bf16)(dyv[i][q] * wc * gd4[i][j][q]);
            sb[kTrOffG + m * kTrLdH + col] = g;
            sb[kTrOffGt + col * kTrLdT + m] = g;
          }
        sw += __shfl_xor(sw, 16, 64);
        sw += __shfl_xor(sw, 32, 64);
        if (l < 16) accum(part + 1024 + col, sw, first);
      }
    }
    __syncthreads();

    // ---- backward
#pragma unroll 1
    for (int layer = 4; layer >= 1; --layer) {
      // G_l^T for the weight gradient
      tile_out(sb + kTrOffGt, 256, p.gt + (size_t)(layer - 1) * 256 * p.ldk, p.ldk, c0);
      // bias gradient: column sums of G, in row order
      if (threadIdx.x < 256) {
        const int n = threadIdx.x;
        float sg = 0.f;
        for (int m = 0; m < kTrainRows; ++m) sg += (float)sb[kTrOffG + m * kTrLdH + n];
        accum(part + 256 * (layer - 1) + n, sg, first);
      }
      if (layer > 1) {
        // G_{l-1} = (G_l W_l) GELU'(Z_{l-1}): rows of G against rows kc of W_l^T
        const __bf16* Wt = p.Wt[layer - 1];
        f32x4 d[2][kTrCB];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < kTrCB; ++j) d[i][j] = zero4;
        for (int k0 = 0; k0 < 256; k0 += 32) {
          bf16x8 b[kTrCB];
#pragma unroll
          for (int j = 0; j < kTrCB; ++j) b[j] = *(const GAS bf16x8*)(Wt + (size_t)(n0 + 16 * j + r) * 256 + k0 + kg);
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const bf16x8 a = *(const lbf16x8*)(sb + kTrOffG + (16 * i + r) * kTrLdH + k0 + kg);
#pragma unroll
            for (int j = 0; j < kTrCB; ++j) d[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], d[i][j], 0, 0, 0);
          }
        }
        __syncthreads();  // every wave is done with G_l and G_l^T
        float zl[2][kTrCB][4];  // Z_{l-1} of this lane's elements, loaded together
#pragma unroll
        for (int j = 0; j < kTrCB; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              zl[i][j][q] = ((const GAS float*)zb)[((layer - 2) * kTrainRows + 16 * i + q4 + q) * 256 + n0 + 16 * j + r];
#pragma unroll
        for (int j = 0; j < kTrCB; ++j) {
          const int col = n0 + 16 * j + r;
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int m = 16 * i + q4 + q;
              const __bf16 g = (__bf16)(d[i][j][q] * gelu_d(zl[i][j][q]));
              sb[kTrOffG + m * kTrLdH + col] = g;
              sb[kTrOffGt + col * kTrLdT + m] = g;
            }
        }
        __syncthreads();
      }
    }
  }
}

// Weight gradients of one pass: dW_l = G_l^T H_{l-1} over its rows (K), one
// workgroup per 16 x 16 block of one layer's gradient (the 16 x 2 blocks of
// layer 1, then 16 x 16 per hidden layer), its four waves taking every fourth
// K step of 32 rows (eight steps' fragments loaded at a time) and their sums
// added in wave order; written on the first pass, added after.  On the last
// pass further workgroups sum the slices of k_mlp_train_rows into the other
// gradient entries, one wave per entry (lane k adds slices k, k + 64, ... in
// order, then a fixed butterfly), and the loss into acc[0].
constexpr int kDwBlocks = 16 * 2 + 3 * 16 * 16;
constexpr int kDwSmallWg = (1281 + 1 + 3) / 4;  // 1281 entries and the loss, four waves per workgroup

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_mlp_train_dw(MlpDw d) {
  const int w = threadIdx.x >> 6;
  const uint32_t l = lane_id();
  if (blockIdx.x >= kDwBlocks) {  // slices and loss (last pass only)
    const int e = (int)(blockIdx.x - kDwBlocks) * 4 + w;
    if (e > 1281) return;
    const float* src = e < 1281 ? d.part + e : d.loss_part;
    const size_t stride = e < 1281 ? (size_t)kTrainSmall : 1;
    float v = 0.f;
    for (int k = (int)l; k < d.n_part; k += 64) v += ((const GAS float*)src)[(size_t)k * stride];
    v = wave_sum_f(v);
    if (l == 0) {
      int64_t o;
      if (e < 1024)
        o = d.off_b[e >> 8] + (e & 255);
      else if (e < 1280)
        o = d.off_wout + (e - 1024);
      else if (e == 1280)
        o = d.off_bout;
      else
        o = -1;
      if (o >= 0) {
        ((GAS float*)d.grad)[o] = v;
      } else {
        ((GAS float*)d.acc)[0] = v;
        if (d.state) {  // device loop: the step's loss and AdamW constants, then one step more
          const uint32_t s = d.state[0] - d.state[1], t = d.state[0] + 1u;
          d.losses[s] = v;
          d.sched[0] = d.lr_sched[s];
          d.sched[1] = (float)(1.0 - pow((double)d.b1, (double)t));
          d.sched[2] = (float)(1.0 - pow((double)d.b2, (double)t));
          d.state[0] = t;
        }
      }
    }
    return;
  }
  int b = blockIdx.x, layer, nb, kb;
  if (b < 32) {
    layer = 0;
    nb = b >> 1;
    kb = b & 1;
  } else {
    b -= 32;
    layer = 1 + (b >> 8);
    nb = (b >> 4) & 15;
    kb = b & 15;
  }
  const int kin = layer == 0 ? 32 : 256;
  const int r = l & 15, kg = (l >> 4) * 8;
  const __bf16* A = d.gt + ((size_t)layer * 256 + 16 * nb + r) * d.ldk + kg;  // G_l^T rows
  const __bf16* B = d.ht + ((size_t)(layer == 0 ? 0 : 32 + (layer - 1) * 256) + 16 * kb + r) * d.ldk + kg;
  const int steps = d.rows / 32;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int s0 = w; s0 < steps; s0 += 32) {
    bf16x8 a[8], bb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int s = min(s0 + 4 * u, steps - 1);  // past the end: a valid step, not used
      a[u] = *(const GAS bf16x8*)(A + 32 * s);
      bb[u] = *(const GAS bf16x8*)(B + 32 * s);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + 4 * u < steps) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], bb[u], acc, 0, 0, 0);
  }
  __shared__ f32x4 red[4][64];
  red[w][l] = acc;
  __syncthreads();
  if (w == 0) {
    const f32x4 v0 = red[0][l], v1 = red[1][l], v2 = red[2][l], v3 = red[3][l];
    GAS float* G = (GAS float*)d.grad + d.off_W[layer];
    const int kc = 16 * kb + r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = 16 * nb + 4 * (l >> 4) + q;
      const float v = ((v0[q] + v1[q]) + v2[q]) + v3[q];
      GAS float* o = G + (size_t)n * kin + kc;
      *o = d.first_pass ? v : *o + v;
    }
  }
}

// AdamW (Loshchilov and Hutter) from the gradient, then the BF16 copies of
// the updated weights.
__global__ __launch_bounds__(256) void k_mlp_train_update(MlpUpdate u) {
  float lr = u.lr, c1 = u.c1, c2 = u.c2;
  if (u.sched) {
    lr = u.sched[0];
    c1 = u.sched[1];
    c2 = u.sched[2];
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < u.n_par; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = ((const GAS float*)u.grad)[i];
    GAS float* P = (GAS float*)u.p;
    GAS float* M = (GAS float*)u.m;
    GAS float* V = (GAS float*)u.v;
    const float mi = u.b1 * M[i] + (1.0f - u.b1) * g;
    const float vi = u.b2 * V[i] + (1.0f - u.b2) * g * g;
    M[i] = mi;
    V[i] = vi;
    const float pi = P[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + u.eps) + u.wd * P[i]);
    P[i] = pi;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
      const int64_t o = i - u.off_W[L];
      if (o >= 0 && o < (int64_t)256 * u.kin[L]) {
        const int rr = (int)(o / u.kin[L]), kk = (int)(o % u.kin[L]);
        const __bf16 v = (__bf16)pi;
        ((GAS __bf16*)u.Wb[L])[o] = v;
        ((GAS __bf16*)u.Wtb[L])[(size_t)kk * 256 + rr] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- inference
// All layers of a 128-row tile in one workgroup.  Each of the four waves owns
// 64 of the 256 output columns for all 128 rows (8 x 4 MFMA blocks, FP32
// accumulators in registers); the layer's input tile is read from LDS, its
// weights from memory (L2-resident, each weight read once per workgroup).
// Between layers the bias + GELU output goes back to the same LDS tile as
// BF16, so activations never reach HBM: per row the kernel reads n_in floats
// and writes one.
constexpr int kInfRows = 128;
constexpr int kInfLd = 256 + 8;  // bf16 per LDS row; the 16-byte pad spreads row reads over banks

typedef __attribute__((address_space(3))) bf16x8 lds_bf16x8;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_infer(MlpInfer p) {
  __shared__ __attribute__((aligned(16))) __bf16 act[kInfRows * kInfLd];
  __shared__ float ypart[4][kInfRows];
  const int w = threadIdx.x >> 6;
  const uint32_t l = lane_id();
  const int r = l & 15, kg = (l >> 4) * 8;
  const int64_t row0 = (int64_t)blockIdx.x * kInfRows;
  const int n0 = w * 64;
  const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[8][4];

  // layer 1: K = 32 (one MFMA step).  The tile's inputs (rows of n_in floats,
  // consecutive in memory) go to the first 32 columns of the LDS tile as
  // BF16, columns n_in .. 31 and rows past n as zeros: one pass of
  // independent unconditional loads, 16 entries per thread, a row's entries in
  // neighbouring lanes.
  {
    bf16x8 b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *(const GAS bf16x8*)(p.W[0] + (size_t)(n0 + 16 * j + r) * 32 + kg);
    const int64_t nrows = p.n - row0;
    float v[kInfRows * 32 / 256];
#pragma unroll
    for (int m = 0; m < kInfRows * 32 / 256; ++m) {
      const int e = (int)threadIdx.x + 256 * m, rr = e >> 5, k = e & 31;
      const bool in = rr < nrows && k < p.n_in;
      // every lane loads (from the tile's first input when its entry is padding), then masks
      const float xv = ((const GAS float*)p.x)[row0 * p.n_in + (in ? rr * p.n_in + k : 0)];
      v[m] = in ? xv : 0.0f;
    }
#pragma unroll
    for (int m = 0; m < kInfRows * 32 / 256; ++m) {
      const int e = (int)threadIdx.x + 256 * m;
      act[(e >> 5) * kInfLd + (e & 31)] = (__bf16)v[m];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bf16x8 a = *(const lds_bf16x8*)((__attribute__((address_space(3))) __bf16*)act + (16 * i + r) * kInfLd + kg);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], zero4, 0, 0, 0);
    }
  }

#pragma unroll 1
  for (int layer = 1; layer < 4; ++layer) {
    // previous layer's output: bias + GELU, BF16, into the LDS tile
    const float* bias = p.bias[layer - 1];
    __syncthreads();  // every wave has finished reading the tile
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + 16 * j + r;
      const float bc = ((const GAS float*)bias)[col];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) act[(16 * i + 4 * (l >> 4) + q) * kInfLd + col] = (__bf16)gelu(acc[i][j][q] + bc);
    }
    __syncthreads();
    const __bf16* W = p.W[layer];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = zero4;
#pragma unroll 2
    for (int k0 = 0; k0 < 256; k0 += 32) {
      bf16x8 b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = *(const GAS bf16x8*)(W + (size_t)(n0 + 16 * j + r) * 256 + k0 + kg);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bf16x8 a = *(const lds_bf16x8*)((__attribute__((address_space(3))) __bf16*)act +
                                              (16 * i + r) * kInfLd + k0 + kg);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
      }
    }
  }

  // output layer from the last hidden layer's accumulators: per row, the
  // wave's 64 columns summed over the 16 lanes that share the row
  const float* b4 = p.bias[3];
  float part[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) part[i][q] = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + 16 * j + r;
    const float bc = ((const GAS float*)b4)[col], wc = ((const GAS float*)p.wout)[col];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) part[i][q] += (float)(__bf16)gelu(acc[i][j][q] + bc) * wc;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v = part[i][q];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if (r == 0) ypart[w][16 * i + 4 * (l >> 4) + q] = v;
    }
  __syncthreads();
  if (threadIdx.x < kInfRows) {
    const int64_t row = row0 + threadIdx.x;
    if (row < p.n) {
      const int t = threadIdx.x;
      ((GAS float*)p.y)[row] = ((const GAS float*)p.bout)[0] + ((ypart[0][t] + ypart[1][t]) + (ypart[2][t] + ypart[3][t]));
    }
  }
}

}  // namespace

hipError_t mlp_infer(const MlpInfer& p, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  const int64_t grid = (p.n + kInfRows - 1) / kInfRows;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  k_mlp_infer<<<(unsigned)grid, 256, 0, s>>>(p);
  return hipGetLastError();
}


size_t mlp_train_lds_bytes() { return kTrLdsBytes; }

int mlp_train_grid(int rows) {
  const int tiles = rows / kTrainRows;
  return tiles < kTrainMaxWg ? tiles : kTrainMaxWg;
}

hipError_t mlp_train_rows(const MlpTrain& p, hipStream_t s) {
  if (p.batch <= 0 || p.batch % kTrainRows || p.rows <= 0 || p.rows % kTrainRows || p.rows > p.ldk ||
      p.row0 < 0 || p.row0 + p.rows > p.batch)
    return hipErrorInvalidValue;
  // the kernel needs more LDS than the default dynamic limit: raise it once per device
  static std::atomic<bool> attr[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!attr[dev].load()) {
    e = hipFuncSetAttribute((const void*)k_mlp_train_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kTrLdsBytes);
    if (e != hipSuccess) return e;
    attr[dev].store(true);
  }
  k_mlp_train_rows<<<mlp_train_grid(p.rows), kTrThreads, kTrLdsBytes, s>>>(p);
  return hipGetLastError();
}

hipError_t mlp_train_dw(const MlpDw& d, hipStream_t s) {
  if (d.rows <= 0 || d.rows % kTrainRows || d.rows > d.ldk || d.n_part <= 0) return hipErrorInvalidValue;
  k_mlp_train_dw<<<kDwBlocks + (d.last_pass ? kDwSmallWg : 0), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t mlp_train_update(const MlpUpdate& u, hipStream_t s) {
  int grid = (int)((u.n_par + 255) / 256);
  if (grid > 4096) grid = 4096;
  k_mlp_train_update<<<grid, 256, 0, s>>>(u);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s) {
  const int n = rows * cols;
  k_to_bf16<<<(n + 255) / 256, 256, 0, s>>>(W, rows, cols, Wb, Wtb);
  return hipGetLastError();
}

}  // namespace rtmc
