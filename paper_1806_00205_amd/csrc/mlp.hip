// Learned surrogate of the yield: an MLP from foam descriptors and (E, cos
// theta) to the RTMC yield, trained on yields the traversal path produces.
// Hidden layers are dense contractions, so they run on gfx950 matrix cores:
// BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16), with bias,
// GELU and its derivative fused into the GEMM epilogues.
//
// One GEMM shape serves the forward and both backward products: C = A * B^T
// with A [M, K] and B [N, K] both K-contiguous (row-major), K a multiple of 32.
//   forward       Z_l  = H_{l-1} W_l^T        (A = H_{l-1} [B, K],  B = W_l [N, K])
//   input grad    dH   = G_l W_l              (A = G_l [B, N],      B = W_l^T [K, N])
//   weight grad   dW_l = G_l^T H_{l-1}        (A = G_l^T [N, B],    B = H_{l-1}^T [K, B])
// so activations and gradients are written in both layouts by the epilogues.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "mlp_kernels.h"

namespace rtmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// erf by Abramowitz and Stegun 7.1.26 (absolute error <= 1.5e-7): branch
// free, one reciprocal and one exponential, far below the BF16 rounding the
// activations then take.
__device__ inline float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  return copysignf(1.0f - poly * __expf(-ax * ax), x);
}

// GELU with the normal CDF, x Phi(x), and its derivative
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ inline float gelu_d(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

// Workgroup tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA blocks of 16 x 16).
// Fragment layout of the 16x16x32 BF16 MFMA (lane l):
//   A: row l % 16, k = 8 (l / 16) .. + 7;  B: column l % 16, same k;
//   C: column l % 16, rows 4 (l / 16) .. + 3.
__global__ __launch_bounds__(256) void k_gemm_nt(MlpGemm g) {
  const int w = threadIdx.x >> 6;
  const uint32_t l = lane_id();
  const int m0 = blockIdx.x * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.y * 64 + (w & 1) * 32;
  const int r = l & 15, kg = (l >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero8 = {};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * i + r;
      a[i] = m < g.M ? *(const GAS bf16x8*)(g.A + (size_t)m * g.lda + k0 + kg) : zero8;
      const int n = n0 + 16 * i + r;
      b[i] = n < g.N ? *(const GAS bf16x8*)(g.B + (size_t)n * g.ldb + k0 + kg) : zero8;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + 16 * j + (l & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * i + 4 * (l >> 4) + q;
        if (m >= g.M) continue;
        const float v = acc[i][j][q];
        if (g.epi == MLP_EPI_F32) {
          g.C[(size_t)m * g.ldc + n] = v;
        } else if (g.epi == MLP_EPI_FWD_GELU) {
          const float z = v + g.bias[n];
          const float h = gelu(z);
          if (g.Z) g.Z[(size_t)m * g.ldz + n] = z;
          g.H[(size_t)m * g.ldh + n] = (__bf16)h;
          if (g.Ht) g.Ht[(size_t)n * g.ldht + m] = (__bf16)h;
        } else {  // MLP_EPI_BWD_GELU: dZ = dH * GELU'(Z)
          const float d = v * gelu_d(g.Zs[(size_t)m * g.ldz + n]);
          g.H[(size_t)m * g.ldh + n] = (__bf16)d;
          if (g.Ht) g.Ht[(size_t)n * g.ldht + m] = (__bf16)d;
        }
      }
    }
}

// Inputs: float [B, n_in] -> bf16 [B, 32] (zero padded) and its transpose [32, B].
__global__ void k_pack_input(const float* __restrict__ x, int B, int n_in, __bf16* __restrict__ X,
                             __bf16* __restrict__ Xt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  for (int k = 0; k < 32; ++k) {
    const __bf16 v = (__bf16)(k < n_in ? x[(size_t)b * n_in + k] : 0.0f);
    X[(size_t)b * 32 + k] = v;
    if (Xt) Xt[(size_t)k * B + b] = v;
  }
}

// Output layer: y = H w + c (one wave per 64 rows, FP32 accumulation).
__global__ void k_out_fwd(const __bf16* __restrict__ H, int B, int width, const float* __restrict__ w,
                          const float* __restrict__ c, float* __restrict__ y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float s = c[0];
  const __bf16* h = H + (size_t)b * width;
  for (int k = 0; k < width; ++k) s += (float)h[k] * w[k];
  y[b] = s;
}

// Loss and output gradient of a batch: dy[b] = 2 (y[b] - t[b]) / B, and
// acc = (mean squared error, sum of dy = the output bias gradient).  One workgroup, each thread summing
// a fixed stride of rows, then a fixed tree: the sums do not depend on
// scheduling, so training is reproducible bit for bit.
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int B, float* __restrict__ dy,
                      float* __restrict__ acc) {
  __shared__ float part[2][256];
  float e = 0.f, g = 0.f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const float d = y[b] - t[b];
    const float gb = 2.0f * d / (float)B;
    dy[b] = gb;
    g += gb;
    e += d * d / (float)B;
  }
  part[0][threadIdx.x] = e;
  part[1][threadIdx.x] = g;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      part[0][threadIdx.x] += part[0][threadIdx.x + s];
      part[1][threadIdx.x] += part[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] = part[0][0];
    acc[1] = part[1][0];
  }
}

// Backward of the output layer into the last hidden layer:
//   G[b, k] = dy[b] w[k] GELU'(Z[b, k]) (bf16, both layouts).
__global__ void k_out_bwd_hidden(const float* __restrict__ dy, const float* __restrict__ w,
                                 const float* __restrict__ Z, int B, int width, __bf16* __restrict__ G,
                                 __bf16* __restrict__ Gt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * width) return;
  const int b = (int)(i / width), k = (int)(i % width);
  const float d = dy[b] * w[k] * gelu_d(Z[i]);
  G[i] = (__bf16)d;
  Gt[(size_t)k * B + b] = (__bf16)d;
}

// Row sums of a [R, B] bf16 matrix into FP32 (bias gradients from G^T), or of
// dy * H^T rows (output weights): out[r] = sum_b Mt[r, b] * (s ? s[b] : 1).
__global__ void k_rowsum(const __bf16* __restrict__ Mt, int R, int B, const float* __restrict__ s,
                         float* __restrict__ out) {
  __shared__ float part[256];
  const int r = blockIdx.x;
  if (r >= R) return;
  float acc = 0.f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) acc += (float)Mt[(size_t)r * B + b] * (s ? s[b] : 1.0f);
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = part[0];
}

// AdamW on the FP32 master parameters (Loshchilov and Hutter), then BF16
// copies of the weight matrices in both layouts.
__global__ void k_adamw(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                        const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
  }
}

// ---- a training loop on the device (one step is replayed as a graph).
// state[0] counts the AdamW steps taken so far, state[1] is its value when
// the loop began, so state[0] - state[1] is the loop's current step s.

// Batch of step s drawn on the device: row r takes row floor(u n / 2^32) of
// (X, y), u the first word of Philox4x32-10 under key seed at counter
// (r, s, 0, 0): uniform sampling with replacement.
__global__ void k_sample_batch(const float* __restrict__ X, const float* __restrict__ y, uint32_t n, int n_in,
                               int batch, uint64_t seed, const uint32_t* __restrict__ state, float* __restrict__ Xb,
                               float* __restrict__ yb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= batch) return;
  const uint32_t s = state[0] - state[1];
  const U4 u = philox(seed, (uint32_t)r, s, 0u, 0u);
  const uint32_t i = __umulhi(u.x, n);
  for (int k = 0; k < n_in; ++k) Xb[(size_t)r * n_in + k] = X[(size_t)i * n_in + k];
  yb[r] = y[i];
}

// AdamW at the loop step's learning rate, bias corrections of step t = state[0] + 1.
__global__ void k_adamw_loop(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, int64_t n, const float* __restrict__ lr_sched,
                             const uint32_t* __restrict__ state, float b1, float b2, float eps, float wd) {
  const uint32_t t = state[0] + 1u;
  const float lr = lr_sched[state[0] - state[1]];
  const float c1 = (float)(1.0 - pow((double)b1, (double)t)), c2 = (float)(1.0 - pow((double)b2, (double)t));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
  }
}

// End of a loop step: its batch loss (before the update) to losses[s]; one step more.
__global__ void k_step_done(uint32_t* state, const float* acc, float* losses) {
  const uint32_t s = state[0] - state[1];
  losses[s] = acc[0];
  state[0] = state[0] + 1u;
}

__global__ void k_to_bf16(const float* __restrict__ W, int rows, int cols, __bf16* __restrict__ Wb,
                          __bf16* __restrict__ Wtb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i % cols;
  const __bf16 v = (__bf16)W[i];
  Wb[i] = v;
  if (Wtb) Wtb[(size_t)c * rows + r] = v;
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

  // layer 1: K = 32 (one MFMA step), inputs straight from memory
  {
    bf16x8 b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *(const GAS bf16x8*)(p.W[0] + (size_t)(n0 + 16 * j + r) * 32 + kg);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t row = row0 + 16 * i + r;
      bf16x8 a = {};
      if (row < p.n) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (kg + e < p.n_in) a[e] = (__bf16)((const GAS float*)p.x)[row * p.n_in + kg + e];
      }
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

hipError_t mlp_gemm(const MlpGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64);
  k_gemm_nt<<<grid, 256, 0, s>>>(g);
  return hipGetLastError();
}

hipError_t mlp_pack_input(const float* x, int B, int n_in, __bf16* X, __bf16* Xt, hipStream_t s) {
  k_pack_input<<<(B + 255) / 256, 256, 0, s>>>(x, B, n_in, X, Xt);
  return hipGetLastError();
}

hipError_t mlp_out_fwd(const __bf16* H, int B, int width, const float* w, const float* c, float* y, hipStream_t s) {
  k_out_fwd<<<(B + 255) / 256, 256, 0, s>>>(H, B, width, w, c, y);
  return hipGetLastError();
}

hipError_t mlp_mse(const float* y, const float* t, int B, float* dy, float* loss_acc, hipStream_t s) {
  k_mse<<<1, 256, 0, s>>>(y, t, B, dy, loss_acc);
  return hipGetLastError();
}

hipError_t mlp_out_bwd_hidden(const float* dy, const float* w, const float* Z, int B, int width, __bf16* G,
                              __bf16* Gt, hipStream_t s) {
  const size_t n = (size_t)B * width;
  k_out_bwd_hidden<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dy, w, Z, B, width, G, Gt);
  return hipGetLastError();
}

hipError_t mlp_rowsum(const __bf16* Mt, int R, int B, const float* scale, float* out, hipStream_t s) {
  k_rowsum<<<R, 256, 0, s>>>(Mt, R, B, scale, out);
  return hipGetLastError();
}

hipError_t mlp_adamw(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, hipStream_t s) {
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  k_adamw<<<grid, 256, 0, s>>>(p, m, v, g, n, lr, b1, b2, eps, wd, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_sample_batch(const float* X, const float* y, uint32_t n, int n_in, int batch, uint64_t seed,
                            const uint32_t* state, float* Xb, float* yb, hipStream_t s) {
  k_sample_batch<<<(batch + 255) / 256, 256, 0, s>>>(X, y, n, n_in, batch, seed, state, Xb, yb);
  return hipGetLastError();
}

hipError_t mlp_adamw_loop(float* p, float* m, float* v, const float* g, int64_t n, const float* lr_sched,
                          const uint32_t* state, float b1, float b2, float eps, float wd, hipStream_t s) {
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  k_adamw_loop<<<grid, 256, 0, s>>>(p, m, v, g, n, lr_sched, state, b1, b2, eps, wd);
  return hipGetLastError();
}

hipError_t mlp_step_done(uint32_t* state, const float* acc, float* losses, hipStream_t s) {
  k_step_done<<<1, 1, 0, s>>>(state, acc, losses);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s) {
  const int n = rows * cols;
  k_to_bf16<<<(n + 255) / 256, 256, 0, s>>>(W, rows, cols, Wb, Wtb);
  return hipGetLastError();
}

}  // namespace rtmc
