// Internal declarations of the surrogate's kernels (mlp.hip), used by the
// host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmc {

// Surrogate MLP pieces (mlp.hip)
enum MlpEpi { MLP_EPI_F32 = 0, MLP_EPI_FWD_GELU = 1, MLP_EPI_BWD_GELU = 2 };

// C = A B^T, A [M, K] and B [N, K] bf16 row-major, K % 32 == 0, FP32 accumulation.
//   MLP_EPI_F32:      C[m, n] (float, ldc)
//   MLP_EPI_FWD_GELU: z = acc + bias[n]; Z[m, n] = z (if Z); H[m, n] = GELU(z) (bf16); Ht[n, m] likewise (if Ht)
//   MLP_EPI_BWD_GELU: d = acc * GELU'(Zs[m, n]); H[m, n] = d (bf16); Ht[n, m] likewise (if Ht)
struct MlpGemm {
  const __bf16* A;
  const __bf16* B;
  int M, N, K, lda, ldb;
  int epi;
  const float* bias;
  float* Z;
  int ldz;
  __bf16* H;
  int ldh;
  __bf16* Ht;
  int ldht;
  float* C;
  int ldc;
  const float* Zs;
};
hipError_t mlp_gemm(const MlpGemm& g, hipStream_t s);
hipError_t mlp_pack_input(const float* x, int B, int n_in, __bf16* X, __bf16* Xt, hipStream_t s);
hipError_t mlp_out_fwd(const __bf16* H, int B, int width, const float* w, const float* c, float* y, hipStream_t s);
hipError_t mlp_mse(const float* y, const float* t, int B, float* dy, float* acc, hipStream_t s);
hipError_t mlp_out_bwd_hidden(const float* dy, const float* w, const float* Z, int B, int width, __bf16* G,
                              __bf16* Gt, hipStream_t s);
hipError_t mlp_rowsum(const __bf16* Mt, int R, int B, const float* scale, float* out, hipStream_t s);
hipError_t mlp_adamw(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, hipStream_t s);
hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s);
// Training loop on the device; state[0] = AdamW steps so far, state[1] = its
// value when the loop began (so the loop's step is their difference).
hipError_t mlp_sample_batch(const float* X, const float* y, uint32_t n, int n_in, int batch, uint64_t seed,
                            const uint32_t* state, float* Xb, float* yb, hipStream_t s);
hipError_t mlp_adamw_loop(float* p, float* m, float* v, const float* g, int64_t n, const float* lr_sched,
                          const uint32_t* state, float b1, float b2, float eps, float wd, hipStream_t s);
hipError_t mlp_step_done(uint32_t* state, const float* acc, float* losses, hipStream_t s);

// Fused inference of the 4 x 256 GELU network: y[r] = wout . H4(x[r]) + bout
// for r < n.  Hidden weights are the bf16 copies in [256, kin] layout
// (kin = 32 for layer 1, columns >= n_in zero); n_in <= 32.
struct MlpInfer {
  const float* x;  // [n, n_in]
  int64_t n;
  int n_in;
  const __bf16* W[4];
  const float* bias[4];
  const float* wout;  // [256]
  const float* bout;  // [1]
  float* y;           // [n]
};
hipError_t mlp_infer(const MlpInfer& p, hipStream_t s);

}  // namespace rtmc
