// Internal declarations of the surrogate's kernels (mlp.hip), used by the
// host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmc {

// Surrogate MLP pieces (mlp.hip)
hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s);
// Training loop on the device; state[0] = AdamW steps so far, state[1] = its
// value when the loop began (so the loop's step is their difference).
// mlp_step_done: the step's loss acc[0] to losses[state[0] - state[1]], then one step more.
hipError_t mlp_step_done(uint32_t* state, const float* acc, float* losses, hipStream_t s);

// Fused training of the 4 x 256 GELU network, two launches per step.
// mlp_train_rows: every workgroup takes tiles of 32 batch rows (tile g, g +
// grid, ...): forward through the four layers with the activations in LDS,
// loss, backward, and its share of every gradient -- the tile's sums over its
// rows -- added into its own slice of `part` (n_par floats per workgroup, in
// the padded parameter layout) and of `loss_part`.  Rows are the given
// (x, t), or drawn: row r of loop step s = state[0] - state[1] is row
// floor(u n_src / 2^32) of (src_x, src_t), u the first word of
// Philox4x32-10(key seed, counter (r, s, 0, 0)).
// mlp_train_update: the gradient as the sum of the workgroups' slices in
// workgroup order (reproducible bit for bit) into grad, the loss into acc[0],
// and, with p set, AdamW and the BF16 weight copies.
constexpr int kTrainRows = 32;     // batch rows per tile
constexpr int kTrainMaxWg = 64;    // most workgroups of mlp_train_rows
size_t mlp_train_lds_bytes();
struct MlpTrain {
  const float* master;     // FP32 parameters (biases and the output layer are read from here)
  const __bf16* W[4];      // W_l [256, kin], kin = 32 for layer 1
  const __bf16* Wt[4];     // W_l^T [kin, 256] (layers 2..4)
  int64_t off_W[4], off_b[4], off_wout, off_bout, n_par;
  int batch;               // multiple of 32
  int n_in;
  const float* x;          // [batch, n_in] given rows, or null to draw them
  const float* t;          // [batch]
  const float* src_x;      // [n_src, n_in] rows to draw from
  const float* src_t;
  uint32_t n_src;
  uint64_t seed;
  const uint32_t* state;
  float* zbuf;             // [grid][3][32][256]: pre-activations of layers 1..3
  float* part;             // [grid][n_par]
  float* loss_part;        // [grid]
};
int mlp_train_grid(int batch);
hipError_t mlp_train_rows(const MlpTrain& p, hipStream_t s);
struct MlpUpdate {
  const float* part;
  const float* loss_part;
  int n_part;              // workgroups that wrote slices
  int64_t n_par;
  float* grad;             // [n_par]
  float* acc;              // acc[0] = loss
  // AdamW when p is set: learning rate lr_sched[state[0] - state[1]] and step
  // t = state[0] + 1 when lr_sched is set, else lr and the bias corrections c1, c2
  float* p;
  float *m, *v;
  const float* lr_sched;
  const uint32_t* state;
  float lr, c1, c2, b1, b2, eps, wd;
  __bf16* Wb[4];           // BF16 copies written after the update
  __bf16* Wtb[4];
  int64_t off_W[4];
  int kin[4];
};
hipError_t mlp_train_update(const MlpUpdate& u, hipStream_t s);

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
