// Internal declarations of the surrogate's kernels (mlp.hip), used by the
// host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmc {

// Surrogate MLP pieces (mlp.hip)
hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s);

// Training of the 4 x 256 GELU network, three launches per step (the batch in
// passes of at most kTrainChunk rows, each pass one mlp_train_rows and one
// mlp_train_dw, then one mlp_train_update).
// mlp_train_rows: every workgroup takes tiles of 32 rows of the pass (tile g,
// g + grid, ...): forward through the four layers with the activations in
// LDS, loss, backward signals; it writes the tiles' X^T, H_l^T and G_l^T (BF16)
// for the weight gradients, and adds the tiles' bias, output-weight and loss
// sums into its own slice of `part` and `loss_part` (written on its first tile
// of the batch, added after).  Rows are the given (x, t), or drawn: batch row
// r of loop step s = state[0] - state[1] is row floor(u n_src / 2^32) of
// (src_x, src_t), u the first word of Philox4x32-10(key seed, counter (r, s, 0, 0)).
// mlp_train_dw: dW_l = G_l^T H_{l-1} over the pass's rows into grad (written on
// the first pass, added after); on the last pass also the sums of the slices
// (in a fixed order) into grad's other entries and the loss into acc[0], and,
// in the device training loop (state set: state[0] = AdamW steps so far,
// state[1] its value when the loop began, s = state[0] - state[1] the loop's
// step), the loss to losses[s], the step's learning rate lr_sched[s] and bias
// corrections 1 - b^(state[0] + 1) to sched[0..2], then state[0] + 1.
// mlp_train_update: AdamW from grad and the BF16 weight copies.
// Every sum has a fixed order, so a step is reproducible bit for bit.
constexpr int kTrainRows = 32;       // batch rows per tile
constexpr int kTrainMaxWg = 256;     // most workgroups of mlp_train_rows
constexpr int kTrainChunk = 16384;   // most rows per pass
constexpr int kTrainSmall = 1288;    // slice entries: b_1..b_4 (4 x 256), w_out (256), b_out, padding
size_t mlp_train_lds_bytes();
struct MlpTrain {
  const float* master;     // FP32 parameters (biases and the output layer are read from here)
  const __bf16* W[4];      // W_l [256, kin], kin = 32 for layer 1
  const __bf16* Wt[4];     // W_l^T [kin, 256] (layers 2..4)
  int64_t off_b[4], off_wout, off_bout;
  int batch;               // rows of the whole batch (the loss is their mean), multiple of 32
  int row0, rows;          // this pass: rows row0 .. row0 + rows - 1 of the batch (rows a multiple of 32)
  int first_pass;          // 1 on the batch's first pass
  int n_in;
  const float* x;          // [batch, n_in] given rows, or null to draw them
  const float* t;          // [batch]
  const float* src_x;      // [n_src, n_in] rows to draw from
  const float* src_t;
  uint32_t n_src;
  uint64_t seed;
  const uint32_t* state;
  float* zbuf;             // [grid][3][32][256]: pre-activations of layers 1..3
  __bf16* gt;              // [4][256][ldk]: G_l^T of the pass's rows
  __bf16* ht;              // [32 + 3 x 256][ldk]: X^T, H_1^T, H_2^T, H_3^T of the pass's rows
  int ldk;                 // row length of gt and ht (>= rows, a multiple of 32)
  float* part;             // [grid][kTrainSmall]
  float* loss_part;        // [grid]
};
int mlp_train_grid(int rows);
hipError_t mlp_train_rows(const MlpTrain& p, hipStream_t s);
struct MlpDw {
  const __bf16* gt;
  const __bf16* ht;
  int ldk, rows, first_pass, last_pass;
  float* grad;             // [n_par] in the padded parameter layout
  int64_t off_W[4], off_b[4], off_wout, off_bout;
  const float* part;       // slices of mlp_train_rows, n_part of them
  const float* loss_part;
  int n_part;
  float* acc;              // acc[0] = loss
  uint32_t* state;         // device training loop only (else null)
  float* losses;
  const float* lr_sched;
  float* sched;            // [3]: lr, c1, c2 of the step
  float b1, b2;
};
hipError_t mlp_train_dw(const MlpDw& d, hipStream_t s);
struct MlpUpdate {
  int64_t n_par;
  const float* grad;       // [n_par]
  // AdamW with learning rate and bias corrections sched[0..2] when sched is
  // set (the device loop), else lr, c1, c2
  float* p;
  float *m, *v;
  const float* sched;
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
