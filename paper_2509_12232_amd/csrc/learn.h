// learn.h -- launch records of the learned-proposal kernels: a 96-256-256-32
// perceptron on the matrix cores (bfloat16 operands, float32 accumulation), its
// training (loss, back-propagation, Adam) and the genotype encode / decode /
// move kernels around it.
#pragma once
#include "dock_internal.h"

namespace dock {

constexpr int kMlpIn = 96, kMlpHidden = 256, kMlpOut = 32;
constexpr int kDesc = 64;              // descriptor features
constexpr int kEncGenes = 32;          // encoded genotype features
constexpr int kEncTorsions = kEncGenes - 7;
constexpr int kMlpRowTile = 32;        // rows per matrix-core tile
constexpr int kWgradChunk = 512;       // rows per partial weight gradient

// Offsets of the packed parameter vector: W1 [96][256], b1, W2 [256][256], b2, W3 [256][32], b3.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;

typedef __bf16 bf16;

// bfloat16 copies of the weights in the two layouts the products read:
//   wt_l  [out][in]  (forward: B operand with the reduction index contiguous)
//   wr_l  [in][out]  (back-propagation of errors through layer l)
struct MlpWeights {
  const float *master;  // packed fp32 parameters (biases are read from here)
  const bf16 *wt1, *wt2, *wt3;
  const bf16 *wr2, *wr3;
  const bf16 *wf;       // the three forward weights in MFMA fragment order (kFragW1/2/3)
};

// Fragment order of a forward weight Bt[N][K] (Bt[n][k] = W[k][n]): for output
// tile t (columns 32 t ..) and reduction step s (k = 16 s ..), the 64 lanes'
// B fragments, lane l holding Bt[32 t + l % 32][16 s + 8 (l / 32) + 0..7], are
// 1 KB contiguous, so a wavefront loads a fragment as whole cache lines.
constexpr int kFragW1 = 0;
constexpr int kFragW2 = kFragW1 + kMlpIn * kMlpHidden;
constexpr int kFragW3 = kFragW2 + kMlpHidden * kMlpHidden;
constexpr int kFragTotal = kFragW3 + kMlpHidden * kMlpOut;

// Activation buffers of one batch of rows (mp = rows rounded up to 32).  "p8"
// copies hold eight consecutive rows interleaved, element (r, c) at
// ((r / 8) * cols + c) * 8 + r % 8: the layout in which the weight-gradient
// products read 16-byte fragments along the row (reduction) index.
struct MlpActs {
  int64_t mp;
  bf16 *a0, *a1, *a2;        // row-major [mp][96 / 256 / 256]
  bf16 *a0p8, *a1p8, *a2p8;  // p8 copies (training only, else null)
  float *y;                  // [mp][32]
};

struct MlpGrads {
  bf16 *g3, *g3p8;    // output error  [mp][32]
  bf16 *g2, *g2p8;    // layer-2 error [mp][256]
  bf16 *g1, *g1p8;    // layer-1 error [mp][256]
  float *partial;     // [ceil(mp / kWgradChunk)][256 * 256] partial weight gradients
  float *loss_part;   // per-block loss partial sums
  float *grads;       // packed fp32 gradients [kMlpParams]
  float *loss;        // [1]
};

// x: fp32 rows [m][96] -> a0 (and a0p8 if set); rows m..mp-1 zero.
hipError_t launch_mlp_input(const float *x, int64_t m, const MlpActs &A, hipStream_t s);
// A training batch of m rows, batch row r taken from source row
// order[row0 + r] (or row0 + r without order): inputs -> a0 and a0p8, targets ->
// tb [mp][32], weights -> wb [mp] (when w is set); padding rows zero.
hipError_t launch_mlp_gather(const float *x, const float *t, const float *w, const int32_t *order, int64_t row0,
                             int64_t m, const MlpActs &A, float *tb, float *wb, hipStream_t s);
// a0 -> a1 -> a2 -> y.
hipError_t launch_mlp_forward(const MlpWeights &W, const MlpActs &A, hipStream_t s);
// loss and all gradients of the batch (m valid rows) into G.grads / G.loss.
hipError_t launch_mlp_backward(const MlpWeights &W, const MlpActs &A, const MlpGrads &G, const float *target,
                               const float *weight, int64_t m, hipStream_t s);
// Adam on the packed parameters; refreshes the bfloat16 copies.
struct AdamStep {
  float lr, beta1, beta2, eps;
  float c1, c2;  // 1 - beta1^t, 1 - beta2^t
};
hipError_t launch_mlp_adam(float *master, float *m, float *v, const float *grads, const AdamStep &a, bf16 *wt1,
                           bf16 *wt2, bf16 *wt3, bf16 *wr2, bf16 *wr3, bf16 *wf, hipStream_t s);
// bfloat16 copies from the packed parameters.
hipError_t launch_mlp_refresh(const float *master, bf16 *wt1, bf16 *wt2, bf16 *wt3, bf16 *wr2, bf16 *wr3, bf16 *wf,
                              hipStream_t s);

// Genotype rows of a population [n_ligs][pop][g_stride] (row r = ligand r / pop).
struct PopRows {
  const LigHeader *hdr;
  const float *desc;  // [n_ligs][64]
  int32_t pop, g_stride;
  int64_t n_rows;
  float lo[3], hi[3];  // translation box
};
// network inputs of rows [row0, row0 + n): fp32 x [n][96], or, when a0 is set,
// bfloat16 a0 [a0_rows][96] with rows n .. a0_rows - 1 zero
hipError_t launch_encode(const PopRows &R, int64_t row0, int64_t n, const float *genotypes, float *x, bf16 *a0,
                         int64_t a0_rows, hipStream_t s);
// encoded moves from -> to, [n_rows][32]
hipError_t launch_moves(const PopRows &R, const float *from, const float *to, float *out, hipStream_t s);
// rank weights of n = n_ligs * pop individuals from their energies
hipError_t launch_rank_weights(int64_t n, int32_t pop, const float *energies, double beta, float *w, hipStream_t s);
// proposals = decode(genotypes, network(encode(genotypes)), alpha_max * u) for
// every row, u in (0, 1] from the Philox stream (individual, generation, ligand,
// proposal purpose); one fused launch (encode, the three layers and decode per
// 32 rows, activations in LDS)
hipError_t launch_propose(const PopRows &R, const MlpWeights &W, const float *genotypes, float alpha_max,
                          uint64_t seed, int32_t generation, float *proposals, hipStream_t s);

}  // namespace dock
