// learn.hip -- the learned proposal on gfx950: a 96-256-256-32 perceptron whose
// products run on the matrix cores (v_mfma_f32_32x32x16_bf16: bfloat16 operands,
// float32 accumulation), its training step (squared-error loss,
// back-propagation, Adam) and the kernels that turn genotypes into network
// inputs and network outputs into proposal genotypes.
//
// Every training product is one wavefront per 32x32 output tile.  Operands are
// kept in HBM in layouts where each lane's eight bfloat16 values of a fragment
// are one 16-byte load: activations row-major (reduction index contiguous) for
// the forward and error products, and eight-row interleaved ("p8") copies for
// the weight-gradient products, whose reduction index is the row.  The fused
// proposal kernel reads a further copy of the forward weights in fragment
// order, where a whole fragment is one contiguous kilobyte.
#include <math.h>

#include "learn.h"
#include "philox.h"

namespace dock {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 frag(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Lane l of a 32x32 accumulator holds column l % 32 and rows
// 8 (r / 4) + 4 (l / 32) + r % 4 of its registers r = 0..15.
__device__ __forceinline__ int acc_row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

__device__ __forceinline__ int64_t p8_index(int64_t row, int cols, int col) {
  return (((row >> 3) * cols + col) << 3) + (row & 7);
}

// ------------------------------------------------------------------- products
enum { kEpiRelu = 0, kEpiOut = 1, kEpiMask = 2 };

// D[mp][N] = A[mp][K] * B, with B given as Bt[N][K]; epilogue by EPI:
//   kEpiRelu: bfloat16(max(D + bias, 0))   -> out (+ out_p8)
//   kEpiOut:  D + bias                      -> out_f32
//   kEpiMask: bfloat16(D where mask > 0)    -> out (+ out_p8)
struct GemmRK {
  const bf16 *A;
  const bf16 *Bt;
  int64_t mp;
  int32_t N, K;
  const float *bias;
  const bf16 *mask;
  bf16 *out;
  bf16 *out_p8;
  float *out_f32;
  int32_t waves_n;  // wavefronts of a block along N (1, 2 or 4)
};

template <int EPI>
__global__ __launch_bounds__(256) void gemm_rk_kernel(GemmRK g) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wm = 4 / g.waves_n;
  const int64_t tm = (int64_t)blockIdx.x * wm + wave / g.waves_n;
  const int tn = blockIdx.y * g.waves_n + wave % g.waves_n;
  if (tm * kMlpRowTile >= g.mp || tn * 32 >= g.N) return;
  const bf16 *a = g.A + (tm * kMlpRowTile + (l & 31)) * g.K + 8 * (l >> 5);
  const bf16 *b = g.Bt + (int64_t)(tn * 32 + (l & 31)) * g.K + 8 * (l >> 5);
  f32x16 acc = {};
  for (int k = 0; k < g.K; k += 16) acc = mfma(frag(a + k), frag(b + k), acc);
  const int col = tn * 32 + (l & 31);
  const float bias = EPI == kEpiMask ? 0.f : g.bias[col];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = tm * kMlpRowTile + acc_row(r, l);
    float v = acc[r] + bias;
    if (EPI == kEpiOut) {
      g.out_f32[row * g.N + col] = v;
      continue;
    }
    if (EPI == kEpiRelu) v = v > 0.f ? v : 0.f;
    if (EPI == kEpiMask) v = (float)g.mask[row * g.N + col] > 0.f ? v : 0.f;
    const bf16 h = (bf16)v;
    g.out[row * g.N + col] = h;
    if (g.out_p8) g.out_p8[p8_index(row, g.N, col)] = h;
  }
}

// partial[c][K][N] = sum over rows m of chunk c of X[m][k] Z[m][n], from the p8
// copies of X [mp][K] and Z [mp][N].
struct GemmWG {
  const bf16 *Xp8;
  const bf16 *Zp8;
  int64_t mp;
  int32_t K, N;
  float *partial;
};

__global__ __launch_bounds__(256) void gemm_wgrad_kernel(GemmWG g) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tiles_n = g.N / 32;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= (g.K / 32) * tiles_n) return;
  const int ti = tile / tiles_n, tn = tile % tiles_n;
  const int64_t m0 = (int64_t)blockIdx.y * kWgradChunk;
  const int64_t m1 = m0 + kWgradChunk < g.mp ? m0 + kWgradChunk : g.mp;
  f32x16 acc = {};
  for (int64_t m = m0; m < m1; m += 16) {
    const int64_t blk = (m >> 3) + (l >> 5);
    acc = mfma(frag(g.Xp8 + ((blk * g.K + ti * 32 + (l & 31)) << 3)),
               frag(g.Zp8 + ((blk * g.N + tn * 32 + (l & 31)) << 3)), acc);
  }
  float *out = g.partial + (int64_t)blockIdx.y * g.K * g.N;
  const int col = tn * 32 + (l & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) out[(ti * 32 + acc_row(r, l)) * g.N + col] = acc[r];
}

// out[i] = sum_c partial[c][i], in chunk order
__global__ void reduce_partial_kernel(const float *partial, int chunks, int n, float *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * n + i];
  out[i] = s;
}

// partial[chunk][c] = sum over the rows m of the chunk (kColsumChunk rows) of
// Z[m][c] (row order); neighbouring threads read neighbouring columns of a row
constexpr int kColsumChunk = 64;

__global__ void colsum_partial_kernel(const bf16 *Z, int64_t mp, int N, float *partial) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int64_t m0 = (int64_t)blockIdx.y * kColsumChunk;
  const int64_t m1 = m0 + kColsumChunk < mp ? m0 + kColsumChunk : mp;
  float s = 0.f;
  for (int64_t m = m0; m < m1; ++m) s += (float)Z[m * N + c];
  partial[(int64_t)blockIdx.y * N + c] = s;
}

// ------------------------------------------------------------ input, loss, Adam
__global__ void mlp_input_kernel(const float *x, int64_t m, int64_t mp, bf16 *a0, bf16 *a0p8) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mp * kMlpIn) return;
  const int64_t row = i / kMlpIn;
  const int c = (int)(i % kMlpIn);
  const bf16 h = (bf16)(row < m ? x[i] : 0.f);
  a0[i] = h;
  if (a0p8) a0p8[p8_index(row, kMlpIn, c)] = h;
}

__global__ void mlp_gather_kernel(const float *x, const float *t, const float *w, const int32_t *order, int64_t row0,
                                  int64_t m, int64_t mp, bf16 *a0, bf16 *a0p8, float *tb, float *wb) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mp) return;
  const int64_t src = r < m ? (order ? (int64_t)order[row0 + r] : row0 + r) : -1;
  for (int c = 0; c < kMlpIn; ++c) {
    const bf16 h = (bf16)(src >= 0 ? x[src * kMlpIn + c] : 0.f);
    a0[r * kMlpIn + c] = h;
    a0p8[p8_index(r, kMlpIn, c)] = h;
  }
  for (int c = 0; c < kMlpOut; ++c) tb[r * kMlpOut + c] = src >= 0 ? t[src * kMlpOut + c] : 0.f;
  if (wb) wb[r] = src >= 0 ? w[src] : 0.f;
}

// g = bfloat16((2 / m) w (y - t)) for valid rows, 0 for padding rows; per-block
// sums of w (y - t)^2 (fixed tree order).
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float *y, const float *t, const float *w, int64_t m,
                                                       int64_t mp, float scale, bf16 *g, bf16 *gp8, float *part) {
  __shared__ float sh[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float sq = 0.f;
  if (i < mp * kMlpOut) {
    const int64_t row = i / kMlpOut;
    const int c = (int)(i % kMlpOut);
    float d = 0.f;
    if (row < m) {
      const float wr = w ? w[row] : 1.f;
      const float e = y[i] - t[row * kMlpOut + c];
      sq = wr * e * e;
      d = scale * wr * e;
    }
    const bf16 h = (bf16)d;
    g[i] = h;
    gp8[p8_index(row, kMlpOut, c)] = h;
  }
  sh[threadIdx.x] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[0] = scale * sum of part[0 .. n): one block of 256 threads, thread t
// summing part[t], part[t + 256], ... in order, then a fixed tree -- the same
// order on every call
__global__ __launch_bounds__(256) void ordered_sum_kernel(const float *part, int n, float scale, float *out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

// Position of Bt[n][k] of a [N][K] forward weight in fragment order.
__device__ __forceinline__ int frag_index(int n, int k, int K) {
  const int t = n >> 5, c = n & 31, s = k >> 4, kk = k & 15;
  return (((t * (K >> 4) + s) * kWave + c + 32 * (kk >> 3)) << 3) + (kk & 7);
}

// bfloat16 copies of weight element e of the packed vector (e < kOffW3 + 256 * 32,
// biases excluded by the caller).
__device__ __forceinline__ void store_weight_copies(int e, float v, bf16 *wt1, bf16 *wt2, bf16 *wt3, bf16 *wr2,
                                                    bf16 *wr3, bf16 *wf) {
  const bf16 h = (bf16)v;
  if (e < kOffB1) {
    const int k = e / kMlpHidden, n = e % kMlpHidden;
    wt1[n * kMlpIn + k] = h;
    wf[kFragW1 + frag_index(n, k, kMlpIn)] = h;
  } else if (e >= kOffW2 && e < kOffB2) {
    const int o = e - kOffW2, k = o / kMlpHidden, n = o % kMlpHidden;
    wt2[n * kMlpHidden + k] = h;
    wr2[k * kMlpHidden + n] = h;
    wf[kFragW2 + frag_index(n, k, kMlpHidden)] = h;
  } else if (e >= kOffW3 && e < kOffB3) {
    const int o = e - kOffW3, k = o / kMlpOut, n = o % kMlpOut;
    wt3[n * kMlpHidden + k] = h;
    wr3[k * kMlpOut + n] = h;
    wf[kFragW3 + frag_index(n, k, kMlpHidden)] = h;
  }
}

__global__ void mlp_refresh_kernel(const float *master, bf16 *wt1, bf16 *wt2, bf16 *wt3, bf16 *wr2, bf16 *wr3,
                                   bf16 *wf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpParams) return;
  store_weight_copies(e, master[e], wt1, wt2, wt3, wr2, wr3, wf);
}

// Adam (Kingma & Ba, ICLR 2015) with bias correction c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void mlp_adam_kernel(float *p, float *m, float *v, const float *grads, AdamStep a, bf16 *wt1, bf16 *wt2,
                                bf16 *wt3, bf16 *wr2, bf16 *wr3, bf16 *wf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpParams) return;
  const float g = grads[e];
  const float mm = a.beta1 * m[e] + (1.f - a.beta1) * g;
  const float vv = a.beta2 * v[e] + (1.f - a.beta2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const float w = p[e] - a.lr * (mm / a.c1) / (sqrtf(vv / a.c2) + a.eps);
  p[e] = w;
  store_weight_copies(e, w, wt1, wt2, wt3, wr2, wr3, wf);
}

// ------------------------------------------------------------------ genotypes
constexpr float kPiF = 3.14159265358979323846f;
constexpr float kTwoPiF = 6.28318530717958647692f;

__device__ __forceinline__ float wrapf(float a) {
  a = fmodf(a, kTwoPiF);
  if (a > kPiF) a -= kTwoPiF;
  else if (a <= -kPiF) a += kTwoPiF;
  return a;
}

// unit quaternion with w >= 0; identity for a zero quaternion
// (selects instead of an early return, so that q stays in registers)
__device__ __forceinline__ void canonical_q(const float *g, float q[4]) {
  const float nn = g[3] * g[3] + g[4] * g[4] + g[5] * g[5] + g[6] * g[6];
  const bool ident = nn < 1e-24f;
  float s = 1.f / sqrtf(ident ? 1.f : nn);
  if (g[3] < 0.f) s = -s;
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = ident ? (c == 0 ? 1.f : 0.f) : g[3 + c] * s;
}

__device__ __forceinline__ void box_half(const PopRows &R, int d, float &c, float &h) {
  c = 0.5f * (R.lo[d] + R.hi[d]);
  h = 0.5f * (R.hi[d] - R.lo[d]);
}

// Network input of one genotype row: 32 encoded genes, then the ligand's 64
// descriptor features.
__device__ void encode_row(const PopRows &R, int64_t r, const float *genotypes, float f[kMlpIn]) {
  const int lig = (int)(r / R.pop);
  const float *g = genotypes + r * R.g_stride;
  const int nt = min(R.hdr[lig].n_tors, kEncTorsions);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float c, h;
    box_half(R, d, c, h);
    f[d] = h > 0.f ? (g[d] - c) / h : 0.f;
  }
  float q[4];
  canonical_q(g, q);
  for (int c = 0; c < 4; ++c) f[3 + c] = q[c];
  for (int k = 0; k < kEncTorsions; ++k) f[7 + k] = k < nt ? g[7 + k] / kPiF : 0.f;
  const float *ds = R.desc + (int64_t)lig * kDesc;
  for (int j = 0; j < kDesc; ++j) f[kEncGenes + j] = ds[j];
}

__global__ void encode_kernel(PopRows R, int64_t row0, int64_t n, const float *genotypes, float *x, bf16 *a0,
                              int64_t a0_rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = a0 ? a0_rows : n;
  if (i >= rows) return;
  float f[kMlpIn];
  if (i < n) {
    encode_row(R, row0 + i, genotypes, f);
  } else {
    for (int j = 0; j < kMlpIn; ++j) f[j] = 0.f;
  }
  if (a0) {
    bf16 *o = a0 + i * kMlpIn;
    for (int j = 0; j < kMlpIn; ++j) o[j] = (bf16)f[j];
  } else {
    float *o = x + i * kMlpIn;
    for (int j = 0; j < kMlpIn; ++j) o[j] = f[j];
  }
}

__global__ void moves_kernel(PopRows R, const float *from, const float *to, float *out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R.n_rows) return;
  const int lig = (int)(r / R.pop);
  const float *a = from + r * R.g_stride, *b = to + r * R.g_stride;
  float *o = out + r * kMlpOut;
  const int nt = min(R.hdr[lig].n_tors, kEncTorsions);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float c, h;
    box_half(R, d, c, h);
    o[d] = h > 0.f ? (b[d] - a[d]) / h : 0.f;
  }
  float qa[4], qb[4];
  canonical_q(a, qa);
  canonical_q(b, qb);
  const float dot = qa[0] * qb[0] + qa[1] * qb[1] + qa[2] * qb[2] + qa[3] * qb[3];
  const float sgn = dot < 0.f ? -1.f : 1.f;
  for (int c = 0; c < 4; ++c) o[3 + c] = sgn * qb[c] - qa[c];
  for (int k = 0; k < kEncTorsions; ++k) o[7 + k] = k < nt ? wrapf(b[7 + k] - a[7 + k]) / kPiF : 0.f;
}

// Proposal of population row r from its network output yy (32 values).
__device__ void decode_row(const PopRows &R, int64_t r, const float *genotypes, const float *yy, float alpha_max,
                           uint64_t seed, int32_t generation, float *prop) {
  const int lig = (int)(r / R.pop), ind = (int)(r % R.pop);
  const float *g = genotypes + r * R.g_stride;
  float *o = prop + r * R.g_stride;
  DrawStream s(seed, (uint64_t)ind, (uint64_t)generation, (uint64_t)lig, kPurposeProposal);
  const float alpha = alpha_max * (float)(1.0 - s.unit());
  // the row copied as is first (genes past the encoded torsions keep their
  // values), in blocks whose loads are issued before their stores
  {
    const float *__restrict__ src = g;
    float *__restrict__ dst = o;
    const int G = R.g_stride;
    for (int j0 = 0; j0 < G; j0 += 8) {
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = src[min(j0 + i, G - 1)];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (j0 + i < G) dst[j0 + i] = v[i];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float c, h;
    box_half(R, d, c, h);
    const float v = g[d] + alpha * h * yy[d];
    o[d] = fminf(fmaxf(v, R.lo[d]), R.hi[d]);
  }
  float q[4];
  canonical_q(g, q);
  for (int c = 0; c < 4; ++c) o[3 + c] = q[c] + alpha * yy[3 + c];
  const int nt = min(R.hdr[lig].n_tors, kEncTorsions);
  for (int k = 0; k < nt; ++k) o[7 + k] = wrapf(g[7 + k] + alpha * kPiF * yy[7 + k]);
}

// ---------------------------------------------------- fused proposal kernel
// One wavefront takes 32 population rows through encode,
// the three layers and decode.  The rows' activations stay in LDS, one padded
// row per individual (the padding puts consecutive rows' 16-byte fragments in
// different banks); weight fragments stream from L2 in fragment order (each a
// contiguous 1 KB), where every wavefront reads the same 196 KB.  The products
// run in the same k order as the per-layer kernels, so the network output is
// the same to the bit.
constexpr int kPropWaves = 4;                     // wavefronts of a workgroup
constexpr int kPropRows = 32 * kPropWaves;        // rows of a workgroup, 32 per wavefront
constexpr int kHStride = kMlpHidden + 8;  // bfloat16 per LDS row

__device__ __forceinline__ bf16x8 lds_frag(const bf16 *h, int l, int k0) {
  return *reinterpret_cast<const bf16x8 *>(h + (l & 31) * kHStride + k0 + 8 * (l >> 5));
}

// acc[t] = h[rows][0..K) * W for NT column tiles of 32, W given in fragment
// order (Bf: the layer's fragments, tile-major, K / 16 steps per tile)
template <int NT, int K>
__device__ __forceinline__ void layer_product(const bf16 *h, const bf16 *Bf, int l, f32x16 acc[NT]) {
  constexpr int KS = K / 16;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x16{};
  const bf16 *b = Bf + 8 * l;
  for (int s = 0; s < KS; ++s) {
    const bf16x8 a = lds_frag(h, l, 16 * s);
    bf16x8 bt[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bt[t] = frag(b + (t * KS + s) * 8 * kWave);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma(a, bt[t], acc[t]);
  }
}

__device__ __forceinline__ uint32_t bf16_bits(float v) { return __builtin_bit_cast(unsigned short, (bf16)v); }

// h[rows][col] = bfloat16(relu(acc + bias[col])), written as bfloat16 pairs.
// Tiles go two at a time: lanes l and l ^ 1 hold columns 2c and 2c + 1 of both
// tiles; the even lane writes the pair of the first tile and the odd lane the
// pair of the second, after swapping one value, so each 32-bit store of 32
// lanes covers 32 consecutive words of one row (no bank conflict).
template <int NT>
__device__ __forceinline__ void store_hidden(bf16 *h, const float *bias, int l, const f32x16 acc[NT]) {
  static_assert(NT % 2 == 0, "tiles in pairs");
  const bool odd = l & 1;
  const int c = l & 31;
#pragma unroll
  for (int t = 0; t < NT; t += 2) {
    const float b0 = bias[t * 32 + c], b1 = bias[(t + 1) * 32 + c];
    const int col = (odd ? (t + 1) * 32 : t * 32) + (c & ~1);   // first column of the pair this lane writes
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v0 = acc[t][r] + b0, v1 = acc[t + 1][r] + b1;
      const uint32_t a = bf16_bits(v0 > 0.f ? v0 : 0.f), bb = bf16_bits(v1 > 0.f ? v1 : 0.f);
      // the even lane sends its second-tile value, the odd lane its first-tile
      // value; quad_perm [1, 0, 3, 2] gives each lane the value of lane l ^ 1
      const uint32_t nb = (uint32_t)__builtin_amdgcn_mov_dpp((int)(odd ? a : bb), 0xB1, 0xF, 0xF, false);
      const uint32_t pair = odd ? (nb | (bb << 16)) : (a | (nb << 16));
      *reinterpret_cast<uint32_t *>(h + acc_row(r, l) * kHStride + col) = pair;
    }
  }
}

struct ProposeLaunch {
  PopRows R;
  MlpWeights W;
  const float *genotypes;
  float *proposals;
  float alpha_max;
  uint64_t seed;
  int32_t generation;
};

// A workgroup of kPropWaves wavefronts, 32 rows each, walks the layers in step
// (the barriers between phases), so the wavefronts of a workgroup load the same
// weight fragments at about the same time and all but the first find them in L1.
__global__ __launch_bounds__(64 * kPropWaves) void propose_kernel(ProposeLaunch P) {
  __shared__ __attribute__((aligned(16))) bf16 h_all[kPropRows * kHStride];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  bf16 *h = h_all + w * 32 * kHStride;             // this wavefront's 32 rows
  const int64_t row0 = (int64_t)blockIdx.x * kPropRows + 32 * w;
  const int64_t r = row0 + (l & 31);
  const bool mine = l < 32;  // lanes 0..31 encode and decode one row each
  if (mine) {
    float f[kMlpIn];
    if (r < P.R.n_rows) {
      encode_row(P.R, r, P.genotypes, f);
    } else {
      for (int j = 0; j < kMlpIn; ++j) f[j] = 0.f;
    }
    // the row as twelve 16-byte stores
#pragma unroll
    for (int j = 0; j < kMlpIn; j += 8) {
      bf16x8 v;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (bf16)f[j + i];
      *reinterpret_cast<bf16x8 *>(h + l * kHStride + j) = v;
    }
  }
  __syncthreads();
  f32x16 acc[kMlpHidden / 32];
  layer_product<kMlpHidden / 32, kMlpIn>(h, P.W.wf + kFragW1, l, acc);
  __syncthreads();
  store_hidden<kMlpHidden / 32>(h, P.W.master + kOffB1, l, acc);
  __syncthreads();
  layer_product<kMlpHidden / 32, kMlpHidden>(h, P.W.wf + kFragW2, l, acc);
  __syncthreads();
  store_hidden<kMlpHidden / 32>(h, P.W.master + kOffB2, l, acc);
  __syncthreads();
  f32x16 out[1];
  layer_product<1, kMlpHidden>(h, P.W.wf + kFragW3, l, out);
  __syncthreads();
  // network outputs as float32 rows in the wavefront's LDS rows, padded to 33
  // floats so that the lanes reading their own rows hit different banks
  constexpr int kYStride = kMlpOut + 1;
  float *y = reinterpret_cast<float *>(h);
  {
    const int col = l & 31;
    const float b = P.W.master[kOffB3 + col];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[acc_row(i, l) * kYStride + col] = out[0][i] + b;
  }
  __syncthreads();
  if (mine && r < P.R.n_rows)
    decode_row(P.R, r, P.genotypes, y + l * kYStride, P.alpha_max, P.seed, P.generation, P.proposals);
}

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int EPI>
static hipError_t gemm_rk(const GemmRK &g, hipStream_t s) {
  GemmRK a = g;
  a.waves_n = a.N >= 128 ? 4 : a.N >= 64 ? 2 : 1;
  const int wm = 4 / a.waves_n;
  const int64_t tiles_m = a.mp / kMlpRowTile;
  dim3 grid(blocks_for(tiles_m, wm), (unsigned)((a.N / 32 + a.waves_n - 1) / a.waves_n));
  hipLaunchKernelGGL(gemm_rk_kernel<EPI>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

static hipError_t wgrad(const bf16 *Xp8, const bf16 *Zp8, int64_t mp, int K, int N, float *partial, float *out,
                        hipStream_t s) {
  const int chunks = (int)((mp + kWgradChunk - 1) / kWgradChunk);
  GemmWG g{Xp8, Zp8, mp, K, N, partial};
  const int tiles = (K / 32) * (N / 32);
  hipLaunchKernelGGL(gemm_wgrad_kernel, dim3(blocks_for(tiles, 4), chunks), dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partial_kernel, dim3(blocks_for(K * N, 256)), dim3(256), 0, s, (const float *)partial,
                     chunks, K * N, out);
  return hipGetLastError();
}

// out[c] = column sums of Z, by chunks of kColsumChunk rows summed in chunk
// order (partial needs ceil(mp / kColsumChunk) * N floats, which the weight
// gradients' ceil(mp / kWgradChunk) * 256 * 256 always cover)
static hipError_t colsum(const bf16 *Z, int64_t mp, int N, float *partial, float *out, hipStream_t s) {
  static_assert(kWgradChunk / kColsumChunk * kMlpHidden <= kMlpHidden * kMlpHidden, "partial buffer size");
  const int chunks = (int)((mp + kColsumChunk - 1) / kColsumChunk);
  hipLaunchKernelGGL(colsum_partial_kernel, dim3(blocks_for(N, 64), chunks), dim3(64), 0, s, Z, mp, N, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partial_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, (const float *)partial,
                     chunks, N, out);
  return hipGetLastError();
}

hipError_t launch_mlp_input(const float *x, int64_t m, const MlpActs &A, hipStream_t s) {
  hipLaunchKernelGGL(mlp_input_kernel, dim3(blocks_for(A.mp * kMlpIn, 256)), dim3(256), 0, s, x, m, A.mp, A.a0,
                     A.a0p8);
  return hipGetLastError();
}

hipError_t launch_mlp_gather(const float *x, const float *t, const float *w, const int32_t *order, int64_t row0,
                             int64_t m, const MlpActs &A, float *tb, float *wb, hipStream_t s) {
  hipLaunchKernelGGL(mlp_gather_kernel, dim3(blocks_for(A.mp, 128)), dim3(128), 0, s, x, t, w, order, row0, m, A.mp,
                     A.a0, A.a0p8, tb, w ? wb : nullptr);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpWeights &W, const MlpActs &A, hipStream_t s) {
  GemmRK g{};
  g.mp = A.mp;
  g.A = A.a0, g.Bt = W.wt1, g.N = kMlpHidden, g.K = kMlpIn, g.bias = W.master + kOffB1;
  g.out = A.a1, g.out_p8 = A.a1p8;
  hipError_t e = gemm_rk<kEpiRelu>(g, s);
  if (e != hipSuccess) return e;
  g.A = A.a1, g.Bt = W.wt2, g.N = kMlpHidden, g.K = kMlpHidden, g.bias = W.master + kOffB2;
  g.out = A.a2, g.out_p8 = A.a2p8;
  if ((e = gemm_rk<kEpiRelu>(g, s)) != hipSuccess) return e;
  g.A = A.a2, g.Bt = W.wt3, g.N = kMlpOut, g.K = kMlpHidden, g.bias = W.master + kOffB3;
  g.out = nullptr, g.out_p8 = nullptr, g.out_f32 = A.y;
  return gemm_rk<kEpiOut>(g, s);
}

hipError_t launch_mlp_backward(const MlpWeights &W, const MlpActs &A, const MlpGrads &G, const float *target,
                               const float *weight, int64_t m, hipStream_t s) {
  const int64_t mp = A.mp;
  const int64_t n_el = mp * kMlpOut;
  const unsigned lb = blocks_for(n_el, 256);
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(lb), dim3(256), 0, s, (const float *)A.y, target, weight, m, mp,
                     (float)(2.0 / (double)m), G.g3, G.g3p8, G.loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, s, (const float *)G.loss_part, (int)lb,
                     (float)(1.0 / (double)m), G.loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // layer 3
  if ((e = wgrad(A.a2p8, G.g3p8, mp, kMlpHidden, kMlpOut, G.partial, G.grads + kOffW3, s)) != hipSuccess) return e;
  if ((e = colsum(G.g3, mp, kMlpOut, G.partial, G.grads + kOffB3, s)) != hipSuccess) return e;
  GemmRK g{};
  g.mp = mp;
  g.A = G.g3, g.Bt = W.wr3, g.N = kMlpHidden, g.K = kMlpOut, g.mask = A.a2, g.out = G.g2, g.out_p8 = G.g2p8;
  if ((e = gemm_rk<kEpiMask>(g, s)) != hipSuccess) return e;
  // layer 2
  if ((e = wgrad(A.a1p8, G.g2p8, mp, kMlpHidden, kMlpHidden, G.partial, G.grads + kOffW2, s)) != hipSuccess)
    return e;
  if ((e = colsum(G.g2, mp, kMlpHidden, G.partial, G.grads + kOffB2, s)) != hipSuccess) return e;
  g.A = G.g2, g.Bt = W.wr2, g.N = kMlpHidden, g.K = kMlpHidden, g.mask = A.a1, g.out = G.g1, g.out_p8 = G.g1p8;
  if ((e = gemm_rk<kEpiMask>(g, s)) != hipSuccess) return e;
  // layer 1
  if ((e = wgrad(A.a0p8, G.g1p8, mp, kMlpIn, kMlpHidden, G.partial, G.grads + kOffW1, s)) != hipSuccess) return e;
  return colsum(G.g1, mp, kMlpHidden, G.partial, G.grads + kOffB1, s);
}

hipError_t launch_mlp_adam(float *master, float *m, float *v, const float *grads, const AdamStep &a, bf16 *wt1,
                           bf16 *wt2, bf16 *wt3, bf16 *wr2, bf16 *wr3, bf16 *wf, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, master, m, v, grads, a,
                     wt1, wt2, wt3, wr2, wr3, wf);
  return hipGetLastError();
}

hipError_t launch_mlp_refresh(const float *master, bf16 *wt1, bf16 *wt2, bf16 *wt3, bf16 *wr2, bf16 *wr3, bf16 *wf,
                              hipStream_t s) {
  hipLaunchKernelGGL(mlp_refresh_kernel, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, master, wt1, wt2, wt3,
                     wr2, wr3, wf);
  return hipGetLastError();
}

hipError_t launch_encode(const PopRows &R, int64_t row0, int64_t n, const float *genotypes, float *x, bf16 *a0,
                         int64_t a0_rows, hipStream_t s) {
  const int64_t rows = a0 ? a0_rows : n;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(encode_kernel, dim3(blocks_for(rows, 128)), dim3(128), 0, s, R, row0, n, genotypes, x, a0,
                     a0_rows);
  return hipGetLastError();
}

// Training weight of individual t (of n_ligs * pop): (1 + beta) (1 - r / pop)^beta
// for its rank r among its ligand's energies (numbers before NaNs, equal
// values by index), in binary64 rounded to float32.
__global__ void rank_weights_kernel(int64_t n, int32_t pop, const float *energies, double beta, float *w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t base = t - t % pop;
  const int i = (int)(t - base);
  const float ei = energies[t];
  const bool ni = ei != ei;
  int r = 0;
  for (int j = 0; j < pop; ++j) {
    const float ej = energies[base + j];
    const bool nj = ej != ej;
    bool before;
    if (nj != ni) before = !nj;
    else if (!ni && ej != ei) before = ej < ei;
    else before = j < i;
    r += (j != i) & before;
  }
  w[t] = (float)((1.0 + beta) * pow(1.0 - (double)r / pop, beta));
}

hipError_t launch_rank_weights(int64_t n, int32_t pop, const float *energies, double beta, float *w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_weights_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, s, n, pop, energies, beta, w);
  return hipGetLastError();
}

hipError_t launch_moves(const PopRows &R, const float *from, const float *to, float *out, hipStream_t s) {
  if (R.n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(moves_kernel, dim3(blocks_for(R.n_rows, 128)), dim3(128), 0, s, R, from, to, out);
  return hipGetLastError();
}

hipError_t launch_propose(const PopRows &R, const MlpWeights &W, const float *genotypes, float alpha_max,
                          uint64_t seed, int32_t generation, float *proposals, hipStream_t s) {
  if (R.n_rows <= 0) return hipSuccess;
  ProposeLaunch P{R, W, genotypes, proposals, alpha_max, seed, generation};
  hipLaunchKernelGGL(propose_kernel, dim3(blocks_for(R.n_rows, kPropRows)), dim3(64 * kPropWaves), 0, s, P);
  return hipGetLastError();
}

}  // namespace dock
