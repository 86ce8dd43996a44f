// api_learn.hip -- host side of the learned-proposal entry points of the C ABI:
// the network handle (parameters, Adam state, bfloat16 weight copies, training
// workspace), inference in row chunks, training steps, and proposals for a
// population.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "api_internal.h"
#include "learn.h"

using namespace dock;

static_assert(DOCK_MLP_PARAMS == kMlpParams, "packed parameter count");
static_assert(DOCK_MLP_IN == kMlpIn && DOCK_MLP_HIDDEN == kMlpHidden && DOCK_MLP_OUT == kMlpOut, "shape");
static_assert(DOCK_DESC == kDesc, "descriptor size");

constexpr int64_t kInferChunk = 65536;  // rows per inference pass (bounds its workspace)

static int64_t pad_rows(int64_t n) { return (n + kMlpRowTile - 1) / kMlpRowTile * kMlpRowTile; }

// Carves 256-byte aligned pieces out of one allocation.
struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    T *p = base ? (T *)(base + off) : nullptr;
    off += (sizeof(T) * count + 255) / 256 * 256;
    return p;
  }
};

// Activation buffers for up to mp rows (p8 copies when training).
static void carve_acts(Carver &c, int64_t mp, bool train, MlpActs &A) {
  A.mp = mp;
  A.a0 = c.take<bf16>(mp * kMlpIn);
  A.a1 = c.take<bf16>(mp * kMlpHidden);
  A.a2 = c.take<bf16>(mp * kMlpHidden);
  A.y = c.take<float>(mp * kMlpOut);
  A.a0p8 = train ? c.take<bf16>(mp * kMlpIn) : nullptr;
  A.a1p8 = train ? c.take<bf16>(mp * kMlpHidden) : nullptr;
  A.a2p8 = train ? c.take<bf16>(mp * kMlpHidden) : nullptr;
}

static void carve_grads(Carver &c, int64_t mp, MlpGrads &G) {
  G.g3 = c.take<bf16>(mp * kMlpOut);
  G.g3p8 = c.take<bf16>(mp * kMlpOut);
  G.g2 = c.take<bf16>(mp * kMlpHidden);
  G.g2p8 = c.take<bf16>(mp * kMlpHidden);
  G.g1 = c.take<bf16>(mp * kMlpHidden);
  G.g1p8 = c.take<bf16>(mp * kMlpHidden);
  G.partial = c.take<float>((size_t)((mp + kWgradChunk - 1) / kWgradChunk) * kMlpHidden * kMlpHidden);
  G.loss_part = c.take<float>((size_t)((mp * kMlpOut + 255) / 256));
  G.grads = c.take<float>(kMlpParams);
  G.loss = c.take<float>(1);
}

struct dock_mlp {
  int device = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr;  // [kMlpParams] each
  bf16 *wt1 = nullptr, *wt2 = nullptr, *wt3 = nullptr, *wr2 = nullptr, *wr3 = nullptr;
  bf16 *wf = nullptr;  // forward weights in fragment order (the fused proposal kernel)
  int64_t adam_t = 0;
  // training workspace for up to ws_rows rows
  char *ws = nullptr;
  int64_t ws_rows = 0;
  MlpActs A{};
  MlpGrads G{};
  float *tb = nullptr, *wb = nullptr;  // gathered targets [rows][32] and weights [rows]
  MlpWeights weights() const { return MlpWeights{master, wt1, wt2, wt3, wr2, wr3, wf}; }
  hipError_t ensure_workspace(int64_t mp) {
    if (mp <= ws_rows) return hipSuccess;
    if (ws) {
      hipError_t e = hipDeviceSynchronize();  // the old workspace may still be in use
      if (e != hipSuccess) return e;
      (void)hipFree(ws);
      ws = nullptr;
      ws_rows = 0;
    }
    Carver sizer{nullptr};
    MlpActs a;
    MlpGrads g;
    carve_acts(sizer, mp, true, a);
    carve_grads(sizer, mp, g);
    sizer.take<float>(mp * kMlpOut);
    sizer.take<float>(mp);
    hipError_t e = hipMalloc((void **)&ws, sizer.off);
    if (e != hipSuccess) return e;
    Carver c{ws};
    carve_acts(c, mp, true, A);
    carve_grads(c, mp, G);
    tb = c.take<float>(mp * kMlpOut);
    wb = c.take<float>(mp);
    ws_rows = mp;
    return hipSuccess;
  }
};

static void free_mlp(dock_mlp *n) {
  for (void *p : {(void *)n->master, (void *)n->m, (void *)n->v, (void *)n->wt1, (void *)n->wt2, (void *)n->wt3,
                  (void *)n->wr2, (void *)n->wr3, (void *)n->wf, (void *)n->ws})
    if (p) (void)hipFree(p);
  delete n;
}

// splitmix64 (Steele, Lea, Flood, OOPSLA 2014): the initial weights' generator
static uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static std::vector<float> initial_params(uint64_t seed) {
  std::vector<float> p(kMlpParams, 0.f);
  uint64_t s = seed;
  auto fill = [&](int off, int fan_in, int count, double scale) {
    const double bound = scale * sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
      p[off + i] = (float)((2.0 * u - 1.0) * bound);
    }
  };
  fill(kOffW1, kMlpIn, kMlpIn * kMlpHidden, 1.0);
  fill(kOffW2, kMlpHidden, kMlpHidden * kMlpHidden, 1.0);
  fill(kOffW3, kMlpHidden, kMlpHidden * kMlpOut, 0.1);
  return p;
}

static hipError_t load_params(dock_mlp *n, const float *host) {
  hipError_t e = hipMemcpy(n->master, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->m, 0, sizeof(float) * kMlpParams);
  if (e == hipSuccess) e = hipMemset(n->v, 0, sizeof(float) * kMlpParams);
  if (e == hipSuccess) e = launch_mlp_refresh(n->master, n->wt1, n->wt2, n->wt3, n->wr2, n->wr3, n->wf, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  n->adam_t = 0;
  return e;
}

extern "C" dock_status dock_mlp_create(int32_t device, uint64_t seed, dock_mlp **out) {
  if (!out) return set_err(DOCK_E_INVALID, "null out");
  *out = nullptr;
  DeviceScope ds(device);
  HIP_TRY(ds.err, "hipSetDevice");
  dock_mlp *n = new dock_mlp();
  n->device = device;
  hipError_t e = hipSuccess;
  for (float **p : {&n->master, &n->m, &n->v})
    if (e == hipSuccess) e = hipMalloc((void **)p, sizeof(float) * kMlpParams);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wt1, sizeof(bf16) * kMlpIn * kMlpHidden);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wt2, sizeof(bf16) * kMlpHidden * kMlpHidden);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wt3, sizeof(bf16) * kMlpHidden * kMlpOut);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wr2, sizeof(bf16) * kMlpHidden * kMlpHidden);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wr3, sizeof(bf16) * kMlpHidden * kMlpOut);
  if (e == hipSuccess) e = hipMalloc((void **)&n->wf, sizeof(bf16) * kFragTotal);
  if (e == hipSuccess) e = load_params(n, initial_params(seed).data());
  if (e != hipSuccess) {
    free_mlp(n);
    return hip_err(e, "network allocation");
  }
  *out = n;
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_destroy(dock_mlp *n) {
  if (!n) return DOCK_OK;
  DeviceScope ds(n->device);
  free_mlp(n);
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_set_params(dock_mlp *n, const float *params) {
  if (!n || !params) return set_err(DOCK_E_INVALID, "null argument");
  for (int i = 0; i < kMlpParams; ++i)
    if (!isfinite(params[i])) return set_err(DOCK_E_INVALID, "non-finite parameter %d", i);
  DeviceScope ds(n->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(load_params(n, params), "parameter upload");
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_get_params(const dock_mlp *n, float *params) {
  if (!n || !params) return set_err(DOCK_E_INVALID, "null argument");
  DeviceScope ds(n->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(hipDeviceSynchronize(), "synchronize");
  HIP_TRY(hipMemcpy(params, n->master, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "parameter download");
  return DOCK_OK;
}

// Inference over n rows in chunks: fill(row0, count, acts) writes the chunk's
// bfloat16 inputs into acts.a0 (rows count .. mp-1 zero); done(row0, count, y)
// consumes the chunk's outputs.
template <class Fill, class Done>
static hipError_t infer_rows(const dock_mlp *net, int64_t n, hipStream_t s, Fill fill, Done done) {
  if (n <= 0) return hipSuccess;
  const int64_t chunk = std::min(pad_rows(n), kInferChunk);
  Carver sizer{nullptr};
  MlpActs a;
  carve_acts(sizer, chunk, false, a);
  char *buf = nullptr;
  hipError_t e = scratch_alloc((void **)&buf, sizer.off, s);
  if (e != hipSuccess) return e;
  Carver c{buf};
  MlpActs A;
  carve_acts(c, chunk, false, A);
  for (int64_t r0 = 0; r0 < n && e == hipSuccess; r0 += chunk) {
    const int64_t cnt = std::min(chunk, n - r0);
    A.mp = pad_rows(cnt);
    e = fill(r0, cnt, A);
    if (e == hipSuccess) e = launch_mlp_forward(net->weights(), A, s);
    if (e == hipSuccess) e = done(r0, cnt, (const float *)A.y);
  }
  hipError_t f = hipFreeAsync(buf, s);
  return e != hipSuccess ? e : f;
}

extern "C" dock_status dock_mlp_forward(const dock_mlp *n, const float *x, int64_t rows, float *y, void *stream) {
  if (!n) return set_err(DOCK_E_INVALID, "null network");
  if (rows < 0) return set_err(DOCK_E_INVALID, "n must be >= 0");
  if (rows == 0) return DOCK_OK;
  if (!x || !y) return set_err(DOCK_E_INVALID, "null x or y");
  DeviceScope ds(n->device);
  HIP_TRY(ds.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = infer_rows(
      n, rows, s, [&](int64_t r0, int64_t cnt, const MlpActs &A) { return launch_mlp_input(x + r0 * kMlpIn, cnt, A, s); },
      [&](int64_t r0, int64_t cnt, const float *yy) {
        return hipMemcpyAsync(y + r0 * kMlpOut, yy, sizeof(float) * cnt * kMlpOut, hipMemcpyDeviceToDevice, s);
      });
  HIP_TRY(e, "network forward");
  return DOCK_OK;
}

// Forward + backward of one batch of m rows (source rows order[row0 ..] or
// row0 ..) into the network's workspace.
static hipError_t batch_gradients(dock_mlp *n, const float *x, const float *target, const float *weight,
                                  const int32_t *order, int64_t row0, int64_t m, hipStream_t s) {
  const int64_t mp = pad_rows(m);
  hipError_t e = n->ensure_workspace(mp);
  if (e != hipSuccess) return e;
  MlpActs A = n->A;
  A.mp = mp;
  e = launch_mlp_gather(x, target, weight, order, row0, m, A, n->tb, n->wb, s);
  if (e == hipSuccess) e = launch_mlp_forward(n->weights(), A, s);
  if (e == hipSuccess) e = launch_mlp_backward(n->weights(), A, n->G, n->tb, weight ? n->wb : nullptr, m, s);
  return e;
}

extern "C" dock_status dock_mlp_gradients(dock_mlp *n, const float *x, const float *target, const float *weight,
                                          int32_t rows, float *grads, float *loss, void *stream) {
  if (!n || !x || !target || !grads || !loss) return set_err(DOCK_E_INVALID, "null argument");
  if (rows < 1 || rows > DOCK_MLP_MAX_BATCH) return set_err(DOCK_E_INVALID, "n must be in 1..%d", DOCK_MLP_MAX_BATCH);
  DeviceScope ds(n->device);
  HIP_TRY(ds.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(batch_gradients(n, x, target, weight, nullptr, 0, rows, s), "network gradients");
  HIP_TRY(hipMemcpyAsync(grads, n->G.grads, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, s), "copy gradients");
  HIP_TRY(hipMemcpyAsync(loss, n->G.loss, sizeof(float), hipMemcpyDeviceToDevice, s), "copy loss");
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_train(dock_mlp *n, const float *x, const float *target, const float *weight,
                                      int64_t n_data, const int32_t *order, int64_t n_rows, int32_t batch,
                                      int32_t n_steps, float lr, float *losses, void *stream) {
  if (!n || !x || !target) return set_err(DOCK_E_INVALID, "null argument");
  if (batch < 1 || batch > DOCK_MLP_MAX_BATCH) return set_err(DOCK_E_INVALID, "batch must be in 1..%d", DOCK_MLP_MAX_BATCH);
  if (n_rows < batch || n_rows % batch != 0) return set_err(DOCK_E_INVALID, "n_rows must be a positive multiple of batch");
  if (n_data < 1 || n_data > 0x7fffffff) return set_err(DOCK_E_INVALID, "n_data must be in 1..2^31-1");
  if (!order && n_rows > n_data) return set_err(DOCK_E_INVALID, "n_rows > n_data without an order");
  if (n_steps < 0) return set_err(DOCK_E_INVALID, "n_steps must be >= 0");
  if (!(lr > 0) || !isfinite(lr)) return set_err(DOCK_E_INVALID, "lr must be positive and finite");
  DeviceScope ds(n->device);
  HIP_TRY(ds.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  if (order) {
    // every row index is checked before any kernel reads through it
    std::vector<int32_t> h(n_rows);
    HIP_TRY(hipMemcpyAsync(h.data(), order, sizeof(int32_t) * n_rows, hipMemcpyDeviceToHost, s), "copy order");
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    for (int64_t i = 0; i < n_rows; ++i)
      if (h[i] < 0 || h[i] >= n_data) return set_err(DOCK_E_INVALID, "order[%lld] = %d outside 0..n_data-1", (long long)i, h[i]);
  }
  for (int32_t st = 0; st < n_steps; ++st) {
    const int64_t off = ((int64_t)st * batch) % n_rows;
    HIP_TRY(batch_gradients(n, x, target, weight, order, off, batch, s), "network gradients");
    if (losses) HIP_TRY(hipMemcpyAsync(losses + st, n->G.loss, sizeof(float), hipMemcpyDeviceToDevice, s), "copy loss");
    n->adam_t += 1;
    AdamStep a{lr, 0.9f, 0.999f, 1e-8f, (float)(1.0 - pow(0.9, (double)n->adam_t)),
               (float)(1.0 - pow(0.999, (double)n->adam_t))};
    HIP_TRY(launch_mlp_adam(n->master, n->m, n->v, n->G.grads, a, n->wt1, n->wt2, n->wt3, n->wr2, n->wr3, n->wf, s), "adam");
  }
  return DOCK_OK;
}

extern "C" dock_status dock_ligand_descriptors(const dock_ligands *L, float *out, void *stream) {
  if (!L || !out) return set_err(DOCK_E_INVALID, "null argument");
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(out, L->desc, sizeof(float) * kDesc * L->n_ligs, hipMemcpyDeviceToDevice, (hipStream_t)stream),
          "copy descriptors");
  return DOCK_OK;
}

static dock_status pop_rows(const dock_ligands *L, const dock_search_params *q, int32_t g_stride, PopRows &R) {
  if (!q) return set_err(DOCK_E_INVALID, "null params");
  if (q->pop_size < 1) return set_err(DOCK_E_INVALID, "pop_size must be >= 1");
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride too small");
  for (int d = 0; d < 3; ++d)
    if (!(q->box_lo[d] <= q->box_hi[d]) || !isfinite(q->box_lo[d]) || !isfinite(q->box_hi[d]))
      return set_err(DOCK_E_INVALID, "empty or non-finite translation box");
  R = make_pop_rows(L, q->pop_size, g_stride, q->box_lo, q->box_hi);
  return DOCK_OK;
}

PopRows make_pop_rows(const dock_ligands *L, int32_t pop, int32_t g_stride, const double lo[3], const double hi[3]) {
  PopRows R{};
  R.hdr = L->hdr;
  R.desc = L->desc;
  R.pop = pop;
  R.g_stride = g_stride;
  R.n_rows = (int64_t)L->n_ligs * pop;
  for (int d = 0; d < 3; ++d) R.lo[d] = (float)lo[d], R.hi[d] = (float)hi[d];
  return R;
}

extern "C" dock_status dock_mlp_features(const dock_ligands *L, const dock_search_params *q, int32_t g_stride,
                                         const float *population, float *x, void *stream) {
  if (!L || !population || !x) return set_err(DOCK_E_INVALID, "null argument");
  PopRows R;
  dock_status st = pop_rows(L, q, g_stride, R);
  if (st) return st;
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_encode(R, 0, R.n_rows, population, x, nullptr, 0, (hipStream_t)stream), "encode launch");
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_moves(const dock_ligands *L, const dock_search_params *q, int32_t g_stride,
                                      const float *from, const float *to, float *out, void *stream) {
  if (!L || !from || !to || !out) return set_err(DOCK_E_INVALID, "null argument");
  PopRows R;
  dock_status st = pop_rows(L, q, g_stride, R);
  if (st) return st;
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_moves(R, from, to, out, (hipStream_t)stream), "moves launch");
  return DOCK_OK;
}

extern "C" dock_status dock_mlp_rank_weights(const dock_ligands *L, const dock_search_params *q, const float *pop_energy,
                                            float beta, float *weight, void *stream) {
  if (!L || !q || !pop_energy || !weight) return set_err(DOCK_E_INVALID, "null argument");
  if (q->pop_size < 1) return set_err(DOCK_E_INVALID, "pop_size must be >= 1");
  if (!isfinite(beta) || !(beta > -1.f)) return set_err(DOCK_E_INVALID, "beta must be finite and > -1");
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_rank_weights((int64_t)L->n_ligs * q->pop_size, q->pop_size, pop_energy, (double)beta, weight,
                              (hipStream_t)stream),
          "rank weights launch");
  return DOCK_OK;
}

hipError_t run_proposals(const dock_mlp *net, const PopRows &R, float alpha_max, uint64_t seed, int32_t generation,
                         const float *population, float *proposals, hipStream_t s) {
  return launch_propose(R, net->weights(), population, alpha_max, seed, generation, proposals, s);
}

int mlp_device(const dock_mlp *net) { return net->device; }

extern "C" dock_status dock_propose(const dock_ligands *L, const dock_mlp *net, const dock_search_params *q,
                                    int32_t generation, float alpha_max, int32_t g_stride, const float *population,
                                    float *proposals, void *stream) {
  if (!L || !net || !population || !proposals) return set_err(DOCK_E_INVALID, "null argument");
  if (net->device != L->device) return set_err(DOCK_E_INVALID, "network and ligands on different devices");
  if (generation < 0) return set_err(DOCK_E_INVALID, "generation must be >= 0");
  if (!(alpha_max > 0) || !isfinite(alpha_max)) return set_err(DOCK_E_INVALID, "alpha_max must be positive and finite");
  PopRows R;
  dock_status st = pop_rows(L, q, g_stride, R);
  if (st) return st;
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(run_proposals(net, R, alpha_max, q->seed, generation, population, proposals, (hipStream_t)stream),
          "proposals");
  return DOCK_OK;
}
