// search.hip -- differential evolution (DE/rand/1/bin, greedy selection) on the
// GPU: the evolutionary search of Sec. V with the pose score as fitness.
//
// The floating-point steps that decide a genotype are done in binary64 with
// contraction switched off, so that every trial genotype is a reproducible
// function of (seed, population, generation, ligand, individual).
#include "dock_internal.h"
#include "philox.h"

namespace dock {

constexpr double kPi = 3.14159265358979323846;

__device__ void init_individual(const DEParams &p, int n_tor, int lig, int i, int g_stride, float *row) {
#pragma clang fp contract(off)
  DrawStream s(p.seed, (uint64_t)i, 0, (uint64_t)lig, kPurposeInit);
  for (int j = 0; j < g_stride; ++j) row[j] = 0.f;
  for (int d = 0; d < 3; ++d) {
    const double u = s.unit();
    const double w = p.hi[d] - p.lo[d];
    const double m = u * w;
    row[d] = (float)(p.lo[d] + m);
  }
  // a point uniform in the unit 4-ball (rejection from the cube [-1,1]^4)
  float q0 = 1.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
  for (int t = 0; t < 64; ++t) {
    const double v0 = 2.0 * s.unit() - 1.0, v1 = 2.0 * s.unit() - 1.0;
    const double v2 = 2.0 * s.unit() - 1.0, v3 = 2.0 * s.unit() - 1.0;
    double nn = v0 * v0;
    nn = nn + v1 * v1;
    nn = nn + v2 * v2;
    nn = nn + v3 * v3;
    if (nn > 0.0 && nn <= 1.0) {
      q0 = (float)v0; q1 = (float)v1; q2 = (float)v2; q3 = (float)v3;
      break;
    }
  }
  row[3] = q0; row[4] = q1; row[5] = q2; row[6] = q3;
  for (int k = 0; k < n_tor; ++k) {
    const double u = s.unit();
    const double m = u * (2.0 * kPi);
    row[7 + k] = (float)(m - kPi);
  }
}

__device__ __forceinline__ int pick_partner(DrawStream &s, int pop, int t0, int t1, int t2, int n_taken) {
  for (int tries = 0; tries < 64; ++tries) {
    const int r = s.index(pop);
    const bool clash = (r == t0) | (n_taken > 1 && r == t1) | (n_taken > 2 && r == t2);
    if (!clash) return r;
  }
  for (int r = (t0 + 1) % pop;; r = (r + 1) % pop) {
    const bool clash = (r == t0) | (n_taken > 1 && r == t1) | (n_taken > 2 && r == t2);
    if (!clash) return r;
  }
}

__device__ void trial_individual(const DEParams &p, int n_tor, int lig, int gen, int i, int g_stride,
                                 const float *__restrict__ pop, float *__restrict__ trial) {
#pragma clang fp contract(off)
  const int P = p.pop, n_genes = 7 + n_tor;
  DrawStream s(p.seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig, kPurposeSelect);
  const int r1 = pick_partner(s, P, i, 0, 0, 1);
  const int r2 = pick_partner(s, P, i, r1, 0, 2);
  const int r3 = pick_partner(s, P, i, r1, r2, 3);
  const int jrand = s.index(n_genes);
  const float *xi = pop + (size_t)i * g_stride, *x1 = pop + (size_t)r1 * g_stride;
  const float *x2 = pop + (size_t)r2 * g_stride, *x3 = pop + (size_t)r3 * g_stride;
  DrawStream c(p.seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig, kPurposeCross);
  for (int j = 0; j < g_stride; ++j) {
    float v = 0.f;
    if (j < n_genes) {
      const double u = c.unit();
      if (u < (double)p.CR || j == jrand) {
        const double diff = (double)x2[j] - (double)x3[j];
        const double step = (double)p.F * diff;
        v = (float)((double)x1[j] + step);
      } else {
        v = xi[j];
      }
      if (j < 3) {
        if ((double)v < p.lo[j]) v = (float)p.lo[j];
        if ((double)v > p.hi[j]) v = (float)p.hi[j];
      } else if (j >= 7) {
        double w = (double)v;
        if (w > kPi) w = w - 2.0 * kPi;
        else if (w <= -kPi) w = w + 2.0 * kPi;
        v = (float)w;
      }
    }
    trial[j] = v;
  }
}

__global__ void de_init_kernel(LigandsDev L, DEParams p, int g_stride, float *pop) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)L.n_ligs * p.pop) return;
  const int lig = (int)(t / p.pop), i = (int)(t % p.pop);
  init_individual(p, L.hdr[lig].n_tors, lig, i, g_stride, pop + t * g_stride);
}

__global__ void de_trials_kernel(LigandsDev L, DEParams p, int gen, int g_stride, const float *pop, float *trials) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)L.n_ligs * p.pop) return;
  const int lig = (int)(t / p.pop), i = (int)(t % p.pop);
  const float *base = pop + (int64_t)lig * p.pop * g_stride;
  trial_individual(p, L.hdr[lig].n_tors, lig, gen, i, g_stride, base, trials + t * g_stride);
}

// One block per ligand: greedy replacement, then the target check.
__global__ void de_select_kernel(int pop, int g_stride, float *population, float *pop_energy,
                                 const float *trials, const float *trial_energy, const float *target,
                                 int32_t *gen_reached, int gen_done) {
  const int lig = blockIdx.x;
  float *P = population + (int64_t)lig * pop * g_stride;
  float *E = pop_energy + (int64_t)lig * pop;
  const float *T = trials + (int64_t)lig * pop * g_stride;
  const float *ET = trial_energy + (int64_t)lig * pop;
  int hit = 0;
  const float tg = (target && gen_reached) ? target[lig] : 0.f;
  for (int i = threadIdx.x; i < pop; i += blockDim.x) {
    const float et = ET[i];
    float e = E[i];
    if (et <= e) {
      for (int j = 0; j < g_stride; ++j) P[(int64_t)i * g_stride + j] = T[(int64_t)i * g_stride + j];
      E[i] = et;
      e = et;
    }
    if (target && gen_reached) hit |= (e <= tg);
  }
  if (target && gen_reached) {
    hit = __syncthreads_or(hit);
    if (threadIdx.x == 0 && hit && gen_reached[lig] < 0) gen_reached[lig] = gen_done;
  }
}

__global__ void de_check_kernel(int pop, const float *pop_energy, const float *target, int32_t *gen_reached,
                                int gen_done, int reset) {
  const int lig = blockIdx.x;
  const float *E = pop_energy + (int64_t)lig * pop;
  int hit = 0;
  for (int i = threadIdx.x; i < pop; i += blockDim.x) hit |= (E[i] <= target[lig]);
  hit = __syncthreads_or(hit);
  if (threadIdx.x == 0) {
    int32_t r = reset ? -1 : gen_reached[lig];
    if (r < 0 && hit) r = gen_done;
    gen_reached[lig] = r;
  }
}

// Best member of the final population: first index of the smallest energy.
__global__ void de_best_kernel(int pop, int g_stride, const float *population, const float *pop_energy,
                               float *best_g, float *best_e) {
  const int lig = blockIdx.x;
  const float *E = pop_energy + (int64_t)lig * pop;
  __shared__ int s_bi;
  if (threadIdx.x == 0) {
    int bi = 0;
    for (int i = 1; i < pop; ++i)
      if (E[i] < E[bi]) bi = i;
    s_bi = bi;
    best_e[lig] = E[bi];
  }
  __syncthreads();
  const float *row = population + ((int64_t)lig * pop + s_bi) * g_stride;
  for (int j = threadIdx.x; j < g_stride; j += blockDim.x) best_g[(int64_t)lig * g_stride + j] = row[j];
}

static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_de_init(const LigandsDev &L, const DEParams &p, int32_t g_stride, float *pop, hipStream_t s) {
  const int64_t n = (int64_t)L.n_ligs * p.pop;
  hipLaunchKernelGGL(de_init_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, s, L, p, g_stride, pop);
  return hipGetLastError();
}

hipError_t launch_de_trials(const LigandsDev &L, const DEParams &p, int32_t gen, int32_t g_stride,
                            const float *pop, float *trials, hipStream_t s) {
  const int64_t n = (int64_t)L.n_ligs * p.pop;
  hipLaunchKernelGGL(de_trials_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, s, L, p, gen, g_stride, pop, trials);
  return hipGetLastError();
}

hipError_t launch_de_select(int32_t n_ligs, int32_t pop, int32_t g_stride, float *population, float *pop_energy,
                            const float *trials, const float *trial_energy, const float *target,
                            int32_t *gen_reached, int32_t gen_done, hipStream_t s) {
  hipLaunchKernelGGL(de_select_kernel, dim3(n_ligs), dim3(256), 0, s, pop, g_stride, population, pop_energy,
                     trials, trial_energy, target, gen_reached, gen_done);
  return hipGetLastError();
}

hipError_t launch_de_check(int32_t n_ligs, int32_t pop, const float *pop_energy, const float *target,
                           int32_t *gen_reached, int32_t gen_done, int32_t reset, hipStream_t s) {
  hipLaunchKernelGGL(de_check_kernel, dim3(n_ligs), dim3(256), 0, s, pop, pop_energy, target, gen_reached,
                     gen_done, reset);
  return hipGetLastError();
}

hipError_t launch_de_best(int32_t n_ligs, int32_t pop, int32_t g_stride, const float *population,
                          const float *pop_energy, float *best_g, float *best_e, hipStream_t s) {
  hipLaunchKernelGGL(de_best_kernel, dim3(n_ligs), dim3(64), 0, s, pop, g_stride, population, pop_energy, best_g,
                     best_e);
  return hipGetLastError();
}

}  // namespace dock
