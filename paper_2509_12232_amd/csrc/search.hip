// search.hip -- differential evolution (DE/rand/1/bin, greedy selection) on the
// GPU: the evolutionary search of Sec. V with the pose score as fitness.
//
// The floating-point steps that decide a genotype are done in binary64 with
// contraction switched off, so that every trial genotype is a reproducible
// function of (seed, population, generation, ligand, individual).
//
// dock_search runs one persistent kernel per ligand-size bucket: each workgroup
// takes the next ligand from a work queue (largest first) and runs its whole
// search -- initial population, then per generation all trials, their scores
// and the greedy selection -- with no other launch or host round trip.  Steps
// without a pose use one lane per individual; scoring gives each individual a
// lane in a block of 64 that 1, 2, 4 or 8 wavefronts build and score together
// (the same bits for every split).
#include <algorithm>

#include "search.h"
#include "philox.h"
#include "score_pose.h"

namespace dock {

constexpr double kPi = 3.14159265358979323846;

// Individual i of the initial population; gene j goes to row[j * gs].
__device__ void init_individual(const DEParams &p, int n_tor, int lig, int i, int g_stride, float *row, int gs) {
#pragma clang fp contract(off)
  DrawStream s(p.seed, (uint64_t)i, 0, (uint64_t)lig, kPurposeInit);
  for (int j = 0; j < g_stride; ++j) row[j * gs] = 0.f;
  for (int d = 0; d < 3; ++d) {
    const double u = s.unit();
    const double w = p.hi[d] - p.lo[d];
    const double m = u * w;
    row[d * gs] = (float)(p.lo[d] + m);
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
  row[3 * gs] = q0; row[4 * gs] = q1; row[5 * gs] = q2; row[6 * gs] = q3;
  for (int k = 0; k < n_tor; ++k) {
    const double u = s.unit();
    const double m = u * (2.0 * kPi);
    row[(7 + k) * gs] = (float)(m - kPi);
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

// Trial i of generation gen.  Gene j of population row r is pop[r * rs + j * gs];
// gene j of the trial goes to trial[j * tgs].  The crossover draws (one per gene
// of the ligand, in gene order) are taken first; the genes are then done in
// blocks of eight whose loads are all issued before their arithmetic, so a
// trial waits for memory once per block rather than once per gene.
static_assert(7 + kMaxTorsions <= 64, "crossover decisions fit one 64-bit mask");
constexpr int kGeneBlock = 8;

__device__ void trial_individual(const DEParams &p, int n_tor, int lig, int gen, int i, int g_stride,
                                 const float *__restrict__ pop, int rs, int gs, float *__restrict__ trial, int tgs) {
#pragma clang fp contract(off)
  const int P = p.pop, n_genes = 7 + n_tor;
  DrawStream s(p.seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig, kPurposeSelect);
  const int r1 = pick_partner(s, P, i, 0, 0, 1);
  const int r2 = pick_partner(s, P, i, r1, 0, 2);
  const int r3 = pick_partner(s, P, i, r1, r2, 3);
  const int jrand = s.index(n_genes);
  const float *xi = pop + (size_t)i * rs, *x1 = pop + (size_t)r1 * rs;
  const float *x2 = pop + (size_t)r2 * rs, *x3 = pop + (size_t)r3 * rs;
  DrawStream c(p.seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig, kPurposeCross);
  uint64_t take = 0;   // bit j: gene j takes the mutant value
  for (int j = 0; j < n_genes; ++j) {
    const double u = c.unit();
    if (u < (double)p.CR || j == jrand) take |= 1ull << j;
  }
  for (int j0 = 0; j0 < g_stride; j0 += kGeneBlock) {
    float a1[kGeneBlock], a2[kGeneBlock], a3[kGeneBlock], ai[kGeneBlock];
#pragma unroll
    for (int k = 0; k < kGeneBlock; ++k) {
      const int j = min(j0 + k, g_stride - 1);   // past the row: a valid gene, not used
      a1[k] = x1[j * gs]; a2[k] = x2[j * gs]; a3[k] = x3[j * gs]; ai[k] = xi[j * gs];
    }
#pragma unroll
    for (int k = 0; k < kGeneBlock; ++k) {
      const int j = j0 + k;
      if (j >= g_stride) break;
      float v = 0.f;
      if (j < n_genes) {
        if ((take >> j) & 1) {
          const double diff = (double)a2[k] - (double)a3[k];
          const double step = (double)p.F * diff;
          v = (float)((double)a1[k] + step);
        } else {
          v = ai[k];
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
      trial[j * tgs] = v;
    }
  }
}

// Copies genes j = h, h + WS, ... (< G) of a gene-major individual from src to
// dst (element j at [j * P]), in blocks whose loads are issued before the stores.
template <int WS>
__device__ __forceinline__ void copy_genes(const float *__restrict__ src, float *__restrict__ dst, int h, int G,
                                           int P) {
  for (int j0 = h; j0 < G; j0 += kGeneBlock * WS) {
    float v[kGeneBlock];
#pragma unroll
    for (int k = 0; k < kGeneBlock; ++k) v[k] = src[min(j0 + k * WS, G - 1) * P];
#pragma unroll
    for (int k = 0; k < kGeneBlock; ++k)
      if (j0 + k * WS < G) dst[(j0 + k * WS) * P] = v[k];
  }
}


__global__ void de_init_kernel(LigandsDev L, DEParams p, int g_stride, float *pop) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)L.n_ligs * p.pop) return;
  const int lig = (int)(t / p.pop), i = (int)(t % p.pop);
  init_individual(p, L.hdr[lig].n_tors, lig, i, g_stride, pop + t * g_stride, 1);
}

__global__ void de_trials_kernel(LigandsDev L, DEParams p, int gen, int g_stride, const float *pop, float *trials) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)L.n_ligs * p.pop) return;
  const int lig = (int)(t / p.pop), i = (int)(t % p.pop);
  const float *base = pop + (int64_t)lig * p.pop * g_stride;
  trial_individual(p, L.hdr[lig].n_tors, lig, gen, i, g_stride, base, g_stride, 1, trials + t * g_stride, 1);
}

// The whole search of one ligand, run by one workgroup of B blocks of WS
// wavefronts.  The per-individual steps without a pose (initial genotypes, DE
// trials, copies) use lane t of the workgroup for individuals t, t + NT, ...;
// a scoring pass gives lane l of block b the individual c + 64 b + l, built and
// scored by the block's WS wavefronts together.  Every wavefront of the
// workgroup takes part in every pass (so all of them meet the same barriers);
// lanes without an individual score individual 0, in bounds, and drop the
// result.  With TAIL (splits 2, 4 and 8, chosen at launch when the population
// ends in a short pass), a generation's last pass, when what is left of the
// population fits in half of each block (32 individuals), scores half blocks
// instead: lanes l and l + 32 share an individual and each takes half of the
// pair and atom work, so the tail of the population costs about half a pass
// (the same energies, bit for bit).  With split 8, wavefronts 0-3 score the
// half block as a split of four, and wavefronts 4-7 only meet its barriers.
// It is a separate instance so that the registers of the half-block code cost
// nothing where no pass uses it.  The population is worked on in a gene-major
// copy W (gene j of individual i at W[j * P + i]), as are the trials, so that
// neighbouring lanes touch neighbouring words; the caller's individual-major
// population is read at the start and written back at the end.
template <int LAYOUT, int WS, bool TAIL>
__device__ void search_ligand(const SearchLaunch &S, int lig, float *my, float *red) {
  const int t = threadIdx.x, NT = blockDim.x;
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave), lane = t % kWave;
  const int h = wave % WS;                          // wavefront within its block
  const int PB = NT / WS;                           // individuals per scoring pass
  const int slot = (wave / WS) * kBlock + lane;     // this lane's individual in a pass
  const LigHeader H = as_const(S.L.hdr)[lig];
  const int P = S.p.pop, G = S.g_stride;
  float *pop = S.population + (int64_t)lig * P * G;
  float *E = S.pop_energy + (int64_t)lig * P;
  float *W = S.work + (int64_t)lig * P * G;
  float *T = S.trials + (int64_t)lig * P * G;
  const bool track = S.target != nullptr && S.gen_reached != nullptr;
  const float tgt = track ? S.target[lig] : 0.f;
  auto score = [&](const float *g, int gs) {
    return score_pose<LAYOUT, WS, 1>(S.L, S.geom, S.ff, S.maps, H, g, gs, my, red, h);
  };
  constexpr bool kHalf = TAIL && WS >= 2;
  constexpr int HWS = WS == 8 ? 4 : WS;   // wavefronts of a block that score a half block
  auto score_half = [&](const float *g, int gs) {
    if constexpr (kHalf) {
      if (WS == HWS || h < HWS) return score_pose<LAYOUT, HWS, 1, true>(S.L, S.geom, S.ff, S.maps, H, g, gs, my, red, h);
      // the barriers that score_pose holds for a split above one (n_tors + 3:
      // the reference coordinates, each torsion, the rigid move, the reduction)
      for (int b = 0; b < H.n_tors + 3; ++b) __syncthreads();
      return 0.f;
    } else {
      return score(g, gs);
    }
  };
  for (int c = 0; c < P; c += NT) {
    const int i = c + t;
    if (i >= P) continue;
    if (S.init) {
      init_individual(S.p, H.n_tors, lig, i, G, W + i, P);
    } else {
      const float *row = pop + (int64_t)i * G;
      for (int j = 0; j < G; ++j) W[j * P + i] = row[j];
    }
  }
  __syncthreads();
  if (S.init) {
    for (int c = 0; c < P; c += PB) {
      const int i = c + slot;
      const float e = score(W + (i < P ? i : 0), P);
      if (i < P && h == 0) E[i] = e;
    }
  }
  // a round of outside proposals (individual-major, one per individual): exact
  // score, greedy replacement -- skipped for a ligand that has already stopped
  // at its target
  if (S.proposals && !(S.stop && !S.init && S.gen_reached && S.gen_reached[lig] >= 0)) {
    const float *Q = S.proposals + (int64_t)lig * P * G;
    for (int c = 0; c < P; c += PB) {
      const int i = c + slot;
      const float *pr = Q + (int64_t)(i < P ? i : 0) * G;
      const float e = score(pr, 1);
      // every wavefront of the block takes the same decision (wavefront 0
      // stores E[i] = e only when e <= E[i], so a late read sees e itself)
      if (i < P && e <= E[i]) {
        for (int j = h; j < G; j += WS) W[j * P + i] = pr[j];
        if (h == 0) E[i] = e;
      }
    }
  }
  __syncthreads();
  int reached = -1;
  if (track) {
    int hit = 0;
    for (int c = 0; c < P; c += NT) {
      const int i = c + t;
      if (i < P) hit |= E[i] <= tgt;
    }
    hit = __syncthreads_or(hit);
    reached = S.init ? -1 : S.gen_reached[lig];
    if (reached < 0 && hit) reached = S.p.first_gen;
  }
  __syncthreads();
  // with S.stop, the search of a ligand ends once its best has reached the target
  const bool stop = track && S.stop;
  const int g_end = (stop && reached >= 0) ? S.p.first_gen : S.p.first_gen + S.p.n_gen;
  for (int gen = S.p.first_gen; gen < g_end; ++gen) {
    // every trial of the generation is drawn from the population as it stood
    for (int c = 0; c < P; c += NT) {
      const int i = c + t;
      if (i < P) trial_individual(S.p, H.n_tors, lig, gen, i, G, W, 1, P, T + i, P);
    }
    __syncthreads();
    int hit = 0;
    for (int c = 0; c < P; c += PB) {
      const bool half = kHalf && P - c <= PB / 2;   // the same for the whole workgroup
      const int i = c + (half ? (wave / WS) * (kBlock / 2) + (lane & (kBlock / 2 - 1)) : slot);
      const float *gi = T + (i < P ? i : 0);
      const float e = half ? score_half(gi, P) : score(gi, P);
      if (i < P && (!half || (lane < kBlock / 2 && h < HWS))) {
        float ei = E[i];
        if (e <= ei) {
          if (half) copy_genes<HWS>(T + i, W + i, h, G, P);
          else copy_genes<WS>(T + i, W + i, h, G, P);
          ei = e;
          if (h == 0) E[i] = e;
        }
        hit |= ei <= tgt;
      }
    }
    if (track) {
      hit = __syncthreads_or(hit);
      if (reached < 0 && hit) reached = gen + 1;
      if (stop && reached >= 0) break;
    } else {
      __syncthreads();
    }
  }
  if (track && t == 0) S.gen_reached[lig] = reached;
  // the population back in the caller's layout
  for (int c = 0; c < P; c += NT) {
    const int i = c + t;
    if (i < P) {
      float *row = pop + (int64_t)i * G;
      for (int j = 0; j < G; ++j) row[j] = W[j * P + i];
    }
  }
  // best member: first index of the smallest energy
  __shared__ int s_best;
  if (t == 0) {
    int bi = 0;
    for (int i = 1; i < P; ++i)
      if (E[i] < E[bi]) bi = i;
    s_best = bi;
    S.best_e[lig] = E[bi];
  }
  __syncthreads();
  const int bi = s_best;
  for (int j = t; j < G; j += NT) S.best_g[(int64_t)lig * G + j] = W[(int64_t)j * P + bi];
  __syncthreads();
}

// Persistent: each workgroup keeps taking ligands from the queue until none is
// left.  Block b of the workgroup keeps its poses' coordinates in its own LDS
// region of lds_atoms * 3 rows of 64 dwords, followed (WS > 1) by WS rows for
// the energy reduction.
// Register budget: at least four wavefronts per SIMD (128 VGPRs) with four or
// eight wavefronts per block, whose LDS per wavefront allows that residency;
// three otherwise.
template <int LAYOUT, int WS, bool TAIL>
__global__ __launch_bounds__(kSearchMaxThreads, WS >= 4 ? 4 : 3) void search_kernel(SearchLaunch S) {
  extern __shared__ float lds[];
  __shared__ int s_q;
  const int block = __builtin_amdgcn_readfirstlane((threadIdx.x / kWave) / WS), lane = threadIdx.x % kWave;
  float *base = lds + (size_t)block * search_block_floats(S.lds_atoms, WS);
  float *my = base + lane;
  float *red = base + 3 * S.lds_atoms * kBlock + lane;
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(S.queue, 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= S.n_order) break;
    search_ligand<LAYOUT, WS, TAIL>(S, S.order[q], my, red);
  }
}

__global__ void fill_i32_kernel(int32_t *p, int32_t n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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

hipError_t launch_fill_i32(int32_t *p, int32_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <int LAYOUT, int WS>
static hipError_t launch_search_t(const SearchLaunch &S, int32_t n_cu, int32_t blocks, hipStream_t s,
                                  const char **step) {
  // Blocks per workgroup, b: up to one per 64 individuals.  Each block's LDS is
  // sized for the bucket's largest ligand, so a larger b can leave fewer
  // wavefronts resident per CU.  Unless the caller fixes b, pick the b that
  // minimises (rounds of resident ligands) x (scoring passes per generation).
  // splits 2, 4 and 8 have a half-block instance (the same kernel otherwise)
  constexpr bool kCanTail = WS >= 2;
  auto kernel = (const void *)search_kernel<LAYOUT, WS, false>;
  auto kernel_tail = (const void *)search_kernel<LAYOUT, WS, kCanTail>;
  const size_t per_block = search_block_floats(S.lds_atoms, WS) * sizeof(float);
  const int max_b = kSearchMaxThreads / (kWave * WS);
  const int want = std::min((S.p.pop + kBlock - 1) / kBlock, max_b);
  // The dynamic LDS allowance is what the CU holds less the kernel's static LDS
  // (its __shared__ variables plus what the compiler adds for block reductions).
  hipFuncAttributes fa;
  *step = "hipFuncGetAttributes";
  if (hipError_t e = hipFuncGetAttributes(&fa, kernel); e != hipSuccess) return e;
  hipFuncAttributes fa_tail;
  if (hipError_t e = hipFuncGetAttributes(&fa_tail, kernel_tail); e != hipSuccess) return e;
  fa.sharedSizeBytes = std::max(fa.sharedSizeBytes, fa_tail.sharedSizeBytes);
  fa.numRegs = std::max(fa.numRegs, fa_tail.numRegs);
  if (fa.sharedSizeBytes >= kLdsPerCU) return hipErrorInvalidConfiguration;
  const size_t max_dyn = kLdsPerCU - fa.sharedSizeBytes;
  const int top_b = std::max(want, std::min(blocks, max_b));
  *step = "hipFuncSetAttribute (largest size)";
  if (per_block * top_b > 65536) {
    for (const void *k : {kernel, kernel_tail}) {
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)std::min<size_t>(max_dyn, per_block * top_b));
      if (e != hipSuccess) return e;
    }
  }
  // Resident workgroups per CU: bounded by the CU's LDS (dynamic + static per
  // workgroup) and by its vector registers (512 per lane per SIMD, allocated in
  // steps of 8, at most 8 wavefronts per SIMD).  The runtime's occupancy query
  // is also taken, and the larger answer used: a workgroup that does not fit
  // waits for a free slot, which a persistent kernel with a work queue tolerates.
  const int vgprs = std::max(8, (fa.numRegs + 7) / 8 * 8);
  const int waves_per_cu = 4 * std::min(8, 512 / vgprs);
  auto resident = [&](int b, int *groups) -> hipError_t {
    *groups = 0;
    if (per_block * b > max_dyn) return hipSuccess;
    *step = "hipOccupancyMaxActiveBlocksPerMultiprocessor";
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(groups, kernel, b * WS * kWave, per_block * b);
    if (e != hipSuccess) return e;
    const int by_lds = (int)(kLdsPerCU / (per_block * b + fa.sharedSizeBytes));
    *groups = std::max(*groups, std::min(by_lds, waves_per_cu / (b * WS)));
    return hipSuccess;
  };
  int best_b = 0, best_groups = 0;
  if (blocks > 0) {
    // the caller's count, lowered to what the LDS of one CU holds
    for (best_b = std::min(blocks, max_b); best_b > 1 && per_block * best_b > max_dyn; --best_b) {
    }
    if (hipError_t e = resident(best_b, &best_groups); e != hipSuccess) return e;
    if (best_groups < 1) return hipErrorInvalidConfiguration;
  } else {
    int64_t best_cost = -1;
    for (int b = 1; b <= want; ++b) {
      int groups = 0;
      if (hipError_t e = resident(b, &groups); e != hipSuccess) return e;
      if (groups < 1) continue;
      const int64_t slots = (int64_t)n_cu * groups;
      const int64_t rounds = (S.n_order + slots - 1) / slots;
      const int64_t passes = (S.p.pop + b * kBlock - 1) / (b * kBlock);
      if (best_cost < 0 || rounds * passes < best_cost) best_cost = rounds * passes, best_b = b, best_groups = groups;
    }
    if (best_b == 0) return hipErrorInvalidConfiguration;
  }
  const size_t lds = per_block * best_b;
  const int64_t grid = std::min<int64_t>(S.n_order, (int64_t)n_cu * best_groups);
  // the half-block instance when the population ends in a pass of at most
  // half a pass (splits 2, 4 and 8)
  const int pass = best_b * kBlock, rem = S.p.pop % pass;
  const bool tail = kCanTail && rem > 0 && 2 * rem <= pass;
  *step = "search kernel launch";
  void (*const fn)(SearchLaunch) = tail ? search_kernel<LAYOUT, WS, kCanTail> : search_kernel<LAYOUT, WS, false>;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(best_b * WS * kWave), lds, s, S);
  return hipGetLastError();
}

template <int LAYOUT>
static hipError_t launch_search_ws(const SearchLaunch &S, int32_t n_cu, SearchShape shape, hipStream_t s,
                                   const char **step) {
  if (shape.split == 8) return launch_search_t<LAYOUT, 8>(S, n_cu, shape.blocks, s, step);
  if (shape.split == 4) return launch_search_t<LAYOUT, 4>(S, n_cu, shape.blocks, s, step);
  if (shape.split == 2) return launch_search_t<LAYOUT, 2>(S, n_cu, shape.blocks, s, step);
  return launch_search_t<LAYOUT, 1>(S, n_cu, shape.blocks, s, step);
}

bool search_shape_fits(int32_t lds_atoms, SearchShape shape) {
  const size_t per_block = search_block_floats(lds_atoms, shape.split) * sizeof(float);
  return per_block * (size_t)std::max(shape.blocks, 1) + 1024 <= kLdsPerCU &&
         std::max(shape.blocks, 1) * shape.split * kWave <= kSearchMaxThreads;
}

hipError_t launch_search(const SearchLaunch &S, int32_t layout, int32_t n_cu, SearchShape shape, hipStream_t s,
                         const char **step) {
  if (S.n_order <= 0) return hipSuccess;
  switch (layout) {
    case kLinear: return launch_search_ws<kLinear>(S, n_cu, shape, s, step);
    case kZPair: return launch_search_ws<kZPair>(S, n_cu, shape, s, step);
    case kYZQuad: return launch_search_ws<kYZQuad>(S, n_cu, shape, s, step);
    case kQuadLine: return launch_search_ws<kQuadLine>(S, n_cu, shape, s, step);
    case kPairLine: return launch_search_ws<kPairLine>(S, n_cu, shape, s, step);
  }
  return hipErrorInvalidValue;
}

}  // namespace dock
