// search.h -- launch records of the differential-evolution kernels.
#pragma once
#include "dock_internal.h"

namespace dock {

struct DEParams {
  int32_t pop, n_gen, first_gen;
  uint64_t seed;
  float F, CR;
  double lo[3], hi[3];
};

hipError_t launch_de_init(const LigandsDev &L, const DEParams &p, int32_t g_stride, float *pop, hipStream_t s);
hipError_t launch_de_trials(const LigandsDev &L, const DEParams &p, int32_t gen, int32_t g_stride,
                            const float *pop, float *trials, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t n, int32_t v, hipStream_t s);

// One persistent search launch over the ligands order[0 .. n_order) (one size
// bucket), taken from the queue counter *queue (which starts at 0).
struct SearchLaunch {
  LigandsDev L;
  MapGeom geom;
  FFConst ff;
  MapData maps;
  DEParams p;
  int32_t g_stride;
  int32_t init;
  float *population;     // [n_ligs][pop][g_stride], in/out
  float *pop_energy;     // [n_ligs][pop], in/out
  float *work;           // [n_ligs][g_stride][pop] scratch: the population, gene-major
  float *trials;         // [n_ligs][g_stride][pop] scratch (trials, gene-major)
  float *best_g;         // [n_ligs][g_stride]
  float *best_e;         // [n_ligs]
  const float *target;   // [n_ligs] or null
  int32_t *gen_reached;  // [n_ligs] or null
  const int32_t *order;
  int32_t n_order;
  int32_t *queue;
  int32_t lds_atoms;     // atom slots per lane in LDS (largest ligand of the launch)
  int32_t stop;          // end a ligand's search once gen_reached is set
  const float *proposals;  // [n_ligs][pop][g_stride] or null: scored and taken greedily before the generations
};

constexpr int kSearchMaxThreads = 768;      // wavefronts per search workgroup: up to 12
constexpr size_t kLdsPerCU = 160 * 1024;    // gfx950 LDS per compute unit

// LDS floats of one pose block of the search kernel: the coordinate columns of
// 64 poses of up to lds_atoms atoms, then (ws > 1) the block's reduction rows.
__host__ __device__ constexpr size_t search_block_floats(int32_t lds_atoms, int32_t ws) {
  return ((size_t)lds_atoms * 3 + block_extra_rows(ws)) * kWave;
}

// Launch shape of a bucket: the split (1, 2, 4 or 8 wavefronts per block of 64
// poses) and the blocks per workgroup (0: chosen from the ligand count and the
// residency the LDS allows).
struct SearchShape {
  int32_t split;
  int32_t blocks;
};

hipError_t launch_search(const SearchLaunch &S, int32_t layout, int32_t n_cu, SearchShape shape, hipStream_t s,
                         const char **step);
// Whether a shape's wavefronts fit one CU's LDS for ligands of up to lds_atoms atoms.
bool search_shape_fits(int32_t lds_atoms, SearchShape shape);

}  // namespace dock
