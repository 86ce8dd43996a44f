// score.hip -- batched pose scoring kernel for gfx950.
//
// One workgroup of WS = 1, 2, 4 or 8 wavefronts scores a block of 64 poses, one
// per lane, the wavefronts splitting each pose's atoms and pair records (the
// same bits for every WS).  Poses of one ligand share every uniform load; a
// block holding poses of several ligands scores it once per ligand, each pass
// keeping the results of its own lanes.
#include "dock_internal.h"
#include "score_pose.h"

#include <algorithm>

namespace dock {

// With four or eight wavefronts per block the register budget is five
// wavefronts per SIMD (96 VGPRs), which a block's LDS allows for ligands of up
// to about 50 atoms.
template <int LAYOUT, int WS>
__global__ __launch_bounds__(kWave * WS, WS >= 4 ? 5 : 1) void score_kernel(ScoreLaunch A, int64_t first) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x % kWave;
  const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t pose = first + (int64_t)blockIdx.x * kBlock + lane;
  const bool live = pose < A.n_poses;
  int lig = -1;
  if (live) {
    if (A.poses_per_ligand > 0) lig = (int)(pose / A.poses_per_ligand);
    else lig = A.pose_ligand ? A.pose_ligand[pose] : 0;
  }
  const bool valid = live & (lig >= 0) & (lig < A.L.n_ligs);
  float e = __builtin_nanf("");
  // lanes past the end read pose 0's genes (in bounds), and their results are dropped
  const float *g = A.genotypes + (live ? pose : 0) * (int64_t)A.g_stride;
  float *my = lds + lane;
  float *red = lds + 3 * A.lds_atoms * kBlock + lane;
  // the same ligand sequence in every wavefront of the block (the same lanes),
  // so all of them meet the same barriers
  uint64_t todo = __ballot(valid);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int cur = __builtin_amdgcn_readlane(lig, leader);
    const LigHeader H = as_const(A.L.hdr)[cur];
    // map loads two atoms ahead with one or two wavefronts per block, one with
    // four or eight (measured on MI355X: there the registers of a second atom
    // cost more residency than its loads hide)
    const float v = score_pose<LAYOUT, WS, WS <= 2 ? 2 : 1>(A.L, A.geom, A.ff, A.maps, H, g, 1, my, red, h);
    if (valid && lig == cur) e = v;
    todo &= ~__ballot(valid && lig == cur);
  }
  if (h == 0 && live) A.energies[pose] = e;
}

// Poses per launch: the grid's work-items (64 WS per block) stay below 2^31.
constexpr int64_t kPosesPerLaunch = (int64_t)1 << 24;

template <int LAYOUT, int WS>
static hipError_t launch_score_ws(const ScoreLaunch &a, hipStream_t s) {
  const size_t lds = ((size_t)a.lds_atoms * 3 + block_extra_rows(WS)) * kBlock * sizeof(float);
  auto fn = score_kernel<LAYOUT, WS>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  for (int64_t first = 0; first < a.n_poses; first += kPosesPerLaunch) {
    const int64_t n = std::min<int64_t>(kPosesPerLaunch, a.n_poses - first);
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kWave * WS), lds, s, a, first);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int LAYOUT>
static hipError_t launch_score_t(const ScoreLaunch &a, hipStream_t s) {
  switch (a.split) {
    case 1: return launch_score_ws<LAYOUT, 1>(a, s);
    case 2: return launch_score_ws<LAYOUT, 2>(a, s);
    case 4: return launch_score_ws<LAYOUT, 4>(a, s);
    case 8: return launch_score_ws<LAYOUT, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_score(const ScoreLaunch &a, hipStream_t s) {
  if (a.n_poses <= 0) return hipSuccess;
  switch (a.layout) {
    case kLinear: return launch_score_t<kLinear>(a, s);
    case kZPair: return launch_score_t<kZPair>(a, s);
    case kYZQuad: return launch_score_t<kYZQuad>(a, s);
    case kQuadLine: return launch_score_t<kQuadLine>(a, s);
    case kPairLine: return launch_score_t<kPairLine>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dock
