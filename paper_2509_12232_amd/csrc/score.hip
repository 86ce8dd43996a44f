// score.hip -- batched pose scoring kernel for gfx950.
//
// One 64-lane workgroup (one wavefront) scores 64 / LP poses with LP = 1, 2 or 4
// lanes per pose (the same bits for every LP).  Poses of one ligand share every
// uniform load; a wavefront holding poses of several ligands walks them one
// ligand at a time (each pass masks the other lanes).
#include "dock_internal.h"
#include "score_pose.h"

namespace dock {

template <int LAYOUT, int LP>
__global__ __launch_bounds__(kWave) void score_kernel(ScoreLaunch A) {
  constexpr int PPW = kWave / LP;  // poses per wavefront; lane p + PPW h is lane h of pose p
  extern __shared__ float lds[];
  const int lane = threadIdx.x;
  const int p = lane % PPW;
  const int64_t pose = (int64_t)blockIdx.x * PPW + p;
  if (pose >= A.n_poses) return;   // all LP lanes of a pose leave together
  int lig;
  if (A.poses_per_ligand > 0) lig = (int)(pose / A.poses_per_ligand);
  else lig = A.pose_ligand ? A.pose_ligand[pose] : 0;
  const bool valid = (lig >= 0) & (lig < A.L.n_ligs);
  float e = __builtin_nanf("");
  const float *g = A.genotypes + pose * (int64_t)A.g_stride;
  float *my = lds + p;
  uint64_t todo = __ballot(valid);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int cur = __builtin_amdgcn_readlane(lig, leader);
    const LigHeader H = A.L.hdr[cur];
    // map loads two atoms ahead with one or two lanes per pose (measured faster
    // on MI355X; with four lanes the extra registers cost more than they hide)
    if (valid && lig == cur) e = score_pose<PPW, LAYOUT, LP, LP <= 2 ? 2 : 1>(A.L, A.geom, A.ff, A.maps, H, g, 1, my);
    todo &= ~__ballot(valid && lig == cur);
  }
  if (lane < PPW) A.energies[pose] = e;
}

template <int LAYOUT, int LP>
static hipError_t launch_score_lp(const ScoreLaunch &a, hipStream_t s) {
  constexpr int PPW = kWave / LP;
  const int64_t blocks = (a.n_poses + PPW - 1) / PPW;
  const size_t lds = (size_t)a.lds_atoms * 3 * PPW * sizeof(float);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)score_kernel<LAYOUT, LP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  auto fn = score_kernel<LAYOUT, LP>;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kWave), lds, s, a);
  return hipGetLastError();
}

template <int LAYOUT>
static hipError_t launch_score_t(const ScoreLaunch &a, hipStream_t s) {
  switch (a.lanes_per_pose) {
    case 1: return launch_score_lp<LAYOUT, 1>(a, s);
    case 2: return launch_score_lp<LAYOUT, 2>(a, s);
    case 4: return launch_score_lp<LAYOUT, 4>(a, s);
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
