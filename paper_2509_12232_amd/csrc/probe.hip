// probe.hip -- roofline probes for the scoring kernel's two halves.
//
// gather_probe: the inter-energy lookups alone (Algorithm 2's map lookups):
// each lane places one ligand rigidly at random (a translation uniform in a
// box, a random orientation) and interpolates its atoms in index order, then
// the next placement, through the same layout and gather code as the scoring
// kernel, at full occupancy and with no other work.  Its rate is the measured
// ceiling for the lookups of that workload's spatial distribution (torsional
// flexibility aside).
//
// pair_probe: the intra-energy pair term alone on register-resident
// coordinates, at full occupancy: the measured VALU ceiling for pair terms.
#include "dock_internal.h"
#include "probe.h"
#include "score_pose.h"

namespace dock {

// Counter-based hash (a 32-bit finaliser) for probe positions; no statistical
// requirement beyond spreading the lookups over the box.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ float unit01(uint32_t h) { return (float)(h >> 8) * (1.0f / 16777216.0f); }

template <int LAYOUT, int U>
__global__ __launch_bounds__(256) void gather_probe_kernel(MapGeom G, MapData M, LigandsDev L, int lig, ProbeBox box,
                                                            int per_lane, uint32_t seed, int64_t n_lanes,
                                                            float *out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)t >= n_lanes) return;
  const LigHeader H = L.hdr[lig];
  const float4 *__restrict__ atoms = L.atoms + H.atom_off;
  const int32_t *__restrict__ types = L.atom_type + H.atom_off;
  float acc = 0.f;
  for (int m = 0; m < per_lane; m += U) {   // U lookups in flight per lane
    Corners<LAYOUT> c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // lookup m + u is atom (m + u) % n of placement (m + u) / n
      const uint32_t place = (uint32_t)(m + u) / (uint32_t)H.n_atoms;
      const int i = (int)((uint32_t)(m + u) - place * (uint32_t)H.n_atoms);
      const uint32_t h = mix32(seed ^ mix32(t * 0x9E3779B9u + place));
      const float tx = box.lo[0] + box.ext[0] * unit01(mix32(h + 1));
      const float ty = box.lo[1] + box.ext[1] * unit01(mix32(h + 2));
      const float tz = box.lo[2] + box.ext[2] * unit01(mix32(h + 3));
      // orientation: normalised point of the cube [-1,1]^4 (isotropic enough for a footprint)
      float qw = 2.f * unit01(mix32(h + 4)) - 1.f, qx = 2.f * unit01(mix32(h + 5)) - 1.f;
      float qy = 2.f * unit01(mix32(h + 6)) - 1.f, qz = 2.f * unit01(mix32(h + 7)) - 1.f;
      const float r = __builtin_amdgcn_rsqf(fmaxf(fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz))), 1e-12f));
      qw *= r; qx *= r; qy *= r; qz *= r;
      const float4 a = atoms[i];
      const float px = fmaf(1.f - 2.f * (qy * qy + qz * qz), a.x, fmaf(2.f * (qx * qy - qw * qz), a.y, fmaf(2.f * (qx * qz + qw * qy), a.z, tx)));
      const float py = fmaf(2.f * (qx * qy + qw * qz), a.x, fmaf(1.f - 2.f * (qx * qx + qz * qz), a.y, fmaf(2.f * (qy * qz - qw * qx), a.z, ty)));
      const float pz = fmaf(2.f * (qx * qz - qw * qy), a.x, fmaf(2.f * (qy * qz + qw * qx), a.y, fmaf(1.f - 2.f * (qx * qx + qy * qy), a.z, tz)));
      c[u] = gather_corners<LAYOUT>(G, M, types[i], a.w, px, py, pz);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += interpolate_corners<LAYOUT>(c[u]);
  }
  out[t] = acc;
}

template <int LAYOUT>
static hipError_t launch_gather_probe_t(const MapGeom &G, const MapData &M, const LigandsDev &L, int32_t lig,
                                        const ProbeBox &box, int64_t n_lanes, int32_t per_lane, int32_t in_flight,
                                        uint32_t seed, float *out, hipStream_t s) {
  const unsigned blocks = (unsigned)((n_lanes + 255) / 256);
  void (*fn)(MapGeom, MapData, LigandsDev, int, ProbeBox, int, uint32_t, int64_t, float *);
  switch (in_flight) {
    case 2: fn = gather_probe_kernel<LAYOUT, 2>; break;
    case 4: fn = gather_probe_kernel<LAYOUT, 4>; break;
    case 8: fn = gather_probe_kernel<LAYOUT, 8>; break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, s, G, M, L, lig, box, per_lane, seed, n_lanes, out);
  return hipGetLastError();
}

hipError_t launch_gather_probe(const MapGeom &G, const MapData &M, int32_t layout, const LigandsDev &L,
                               int32_t lig, const ProbeBox &box, int64_t n_lanes, int32_t per_lane,
                               int32_t in_flight, uint32_t seed, float *out, hipStream_t s) {
  switch (layout) {
    case kLinear: return launch_gather_probe_t<kLinear>(G, M, L, lig, box, n_lanes, per_lane, in_flight, seed, out, s);
    case kZPair: return launch_gather_probe_t<kZPair>(G, M, L, lig, box, n_lanes, per_lane, in_flight, seed, out, s);
    case kYZQuad: return launch_gather_probe_t<kYZQuad>(G, M, L, lig, box, n_lanes, per_lane, in_flight, seed, out, s);
    case kQuadLine:
      return launch_gather_probe_t<kQuadLine>(G, M, L, lig, box, n_lanes, per_lane, in_flight, seed, out, s);
    case kPairLine:
      return launch_gather_probe_t<kPairLine>(G, M, L, lig, box, n_lanes, per_lane, in_flight, seed, out, s);
  }
  return hipErrorInvalidValue;
}

// Pair terms on coordinates held in registers: each lane evaluates per_lane pair
// terms with synthetic coordinates and coefficients.
__global__ __launch_bounds__(256) void pair_probe_kernel(FFConst F, int per_lane, int64_t n_lanes, float *out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)t >= n_lanes) return;
  const uint32_t h = mix32(t);
  float x = 3.f * unit01(h), y = 3.f * unit01(mix32(h + 1)), z = 3.f * unit01(mix32(h + 2));
  PairRec P{0, 1.2e5f, 0.9f, -30.f, 0.002f};
  float acc = 0.f;
  constexpr int U = 4;
  for (int m = 0; m < per_lane; m += U) {
    float e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) e[u] = pair_term<false>(F, P, x + 0.5f * u, y - 0.25f * u, z + (float)m * 1e-6f);
    acc += (e[0] + e[1]) + (e[2] + e[3]);
    x += 1e-3f;
  }
  out[t] = acc;
}

hipError_t launch_pair_probe(const FFConst &F, int64_t n_lanes, int32_t per_lane, float *out, hipStream_t s) {
  const unsigned blocks = (unsigned)((n_lanes + 255) / 256);
  hipLaunchKernelGGL(pair_probe_kernel, dim3(blocks), dim3(256), 0, s, F, per_lane, n_lanes, out);
  return hipGetLastError();
}

}  // namespace dock
