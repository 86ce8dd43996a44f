// score_pose.h -- device code that builds one pose from its genotype and scores
// it (Sec. V: Algorithm 1 followed by Algorithm 2), one pose per lane.
//
// Mapping: every lane owns one pose.  All ligand data (atoms, torsions, pairs)
// is uniform across the wavefront and arrives through scalar loads, so every
// loop below is a scalar loop with no divergence.  Each lane keeps its pose's
// atom coordinates in its own LDS column: coordinate c of atom i at
// my[(3 i + c) * STRIDE], STRIDE = lanes sharing one LDS row, which makes every
// LDS access of a wavefront hit 64 consecutive dwords (no bank conflicts).
#pragma once
#include "dock_internal.h"

namespace dock {

__device__ __forceinline__ float lerp1(float a, float b, float t) { return fmaf(t, b - a, a); }

// Trilinear interpolation of (T_type + q E + |q| D) at one atom; 0 outside the
// closed grid box (Algorithm 2's "nearby" test).
__device__ __forceinline__ float atom_inter(const MapGeom &G, const float *__restrict__ maps, int type,
                                            float q, float px, float py, float pz) {
  const float ux = (px - G.ox) * G.inv_h;
  const float uy = (py - G.oy) * G.inv_h;
  const float uz = (pz - G.oz) * G.inv_h;
  const float mx = (float)(G.nx - 1), my = (float)(G.ny - 1), mz = (float)(G.nz - 1);
  const bool inside = (ux >= 0.f) & (ux <= mx) & (uy >= 0.f) & (uy <= my) & (uz >= 0.f) & (uz <= mz);
  // cell index clamped into [0, n-2] so that every load stays in bounds, also
  // for atoms outside the box (whose contribution is then discarded)
  const float fcx = fminf(fmaxf(floorf(ux), 0.f), mx - 1.f);
  const float fcy = fminf(fmaxf(floorf(uy), 0.f), my - 1.f);
  const float fcz = fminf(fmaxf(floorf(uz), 0.f), mz - 1.f);
  const float fx = ux - fcx, fy = uy - fcy, fz = uz - fcz;
  const int nx = G.nx, nxy = G.nx * G.ny;
  const int plane = nxy * G.nz;
  const int idx = (int)fcx + nx * (int)fcy + nxy * (int)fcz;
  const float *T = maps + (size_t)type * plane;
  const float *E = maps + (size_t)G.n_types * plane;
  const float *D = E + plane;
  const float aq = fabsf(q);
  float v[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int o = idx + (b & 1) + ((b >> 1) & 1) * nx + ((b >> 2) & 1) * nxy;
    v[b] = fmaf(aq, D[o], fmaf(q, E[o], T[o]));
  }
  const float c00 = lerp1(v[0], v[1], fx), c10 = lerp1(v[2], v[3], fx);
  const float c01 = lerp1(v[4], v[5], fx), c11 = lerp1(v[6], v[7], fx);
  const float c0 = lerp1(c00, c10, fy), c1 = lerp1(c01, c11, fy);
  const float e = lerp1(c0, c1, fz);
  return inside ? e : 0.f;
}

// One non-bonded pair term.  hb selects the 12-10 attractive exponent.
template <bool HB>
__device__ __forceinline__ float pair_term(const FFConst &F, const PairRec &P, float dx, float dy, float dz) {
  float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  r2 = fmaxf(r2, F.rmin2);
  const float ir = __builtin_amdgcn_rsqf(r2);
  const float ir2 = ir * ir;
  const float ir6 = ir2 * ir2 * ir2;
  const float ir12 = ir6 * ir6;
  const float att = HB ? ir6 * ir2 * ir2 : ir6;
  const float vdw = fminf(fmaf(P.A, ir12, -P.B * att), F.e_cap);
  const float r = r2 * ir;
  const float ex = __builtin_amdgcn_exp2f(r * F.diel_c);
  const float inv_eps = fmaf(F.k, ex, 1.f) * __builtin_amdgcn_rcpf(fmaf(F.Ak, ex, F.eps0));
  const float elec = P.qq * ir * inv_eps;
  const float gs = __builtin_amdgcn_exp2f(r2 * F.gauss_c);
  return fmaf(P.sv, gs, vdw + elec);
}

template <int STRIDE>
__device__ __forceinline__ float &at(float *my, int atom, int c) {
  return my[(3 * atom + c) * STRIDE];
}

// Energy of the pose given by genotype row g (per lane) for ligand header H
// (uniform).  Non-finite genes give NaN.
template <int STRIDE>
__device__ float score_pose(const LigandsDev &L, const MapGeom &G, const FFConst &F,
                            const float *__restrict__ maps, const LigHeader &H,
                            const float *__restrict__ g, float *__restrict__ my) {
  const int n = H.n_atoms;
  const float4 *__restrict__ atoms = L.atoms + H.atom_off;
  const int32_t *__restrict__ types = L.atom_type + H.atom_off;

  // reference conformation (centred) into this lane's LDS column
  for (int i = 0; i < n; ++i) {
    const float4 a = atoms[i];
    at<STRIDE>(my, i, 0) = a.x;
    at<STRIDE>(my, i, 1) = a.y;
    at<STRIDE>(my, i, 2) = a.z;
  }

  bool bad = false;
  // Algorithm 1, rotatable bonds: rotate each fragment about its current bond
  // axis.  Rotations about current axes commute on a tree, so the torsion order
  // of the genotype is used as is.
  const TorRec *__restrict__ tors = L.tors + H.tor_off;
  for (int k = 0; k < H.n_tors; ++k) {
    const TorRec T = tors[k];
    const float th = g[7 + T.gene];
    bad |= !__builtin_isfinite(th);
    const float ax = at<STRIDE>(my, T.a, 0), ay = at<STRIDE>(my, T.a, 1), az = at<STRIDE>(my, T.a, 2);
    float ux = at<STRIDE>(my, T.lo, 0) - ax, uy = at<STRIDE>(my, T.lo, 1) - ay, uz = at<STRIDE>(my, T.lo, 2) - az;
    const float il = __builtin_amdgcn_rsqf(fmaf(ux, ux, fmaf(uy, uy, uz * uz)));
    ux *= il; uy *= il; uz *= il;
    float s, c;
    sincosf(th, &s, &c);
    const float oc = 1.f - c;
    const float r00 = fmaf(ux * ux, oc, c), r01 = fmaf(ux * uy, oc, -uz * s), r02 = fmaf(ux * uz, oc, uy * s);
    const float r10 = fmaf(uy * ux, oc, uz * s), r11 = fmaf(uy * uy, oc, c), r12 = fmaf(uy * uz, oc, -ux * s);
    const float r20 = fmaf(uz * ux, oc, -uy * s), r21 = fmaf(uz * uy, oc, ux * s), r22 = fmaf(uz * uz, oc, c);
    for (int i = T.lo + 1; i < T.hi; ++i) {
      const float vx = at<STRIDE>(my, i, 0) - ax, vy = at<STRIDE>(my, i, 1) - ay, vz = at<STRIDE>(my, i, 2) - az;
      at<STRIDE>(my, i, 0) = ax + fmaf(r00, vx, fmaf(r01, vy, r02 * vz));
      at<STRIDE>(my, i, 1) = ay + fmaf(r10, vx, fmaf(r11, vy, r12 * vz));
      at<STRIDE>(my, i, 2) = az + fmaf(r20, vx, fmaf(r21, vy, r22 * vz));
    }
  }

  // Algorithm 1, rigid part: rotate about the ligand origin, then translate
  const float tx = g[0], ty = g[1], tz = g[2];
  float qw = g[3], qx = g[4], qy = g[5], qz = g[6];
  bad |= !(__builtin_isfinite(tx) & __builtin_isfinite(ty) & __builtin_isfinite(tz) & __builtin_isfinite(qw) &
           __builtin_isfinite(qx) & __builtin_isfinite(qy) & __builtin_isfinite(qz));
  const float nn = fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
  if (nn < 1e-24f) {
    qw = 1.f; qx = qy = qz = 0.f;
  } else {
    const float r = __builtin_amdgcn_rsqf(nn);
    qw *= r; qx *= r; qy *= r; qz *= r;
  }
  const float R00 = 1.f - 2.f * (qy * qy + qz * qz), R01 = 2.f * (qx * qy - qw * qz), R02 = 2.f * (qx * qz + qw * qy);
  const float R10 = 2.f * (qx * qy + qw * qz), R11 = 1.f - 2.f * (qx * qx + qz * qz), R12 = 2.f * (qy * qz - qw * qx);
  const float R20 = 2.f * (qx * qz - qw * qy), R21 = 2.f * (qy * qz + qw * qx), R22 = 1.f - 2.f * (qx * qx + qy * qy);

  // Algorithm 2, inter-energy loop (fused with the rigid move of each atom)
  float inter = 0.f;
  for (int i = 0; i < n; ++i) {
    const float px = at<STRIDE>(my, i, 0), py = at<STRIDE>(my, i, 1), pz = at<STRIDE>(my, i, 2);
    const float wx = fmaf(R00, px, fmaf(R01, py, fmaf(R02, pz, tx)));
    const float wy = fmaf(R10, px, fmaf(R11, py, fmaf(R12, pz, ty)));
    const float wz = fmaf(R20, px, fmaf(R21, py, fmaf(R22, pz, tz)));
    at<STRIDE>(my, i, 0) = wx;
    at<STRIDE>(my, i, 1) = wy;
    at<STRIDE>(my, i, 2) = wz;
    inter += atom_inter(G, maps, types[i], atoms[i].w, wx, wy, wz);
  }

  // Algorithm 2, intra-energy loop over the non-bonded pairs
  float intra = 0.f;
  const PairRec *__restrict__ pairs = L.pairs + H.pair_off;
#pragma unroll 4
  for (int p = 0; p < H.n_pairs; ++p) {
    const PairRec P = pairs[p];
    const float dx = at<STRIDE>(my, P.i, 0) - at<STRIDE>(my, P.j, 0);
    const float dy = at<STRIDE>(my, P.i, 1) - at<STRIDE>(my, P.j, 1);
    const float dz = at<STRIDE>(my, P.i, 2) - at<STRIDE>(my, P.j, 2);
    intra += pair_term<false>(F, P, dx, dy, dz);
  }
  for (int p = H.n_pairs; p < H.n_pairs + H.n_pairs_hb; ++p) {
    const PairRec P = pairs[p];
    const float dx = at<STRIDE>(my, P.i, 0) - at<STRIDE>(my, P.j, 0);
    const float dy = at<STRIDE>(my, P.i, 1) - at<STRIDE>(my, P.j, 1);
    const float dz = at<STRIDE>(my, P.i, 2) - at<STRIDE>(my, P.j, 2);
    intra += pair_term<true>(F, P, dx, dy, dz);
  }
  const float e = inter + intra;
  return bad ? __builtin_nanf("") : e;
}

}  // namespace dock
