// score_pose.h -- device code that builds one pose from its genotype and scores
// it (Sec. V: Algorithm 1 followed by Algorithm 2), with one, two, four or eight
// wavefronts sharing a block of poses.
//
// Mapping: a block of 64 poses, one per lane, is built and scored by WS = 1, 2,
// 4 or 8 wavefronts together (the "split"): lane l of each of them works on
// pose l, and wavefront h of the block takes its share of the atoms and of the
// pair records.  All ligand data (atoms, torsions, pairs) is uniform across a
// wavefront and arrives through scalar loads, so every loop below is a scalar
// loop and every pair record is an instruction operand as loaded (in a half
// block, described at score_pose, records and atoms differ between the two lane
// halves and arrive by vector loads; the loops stay scalar).  A pose's
// atom coordinates live in an LDS column shared by its WS lanes: coordinate c
// of atom i at my[(3 i + c) * 64], so the lanes that read the same atom hit
// consecutive dwords.
#pragma once
#include "dock_internal.h"

namespace dock {

__device__ __forceinline__ float lerp1(float a, float b, float t) { return fmaf(t, b - a, a); }

// Raw map values of one atom's grid cell, as loaded for the layout, plus what
// is needed to finish the interpolation later.  v[b] of the combined value is
// corner (x + (b&1), y + (b>>1 & 1), z + (b>>2 & 1)).
template <int LAYOUT>
struct Corners;

template <>
struct Corners<kLinear> {
  float t[8], e[8], d[8];
  float fx, fy, fz, q, aq;
  bool inside;
  __device__ __forceinline__ void combine(float v[8]) const {
#pragma unroll
    for (int b = 0; b < 8; ++b) v[b] = fmaf(aq, d[b], fmaf(q, e[b], t[b]));
  }
};

template <>
struct Corners<kZPair> {
  float2 t00, t10, t01, t11;   // (z, z+1) at x/x+1, y/y+1
  float4 d00, d10, d01, d11;   // (E z, E z+1, D z, D z+1)
  float fx, fy, fz, q, aq;
  bool inside;
  __device__ __forceinline__ void combine(float v[8]) const {
    v[0] = fmaf(aq, d00.z, fmaf(q, d00.x, t00.x));
    v[1] = fmaf(aq, d10.z, fmaf(q, d10.x, t10.x));
    v[2] = fmaf(aq, d01.z, fmaf(q, d01.x, t01.x));
    v[3] = fmaf(aq, d11.z, fmaf(q, d11.x, t11.x));
    v[4] = fmaf(aq, d00.w, fmaf(q, d00.y, t00.y));
    v[5] = fmaf(aq, d10.w, fmaf(q, d10.y, t10.y));
    v[6] = fmaf(aq, d01.w, fmaf(q, d01.y, t01.y));
    v[7] = fmaf(aq, d11.w, fmaf(q, d11.y, t11.y));
  }
};

template <>
struct Corners<kYZQuad> {
  float4 t0, t1, e0, d0, e1, d1;   // quads (y z, y+1 z, y z+1, y+1 z+1) at x and x+1
  float fx, fy, fz, q, aq;
  bool inside;
  __device__ __forceinline__ void combine(float v[8]) const {
    v[0] = fmaf(aq, d0.x, fmaf(q, e0.x, t0.x));
    v[1] = fmaf(aq, d1.x, fmaf(q, e1.x, t1.x));
    v[2] = fmaf(aq, d0.y, fmaf(q, e0.y, t0.y));
    v[3] = fmaf(aq, d1.y, fmaf(q, e1.y, t1.y));
    v[4] = fmaf(aq, d0.z, fmaf(q, e0.z, t0.z));
    v[5] = fmaf(aq, d1.z, fmaf(q, e1.z, t1.z));
    v[6] = fmaf(aq, d0.w, fmaf(q, e0.w, t0.w));
    v[7] = fmaf(aq, d1.w, fmaf(q, e1.w, t1.w));
  }
};

template <>
struct Corners<kQuadLine> {
  float4 t0, t1, s0, s1;   // type and signed quads (y z, y+1 z, y z+1, y+1 z+1) at x and x+1
  float fx, fy, fz, q, aq;
  bool inside;
  __device__ __forceinline__ void combine(float v[8]) const {
    v[0] = fmaf(q, s0.x, t0.x);
    v[1] = fmaf(q, s1.x, t1.x);
    v[2] = fmaf(q, s0.y, t0.y);
    v[3] = fmaf(q, s1.y, t1.y);
    v[4] = fmaf(q, s0.z, t0.z);
    v[5] = fmaf(q, s1.z, t1.z);
    v[6] = fmaf(q, s0.w, t0.w);
    v[7] = fmaf(q, s1.w, t1.w);
  }
};

// kPairLine loads the same four quads, from one line.
template <>
struct Corners<kPairLine> : Corners<kQuadLine> {};

// Trilinear interpolation of (T_type + q E + |q| D) from loaded corners; 0 outside
// the closed grid box (Algorithm 2's "nearby" test).
template <int LAYOUT>
__device__ __forceinline__ float interpolate_corners(const Corners<LAYOUT> &C) {
  float v[8];
  C.combine(v);
  const float c00 = lerp1(v[0], v[1], C.fx), c10 = lerp1(v[2], v[3], C.fx);
  const float c01 = lerp1(v[4], v[5], C.fx), c11 = lerp1(v[6], v[7], C.fx);
  const float c0 = lerp1(c00, c10, C.fy), c1 = lerp1(c01, c11, C.fy);
  const float e = lerp1(c0, c1, C.fz);
  return C.inside ? e : 0.f;
}

// Cell of an atom at p and the loads of its corner values.
template <int LAYOUT>
__device__ __forceinline__ Corners<LAYOUT> gather_corners(const MapGeom &G, const MapData &M, int type, float q,
                                                          float px, float py, float pz) {
  Corners<LAYOUT> C;
  const float ux = (px - G.ox) * G.inv_h;
  const float uy = (py - G.oy) * G.inv_h;
  const float uz = (pz - G.oz) * G.inv_h;
  const float mx = (float)(G.nx - 1), my = (float)(G.ny - 1), mz = (float)(G.nz - 1);
  C.inside = (ux >= 0.f) & (ux <= mx) & (uy >= 0.f) & (uy <= my) & (uz >= 0.f) & (uz <= mz);
  // cell index clamped into [0, n-2] so that every load stays in bounds, also
  // for atoms outside the box (whose contribution is then discarded)
  const float fcx = fminf(fmaxf(floorf(ux), 0.f), mx - 1.f);
  const float fcy = fminf(fmaxf(floorf(uy), 0.f), my - 1.f);
  const float fcz = fminf(fmaxf(floorf(uz), 0.f), mz - 1.f);
  C.fx = ux - fcx;
  C.fy = uy - fcy;
  C.fz = uz - fcz;
  C.q = q;
  C.aq = fabsf(q);
  const int cx = (int)fcx, cy = (int)fcy, cz = (int)fcz;
  const int nx = G.nx;
  if constexpr (LAYOUT == kLinear) {
    const int nxy = G.nx * G.ny;
    const int plane = nxy * G.nz;
    const int idx = cx + nx * cy + nxy * cz;
    const float *T = M.lin + (size_t)type * plane;
    const float *E = M.lin + (size_t)G.n_types * plane;
    const float *D = E + plane;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int o = idx + (b & 1) + ((b >> 1) & 1) * nx + ((b >> 2) & 1) * nxy;
      C.t[b] = T[o];
      C.e[b] = E[o];
      C.d[b] = D[o];
    }
  } else if constexpr (LAYOUT == kZPair) {
    const int e = cx + nx * (cy + G.ny * cz);
    const float2 *T = M.tz + (size_t)type * M.t_stride;
    C.t00 = T[e]; C.t10 = T[e + 1]; C.t01 = T[e + nx]; C.t11 = T[e + nx + 1];
    C.d00 = M.edz[e]; C.d10 = M.edz[e + 1]; C.d01 = M.edz[e + nx]; C.d11 = M.edz[e + nx + 1];
  } else if constexpr (LAYOUT == kYZQuad) {
    const int e = cx + nx * (cy + (G.ny - 1) * cz);
    const float4 *T = M.tq + (size_t)type * M.t_stride;
    C.t0 = T[e]; C.t1 = T[e + 1];
    C.e0 = M.edq[2 * e]; C.d0 = M.edq[2 * e + 1]; C.e1 = M.edq[2 * e + 2]; C.d1 = M.edq[2 * e + 3];
  } else if constexpr (LAYOUT == kQuadLine) {
    // line k = cx / 7 of row (cy, cz), slot cx - 7k in [0, 6]: both quads in one line
    const int k = cx / kLineCells;
    const int e = ((cz * (G.ny - 1) + cy) * M.nxb + k) * kLineQuads + (cx - k * kLineCells);
    const float4 *T = M.lq + (size_t)type * M.t_stride;
    const float4 *Sg = M.lq + (size_t)(G.n_types + (q < 0.f ? 1 : 0)) * M.t_stride;
    C.t0 = T[e]; C.t1 = T[e + 1];
    C.s0 = Sg[e]; C.s1 = Sg[e + 1];
  } else {
    // line k = cx / 3 of row (cy, cz) in the atom's (type, sign) copy, node slot
    // cx - 3k in [0, 2]: (T, S) of node x, then of node x + 1, 64 contiguous bytes
    const int k = cx / kPairCells;
    const int e = ((cz * (G.ny - 1) + cy) * M.nxb + k) * (2 * kPairNodes) + 2 * (cx - k * kPairCells);
    const float4 *B = M.pq + (size_t)(2 * type + (q < 0.f ? 1 : 0)) * M.t_stride;
    C.t0 = B[e]; C.s0 = B[e + 1];
    C.t1 = B[e + 2]; C.s1 = B[e + 3];
  }
  return C;
}

// One non-bonded pair term.  hb selects the 12-10 attractive exponent.
template <bool HB>
__device__ __forceinline__ float pair_term(const FFConst &F, const PairRec &P, float dx, float dy, float dz) {
  // The two clamps compare bit patterns as integers: that orders floats the
  // way fmaxf / fminf do whenever the bound is positive (r2 and rmin2 are
  // non-negative; a negative vdw is a negative integer, below any positive
  // cap), and an integer max or min takes the scalar bound as an operand with
  // no quieting step.
  float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  r2 = __int_as_float(max(__float_as_int(r2), __float_as_int(F.rmin2)));
  const float ir = __builtin_amdgcn_rsqf(r2);
  const float ir2 = ir * ir;
  const float ir6 = ir2 * ir2 * ir2;
  const float ir12 = ir6 * ir6;
  const float att = HB ? ir6 * ir2 * ir2 : ir6;
  const float vdw = __int_as_float(min(__float_as_int(fmaf(P.A, ir12, -P.B * att)), __float_as_int(F.e_cap)));
  const float r = r2 * ir;
  const float ex = __builtin_amdgcn_exp2f(r * F.diel_c);
  const float inv_eps = fmaf(F.k, ex, 1.f) * __builtin_amdgcn_rcpf(fmaf(F.Ak, ex, F.eps0));
  const float elec = P.qq * ir * inv_eps;
  const float gs = __builtin_amdgcn_exp2f(r2 * F.gauss_c);
  return fmaf(P.sv, gs, vdw + elec);
}

__device__ __forceinline__ float &at(float *my, int atom, int c) { return my[(3 * atom + c) * kBlock]; }

// The ligand tables as constant memory: the kernels never write them, and
// uniform loads through these pointers become scalar loads even in kernels
// that also store to global memory.  (The host pass of the compiler, which
// only checks the kernels' syntax, sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
#else
template <class T>
using cptr = const T *;
#endif
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

// R consecutive pair records (uniform, so scalar operands as loaded).
template <int R>
struct PairSlice {
  PairRec r[R];
  __device__ __forceinline__ void load(cptr<PairRec> p) {
#pragma unroll
    for (int u = 0; u < R; ++u) r[u] = p[u];
  }
};

// The atoms' coordinates of the R pairs of a slice, read from this lane's column.
template <int R>
struct SliceCoords {
  float xi[R], yi[R], zi[R], xj[R], yj[R], zj[R];
  __device__ __forceinline__ void load(const PairSlice<R> &S, float *my) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = S.r[u].ij & 0xffff, j = S.r[u].ij >> 16;
      xi[u] = at(my, i, 0); yi[u] = at(my, i, 1); zi[u] = at(my, i, 2);
      xj[u] = at(my, j, 0); yj[u] = at(my, j, 1); zj[u] = at(my, j, 2);
    }
  }
};

// Balanced pairwise sum of N values (N a power of two): the order in which a
// pose's partial sums are combined, the same for every split.
template <int N>
__device__ __forceinline__ float tree_sum(const float *v) {
  if constexpr (N == 1) {
    return v[0];
  } else {
    return tree_sum<N / 2>(v) + tree_sum<N / 2>(v + N / 2);
  }
}

// Barrier of the wavefronts that share pose blocks (the workgroup), ordering
// their LDS writes before the reads that follow.
template <int WS>
__device__ __forceinline__ void block_sync() {
  if constexpr (WS > 1) __syncthreads();
}

// Energy of the pose whose gene j is g[j * gs] for ligand header H (uniform),
// computed by the WS wavefronts of a block together; this is wavefront h.  my
// is this lane's LDS column, red this lane's slot of the block's reduction area
// (WS floats at red[w * kBlock], w < WS; unused for WS = 1).  Every wavefront
// of the workgroup calls this the same number of times with the same ligand
// (each call holds n_tors + 3 workgroup barriers for WS > 1); lanes with no
// pose of that ligand compute a value that the caller discards.
//
// The energy is the balanced pairwise sum of kParts = 8 partial sums p_u:
//   p_u = (inter over atoms i with i % 8 == u, in index order)
//       + (record u of every pair group, in group order, then the 12-10 pairs p
//          with p % 8 == u, in index order),
// and wavefront h owns p_u for u in [h R, (h + 1) R), R = 8 / WS.  Every split
// therefore adds the same terms in the same order and gives the same bits.
// Every wavefront returns the energy.  Non-finite genes give NaN.  AHEAD: how
// many atoms ahead of its interpolation an atom's map loads are issued (more
// loads in flight, more registers); it does not change the result.
//
// HALF (WS < 8): a half block, 32 poses on lanes 0-31 with lane l + 32 given the
// genes of pose l.  The two lanes build the same pose into their own columns;
// the energy loops then run as if the block had 2 WS wavefronts, lane half s of
// wavefront h acting as wavefront 2 h + s, which owns the first (s = 0) or the
// second half of wavefront h's partial sums.  Records and atoms then differ
// between the halves and arrive by vector loads.  The two halves' subtotals
// are the two subtrees of wavefront h's share, so the energy has the same bits
// as in a full block.
template <int LAYOUT, int WS, int AHEAD, bool HALF = false>
__device__ float score_pose(const LigandsDev &L, const MapGeom &G, const FFConst &F, const MapData &maps,
                            const LigHeader &H, const float *__restrict__ g, int gs, float *__restrict__ my,
                            float *__restrict__ red, int h) {
  static_assert(WS == 1 || WS == 2 || WS == 4 || WS == 8, "one, two, four or eight wavefronts per block");
  static_assert(!HALF || WS < 8, "a half block needs two partial sums per wavefront");
  constexpr int WV = HALF ? 2 * WS : WS;  // wavefronts of the energy loops
  constexpr int R = kParts / WV;      // partial sums (and records of a group) per energy-loop wavefront
  constexpr int SL = R < 4 ? R : 4;   // records evaluated per step of the pair loop
  constexpr int NP = R / SL;          // steps per pair group
  const int n = H.n_atoms;
  const cptr<float4> atoms = as_const(L.atoms) + H.atom_off;
  const cptr<int32_t> types = as_const(L.atom_type) + H.atom_off;

  bool bad = false;
  // the genes are requested before they are needed: the rigid ones here, each
  // torsion angle one torsion ahead
  const float tx = g[0], ty = g[gs], tz = g[2 * gs];
  float qw = g[3 * gs], qx = g[4 * gs], qy = g[5 * gs], qz = g[6 * gs];
  const cptr<TorRec> tors = as_const(L.tors) + H.tor_off;
  float th_next = H.n_tors > 0 ? g[(7 + tors[0].gene) * gs] : 0.f;
  // reference conformation (centred) into the pose's LDS column
  for (int i = h; i < n; i += WS) {
    const float4 a = atoms[i];
    at(my, i, 0) = a.x;
    at(my, i, 1) = a.y;
    at(my, i, 2) = a.z;
  }
  block_sync<WS>();

  // Algorithm 1, rotatable bonds: rotate each fragment about its current bond
  // axis.  Rotations about current axes commute on a tree, so the torsion order
  // of the genotype is used as is.
  for (int k = 0; k < H.n_tors; ++k) {
    const TorRec T = tors[k];
    const float th = th_next;
    if (k + 1 < H.n_tors) th_next = g[(7 + tors[k + 1].gene) * gs];
    bad |= !__builtin_isfinite(th);
    float s, c;
    sincosf(th, &s, &c);
    const float ax = at(my, T.a, 0), ay = at(my, T.a, 1), az = at(my, T.a, 2);
    float ux = at(my, T.lo, 0) - ax, uy = at(my, T.lo, 1) - ay, uz = at(my, T.lo, 2) - az;
    const float il = __builtin_amdgcn_rsqf(fmaf(ux, ux, fmaf(uy, uy, uz * uz)));
    ux *= il; uy *= il; uz *= il;
    const float oc = 1.f - c;
    const float r00 = fmaf(ux * ux, oc, c), r01 = fmaf(ux * uy, oc, -uz * s), r02 = fmaf(ux * uz, oc, uy * s);
    const float r10 = fmaf(uy * ux, oc, uz * s), r11 = fmaf(uy * uy, oc, c), r12 = fmaf(uy * uz, oc, -ux * s);
    const float r20 = fmaf(uz * ux, oc, -uy * s), r21 = fmaf(uz * uy, oc, ux * s), r22 = fmaf(uz * uz, oc, c);
    for (int i = T.lo + 1 + h; i < T.hi; i += WS) {
      const float vx = at(my, i, 0) - ax, vy = at(my, i, 1) - ay, vz = at(my, i, 2) - az;
      at(my, i, 0) = ax + fmaf(r00, vx, fmaf(r01, vy, r02 * vz));
      at(my, i, 1) = ay + fmaf(r10, vx, fmaf(r11, vy, r12 * vz));
      at(my, i, 2) = az + fmaf(r20, vx, fmaf(r21, vy, r22 * vz));
    }
    block_sync<WS>();
  }

  // Algorithm 1, rigid part: rotate about the ligand origin, then translate
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

  for (int i = h; i < n; i += WS) {
    const float px = at(my, i, 0), py = at(my, i, 1), pz = at(my, i, 2);
    at(my, i, 0) = fmaf(R00, px, fmaf(R01, py, fmaf(R02, pz, tx)));
    at(my, i, 1) = fmaf(R10, px, fmaf(R11, py, fmaf(R12, pz, ty)));
    at(my, i, 2) = fmaf(R20, px, fmaf(R21, py, fmaf(R22, pz, tz)));
  }
  block_sync<WS>();

  // Algorithm 2: the inter-energy loop over atoms and the intra-energy loop over
  // pairs, interleaved.  Iteration k issues the map loads of the wavefront's
  // atom of slot k + AHEAD, then evaluates the k-th of equal slices of the pair
  // groups, then interpolates the atom of slot k from loads issued AHEAD
  // iterations earlier, so the pair arithmetic covers the latency of the
  // gathers.  The wavefront's records form a stream of steps of SL records
  // (NP steps per group); the coordinates of step s+1 and the records of step
  // s+2 are requested before step s is evaluated (the list ends with spare zero
  // groups to read past).
  // the energy loops' wavefront index (per lane for a half block)
  const int hv = HALF ? 2 * h + (int)(__lane_id() >> 5) : h;
  const cptr<PairRec> pairs = as_const(L.pairs) + H.pair_off + hv * R;
  auto step_ptr = [&](int st) { return pairs + kParts * (st / NP) + (st % NP) * SL; };
  const int ng = H.n_groups;
  // The wavefront's atoms in index order: slot k is atom 8 (k / R) + h R + k % R,
  // of class h R + k % R; wavefront 0 has the most slots, the others skip their
  // last.
  const int slots = R * (n / kParts) + min(n % kParts, R);
  auto atom_of = [&](int slot) { return kParts * (slot / R) + hv * R + slot % R; };
  float inter[R], intra[R];
#pragma unroll
  for (int u = 0; u < R; ++u) inter[u] = intra[u] = 0.f;
  // ring[d] holds the loads of the atom of slot k + d
  Corners<LAYOUT> ring[AHEAD + 1];
  auto gather = [&](int slot) {
    const int i = min(atom_of(slot), n - 1);
    return gather_corners<LAYOUT>(G, maps, types[i], atoms[i].w, at(my, i, 0), at(my, i, 1), at(my, i, 2));
  };
#pragma unroll
  for (int d = 0; d < AHEAD; ++d)
    if (d < slots) ring[d] = gather(d);
  // the pair terms of one step (records P, coordinates X) into its partial sums
  auto eval = [&](const PairSlice<SL> &P, const SliceCoords<SL> &X, int part) {
#pragma unroll
    for (int u = 0; u < SL; ++u)
      intra[part * SL + u] += pair_term<false>(F, P.r[u], X.xi[u] - X.xj[u], X.yi[u] - X.yj[u], X.zi[u] - X.zj[u]);
  };
  // Steps go two at a time with two coordinate sets used in turn (X0 for even
  // steps, X1 for odd ones), so no coordinates are copied between steps.  A:
  // records of the current step, B: of the next; X0: coordinates of A.
  PairSlice<SL> A, B;
  A.load(step_ptr(0));
  B.load(step_ptr(1));
  SliceCoords<SL> X0, X1;
  X0.load(A, my);
  for (int k = 0; k < slots; ++k) {
    const int ka = k + AHEAD;
    if (ka < slots) ring[AHEAD] = gather(ka);
    // this slot's steps: its equal share of the pair groups, NP steps each
    // (for NP = 2 both bounds are even, so a step's partial-sum block is its
    // position in the pair)
    const int s1 = NP * (((k + 1) * ng) / slots);
    int st = NP * ((k * ng) / slots);
    for (; st + 1 < s1; st += 2) {
      X1.load(B, my);
      PairSlice<SL> C;
      C.load(step_ptr(st + 2));
      eval(A, X0, 0);
      X0.load(C, my);
      PairSlice<SL> D;
      D.load(step_ptr(st + 3));
      eval(B, X1, NP - 1);
      A = C;
      B = D;
    }
    if (st < s1) {   // one step left (NP = 1 only)
      X1.load(B, my);
      PairSlice<SL> C;
      C.load(step_ptr(st + 2));
      eval(A, X0, 0);
      A = B;
      B = C;
      X0 = X1;
    }
    const float v = interpolate_corners<LAYOUT>(ring[0]);
    if (atom_of(k) < n) {
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (k % R == u) inter[u] += v;
    }
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) ring[d] = ring[d + 1];
  }
  // 12-10 pairs, kParts at a time (past the end: all-zero records, which add +0)
  const cptr<PairRec> hb = as_const(L.pairs) + H.hb_off;
  for (int p = 0; p < H.n_pairs_hb; p += kParts) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int q = p + hv * R + u;
      PairRec P{0, 0.f, 0.f, 0.f, 0.f};
      if (q < H.n_pairs_hb) P = hb[q];
      const int i = P.ij & 0xffff, j = P.ij >> 16;
      intra[u] += pair_term<true>(F, P, at(my, i, 0) - at(my, j, 0), at(my, i, 1) - at(my, j, 1),
                                  at(my, i, 2) - at(my, j, 2));
    }
  }
  float part[R];
#pragma unroll
  for (int u = 0; u < R; ++u) part[u] = inter[u] + intra[u];
  // this wavefront's share (the subtree of its partial sums), then, through
  // LDS, the shares of the block's wavefronts in the same tree
  float e = tree_sum<R>(part);
  // a half block: the other half's subtree (addition commutes, so both halves
  // hold the same sum)
  if constexpr (HALF) e = e + __shfl_xor(e, 32);
  if constexpr (WS > 1) {
    red[h * kBlock] = e;
    block_sync<WS>();
    float share[WS];
#pragma unroll
    for (int w = 0; w < WS; ++w) share[w] = red[w * kBlock];
    e = tree_sum<WS>(share);
  }
  return bad ? __builtin_nanf("") : e;
}

}  // namespace dock
