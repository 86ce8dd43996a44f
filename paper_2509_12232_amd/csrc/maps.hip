// maps.hip -- AutoGrid-like grid-map construction on the GPU (Sec. V: the fixed
// receptor is turned into per-type, electrostatic and desolvation maps).
//
// One thread per grid node; receptor atoms stream through LDS in tiles shared by
// the 256 threads of a block.  Per-type accumulators live in registers (the
// loop over types is unrolled to the compile-time maximum and predicated).
#include "maps.h"

namespace dock {

constexpr int kMapBlock = 256;

__global__ __launch_bounds__(kMapBlock) void build_maps_kernel(MapBuild M) {
  __shared__ float4 s_rec[kMapBlock];
  __shared__ int s_type[kMapBlock];
  const MapGeom &G = M.geom;
  const int64_t plane = (int64_t)G.nx * G.ny * G.nz;
  const int64_t node = (int64_t)blockIdx.x * kMapBlock + threadIdx.x;
  const bool live = node < plane;
  const int ix = (int)(node % G.nx), iy = (int)((node / G.nx) % G.ny), iz = (int)(node / ((int64_t)G.nx * G.ny));
  const float h = M.h;
  const float px = fmaf((float)ix, h, G.ox), py = fmaf((float)iy, h, G.oy), pz = fmaf((float)iz, h, G.oz);
  const int NT = G.n_types;
  float T[kMaxTypes];
#pragma unroll
  for (int a = 0; a < kMaxTypes; ++a) T[a] = 0.f;
  float E = 0.f, D = 0.f;
  for (int base = 0; base < M.n_rec; base += kMapBlock) {
    const int r = base + threadIdx.x;
    if (r < M.n_rec) {
      s_rec[threadIdx.x] = M.rec[r];
      s_type[threadIdx.x] = M.rec_type[r];
    }
    __syncthreads();
    const int cnt = min(kMapBlock, M.n_rec - base);
    for (int k = 0; k < cnt; ++k) {
      const float4 R = s_rec[k];
      const int tr = s_type[k];
      const float dx = px - R.x, dy = py - R.y, dz = pz - R.z;
      const float r2 = fmaxf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), M.rmin2);
      const float ir = __builtin_amdgcn_rsqf(r2);
      const float ir2 = ir * ir, ir6 = ir2 * ir2 * ir2, ir10 = ir6 * ir2 * ir2, ir12 = ir6 * ir6;
      const float rr = r2 * ir;
      const float gs = __builtin_amdgcn_exp2f(r2 * M.ff.gauss_c);
      const float ex = __builtin_amdgcn_exp2f(rr * M.ff.diel_c);
      const float inv_eps = fmaf(M.ff.k, ex, 1.f) * __builtin_amdgcn_rcpf(fmaf(M.ff.Ak, ex, M.ff.eps0));
      E = fmaf(M.coulomb * R.w, ir * inv_eps, E);
      const float vr = M.vol[tr];
      D = fmaf(M.qsolpar * vr, gs, D);
      const float Sr = fmaf(M.qsolpar, fabsf(R.w), M.solpar[tr]);
#pragma unroll
      for (int a = 0; a < kMaxTypes; ++a) {
        if (a < NT) {
          const int c = a * NT + tr;
          const float att = M.hb[c] ? ir10 : ir6;
          const float vdw = fminf(fmaf(M.A[c], ir12, -M.B[c] * att), M.e_cap);
          const float sv = fmaf(M.solpar[a], vr, Sr * M.vol[a]);
          T[a] += fmaf(sv, gs, vdw);
        }
      }
    }
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int a = 0; a < kMaxTypes; ++a)
    if (a < NT) M.maps[a * plane + node] = fminf(T[a], M.map_cap);
  M.maps[NT * plane + node] = fminf(fmaxf(E, -M.map_cap), M.map_cap);
  M.maps[(NT + 1) * plane + node] = fminf(D, M.map_cap);
}

hipError_t launch_build_maps(const MapBuild &m, hipStream_t s) {
  const int64_t plane = (int64_t)m.geom.nx * m.geom.ny * m.geom.nz;
  const unsigned blocks = (unsigned)((plane + kMapBlock - 1) / kMapBlock);
  hipLaunchKernelGGL(build_maps_kernel, dim3(blocks), dim3(kMapBlock), 0, s, m);
  return hipGetLastError();
}

}  // namespace dock

namespace dock {

// One thread per element of the packed grid; every type map plus the E/D record.
__global__ void relayout_kernel(MapGeom g, int32_t layout, const float *__restrict__ lin, void *types_out,
                                float4 *__restrict__ ed_out) {
  if (layout != kZPair && layout != kYZQuad) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int py = layout == kYZQuad ? ny - 1 : ny;
  const int64_t n_el = (int64_t)nx * py * (nz - 1);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_el) return;
  const int x = (int)(e % nx), y = (int)((e / nx) % py), z = (int)(e / ((int64_t)nx * py));
  const int64_t plane = (int64_t)nx * ny * nz;
  auto at = [&](int m, int xx, int yy, int zz) { return lin[m * plane + ((int64_t)zz * ny + yy) * nx + xx]; };
  const int E = g.n_types, D = g.n_types + 1;
  if (layout == kZPair) {
    float2 *T = (float2 *)types_out;
    for (int t = 0; t < g.n_types; ++t) T[t * n_el + e] = make_float2(at(t, x, y, z), at(t, x, y, z + 1));
    ed_out[e] = make_float4(at(E, x, y, z), at(E, x, y, z + 1), at(D, x, y, z), at(D, x, y, z + 1));
  } else {
    float4 *T = (float4 *)types_out;
    for (int t = 0; t < g.n_types; ++t)
      T[t * n_el + e] = make_float4(at(t, x, y, z), at(t, x, y + 1, z), at(t, x, y, z + 1), at(t, x, y + 1, z + 1));
    ed_out[2 * e] = make_float4(at(E, x, y, z), at(E, x, y + 1, z), at(E, x, y, z + 1), at(E, x, y + 1, z + 1));
    ed_out[2 * e + 1] = make_float4(at(D, x, y, z), at(D, x, y + 1, z), at(D, x, y, z + 1), at(D, x, y + 1, z + 1));
  }
}

// kQuadLine: one thread per quad slot of one map; it writes that slot of every
// map (types, then S+ = E + D and S- = E - D).  Slots past the row's last node
// (x >= nx in a row's last line) are zero and never read.
__global__ void relayout_lines_kernel(MapGeom g, int32_t nxb, int64_t t_stride, const float *__restrict__ lin,
                                      float4 *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= t_stride) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int slot = (int)(e % kLineQuads);
  const int64_t line = e / kLineQuads;
  const int k = (int)(line % nxb);
  const int y = (int)((line / nxb) % (ny - 1));
  const int z = (int)(line / ((int64_t)nxb * (ny - 1)));
  const int x = k * kLineCells + slot;
  const int64_t plane = (int64_t)nx * ny * nz;
  if (x >= nx) {
    for (int m = 0; m < g.n_types + 2; ++m) out[m * t_stride + e] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  auto quad = [&](int m) {
    const float *M = lin + m * plane;
    const int64_t o = ((int64_t)z * ny + y) * nx + x;
    return make_float4(M[o], M[o + nx], M[o + (int64_t)nx * ny], M[o + (int64_t)nx * ny + nx]);
  };
  for (int t = 0; t < g.n_types; ++t) out[t * t_stride + e] = quad(t);
  const float4 E = quad(g.n_types), D = quad(g.n_types + 1);
  out[g.n_types * t_stride + e] = make_float4(E.x + D.x, E.y + D.y, E.z + D.z, E.w + D.w);
  out[(g.n_types + 1) * t_stride + e] = make_float4(E.x - D.x, E.y - D.y, E.z - D.z, E.w - D.w);
}

// kPairLine: one thread per node slot of a line (slot j of line k is node
// x = kPairCells k + j); it writes that slot's type quad and signed quad in
// every (type, sign) copy.  Slots past the row's last node are zero and never
// read.  S+ and S- are rounded exactly as in kQuadLine, so the two layouts give
// the same energies.
__global__ void relayout_pairs_kernel(MapGeom g, int32_t nxb, int64_t t_stride, const float *__restrict__ lin,
                                      float4 *__restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // node slot index
  if (n >= t_stride / 2) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int slot = (int)(n % kPairNodes);
  const int64_t line = n / kPairNodes;
  const int k = (int)(line % nxb);
  const int y = (int)((line / nxb) % (ny - 1));
  const int z = (int)(line / ((int64_t)nxb * (ny - 1)));
  const int x = k * kPairCells + slot;
  const int64_t e = 2 * n;   // quad index of the slot's type quad within a copy
  const int64_t plane = (int64_t)nx * ny * nz;
  if (x >= nx) {
    for (int c = 0; c < 2 * g.n_types; ++c) {
      out[c * t_stride + e] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[c * t_stride + e + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  auto quad = [&](int m) {
    const float *M = lin + m * plane;
    const int64_t o = ((int64_t)z * ny + y) * nx + x;
    return make_float4(M[o], M[o + nx], M[o + (int64_t)nx * ny], M[o + (int64_t)nx * ny + nx]);
  };
  const float4 E = quad(g.n_types), D = quad(g.n_types + 1);
  const float4 Sp = make_float4(E.x + D.x, E.y + D.y, E.z + D.z, E.w + D.w);
  const float4 Sm = make_float4(E.x - D.x, E.y - D.y, E.z - D.z, E.w - D.w);
  for (int t = 0; t < g.n_types; ++t) {
    const float4 T = quad(t);
    out[(2 * t) * t_stride + e] = T;
    out[(2 * t) * t_stride + e + 1] = Sp;
    out[(2 * t + 1) * t_stride + e] = T;
    out[(2 * t + 1) * t_stride + e + 1] = Sm;
  }
}

hipError_t launch_relayout_pairs(const MapGeom &g, int32_t nxb, int64_t t_stride, const float *lin, float4 *out,
                                 hipStream_t s) {
  const int64_t nodes = t_stride / 2;
  hipLaunchKernelGGL(relayout_pairs_kernel, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s, g, nxb,
                     t_stride, lin, out);
  return hipGetLastError();
}

hipError_t launch_relayout_lines(const MapGeom &g, int32_t nxb, int64_t t_stride, const float *lin, float4 *out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(relayout_lines_kernel, dim3((unsigned)((t_stride + 255) / 256)), dim3(256), 0, s, g, nxb,
                     t_stride, lin, out);
  return hipGetLastError();
}

hipError_t launch_relayout(const MapGeom &g, int32_t layout, const float *lin, void *types_out, float4 *ed_out,
                           hipStream_t s) {
  if (layout != kZPair && layout != kYZQuad) return hipErrorInvalidValue;
  const int py = layout == kYZQuad ? g.ny - 1 : g.ny;
  const int64_t n_el = (int64_t)g.nx * py * (g.nz - 1);
  hipLaunchKernelGGL(relayout_kernel, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, s, g, layout, lin,
                     types_out, ed_out);
  return hipGetLastError();
}

}  // namespace dock
