// maps.h -- launch records of the grid-map builder.
#pragma once
#include "dock_internal.h"

namespace dock {

struct MapBuild {
  MapGeom geom;
  int32_t n_rec;
  const float4 *rec;       // x, y, z, charge
  const int32_t *rec_type;
  // per (probe type, receptor type): A, B and the 12-10 flag; per type: solpar, vol
  const float *A, *B;
  const int32_t *hb;
  const float *solpar, *vol;
  float qsolpar, coulomb, e_cap, map_cap, rmin2, h;
  FFConst ff;
  float *maps;
};

hipError_t launch_build_maps(const MapBuild &m, hipStream_t s);

// Derive a packed layout from the linear maps (buffers sized by the caller).
hipError_t launch_relayout(const MapGeom &g, int32_t layout, const float *lin, void *types_out, float4 *ed_out,
                           hipStream_t s);

// The kQuadLine copy: (n_types + 2) maps of t_stride quads, nxb lines per row.
hipError_t launch_relayout_lines(const MapGeom &g, int32_t nxb, int64_t t_stride, const float *lin, float4 *out,
                                 hipStream_t s);
// The kPairLine copy: 2 n_types copies of t_stride quads, nxb lines per row.
hipError_t launch_relayout_pairs(const MapGeom &g, int32_t nxb, int64_t t_stride, const float *lin, float4 *out,
                                 hipStream_t s);

}  // namespace dock
