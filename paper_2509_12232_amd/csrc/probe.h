// probe.h -- launchers of the roofline probes (measurement aids).
#pragma once
#include "dock_internal.h"

namespace dock {

// Lookups of the gather probe: rigid placements of one ligand's reference atoms,
// translation uniform in [lo, lo + ext], random orientation, random atom.
struct ProbeBox {
  float lo[3], ext[3];
};

hipError_t launch_gather_probe(const MapGeom &G, const MapData &M, int32_t layout, const LigandsDev &L,
                               int32_t lig, const ProbeBox &box, int64_t n_lanes, int32_t per_lane,
                               int32_t in_flight, uint32_t seed, float *out, hipStream_t s);
hipError_t launch_pair_probe(const FFConst &F, int64_t n_lanes, int32_t per_lane, float *out, hipStream_t s);

}  // namespace dock
