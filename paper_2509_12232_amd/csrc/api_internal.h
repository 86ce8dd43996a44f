// api_internal.h -- host-side records shared by the translation units that
// implement the C ABI: error reporting, device scoping and the handle types.
#pragma once
#include <stdarg.h>

#include <mutex>
#include <string>
#include <vector>

#include "dock.h"
#include "dock_internal.h"

// Sets the calling thread's error message and returns st.
dock_status set_err(dock_status st, const char *fmt, ...);
// Maps a HIP error to DOCK_E_NOMEM / DOCK_E_DEVICE with the failing step's name.
dock_status hip_err(hipError_t e, const char *what);

// Stream-ordered scratch from the library's own memory pool of the current
// device.  The pool keeps freed memory (its release threshold is unlimited), so
// repeated calls reuse their scratch instead of mapping it again; it lives
// until the process ends.  Free with hipFreeAsync on a stream.
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s);

#define HIP_TRY(expr, what)                  \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return hip_err(e_, what); \
  } while (0)

namespace dock {

// Makes `device` current for the scope of an API call.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int device) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != device) err = hipSetDevice(device);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  *dst = nullptr;
  if (src.empty()) return hipMalloc((void **)dst, sizeof(T));  // keep a valid pointer
  hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace dock

struct dock_pocket {
  int device = 0;
  dock::MapGeom geom{};
  dock::FFConst ffc{};
  int n_types = 0;
  std::vector<float> Rii, epsii, vol, solpar;
  std::vector<uint8_t> hbond;
  float coulomb = 0, qsolpar = 0;
  float *maps = nullptr;      // ABI layout
  int64_t plane = 0;
  int32_t layout = dock::kLinear;    // layout the scoring kernel reads
  int32_t n_cu = 1;            // compute units of the device (persistent launch size)
  std::string arch;            // device architecture name (keys the autotuner's cache)
  void *tpack = nullptr;       // packed type maps (kQuadLine, kPairLine: all maps)
  float4 *edpack = nullptr;    // packed electrostatic/desolvation records
  int64_t t_stride = 0;
  int32_t nxb = 0;
  dock::MapData view() const {
    dock::MapData m{};
    m.lin = maps;
    m.t_stride = t_stride;
    m.nxb = nxb;
    if (layout == dock::kZPair) m.tz = (const float2 *)tpack, m.edz = edpack;
    if (layout == dock::kYZQuad) m.tq = (const float4 *)tpack, m.edq = edpack;
    if (layout == dock::kQuadLine) m.lq = (const float4 *)tpack;
    if (layout == dock::kPairLine) m.pq = (const float4 *)tpack;
    return m;
  }
};

// Ligands with (previous bucket's upper, upper] atoms: order[offset .. offset + count).
struct LigandBucket {
  int32_t upper;      // atom-count bound of the bucket
  int32_t lds_atoms;  // largest ligand actually in it (sizes the LDS of its launch)
  int32_t offset, count;
  int32_t split;           // launch shape of its search kernel: wavefronts per block of 64 poses
  int32_t blocks;          // blocks per workgroup (0: chosen at launch)
  int32_t fixed;           // 1: shape set by the caller or the autotuner
  int64_t cost;            // sum of atoms + pairs over its ligands (work estimate)
};

struct dock_ligands {
  int device = 0;
  int n_ligs = 0;
  int max_atoms = 0, max_tors = 0;
  int32_t layout = dock::kLinear;   // map layout of the pocket the set was created for
  std::vector<dock::LigHeader> hdr_host;
  std::vector<int32_t> pair_count;
  dock::LigHeader *hdr = nullptr;
  float4 *atoms = nullptr;
  int32_t *atom_type = nullptr;
  dock::TorRec *tors = nullptr;
  dock::PairRec *pairs = nullptr;
  // ligands grouped by atom count; within a group, costliest first
  std::vector<LigandBucket> buckets;
  int32_t *order = nullptr;
  float *desc = nullptr;  // [n_ligs][64] descriptor features (learned proposal)
  // side streams for concurrent bucket launches (created on first use)
  mutable std::mutex side_mu;
  mutable std::vector<hipStream_t> side;
  // Three side streams: with the caller's stream, one for each of the four
  // hardware queues the HIP runtime gives a process by default.  With more
  // streams than queues, two streams share a queue and run in order, and which
  // two is up to the runtime (measured on MI355X: with four side streams the
  // 1000-ligand search took 57 ms eagerly against 46 ms with three or five).
  static constexpr size_t kSideStreams = 3;
  hipError_t ensure_side_streams() const {
    while (side.size() < kSideStreams) {
      hipStream_t st = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
      side.push_back(st);
    }
    return hipSuccess;
  }
  dock::LigandsDev view() const { return dock::LigandsDev{hdr, atoms, atom_type, tors, pairs, n_ligs}; }
};

// ------------------------------------------------------------ learned proposal
#include "learn.h"

// Rows of a population [n_ligs][pop][g_stride] of L with translation box lo..hi.
dock::PopRows make_pop_rows(const dock_ligands *L, int32_t pop, int32_t g_stride, const double lo[3],
                            const double hi[3]);
// proposals = dock_propose's proposals of population (rows R), enqueued on s.
hipError_t run_proposals(const dock_mlp *net, const dock::PopRows &R, float alpha_max, uint64_t seed,
                         int32_t generation, const float *population, float *proposals, hipStream_t s);
int mlp_device(const dock_mlp *net);
