// dock_internal.h -- records shared by the host side of the library and its
// gfx950 kernels.  Everything the kernels read about a ligand is laid out so a
// wavefront can fetch it with scalar (uniform) loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dock {

constexpr int kMaxAtoms = 96;
constexpr int kMaxTorsions = 32;
constexpr int kMaxTypes = 32;
constexpr int kWave = 64;
constexpr int kBlock = kWave;   // poses per scoring block: one per lane
// A pose's energy is the sum of kParts partial sums, each accumulated in a
// fixed order and combined by a balanced tree; the 12-6 pair records come in
// groups of kParts, record u of a group belonging to partial sum u.
constexpr int kParts = 8;
constexpr int kMaxSplit = 8;    // wavefronts sharing a block of poses: 1, 2, 4 or 8

// Rows of kBlock floats a block of poses keeps in LDS besides its coordinate
// columns, when ws wavefronts share it: the energy reduction, one row each.
__host__ __device__ constexpr int block_extra_rows(int ws) { return ws > 1 ? ws : 0; }

// Per ligand.  Atoms are renumbered in depth-first pre-order from the root
// (atom 0), so every rotatable bond's moving fragment is one contiguous range.
// Pairs: the 12-6 pairs in groups of kParts (the last group padded with records
// whose coefficients are all zero, which contribute exactly 0), two further
// all-zero groups that the kernel may prefetch past the end, then the 12-10 pairs.
struct alignas(32) LigHeader {
  int32_t n_atoms;
  int32_t n_tors;
  int32_t n_groups;    // groups of kParts 12-6 pair records
  int32_t n_pairs_hb;  // 12-10 pairs, starting at hb_off
  int32_t atom_off;    // into atoms[] / atom_type[]
  int32_t tor_off;     // into tors[]
  int32_t pair_off;    // into pairs[]
  int32_t hb_off;      // into pairs[]
};

// Rotatable bond: axis from atom a (root side) to atom lo (the far atom, first of
// its fragment); the fragment is atoms [lo, hi).  gene = index of its angle in
// the genotype's torsion block.
struct alignas(16) TorRec {
  int32_t a, lo, hi, gene;
};

// Non-bonded pair with its precomputed coefficients (20 bytes, so the pair table
// of a typical ligand fits the scalar data cache).
struct PairRec {
  int32_t ij;    // i | j << 16
  float A, B;    // repulsive / attractive coefficients of the 12-6 or 12-10 term
  float qq;      // coulomb * q_i * q_j
  float sv;      // S_i vol_j + S_j vol_i
};
static_assert(sizeof(PairRec) == 20, "PairRec is five dwords");

struct MapGeom {
  int32_t nx, ny, nz, n_types;
  float ox, oy, oz, inv_h;
};

// Device layouts of the maps used by the scoring kernel.  The ABI layout is
// kept as is (kLinear); the packed layouts duplicate neighbouring nodes so that
// the eight corners of a cell come from fewer cache lines:
//   kZPair:  per type, float2 (M[x,y,z], M[x,y,z+1]) over z < nz-1; the x and
//            x+1 elements of a row are adjacent (16 B), so a cell needs two rows.
//            Electrostatic + desolvation as float4 (E, E_z+1, D, D_z+1).
//   kYZQuad: per type, float4 (M[x,y,z], M[x,y+1,z], M[x,y,z+1], M[x,y+1,z+1])
//            over y < ny-1, z < nz-1; a cell is the two adjacent elements x, x+1
//            (32 B).  Electrostatic + desolvation as two float4 quads per node.
//   kQuadLine: the yz-quads of kYZQuad cut into 128-byte lines of eight
//            x-consecutive quads, x = 7k .. 7k+7 in line k (consecutive lines
//            of a row share one quad), so the two quads of a cell never straddle
//            a line.  The electrostatic and desolvation maps are replaced by two
//            signed maps S+ = E + D and S- = E - D: since q E + |q| D equals
//            q S+ for q >= 0 and q S- for q < 0, one lookup reads a type quad pair
//            and one signed quad pair, exactly two cache lines.
//   kPairLine: one copy per (atom type, charge sign): node x of a row is its
//            type quad followed by its signed quad (32 B), four x-consecutive
//            nodes to a 128-byte line, x = 3k .. 3k+3 in line k, so a lookup
//            (both nodes of its cell, both quads of each) is 64 contiguous
//            bytes of one cache line.  2 n_types copies, about 14x the ABI maps.
enum MapLayout : int32_t { kLinear = 0, kZPair = 1, kYZQuad = 2, kQuadLine = 3, kPairLine = 4 };

// Quads per line of kQuadLine and the cells (x steps) a line covers.
constexpr int kLineQuads = 8;
constexpr int kLineCells = kLineQuads - 1;
// Nodes per line of kPairLine (two quads each) and the cells a line covers.
constexpr int kPairNodes = 4;
constexpr int kPairCells = kPairNodes - 1;

struct MapData {
  const float *lin;      // [n_types+2][nz][ny][nx]
  const float2 *tz;      // kZPair types:  [n_types][nz-1][ny][nx]
  const float4 *edz;     // kZPair E/D:    [nz-1][ny][nx]
  const float4 *tq;      // kYZQuad types: [n_types][nz-1][ny-1][nx]
  const float4 *edq;     // kYZQuad E/D:   [nz-1][ny-1][nx][2]
  const float4 *lq;      // kQuadLine:     [n_types + 2][nz-1][ny-1][nxb][kLineQuads], maps n_types and
                         //                n_types+1 are S+ and S-
  const float4 *pq;      // kPairLine:     [2 n_types][nz-1][ny-1][nxb][kPairNodes][2]: copy 2t + s
                         //                holds type t's quads and S+ (s = 0) or S- (s = 1)
  int64_t t_stride;      // elements (quads) per map (kPairLine: per copy) in the packed layout
  int32_t nxb;           // lines per (y, z) row: kQuadLine (nx - 2) / kLineCells + 1,
                         // kPairLine (nx - 2) / kPairCells + 1
};

struct FFConst {
  float e_cap, rmin2;
  float eps0, Ak;     // dielectric: 1/eps(r) = (1 + k e) / (eps0 + A k e), e = exp(-lambda B r)
  float k, diel_c;    // diel_c = -lambda * B * log2(e)
  float gauss_c;      // -log2(e) / (2 sigma^2)
  float pad;
};

struct LigandsDev {
  const LigHeader *hdr;
  const float4 *atoms;     // x, y, z (centred reference), charge
  const int32_t *atom_type;
  const TorRec *tors;
  const PairRec *pairs;
  int32_t n_ligs;
};

struct ScoreLaunch {
  LigandsDev L;
  MapGeom geom;
  FFConst ff;
  MapData maps;
  int32_t layout;
  const int32_t *pose_ligand;  // may be null
  int32_t poses_per_ligand;    // > 0: ligand = pose / poses_per_ligand (pose_ligand ignored)
  const float *genotypes;
  int32_t g_stride;
  int64_t n_poses;
  float *energies;
  int32_t lds_atoms;           // atom slots per pose in LDS
  int32_t split;               // wavefronts per block of 64 poses: 1, 2, 4 or 8
};

// Launchers (one translation unit per kernel family).
hipError_t launch_score(const ScoreLaunch &a, hipStream_t s);

}  // namespace dock

