// api.hip -- host side of the C ABI declared in include/dock.h: argument
// validation, ligand preprocessing, device memory ownership and kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <numeric>
#include <vector>

#include "api_internal.h"
#include "maps.h"
#include "search.h"
#include "probe.h"

using namespace dock;

// ------------------------------------------------------------------------------ errors
static thread_local char g_err[512];

dock_status set_err(dock_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

dock_status hip_err(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) return set_err(DOCK_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_err(DOCK_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *dock_last_error(void) { return g_err; }

hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s) {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = pools.find(device);
    if (it != pools.end()) {
      pool = it->second;
    } else {
      hipMemPoolProps props{};
      props.allocType = hipMemAllocationTypePinned;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = device;
      e = hipMemPoolCreate(&pool, &props);
      if (e != hipSuccess) return e;
      uint64_t keep = UINT64_MAX;
      e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return e;
      }
      pools[device] = pool;
    }
  }
  return hipMallocFromPoolAsync(p, bytes, pool, s);
}
extern "C" int32_t dock_version(void) { return 2; }

// ------------------------------------------------------------------------------ handles
// Packed layout for the scoring kernel: the pair-line layout (one cache line
// per lookup, about 14x the ABI maps) while its copy stays within kPairBudget
// bytes; else the quad-line layout (two lines per lookup, about 4.6x) within
// kQuadBudget; else the z-pair layout (2x).  Random lookups are bound by the
// lines in flight per CU, so halving the lines per lookup outweighs the pair-line
// copy outgrowing the 256 MB Infinity Cache (measured on MI355X with fourteen
// 100^3 maps: 58 against 37 G lookups/s).
static constexpr double kPairBudget = 8.0 * 1024 * 1024 * 1024;
static constexpr double kQuadBudget = 512.0 * 1024 * 1024;

static int64_t line_blocks(const MapGeom &g) { return (g.nx - 2) / kLineCells + 1; }
static int64_t line_stride(const MapGeom &g) {
  return (int64_t)(g.nz - 1) * (g.ny - 1) * line_blocks(g) * kLineQuads;
}
static int64_t pair_blocks(const MapGeom &g) { return (g.nx - 2) / kPairCells + 1; }
static int64_t pair_stride(const MapGeom &g) {
  return (int64_t)(g.nz - 1) * (g.ny - 1) * pair_blocks(g) * (2 * kPairNodes);
}
// Largest element index of one map (or copy) of each line layout, which the
// gather computes in 32 bits.
static double line_elements(const int32_t dims[3]) {
  return (double)(dims[2] - 1) * (dims[1] - 1) * ((dims[0] - 2) / kLineCells + 1) * kLineQuads;
}
static double pair_elements(const int32_t dims[3]) {
  return (double)(dims[2] - 1) * (dims[1] - 1) * ((dims[0] - 2) / kPairCells + 1) * (2 * kPairNodes);
}

static int32_t choose_layout(const MapGeom &g, int32_t requested) {
  if (requested != DOCK_LAYOUT_AUTO) return requested;
  const int32_t dims[3] = {g.nx, g.ny, g.nz};
  const double pair_bytes = (double)pair_stride(g) * 16.0 * (2 * g.n_types);
  if (pair_bytes <= kPairBudget && pair_elements(dims) <= 2147483647.0) return kPairLine;
  const double bytes = (double)line_stride(g) * 16.0 * (g.n_types + 2);
  return bytes <= kQuadBudget ? kQuadLine : kZPair;
}

static bool valid_layout(int32_t layout) {
  return layout == DOCK_LAYOUT_AUTO || layout == DOCK_LAYOUT_LINEAR || layout == DOCK_LAYOUT_ZPAIR ||
         layout == DOCK_LAYOUT_YZQUAD || layout == DOCK_LAYOUT_QUADLINE || layout == DOCK_LAYOUT_PAIRLINE;
}

// Builds the packed copy of p->maps (already on the device).
static hipError_t pack_maps(dock_pocket *p, int32_t requested) {
  p->layout = choose_layout(p->geom, requested);
  if (p->layout == kPairLine) {
    p->nxb = (int32_t)pair_blocks(p->geom);
    p->t_stride = pair_stride(p->geom);
    hipError_t e = hipMalloc(&p->tpack, (size_t)p->t_stride * 16 * (2 * p->geom.n_types));
    if (e == hipSuccess)
      e = launch_relayout_pairs(p->geom, p->nxb, p->t_stride, p->maps, (float4 *)p->tpack, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    return e;
  }
  if (p->layout == kQuadLine) {
    p->nxb = (int32_t)line_blocks(p->geom);
    p->t_stride = line_stride(p->geom);
    hipError_t e = hipMalloc(&p->tpack, (size_t)p->t_stride * 16 * (p->geom.n_types + 2));
    if (e == hipSuccess)
      e = launch_relayout_lines(p->geom, p->nxb, p->t_stride, p->maps, (float4 *)p->tpack, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    return e;
  }
  if (p->layout != kZPair && p->layout != kYZQuad) return hipSuccess;  // kLinear reads p->maps directly
  const MapGeom &g = p->geom;
  const int py = p->layout == kYZQuad ? g.ny - 1 : g.ny;
  const int64_t n_el = (int64_t)g.nx * py * (g.nz - 1);
  const size_t tbytes = (size_t)n_el * g.n_types * (p->layout == kYZQuad ? 16 : 8);
  const size_t edbytes = (size_t)n_el * (p->layout == kYZQuad ? 32 : 16);
  p->t_stride = n_el;
  hipError_t e = hipMalloc(&p->tpack, tbytes);
  if (e == hipSuccess) e = hipMalloc((void **)&p->edpack, edbytes);
  if (e == hipSuccess) e = launch_relayout(g, p->layout, p->maps, p->tpack, p->edpack, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  return e;
}

static void free_pocket(dock_pocket *p) {
  for (void *q : {(void *)p->maps, p->tpack, (void *)p->edpack})
    if (q) (void)hipFree(q);
  delete p;
}

// ------------------------------------------------------------------------------ pockets
static dock_status check_ff(const dock_forcefield *ff) {
  if (!ff) return set_err(DOCK_E_INVALID, "null force field");
  if (ff->n_types < 1 || ff->n_types > kMaxTypes)
    return set_err(DOCK_E_INVALID, "n_types must be in 1..%d", kMaxTypes);
  if (!ff->Rii || !ff->epsii || !ff->vol || !ff->solpar || !ff->hbond)
    return set_err(DOCK_E_INVALID, "null force-field array");
  for (int t = 0; t < ff->n_types; ++t)
    if (!(isfinite(ff->Rii[t]) && isfinite(ff->epsii[t]) && ff->epsii[t] >= 0 && isfinite(ff->vol[t]) &&
          isfinite(ff->solpar[t])))
      return set_err(DOCK_E_INVALID, "non-finite or negative force-field entry for type %d", t);
  for (int a = 0; a < ff->n_types; ++a)
    for (int b = 0; b < ff->n_types; ++b)
      if (ff->hbond[a * ff->n_types + b] > 1 || ff->hbond[a * ff->n_types + b] != ff->hbond[b * ff->n_types + a])
        return set_err(DOCK_E_INVALID, "hbond table must be symmetric 0/1");
  if (!(ff->sigma > 0) || !(ff->r_min > 0) || !(ff->e_cap > 0) || !isfinite(ff->e_cap) || !isfinite(ff->coulomb) ||
      !isfinite(ff->diel_A) || !isfinite(ff->diel_eps0) || !isfinite(ff->diel_lambda) || !isfinite(ff->diel_k) ||
      !isfinite(ff->qsolpar) || !(ff->map_cap > 0))
    return set_err(DOCK_E_INVALID, "bad force-field constant");
  return DOCK_OK;
}

static dock_status check_grid(const dock_grid *g, int n_types, int32_t layout) {
  if (!g) return set_err(DOCK_E_INVALID, "null grid");
  if (g->n_types != n_types) return set_err(DOCK_E_INVALID, "grid n_types %d != force field %d", g->n_types, n_types);
  for (int d = 0; d < 3; ++d)
    if (g->dims[d] < 2) return set_err(DOCK_E_INVALID, "grid dims must be >= 2");
  if (!(g->spacing > 0) || !isfinite(g->spacing)) return set_err(DOCK_E_INVALID, "spacing must be > 0");
  for (int d = 0; d < 3; ++d)
    if (!isfinite(g->origin[d])) return set_err(DOCK_E_INVALID, "non-finite origin");
  const double total = (double)g->dims[0] * g->dims[1] * g->dims[2] * (n_types + 2);
  if (total > 2147483647.0) return set_err(DOCK_E_INVALID, "maps larger than 2^31 values");
  // the line layouts' gathers index one map (or copy) with 32-bit element indices
  if (layout == DOCK_LAYOUT_QUADLINE && line_elements(g->dims) > 2147483647.0)
    return set_err(DOCK_E_INVALID, "grid too large for the quad-line layout");
  if (layout == DOCK_LAYOUT_PAIRLINE && pair_elements(g->dims) > 2147483647.0)
    return set_err(DOCK_E_INVALID, "grid too large for the pair-line layout");
  return DOCK_OK;
}

static void fill_pocket_ff(dock_pocket *p, const dock_forcefield *ff) {
  const int nt = ff->n_types;
  p->n_types = nt;
  p->Rii.assign(ff->Rii, ff->Rii + nt);
  p->epsii.assign(ff->epsii, ff->epsii + nt);
  p->vol.assign(ff->vol, ff->vol + nt);
  p->solpar.assign(ff->solpar, ff->solpar + nt);
  p->hbond.assign(ff->hbond, ff->hbond + nt * nt);
  p->coulomb = ff->coulomb;
  p->qsolpar = ff->qsolpar;
  const double LOG2E = 1.4426950408889634;
  const double B = (double)ff->diel_eps0 - ff->diel_A;
  FFConst &c = p->ffc;
  c.e_cap = ff->e_cap;
  c.rmin2 = (float)((double)ff->r_min * ff->r_min);
  c.eps0 = ff->diel_eps0;
  c.Ak = (float)((double)ff->diel_A * ff->diel_k);
  c.k = ff->diel_k;
  c.diel_c = (float)(-(double)ff->diel_lambda * B * LOG2E);
  c.gauss_c = (float)(-LOG2E / (2.0 * (double)ff->sigma * ff->sigma));
  c.pad = 0;
}

static hipError_t fill_device_info(dock_pocket *p) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, p->device);
  if (e == hipSuccess) {
    p->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    // the architecture name without its feature suffixes (gfx950:sramecc+:xnack- -> gfx950)
    std::string arch(prop.gcnArchName);
    p->arch = arch.substr(0, arch.find(':'));
    if (p->arch.empty()) p->arch = "unknown";
  }
  return e;
}

static void fill_geom(dock_pocket *p, const dock_grid *g) {
  p->geom = MapGeom{g->dims[0], g->dims[1], g->dims[2], g->n_types, g->origin[0], g->origin[1], g->origin[2],
                    (float)(1.0 / (double)g->spacing)};
  p->plane = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
}

extern "C" dock_status dock_create_pocket(const dock_grid *grid, const float *maps, int32_t maps_on_device,
                                          const dock_forcefield *ff, int32_t layout, int32_t device,
                                          dock_pocket **out) {
  if (!out) return set_err(DOCK_E_INVALID, "null out");
  *out = nullptr;
  if (!valid_layout(layout)) return set_err(DOCK_E_INVALID, "unknown layout %d", layout);
  dock_status st = check_ff(ff);
  if (st) return st;
  if ((st = check_grid(grid, ff->n_types, layout))) return st;
  if (!maps) return set_err(DOCK_E_INVALID, "null maps");
  DeviceScope ds(device);
  HIP_TRY(ds.err, "hipSetDevice");
  dock_pocket *p = new dock_pocket();
  p->device = device;
  fill_pocket_ff(p, ff);
  fill_geom(p, grid);
  const size_t bytes = sizeof(float) * p->plane * (ff->n_types + 2);
  hipError_t e = fill_device_info(p);
  if (e == hipSuccess) e = hipMalloc((void **)&p->maps, bytes);
  if (e == hipSuccess)
    e = hipMemcpy(p->maps, maps, bytes, maps_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  if (e == hipSuccess) e = pack_maps(p, layout);
  if (e != hipSuccess) {
    free_pocket(p);
    return hip_err(e, "pocket maps");
  }
  *out = p;
  return DOCK_OK;
}

extern "C" dock_status dock_create_pocket_from_receptor(const dock_grid *grid, const dock_forcefield *ff,
                                                        int32_t n_atoms, const float *xyz, const int32_t *type,
                                                        const float *charge, int32_t layout, int32_t device,
                                                        dock_pocket **out) {
  if (!out) return set_err(DOCK_E_INVALID, "null out");
  *out = nullptr;
  if (!valid_layout(layout)) return set_err(DOCK_E_INVALID, "unknown layout %d", layout);
  dock_status st = check_ff(ff);
  if (st) return st;
  if ((st = check_grid(grid, ff->n_types, layout))) return st;
  if (n_atoms < 0 || (n_atoms > 0 && (!xyz || !type || !charge)))
    return set_err(DOCK_E_INVALID, "bad receptor arrays");
  const int nt = ff->n_types;
  std::vector<float4> rec(n_atoms);
  std::vector<int32_t> rt(type, type + n_atoms);
  for (int i = 0; i < n_atoms; ++i) {
    if (type[i] < 0 || type[i] >= nt) return set_err(DOCK_E_INVALID, "receptor atom %d type out of range", i);
    rec[i] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], charge[i]);
  }
  std::vector<float> A(nt * nt), B(nt * nt);
  std::vector<int32_t> hb(nt * nt);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      const double req = 0.5 * ((double)ff->Rii[a] + ff->Rii[b]);
      const double eps = sqrt((double)ff->epsii[a] * ff->epsii[b]);
      const bool h = ff->hbond[a * nt + b] != 0;
      A[a * nt + b] = (float)((h ? 5.0 : 1.0) * eps * pow(req, 12));
      B[a * nt + b] = (float)((h ? 6.0 : 2.0) * eps * pow(req, h ? 10 : 6));
      hb[a * nt + b] = h;
    }
  DeviceScope ds(device);
  HIP_TRY(ds.err, "hipSetDevice");
  dock_pocket *p = new dock_pocket();
  p->device = device;
  fill_pocket_ff(p, ff);
  fill_geom(p, grid);
  float4 *d_rec = nullptr;
  int32_t *d_rt = nullptr, *d_hb = nullptr;
  float *d_A = nullptr, *d_B = nullptr, *d_sol = nullptr, *d_vol = nullptr;
  hipError_t e = fill_device_info(p);
  if (e == hipSuccess) e = upload(&d_rec, rec);
  if (e == hipSuccess) e = upload(&d_rt, rt);
  if (e == hipSuccess) e = upload(&d_A, A);
  if (e == hipSuccess) e = upload(&d_B, B);
  if (e == hipSuccess) e = upload(&d_hb, hb);
  if (e == hipSuccess) e = upload(&d_sol, p->solpar);
  if (e == hipSuccess) e = upload(&d_vol, p->vol);
  if (e == hipSuccess) e = hipMalloc((void **)&p->maps, sizeof(float) * p->plane * (nt + 2));
  if (e == hipSuccess) {
    MapBuild m{};
    m.geom = p->geom;
    m.n_rec = n_atoms;
    m.rec = d_rec;
    m.rec_type = d_rt;
    m.A = d_A;
    m.B = d_B;
    m.hb = d_hb;
    m.solpar = d_sol;
    m.vol = d_vol;
    m.qsolpar = ff->qsolpar;
    m.coulomb = ff->coulomb;
    m.e_cap = ff->e_cap;
    m.map_cap = ff->map_cap;
    m.rmin2 = p->ffc.rmin2;
    m.h = grid->spacing;
    m.ff = p->ffc;
    m.maps = p->maps;
    e = launch_build_maps(m, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = pack_maps(p, layout);
  }
  for (void *q : {(void *)d_rec, (void *)d_rt, (void *)d_A, (void *)d_B, (void *)d_hb, (void *)d_sol, (void *)d_vol})
    if (q) (void)hipFree(q);
  if (e != hipSuccess) {
    free_pocket(p);
    return hip_err(e, "map build");
  }
  *out = p;
  return DOCK_OK;
}

extern "C" dock_status dock_pocket_maps(const dock_pocket *p, float *maps_out, void *stream) {
  if (!p || !maps_out) return set_err(DOCK_E_INVALID, "null argument");
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(maps_out, p->maps, sizeof(float) * p->plane * (p->n_types + 2), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream),
          "copy maps");
  return DOCK_OK;
}

extern "C" dock_status dock_pocket_layout(const dock_pocket *p, int32_t *layout) {
  if (!p || !layout) return set_err(DOCK_E_INVALID, "null argument");
  *layout = p->layout;
  return DOCK_OK;
}

extern "C" dock_status dock_destroy_pocket(dock_pocket *p) {
  if (!p) return DOCK_OK;
  DeviceScope ds(p->device);
  free_pocket(p);
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ ligands
namespace {

struct PrepOut {
  std::vector<float4> atoms;
  std::vector<int32_t> types;
  std::vector<TorRec> tors;
  std::vector<PairRec> pairs;  // 12-6 groups, two spare zero groups, then 12-10 pairs
  int n_plain = 0, n_hb = 0, n_groups = 0;
  float desc[64];  // descriptor features of the learned proposal
};

// Root at atom 0; depth-first pre-order renumbering so each rotatable bond's far
// side is one index range; rigid fragments; pairs >= 4 bonds apart across
// fragments; per-pair coefficients.
dock_status prep_ligand(const dock_pocket *P, const dock_ligand_desc &d, int lig, PrepOut &o) {
  const int n = d.n_atoms, nt = d.n_torsions;
  if (n < 1) return set_err(DOCK_E_INVALID, "ligand %d: n_atoms must be >= 1", lig);
  if (n > kMaxAtoms) return set_err(DOCK_E_UNSUPPORTED, "ligand %d: %d atoms > %d", lig, n, kMaxAtoms);
  if (nt < 0) return set_err(DOCK_E_INVALID, "ligand %d: negative n_torsions", lig);
  if (nt > kMaxTorsions) return set_err(DOCK_E_UNSUPPORTED, "ligand %d: %d torsions > %d", lig, nt, kMaxTorsions);
  if (nt > n - 1) return set_err(DOCK_E_INVALID, "ligand %d: more torsions than bonds", lig);
  if (!d.xyz || !d.type || !d.charge || (n > 1 && !d.bonds) || (nt > 0 && !d.torsion_bonds))
    return set_err(DOCK_E_INVALID, "ligand %d: null array", lig);
  for (int i = 0; i < n; ++i) {
    if (d.type[i] < 0 || d.type[i] >= P->n_types) return set_err(DOCK_E_INVALID, "ligand %d: atom type out of range", lig);
    if (!isfinite(d.xyz[3 * i]) || !isfinite(d.xyz[3 * i + 1]) || !isfinite(d.xyz[3 * i + 2]) || !isfinite(d.charge[i]))
      return set_err(DOCK_E_INVALID, "ligand %d: non-finite coordinate or charge", lig);
  }
  // n - 1 distinct bonds form a tree exactly when none of them closes a cycle
  // (union-find); a repeated bond is invalid, a cycle is a ring
  std::vector<std::vector<int>> adj(n);
  {
    std::vector<int> comp(n);
    std::iota(comp.begin(), comp.end(), 0);
    auto find = [&](int x) {
      while (comp[x] != x) x = comp[x] = comp[comp[x]];
      return x;
    };
    for (int k = 0; k < n - 1; ++k) {
      const int a = d.bonds[2 * k], b = d.bonds[2 * k + 1];
      if (a < 0 || a >= n || b < 0 || b >= n || a == b)
        return set_err(DOCK_E_INVALID, "ligand %d: bad bond %d", lig, k);
      if (std::find(adj[a].begin(), adj[a].end(), b) != adj[a].end())
        return set_err(DOCK_E_INVALID, "ligand %d: repeated bond %d", lig, k);
      const int ra = find(a), rb = find(b);
      if (ra == rb)
        return set_err(DOCK_E_UNSUPPORTED, "ligand %d: the bonds close a ring (rings are not supported)", lig);
      comp[ra] = rb;
      adj[a].push_back(b);
      adj[b].push_back(a);
    }
  }
  // depth-first pre-order from the root
  std::vector<int> parent(n, -1), order, pos(n, -1), size(n, 1);
  order.reserve(n);
  {
    std::vector<int> stack{0};
    pos[0] = 0;
    std::vector<char> seen(n, 0);
    seen[0] = 1;
    while (!stack.empty()) {
      const int u = stack.back();
      stack.pop_back();
      pos[u] = (int)order.size();
      order.push_back(u);
      for (int k = (int)adj[u].size() - 1; k >= 0; --k) {
        const int v = adj[u][k];
        if (v == parent[u]) continue;
        if (seen[v]) return set_err(DOCK_E_UNSUPPORTED, "ligand %d: the bonds close a ring (rings are not supported)", lig);
        seen[v] = 1;
        parent[v] = u;
        stack.push_back(v);
      }
    }
    if ((int)order.size() != n) return set_err(DOCK_E_INVALID, "ligand %d: bonds do not form a tree", lig);
    for (int k = n - 1; k > 0; --k) size[parent[order[k]]] += size[order[k]];
  }
  // rotatable bonds
  std::vector<char> rot(n > 1 ? n - 1 : 1, 0);
  o.tors.clear();
  for (int k = 0; k < nt; ++k) {
    const int bi = d.torsion_bonds[k];
    if (bi < 0 || bi >= n - 1) return set_err(DOCK_E_INVALID, "ligand %d: torsion bond index out of range", lig);
    if (rot[bi]) return set_err(DOCK_E_INVALID, "ligand %d: repeated torsion bond", lig);
    rot[bi] = 1;
    int a = d.bonds[2 * bi], b = d.bonds[2 * bi + 1];
    if (adj[a].size() < 2 || adj[b].size() < 2)
      return set_err(DOCK_E_INVALID, "ligand %d: torsion on a terminal bond", lig);
    if (parent[a] == b) std::swap(a, b);  // a on the root side
    o.tors.push_back(TorRec{pos[a], pos[b], pos[b] + size[b], k});
  }
  // rigid fragments (union-find over the non-rotatable bonds)
  std::vector<int> uf(n);
  std::iota(uf.begin(), uf.end(), 0);
  auto find = [&](int x) {
    while (uf[x] != x) x = uf[x] = uf[uf[x]];
    return x;
  };
  for (int k = 0; k < n - 1; ++k)
    if (!rot[k]) uf[find(d.bonds[2 * k])] = find(d.bonds[2 * k + 1]);
  // bond-graph distances
  std::vector<int> dist((size_t)n * n, -1), q(n);
  for (int s = 0; s < n; ++s) {
    int *ds = &dist[(size_t)s * n];
    int h = 0, t = 0;
    ds[s] = 0;
    q[t++] = s;
    while (h < t) {
      const int u = q[h++];
      for (int v : adj[u])
        if (ds[v] < 0) ds[v] = ds[u] + 1, q[t++] = v;
    }
  }
  // centred reference conformation, in the new order
  double c[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) c[k] += d.xyz[3 * i + k];
  for (int k = 0; k < 3; ++k) c[k] /= n;
  o.atoms.resize(n);
  o.types.resize(n);
  for (int i = 0; i < n; ++i) {
    const int u = order[i];
    o.atoms[i] = make_float4((float)(d.xyz[3 * u] - c[0]), (float)(d.xyz[3 * u + 1] - c[1]),
                             (float)(d.xyz[3 * u + 2] - c[2]), d.charge[u]);
    o.types[i] = d.type[u];
  }
  // pairs with coefficients (computed in binary64, stored as float)
  std::vector<PairRec> plain, hb;
  for (int u = 0; u < n; ++u)
    for (int v = u + 1; v < n; ++v) {
      if (dist[(size_t)u * n + v] < 4 || find(u) == find(v)) continue;
      const int tu = d.type[u], tv = d.type[v];
      const double req = 0.5 * ((double)P->Rii[tu] + P->Rii[tv]);
      const double eps = sqrt((double)P->epsii[tu] * P->epsii[tv]);
      const bool h = P->hbond[tu * P->n_types + tv] != 0;
      const double A = (h ? 5.0 : 1.0) * eps * pow(req, 12);
      const double B = (h ? 6.0 : 2.0) * eps * pow(req, h ? 10 : 6);
      const double qu = d.charge[u], qv = d.charge[v];
      const double Su = (double)P->solpar[tu] + (double)P->qsolpar * fabs(qu);
      const double Sv = (double)P->solpar[tv] + (double)P->qsolpar * fabs(qv);
      PairRec r{};
      r.ij = std::min(pos[u], pos[v]) | (std::max(pos[u], pos[v]) << 16);
      r.A = (float)A;
      r.B = (float)B;
      r.qq = (float)((double)P->coulomb * qu * qv);
      r.sv = (float)(Su * P->vol[tv] + Sv * P->vol[tu]);
      (h ? hb : plain).push_back(r);
    }
  // sort by (i, j); ij packs i in the low half, so compare the halves explicitly
  auto by_ij = [](const PairRec &x, const PairRec &y) {
    const int xi = x.ij & 0xffff, yi = y.ij & 0xffff;
    return xi != yi ? xi < yi : (x.ij >> 16) < (y.ij >> 16);
  };
  std::sort(plain.begin(), plain.end(), by_ij);
  std::sort(hb.begin(), hb.end(), by_ij);
  o.n_plain = (int)plain.size();
  o.n_hb = (int)hb.size();
  o.n_groups = (o.n_plain + kParts - 1) / kParts;
  // 12-6 pairs padded to whole groups of kParts, two spare all-zero groups, then 12-10 pairs
  o.pairs = plain;
  o.pairs.resize((size_t)kParts * (o.n_groups + 2), PairRec{0, 0.f, 0.f, 0.f, 0.f});
  o.pairs.insert(o.pairs.end(), hb.begin(), hb.end());
  // descriptor: type fractions, torsion and atom counts, charge statistics,
  // radius of gyration of the reference conformation, pair count
  double f[64] = {0};
  double rg2 = 0, qa = 0, qs = 0;
  for (int i = 0; i < n; ++i) {
    f[d.type[i]] += 1.0 / n;
    qa += fabs((double)d.charge[i]);
    qs += d.charge[i];
    for (int k = 0; k < 3; ++k) {
      const double x = d.xyz[3 * i + k] - c[k];
      rg2 += x * x;
    }
  }
  f[32] = nt / 20.0;
  f[33] = n / 96.0;
  f[34] = qa / n;
  f[35] = qs / n;
  f[36] = sqrt(rg2 / n) / 10.0;
  f[37] = (o.n_plain + o.n_hb) / 4096.0;
  for (int j = 0; j < 64; ++j) o.desc[j] = (float)f[j];
  return DOCK_OK;
}

}  // namespace

static void free_ligands(dock_ligands *L) {
  for (hipStream_t st : L->side) (void)hipStreamDestroy(st);
  for (void *q : {(void *)L->hdr, (void *)L->atoms, (void *)L->atom_type, (void *)L->tors, (void *)L->pairs,
                  (void *)L->order, (void *)L->desc})
    if (q) (void)hipFree(q);
  delete L;
}

extern "C" dock_status dock_create_ligands(const dock_pocket *pocket, const dock_ligand_desc *ligands,
                                           int32_t n_ligands, dock_ligands **out) {
  if (!out) return set_err(DOCK_E_INVALID, "null out");
  *out = nullptr;
  if (!pocket || !ligands) return set_err(DOCK_E_INVALID, "null argument");
  if (n_ligands < 1) return set_err(DOCK_E_INVALID, "n_ligands must be >= 1");
  std::vector<LigHeader> hdr(n_ligands);
  std::vector<int32_t> pair_count(n_ligands);
  std::vector<float4> atoms;
  std::vector<int32_t> types;
  std::vector<TorRec> tors;
  std::vector<PairRec> pairs;
  std::vector<float> desc;
  int max_atoms = 1, max_tors = 0;
  PrepOut o;
  for (int l = 0; l < n_ligands; ++l) {
    dock_status st = prep_ligand(pocket, ligands[l], l, o);
    if (st) return st;
    LigHeader &h = hdr[l];
    h.n_atoms = (int)o.atoms.size();
    h.n_tors = (int)o.tors.size();
    h.n_groups = o.n_groups;
    h.n_pairs_hb = o.n_hb;
    h.atom_off = (int)atoms.size();
    h.tor_off = (int)tors.size();
    h.pair_off = (int)pairs.size();
    h.hb_off = h.pair_off + kParts * (o.n_groups + 2);
    pair_count[l] = o.n_plain + o.n_hb;
    if ((double)pairs.size() + o.pairs.size() > 2.0e9) return set_err(DOCK_E_UNSUPPORTED, "ligand set too large");
    atoms.insert(atoms.end(), o.atoms.begin(), o.atoms.end());
    types.insert(types.end(), o.types.begin(), o.types.end());
    tors.insert(tors.end(), o.tors.begin(), o.tors.end());
    pairs.insert(pairs.end(), o.pairs.begin(), o.pairs.end());
    desc.insert(desc.end(), o.desc, o.desc + 64);
    max_atoms = std::max(max_atoms, h.n_atoms);
    max_tors = std::max(max_tors, h.n_tors);
  }
  DeviceScope ds(pocket->device);
  HIP_TRY(ds.err, "hipSetDevice");
  dock_ligands *L = new dock_ligands();
  L->device = pocket->device;
  L->layout = pocket->layout;
  L->n_ligs = n_ligands;
  L->max_atoms = max_atoms;
  L->max_tors = max_tors;
  L->hdr_host = hdr;
  L->pair_count = pair_count;
  // size buckets for the search launches (LDS is sized per bucket); the work of a
  // ligand's search grows with atoms + pairs, and the costliest go first
  std::vector<int32_t> order;
  int lo = 0;
  for (int ub : {16, 32, 48, 64, kMaxAtoms}) {
    std::vector<int32_t> ids;
    for (int l = 0; l < n_ligands; ++l)
      if (hdr[l].n_atoms > lo && hdr[l].n_atoms <= ub) ids.push_back(l);
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
      return hdr[x].n_atoms + pair_count[x] > hdr[y].n_atoms + pair_count[y];
    });
    int mx = 1;
    int64_t cost = 0;
    for (int32_t l : ids) mx = std::max(mx, hdr[l].n_atoms), cost += hdr[l].n_atoms + pair_count[l];
    // default shape (until tuned or set): blocks split over four wavefronts once
    // the LDS of their coordinates limits residency
    L->buckets.push_back(
        LigandBucket{ub, mx, (int32_t)order.size(), (int32_t)ids.size(), mx > 16 ? 4 : 1, 0, 0, cost});
    order.insert(order.end(), ids.begin(), ids.end());
    lo = ub;
  }
  hipError_t e = upload(&L->hdr, hdr);
  if (e == hipSuccess) e = upload(&L->atoms, atoms);
  if (e == hipSuccess) e = upload(&L->atom_type, types);
  if (e == hipSuccess) e = upload(&L->tors, tors);
  if (e == hipSuccess) e = upload(&L->pairs, pairs);
  if (e == hipSuccess) e = upload(&L->order, order);
  if (e == hipSuccess) e = upload(&L->desc, desc);
  if (e != hipSuccess) {
    free_ligands(L);
    return hip_err(e, "ligand upload");
  }
  *out = L;
  return DOCK_OK;
}

extern "C" dock_status dock_ligand_pair_count(const dock_ligands *L, int32_t lig, int32_t *n_pairs) {
  if (!L || !n_pairs) return set_err(DOCK_E_INVALID, "null argument");
  if (lig < 0 || lig >= L->n_ligs) return set_err(DOCK_E_INVALID, "ligand index out of range");
  *n_pairs = L->pair_count[lig];
  return DOCK_OK;
}

extern "C" dock_status dock_destroy_ligands(dock_ligands *L) {
  if (!L) return DOCK_OK;
  DeviceScope ds(L->device);
  free_ligands(L);
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ scoring
// Split of the scoring kernel (wavefronts per block of 64 poses): 0 = automatic
// (score_split_auto).
static std::atomic<int32_t> g_score_split{0};

// Automatic split.  A block's LDS (3 floats per atom per pose, 64 poses) is
// shared by its wavefronts, so a larger split keeps more wavefronts resident
// per CU for the same LDS, at the cost of the pose build's barriers and of the
// per-torsion setup each wavefront repeats.  Measured on MI355X (fourteen
// 100^3 maps in the pair-line layout, 2e6 random poses of one ligand of each
// size, M poses/s for splits 1 / 2 / 4 / 8): 12 atoms 4846 / 5054 / 4981 /
// 3783; 24 atoms 2100 / 2362 / 2429 / 1999; 48 atoms 421 / 689 / 955 / 795;
// 64 atoms 162 / 326 / 458 / 432; 96 atoms 49 / 104 / 142 / 206.  Four
// wavefronts up to 64 atoms (within 2% of the fastest at 12), eight above.
static int32_t score_split_auto(int32_t max_atoms, int32_t layout) {
  (void)layout;
  return max_atoms > 64 ? 8 : 4;
}

static int32_t score_split(const dock_ligands *L, int32_t layout) {
  const int32_t ws = g_score_split.load();
  return ws ? ws : score_split_auto(L->max_atoms, layout);
}

extern "C" dock_status dock_score_set_split(int32_t split) {
  if (split != 0 && split != 1 && split != 2 && split != 4 && split != 8)
    return set_err(DOCK_E_INVALID, "split must be 0, 1, 2, 4 or 8");
  g_score_split.store(split);
  return DOCK_OK;
}

extern "C" dock_status dock_score_split(const dock_ligands *L, int32_t *split) {
  if (!L || !split) return set_err(DOCK_E_INVALID, "null argument");
  *split = score_split(L, L->layout);
  return DOCK_OK;
}

static ScoreLaunch make_score(const dock_pocket *p, const dock_ligands *L) {
  ScoreLaunch a{};
  a.L = L->view();
  a.geom = p->geom;
  a.ff = p->ffc;
  a.maps = p->view();
  a.layout = p->layout;
  a.lds_atoms = L->max_atoms;
  a.split = score_split(L, p->layout);
  return a;
}

static dock_status check_pair(const dock_pocket *p, const dock_ligands *L) {
  if (!p || !L) return set_err(DOCK_E_INVALID, "null handle");
  if (p->device != L->device) return set_err(DOCK_E_INVALID, "pocket and ligands on different devices");
  return DOCK_OK;
}

extern "C" dock_status dock_score_poses(const dock_pocket *p, const dock_ligands *L, const int32_t *pose_ligand,
                                        const float *genotypes, int32_t g_stride, int64_t n_poses, float *energies,
                                        void *stream) {
  dock_status st = check_pair(p, L);
  if (st) return st;
  if (n_poses < 0) return set_err(DOCK_E_INVALID, "n_poses must be >= 0");
  if (n_poses == 0) return DOCK_OK;
  if (!genotypes || !energies) return set_err(DOCK_E_INVALID, "null genotypes or energies");
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride %d < 7 + %d torsions", g_stride, L->max_tors);
  if (n_poses > ((int64_t)1 << 37)) return set_err(DOCK_E_INVALID, "n_poses too large");
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  ScoreLaunch a = make_score(p, L);
  a.pose_ligand = pose_ligand;
  a.poses_per_ligand = 0;
  a.genotypes = genotypes;
  a.g_stride = g_stride;
  a.n_poses = n_poses;
  a.energies = energies;
  HIP_TRY(launch_score(a, (hipStream_t)stream), "score launch");
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ search
static dock_status check_params(const dock_search_params *q) {
  if (!q) return set_err(DOCK_E_INVALID, "null params");
  if (q->pop_size < 4) return set_err(DOCK_E_INVALID, "pop_size must be >= 4");
  if (q->pop_size > (1 << 20)) return set_err(DOCK_E_INVALID, "pop_size too large");
  if (q->n_generations < 0) return set_err(DOCK_E_INVALID, "n_generations must be >= 0");
  if (q->first_generation < 0) return set_err(DOCK_E_INVALID, "first_generation must be >= 0");
  if (!isfinite(q->F) || !isfinite(q->CR)) return set_err(DOCK_E_INVALID, "non-finite F or CR");
  for (int d = 0; d < 3; ++d)
    if (!(q->box_lo[d] <= q->box_hi[d]) || !isfinite(q->box_lo[d]) || !isfinite(q->box_hi[d]))
      return set_err(DOCK_E_INVALID, "empty or non-finite translation box");
  return DOCK_OK;
}

static DEParams de_params(const dock_search_params *q) {
  DEParams p{};
  p.pop = q->pop_size;
  p.n_gen = q->n_generations;
  p.first_gen = q->first_generation;
  p.seed = q->seed;
  p.F = q->F;
  p.CR = q->CR;
  for (int d = 0; d < 3; ++d) p.lo[d] = q->box_lo[d], p.hi[d] = q->box_hi[d];
  return p;
}

extern "C" dock_status dock_de_init(const dock_ligands *L, const dock_search_params *q, int32_t g_stride,
                                    float *population, void *stream) {
  if (!L || !population) return set_err(DOCK_E_INVALID, "null argument");
  dock_status st = check_params(q);
  if (st) return st;
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride too small");
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_de_init(L->view(), de_params(q), g_stride, population, (hipStream_t)stream), "de_init launch");
  return DOCK_OK;
}

extern "C" dock_status dock_de_trials(const dock_ligands *L, const dock_search_params *q, int32_t generation,
                                      int32_t g_stride, const float *population, float *trials, void *stream) {
  if (!L || !population || !trials) return set_err(DOCK_E_INVALID, "null argument");
  dock_status st = check_params(q);
  if (st) return st;
  if (generation < 0) return set_err(DOCK_E_INVALID, "generation must be >= 0");
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride too small");
  DeviceScope ds(L->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_de_trials(L->view(), de_params(q), generation, g_stride, population, trials, (hipStream_t)stream),
          "de_trials launch");
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ search shapes
namespace {

// Launch shapes found by the autotuner, for the whole process, keyed by what
// decides them: the kind of device (architecture and compute units), map layout
// and size, the bucket and its largest ligand, the population size.  The key
// names no device index, so shapes saved to a file apply to any device of the
// same kind.
struct ShapeKey {
  std::string arch;
  int n_cu, layout, nx, ny, nz, n_types, upper, lds_atoms, pop;
  bool operator<(const ShapeKey &o) const {
    return std::tie(arch, n_cu, layout, nx, ny, nz, n_types, upper, lds_atoms, pop) <
           std::tie(o.arch, o.n_cu, o.layout, o.nx, o.ny, o.nz, o.n_types, o.upper, o.lds_atoms, o.pop);
  }
};
std::mutex g_shape_mu;
std::map<ShapeKey, SearchShape> g_shapes;

ShapeKey shape_key(const dock_pocket *p, const LigandBucket &B, int pop) {
  return ShapeKey{p->arch, p->n_cu, p->layout, p->geom.nx, p->geom.ny, p->geom.nz, p->geom.n_types,
                  B.upper, B.lds_atoms, pop};
}

constexpr const char *kTuneHeader = "# dock search shapes v2: arch n_cu layout nx ny nz n_types bucket_upper "
                                    "largest_ligand pop split blocks_per_group";

}  // namespace

// The shape a bucket's search launch uses: the one set on the handle, else a
// tuned one for the same key, else the bucket's default.
static SearchShape bucket_shape(const dock_pocket *p, const LigandBucket &B, int pop) {
  if (!B.fixed) {
    std::lock_guard<std::mutex> g(g_shape_mu);
    auto it = g_shapes.find(shape_key(p, B, pop));
    if (it != g_shapes.end()) return it->second;
  }
  return SearchShape{B.split, B.blocks};
}

// One pass of the persistent search kernels over every size bucket, generations
// [S.p.first_gen, S.p.first_gen + S.p.n_gen): the buckets run concurrently on the
// handle's side streams (forked from and joined back to s), so that small
// buckets do not leave the GPU idle while the last ligands of another finish.
// Costliest bucket first, each onto the side stream with the least work so far,
// so the longest bucket never waits behind another.  With serial set, the
// buckets run one after another on s instead (the same order, no side streams
// and no events).
static hipError_t search_pass(const dock_pocket *p, const dock_ligands *L, SearchLaunch S, int32_t *queues,
                              hipStream_t s, const char **step, bool serial) {
  const int nb = (int)L->buckets.size();
  *step = "queue reset";
  hipError_t e = launch_fill_i32(queues, nb, 0, s);
  if (serial) {
    int by_cost[DOCK_SEARCH_BUCKETS];
    int m = 0;
    for (int b = 0; b < nb && m < DOCK_SEARCH_BUCKETS; ++b)
      if (L->buckets[b].count > 0) by_cost[m++] = b;
    std::stable_sort(by_cost, by_cost + m, [&](int x, int y) { return L->buckets[x].cost > L->buckets[y].cost; });
    for (int k = 0; k < m && e == hipSuccess; ++k) {
      const LigandBucket &B = L->buckets[by_cost[k]];
      S.order = L->order + B.offset;
      S.n_order = B.count;
      S.queue = queues + by_cost[k];
      S.lds_atoms = B.lds_atoms;
      e = launch_search(S, p->layout, p->n_cu, bucket_shape(p, B, S.p.pop), s, step);
    }
    return e;
  }
  std::lock_guard<std::mutex> guard(L->side_mu);
  if (e == hipSuccess) *step = "side streams", e = L->ensure_side_streams();
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, s);
  std::vector<int> by_cost;
  for (int b = 0; b < nb; ++b)
    if (L->buckets[b].count > 0) by_cost.push_back(b);
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&](int x, int y) { return L->buckets[x].cost > L->buckets[y].cost; });
  std::vector<int64_t> load(L->side.size(), 0);
  for (int b : by_cost) {
    if (e != hipSuccess) break;
    const LigandBucket &B = L->buckets[b];
    const size_t k = std::min_element(load.begin(), load.end()) - load.begin();
    load[k] += B.cost;
    hipStream_t side = L->side[k];
    *step = "side streams";
    e = hipStreamWaitEvent(side, fork, 0);
    S.order = L->order + B.offset;
    S.n_order = B.count;
    S.queue = queues + b;
    S.lds_atoms = B.lds_atoms;
    if (e == hipSuccess) e = launch_search(S, p->layout, p->n_cu, bucket_shape(p, B, S.p.pop), side, step);
    hipEvent_t done = nullptr;
    if (e == hipSuccess) *step = "side streams", e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e == hipSuccess) {
      joins.push_back(done);
      e = hipEventRecord(done, side);
    }
  }
  for (hipEvent_t ev : joins) {
    hipError_t w = hipStreamWaitEvent(s, ev, 0);
    if (e == hipSuccess) e = w;
    (void)hipEventDestroy(ev);
  }
  if (fork) (void)hipEventDestroy(fork);
  return e;
}

static dock_status check_search(const dock_pocket *p, const dock_ligands *L, const dock_search_params *q,
                                int32_t g_stride, const float *population, const float *pop_energy,
                                const float *best_genotypes, const float *best_energies, const float *target,
                                const int32_t *gen_reached) {
  dock_status st = check_pair(p, L);
  if (st) return st;
  if ((st = check_params(q))) return st;
  if (!population || !pop_energy || !best_genotypes || !best_energies)
    return set_err(DOCK_E_INVALID, "null output buffer");
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride too small");
  if ((int64_t)q->first_generation + q->n_generations > 0x7fffffff) return set_err(DOCK_E_INVALID, "too many generations");
  if (q->stop_at_target && !(target && gen_reached))
    return set_err(DOCK_E_INVALID, "stop_at_target needs target and gen_reached");
  const dock_mlp *net = q->proposal;
  if (net) {
    if (mlp_device(net) != p->device) return set_err(DOCK_E_INVALID, "proposal network on another device");
    if (!(q->proposal_step > 0) || !isfinite(q->proposal_step))
      return set_err(DOCK_E_INVALID, "proposal_step must be positive and finite");
    if (q->proposal_every < 0) return set_err(DOCK_E_INVALID, "proposal_every must be >= 0");
  }
  return DOCK_OK;
}

// Scratch of one search: trials and the gene-major population, [n_ligs][g_stride][pop]
// each, and one queue counter per bucket.
struct SearchScratch {
  float *trials = nullptr, *work = nullptr;
  int32_t *queues = nullptr;
};

// Enqueues a whole search (validated arguments, scratch in place) on s.
static hipError_t enqueue_search(const dock_pocket *p, const dock_ligands *L, const dock_search_params *q,
                                 int32_t g_stride, float *population, float *pop_energy, float *best_genotypes,
                                 float *best_energies, const float *target, int32_t *gen_reached,
                                 const SearchScratch &X, hipStream_t s, const char **step, bool serial = false) {
  const bool track = target && gen_reached;
  const dock_mlp *net = q->proposal;
  const int P = q->pop_size;
  SearchLaunch S{};
  S.L = L->view();
  S.geom = p->geom;
  S.ff = p->ffc;
  S.maps = p->view();
  S.p = de_params(q);
  S.g_stride = g_stride;
  S.init = q->init ? 1 : 0;
  S.population = population;
  S.pop_energy = pop_energy;
  S.best_g = best_genotypes;
  S.best_e = best_energies;
  S.target = track ? target : nullptr;
  S.gen_reached = track ? gen_reached : nullptr;
  S.stop = q->stop_at_target ? 1 : 0;
  S.trials = X.trials;
  S.work = X.work;
  if (!net) return search_pass(p, L, S, X.queues, s, step, serial);
  // Learned proposals: a round fills the trial buffer with one proposal per
  // individual; the next persistent pass scores them and takes each greedily
  // before its generations (the pass's DE trials reuse that buffer afterwards).
  const PopRows R = make_pop_rows(L, P, g_stride, q->box_lo, q->box_hi);
  const int g0 = q->first_generation, g_end = g0 + q->n_generations;
  const int every = q->proposal_every;
  auto propose = [&](int gen) {
    *step = "proposals";
    return run_proposals(net, R, q->proposal_step, q->seed, gen, population, S.trials, s);
  };
  hipError_t e = hipSuccess;
  bool pending = false;
  if (q->init) {
    // the initial population and its scores, then the first round
    SearchLaunch T = S;
    T.p.n_gen = 0;
    e = search_pass(p, L, T, X.queues, s, step, serial);
    if (e == hipSuccess) e = propose(g0);
    pending = true;
  } else if (every > 0 && g0 > 0 && g0 % every == 0 && g0 < q->proposal_until && g0 < g_end) {
    // later rounds come before the generations g > 0 that are multiples of
    // proposal_every (g < proposal_until), so a search split into resumed
    // calls runs the same rounds as one call
    e = propose(g0);
    pending = true;
  }
  int g = g0;
  while (e == hipSuccess) {
    int seg_end = g_end;
    if (every > 0) {
      const int64_t nb = ((int64_t)g / every + 1) * every;
      if (nb < q->proposal_until && nb < g_end) seg_end = (int)nb;
    }
    SearchLaunch T = S;
    T.init = 0;
    T.p.first_gen = g;
    T.p.n_gen = seg_end - g;
    T.proposals = pending ? S.trials : nullptr;
    e = search_pass(p, L, T, X.queues, s, step, serial);
    pending = false;
    g = seg_end;
    if (g >= g_end) break;
    if (e == hipSuccess) e = propose(g);
    pending = true;
  }
  return e;
}

extern "C" dock_status dock_search(const dock_pocket *p, const dock_ligands *L, const dock_search_params *q,
                                   int32_t g_stride, float *population, float *pop_energy, float *best_genotypes,
                                   float *best_energies, const float *target, int32_t *gen_reached, void *stream) {
  dock_status st = check_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target,
                                gen_reached);
  if (st) return st;
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t nf = (size_t)L->n_ligs * q->pop_size * g_stride;
  SearchScratch X;
  const char *step = "search buffers";
  hipError_t e = scratch_alloc((void **)&X.trials, sizeof(float) * nf, s);
  if (e == hipSuccess) e = scratch_alloc((void **)&X.work, sizeof(float) * nf, s);
  if (e == hipSuccess) e = scratch_alloc((void **)&X.queues, sizeof(int32_t) * L->buckets.size(), s);
  if (e == hipSuccess)
    e = enqueue_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target, gen_reached,
                       X, s, &step);
  if (X.queues) (void)hipFreeAsync(X.queues, s);
  if (X.work) (void)hipFreeAsync(X.work, s);
  if (X.trials) (void)hipFreeAsync(X.trials, s);
  if (e != hipSuccess) return hip_err(e, step);
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ search without allocation
// The fixed scratch of dock_search_no_alloc, one copy per device: 256 bytes of
// bucket queue counters, then the trials and the gene-major population, each
// rounded up to 256 bytes.  In host code `scratch` only names the array; its
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[DOCK_NO_ALLOC_SCRATCH_BYTES];

namespace {
constexpr size_t kScratchQueueBytes = 256;
static_assert(DOCK_SEARCH_BUCKETS * sizeof(int32_t) <= kScratchQueueBytes, "queue counters fit their slot");
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_ptr;   // device ordinal -> device address of `scratch`

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Device address of this device's scratch (the device current).
hipError_t scratch_address(int device, unsigned char **out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = (unsigned char *)ptr;
  *out = (unsigned char *)ptr;
  return hipSuccess;
}
}  // namespace

extern "C" dock_status dock_search_no_alloc(const dock_pocket *p, const dock_ligands *L, const dock_search_params *q,
                                           int32_t g_stride, float *population, float *pop_energy,
                                           float *best_genotypes, float *best_energies, const float *target,
                                           int32_t *gen_reached, void *stream) {
  dock_status st = check_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target,
                                gen_reached);
  if (st) return st;
  const size_t nf = (size_t)L->n_ligs * q->pop_size * g_stride;
  const size_t arr = round256(sizeof(float) * nf);
  if (nf > ((size_t)DOCK_NO_ALLOC_SCRATCH_BYTES - kScratchQueueBytes) / (2 * sizeof(float)) ||
      kScratchQueueBytes + 2 * arr > (size_t)DOCK_NO_ALLOC_SCRATCH_BYTES)
    return set_err(DOCK_E_INVALID,
                   "search needs %zu bytes of scratch (n_ligands x pop_size x g_stride = %zu floats, twice), more "
                   "than the fixed %u of dock_search_no_alloc",
                   kScratchQueueBytes + 2 * arr, nf, (unsigned)DOCK_NO_ALLOC_SCRATCH_BYTES);
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  unsigned char *base = nullptr;
  HIP_TRY(scratch_address(p->device, &base), "hipGetSymbolAddress(scratch)");
  SearchScratch X;
  X.queues = (int32_t *)base;
  X.trials = (float *)(base + kScratchQueueBytes);
  X.work = (float *)(base + kScratchQueueBytes + arr);
  const char *step = "search";
  hipError_t e = enqueue_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target,
                                gen_reached, X, (hipStream_t)stream, &step, true);
  if (e != hipSuccess) return hip_err(e, step);
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ search plans
struct dock_search_plan {
  int device = 0;
  SearchScratch X;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void free_plan(dock_search_plan *P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (void *b : {(void *)P->X.trials, (void *)P->X.work, (void *)P->X.queues})
    if (b) (void)hipFree(b);
  delete P;
}

extern "C" dock_status dock_search_plan_create(const dock_pocket *p, const dock_ligands *L,
                                               const dock_search_params *q, int32_t g_stride, float *population,
                                               float *pop_energy, float *best_genotypes, float *best_energies,
                                               const float *target, int32_t *gen_reached, dock_search_plan **out) {
  if (!out) return set_err(DOCK_E_INVALID, "null out");
  *out = nullptr;
  dock_status st = check_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target,
                                gen_reached);
  if (st) return st;
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  dock_search_plan *P = new dock_search_plan();
  P->device = p->device;
  const size_t nf = (size_t)L->n_ligs * q->pop_size * g_stride;
  const char *step = "plan buffers";
  hipError_t e = hipMalloc((void **)&P->X.trials, sizeof(float) * nf);
  if (e == hipSuccess) e = hipMalloc((void **)&P->X.work, sizeof(float) * nf);
  if (e == hipSuccess) e = hipMalloc((void **)&P->X.queues, sizeof(int32_t) * L->buckets.size());
  // capture on a private stream (default priority); the side streams join the
  // capture through the fork/join events
  hipStream_t cs = nullptr;
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> guard(L->side_mu);
    e = L->ensure_side_streams();  // created before the capture starts
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) {
    step = "graph capture";
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      hipError_t w = enqueue_search(p, L, q, g_stride, population, pop_energy, best_genotypes, best_energies, target,
                                    gen_reached, P->X, cs, &step);
      hipError_t c = hipStreamEndCapture(cs, &P->graph);
      e = w != hipSuccess ? w : c;
    }
  }
  if (e == hipSuccess) step = "graph instantiate", e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    free_plan(P);
    return hip_err(e, step);
  }
  *out = P;
  return DOCK_OK;
}

extern "C" dock_status dock_search_plan_launch(dock_search_plan *P, void *stream) {
  if (!P) return set_err(DOCK_E_INVALID, "null plan");
  DeviceScope ds(P->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(hipGraphLaunch(P->exec, (hipStream_t)stream), "graph launch");
  return DOCK_OK;
}

extern "C" dock_status dock_search_plan_destroy(dock_search_plan *P) {
  if (!P) return DOCK_OK;
  DeviceScope ds(P->device);
  free_plan(P);
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ shapes and autotuner
extern "C" dock_status dock_search_shapes(const dock_ligands *L, dock_search_shape *shapes) {
  if (!L || !shapes) return set_err(DOCK_E_INVALID, "null argument");
  for (size_t b = 0; b < L->buckets.size(); ++b)
    shapes[b] = dock_search_shape{L->buckets[b].upper, L->buckets[b].split, L->buckets[b].blocks};
  return DOCK_OK;
}

extern "C" dock_status dock_search_set_shapes(dock_ligands *L, const dock_search_shape *shapes) {
  if (!L || !shapes) return set_err(DOCK_E_INVALID, "null argument");
  for (size_t b = 0; b < L->buckets.size(); ++b) {
    const dock_search_shape &x = shapes[b];
    if (x.max_atoms != L->buckets[b].upper) return set_err(DOCK_E_INVALID, "bucket %d bound must be %d", (int)b, L->buckets[b].upper);
    if (x.split != 1 && x.split != 2 && x.split != 4 && x.split != 8)
      return set_err(DOCK_E_INVALID, "split must be 1, 2, 4 or 8");
    if (x.blocks_per_group < 0 || x.blocks_per_group * x.split * kWave > kSearchMaxThreads)
      return set_err(DOCK_E_INVALID, "blocks_per_group must be in 0..%d for split %d",
                     kSearchMaxThreads / (kWave * x.split), x.split);
  }
  std::lock_guard<std::mutex> guard(L->side_mu);
  for (size_t b = 0; b < L->buckets.size(); ++b) {
    L->buckets[b].split = shapes[b].split;
    L->buckets[b].blocks = shapes[b].blocks_per_group;
    L->buckets[b].fixed = 1;
  }
  return DOCK_OK;
}

extern "C" dock_status dock_search_autotune(const dock_pocket *p, dock_ligands *L, const dock_search_params *q,
                                            int32_t g_stride, int32_t tune_generations, void *stream) {
  dock_status st = check_pair(p, L);
  if (st) return st;
  if ((st = check_params(q))) return st;
  if (g_stride < 7 + L->max_tors) return set_err(DOCK_E_INVALID, "g_stride too small");
  if (tune_generations < 1 || tune_generations > 1000) return set_err(DOCK_E_INVALID, "tune_generations must be in 1..1000");
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int P = q->pop_size;
  const int64_t n = (int64_t)L->n_ligs * P;
  // scratch state of a search over the whole set (the timed runs touch one bucket each)
  SearchLaunch S{};
  S.L = L->view();
  S.geom = p->geom;
  S.ff = p->ffc;
  S.maps = p->view();
  S.p = de_params(q);
  S.p.first_gen = 0;
  S.p.n_gen = tune_generations;
  S.g_stride = g_stride;
  S.init = 1;
  float *buf = nullptr;
  int32_t *queue = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  const char *step = "autotune buffers";
  const size_t nf = (size_t)n * g_stride;
  hipError_t e = hipMalloc((void **)&buf, sizeof(float) * (3 * nf + n + (size_t)L->n_ligs * (g_stride + 1)));
  if (e == hipSuccess) e = hipMalloc((void **)&queue, sizeof(int32_t));
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e == hipSuccess) {
    S.population = buf;
    S.trials = buf + nf;
    S.work = buf + 2 * nf;
    S.pop_energy = buf + 3 * nf;
    S.best_g = S.pop_energy + n;
    S.best_e = S.best_g + (size_t)L->n_ligs * g_stride;
  }
  for (size_t b = 0; b < L->buckets.size() && e == hipSuccess; ++b) {
    LigandBucket &B = L->buckets[b];
    if (B.count == 0) continue;
    {
      std::lock_guard<std::mutex> g(g_shape_mu);
      auto it = g_shapes.find(shape_key(p, B, P));
      if (it != g_shapes.end()) {
        std::lock_guard<std::mutex> guard(L->side_mu);
        B.split = it->second.split, B.blocks = it->second.blocks, B.fixed = 1;
        continue;
      }
    }
    S.order = L->order + B.offset;
    S.n_order = B.count;
    S.queue = queue;
    S.lds_atoms = B.lds_atoms;
    SearchShape best{0, 0};
    float best_ms = 0.f;
    for (int ws = 1; ws <= kMaxSplit && e == hipSuccess; ws *= 2) {
      const int max_b = std::min(kSearchMaxThreads / (kWave * ws), (P + kBlock - 1) / kBlock);
      for (int nb = 1; nb <= max_b && e == hipSuccess; ++nb) {
        const SearchShape shape{ws, nb};
        if (!search_shape_fits(B.lds_atoms, shape)) continue;
        float ms = 0.f;
        // a warm-up run, then the timed one
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
          step = "autotune run";
          e = launch_fill_i32(queue, 1, 0, s);
          if (e == hipSuccess) e = hipEventRecord(t0, s);
          if (e == hipSuccess) e = launch_search(S, p->layout, p->n_cu, shape, s, &step);
          if (e == hipErrorInvalidConfiguration) {  // this shape does not fit the CU: skip it
            (void)hipGetLastError();
            e = hipSuccess;
            ms = -1.f;
            break;
          }
          if (e == hipSuccess) e = hipEventRecord(t1, s);
          if (e == hipSuccess) e = hipEventSynchronize(t1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        }
        if (e == hipSuccess && ms >= 0.f && (best.split == 0 || ms < best_ms)) best = shape, best_ms = ms;
      }
    }
    if (e != hipSuccess || best.split == 0) break;
    {
      std::lock_guard<std::mutex> guard(L->side_mu);
      B.split = best.split;
      B.blocks = best.blocks;
      B.fixed = 1;
    }
    std::lock_guard<std::mutex> g(g_shape_mu);
    g_shapes[shape_key(p, B, P)] = best;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (queue) (void)hipFree(queue);
  if (buf) (void)hipFree(buf);
  if (e != hipSuccess) return hip_err(e, step);
  return DOCK_OK;
}

// The autotuner's cache as a text file: a header line, then one shape per line.
extern "C" dock_status dock_search_tune_save(const char *path) {
  if (!path) return set_err(DOCK_E_INVALID, "null path");
  std::string text = std::string(kTuneHeader) + "\n";
  {
    std::lock_guard<std::mutex> g(g_shape_mu);
    char line[256];
    for (const auto &kv : g_shapes) {
      const ShapeKey &k = kv.first;
      snprintf(line, sizeof line, "%s %d %d %d %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.n_cu, k.layout, k.nx,
               k.ny, k.nz, k.n_types, k.upper, k.lds_atoms, k.pop, kv.second.split, kv.second.blocks);
      text += line;
    }
  }
  FILE *f = fopen(path, "w");
  if (!f) return set_err(DOCK_E_INVALID, "cannot write %s", path);
  const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return set_err(DOCK_E_INVALID, "cannot write %s", path);
  return DOCK_OK;
}

extern "C" dock_status dock_search_tune_load(const char *path) {
  if (!path) return set_err(DOCK_E_INVALID, "null path");
  FILE *f = fopen(path, "r");
  if (!f) return set_err(DOCK_E_INVALID, "cannot read %s", path);
  std::vector<std::pair<ShapeKey, SearchShape>> entries;
  char line[512];
  int n_line = 0;
  dock_status st = DOCK_OK;
  while (fgets(line, sizeof line, f)) {
    ++n_line;
    if (line[0] == '#' || line[0] == '\n' || line[0] == '\0') continue;
    char arch[64];
    ShapeKey k{};
    SearchShape sh{};
    char extra[2];
    const int got = sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %1s", arch, &k.n_cu, &k.layout, &k.nx, &k.ny,
                           &k.nz, &k.n_types, &k.upper, &k.lds_atoms, &k.pop, &sh.split, &sh.blocks, extra);
    const bool valid = got == 12 && k.n_cu > 0 && k.layout >= kLinear && k.layout <= kPairLine && k.nx >= 2 &&
                       k.ny >= 2 && k.nz >= 2 && k.n_types >= 1 && k.n_types <= kMaxTypes && k.upper >= 1 &&
                       k.upper <= kMaxAtoms && k.lds_atoms >= 1 && k.lds_atoms <= k.upper && k.pop >= 4 &&
                       (sh.split == 1 || sh.split == 2 || sh.split == 4 || sh.split == 8) && sh.blocks >= 0 &&
                       sh.blocks * sh.split * kWave <= kSearchMaxThreads;
    if (!valid) {
      st = set_err(DOCK_E_INVALID, "%s line %d: not a search shape", path, n_line);
      break;
    }
    k.arch = arch;
    entries.emplace_back(k, sh);
  }
  if (st == DOCK_OK && ferror(f)) st = set_err(DOCK_E_INVALID, "cannot read %s", path);
  fclose(f);
  if (st) return st;
  std::lock_guard<std::mutex> g(g_shape_mu);
  for (const auto &kv : entries) g_shapes[kv.first] = kv.second;
  return DOCK_OK;
}

// ------------------------------------------------------------------------------ probes
extern "C" dock_status dock_gather_probe(const dock_pocket *p, const dock_ligands *L, int32_t lig,
                                         const float box_lo[3], const float box_hi[3], int64_t n_lanes,
                                         int32_t per_lane, int32_t in_flight, uint64_t seed, float *out,
                                         void *stream) {
  dock_status st = check_pair(p, L);
  if (st) return st;
  if (!box_lo || !box_hi || !out) return set_err(DOCK_E_INVALID, "null argument");
  if (lig < 0 || lig >= L->n_ligs) return set_err(DOCK_E_INVALID, "ligand index out of range");
  if (in_flight != 2 && in_flight != 4 && in_flight != 8) return set_err(DOCK_E_INVALID, "in_flight must be 2, 4 or 8");
  if (n_lanes < 1 || n_lanes > ((int64_t)1 << 31) || per_lane < in_flight || per_lane % in_flight)
    return set_err(DOCK_E_INVALID, "n_lanes in 1..2^31, per_lane a positive multiple of in_flight");
  ProbeBox box{};
  for (int d = 0; d < 3; ++d) {
    if (!(box_lo[d] <= box_hi[d])) return set_err(DOCK_E_INVALID, "empty probe box");
    box.lo[d] = box_lo[d];
    box.ext[d] = box_hi[d] - box_lo[d];
  }
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_gather_probe(p->geom, p->view(), p->layout, L->view(), lig, box, n_lanes, per_lane, in_flight,
                              (uint32_t)seed, out, (hipStream_t)stream),
          "gather probe launch");
  return DOCK_OK;
}

extern "C" dock_status dock_pair_probe(const dock_pocket *p, int64_t n_lanes, int32_t per_lane, float *out,
                                       void *stream) {
  if (!p || !out) return set_err(DOCK_E_INVALID, "null argument");
  if (n_lanes < 1 || n_lanes > ((int64_t)1 << 31) || per_lane < 4 || per_lane % 4)
    return set_err(DOCK_E_INVALID, "n_lanes in 1..2^31, per_lane a positive multiple of 4");
  DeviceScope ds(p->device);
  HIP_TRY(ds.err, "hipSetDevice");
  HIP_TRY(launch_pair_probe(p->ffc, n_lanes, per_lane, out, (hipStream_t)stream), "pair probe launch");
  return DOCK_OK;
}
