/* oracle.c -- plain FP64 CPU oracle for the muDock docking hot path.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.
 *
 * What it computes, in the paper's order:
 *   - docking of one individual (Sec. V, Algorithm 1): rotatable-bond fragment
 *     rotations, then the rigid rotation about the ligand origin and the
 *     translation;
 *   - scoring of a docked ligand (Sec. V, Algorithm 2): an inter-energy loop over
 *     ligand atoms that looks up precomputed per-type, electrostatic and
 *     desolvation grid maps when the atom is near the protein, and an
 *     intra-energy loop over ligand atom pairs that evaluates van der Waals /
 *     hydrogen-bond, electrostatic and desolvation terms; the score is their sum;
 *   - the grid maps themselves, AutoGrid-style (Sec. V): a probe of each type at
 *     every node, summed over receptor atoms;
 *   - an evolutionary search whose fitness is the score (Sec. V; here plain
 *     DE/rand/1/bin with greedy selection, driven by Philox4x64-10 of Salmon et
 *     al., SC'11).
 * The paper fixes the loop structure and the term list but no formulas; the
 * readings used here (functional forms, constants as input data, the pair
 * exclusion rule, the grid-box "nearby" test) are listed in the design notes.
 *
 * Plain loops, binary64 everywhere, no contraction, no reordering beyond what
 * the definitions state.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static _Thread_local char g_err[512];

const char *oracle_last_error(void) { return g_err; }

static int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

/* ===================================================================================
 * Ligand preprocessing: root, torsion orientation, moving sets, rigid fragments,
 * non-bonded pair list.
 * =================================================================================== */
typedef struct {
  int n, nt;
  double *x;          /* [n][3] reference conformation minus its centroid */
  int *type;
  double *q;
  int *tor_a, *tor_b; /* oriented: tor_a nearer the root (atom 0) */
  uint8_t *moving;    /* [nt][n] */
  int *frag;          /* rigid fragment id per atom */
  int64_t n_pairs;
  int *pi, *pj;
} prep_t;

static void prep_free(prep_t *p) {
  if (!p) return;
  free(p->x); free(p->type); free(p->q); free(p->tor_a); free(p->tor_b);
  free(p->moving); free(p->frag); free(p->pi); free(p->pj);
  memset(p, 0, sizeof *p);
}

static int find_root(int *uf, int a) {
  while (uf[a] != a) a = uf[a];
  return a;
}

static int prep_ligand(const ora_ligand *lig, int n_types, prep_t *P) {
  memset(P, 0, sizeof *P);
  const int n = lig->n_atoms, nt = lig->n_torsions;
  if (n < 1) return fail(ORA_E_INVALID, "n_atoms must be >= 1");
  if (nt < 0 || nt > (n > 1 ? n - 1 : 0)) return fail(ORA_E_INVALID, "bad n_torsions %d", nt);
  if (!lig->xyz || !lig->type || !lig->charge || (n > 1 && !lig->bonds) || (nt > 0 && !lig->torsion_bonds))
    return fail(ORA_E_INVALID, "null ligand array");
  for (int i = 0; i < n; i++)
    if (lig->type[i] < 0 || lig->type[i] >= n_types) return fail(ORA_E_INVALID, "atom type out of range");

  /* adjacency of the bond graph */
  int *deg = calloc(n, sizeof(int));
  int *adj = malloc(sizeof(int) * (size_t)n * n); /* adj[i*n + k]: k-th neighbour of i */
  int *adjb = malloc(sizeof(int) * (size_t)n * n); /* bond index of that neighbour edge */
  int *depth = malloc(sizeof(int) * n), *parent = malloc(sizeof(int) * n), *queue = malloc(sizeof(int) * n);
  int rc = ORA_OK;
  for (int k = 0; k < n - 1; k++) {
    int a = lig->bonds[2 * k], b = lig->bonds[2 * k + 1];
    if (a < 0 || a >= n || b < 0 || b >= n || a == b) { rc = fail(ORA_E_INVALID, "bad bond %d", k); goto out; }
    adj[a * n + deg[a]] = b; adjb[a * n + deg[a]] = k; deg[a]++;
    adj[b * n + deg[b]] = a; adjb[b * n + deg[b]] = k; deg[b]++;
  }
  /* breadth-first walk from the root: n-1 edges that reach every atom form a tree */
  for (int i = 0; i < n; i++) depth[i] = -1;
  depth[0] = 0; parent[0] = -1;
  int head = 0, tail = 0;
  queue[tail++] = 0;
  while (head < tail) {
    int a = queue[head++];
    for (int k = 0; k < deg[a]; k++) {
      int b = adj[a * n + k];
      if (depth[b] < 0) { depth[b] = depth[a] + 1; parent[b] = a; queue[tail++] = b; }
    }
  }
  if (tail != n) { rc = fail(ORA_E_INVALID, "bonds do not form a tree"); goto out; }

  P->n = n; P->nt = nt;
  P->x = malloc(sizeof(double) * 3 * n);
  P->type = malloc(sizeof(int) * n);
  P->q = malloc(sizeof(double) * n);
  P->tor_a = malloc(sizeof(int) * (nt ? nt : 1));
  P->tor_b = malloc(sizeof(int) * (nt ? nt : 1));
  P->moving = calloc((size_t)(nt ? nt : 1) * n, 1);
  P->frag = malloc(sizeof(int) * n);

  /* centroid of the reference conformation is the ligand origin */
  double c[3] = {0, 0, 0};
  for (int i = 0; i < n; i++)
    for (int d = 0; d < 3; d++) c[d] += (double)lig->xyz[3 * i + d];
  for (int d = 0; d < 3; d++) c[d] /= n;
  for (int i = 0; i < n; i++) {
    for (int d = 0; d < 3; d++) P->x[3 * i + d] = (double)lig->xyz[3 * i + d] - c[d];
    P->type[i] = lig->type[i];
    P->q[i] = (double)lig->charge[i];
  }

  /* torsions: orient each rotatable bond away from the root; the moving set is
   * the subtree hanging from the far end */
  uint8_t *is_rot = calloc(n > 1 ? n - 1 : 1, 1);
  for (int k = 0; k < nt; k++) {
    int bi = lig->torsion_bonds[k];
    if (bi < 0 || bi >= n - 1) { free(is_rot); rc = fail(ORA_E_INVALID, "torsion bond index out of range"); goto out; }
    if (is_rot[bi]) { free(is_rot); rc = fail(ORA_E_INVALID, "duplicate torsion bond"); goto out; }
    is_rot[bi] = 1;
    int a = lig->bonds[2 * bi], b = lig->bonds[2 * bi + 1];
    if (deg[a] < 2 || deg[b] < 2) { free(is_rot); rc = fail(ORA_E_INVALID, "torsion on a terminal bond"); goto out; }
    if (depth[a] > depth[b]) { int t = a; a = b; b = t; }
    P->tor_a[k] = a; P->tor_b[k] = b;
    for (int i = 0; i < n; i++) {
      for (int w = i; w >= 0; w = parent[w])
        if (w == b) { P->moving[(size_t)k * n + i] = 1; break; }
    }
  }

  /* rigid fragments: connected components after removing rotatable bonds */
  int *uf = malloc(sizeof(int) * n);
  for (int i = 0; i < n; i++) uf[i] = i;
  for (int k = 0; k < n - 1; k++) {
    if (is_rot[k]) continue;
    int ra = find_root(uf, lig->bonds[2 * k]), rb = find_root(uf, lig->bonds[2 * k + 1]);
    if (ra != rb) uf[rb] = ra;
  }
  for (int i = 0; i < n; i++) P->frag[i] = find_root(uf, i);
  free(uf);
  free(is_rot);

  /* graph distances (one breadth-first walk per atom) and the pair list:
   * i<j, at least four bonds apart, in different rigid fragments */
  int *dist = malloc(sizeof(int) * (size_t)n * n);
  for (int s = 0; s < n; s++) {
    int *ds = dist + (size_t)s * n;
    for (int i = 0; i < n; i++) ds[i] = -1;
    ds[s] = 0; head = tail = 0; queue[tail++] = s;
    while (head < tail) {
      int a = queue[head++];
      for (int k = 0; k < deg[a]; k++) {
        int b = adj[a * n + k];
        if (ds[b] < 0) { ds[b] = ds[a] + 1; queue[tail++] = b; }
      }
    }
  }
  int64_t np = 0;
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++)
      if (dist[(size_t)i * n + j] >= 4 && P->frag[i] != P->frag[j]) np++;
  P->n_pairs = np;
  P->pi = malloc(sizeof(int) * (np ? np : 1));
  P->pj = malloc(sizeof(int) * (np ? np : 1));
  np = 0;
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++)
      if (dist[(size_t)i * n + j] >= 4 && P->frag[i] != P->frag[j]) { P->pi[np] = i; P->pj[np] = j; np++; }
  free(dist);
out:
  free(deg); free(adj); free(adjb); free(depth); free(parent); free(queue);
  if (rc != ORA_OK) prep_free(P);
  return rc;
}

int oracle_ligand_info(const ora_ligand *lig, int n_types, int32_t *pairs, int64_t max_pairs,
                       int64_t *n_pairs, int32_t *frag, uint8_t *moving, int32_t *axis) {
  prep_t P;
  int rc = prep_ligand(lig, n_types, &P);
  if (rc) return rc;
  *n_pairs = P.n_pairs;
  if (pairs)
    for (int64_t p = 0; p < P.n_pairs && p < max_pairs; p++) { pairs[2 * p] = P.pi[p]; pairs[2 * p + 1] = P.pj[p]; }
  if (frag) for (int i = 0; i < P.n; i++) frag[i] = P.frag[i];
  if (moving) memcpy(moving, P.moving, (size_t)P.nt * P.n);
  if (axis) for (int k = 0; k < P.nt; k++) { axis[2 * k] = P.tor_a[k]; axis[2 * k + 1] = P.tor_b[k]; }
  prep_free(&P);
  return ORA_OK;
}

/* ===================================================================================
 * Algorithm 1: dock one individual.
 * Genotype: t(3) translation in Angstrom, q(4) = (w,x,y,z) orientation
 * quaternion (normalised here), theta(n_torsions) radians.
 * =================================================================================== */
static int genes_finite(const float *g, int n_genes) {
  for (int j = 0; j < n_genes; j++)
    if (!isfinite((double)g[j])) return 0;
  return 1;
}

static void build_pose(const prep_t *P, const float *g, double *X) {
  const int n = P->n;
  memcpy(X, P->x, sizeof(double) * 3 * n);
  /* rotatable-bond fragments: rotate the moving subtree about the current bond
   * axis a->b by theta (right-hand rule, Rodrigues' formula) */
  for (int k = 0; k < P->nt; k++) {
    const double th = (double)g[7 + k];
    const int a = P->tor_a[k], b = P->tor_b[k];
    double u[3], len = 0;
    for (int d = 0; d < 3; d++) { u[d] = X[3 * b + d] - X[3 * a + d]; len += u[d] * u[d]; }
    len = sqrt(len);
    for (int d = 0; d < 3; d++) u[d] /= len;
    const double c = cos(th), s = sin(th);
    const double ax = X[3 * a], ay = X[3 * a + 1], az = X[3 * a + 2];
    for (int i = 0; i < n; i++) {
      if (!P->moving[(size_t)k * n + i]) continue;
      const double v[3] = {X[3 * i] - ax, X[3 * i + 1] - ay, X[3 * i + 2] - az};
      const double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
      const double ud = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
      X[3 * i] = ax + (v[0] * c + cr[0] * s + u[0] * ud * (1.0 - c));
      X[3 * i + 1] = ay + (v[1] * c + cr[1] * s + u[1] * ud * (1.0 - c));
      X[3 * i + 2] = az + (v[2] * c + cr[2] * s + u[2] * ud * (1.0 - c));
    }
  }
  /* rotation about the ligand origin, then translation */
  double w = g[3], x = g[4], y = g[5], z = g[6];
  const double nn = w * w + x * x + y * y + z * z;
  if (nn < 1e-24) { w = 1; x = y = z = 0; }
  else { const double r = sqrt(nn); w /= r; x /= r; y /= r; z /= r; }
  const double R[9] = {
      1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
      2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
      2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  for (int i = 0; i < n; i++) {
    const double p0 = X[3 * i], p1 = X[3 * i + 1], p2 = X[3 * i + 2];
    for (int d = 0; d < 3; d++)
      X[3 * i + d] = (R[3 * d] * p0 + R[3 * d + 1] * p1 + R[3 * d + 2] * p2) + (double)g[d];
  }
}

int oracle_pose(const ora_ligand *lig, int n_types, const float *genotype, double *xyz_out) {
  prep_t P;
  int rc = prep_ligand(lig, n_types, &P);
  if (rc) return rc;
  build_pose(&P, genotype, xyz_out);
  prep_free(&P);
  return ORA_OK;
}

/* ===================================================================================
 * Algorithm 2, inter-energy loop: grid-map lookup for atoms inside the grid box.
 * =================================================================================== */
static double map_at(const ora_grid *G, int m, int i, int j, int k) {
  const size_t nx = G->dims[0], ny = G->dims[1], nz = G->dims[2];
  return (double)G->maps[(((size_t)m * nz + k) * ny + j) * nx + i];
}

/* trilinear interpolation of map m in cell c with fractions f */
static double trilinear(const ora_grid *G, int m, const int c[3], const double f[3]) {
  double s = 0;
  for (int b = 0; b < 8; b++) {
    const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
    const double w = (bx ? f[0] : 1 - f[0]) * (by ? f[1] : 1 - f[1]) * (bz ? f[2] : 1 - f[2]);
    s += w * map_at(G, m, c[0] + bx, c[1] + by, c[2] + bz);
  }
  return s;
}

/* energy of one atom at p: 0 outside the closed grid box */
static double atom_inter(const ora_grid *G, const double p[3], int type, double q) {
  double u[3], f[3];
  int c[3];
  for (int d = 0; d < 3; d++) {
    u[d] = (p[d] - G->origin[d]) / G->spacing;
    if (!(u[d] >= 0.0 && u[d] <= (double)(G->dims[d] - 1))) return 0.0;
  }
  for (int d = 0; d < 3; d++) {
    int cd = (int)floor(u[d]);
    if (cd > G->dims[d] - 2) cd = G->dims[d] - 2;
    c[d] = cd;
    f[d] = u[d] - cd;
  }
  const double t = trilinear(G, type, c, f);
  const double e = trilinear(G, G->n_types, c, f);
  const double s = trilinear(G, G->n_types + 1, c, f);
  return t + q * e + fabs(q) * s;
}

int oracle_inter_atoms(const ora_grid *G, int n_atoms, const double *xyz, const int32_t *type,
                       const double *charge, double *per_atom) {
  for (int d = 0; d < 3; d++)
    if (G->dims[d] < 2) return fail(ORA_E_INVALID, "grid dims must be >= 2");
  for (int i = 0; i < n_atoms; i++) {
    if (type[i] < 0 || type[i] >= G->n_types) return fail(ORA_E_INVALID, "type out of range");
    per_atom[i] = atom_inter(G, xyz + 3 * i, type[i], charge[i]);
  }
  return ORA_OK;
}

/* ===================================================================================
 * Pair terms (Algorithm 2, intra-energy loop; the same pieces build the maps).
 * =================================================================================== */
/* van der Waals (12-6) or hydrogen bond (12-10), well depth -eps at r_eq,
 * capped at e_cap from above */
static double vdw_hb(const ora_ff *ff, int ti, int tj, double r) {
  const double req = 0.5 * (ff->Rii[ti] + ff->Rii[tj]);
  const double eps = sqrt(ff->epsii[ti] * ff->epsii[tj]);
  double e;
  if (ff->hbond[ti * ff->n_types + tj]) {
    const double A = 5.0 * eps * pow(req, 12), B = 6.0 * eps * pow(req, 10);
    e = A / pow(r, 12) - B / pow(r, 10);
  } else {
    const double A = eps * pow(req, 12), B = 2.0 * eps * pow(req, 6);
    e = A / pow(r, 12) - B / pow(r, 6);
  }
  return e < ff->e_cap ? e : ff->e_cap;
}

/* sigmoidal distance-dependent dielectric */
static double dielectric(const ora_ff *ff, double r) {
  const double B = ff->diel_eps0 - ff->diel_A;
  return ff->diel_A + B / (1.0 + ff->diel_k * exp(-ff->diel_lambda * B * r));
}

static double gauss(const ora_ff *ff, double r) {
  return exp(-(r * r) / (2.0 * ff->sigma * ff->sigma));
}

double oracle_pair_energy(const ora_ff *ff, int ti, int tj, double qi, double qj, double r) {
  if (r < ff->r_min) r = ff->r_min;
  const double Si = ff->solpar[ti] + ff->qsolpar * fabs(qi);
  const double Sj = ff->solpar[tj] + ff->qsolpar * fabs(qj);
  const double vdw = vdw_hb(ff, ti, tj, r);
  const double elec = ff->coulomb * qi * qj / (dielectric(ff, r) * r);
  const double desolv = (Si * ff->vol[tj] + Sj * ff->vol[ti]) * gauss(ff, r);
  return vdw + elec + desolv;
}

static double distance3(const double *a, const double *b) {
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

static double intra_energy(const prep_t *P, const ora_ff *ff, const double *X) {
  double s = 0;
  for (int64_t p = 0; p < P->n_pairs; p++) {
    const int i = P->pi[p], j = P->pj[p];
    s += oracle_pair_energy(ff, P->type[i], P->type[j], P->q[i], P->q[j], distance3(X + 3 * i, X + 3 * j));
  }
  return s;
}

int oracle_intra_xyz(const ora_ligand *lig, const ora_ff *ff, const double *xyz, double *out) {
  prep_t P;
  int rc = prep_ligand(lig, ff->n_types, &P);
  if (rc) return rc;
  *out = intra_energy(&P, ff, xyz);
  prep_free(&P);
  return ORA_OK;
}

int oracle_brute_inter(const ora_ff *ff, int n_lig, const double *lig_xyz, const int32_t *lig_type,
                       const double *lig_q, int n_rec, const double *rec_xyz, const int32_t *rec_type,
                       const double *rec_q, double *out) {
  double s = 0;
  for (int i = 0; i < n_lig; i++)
    for (int j = 0; j < n_rec; j++)
      s += oracle_pair_energy(ff, lig_type[i], rec_type[j], lig_q[i], rec_q[j],
                              distance3(lig_xyz + 3 * i, rec_xyz + 3 * j));
  *out = s;
  return ORA_OK;
}

/* ===================================================================================
 * Scoring of a batch of poses.
 * =================================================================================== */
static double score_one(const prep_t *P, const ora_grid *G, const ora_ff *ff, const float *g,
                        double *X, double *inter_out, double *intra_out) {
  if (!genes_finite(g, 7 + P->nt)) {
    if (inter_out) *inter_out = NAN;
    if (intra_out) *intra_out = NAN;
    return NAN;
  }
  build_pose(P, g, X);
  double inter = 0;
  for (int i = 0; i < P->n; i++) inter += atom_inter(G, X + 3 * i, P->type[i], P->q[i]);
  const double intra = intra_energy(P, ff, X);
  if (inter_out) *inter_out = inter;
  if (intra_out) *intra_out = intra;
  return inter + intra;
}

typedef struct {
  const ora_grid *G;
  const ora_ff *ff;
  const prep_t *preps;
  const int32_t *pose_ligand;
  const float *gen;
  int g_stride;
  int64_t lo, hi;
  double *E, *Ei, *Ea;
  int max_atoms;
} score_task;

static void *score_worker(void *arg) {
  score_task *t = arg;
  double *X = malloc(sizeof(double) * 3 * t->max_atoms);
  for (int64_t p = t->lo; p < t->hi; p++) {
    const int l = t->pose_ligand ? t->pose_ligand[p] : 0;
    double ei, ea;
    t->E[p] = score_one(&t->preps[l], t->G, t->ff, t->gen + (size_t)p * t->g_stride, X, &ei, &ea);
    if (t->Ei) t->Ei[p] = ei;
    if (t->Ea) t->Ea[p] = ea;
  }
  free(X);
  return NULL;
}

static int check_grid(const ora_grid *G, const ora_ff *ff) {
  if (!G || !G->maps) return fail(ORA_E_INVALID, "null grid");
  if (G->n_types != ff->n_types) return fail(ORA_E_INVALID, "grid/forcefield n_types mismatch");
  for (int d = 0; d < 3; d++)
    if (G->dims[d] < 2) return fail(ORA_E_INVALID, "grid dims must be >= 2");
  if (!(G->spacing > 0)) return fail(ORA_E_INVALID, "spacing must be > 0");
  return ORA_OK;
}

static int prep_all(const ora_ligand *ligs, int n_ligs, int n_types, prep_t **out, int *max_atoms) {
  prep_t *preps = calloc(n_ligs, sizeof(prep_t));
  *max_atoms = 1;
  for (int l = 0; l < n_ligs; l++) {
    int rc = prep_ligand(&ligs[l], n_types, &preps[l]);
    if (rc) {
      for (int k = 0; k < l; k++) prep_free(&preps[k]);
      free(preps);
      return rc;
    }
    if (preps[l].n > *max_atoms) *max_atoms = preps[l].n;
  }
  *out = preps;
  return ORA_OK;
}

int oracle_score_poses(const ora_grid *G, const ora_ff *ff, const ora_ligand *ligs, int n_ligs,
                       const int32_t *pose_ligand, const float *genotypes, int g_stride,
                       int64_t n_poses, double *energies, double *inter, double *intra, int n_threads) {
  int rc = check_grid(G, ff);
  if (rc) return rc;
  if (n_ligs < 1) return fail(ORA_E_INVALID, "n_ligs must be >= 1");
  if (n_poses < 0) return fail(ORA_E_INVALID, "n_poses must be >= 0");
  prep_t *preps;
  int max_atoms;
  rc = prep_all(ligs, n_ligs, ff->n_types, &preps, &max_atoms);
  if (rc) return rc;
  for (int l = 0; l < n_ligs; l++)
    if (g_stride < 7 + preps[l].nt) { rc = fail(ORA_E_INVALID, "g_stride too small"); goto done; }
  if (pose_ligand)
    for (int64_t p = 0; p < n_poses; p++)
      if (pose_ligand[p] < 0 || pose_ligand[p] >= n_ligs) { rc = fail(ORA_E_INVALID, "pose_ligand out of range"); goto done; }
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  {
    pthread_t th[256];
    score_task tasks[256];
    const int64_t chunk = (n_poses + n_threads - 1) / n_threads;
    for (int t = 0; t < n_threads; t++) {
      int64_t lo = t * chunk, hi = lo + chunk;
      if (lo > n_poses) lo = n_poses;
      if (hi > n_poses) hi = n_poses;
      tasks[t] = (score_task){G, ff, preps, pose_ligand, genotypes, g_stride, lo, hi, energies, inter, intra, max_atoms};
      pthread_create(&th[t], NULL, score_worker, &tasks[t]);
    }
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  }
done:
  for (int l = 0; l < n_ligs; l++) prep_free(&preps[l]);
  free(preps);
  return rc;
}

/* ===================================================================================
 * Grid maps (AutoGrid-like precomputation, Sec. V): at every node, a probe of each
 * ligand type against all receptor atoms; plus the electrostatic potential and the
 * charge-independent part of desolvation.
 * =================================================================================== */
typedef struct {
  const ora_ff *ff;
  int n_rec;
  const double *rx;
  const int32_t *rt;
  const double *rq;
  int dims[3];
  double origin[3], h;
  float *maps;
  int z0, z1;
  const double *A, *B;   /* [n_types][n_types] repulsive / attractive coefficients */
} map_task;

/* the van der Waals / hydrogen-bond coefficients of a type pair (same values as
 * vdw_hb computes inline) */
static void vdw_coeffs(const ora_ff *ff, int ti, int tj, double *A, double *B) {
  const double req = 0.5 * (ff->Rii[ti] + ff->Rii[tj]);
  const double eps = sqrt(ff->epsii[ti] * ff->epsii[tj]);
  if (ff->hbond[ti * ff->n_types + tj]) { *A = 5.0 * eps * pow(req, 12); *B = 6.0 * eps * pow(req, 10); }
  else { *A = eps * pow(req, 12); *B = 2.0 * eps * pow(req, 6); }
}

static void *map_worker(void *arg) {
  map_task *t = arg;
  const ora_ff *ff = t->ff;
  const int NT = ff->n_types;
  const size_t nx = t->dims[0], ny = t->dims[1], nz = t->dims[2];
  double *T = malloc(sizeof(double) * NT);
  for (int k = t->z0; k < t->z1; k++)
    for (size_t j = 0; j < ny; j++)
      for (size_t i = 0; i < nx; i++) {
        const double p[3] = {t->origin[0] + i * t->h, t->origin[1] + j * t->h, t->origin[2] + k * t->h};
        double E = 0, D = 0;
        for (int a = 0; a < NT; a++) T[a] = 0;
        for (int r = 0; r < t->n_rec; r++) {
          double dist = distance3(p, t->rx + 3 * r);
          if (dist < ff->r_min) dist = ff->r_min;
          const int tr = t->rt[r];
          const double qr = t->rq[r];
          const double G = gauss(ff, dist);
          const double Sr = ff->solpar[tr] + ff->qsolpar * fabs(qr);
          const double r6 = pow(dist, 6), r10 = pow(dist, 10), r12 = pow(dist, 12);
          for (int a = 0; a < NT; a++) {
            const double A = t->A[a * NT + tr], B = t->B[a * NT + tr];
            double vdw = ff->hbond[a * NT + tr] ? A / r12 - B / r10 : A / r12 - B / r6;
            if (vdw > ff->e_cap) vdw = ff->e_cap;
            T[a] += vdw + (ff->solpar[a] * ff->vol[tr] + Sr * ff->vol[a]) * G;
          }
          E += ff->coulomb * qr / (dielectric(ff, dist) * dist);
          D += ff->qsolpar * ff->vol[tr] * G;
        }
        const size_t node = ((size_t)k * ny + j) * nx + i, plane = nx * ny * nz;
        for (int a = 0; a < NT; a++) t->maps[a * plane + node] = (float)(T[a] < ff->map_cap ? T[a] : ff->map_cap);
        double Ec = E;
        if (Ec > ff->map_cap) Ec = ff->map_cap;
        if (Ec < -ff->map_cap) Ec = -ff->map_cap;
        t->maps[NT * plane + node] = (float)Ec;
        t->maps[(NT + 1) * plane + node] = (float)(D < ff->map_cap ? D : ff->map_cap);
      }
  free(T);
  return NULL;
}

int oracle_build_maps(const ora_ff *ff, int n_rec, const double *rec_xyz, const int32_t *rec_type,
                      const double *rec_q, const int dims[3], const double origin[3], double spacing,
                      float *maps_out, int n_threads) {
  for (int d = 0; d < 3; d++)
    if (dims[d] < 2) return fail(ORA_E_INVALID, "grid dims must be >= 2");
  for (int r = 0; r < n_rec; r++)
    if (rec_type[r] < 0 || rec_type[r] >= ff->n_types) return fail(ORA_E_INVALID, "receptor type out of range");
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  if (n_threads > dims[2]) n_threads = dims[2];
  const int NT = ff->n_types;
  double *A = malloc(sizeof(double) * NT * NT), *B = malloc(sizeof(double) * NT * NT);
  for (int a = 0; a < NT; a++)
    for (int b = 0; b < NT; b++) vdw_coeffs(ff, a, b, &A[a * NT + b], &B[a * NT + b]);
  pthread_t th[256];
  map_task tasks[256];
  for (int t = 0; t < n_threads; t++) {
    tasks[t] = (map_task){ff, n_rec, rec_xyz, rec_type, rec_q, {dims[0], dims[1], dims[2]},
                          {origin[0], origin[1], origin[2]}, spacing, maps_out,
                          (int)((int64_t)dims[2] * t / n_threads), (int)((int64_t)dims[2] * (t + 1) / n_threads),
                          A, B};
    pthread_create(&th[t], NULL, map_worker, &tasks[t]);
  }
  for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  free(A); free(B);
  return ORA_OK;
}

/* ===================================================================================
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128
 * multiplications whose halves are mixed with the other counter words and the
 * round key; the key is bumped by two Weyl constants between rounds.
 * =================================================================================== */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    const unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One stream of 32-bit draws per (individual, generation, ligand, purpose):
 * draw n is half (n & 1: 0 low, 1 high) of 64-bit word (n >> 1) & 3 of the block
 * with counter (individual, generation, ligand, purpose << 32 | n >> 3), key (seed, 0). */
enum { PURPOSE_INIT = 1, PURPOSE_SELECT = 2, PURPOSE_CROSS = 3 };

typedef struct {
  uint64_t key[2];
  uint64_t c0, c1, c2, purpose;
  uint64_t n;
} stream_t;

static stream_t stream_make(uint64_t seed, uint64_t indiv, uint64_t gen, uint64_t lig, uint64_t purpose) {
  stream_t s = {{seed, 0}, indiv, gen, lig, purpose, 0};
  return s;
}

static uint32_t draw_u32(stream_t *s) {
  const uint64_t ctr[4] = {s->c0, s->c1, s->c2, (s->purpose << 32) | (s->n >> 3)};
  uint64_t out[4];
  oracle_philox4x64(ctr, s->key, out);
  const uint64_t w = out[(s->n >> 1) & 3];
  const uint32_t v = (s->n & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
  s->n++;
  return v;
}

/* uniform in [0,1) on the 2^-24 lattice */
static double draw_unit(stream_t *s) { return (double)(draw_u32(s) >> 8) / 16777216.0; }

/* uniform integer in [0, n) */
static int draw_index(stream_t *s, int n) { return (int)(((uint64_t)draw_u32(s) * (uint64_t)n) >> 32); }

/* ===================================================================================
 * Differential evolution, DE/rand/1/bin.
 * =================================================================================== */
static const double PI = 3.14159265358979323846;

static void de_init_one(const ora_search_params *p, int n_tor, int lig_id, int i, int g_stride, float *row) {
  stream_t s = stream_make(p->seed, (uint64_t)i, 0, (uint64_t)lig_id, PURPOSE_INIT);
  for (int j = 0; j < g_stride; j++) row[j] = 0.0f;
  for (int d = 0; d < 3; d++) {
    const double u = draw_unit(&s);
    row[d] = (float)(p->box_lo[d] + u * (p->box_hi[d] - p->box_lo[d]));
  }
  /* orientation: a point drawn uniformly in the unit 4-ball (rejection from the
   * cube), whose direction is uniform on the rotation group */
  row[3] = 1.0f; row[4] = row[5] = row[6] = 0.0f;
  for (int tries = 0; tries < 64; tries++) {
    double v[4], nn = 0;
    for (int c = 0; c < 4; c++) { v[c] = 2.0 * draw_unit(&s) - 1.0; nn += v[c] * v[c]; }
    if (nn > 0.0 && nn <= 1.0) {
      for (int c = 0; c < 4; c++) row[3 + c] = (float)v[c];
      break;
    }
  }
  for (int k = 0; k < n_tor; k++) {
    const double u = draw_unit(&s);
    row[7 + k] = (float)(u * (2.0 * PI) - PI);
  }
}

static int pick_partner(stream_t *s, int pop, const int *taken, int n_taken) {
  for (int tries = 0; tries < 64; tries++) {
    const int r = draw_index(s, pop);
    int clash = 0;
    for (int k = 0; k < n_taken; k++) clash |= (r == taken[k]);
    if (!clash) return r;
  }
  for (int r = (taken[0] + 1) % pop;; r = (r + 1) % pop) {
    int clash = 0;
    for (int k = 0; k < n_taken; k++) clash |= (r == taken[k]);
    if (!clash) return r;
  }
}

static void de_trial_one(const ora_search_params *p, int n_tor, int lig_id, int gen, int i, int g_stride,
                         const float *pop, float *trial) {
  const int P = p->pop_size, n_genes = 7 + n_tor;
  stream_t s = stream_make(p->seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig_id, PURPOSE_SELECT);
  int taken[4] = {i, 0, 0, 0};
  taken[1] = pick_partner(&s, P, taken, 1);
  taken[2] = pick_partner(&s, P, taken, 2);
  taken[3] = pick_partner(&s, P, taken, 3);
  const int jrand = draw_index(&s, n_genes);
  const float *xi = pop + (size_t)i * g_stride, *x1 = pop + (size_t)taken[1] * g_stride;
  const float *x2 = pop + (size_t)taken[2] * g_stride, *x3 = pop + (size_t)taken[3] * g_stride;
  stream_t sc = stream_make(p->seed, (uint64_t)i, (uint64_t)gen, (uint64_t)lig_id, PURPOSE_CROSS);
  for (int j = 0; j < g_stride; j++) trial[j] = 0.0f;
  for (int j = 0; j < n_genes; j++) {
    const double u = draw_unit(&sc);
    float v;
    if (u < p->CR || j == jrand) {
      const double diff = (double)x2[j] - (double)x3[j];
      const double step = p->F * diff;
      v = (float)((double)x1[j] + step);
    } else {
      v = xi[j];
    }
    if (j < 3) {
      if ((double)v < p->box_lo[j]) v = (float)p->box_lo[j];
      if ((double)v > p->box_hi[j]) v = (float)p->box_hi[j];
    } else if (j >= 7) {
      double w = (double)v;
      if (w > PI) w -= 2.0 * PI;
      else if (w <= -PI) w += 2.0 * PI;
      v = (float)w;
    }
    trial[j] = v;
  }
}

static int check_params(const ora_search_params *p) {
  if (p->pop_size < 4) return fail(ORA_E_INVALID, "pop_size must be >= 4");
  if (p->n_generations < 0) return fail(ORA_E_INVALID, "n_generations must be >= 0");
  for (int d = 0; d < 3; d++)
    if (!(p->box_lo[d] <= p->box_hi[d])) return fail(ORA_E_INVALID, "empty translation box");
  return ORA_OK;
}

int oracle_de_init(const ora_ligand *lig, const ora_search_params *p, int lig_id, int g_stride, float *population) {
  int rc = check_params(p);
  if (rc) return rc;
  if (g_stride < 7 + lig->n_torsions) return fail(ORA_E_INVALID, "g_stride too small");
  for (int i = 0; i < p->pop_size; i++)
    de_init_one(p, lig->n_torsions, lig_id, i, g_stride, population + (size_t)i * g_stride);
  return ORA_OK;
}

int oracle_de_trials(const ora_ligand *lig, const ora_search_params *p, int lig_id, int generation, int g_stride,
                     const float *population, float *trials) {
  int rc = check_params(p);
  if (rc) return rc;
  if (g_stride < 7 + lig->n_torsions) return fail(ORA_E_INVALID, "g_stride too small");
  for (int i = 0; i < p->pop_size; i++)
    de_trial_one(p, lig->n_torsions, lig_id, generation, i, g_stride, population, trials + (size_t)i * g_stride);
  return ORA_OK;
}

typedef struct {
  const ora_grid *G;
  const ora_ff *ff;
  const prep_t *preps;
  const ora_search_params *p;
  int g_stride;
  float *population;
  double *pop_energy;
  float *best_genotype;
  double *best_energy;
  const double *target;
  int32_t *gen_reached;
  int next;           /* next ligand to take (shared, under lock) */
  int n_ligs;
  pthread_mutex_t lock;
  int max_atoms;
} search_ctx;

static void search_ligand(search_ctx *c, int l) {
  const prep_t *P = &c->preps[l];
  const ora_search_params *p = c->p;
  const int NP = p->pop_size, S = c->g_stride;
  float *pop = c->population + (size_t)l * NP * S;
  double *E = c->pop_energy + (size_t)l * NP;
  float *trials = malloc(sizeof(float) * (size_t)NP * S);
  double *Et = malloc(sizeof(double) * NP);
  double *X = malloc(sizeof(double) * 3 * c->max_atoms);
  if (p->init) {
    for (int i = 0; i < NP; i++) de_init_one(p, P->nt, l, i, S, pop + (size_t)i * S);
    for (int i = 0; i < NP; i++) E[i] = score_one(P, c->G, c->ff, pop + (size_t)i * S, X, NULL, NULL);
  }
  int reached = -1;
  if (c->gen_reached && !p->init) reached = c->gen_reached[l];
  const double tgt = c->target ? c->target[l] : -INFINITY;
#define POP_BEST_REACHES(gdone)                                              \
  do {                                                                       \
    if (c->target && reached < 0) {                                          \
      for (int i_ = 0; i_ < NP; i_++)                                        \
        if (E[i_] <= tgt) { reached = (gdone); break; }                      \
    }                                                                        \
  } while (0)
  POP_BEST_REACHES(p->first_generation);
  for (int g = p->first_generation; g < p->first_generation + p->n_generations; g++) {
    for (int i = 0; i < NP; i++) de_trial_one(p, P->nt, l, g, i, S, pop, trials + (size_t)i * S);
    for (int i = 0; i < NP; i++) Et[i] = score_one(P, c->G, c->ff, trials + (size_t)i * S, X, NULL, NULL);
    for (int i = 0; i < NP; i++)
      if (Et[i] <= E[i]) {
        memcpy(pop + (size_t)i * S, trials + (size_t)i * S, sizeof(float) * S);
        E[i] = Et[i];
      }
    POP_BEST_REACHES(g + 1);
  }
#undef POP_BEST_REACHES
  int bi = 0;
  for (int i = 1; i < NP; i++)
    if (E[i] < E[bi]) bi = i;
  memcpy(c->best_genotype + (size_t)l * S, pop + (size_t)bi * S, sizeof(float) * S);
  c->best_energy[l] = E[bi];
  if (c->gen_reached) c->gen_reached[l] = reached;
  free(trials); free(Et); free(X);
}

static void *search_worker(void *arg) {
  search_ctx *c = arg;
  for (;;) {
    pthread_mutex_lock(&c->lock);
    const int l = c->next < c->n_ligs ? c->next++ : -1;
    pthread_mutex_unlock(&c->lock);
    if (l < 0) break;
    search_ligand(c, l);
  }
  return NULL;
}

int oracle_search(const ora_grid *G, const ora_ff *ff, const ora_ligand *ligs, int n_ligs,
                  const ora_search_params *p, int g_stride, float *population, double *pop_energy,
                  float *best_genotype, double *best_energy, const double *target, int32_t *gen_reached,
                  int n_threads) {
  int rc = check_grid(G, ff);
  if (rc) return rc;
  rc = check_params(p);
  if (rc) return rc;
  if (n_ligs < 1) return fail(ORA_E_INVALID, "n_ligs must be >= 1");
  prep_t *preps;
  int max_atoms;
  rc = prep_all(ligs, n_ligs, ff->n_types, &preps, &max_atoms);
  if (rc) return rc;
  for (int l = 0; l < n_ligs; l++)
    if (g_stride < 7 + preps[l].nt) { rc = fail(ORA_E_INVALID, "g_stride too small"); goto done; }
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  {
    search_ctx c = {G, ff, preps, p, g_stride, population, pop_energy, best_genotype, best_energy,
                    target, gen_reached, 0, n_ligs, PTHREAD_MUTEX_INITIALIZER, max_atoms};
    pthread_t th[256];
    for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, search_worker, &c);
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  }
done:
  for (int l = 0; l < n_ligs; l++) prep_free(&preps[l]);
  free(preps);
  return rc;
}
