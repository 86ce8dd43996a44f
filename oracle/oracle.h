/* oracle.h -- plain FP64 CPU oracle for the muDock docking hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark call into this library.  It shares no code with
 * the HIP library: it is written from the paper (Sec. V, Algorithms 1 and 2) and
 * the readings recorded beside it, in plain, slow, obviously-checkable loops.
 *
 * Every floating-point computation is IEEE binary64 without contraction
 * (built with -ffp-contract=off, no fast-math).  Inputs arrive as float32 values
 * (coordinates, charges, maps, genotypes) or as doubles holding float32 values
 * (force-field data), and are promoted exactly.
 */
#ifndef DOCK_ORACLE_H
#define DOCK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_E_INVALID = 1, ORA_E_NOMEM = 2 };

/* Force-field data: per-type table plus the constants of the pair terms. */
typedef struct {
  int n_types;
  const double *Rii, *epsii, *vol, *solpar;  /* [n_types] */
  const uint8_t *hbond;                      /* [n_types*n_types], 1 -> 12-10 */
  double coulomb, diel_A, diel_eps0, diel_lambda, diel_k;
  double sigma, qsolpar, e_cap, r_min, map_cap;
} ora_ff;

/* Grid maps: [n_types+2][nz][ny][nx] float32, x fastest; map n_types is the
 * electrostatic map, n_types+1 the desolvation map.  Node (i,j,k) sits at
 * origin + (i,j,k)*spacing. */
typedef struct {
  int n_types;
  int dims[3];
  double origin[3];
  double spacing;
  const float *maps;
} ora_grid;

/* One ligand: reference conformation, types, charges, bond tree, rotatable bonds. */
typedef struct {
  int n_atoms, n_torsions;
  const float *xyz;            /* [n_atoms][3] */
  const int32_t *type;         /* [n_atoms] */
  const float *charge;         /* [n_atoms] */
  const int32_t *bonds;        /* [n_atoms-1][2] */
  const int32_t *torsion_bonds;/* [n_torsions] indices into bonds */
} ora_ligand;

const char *oracle_last_error(void);

/* Preprocessing outputs for tests: non-bonded pair list, rigid fragment ids and
 * per-torsion moving-atom masks.  pairs: [max_pairs][2]; frag: [n_atoms];
 * moving: [n_torsions][n_atoms] (1 if the atom is rotated by that torsion);
 * axis: [n_torsions][2] oriented (a,b), a nearer the root.  Returns the number
 * of pairs in *n_pairs. */
int oracle_ligand_info(const ora_ligand *lig, int n_types, int32_t *pairs, int64_t max_pairs,
                       int64_t *n_pairs, int32_t *frag, uint8_t *moving, int32_t *axis);

/* Pose build only: xyz_out [n_atoms][3] in Angstrom. */
int oracle_pose(const ora_ligand *lig, int n_types, const float *genotype, double *xyz_out);

/* Energies of n_poses poses.  pose_ligand may be NULL (all ligand 0).
 * energies[n_poses] total; inter/intra may be NULL. */
int oracle_score_poses(const ora_grid *grid, const ora_ff *ff, const ora_ligand *ligs, int n_ligs,
                       const int32_t *pose_ligand, const float *genotypes, int g_stride,
                       int64_t n_poses, double *energies, double *inter, double *intra,
                       int n_threads);

/* Inter energy of explicit atom positions (for interpolation pins). */
int oracle_inter_atoms(const ora_grid *grid, int n_atoms, const double *xyz, const int32_t *type,
                       const double *charge, double *per_atom);

/* Intra energy of explicit atom positions of one ligand. */
int oracle_intra_xyz(const ora_ligand *lig, const ora_ff *ff, const double *xyz, double *out);

/* Pair potential between two atoms at distance r (for closed-form pins). */
double oracle_pair_energy(const ora_ff *ff, int ti, int tj, double qi, double qj, double r);

/* Brute-force ligand-receptor energy of explicit positions (sum of the pair
 * potential over all ligand x receptor atom pairs, no grid). */
int oracle_brute_inter(const ora_ff *ff, int n_lig, const double *lig_xyz, const int32_t *lig_type,
                       const double *lig_q, int n_rec, const double *rec_xyz,
                       const int32_t *rec_type, const double *rec_q, double *out);

/* Grid maps from a receptor: maps_out [n_types+2][nz][ny][nx] float32. */
int oracle_build_maps(const ora_ff *ff, int n_rec, const double *rec_xyz, const int32_t *rec_type,
                      const double *rec_q, const int dims[3], const double origin[3], double spacing,
                      float *maps_out, int n_threads);

/* Philox4x64-10 block function. */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

typedef struct {
  int pop_size, n_generations;
  uint64_t seed;
  double F, CR;                  /* float32 values */
  double box_lo[3], box_hi[3];   /* translation bounds */
  int init;                      /* 1: draw the initial population; 0: resume from the given one */
  int first_generation;          /* absolute index of the first generation run by this call */
} ora_search_params;

/* Initial population for ligand lig_id (pop_size rows of g_stride floats). */
int oracle_de_init(const ora_ligand *lig, const ora_search_params *p, int lig_id, int g_stride,
                   float *population);

/* Trial population of one generation, from a given population. */
int oracle_de_trials(const ora_ligand *lig, const ora_search_params *p, int lig_id, int generation,
                     int g_stride, const float *population, float *trials);

/* Plain differential evolution over n_ligs ligands (ligand l uses id l).
 * population [n_ligs][pop][g_stride] and pop_energy [n_ligs][pop] are in/out.
 * best_genotype [n_ligs][g_stride], best_energy [n_ligs] out.  target may be
 * NULL; gen_reached [n_ligs] (may be NULL) gets the number of completed
 * generations at which the population best first reached target, or -1. */
int oracle_search(const ora_grid *grid, const ora_ff *ff, const ora_ligand *ligs, int n_ligs,
                  const ora_search_params *p, int g_stride, float *population, double *pop_energy,
                  float *best_genotype, double *best_energy, const double *target,
                  int32_t *gen_reached, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
