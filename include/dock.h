/* dock.h -- C ABI of the MI355X (gfx950) docking hot path.
 *
 * The problem follows the muDock mini-app of "Towards High-Performance and
 * Portable Molecular Docking on CPUs through Vectorization" (arXiv 2509.12232):
 *   - a receptor whose fixed structure is precomputed into 3-D grid maps, one per
 *     ligand atom type plus electrostatic and desolvation maps (Sec. V);
 *   - ligands made of typed, charged atoms joined by a bond tree with rotatable
 *     bonds (Sec. V, Algorithm 1);
 *   - a pose (individual) = translation + orientation + one angle per rotatable
 *     bond (Sec. II, Sec. V);
 *   - its score = inter energy (map lookups for atoms near the protein) + intra
 *     energy (ligand atom pairs), Sec. V, Algorithm 2;
 *   - an evolutionary search for the best-scoring pose with the score as fitness
 *     (Sec. V), here plain differential evolution.
 *
 * Conventions for every entry point:
 *   - Units: Angstrom, kcal/mol, elementary charge, radians.
 *   - Every call returns a dock_status; on failure dock_last_error() holds a
 *     message (thread-local, valid until the next dock_* call on that thread).
 *   - Argument validation happens on the host before anything is enqueued; a
 *     failed validation enqueues nothing.
 *   - "device" pointers are HIP device memory of the handle's device; "host"
 *     pointers are ordinary host memory.  create_* calls copy what they keep, so
 *     the caller may free its inputs on return.  Outputs are caller-allocated.
 *     The library never frees caller memory.
 *   - stream is a hipStream_t (NULL = the legacy default stream) of the handle's
 *     device.  Compute calls only enqueue work; the caller synchronises.
 *   - Handles are immutable after creation, so concurrent compute calls on
 *     different streams are allowed.  Destroy a handle only after the work that
 *     uses it has completed.
 */
#ifndef DOCK_H
#define DOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DOCK_OK = 0,
  DOCK_E_INVALID = 1,     /* bad argument or descriptor */
  DOCK_E_NOMEM = 2,       /* device allocation failed */
  DOCK_E_DEVICE = 3,      /* HIP runtime error */
  DOCK_E_UNSUPPORTED = 4  /* valid input outside what this build supports (e.g. > 96 atoms) */
} dock_status;

/* Message for the last failure on this thread ("" if none). */
const char *dock_last_error(void);

/* ABI version, incremented on incompatible changes. */
int32_t dock_version(void);

typedef struct dock_pocket dock_pocket;    /* maps + force field, on one device */
typedef struct dock_ligands dock_ligands;  /* preprocessed ligand set, on the pocket's device */

/* Force-field data (host pointers, copied).  The paper names the four terms
 * (electrostatic, van der Waals, hydrogen bond, desolvation; Algorithm 2) but
 * gives no constants, so all of them are inputs.  Pair potential between atoms
 * i, j at distance r' = max(r, r_min):
 *   vdW/H-bond: min(A r'^-12 - B r'^-p, e_cap), r_eq = (Rii_i+Rii_j)/2,
 *               eps = sqrt(epsii_i epsii_j); p = 6: A = eps r_eq^12, B = 2 eps r_eq^6;
 *               p = 10 when hbond[t_i*n_types+t_j]: A = 5 eps r_eq^12, B = 6 eps r_eq^10
 *   electrostatic: coulomb q_i q_j / (eps(r') r'),
 *               eps(r) = diel_A + (diel_eps0 - diel_A) / (1 + diel_k exp(-diel_lambda (diel_eps0 - diel_A) r))
 *   desolvation: (S_i vol_j + S_j vol_i) exp(-r'^2 / (2 sigma^2)), S = solpar + qsolpar |q|
 * e_cap (the cap on the repulsive term), r_min, sigma and map_cap must be
 * positive and finite.  map_cap clamps the maps built by
 * dock_create_pocket_from_receptor. */
typedef struct {
  int32_t n_types;                          /* 1..32 */
  const float *Rii, *epsii, *vol, *solpar;  /* [n_types] */
  const uint8_t *hbond;                     /* [n_types*n_types], symmetric, 0 or 1 */
  float coulomb, diel_A, diel_eps0, diel_lambda, diel_k;
  float sigma, qsolpar, e_cap, r_min, map_cap;
} dock_forcefield;

/* Grid geometry: dims[d] >= 2 nodes per axis; node (i,j,k) at origin + (i,j,k)*spacing.
 * Maps are float32 [n_types+2][nz][ny][nx], x fastest: maps 0..n_types-1 are the
 * per-type maps, map n_types the electrostatic map (per unit charge), map
 * n_types+1 the desolvation map (per unit |charge|). */
typedef struct {
  int32_t n_types;
  int32_t dims[3];
  float origin[3];
  float spacing;
} dock_grid;

/* Device layout of the maps read by the scoring kernel (the ABI layout above is
 * always kept as well).  The packed layouts duplicate neighbouring nodes so the
 * eight corners of a grid cell come from fewer cache lines:
 *   DOCK_LAYOUT_LINEAR  the ABI layout itself (1x memory);
 *   DOCK_LAYOUT_ZPAIR   node pairs along z, x-neighbours adjacent (2x);
 *   DOCK_LAYOUT_YZQUAD  node quads over y and z, x-neighbours adjacent (4x);
 *   DOCK_LAYOUT_QUADLINE the yz-quads cut into 128-byte lines of eight
 *                       x-consecutive quads that overlap by one, so a cell
 *                       never straddles a line; the electrostatic and
 *                       desolvation maps stored as E + D and E - D, of which
 *                       an atom reads the one of its charge's sign (q E + |q| D
 *                       is q (E + D) for q >= 0 and q (E - D) for q < 0): two
 *                       cache lines per lookup (about 4.6x);
 *   DOCK_LAYOUT_PAIRLINE one copy per (atom type, charge sign), each node's
 *                       type quad followed by its E + D or E - D quad, four
 *                       x-consecutive nodes to a 128-byte line (consecutive
 *                       lines share one node): one cache line per lookup
 *                       (about 14x for 12 types);
 *   DOCK_LAYOUT_AUTO    the pair-line layout if its copy fits 8 GiB, else the
 *                       quad-line layout if its copy fits 512 MiB, else z-pair.
 * Results do not depend on the layout beyond float rounding of the same terms;
 * the quad-line and pair-line layouts give the same bits. */
enum {
  DOCK_LAYOUT_AUTO = -1,
  DOCK_LAYOUT_LINEAR = 0,
  DOCK_LAYOUT_ZPAIR = 1,
  DOCK_LAYOUT_YZQUAD = 2,
  DOCK_LAYOUT_QUADLINE = 3,
  DOCK_LAYOUT_PAIRLINE = 4
};

/* Create a pocket from precomputed maps (Sec. V: maps precomputed around the
 * receptor, AutoGrid-style).  maps: host (maps_on_device = 0) or device (1)
 * pointer in the layout above.  layout: one of DOCK_LAYOUT_*.  device: HIP
 * device ordinal.  *out receives the handle.  Synchronous.  Errors:
 * DOCK_E_INVALID (null pointers, n_types mismatch, dims < 2, spacing <= 0, map
 * larger than 2^31 floats, unknown layout, a quad-line or pair-line map of more
 * than 2^31 elements), DOCK_E_NOMEM, DOCK_E_DEVICE. */
dock_status dock_create_pocket(const dock_grid *grid, const float *maps, int32_t maps_on_device,
                               const dock_forcefield *ff, int32_t layout, int32_t device, dock_pocket **out);

/* Create a pocket by building the maps on the GPU from receptor atoms (the
 * AutoGrid-like step of Sec. V: a probe of each type at every node, summed over
 * all receptor atoms with the pair potential above; the electrostatic map is the
 * Coulomb term per unit probe charge, the desolvation map the qsolpar part per
 * unit |probe charge|; type and desolvation maps are clamped above at map_cap,
 * the electrostatic map to [-map_cap, map_cap]).  xyz [n_atoms][3], type
 * [n_atoms], charge [n_atoms]: host pointers.  layout as dock_create_pocket.
 * Synchronous: returns when the maps are built.  Errors as dock_create_pocket,
 * plus receptor types out of range. */
dock_status dock_create_pocket_from_receptor(const dock_grid *grid, const dock_forcefield *ff,
                                             int32_t n_atoms, const float *xyz, const int32_t *type,
                                             const float *charge, int32_t layout, int32_t device,
                                             dock_pocket **out);

/* The DOCK_LAYOUT_* (never AUTO) the pocket's scoring kernel reads. */
dock_status dock_pocket_layout(const dock_pocket *pocket, int32_t *layout);

/* Copy the pocket's maps (layout above) into maps_out: a device pointer of
 * (n_types+2)*nx*ny*nz floats.  Enqueued on stream. */
dock_status dock_pocket_maps(const dock_pocket *pocket, float *maps_out, void *stream);

dock_status dock_destroy_pocket(dock_pocket *pocket);

/* One ligand (host pointers, copied).  Atom 0 is the root: each rotatable bond
 * moves the side away from atom 0 (Algorithm 1, rotamer fragments). */
typedef struct {
  int32_t n_atoms;              /* 1..96 */
  int32_t n_torsions;           /* 0..32 */
  const float *xyz;             /* [n_atoms][3] reference conformation */
  const int32_t *type;          /* [n_atoms] in [0, n_types) */
  const float *charge;          /* [n_atoms] */
  const int32_t *bonds;         /* [n_atoms-1][2] distinct bonds that must form a tree: bonds that
                                   close a ring (and so leave some atom unconnected) are
                                   DOCK_E_UNSUPPORTED; a repeated or self bond is DOCK_E_INVALID */
  const int32_t *torsion_bonds; /* [n_torsions] distinct indices into bonds, neither end of degree 1 */
} dock_ligand_desc;

/* Preprocess a ligand set for a pocket: root at atom 0, ligand origin at the
 * centroid of the reference conformation, intra pairs = atom pairs at least four
 * bonds apart that lie in different rigid fragments (Algorithm 2's pair loop; no
 * distance cutoff).  Errors: DOCK_E_INVALID (bonds out of range, repeated or
 * joining an atom to itself, torsion on a terminal or repeated bond, type out
 * of range, non-finite input, n_ligands < 1), DOCK_E_UNSUPPORTED (> 96 atoms,
 * > 32 torsions, bonds that close a ring), DOCK_E_NOMEM, DOCK_E_DEVICE. */
dock_status dock_create_ligands(const dock_pocket *pocket, const dock_ligand_desc *ligands,
                                int32_t n_ligands, dock_ligands **out);

/* Number of intra pairs of ligand lig (host query). */
dock_status dock_ligand_pair_count(const dock_ligands *ligs, int32_t lig, int32_t *n_pairs);

dock_status dock_destroy_ligands(dock_ligands *ligs);

/* Score n_poses poses (Algorithms 1 and 2 for each): pose p of ligand
 * pose_ligand[p] is built from genotypes[p*g_stride ...] = t(3), q(4) = (w,x,y,z)
 * (normalised here; |q|^2 < 1e-24 means identity), theta(n_torsions) in the
 * ligand's torsion order; then energies[p] = inter + intra in kcal/mol, FP32.
 * Inter: each atom inside the closed grid box adds the trilinear interpolation
 * of T_type + q E + |q| D; atoms outside add 0.
 * pose_ligand: device [n_poses] or NULL (every pose is ligand 0); an index out of
 * range yields NaN for that pose.  genotypes: device [n_poses][g_stride], g_stride
 * >= 7 + the largest n_torsions of the set.  energies: device [n_poses].  A pose
 * with a non-finite gene scores NaN.  n_poses = 0 is a no-op.
 * Errors: DOCK_E_INVALID (null handles/pointers, g_stride too small, handles of
 * different devices), DOCK_E_DEVICE (launch failure). */
dock_status dock_score_poses(const dock_pocket *pocket, const dock_ligands *ligs,
                             const int32_t *pose_ligand, const float *genotypes, int32_t g_stride,
                             int64_t n_poses, float *energies, void *stream);

/* Launch shape of dock_score_poses (a tuning knob; energies are bit-identical
 * for every shape).  Poses are scored in blocks of 64, one per lane; split =
 * 1, 2, 4 or 8 wavefronts build and score a block together, sharing its LDS (3
 * floats per atom per pose) and splitting each pose's atoms and pair records,
 * so more wavefronts stay resident for large ligands; 0 restores the automatic
 * choice by the set's largest ligand.  Process-wide; takes effect at the next
 * call.  Errors: DOCK_E_INVALID for any other value. */
dock_status dock_score_set_split(int32_t split);

/* The split dock_score_poses uses for ligand set ligs (the setting above, or
 * the automatic choice).  Errors: DOCK_E_INVALID (null argument). */
dock_status dock_score_split(const dock_ligands *ligs, int32_t *split);

/* Differential evolution (DE/rand/1/bin, greedy selection) as the evolutionary
 * search of Sec. V.  Random draws come from Philox4x64-10 (Salmon et al., SC'11)
 * with key (seed, 0) and counter (individual, generation, ligand, purpose << 32 |
 * block); ligand l of the set uses ligand id l. */
typedef struct dock_mlp dock_mlp;          /* learned proposal network, on one device */

typedef struct {
  int32_t pop_size;         /* >= 4 */
  int32_t n_generations;    /* >= 0 */
  uint64_t seed;
  float F, CR;              /* differential weight, crossover rate */
  double box_lo[3], box_hi[3];  /* translation bounds (init range and clamp) */
  int32_t init;             /* 1: draw and score the initial population; 0: resume */
  int32_t first_generation; /* absolute index of the first generation this call runs */
  int32_t stop_at_target;   /* 1: a ligand stops once its population best is <= its target
                               (needs target and gen_reached); 0: run every generation */
  /* Learned proposal (not part of the paper's search; NULL = plain DE).  A
   * proposal round replaces each individual by dock_propose's proposal when the
   * proposal scores <= the individual (the search's own greedy rule).  Rounds run
   * right after the initial population (init = 1) and before every generation g
   * of the call that is a positive multiple of proposal_every (> 0) with g <
   * proposal_until -- absolute generation indices, so a search split into
   * resumed calls runs the same rounds as one call. */
  const dock_mlp *proposal;
  float proposal_step;      /* alpha_max of dock_propose, > 0 */
  int32_t proposal_every;   /* >= 0 (0: only the round after the initial population) */
  int32_t proposal_until;   /* generation bound of the later rounds */
} dock_search_params;

/* Initial population: rows [n_ligands][pop_size][g_stride] on device, genes
 * beyond 7 + n_torsions set to 0.  Translation uniform in the box, orientation a
 * uniform point of the unit 4-ball (uniform rotation once normalised), torsions
 * uniform in [-pi, pi). */
dock_status dock_de_init(const dock_ligands *ligs, const dock_search_params *params, int32_t g_stride,
                         float *population, void *stream);

/* Trial genotypes of one generation from a population (both device
 * [n_ligands][pop_size][g_stride]).  Gene j of trial i takes x_r1 + F (x_r2 - x_r3)
 * (binary64 arithmetic, rounded to float32) when a uniform draw is < CR or
 * j = j_rand, else x_i; translations are clamped to the box, torsions wrapped
 * once into (-pi, pi]. */
dock_status dock_de_trials(const dock_ligands *ligs, const dock_search_params *params, int32_t generation,
                           int32_t g_stride, const float *population, float *trials, void *stream);

/* Full search.  population [n_ligands][pop_size][g_stride] and pop_energy
 * [n_ligands][pop_size] (device) are in/out: with init = 1 they are overwritten
 * by the initial population and its scores; with init = 0 they are the state to
 * resume from (resume with first_generation = generations already run gives
 * exactly the result of one uninterrupted run).  best_genotypes
 * [n_ligands][g_stride] and best_energies [n_ligands] (device) receive the best
 * member of the final population (ties: lowest index).  target [n_ligands]
 * (device, may be NULL) and gen_reached [n_ligands] (device, may be NULL,
 * in/out): gen_reached records the number of completed generations at which the
 * population best first reached <= target (-1 while not reached; with init = 1
 * it is reset first).  Scratch (the trials and a gene-major copy of the
 * population, 2 x n_ligands x pop_size x g_stride floats) comes stream-ordered
 * from a memory pool the library keeps per device, which holds freed memory for
 * the next call until the process ends.  Errors as dock_score_poses plus bad
 * parameters, DOCK_E_NOMEM. */
dock_status dock_search(const dock_pocket *pocket, const dock_ligands *ligs, const dock_search_params *params,
                        int32_t g_stride, float *population, float *pop_energy, float *best_genotypes,
                        float *best_energies, const float *target, int32_t *gen_reached, void *stream);

/* The same search as dock_search, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It allocates nothing: its scratch (the bucket queue
 * counters, the trials and the gene-major population copy) lives in one fixed
 * area of DOCK_NO_ALLOC_SCRATCH_BYTES per device, reserved when the library's
 * device code is loaded on that device and held until the process ends.  The
 * area holds 256 bytes of counters and two arrays of n_ligands x pop_size x
 * g_stride floats, each rounded up to 256 bytes; a larger search is rejected
 * with DOCK_E_INVALID before anything is enqueued.  The size buckets run one
 * after another on stream (no side streams, no events), so results are the
 * same bits as dock_search's and only the overlap of buckets is lost.  Every
 * call on a device shares that device's area, which keeps the last call's
 * contents: calls that overlap on one device (on different streams, or from
 * different threads) race and give undefined results; calls ordered on one
 * stream are safe.  Arguments, in/out buffers and other errors as dock_search. */
#define DOCK_NO_ALLOC_SCRATCH_BYTES (64u << 20)
dock_status dock_search_no_alloc(const dock_pocket *pocket, const dock_ligands *ligs, const dock_search_params *params,
                                 int32_t g_stride, float *population, float *pop_energy, float *best_genotypes,
                                 float *best_energies, const float *target, int32_t *gen_reached, void *stream);

/* ---- Search plans: one captured graph per search -------------------------------
 * A plan holds its own scratch (trials and the gene-major population copy,
 * 2 x n_ligands x pop_size x g_stride floats, and the bucket queues) and the
 * whole search -- every bucket's persistent launch on the side streams, the
 * proposal rounds of a learned search, the joins -- captured once into a HIP
 * graph.  Launching it enqueues the same search as dock_search with the
 * arguments given at creation (the same pointers; their contents are read at
 * launch time), as one graph launch, with no allocation.  The launch shapes
 * in force at creation are the ones captured.  Launches of one plan must not
 * overlap (they share its scratch).  Errors as dock_search. */
typedef struct dock_search_plan dock_search_plan;
dock_status dock_search_plan_create(const dock_pocket *pocket, const dock_ligands *ligs,
                                    const dock_search_params *params, int32_t g_stride, float *population,
                                    float *pop_energy, float *best_genotypes, float *best_energies,
                                    const float *target, int32_t *gen_reached, dock_search_plan **out);
dock_status dock_search_plan_launch(dock_search_plan *plan, void *stream);
dock_status dock_search_plan_destroy(dock_search_plan *plan);

/* ---- Launch shapes of the search and their autotuner --------------------------
 * dock_search runs one persistent kernel per ligand-size bucket (atom counts
 * up to 16, 32, 48, 64, 96); a workgroup runs one ligand's search at a time.
 * Its shape: the split (1, 2, 4 or 8 wavefronts build and score a block of 64
 * individuals together, splitting their atoms and pair records and sharing
 * the block's LDS) and blocks per workgroup (1 up to 12 / split, 0 = chosen at
 * launch from the ligand count and the LDS residency).  Energies, and hence
 * search results, do not depend on the shape: every form sums the same
 * partial sums in the same order.  Shapes are launch configuration kept in
 * the ligand handle (the one exception to its immutability): set or tune them
 * while no search on the handle is in flight. */
#define DOCK_SEARCH_BUCKETS 5
typedef struct {
  int32_t max_atoms;        /* the bucket's upper atom count (read-only: 16, 32, 48, 64, 96) */
  int32_t split;            /* wavefronts per block of 64 individuals: 1, 2, 4 or 8 */
  int32_t blocks_per_group; /* 0..12 / split (0..1 for split 8) */
} dock_search_shape;

/* The handle's shapes, host dock_search_shape[DOCK_SEARCH_BUCKETS]: the
 * defaults, the ones set below, or the ones the autotuner fixed (timed or found
 * in its cache).  A search of a bucket whose shape is not fixed uses a cached
 * shape for its pocket and population size if there is one. */
dock_status dock_search_shapes(const dock_ligands *ligs, dock_search_shape *shapes);
/* Fixes the shapes (host array as above; max_atoms must match). */
dock_status dock_search_set_shapes(dock_ligands *ligs, const dock_search_shape *shapes);
/* Autotuner: for every non-empty bucket, times a search of tune_generations
 * generations (params' pop_size, seed, box) of the bucket's ligands for every
 * shape (split 1, 2, 4 and 8 x 1 up to 12 / split blocks, at most one block
 * per 64 individuals), warm-up run first,
 * with HIP events on stream, and fixes the fastest.  Results are cached for the
 * process under (device architecture and compute-unit count, map layout and
 * dimensions, bucket, its largest ligand, pop_size); a cached bucket is not
 * timed again, and dock_search uses cached shapes for handles whose shapes were
 * not fixed.  Synchronous; allocates and frees its own scratch state;
 * 1 <= tune_generations <= 1000. */
dock_status dock_search_autotune(const dock_pocket *pocket, dock_ligands *ligs, const dock_search_params *params,
                                 int32_t g_stride, int32_t tune_generations, void *stream);

/* The autotuner's cache as a file, so that a later process (on a device of the
 * same architecture and compute-unit count) uses tuned shapes without timing
 * them again.  dock_search_tune_save writes every cached shape of this process
 * to the text file at path (a header line, then one line per shape: arch n_cu
 * layout nx ny nz n_types bucket_upper largest_ligand pop split
 * blocks_per_group), replacing the file.  dock_search_tune_load reads such a
 * file and merges it into this process's cache (an entry with the same key is
 * replaced); if any line is malformed or out of range nothing is loaded.
 * Host-only; no device is touched.  Errors: DOCK_E_INVALID (null path, the
 * file cannot be written or read, a malformed line). */
dock_status dock_search_tune_save(const char *path);
dock_status dock_search_tune_load(const char *path);

/* ---- Learned proposal --------------------------------------------------------
 * An addition to the paper's method (whose search, Sec. V, has no learned
 * part): a perceptron 96 -> 256 -> 256 -> 32 with ReLU hidden layers proposes
 * genotype moves; every proposal is scored by the exact function and kept only
 * by the search's greedy rule, so plain DE remains the judge.  Matrix products
 * run on the matrix cores with bfloat16 operands (inputs, weights, hidden
 * activations and back-propagated errors rounded to nearest-even bfloat16) and
 * float32 accumulation; everything else is float32.
 *
 * Network input of an individual (96 features): 32 encoded genes -- (t_d - c_d) /
 * h_d for the box centre c and half-width h (0 where h = 0), the unit quaternion
 * with w >= 0 (identity for |q|^2 < 1e-24), theta_k / pi for k < min(n_torsions,
 * 25), zeros -- then the ligand's 64 descriptor features.  Output (32): a move
 * in the same encoding.
 *
 * Parameters, packed float32 (DOCK_MLP_PARAMS values): W1 [96][256] (input
 * major), b1 [256], W2 [256][256], b2 [256], W3 [256][32], b3 [32]; layer l
 * computes a_l = relu(a_{l-1} W_l + b_l), the last without relu. */
#define DOCK_MLP_IN 96
#define DOCK_MLP_HIDDEN 256
#define DOCK_MLP_OUT 32
#define DOCK_MLP_PARAMS 98848
#define DOCK_DESC 64
#define DOCK_MLP_MAX_BATCH 65536

/* New network on a device: He-uniform weights from seed (U(+-sqrt(6 / fan_in)),
 * the last layer scaled by 0.1), zero biases, zero Adam state. */
dock_status dock_mlp_create(int32_t device, uint64_t seed, dock_mlp **out);
dock_status dock_mlp_destroy(dock_mlp *net);
/* Replace the parameters (host float[DOCK_MLP_PARAMS], finite) and reset the
 * Adam state; synchronous. */
dock_status dock_mlp_set_params(dock_mlp *net, const float *params);
/* Copy the parameters out (host float[DOCK_MLP_PARAMS]); synchronous. */
dock_status dock_mlp_get_params(const dock_mlp *net, float *params);
/* y [n][32] = network(x [n][96]) (both device float32), n >= 0. */
dock_status dock_mlp_forward(const dock_mlp *net, const float *x, int64_t n, float *y, void *stream);
/* Loss (1/n) sum_i w_i sum_j (y_ij - target_ij)^2 of rows x [n][96] against
 * target [n][32] with weights w [n] (NULL = 1), and its gradients by
 * back-propagation: grads (device float[DOCK_MLP_PARAMS], packed like the
 * parameters) and loss (device float[1]).  1 <= n <= DOCK_MLP_MAX_BATCH.  Uses
 * the network's training workspace: calls on one network must not overlap. */
dock_status dock_mlp_gradients(dock_mlp *net, const float *x, const float *target, const float *weight, int32_t n,
                               float *grads, float *loss, void *stream);
/* n_steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * minibatches of `batch` rows of the data set x [n_data][96], target
 * [n_data][32], weight [n_data] (NULL = 1).  The rows trained on are
 * order[0 .. n_rows) (device int32, each in [0, n_data), checked on the host
 * with a synchronous copy), or 0 .. n_rows-1 when order is NULL (then n_rows <=
 * n_data); step s takes positions (s * batch) mod n_rows onwards.  n_rows must
 * be a multiple of batch, 1 <= batch <= DOCK_MLP_MAX_BATCH.  losses (device
 * float[n_steps], may be NULL) receives each step's loss before its update.
 * Calls on one network must not overlap. */
dock_status dock_mlp_train(dock_mlp *net, const float *x, const float *target, const float *weight, int64_t n_data,
                           const int32_t *order, int64_t n_rows, int32_t batch, int32_t n_steps, float lr,
                           float *losses, void *stream);

/* Descriptor of every ligand, out [n_ligands][64] (device float32): [0, 32) the
 * fraction of its atoms of each type; 32 torsions / 20; 33 atoms / 96; 34 mean
 * |charge|; 35 mean charge; 36 radius of gyration / 10 A; 37 intra pairs / 4096;
 * the rest 0. */
dock_status dock_ligand_descriptors(const dock_ligands *ligs, float *out, void *stream);

/* Network inputs x [n_ligands * pop_size][96] (device) of a population
 * [n_ligands][pop_size][g_stride] (device); params supplies pop_size and the box. */
dock_status dock_mlp_features(const dock_ligands *ligs, const dock_search_params *params, int32_t g_stride,
                              const float *population, float *x, void *stream);

/* Encoded moves out [n_ligands * pop_size][32] (device) from population `from` to
 * population `to` (same shape): (t_to - t_from) / h; q_to' - q_from' for the
 * canonical unit quaternions with q_to' of the sign nearer q_from';
 * wrap(theta_to - theta_from) / pi for the first min(n_torsions, 25); zeros. */
dock_status dock_mlp_moves(const dock_ligands *ligs, const dock_search_params *params, int32_t g_stride,
                           const float *from, const float *to, float *out, void *stream);

/* Training weights from a population's energies (one snapshot of a search's
 * energy trace), for dock_mlp_train's weight argument: individual i of ligand
 * l, of rank r among the ligand's pop_size energies (0 = the lowest; equal
 * energies ranked by index; NaN after every number), gets weight[l * pop_size
 * + i] = (1 + beta) (1 - r / pop_size)^beta, in binary64 rounded to float32.
 * beta = 0 gives 1 everywhere; beta > 0 favours the individuals nearer their
 * ligand's best (the weights of a ligand average about 1).  pop_energy
 * [n_ligands][pop_size] and weight [n_ligands * pop_size] are device buffers;
 * params supplies pop_size.  Cost O(pop_size) per individual.  Errors:
 * DOCK_E_INVALID (null arguments, pop_size < 1, beta not finite or <= -1). */
dock_status dock_mlp_rank_weights(const dock_ligands *ligs, const dock_search_params *params, const float *pop_energy,
                                  float beta, float *weight, void *stream);

/* Proposals (same shape as population, device): for individual i of ligand l,
 * y = network(features), alpha = alpha_max (1 - u) with u the first uniform of
 * the Philox stream (i, generation, l, purpose 4) (so alpha in (0, alpha_max]),
 * then t + alpha h y_t clamped to the box; canonical q + alpha y_q; wrap(theta_k +
 * alpha pi y_k) for k < min(n_torsions, 25); other genes copied. */
dock_status dock_propose(const dock_ligands *ligs, const dock_mlp *net, const dock_search_params *params,
                         int32_t generation, float alpha_max, int32_t g_stride, const float *population,
                         float *proposals, void *stream);

/* ---- Roofline probes: measurement aids, not steps of the docking path. ---- */

/* Map lookups alone, as the inter-energy loop of Algorithm 2 performs them: each
 * of n_lanes lanes interpolates per_lane atoms of ligand lig: its reference
 * conformation placed rigidly with a random orientation and a translation
 * uniform in [box_lo, box_hi] (host float[3] each), atoms in index order, then
 * the next placement, through the pocket's device layout and the scoring
 * kernel's gather code, and writes the sum of its values to out[lane] (device
 * float[n_lanes]).  Each lane keeps
 * in_flight (2, 4 or 8) lookups in flight: issues their loads, then
 * interpolates them.  Timing it (at the fastest in_flight) gives the measured
 * rate of random lookups for that workload's spatial distribution.
 * Errors: DOCK_E_INVALID (null pointers, handles of different devices, lig out
 * of range, empty box, n_lanes outside 1..2^31, in_flight not 2, 4 or 8,
 * per_lane not a positive multiple of in_flight), DOCK_E_DEVICE. */
dock_status dock_gather_probe(const dock_pocket *pocket, const dock_ligands *ligs, int32_t lig,
                              const float box_lo[3], const float box_hi[3], int64_t n_lanes, int32_t per_lane,
                              int32_t in_flight, uint64_t seed, float *out, void *stream);

/* Intra-energy pair terms alone (Algorithm 2's pair loop body) on register
 * coordinates: n_lanes lanes evaluate per_lane 12-6 pair terms each with the
 * pocket's force-field constants and write their sums to out[lane] (device
 * float[n_lanes]).  Timing it gives the measured VALU rate of pair terms.
 * Errors: DOCK_E_INVALID (null pointers, n_lanes outside 1..2^31, per_lane not
 * a positive multiple of 4), DOCK_E_DEVICE. */
dock_status dock_pair_probe(const dock_pocket *pocket, int64_t n_lanes, int32_t per_lane, float *out,
                            void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DOCK_H */
