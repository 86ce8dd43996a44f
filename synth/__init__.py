"""Seeded synthetic inputs for the docking hot path.

This module serves both the FP64 CPU oracle (``oracle/``) and the HIP library
(``paper_2509_12232_amd``).  It produces *inputs only*: ligand topologies and
reference conformations, a receptor, per-type force-field data, grid geometry
and batches of genotypes.  It holds none of the scoring, pose-building or search
arithmetic; that lives, independently written, on each side.

Every floating-point value it returns is rounded to float32 once, so that the
FP32 device path and the FP64 oracle (which promotes the float32 value) see
exactly the same numbers.

The paper's inputs (a set of drug-like ligands and one receptor complex, Sec. VII)
are not available; these generators stand in for them with the same structure:
tree-shaped heavy-atom ligands with rotatable bonds, typed and charged atoms, and
a receptor whose fixed structure is turned into grid maps around a pocket.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ForceField", "Ligand", "Receptor", "Grid",
    "forcefield", "make_ligand", "make_receptor", "make_grid",
    "sample_genotypes", "pocket_box", "CONFIGS", "config_ligands",
]

f32 = np.float32


# --------------------------------------------------------------------------------------
# force-field data (a table of numbers, not arithmetic)
# --------------------------------------------------------------------------------------
@dataclass
class ForceField:
    """Per-type parameters and global constants of the pair potential.

    The paper names the four interaction terms (electrostatic, van der Waals,
    hydrogen bond, desolvation; Sec. V, Algorithm 2) but prints no constants.
    The values below are the synthetic type table and literature-style constants
    both implementations receive as input data.
    """
    n_types: int
    Rii: np.ndarray          # [n_types] equilibrium radius, Angstrom
    epsii: np.ndarray        # [n_types] well depth, kcal/mol
    vol: np.ndarray          # [n_types] atomic solvation volume, Angstrom^3
    solpar: np.ndarray       # [n_types] atomic solvation parameter
    hbond: np.ndarray        # [n_types, n_types] uint8: 1 -> 12-10 pair, 0 -> 12-6
    coulomb: float = float(f32(332.06363))
    diel_A: float = float(f32(-8.5525))
    diel_eps0: float = float(f32(78.4))
    diel_lambda: float = float(f32(0.003627))
    diel_k: float = float(f32(7.7839))
    sigma: float = float(f32(3.6))
    qsolpar: float = float(f32(0.01097))
    e_cap: float = float(f32(10.0))
    r_min: float = float(f32(0.1))
    map_cap: float = float(f32(10.0))


def forcefield(n_types: int, *, solpar: float = 0.0, hbond_pairs=()) -> ForceField:
    """Synthetic type table: R = 3.0+0.1t, eps = 0.05+0.015t, vol = 10+2t."""
    t = np.arange(n_types, dtype=np.float64)
    hb = np.zeros((n_types, n_types), dtype=np.uint8)
    for a, b in hbond_pairs:
        hb[a, b] = hb[b, a] = 1
    return ForceField(
        n_types=n_types,
        Rii=(3.0 + 0.1 * t).astype(f32),
        epsii=(0.05 + 0.015 * t).astype(f32),
        vol=(10.0 + 2.0 * t).astype(f32),
        solpar=np.full(n_types, solpar, dtype=f32),
        hbond=hb,
    )


# --------------------------------------------------------------------------------------
# ligands: seeded random tree walk
# --------------------------------------------------------------------------------------
@dataclass
class Ligand:
    xyz: np.ndarray            # [n_atoms, 3] float32 reference conformation (centred)
    type: np.ndarray           # [n_atoms] int32
    charge: np.ndarray         # [n_atoms] float32
    bonds: np.ndarray          # [n_atoms-1, 2] int32 (a tree)
    torsion_bonds: np.ndarray  # [n_torsions] int32 indices into bonds

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_torsions(self) -> int:
        return int(self.torsion_bonds.shape[0])


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_ligand(seed: int, lig_id: int, n_atoms: int, n_torsions: int, n_types: int,
                *, bond: float = 1.5, min_13: float = 2.4, min_nb: float = 3.0) -> Ligand:
    """Tree-walk ligand: each new atom hangs off a random parent of degree < 4 at
    ``bond`` Angstrom in a uniform direction, accepted only if it keeps 1-3
    distances >= ``min_13`` and every other non-bonded distance >= ``min_nb``
    (at most 100 directions per parent draw).  Types are uniform, charges
    U(-0.5, 0.5).  Rotatable bonds are drawn without replacement from the bonds
    whose two ends both have degree >= 2, capped at the number available."""
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    rng = np.random.default_rng([seed, lig_id, 0x11AA])
    pos = np.zeros((n_atoms, 3))
    deg = np.zeros(n_atoms, dtype=np.int64)
    nbr: list[list[int]] = [[] for _ in range(n_atoms)]
    bonds = []
    for a in range(1, n_atoms):
        placed = False
        for _attempt in range(10000):
            cand = np.flatnonzero(deg[:a] < 4)
            parent = int(rng.choice(cand))
            lim = np.full(a, min_nb)
            lim[nbr[parent]] = min_13
            lim[parent] = 0.0
            cands = pos[parent] + bond * _unit_vectors(rng, 100)          # [100, 3]
            dist = np.linalg.norm(cands[:, None, :] - pos[None, :a, :], axis=2)
            ok = np.flatnonzero(np.all(dist >= lim[None, :], axis=1))
            if ok.size:
                pos[a] = cands[ok[0]]
                placed = True
                break
        if not placed:
            raise RuntimeError("tree walk failed to place an atom")
        bonds.append((parent, a))
        deg[parent] += 1
        deg[a] += 1
        nbr[parent].append(a)
        nbr[a].append(parent)
    pos -= pos.mean(axis=0)
    bonds_arr = np.array(bonds, dtype=np.int32).reshape(-1, 2)
    eligible = [k for k, (a, b) in enumerate(bonds) if deg[a] >= 2 and deg[b] >= 2]
    n_t = min(n_torsions, len(eligible))
    tors = np.sort(rng.choice(np.array(eligible, dtype=np.int64), size=n_t, replace=False)) \
        if n_t > 0 else np.zeros(0, dtype=np.int64)
    return Ligand(
        xyz=pos.astype(f32),
        type=rng.integers(0, n_types, size=n_atoms).astype(np.int32),
        charge=rng.uniform(-0.5, 0.5, size=n_atoms).astype(f32),
        bonds=bonds_arr,
        torsion_bonds=np.asarray(tors, dtype=np.int32),
    )


# --------------------------------------------------------------------------------------
# receptor and grid geometry
# --------------------------------------------------------------------------------------
@dataclass
class Receptor:
    xyz: np.ndarray     # [n, 3] float32
    type: np.ndarray    # [n] int32
    charge: np.ndarray  # [n] float32


CENTRE = np.array([1.0, 2.0, 3.0])


def make_receptor(seed: int, n_atoms: int, n_types: int, *, box: float = 30.0,
                  pocket_radius: float = 8.0, centre=CENTRE) -> Receptor:
    """Receptor atoms uniform in a cube of side ``box`` around ``centre``, none
    inside the pocket sphere of radius ``pocket_radius``."""
    rng = np.random.default_rng([seed, 0x5EC])
    out = np.zeros((0, 3))
    while out.shape[0] < n_atoms:
        p = rng.uniform(-box / 2, box / 2, size=(2 * n_atoms, 3))
        p = p[np.linalg.norm(p, axis=1) >= pocket_radius]
        out = np.concatenate([out, p])
    out = out[:n_atoms] + np.asarray(centre)
    return Receptor(
        xyz=out.astype(f32),
        type=rng.integers(0, n_types, size=n_atoms).astype(np.int32),
        charge=rng.uniform(-0.5, 0.5, size=n_atoms).astype(f32),
    )


@dataclass
class Grid:
    dims: tuple            # nodes per axis (nx, ny, nz)
    origin: tuple          # Angstrom; float32-representable
    spacing: float         # Angstrom; float32-representable
    n_types: int

    @property
    def n_maps(self) -> int:
        return self.n_types + 2

    def upper(self) -> np.ndarray:
        return np.asarray(self.origin) + (np.asarray(self.dims) - 1) * self.spacing


def make_grid(n: int | tuple, n_types: int, *, spacing: float = 0.375, centre=CENTRE) -> Grid:
    """Grid of ``n`` nodes per axis centred on the pocket centre."""
    dims = (n, n, n) if isinstance(n, int) else tuple(n)
    h = float(f32(spacing))
    origin = tuple(float(f32(c - (d - 1) * h / 2)) for c, d in zip(centre, dims))
    return Grid(dims=dims, origin=origin, spacing=h, n_types=n_types)


def pocket_box(grid: Grid, half: float = 8.0, centre=CENTRE):
    """Translation box: cube centre +- ``half`` Angstrom, intersected with the grid box."""
    lo = np.maximum(np.asarray(centre) - half, np.asarray(grid.origin))
    hi = np.minimum(np.asarray(centre) + half, grid.upper())
    return lo.astype(f32).astype(np.float64), hi.astype(f32).astype(np.float64)


# --------------------------------------------------------------------------------------
# genotype batches
# --------------------------------------------------------------------------------------
def sample_genotypes(seed: int, n: int, n_torsions: int, g_stride: int, box_lo, box_hi) -> np.ndarray:
    """``n`` genotypes [t(3), q(4), theta(n_torsions), zero pad] as float32:
    t uniform in the box, q uniform on the rotation group (Shoemake's subgroup
    algorithm), torsions uniform in (-pi, pi)."""
    if g_stride < 7 + n_torsions:
        raise ValueError("g_stride too small")
    rng = np.random.default_rng([seed, 0x6E0])
    g = np.zeros((n, g_stride), dtype=f32)
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    g[:, 0:3] = (lo + rng.random((n, 3)) * (hi - lo)).astype(f32)
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    g[:, 3] = (b * np.cos(2 * np.pi * u3)).astype(f32)   # w
    g[:, 4] = (a * np.sin(2 * np.pi * u2)).astype(f32)   # x
    g[:, 5] = (a * np.cos(2 * np.pi * u2)).astype(f32)   # y
    g[:, 6] = (b * np.sin(2 * np.pi * u3)).astype(f32)   # z
    if n_torsions:
        g[:, 7:7 + n_torsions] = rng.uniform(-np.pi, np.pi, size=(n, n_torsions)).astype(f32)
    return g


# --------------------------------------------------------------------------------------
# the five workload recipes
# --------------------------------------------------------------------------------------
@dataclass
class Config:
    name: str
    n_types: int
    grid_n: int
    receptor_atoms: int = 2000
    ligand_atoms: tuple = ()      # explicit per-ligand atom counts (filled by config_ligands)
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # one 24-atom ligand, 6 torsions, 8 types, 40^3 grid; DE 64 x 100
    0: dict(name="single-ligand DE", n_types=8, grid_n=40, n_ligands=1, atoms=24, torsions=6,
            pop=64, gens=100),
    # scoring microbench: one 40-atom, 10-torsion ligand, 12 types, 100^3 grid, 1e7 poses
    1: dict(name="scoring microbench", n_types=12, grid_n=100, n_ligands=1, atoms=40, torsions=10,
            n_poses=10_000_000),
    # 1000 ligands, atoms U{10..60}, torsions U{0..15}; 8 types, 64^3; DE 128 x 200
    2: dict(name="plain DE batch", n_types=8, grid_n=64, n_ligands=1000, atoms=(10, 60),
            torsions=(0, 15), pop=128, gens=200),
    # 10000 ligands lognormal(ln 32, 0.5) clipped 8..96, torsions 0..20; 12 types, 80^3; 150 x 300
    3: dict(name="uneven persistent batch", n_types=12, grid_n=80, n_ligands=10_000,
            atoms="lognormal", torsions=(0, 20), pop=150, gens=300),
    # learned proposal vs plain DE on config 3's batch; the network is trained on
    # plain runs over a disjoint set of 5000 ligands (ids 100000..104999) drawn
    # from the same size distribution
    4: dict(name="learned proposal vs plain", n_types=12, grid_n=80, n_ligands=5_000, first_id=100_000,
            atoms="lognormal", torsions=(0, 20), pop=150, gens=300, tuples=1_000_000),
    # validation batch for the learned proposal's round schedule: 2000 more
    # ligands of the same size law (ids 200000..201999), disjoint from the
    # training set and from the batch the comparison is reported on
    5: dict(name="proposal schedule validation", n_types=12, grid_n=80, n_ligands=2_000, first_id=200_000,
            atoms="lognormal", torsions=(0, 20), pop=150, gens=300),
}


def config_ligand_sizes(cfg_id: int, seed: int = 1):
    """Per-ligand (n_atoms, requested n_torsions) for a workload recipe."""
    c = CONFIGS[cfg_id]
    n = c["n_ligands"]
    rng = np.random.default_rng([seed, cfg_id, 0x512E])
    if isinstance(c["atoms"], int):
        atoms = np.full(n, c["atoms"])
    elif c["atoms"] == "lognormal":
        atoms = np.clip(np.rint(np.exp(math.log(32.0) + 0.5 * rng.normal(size=n))), 8, 96).astype(int)
    else:
        lo, hi = c["atoms"]
        atoms = rng.integers(lo, hi + 1, size=n)
    if isinstance(c["torsions"], int):
        tors = np.full(n, c["torsions"])
    else:
        lo, hi = c["torsions"]
        tors = rng.integers(lo, hi + 1, size=n)
    return atoms.astype(int), tors.astype(int)


def _make_ligand_args(args):
    return make_ligand(*args)


def config_ligands(cfg_id: int, seed: int = 1, count: int | None = None, workers: int = 1):
    """The first ``count`` ligands of a workload recipe (all of them by default).
    Every ligand has its own seed, so ``workers`` > 1 (a process pool) gives the
    same ligands."""
    c = CONFIGS[cfg_id]
    atoms, tors = config_ligand_sizes(cfg_id, seed)
    m = len(atoms) if count is None else min(count, len(atoms))
    first = c.get("first_id", 0)
    args = [(seed, first + i, int(atoms[i]), int(tors[i]), c["n_types"]) for i in range(m)]
    if workers <= 1 or m < 64:
        return [make_ligand(*a) for a in args]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make_ligand_args, args, chunksize=64))
