"""Shared construction of seeded test systems (inputs only) and the parity rule."""
from __future__ import annotations

import functools

import numpy as np

import synth

# FP32 GPU energy vs FP64 oracle energy on identical inputs
REL_TOL = 1e-4
ABS_TOL = 1e-3


def within_tol(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(gpu - ref) <= np.maximum(REL_TOL * np.abs(ref), ABS_TOL)


def assert_energies_match(gpu, ref, mask=None, what="energies"):
    ok = within_tol(gpu, ref)
    nan_both = np.isnan(gpu) & np.isnan(ref)
    ok = ok | nan_both
    if mask is not None:
        ok = ok | ~mask
    if not ok.all():
        bad = np.flatnonzero(~ok)
        i = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {len(ok)} outside tolerance; first at {i}: "
                             f"gpu={gpu[i]!r} oracle={ref[i]!r}")


@functools.lru_cache(maxsize=None)
def system(cfg: int, grid_n: int | None = None, n_rec: int = 2000, seed: int = 1, solpar: float = 0.0,
           hbond: bool = False):
    """(ff, receptor, grid) for a workload recipe, optionally with a smaller grid."""
    import oracle  # test infrastructure only
    c = synth.CONFIGS[cfg]
    nt = c["n_types"]
    ff = synth.forcefield(nt, solpar=solpar, hbond_pairs=[(0, 1), (2, 3)] if hbond else ())
    rec = synth.make_receptor(seed, n_rec, nt)
    grid = synth.make_grid(grid_n or c["grid_n"], nt)
    maps = oracle.build_maps(ff, rec, grid)
    return ff, rec, grid, maps


def near_face_mask(ora, grid, ligands, genotypes, pose_ligand=None, margin=1e-4):
    """True for poses with no atom within ``margin`` cells of a grid face (FP64 pose)."""
    lo = np.asarray(grid.origin)
    hi_cells = np.asarray(grid.dims) - 1
    keep = np.ones(len(genotypes), bool)
    for p in range(len(genotypes)):
        lig = ligands[0 if pose_ligand is None else int(pose_ligand[p])]
        X = ora.pose(lig, grid.n_types, genotypes[p])
        u = (X - lo) / grid.spacing
        if np.any(np.abs(u) < margin) or np.any(np.abs(u - hi_cells) < margin):
            keep[p] = False
    return keep
