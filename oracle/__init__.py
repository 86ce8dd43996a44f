"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the HIP library
and its binding) never does, and shares no code with it.

Arguments are the plain records produced by ``synth`` (ligands, receptor,
force field, grid); arrays are passed by pointer through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

__all__ = ["build", "load", "score_poses", "build_maps", "pose", "ligand_info", "inter_atoms",
           "intra_xyz", "pair_energy", "brute_inter", "philox4x64", "de_init", "de_trials",
           "search", "SearchParams", "default_threads"]


def build(out: str | None = None, extra_flags=()) -> str:
    """Compile ``liboracle.so`` with gcc (IEEE binary64, no contraction, no
    fast-math); ``out`` and ``extra_flags`` serve other builds of the same source
    (the tests' instrumented one)."""
    path = out or _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", *extra_flags, _SRC, "-o", path + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


_lib = None


def load():
    """Load the built library (building it only if no build exists)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")   # another build of the same source (the sanitized one)
        if path is None:
            path = _LIB
            if not os.path.exists(path):
                build()
        lib = C.CDLL(path)
        lib.oracle_last_error.restype = C.c_char_p
        lib.oracle_pair_energy.restype = C.c_double
        lib.oracle_pair_energy.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double]
        _lib = lib
    return _lib


def default_threads() -> int:
    n = os.cpu_count() or 1
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return max(1, min(n, 16))


# ----------------------------------------------------------------------------- structs
class _FF(C.Structure):
    _fields_ = [("n_types", C.c_int),
                ("Rii", C.c_void_p), ("epsii", C.c_void_p), ("vol", C.c_void_p), ("solpar", C.c_void_p),
                ("hbond", C.c_void_p),
                ("coulomb", C.c_double), ("diel_A", C.c_double), ("diel_eps0", C.c_double),
                ("diel_lambda", C.c_double), ("diel_k", C.c_double),
                ("sigma", C.c_double), ("qsolpar", C.c_double), ("e_cap", C.c_double),
                ("r_min", C.c_double), ("map_cap", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("n_types", C.c_int), ("dims", C.c_int * 3), ("origin", C.c_double * 3),
                ("spacing", C.c_double), ("maps", C.c_void_p)]


class _Lig(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("n_torsions", C.c_int), ("xyz", C.c_void_p),
                ("type", C.c_void_p), ("charge", C.c_void_p), ("bonds", C.c_void_p),
                ("torsion_bonds", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("pop_size", C.c_int), ("n_generations", C.c_int), ("seed", C.c_uint64),
                ("F", C.c_double), ("CR", C.c_double),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("init", C.c_int), ("first_generation", C.c_int)]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def arr(self, a, dtype):
        a = _c(a, dtype)
        self.bufs.append(a)
        return _ptr(a) if a.size else None


def _ff(ff, keep: _Keep) -> _FF:
    return _FF(ff.n_types, keep.arr(ff.Rii, np.float64), keep.arr(ff.epsii, np.float64),
               keep.arr(ff.vol, np.float64), keep.arr(ff.solpar, np.float64),
               keep.arr(np.asarray(ff.hbond).reshape(-1), np.uint8),
               ff.coulomb, ff.diel_A, ff.diel_eps0, ff.diel_lambda, ff.diel_k,
               ff.sigma, ff.qsolpar, ff.e_cap, ff.r_min, ff.map_cap)


def _grid(grid, maps, keep: _Keep) -> _Grid:
    m = keep.arr(maps, np.float32)
    return _Grid(grid.n_types, (C.c_int * 3)(*grid.dims), (C.c_double * 3)(*grid.origin),
                 grid.spacing, m)


def _lig(lig, keep: _Keep) -> _Lig:
    return _Lig(lig.n_atoms, lig.n_torsions, keep.arr(lig.xyz, np.float32), keep.arr(lig.type, np.int32),
                keep.arr(lig.charge, np.float32), keep.arr(lig.bonds, np.int32),
                keep.arr(lig.torsion_bonds, np.int32))


def _ligs(ligands, keep: _Keep):
    arr = (_Lig * len(ligands))()
    for i, l in enumerate(ligands):
        arr[i] = _lig(l, keep)
    return arr


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle: " + load().oracle_last_error().decode())


# ----------------------------------------------------------------------------- API
def score_poses(grid, maps, ff, ligands, genotypes, pose_ligand=None, n_threads=None, parts=False):
    """FP64 energies of a batch of poses; with ``parts`` also (inter, intra)."""
    lib = load()
    keep = _Keep()
    G = _grid(grid, maps, keep)
    F = _ff(ff, keep)
    L = _ligs(ligands, keep)
    g = _c(genotypes, np.float32)
    n = g.shape[0]
    pl = None if pose_ligand is None else _c(pose_ligand, np.int32)
    E = np.empty(n, np.float64)
    Ei = np.empty(n, np.float64) if parts else None
    Ea = np.empty(n, np.float64) if parts else None
    rc = lib.oracle_score_poses(C.byref(G), C.byref(F), L, len(ligands),
                                C.c_void_p(None if pl is None else _ptr(pl)), C.c_void_p(_ptr(g)),
                                g.shape[1], C.c_int64(n), C.c_void_p(_ptr(E)),
                                C.c_void_p(None if Ei is None else _ptr(Ei)),
                                C.c_void_p(None if Ea is None else _ptr(Ea)),
                                n_threads or default_threads())
    _check(rc)
    return (E, Ei, Ea) if parts else E


def build_maps(ff, receptor, grid, n_threads=None) -> np.ndarray:
    """AutoGrid-style maps [n_types+2, nz, ny, nx] float32."""
    lib = load()
    keep = _Keep()
    F = _ff(ff, keep)
    nx, ny, nz = grid.dims
    out = np.empty((ff.n_types + 2, nz, ny, nx), np.float32)
    rx = _c(receptor.xyz, np.float64)
    rt = _c(receptor.type, np.int32)
    rq = _c(receptor.charge, np.float64)
    rc = lib.oracle_build_maps(C.byref(F), len(rt), C.c_void_p(_ptr(rx)), C.c_void_p(_ptr(rt)),
                               C.c_void_p(_ptr(rq)), (C.c_int * 3)(*grid.dims),
                               (C.c_double * 3)(*grid.origin), C.c_double(grid.spacing),
                               C.c_void_p(_ptr(out)), n_threads or default_threads())
    _check(rc)
    return out


def pose(ligand, n_types, genotype) -> np.ndarray:
    lib = load()
    keep = _Keep()
    L = _lig(ligand, keep)
    g = _c(genotype, np.float32)
    out = np.empty((ligand.n_atoms, 3), np.float64)
    _check(lib.oracle_pose(C.byref(L), n_types, C.c_void_p(_ptr(g)), C.c_void_p(_ptr(out))))
    return out


def ligand_info(ligand, n_types):
    """(pairs [P,2], frag [n], moving [n_tor, n] bool, axis [n_tor, 2])."""
    lib = load()
    keep = _Keep()
    L = _lig(ligand, keep)
    n, nt = ligand.n_atoms, ligand.n_torsions
    maxp = n * (n - 1) // 2
    pairs = np.empty((max(maxp, 1), 2), np.int32)
    npairs = C.c_int64(0)
    frag = np.empty(n, np.int32)
    moving = np.empty((max(nt, 1), n), np.uint8)
    axis = np.empty((max(nt, 1), 2), np.int32)
    _check(lib.oracle_ligand_info(C.byref(L), n_types, C.c_void_p(_ptr(pairs)), C.c_int64(maxp),
                                  C.byref(npairs), C.c_void_p(_ptr(frag)), C.c_void_p(_ptr(moving)),
                                  C.c_void_p(_ptr(axis))))
    return pairs[:npairs.value].copy(), frag, moving[:nt].astype(bool), axis[:nt].copy()


def inter_atoms(grid, maps, xyz, types, charges) -> np.ndarray:
    lib = load()
    keep = _Keep()
    G = _grid(grid, maps, keep)
    x = _c(xyz, np.float64).reshape(-1, 3)
    t = _c(types, np.int32)
    q = _c(charges, np.float64)
    out = np.empty(len(t), np.float64)
    _check(lib.oracle_inter_atoms(C.byref(G), len(t), C.c_void_p(_ptr(x)), C.c_void_p(_ptr(t)),
                                  C.c_void_p(_ptr(q)), C.c_void_p(_ptr(out))))
    return out


def intra_xyz(ligand, ff, xyz) -> float:
    lib = load()
    keep = _Keep()
    L = _lig(ligand, keep)
    F = _ff(ff, keep)
    x = _c(xyz, np.float64)
    out = C.c_double(0)
    _check(lib.oracle_intra_xyz(C.byref(L), C.byref(F), C.c_void_p(_ptr(x)), C.byref(out)))
    return out.value


def pair_energy(ff, ti, tj, qi, qj, r) -> float:
    lib = load()
    keep = _Keep()
    F = _ff(ff, keep)
    return lib.oracle_pair_energy(C.byref(F), int(ti), int(tj), float(qi), float(qj), float(r))


def brute_inter(ff, lig_xyz, lig_type, lig_q, receptor) -> float:
    lib = load()
    keep = _Keep()
    F = _ff(ff, keep)
    lx = _c(lig_xyz, np.float64)
    lt = _c(lig_type, np.int32)
    lq = _c(lig_q, np.float64)
    rx = _c(receptor.xyz, np.float64)
    rt = _c(receptor.type, np.int32)
    rq = _c(receptor.charge, np.float64)
    out = C.c_double(0)
    _check(lib.oracle_brute_inter(C.byref(F), len(lt), C.c_void_p(_ptr(lx)), C.c_void_p(_ptr(lt)),
                                  C.c_void_p(_ptr(lq)), len(rt), C.c_void_p(_ptr(rx)),
                                  C.c_void_p(_ptr(rt)), C.c_void_p(_ptr(rq)), C.byref(out)))
    return out.value


def philox4x64(ctr, key) -> np.ndarray:
    lib = load()
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib.oracle_philox4x64(c, k, o)
    return np.array(list(o), dtype=np.uint64)


@dataclass
class SearchParams:
    pop_size: int
    n_generations: int
    seed: int
    box_lo: tuple
    box_hi: tuple
    F: float = 0.5
    CR: float = 0.9
    init: int = 1
    first_generation: int = 0

    def _c(self) -> _Params:
        return _Params(self.pop_size, self.n_generations, self.seed,
                       float(np.float32(self.F)), float(np.float32(self.CR)),
                       (C.c_double * 3)(*self.box_lo), (C.c_double * 3)(*self.box_hi),
                       self.init, self.first_generation)


def de_init(ligand, params: SearchParams, lig_id: int, g_stride: int) -> np.ndarray:
    lib = load()
    keep = _Keep()
    L = _lig(ligand, keep)
    P = params._c()
    out = np.zeros((params.pop_size, g_stride), np.float32)
    _check(lib.oracle_de_init(C.byref(L), C.byref(P), lig_id, g_stride, C.c_void_p(_ptr(out))))
    return out


def de_trials(ligand, params: SearchParams, lig_id: int, generation: int, population) -> np.ndarray:
    lib = load()
    keep = _Keep()
    L = _lig(ligand, keep)
    P = params._c()
    pop = _c(population, np.float32)
    out = np.zeros_like(pop)
    _check(lib.oracle_de_trials(C.byref(L), C.byref(P), lig_id, generation, pop.shape[1],
                                C.c_void_p(_ptr(pop)), C.c_void_p(_ptr(out))))
    return out


def search(grid, maps, ff, ligands, params: SearchParams, g_stride: int, population=None,
           pop_energy=None, target=None, gen_reached=None, n_threads=None):
    """Plain DE over all ligands.  Returns dict with population, pop_energy,
    best_genotype, best_energy, gen_reached (arrays are updated copies)."""
    lib = load()
    keep = _Keep()
    G = _grid(grid, maps, keep)
    F = _ff(ff, keep)
    L = _ligs(ligands, keep)
    P = params._c()
    nl = len(ligands)
    pop = np.zeros((nl, params.pop_size, g_stride), np.float32) if population is None \
        else _c(population, np.float32).copy()
    pe = np.zeros((nl, params.pop_size), np.float64) if pop_energy is None \
        else _c(pop_energy, np.float64).copy()
    bg = np.zeros((nl, g_stride), np.float32)
    be = np.zeros(nl, np.float64)
    tg = None if target is None else _c(target, np.float64)
    gr = np.full(nl, -1, np.int32) if gen_reached is None else _c(gen_reached, np.int32).copy()
    rc = lib.oracle_search(C.byref(G), C.byref(F), L, nl, C.byref(P), g_stride,
                           C.c_void_p(_ptr(pop)), C.c_void_p(_ptr(pe)), C.c_void_p(_ptr(bg)),
                           C.c_void_p(_ptr(be)), C.c_void_p(None if tg is None else _ptr(tg)),
                           C.c_void_p(_ptr(gr)), n_threads or default_threads())
    _check(rc)
    return dict(population=pop, pop_energy=pe, best_genotype=bg, best_energy=be, gen_reached=gr)
