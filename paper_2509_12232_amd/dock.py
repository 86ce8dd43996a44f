"""ctypes binding of ``libdock.so`` (include/dock.h), same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the library's HIP
kernels.  Device buffers are torch tensors on the pocket's device; their
``data_ptr()`` and the current HIP stream are handed to the library.  If the
library has not been built, importing this module raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdock.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2509_12232_amd.build.build() "
                      "(hipcc --offload-arch=gfx950) first")

_lib = C.CDLL(LIB_PATH)

DOCK_OK, DOCK_E_INVALID, DOCK_E_NOMEM, DOCK_E_DEVICE, DOCK_E_UNSUPPORTED = range(5)
(DOCK_LAYOUT_AUTO, DOCK_LAYOUT_LINEAR, DOCK_LAYOUT_ZPAIR, DOCK_LAYOUT_YZQUAD, DOCK_LAYOUT_QUADLINE,
 DOCK_LAYOUT_PAIRLINE) = -1, 0, 1, 2, 3, 4
_STATUS = {1: "DOCK_E_INVALID", 2: "DOCK_E_NOMEM", 3: "DOCK_E_DEVICE", 4: "DOCK_E_UNSUPPORTED"}


class DockError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _FF(C.Structure):
    _fields_ = [("n_types", C.c_int32),
                ("Rii", C.c_void_p), ("epsii", C.c_void_p), ("vol", C.c_void_p), ("solpar", C.c_void_p),
                ("hbond", C.c_void_p),
                ("coulomb", C.c_float), ("diel_A", C.c_float), ("diel_eps0", C.c_float),
                ("diel_lambda", C.c_float), ("diel_k", C.c_float),
                ("sigma", C.c_float), ("qsolpar", C.c_float), ("e_cap", C.c_float), ("r_min", C.c_float),
                ("map_cap", C.c_float)]


class _Grid(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("dims", C.c_int32 * 3), ("origin", C.c_float * 3),
                ("spacing", C.c_float)]


class _LigDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_torsions", C.c_int32), ("xyz", C.c_void_p), ("type", C.c_void_p),
                ("charge", C.c_void_p), ("bonds", C.c_void_p), ("torsion_bonds", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("pop_size", C.c_int32), ("n_generations", C.c_int32), ("seed", C.c_uint64),
                ("F", C.c_float), ("CR", C.c_float),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("init", C.c_int32), ("first_generation", C.c_int32), ("stop_at_target", C.c_int32),
                ("proposal", C.c_void_p), ("proposal_step", C.c_float), ("proposal_every", C.c_int32),
                ("proposal_until", C.c_int32)]


_P = C.c_void_p
_lib.dock_last_error.restype = C.c_char_p
_lib.dock_version.restype = C.c_int32
_SIGS = {
    "dock_create_pocket": [_P, _P, C.c_int32, _P, C.c_int32, C.c_int32, _P],
    "dock_create_pocket_from_receptor": [_P, _P, C.c_int32, _P, _P, _P, C.c_int32, C.c_int32, _P],
    "dock_pocket_layout": [_P, _P],
    "dock_pocket_maps": [_P, _P, _P],
    "dock_destroy_pocket": [_P],
    "dock_create_ligands": [_P, _P, C.c_int32, _P],
    "dock_ligand_pair_count": [_P, C.c_int32, _P],
    "dock_destroy_ligands": [_P],
    "dock_score_poses": [_P, _P, _P, _P, C.c_int32, C.c_int64, _P, _P],
    "dock_score_set_split": [C.c_int32],
    "dock_score_split": [_P, _P],
    "dock_de_init": [_P, _P, C.c_int32, _P, _P],
    "dock_de_trials": [_P, _P, C.c_int32, C.c_int32, _P, _P, _P],
    "dock_search": [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P],
    "dock_search_no_alloc": [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P],
    "dock_gather_probe": [_P, _P, C.c_int32, _P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_uint64, _P, _P],
    "dock_pair_probe": [_P, C.c_int64, C.c_int32, _P, _P],
    "dock_search_plan_create": [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P],
    "dock_search_plan_launch": [_P, _P],
    "dock_search_plan_destroy": [_P],
    "dock_search_shapes": [_P, _P],
    "dock_search_set_shapes": [_P, _P],
    "dock_search_autotune": [_P, _P, _P, C.c_int32, C.c_int32, _P],
    "dock_search_tune_save": [C.c_char_p],
    "dock_search_tune_load": [C.c_char_p],
    "dock_mlp_create": [C.c_int32, C.c_uint64, _P],
    "dock_mlp_destroy": [_P],
    "dock_mlp_set_params": [_P, _P],
    "dock_mlp_get_params": [_P, _P],
    "dock_mlp_forward": [_P, _P, C.c_int64, _P, _P],
    "dock_mlp_gradients": [_P, _P, _P, _P, C.c_int32, _P, _P, _P],
    "dock_mlp_train": [_P, _P, _P, _P, C.c_int64, _P, C.c_int64, C.c_int32, C.c_int32, C.c_float, _P, _P],
    "dock_ligand_descriptors": [_P, _P, _P],
    "dock_mlp_features": [_P, _P, C.c_int32, _P, _P, _P],
    "dock_mlp_moves": [_P, _P, C.c_int32, _P, _P, _P, _P],
    "dock_propose": [_P, _P, _P, C.c_int32, C.c_float, C.c_int32, _P, _P, _P],
    "dock_mlp_rank_weights": [_P, _P, _P, C.c_float, _P, _P],
}
DOCK_MLP_IN, DOCK_MLP_HIDDEN, DOCK_MLP_OUT, DOCK_MLP_PARAMS, DOCK_DESC = 96, 256, 32, 98848, 64
DOCK_MLP_MAX_BATCH = 65536
DOCK_NO_ALLOC_SCRATCH_BYTES = 64 << 20
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int


def _check(st: int):
    if st != DOCK_OK:
        raise DockError(st, _lib.dock_last_error().decode())


def dock_version() -> int:
    return int(_lib.dock_version())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _bufs(device: int, *specs):
    """Device pointers (None for None) of the torch tensors in specs, each given
    as (tensor, dtype name, what, least element count).  Every tensor is checked
    -- type, dtype and length first, for all of them, then that it lies
    contiguous on the handle's device -- before any pointer reaches the library,
    whose kernels write through them."""
    import torch
    for t, dtype_name, what, need in specs:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what}: expected a torch tensor")
        if str(t.dtype) != f"torch.{dtype_name}":
            raise TypeError(f"{what}: expected {dtype_name}, got {t.dtype}")
        if t.numel() < need:
            raise ValueError(f"{what}: {t.numel()} elements, at least {need} needed")
    out = []
    for t, _, what, _ in specs:
        if t is None:
            out.append(None)
            continue
        if not t.is_cuda:
            raise TypeError(f"{what}: expected a device tensor")
        if t.device.index != device:
            raise ValueError(f"{what}: on device {t.device.index}, the handle is on device {device}")
        if not t.is_contiguous():
            raise ValueError(f"{what}: tensor must be contiguous")
        out.append(C.c_void_p(t.data_ptr()))
    return out


def _buf(t, dtype_name: str, what: str, need: int, device: int):
    """_bufs for one tensor."""
    return _bufs(device, (t, dtype_name, what, need))[0]


def _rows(t, what: str) -> int:
    """Row count of a 2-D (or higher) tensor argument."""
    if t is None or t.dim() < 2:
        raise ValueError(f"{what}: expected a tensor of at least two dimensions")
    return int(t.shape[0])


class _Keep:
    def __init__(self):
        self.bufs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.bufs.append(a)
        return C.c_void_p(a.ctypes.data) if a.size else None


def _ff_struct(ff, keep: _Keep) -> _FF:
    return _FF(ff.n_types, keep.arr(ff.Rii, np.float32), keep.arr(ff.epsii, np.float32),
               keep.arr(ff.vol, np.float32), keep.arr(ff.solpar, np.float32),
               keep.arr(np.asarray(ff.hbond).reshape(-1), np.uint8),
               ff.coulomb, ff.diel_A, ff.diel_eps0, ff.diel_lambda, ff.diel_k,
               ff.sigma, ff.qsolpar, ff.e_cap, ff.r_min, ff.map_cap)


def _grid_struct(grid) -> _Grid:
    return _Grid(grid.n_types, (C.c_int32 * 3)(*grid.dims), (C.c_float * 3)(*grid.origin), grid.spacing)


class Pocket:
    """Owner of a dock_pocket handle."""

    def __init__(self, handle: C.c_void_p, grid, device: int):
        self.handle = handle
        self.grid = grid
        self.device = device
        # held here: module globals may already be gone when __del__ runs at exit
        self._destroy = _lib.dock_destroy_pocket

    @property
    def layout(self) -> int:
        out = C.c_int32(0)
        _check(_lib.dock_pocket_layout(self.handle, C.byref(out)))
        return out.value

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "_destroy", None):
            self._destroy(self.handle)
            self.handle = None


class Ligands:
    """Owner of a dock_ligands handle."""

    def __init__(self, handle: C.c_void_p, n: int, max_torsions: int, pocket: Pocket):
        self.handle = handle
        self.n = n
        self.max_torsions = max_torsions
        self.pocket = pocket  # keeps the pocket alive
        self._destroy = _lib.dock_destroy_ligands

    def pair_count(self, lig: int) -> int:
        out = C.c_int32(0)
        _check(_lib.dock_ligand_pair_count(self.handle, lig, C.byref(out)))
        return out.value

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "_destroy", None):
            self._destroy(self.handle)
            self.handle = None


def dock_create_pocket(grid, maps, ff, device: int = 0, layout: int = DOCK_LAYOUT_AUTO) -> Pocket:
    """maps: host numpy array or device tensor, float32 [n_types+2, nz, ny, nx]."""
    keep = _Keep()
    F = _ff_struct(ff, keep)
    G = _grid_struct(grid)
    out = C.c_void_p()
    if isinstance(maps, np.ndarray):
        ptr, on_dev = keep.arr(maps, np.float32), 0
    else:
        ptr, on_dev = _buf(maps, "float32", "maps", (grid.n_types + 2) * int(np.prod(grid.dims)), device), 1
    _check(_lib.dock_create_pocket(C.byref(G), ptr, on_dev, C.byref(F), layout, device, C.byref(out)))
    return Pocket(out, grid, device)


def dock_create_pocket_from_receptor(grid, ff, receptor, device: int = 0, layout: int = DOCK_LAYOUT_AUTO) -> Pocket:
    keep = _Keep()
    F = _ff_struct(ff, keep)
    G = _grid_struct(grid)
    out = C.c_void_p()
    n = int(len(receptor.type))
    _check(_lib.dock_create_pocket_from_receptor(C.byref(G), C.byref(F), n, keep.arr(receptor.xyz, np.float32),
                                                 keep.arr(receptor.type, np.int32),
                                                 keep.arr(receptor.charge, np.float32), layout, device,
                                                 C.byref(out)))
    return Pocket(out, grid, device)


def dock_pocket_maps(pocket: Pocket, maps_out, stream=None):
    g = pocket.grid
    need = (g.n_types + 2) * int(np.prod(g.dims))
    _check(_lib.dock_pocket_maps(pocket.handle, _buf(maps_out, "float32", "maps_out", need, pocket.device),
                                 _stream(stream)))


def dock_create_ligands(pocket: Pocket, ligands) -> Ligands:
    keep = _Keep()
    arr = (_LigDesc * len(ligands))()
    for i, l in enumerate(ligands):
        arr[i] = _LigDesc(int(l.xyz.shape[0]), int(len(l.torsion_bonds)), keep.arr(l.xyz, np.float32),
                          keep.arr(l.type, np.int32), keep.arr(l.charge, np.float32),
                          keep.arr(l.bonds, np.int32), keep.arr(l.torsion_bonds, np.int32))
    out = C.c_void_p()
    _check(_lib.dock_create_ligands(pocket.handle, arr, len(ligands), C.byref(out)))
    max_t = max(int(len(l.torsion_bonds)) for l in ligands)
    return Ligands(out, len(ligands), max_t, pocket)


def dock_score_poses(pocket: Pocket, ligs: Ligands, genotypes, energies, pose_ligand=None, stream=None):
    """genotypes: float32 [n, g_stride] device tensor; energies: float32 [n] device tensor."""
    n = _rows(genotypes, "genotypes")
    gs = int(np.prod(genotypes.shape[1:]))
    pl, g, e = _bufs(pocket.device, (pose_ligand, "int32", "pose_ligand", n),
                     (genotypes, "float32", "genotypes", n * gs), (energies, "float32", "energies", n))
    _check(_lib.dock_score_poses(pocket.handle, ligs.handle, pl, g, gs, n, e, _stream(stream)))


def dock_score_set_split(split: int):
    """Wavefronts per block of 64 poses of the scoring kernel (1, 2, 4 or 8; 0 =
    automatic), process-wide."""
    _check(_lib.dock_score_set_split(int(split)))


def dock_score_split(ligs: Ligands) -> int:
    out = C.c_int32()
    _check(_lib.dock_score_split(ligs.handle, C.byref(out)))
    return out.value


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
    stop_at_target: int = 0
    proposal: "Mlp | None" = None
    proposal_step: float = 1.0
    proposal_every: int = 0
    proposal_until: int = 1 << 30

    def _c(self) -> _Params:
        return _Params(self.pop_size, self.n_generations, self.seed, self.F, self.CR,
                       (C.c_double * 3)(*self.box_lo), (C.c_double * 3)(*self.box_hi), self.init,
                       self.first_generation, self.stop_at_target,
                       self.proposal.handle if self.proposal is not None else None, self.proposal_step,
                       self.proposal_every, self.proposal_until)


def _pop_sizes(ligs: Ligands, params: SearchParams, population):
    """(g_stride, elements of a population, of its energies) for a population tensor."""
    g = int(population.shape[-1])
    n = ligs.n * max(int(params.pop_size), 0)
    return g, n * g, n


def dock_de_init(ligs: Ligands, params: SearchParams, population, stream=None):
    P = params._c()
    g, npg, _ = _pop_sizes(ligs, params, population)
    _check(_lib.dock_de_init(ligs.handle, C.byref(P), g,
                             _buf(population, "float32", "population", npg, ligs.pocket.device), _stream(stream)))


def dock_de_trials(ligs: Ligands, params: SearchParams, generation: int, population, trials, stream=None):
    P = params._c()
    g, npg, _ = _pop_sizes(ligs, params, population)
    pp, tp = _bufs(ligs.pocket.device, (population, "float32", "population", npg), (trials, "float32", "trials", npg))
    _check(_lib.dock_de_trials(ligs.handle, C.byref(P), generation, g, pp, tp, _stream(stream)))


def dock_search(pocket: Pocket, ligs: Ligands, params: SearchParams, population, pop_energy, best_genotypes,
                best_energies, target=None, gen_reached=None, stream=None):
    P = params._c()
    args = _search_buffers(pocket, ligs, params, population, pop_energy, best_genotypes, best_energies, target,
                           gen_reached)
    _check(_lib.dock_search(pocket.handle, ligs.handle, C.byref(P), *args, _stream(stream)))


def dock_search_no_alloc(pocket: Pocket, ligs: Ligands, params: SearchParams, population, pop_energy,
                         best_genotypes, best_energies, target=None, gen_reached=None, stream=None):
    """dock_search on the library's fixed per-device scratch (no allocation)."""
    P = params._c()
    args = _search_buffers(pocket, ligs, params, population, pop_energy, best_genotypes, best_energies, target,
                           gen_reached)
    _check(_lib.dock_search_no_alloc(pocket.handle, ligs.handle, C.byref(P), *args, _stream(stream)))


def _search_buffers(pocket: Pocket, ligs: Ligands, params: SearchParams, population, pop_energy, best_genotypes,
                    best_energies, target, gen_reached):
    """g_stride and the checked pointers of a search's buffers."""
    g, npg, npe = _pop_sizes(ligs, params, population)
    n = ligs.n
    return (g, *_bufs(pocket.device, (population, "float32", "population", npg),
                      (pop_energy, "float32", "pop_energy", npe), (best_genotypes, "float32", "best_genotypes", n * g),
                      (best_energies, "float32", "best_energies", n), (target, "float32", "target", n),
                      (gen_reached, "int32", "gen_reached", n)))


def dock_gather_probe(pocket: Pocket, ligs: Ligands, lig: int, box_lo, box_hi, out, per_lane: int, seed: int = 1,
                      stream=None, in_flight: int = 4):
    """Random map lookups alone (roofline probe); out: float32 device tensor, one value per lane;
    in_flight: lookups each lane keeps in flight (2, 4 or 8)."""
    lo = (C.c_float * 3)(*box_lo)
    hi = (C.c_float * 3)(*box_hi)
    _check(_lib.dock_gather_probe(pocket.handle, ligs.handle, lig, lo, hi, int(out.numel()), per_lane, in_flight,
                                  seed, _buf(out, "float32", "out", 0, pocket.device), _stream(stream)))


def dock_pair_probe(pocket: Pocket, out, per_lane: int, stream=None):
    """Pair terms alone on register coordinates (roofline probe)."""
    _check(_lib.dock_pair_probe(pocket.handle, int(out.numel()), per_lane,
                                _buf(out, "float32", "out", 0, pocket.device), _stream(stream)))


# ---------------------------------------------------------------- search plans
class SearchPlan:
    """Owner of a dock_search_plan (a search captured into one HIP graph).  Keeps
    the buffers it was created with alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep
        self._destroy = _lib.dock_search_plan_destroy

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "_destroy", None):
            self._destroy(self.handle)
            self.handle = None


def dock_search_plan_create(pocket: Pocket, ligs: Ligands, params: SearchParams, population, pop_energy,
                            best_genotypes, best_energies, target=None, gen_reached=None) -> SearchPlan:
    P = params._c()
    out = C.c_void_p()
    args = _search_buffers(pocket, ligs, params, population, pop_energy, best_genotypes, best_energies, target,
                           gen_reached)
    _check(_lib.dock_search_plan_create(pocket.handle, ligs.handle, C.byref(P), *args, C.byref(out)))
    return SearchPlan(out, (pocket, ligs, params.proposal, population, pop_energy, best_genotypes, best_energies,
                            target, gen_reached))


def dock_search_plan_launch(plan: SearchPlan, stream=None):
    _check(_lib.dock_search_plan_launch(plan.handle, _stream(stream)))


# ---------------------------------------------------------------- search launch shapes
DOCK_SEARCH_BUCKETS = 5


class _Shape(C.Structure):
    _fields_ = [("max_atoms", C.c_int32), ("split", C.c_int32), ("blocks_per_group", C.c_int32)]


def dock_search_shapes(ligs: Ligands):
    """[(max_atoms, split, blocks_per_group)] per ligand-size bucket."""
    arr = (_Shape * DOCK_SEARCH_BUCKETS)()
    _check(_lib.dock_search_shapes(ligs.handle, arr))
    return [(a.max_atoms, a.split, a.blocks_per_group) for a in arr]


def dock_search_set_shapes(ligs: Ligands, shapes):
    arr = (_Shape * DOCK_SEARCH_BUCKETS)(*[_Shape(*x) for x in shapes])
    _check(_lib.dock_search_set_shapes(ligs.handle, arr))


def dock_search_tune_save(path):
    """Write the autotuner's cached shapes (this process) to a text file."""
    _check(_lib.dock_search_tune_save(os.fsencode(path)))


def dock_search_tune_load(path):
    """Merge shapes saved by dock_search_tune_save into this process's cache."""
    _check(_lib.dock_search_tune_load(os.fsencode(path)))


def dock_search_autotune(pocket: Pocket, ligs: Ligands, params: SearchParams, g_stride: int,
                         tune_generations: int = 3, stream=None):
    P = params._c()
    _check(_lib.dock_search_autotune(pocket.handle, ligs.handle, C.byref(P), g_stride, tune_generations,
                                     _stream(stream)))


# ---------------------------------------------------------------- learned proposal
class Mlp:
    """Owner of a dock_mlp handle (the learned-proposal network)."""

    def __init__(self, handle: C.c_void_p, device: int):
        self.handle = handle
        self.device = device
        self._destroy = _lib.dock_mlp_destroy

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "_destroy", None):
            self._destroy(self.handle)
            self.handle = None


def dock_mlp_create(device: int = 0, seed: int = 1) -> Mlp:
    out = C.c_void_p()
    _check(_lib.dock_mlp_create(device, seed, C.byref(out)))
    return Mlp(out, device)


def dock_mlp_set_params(net: Mlp, params):
    keep = _Keep()
    p = np.asarray(params, dtype=np.float32).reshape(-1)
    if p.size != DOCK_MLP_PARAMS:
        raise ValueError(f"expected {DOCK_MLP_PARAMS} parameters")
    _check(_lib.dock_mlp_set_params(net.handle, keep.arr(p, np.float32)))


def dock_mlp_get_params(net: Mlp) -> np.ndarray:
    out = np.empty(DOCK_MLP_PARAMS, np.float32)
    _check(_lib.dock_mlp_get_params(net.handle, C.c_void_p(out.ctypes.data)))
    return out


def dock_mlp_forward(net: Mlp, x, y, stream=None):
    """x: float32 [n, 96] device tensor; y: float32 [n, 32] device tensor."""
    n = _rows(x, "x")
    xp, yp = _bufs(net.device, (x, "float32", "x", n * DOCK_MLP_IN), (y, "float32", "y", n * DOCK_MLP_OUT))
    _check(_lib.dock_mlp_forward(net.handle, xp, n, yp, _stream(stream)))


def dock_mlp_gradients(net: Mlp, x, target, grads, loss, weight=None, stream=None):
    n = _rows(x, "x")
    xp, tp, wp, gp, lp = _bufs(net.device, (x, "float32", "x", n * DOCK_MLP_IN),
                               (target, "float32", "target", n * DOCK_MLP_OUT), (weight, "float32", "weight", n),
                               (grads, "float32", "grads", DOCK_MLP_PARAMS), (loss, "float32", "loss", 1))
    _check(_lib.dock_mlp_gradients(net.handle, xp, tp, wp, n, gp, lp, _stream(stream)))


def dock_mlp_train(net: Mlp, x, target, batch: int, n_steps: int, lr: float, weight=None, order=None, losses=None,
                   stream=None):
    """Adam steps on minibatches of the data set x [n, 96] / target [n, 32]: the rows
    order[0..] (int32 device tensor of row indices) or all rows in order."""
    n = _rows(x, "x")
    n_rows = n if order is None else int(order.numel())
    xp, tp, wp, op, lp = _bufs(net.device, (x, "float32", "x", n * DOCK_MLP_IN),
                               (target, "float32", "target", n * DOCK_MLP_OUT), (weight, "float32", "weight", n),
                               (order, "int32", "order", 0), (losses, "float32", "losses", max(n_steps, 0)))
    _check(_lib.dock_mlp_train(net.handle, xp, tp, wp, n, op, n_rows, batch, n_steps, lr, lp, _stream(stream)))


def dock_ligand_descriptors(ligs: Ligands, out, stream=None):
    _check(_lib.dock_ligand_descriptors(ligs.handle, _buf(out, "float32", "out", ligs.n * DOCK_DESC,
                                                          ligs.pocket.device), _stream(stream)))


def dock_mlp_features(ligs: Ligands, params: SearchParams, population, x, stream=None):
    P = params._c()
    g, npg, n = _pop_sizes(ligs, params, population)
    pp, xp = _bufs(ligs.pocket.device, (population, "float32", "population", npg),
                   (x, "float32", "x", n * DOCK_MLP_IN))
    _check(_lib.dock_mlp_features(ligs.handle, C.byref(P), g, pp, xp, _stream(stream)))


def dock_mlp_moves(ligs: Ligands, params: SearchParams, from_pop, to_pop, out, stream=None):
    P = params._c()
    g, npg, n = _pop_sizes(ligs, params, from_pop)
    fp, tp, op = _bufs(ligs.pocket.device, (from_pop, "float32", "from", npg), (to_pop, "float32", "to", npg),
                       (out, "float32", "out", n * DOCK_MLP_OUT))
    _check(_lib.dock_mlp_moves(ligs.handle, C.byref(P), g, fp, tp, op, _stream(stream)))


def dock_propose(ligs: Ligands, net: Mlp, params: SearchParams, generation: int, alpha_max: float, population,
                 proposals, stream=None):
    P = params._c()
    g, npg, _ = _pop_sizes(ligs, params, population)
    pp, qp = _bufs(ligs.pocket.device, (population, "float32", "population", npg),
                   (proposals, "float32", "proposals", npg))
    _check(_lib.dock_propose(ligs.handle, net.handle, C.byref(P), generation, alpha_max, g, pp, qp,
                             _stream(stream)))


def dock_mlp_rank_weights(ligs: Ligands, params: SearchParams, pop_energy, beta: float, weight, stream=None):
    """Training weights (1 + beta)(1 - rank / pop)^beta from a population's energies."""
    P = params._c()
    n = ligs.n * max(int(params.pop_size), 0)
    ep, wp = _bufs(ligs.pocket.device, (pop_energy, "float32", "pop_energy", n), (weight, "float32", "weight", n))
    _check(_lib.dock_mlp_rank_weights(ligs.handle, C.byref(P), ep, float(beta), wp, _stream(stream)))
