"""GPU parity of pose scoring (Algorithms 1 and 2 per pose) against the FP64
oracle on identical seeded inputs, through the C ABI."""
import numpy as np
import pytest

import synth
from tests._systems import assert_energies_match, near_face_mask, system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dk():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock
    return dock


def _gpu_energies(dk, pocket, ligs, g, pose_ligand=None):
    import torch
    gt = torch.from_numpy(np.ascontiguousarray(g)).cuda()
    e = torch.full((len(g),), 12345.0, dtype=torch.float32, device="cuda")
    pl = None if pose_ligand is None else torch.from_numpy(np.asarray(pose_ligand, np.int32)).cuda()
    dk.dock_score_poses(pocket, ligs, gt, e, pose_ligand=pl)
    torch.cuda.synchronize()
    return e.cpu().numpy()


@pytest.mark.parametrize("layout", [0, 1, 2, 3, 4])
def test_config0_single_ligand_parity(dk, ora, layout):
    """24-atom, 6-torsion ligand on 40^3 maps: 4133 random poses (64 full tiles +
    a ragged tail), for each device map layout."""
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    print("case: config0 single ligand, 4133 poses, layout", layout, flush=True)
    pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
    assert pocket.layout == layout
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    g = synth.sample_genotypes(11, 4133, 6, 13, lo, hi)
    e_gpu = _gpu_energies(dk, pocket, ligs, g)
    e_ref = ora.score_poses(grid, maps, ff, [lig], g)
    keep = near_face_mask(ora, grid, [lig], g)
    assert keep.mean() > 0.95
    assert_energies_match(e_gpu, e_ref, keep)


def test_pair_line_gives_the_quad_line_bits(dk):
    """The pair-line and quad-line layouts hold the same rounded values (type
    quads, E + D and E - D quads) and the kernel interpolates them in the same
    order, so energies are the same bits for every scoring split, for atoms
    of both charge signs and for poses reaching past the grid box."""
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    assert (lig.charge > 0).any() and (lig.charge < 0).any()
    lo = np.asarray(grid.origin) - 1.0
    hi = np.asarray(grid.upper()) + 1.0
    g = synth.sample_genotypes(12, 2077, 6, 13, lo, hi)
    got = {}
    try:
        for layout in (3, 4):
            pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
            ligs = dk.dock_create_ligands(pocket, [lig])
            for lp in (1, 2, 4, 8):
                print("case: quad-line vs pair-line bits, layout", layout, "split", lp, flush=True)
                dk.dock_score_set_split(lp)
                got[layout, lp] = _gpu_energies(dk, pocket, ligs, g)
    finally:
        dk.dock_score_set_split(0)
    for lp in (1, 2, 4, 8):
        assert np.array_equal(got[3, lp].view(np.uint32), got[4, lp].view(np.uint32)), lp
    assert np.isfinite(got[4, 1]).all()


@pytest.mark.parametrize("dims", [(2, 2, 2), (9, 3, 5), (16, 7, 4), (23, 11, 6)])
def test_odd_grid_dims_every_layout(dk, ora, dims):
    """Non-cubic grids whose x extent leaves the quad-line and pair-line layouts
    a partly filled last line per row (and the 2-node minimum), with poses spread
    over and past the grid box, for every device layout."""
    import oracle
    nt = 8
    ff = synth.forcefield(nt)
    rec = synth.make_receptor(3, 400, nt)
    grid = synth.make_grid(dims, nt, spacing=1.0)
    maps = oracle.build_maps(ff, rec, grid)
    lig = synth.make_ligand(2, 0, 12, 3, nt)
    lo = np.asarray(grid.origin) - 2.0
    hi = np.asarray(grid.upper()) + 2.0
    g = synth.sample_genotypes(21, 700, 3, 10, lo, hi)
    e_ref = ora.score_poses(grid, maps, ff, [lig], g)
    keep = near_face_mask(ora, grid, [lig], g)
    for layout in (0, 1, 2, 3, 4):
        print("case: grid dims", dims, "layout", layout, flush=True)
        pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
        ligs = dk.dock_create_ligands(pocket, [lig])
        assert_energies_match(_gpu_energies(dk, pocket, ligs, g), e_ref, keep)


def test_mixed_ligands_per_wave_with_hbond_and_solvation(dk, ora):
    """Ten ligands of 10-60 atoms interleaved at random across wavefronts, with
    12-10 pairs and non-zero per-type solvation switched on."""
    ff, rec, grid, maps = system(2, grid_n=48, solpar=-0.0011, hbond=True)
    atoms, tors = synth.config_ligand_sizes(2)
    ligands = [synth.make_ligand(1, i, int(atoms[i]), int(tors[i]), 8) for i in range(10)]
    print("case: mixed ligands", [l.n_atoms for l in ligands], flush=True)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    stride = 7 + max(l.n_torsions for l in ligands)
    lo, hi = synth.pocket_box(grid, half=4.0)
    rng = np.random.default_rng(5)
    n = 3000
    pl = rng.integers(0, 10, n).astype(np.int32)
    g = synth.sample_genotypes(12, n, stride - 7, stride, lo, hi)
    for p in range(n):     # genes past a ligand's own torsions are padding
        g[p, 7 + ligands[pl[p]].n_torsions:] = 0
    e_gpu = _gpu_energies(dk, pocket, ligs, g, pl)
    e_ref = ora.score_poses(grid, maps, ff, ligands, g, pose_ligand=pl)
    keep = near_face_mask(ora, grid, ligands, g, pl)
    assert_energies_match(e_gpu, e_ref, keep)
    # grouped by ligand gives the same numbers
    order = np.argsort(pl, kind="stable")
    e2 = _gpu_energies(dk, pocket, ligs, g[order], pl[order])
    np.testing.assert_array_equal(e2, e_gpu[order])


def test_edge_ligands(dk, ora):
    """One atom (no pairs, no torsions), a rigid 12-atom ligand, and the largest
    supported ligand (96 atoms, 20 torsions)."""
    ff, rec, grid, maps = system(0)
    one = synth.Ligand(np.array([[0.3, -0.2, 0.1]], np.float32), np.array([3], np.int32),
                       np.array([0.25], np.float32), np.zeros((0, 2), np.int32), np.zeros(0, np.int32))
    rigid = synth.make_ligand(1, 3, 12, 0, 8)
    big = synth.make_ligand(1, 4, 96, 20, 8)
    ligands = [one, rigid, big]
    print("case: edge ligands 1/12/96 atoms", flush=True)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    assert ligs.pair_count(0) == 0
    lo, hi = synth.pocket_box(grid, half=3.0)
    n = 600
    pl = np.repeat(np.arange(3, dtype=np.int32), n // 3)
    g = synth.sample_genotypes(13, n, 20, 27, lo, hi)
    g[pl != 2, 7:] = 0
    e_gpu = _gpu_energies(dk, pocket, ligs, g, pl)
    e_ref = ora.score_poses(grid, maps, ff, ligands, g, pose_ligand=pl)
    keep = near_face_mask(ora, grid, ligands, g, pl)
    assert_energies_match(e_gpu, e_ref, keep)


def test_outside_box_nan_and_bad_ligand_index(dk, ora):
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    g = np.zeros((5, 13), np.float32)
    g[:, 3] = 1
    g[0, 0:3] = (100.0, 100.0, 100.0)     # whole ligand outside the maps: intra only
    g[1, 8] = np.nan
    g[2, 4] = np.inf
    g[3, 3:7] = 0                         # zero quaternion = identity
    pl = np.array([0, 0, 0, 0, 7], np.int32)
    e_gpu = _gpu_energies(dk, pocket, ligs, g, pl)
    e_ref = ora.score_poses(grid, maps, ff, [lig], g[:4])
    _, _, intra = ora.score_poses(grid, maps, ff, [lig], g[:1], parts=True)
    assert_energies_match(e_gpu[:4], e_ref)
    assert e_ref[0] == pytest.approx(intra[0])
    assert np.isnan(e_gpu[1]) and np.isnan(e_gpu[2]) and np.isnan(e_gpu[4])


def test_empty_batch_and_invalid_args(dk):
    import torch
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    g = torch.zeros((0, 13), dtype=torch.float32, device="cuda")
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    dk.dock_score_poses(pocket, ligs, g, e)
    with pytest.raises(dk.DockError):
        dk.dock_score_poses(pocket, ligs, torch.zeros((4, 12), dtype=torch.float32, device="cuda"),
                            torch.zeros(4, dtype=torch.float32, device="cuda"))
    too_big = synth.make_ligand(1, 0, 24, 6, 8)
    too_big.type = too_big.type + 8
    with pytest.raises(dk.DockError):
        dk.dock_create_ligands(pocket, [too_big])


def test_ring_is_unsupported(dk):
    """Bonds that close a ring are valid chemistry outside what this build
    supports (the rotatable-bond tree of Algorithm 1): DOCK_E_UNSUPPORTED,
    wherever the ring lies.  A repeated bond is invalid input."""
    import dataclasses
    ff, rec, grid, maps = system(0)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    lig = synth.make_ligand(1, 0, 6, 0, 8)
    for bonds in ([[0, 1], [1, 2], [2, 3], [3, 0], [4, 5]],    # ring through the root atom
                  [[0, 1], [1, 2], [3, 4], [4, 5], [5, 3]]):   # ring apart from it
        ring = dataclasses.replace(lig, bonds=np.array(bonds, np.int32))
        with pytest.raises(dk.DockError) as ei:
            dk.dock_create_ligands(pocket, [ring])
        assert ei.value.status == dk.DOCK_E_UNSUPPORTED and "ring" in str(ei.value), bonds
    for bonds in ([[0, 1], [1, 2], [2, 3], [3, 4], [4, 3]], [[0, 1], [1, 2], [2, 2], [3, 4], [4, 5]]):
        bad = dataclasses.replace(lig, bonds=np.array(bonds, np.int32))
        with pytest.raises(dk.DockError) as ei:
            dk.dock_create_ligands(pocket, [bad])
        assert ei.value.status == dk.DOCK_E_INVALID, bonds
    dk.dock_create_ligands(pocket, [lig])


def test_deterministic_across_calls(dk):
    import torch
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    g = synth.sample_genotypes(14, 5000, 6, 13, lo, hi)
    a = _gpu_energies(dk, pocket, ligs, g)
    b = _gpu_energies(dk, pocket, ligs, g)
    assert np.array_equal(a, b, equal_nan=True)


def test_split_same_bits(dk, ora):
    """Every scoring launch shape (1, 2, 4 or 8 wavefronts per block of 64 poses)
    gives the same bits, on ligands of 1-96 atoms mixed within blocks with a
    ragged pose count; the one-wavefront shape also matches the oracle."""
    ff, rec, grid, maps = system(2, grid_n=48, solpar=-0.0011, hbond=True)
    sizes = [(1, 0), (7, 1), (24, 6), (40, 10), (61, 12), (96, 20)]
    ligands = [synth.make_ligand(4, i, a, t, 8) for i, (a, t) in enumerate(sizes)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    stride = 7 + max(l.n_torsions for l in ligands)
    lo, hi = synth.pocket_box(grid, half=4.0)
    rng = np.random.default_rng(9)
    n = 1001
    pl = rng.integers(0, len(ligands), n).astype(np.int32)
    g = synth.sample_genotypes(13, n, stride - 7, stride, lo, hi)
    for p in range(n):
        g[p, 7 + ligands[pl[p]].n_torsions:] = 0
    runs = {}
    try:
        for lp in (1, 2, 4, 8):
            print("case: scoring split", lp, flush=True)
            dk.dock_score_set_split(lp)
            assert dk.dock_score_split(ligs) == lp
            runs[lp] = _gpu_energies(dk, pocket, ligs, g, pl)
    finally:
        dk.dock_score_set_split(0)
    np.testing.assert_array_equal(runs[2], runs[1])
    np.testing.assert_array_equal(runs[4], runs[1])
    np.testing.assert_array_equal(runs[8], runs[1])
    sub = np.arange(0, n, 7)
    e_ref = ora.score_poses(grid, maps, ff, ligands, g[sub], pose_ligand=pl[sub])
    keep = near_face_mask(ora, grid, ligands, g[sub], pl[sub])
    assert_energies_match(runs[1][sub], e_ref, keep)
    with pytest.raises(dk.DockError):
        dk.dock_score_set_split(3)


def test_automatic_split(dk):
    """The automatic scoring split follows the set's largest ligand (the fastest
    measured at each size): four wavefronts per block of 64 poses up to 64
    atoms, eight above, for every map layout; a fixed setting overrides it and
    0 restores it."""
    ff, rec, grid, maps = system(0)
    dk.dock_score_set_split(0)
    for layout in (dk.DOCK_LAYOUT_PAIRLINE, dk.DOCK_LAYOUT_QUADLINE, dk.DOCK_LAYOUT_ZPAIR):
        pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
        for atoms in (5, 16, 40, 64, 65, 96):
            ligs = dk.dock_create_ligands(pocket, [synth.make_ligand(1, 900 + atoms, 12, 2, 8),
                                                   synth.make_ligand(1, atoms, atoms, 3, 8)])
            assert dk.dock_score_split(ligs) == (4 if atoms <= 64 else 8), (layout, atoms)
    try:
        dk.dock_score_set_split(1)
        assert dk.dock_score_split(ligs) == 1
    finally:
        dk.dock_score_set_split(0)
    assert dk.dock_score_split(ligs) == 8


def test_max_torsions_and_types(dk, ora):
    """The limits of the ABI at once: 32 atom types (34 maps) and a ligand with
    32 torsions (39 genes), for every map layout and scoring split, plus
    the DE trial of a 39-gene genotype bit for bit against the oracle."""
    import torch
    import oracle
    nt = 32
    ff = synth.forcefield(nt)
    rec = synth.make_receptor(5, 400, nt)
    grid = synth.make_grid(40, nt)
    maps = oracle.build_maps(ff, rec, grid)
    lig = synth.make_ligand(1, 700, 70, 32, nt)
    assert lig.n_torsions == 32
    lo, hi = synth.pocket_box(grid, half=2.0)
    g = synth.sample_genotypes(17, 333, 32, 39, lo, hi)
    e_ref = ora.score_poses(grid, maps, ff, [lig], g)
    keep = near_face_mask(ora, grid, [lig], g)
    try:
        for layout in (0, 1, 2, 3, 4):
            pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
            ligs = dk.dock_create_ligands(pocket, [lig])
            for lp in (1, 2, 4, 8):
                print("case: 32 types, 32 torsions, layout", layout, "split", lp, flush=True)
                dk.dock_score_set_split(lp)
                assert_energies_match(_gpu_energies(dk, pocket, ligs, g), e_ref, keep)
    finally:
        dk.dock_score_set_split(0)
    P = 40
    params = dict(pop_size=P, n_generations=1, seed=9, box_lo=tuple(lo), box_hi=tuple(hi))
    pop = ora.de_init(lig, ora.SearchParams(**params), 0, 39)[None]
    tr = torch.zeros((1, P, 39), dtype=torch.float32, device="cuda")
    dk.dock_de_trials(ligs, dk.SearchParams(**params), 4, torch.from_numpy(pop).cuda(), tr)
    torch.cuda.synchronize()
    ref = ora.de_trials(lig, ora.SearchParams(**params), 0, 4, pop[0])
    assert np.array_equal(tr.cpu().numpy()[0].view(np.uint32), ref.view(np.uint32))
