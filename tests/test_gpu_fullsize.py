"""Full-size parity for the scoring microbenchmark workload (10^7 random poses of
one 40-atom, 10-torsion ligand on fourteen 100^3 maps), in the launch
configuration the benchmark times: every pose is scored on the GPU, a seeded
random sample is scored by the FP64 oracle, and properties that hold at any
size are checked on all of them."""
import numpy as np
import pytest

import synth
from tests._systems import assert_energies_match, near_face_mask

pytestmark = pytest.mark.gpu

N_POSES = 10_000_000
N_SAMPLE = 20_000


def test_config1_full_size_sampled_parity(ora):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock as dk
    c = synth.CONFIGS[1]
    nt = c["n_types"]
    ff = synth.forcefield(nt)
    rec = synth.make_receptor(1, 2000, nt)
    grid = synth.make_grid(c["grid_n"], nt)
    lig = synth.make_ligand(1, 0, c["atoms"], c["torsions"], nt)
    print("case: config1 full size, oracle maps 100^3", flush=True)
    maps = ora.build_maps(ff, rec, grid)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    assert pocket.layout == dk.DOCK_LAYOUT_QUADLINE
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    g = synth.sample_genotypes(1, N_POSES, lig.n_torsions, 7 + lig.n_torsions, lo, hi)
    gt = torch.from_numpy(g).cuda()
    e = torch.empty(N_POSES, dtype=torch.float32, device="cuda")
    dk.dock_score_poses(pocket, ligs, gt, e)
    torch.cuda.synchronize()
    e_all = e.cpu().numpy()
    # any size: every pose got a finite score (all genes are finite)
    assert np.isfinite(e_all).all()
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(N_POSES, N_SAMPLE, replace=False))
    idx = np.concatenate([idx, [0, N_POSES - 1]])
    ref = ora.score_poses(grid, maps, ff, [lig], g[idx])
    keep = near_face_mask(ora, grid, [lig], g[idx])
    assert keep.mean() > 0.99
    assert_energies_match(e_all[idx], ref, keep, what="config1 sample")
    # the same poses scored alone give the same values as inside the full batch
    e2 = torch.empty(len(idx), dtype=torch.float32, device="cuda")
    dk.dock_score_poses(pocket, ligs, torch.from_numpy(g[idx]).cuda(), e2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(e2.cpu().numpy(), e_all[idx])
