"""GPU map builder (AutoGrid-like step, Sec. V) against the oracle's FP64 maps."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_gpu_maps_match_oracle(ora):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock as dk
    nt = 8
    ff = synth.forcefield(nt, solpar=-0.0009, hbond_pairs=[(1, 5)])
    rec = synth.make_receptor(3, 700, nt)
    grid = synth.make_grid((21, 18, 23), nt, spacing=0.5)
    ref = ora.build_maps(ff, rec, grid)
    pocket = dk.dock_create_pocket_from_receptor(grid, ff, rec)
    out = torch.zeros(ref.size, dtype=torch.float32, device="cuda")
    dk.dock_pocket_maps(pocket, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(ref.shape)
    # FP32 accumulation of <= 700 bounded terms per node
    tol = 2e-3 + 1e-4 * np.abs(ref)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()))
    # clamps hold exactly
    assert got[:nt].max() <= ff.map_cap and got[nt].min() >= -ff.map_cap and got[nt + 1].max() <= ff.map_cap


@pytest.mark.parametrize("variant", ["plain", "hbond_solpar"])
def test_gpu_built_maps_give_oracle_energies(ora, variant):
    """Energies scored on a pocket whose maps the GPU built from the receptor
    match the oracle's energies on the oracle's own maps (the same receptor, FP64
    build), within the energy tolerance: 1e-4 relative or 1e-3 kcal/mol, per pose
    (the single-ligand workload's 2000-atom receptor and 40^3 grid; 24-atom
    ligand; 3000 poses in the pocket box; poses with an atom within 1e-4 cells
    of a face excluded)."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock as dk
    from tests._systems import assert_energies_match, near_face_mask
    nt = 8
    ff = synth.forcefield(nt, solpar=-0.0009, hbond_pairs=[(1, 5), (2, 2)]) if variant != "plain" \
        else synth.forcefield(nt)
    rec = synth.make_receptor(1, 2000, nt)
    grid = synth.make_grid(40, nt)
    lig = synth.make_ligand(1, 0, 24, 6, nt)
    print("case: GPU-built maps, energies,", variant, flush=True)
    pocket = dk.dock_create_pocket_from_receptor(grid, ff, rec)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    g = synth.sample_genotypes(11, 3000, lig.n_torsions, 7 + lig.n_torsions, lo, hi)
    e = torch.empty(len(g), dtype=torch.float32, device="cuda")
    dk.dock_score_poses(pocket, ligs, torch.from_numpy(g).cuda(), e)
    torch.cuda.synchronize()
    got = e.cpu().numpy()
    ref = ora.score_poses(grid, ora.build_maps(ff, rec, grid), ff, [lig], g)
    keep = near_face_mask(ora, grid, [lig], g)
    assert keep.mean() > 0.9
    assert np.isfinite(got[keep]).all()
    assert_energies_match(got, ref, keep, what=f"energies on GPU-built maps ({variant})")
