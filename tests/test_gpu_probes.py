"""The roofline probes run through the C ABI and reject bad arguments."""
import numpy as np
import pytest

import synth
from tests._systems import system

pytestmark = pytest.mark.gpu


def test_probes_run_and_validate():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock as dk
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    lo, hi = synth.pocket_box(grid)
    for layout in (0, 1, 2, 3, 4):
        pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
        ligs = dk.dock_create_ligands(pocket, [lig])
        for in_flight in (2, 4, 8):
            out = torch.full((1000,), np.nan, dtype=torch.float32, device="cuda")   # not a multiple of 256
            dk.dock_gather_probe(pocket, ligs, 0, lo, hi, out, 8, in_flight=in_flight)
            torch.cuda.synchronize()
            assert torch.isfinite(out).all()
    out = torch.full((777,), np.nan, dtype=torch.float32, device="cuda")
    dk.dock_pair_probe(pocket, out, 16)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    with pytest.raises(dk.DockError):
        dk.dock_gather_probe(pocket, ligs, 1, lo, hi, out, 8)      # ligand index out of range
    with pytest.raises(dk.DockError):
        dk.dock_gather_probe(pocket, ligs, 0, lo, hi, out, 8, in_flight=3)
    with pytest.raises(dk.DockError):
        dk.dock_gather_probe(pocket, ligs, 0, lo, hi, out, 12, in_flight=8)   # not a multiple
    with pytest.raises(dk.DockError):
        dk.dock_pair_probe(pocket, out, 6)                         # per_lane not a multiple of 4
