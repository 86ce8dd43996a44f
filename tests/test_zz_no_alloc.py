"""dock_search_no_alloc, the search on the library's fixed per-device scratch,
against dock_search on the same inputs: the same bits for every output, on two
calls in a row (the second one smaller, so it runs on what the first left in
the scratch), and a search too large for the scratch rejected before any work."""
import numpy as np
import pytest

import synth
from tests._systems import system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dk():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_12232_amd import dock
    return dock


def _buffers(n, pop, stride, with_target):
    import torch
    b = dict(pop=torch.zeros((n, pop, stride), dtype=torch.float32, device="cuda"),
             pe=torch.zeros((n, pop), dtype=torch.float32, device="cuda"),
             bg=torch.zeros((n, stride), dtype=torch.float32, device="cuda"),
             be=torch.zeros(n, dtype=torch.float32, device="cuda"),
             gr=torch.full((n,), -7, dtype=torch.int32, device="cuda") if with_target else None)
    return b


def _search(fn, pocket, ligs, params, b, target):
    fn(pocket, ligs, params, b["pop"], b["pe"], b["bg"], b["be"], target=target, gen_reached=b["gr"])


def _bits(b):
    return {k: v.cpu().numpy().view(np.uint32 if v.dtype.is_floating_point else np.int32)
            for k, v in b.items() if v is not None}


def test_no_alloc_search_matches_dock_search_twice(dk):
    import torch
    ff, rec, grid, maps = system(2, grid_n=48)
    atoms, tors = synth.config_ligand_sizes(2)
    ligands = [synth.make_ligand(1, i, int(atoms[i]), int(tors[i]), 8) for i in range(24)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    lo, hi = synth.pocket_box(grid)
    net = dk.dock_mlp_create(0, 5)
    # call 1: 24 ligands, pop 96, 14 generations, proposal rounds from a seeded
    # network, targets recorded (no stop); call 2: 7 ligands, pop 40, 9 plain generations
    cases = [
        (ligands, dict(pop_size=96, n_generations=14, seed=3, proposal=net, proposal_step=1.0, proposal_every=5,
                       proposal_until=100), True),
        (ligands[:7], dict(pop_size=40, n_generations=9, seed=4), False),
    ]
    for k, (ls, kw, with_target) in enumerate(cases):
        print(f"no-alloc case {k}: {len(ls)} ligands, pop {kw['pop_size']}, {kw['n_generations']} generations",
              flush=True)
        ligs = dk.dock_create_ligands(pocket, ls)
        stride = 7 + max(l.n_torsions for l in ls)
        params = dk.SearchParams(box_lo=tuple(lo), box_hi=tuple(hi), **kw)
        target = None
        if with_target:
            # a level about half of the ligands reach within the run
            pre = _buffers(len(ls), kw["pop_size"], stride, False)
            _search(dk.dock_search, pocket, ligs, dk.SearchParams(box_lo=tuple(lo), box_hi=tuple(hi),
                                                                   **dict(kw, n_generations=4)), pre, None)
            target = pre["be"] - 0.5
        ref = _buffers(len(ls), kw["pop_size"], stride, with_target)
        got = _buffers(len(ls), kw["pop_size"], stride, with_target)
        _search(dk.dock_search, pocket, ligs, params, ref, target)
        _search(dk.dock_search_no_alloc, pocket, ligs, params, got, target)
        torch.cuda.synchronize()
        r, g = _bits(ref), _bits(got)
        for name in r:
            assert np.array_equal(r[name], g[name]), (k, name)
        if with_target:
            gr = ref["gr"].cpu().numpy()
            assert (gr >= 0).any() and (gr >= -1).all(), gr
        assert np.isfinite(ref["pe"].cpu().numpy()).all()


def test_no_alloc_rejects_a_search_beyond_its_scratch(dk):
    import torch
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    stride = 13
    # one ligand x pop x 13 floats, twice, just over the fixed scratch
    pop = (dk.DOCK_NO_ALLOC_SCRATCH_BYTES - 256) // (2 * 4 * stride) + 1
    b = _buffers(1, pop, stride, False)
    b["pe"].fill_(3.0)
    params = dk.SearchParams(pop_size=pop, n_generations=1, seed=1, box_lo=tuple(lo), box_hi=tuple(hi))
    with pytest.raises(dk.DockError) as ei:
        _search(dk.dock_search_no_alloc, pocket, ligs, params, b, None)
    assert ei.value.status == dk.DOCK_E_INVALID and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((b["pe"] == 3.0).all())   # nothing was enqueued
