"""MI355X (gfx950) docking hot path: batched pose scoring and differential
evolution behind the C ABI of include/dock.h.

``paper_2509_12232_amd.dock`` is the binding (importing it requires the built
``libdock.so``); ``paper_2509_12232_amd.build`` compiles it with hipcc;
``paper_2509_12232_amd.proposal`` sequences ABI calls into the learned
proposal's training recipe and the time-to-target runs.

A minimal session (device buffers are torch tensors on ``cuda:0``)::

    import torch, synth
    from paper_2509_12232_amd import dock as dk
    ff = synth.forcefield(12)
    grid = synth.make_grid(80, 12)
    pocket = dk.dock_create_pocket_from_receptor(grid, ff, synth.make_receptor(1, 2000, 12))
    ligs = dk.dock_create_ligands(pocket, synth.config_ligands(3, count=100))
    lo, hi = synth.pocket_box(grid)
    # score poses: genotypes [n][g_stride] = t(3), q(4), torsions, zero padding
    g = torch.from_numpy(synth.sample_genotypes(1, 10_000, 20, 27, lo, hi)).cuda()
    e = torch.empty(10_000, device="cuda")
    dk.dock_score_poses(pocket, ligs, g, e, pose_ligand=torch.zeros(10_000, dtype=torch.int32, device="cuda"))
    # search every ligand (launch shapes tuned once per process, or loaded)
    p = dk.SearchParams(pop_size=150, n_generations=300, seed=1, box_lo=tuple(lo), box_hi=tuple(hi))
    dk.dock_search_autotune(pocket, ligs, p, 27)
    pop = torch.zeros((ligs.n, 150, 27), device="cuda")
    pe, bg, be = torch.zeros((ligs.n, 150), device="cuda"), torch.zeros((ligs.n, 27), device="cuda"), \\
        torch.zeros(ligs.n, device="cuda")
    dk.dock_search(pocket, ligs, p, pop, pe, bg, be)   # best energies in be, genotypes in bg
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdock.so")
