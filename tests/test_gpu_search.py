"""GPU parity of the differential-evolution search (the paper's evolutionary
search with the score as fitness, Sec. V): bit-identical random streams and
trial genotypes against the oracle, exact resume, and best-score distributions."""
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


def _ligs_cfg2(n):
    atoms, tors = synth.config_ligand_sizes(2)
    return [synth.make_ligand(1, i, int(atoms[i]), int(tors[i]), 8) for i in range(n)]


def _params(mod, lo, hi, **kw):
    base = dict(pop_size=64, n_generations=5, seed=1, box_lo=tuple(lo), box_hi=tuple(hi))
    base.update(kw)
    return mod.SearchParams(**base)


def test_init_population_bit_identical(dk, ora):
    import torch
    ff, rec, grid, maps = system(2, grid_n=48)
    ligands = _ligs_cfg2(6)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    P = 37
    pop = torch.full((6, P, stride), 9.0, dtype=torch.float32, device="cuda")
    dk.dock_de_init(ligs, _params(dk, lo, hi, pop_size=P, seed=99), pop)
    torch.cuda.synchronize()
    got = pop.cpu().numpy()
    for l, lig in enumerate(ligands):
        ref = ora.de_init(lig, _params(ora, lo, hi, pop_size=P, seed=99), l, stride)
        assert np.array_equal(got[l].view(np.uint32), ref.view(np.uint32)), l


def test_init_population_bit_identical_a_million(dk, ora):
    """The device and host Philox4x64-10 streams over 10^6 counters: the initial
    population of 10^6 individuals (each draws from its own stream, counter
    (individual, 0, ligand, purpose)) for two ligands and two seeds, bit for
    bit against the oracle's."""
    import torch
    ff, rec, grid, maps = system(0)
    ligands = [synth.make_ligand(1, 0, 24, 6, 8), synth.make_ligand(1, 7, 30, 9, 8)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 16
    P = 500_000
    for seed in (1, 0xFFFFFFFFFFFF):
        print("case: initial population of 2 x 500000, seed", seed, flush=True)
        pop = torch.full((2, P, stride), 7.0, dtype=torch.float32, device="cuda")
        dk.dock_de_init(ligs, _params(dk, lo, hi, pop_size=P, seed=seed), pop)
        torch.cuda.synchronize()
        got = pop.cpu().numpy()
        for l, lig in enumerate(ligands):
            ref = ora.de_init(lig, _params(ora, lo, hi, pop_size=P, seed=seed), l, stride)
            assert np.array_equal(got[l].view(np.uint32), ref.view(np.uint32)), (seed, l)


def test_trials_bit_identical(dk, ora):
    import torch
    ff, rec, grid, maps = system(2, grid_n=48)
    ligands = _ligs_cfg2(5)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    P = 50
    rng = np.random.default_rng(3)
    pop = np.zeros((5, P, stride), np.float32)
    for l, lig in enumerate(ligands):
        pop[l] = ora.de_init(lig, _params(ora, lo, hi, pop_size=P), l, stride)
        pop[l, :, :3] += rng.normal(0, 3, (P, 3)).astype(np.float32)   # some outside the box: clamp path
    for gen, (F, CR) in enumerate([(0.5, 0.9), (0.8, 0.3), (1.7, 1.0)]):
        tr = torch.zeros((5, P, stride), dtype=torch.float32, device="cuda")
        dk.dock_de_trials(ligs, _params(dk, lo, hi, pop_size=P, F=F, CR=CR, seed=5), gen + 3,
                          torch.from_numpy(pop).cuda(), tr)
        torch.cuda.synchronize()
        got = tr.cpu().numpy()
        for l, lig in enumerate(ligands):
            ref = ora.de_trials(lig, _params(ora, lo, hi, pop_size=P, F=F, CR=CR, seed=5), l, gen + 3, pop[l])
            assert np.array_equal(got[l].view(np.uint32), ref.view(np.uint32)), (gen, l)


def _run_gpu_search(dk, pocket, ligs, params, n_lig, stride, population=None, pop_energy=None, target=None,
                    gen_reached=None):
    import torch
    P = params.pop_size
    pop = torch.zeros((n_lig, P, stride), dtype=torch.float32, device="cuda") if population is None \
        else population.clone()
    pe = torch.zeros((n_lig, P), dtype=torch.float32, device="cuda") if pop_energy is None else pop_energy.clone()
    bg = torch.zeros((n_lig, stride), dtype=torch.float32, device="cuda")
    be = torch.zeros(n_lig, dtype=torch.float32, device="cuda")
    gr = None
    if target is not None:
        gr = torch.full((n_lig,), -1, dtype=torch.int32, device="cuda") if gen_reached is None else gen_reached.clone()
    dk.dock_search(pocket, ligs, params, pop, pe, bg, be, target=target, gen_reached=gr)
    torch.cuda.synchronize()
    return pop, pe, bg, be, gr


def test_resume_bit_identical_on_gpu(dk):
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    full = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=20), 1, 13)
    a = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=8), 1, 13)
    b = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=12, init=0, first_generation=8), 1, 13,
                        population=a[0], pop_energy=a[1])
    for x, y in zip(full[:4], b[:4]):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_search_energies_are_scores_and_improve(dk, ora):
    """After a GPU search every stored energy is the oracle score of its stored
    genotype (within tolerance), and the best improves on the initial population."""
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    p0 = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=0), 1, 13)
    p = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=100), 1, 13)
    pop = p[0].cpu().numpy()[0]
    pe = p[1].cpu().numpy()[0]
    ref = ora.score_poses(grid, maps, ff, [lig], pop)
    from tests._systems import assert_energies_match
    assert_energies_match(pe, ref)
    assert float(p[3].cpu()[0]) < float(p0[3].cpu()[0])
    assert float(p[3].cpu()[0]) == pe.min()


def _lockstep(dk, ora, pocket, ligs, grid, maps, ff, ligands, lo, hi, stride, pop, gens, seed):
    """The GPU search and the oracle's search of the same ligands from the same
    seed, each resumed one generation at a time from its own state (a resumed
    search is the uninterrupted one bit for bit, on both sides) and compared
    after every generation until every ligand's populations differ.  Returns
    (GPU best energies, oracle best energies, first diverging generation per
    ligand: the number of completed generations after which the two
    populations first differ, -1 if they never do)."""
    import torch
    nl = len(ligands)
    first = np.full(nl, -1)

    def cmp(g, gpu_pop, ora_pop):
        same = np.all(gpu_pop.cpu().numpy().view(np.uint32) == ora_pop.view(np.uint32), axis=(1, 2))
        first[(first < 0) & ~same] = g

    kw = dict(pop_size=pop, seed=seed)
    gs = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=0, **kw), nl, stride)
    os_ = ora.search(grid, maps, ff, ligands, _params(ora, lo, hi, n_generations=0, **kw), stride)
    cmp(0, gs[0], os_["population"])
    g = 0
    while g < gens:
        # one generation at a time while some ligand still agrees, then the rest at once
        step = 1 if np.any(first < 0) else gens - g
        gp = _params(dk, lo, hi, n_generations=step, init=0, first_generation=g, **kw)
        op = _params(ora, lo, hi, n_generations=step, init=0, first_generation=g, **kw)
        gs = _run_gpu_search(dk, pocket, ligs, gp, nl, stride, population=gs[0], pop_energy=gs[1])
        os_ = ora.search(grid, maps, ff, ligands, op, stride, population=os_["population"],
                         pop_energy=os_["pop_energy"])
        g += step
        if step == 1:
            cmp(g, gs[0], os_["population"])
    torch.cuda.synchronize()
    return gs[3].cpu().numpy().astype(np.float64), os_["best_energy"], first


def test_search_matches_oracle_lockstep_then_distribution(dk, ora):
    """Config 0 (24 atoms, 6 torsions, 40^3 maps; population 64, 100 generations)
    for 8 seeds.  Both sides draw the same random streams, so they agree exactly
    until a near-tie selection flips between FP32 and FP64; the first diverging
    generation of every run is reported, and none may come before generation
    10.  The best scores must agree in distribution: medians within 0.1
    kcal/mol and a two-sample KS p > 0.01."""
    from scipy.stats import ks_2samp
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    gpu_best, ora_best, firsts = [], [], []
    for seed in range(1, 9):
        gb, ob, first = _lockstep(dk, ora, pocket, ligs, grid, maps, ff, [lig], lo, hi, 13, 64, 100, seed)
        gpu_best.append(gb[0])
        ora_best.append(ob[0])
        firsts.append(int(first[0]))
    print("config 0: gpu best", np.round(gpu_best, 3), "oracle best", np.round(ora_best, 3), flush=True)
    print("config 0: first diverging generation per seed (-1: never)", firsts, flush=True)
    assert all(f < 0 or f >= 10 for f in firsts), firsts
    assert abs(np.median(gpu_best) - np.median(ora_best)) < 0.1
    assert ks_2samp(gpu_best, ora_best).pvalue > 0.01


def test_half_block_search_matches_oracle_lockstep(dk, ora):
    """Population 150 with one block per workgroup ends every generation with a
    half-block pass (22 individuals, two lanes each).  With splits 2, 4 and 8
    the GPU search stays in lockstep with the oracle's for at least 10
    generations (the oracle scores in FP64, so a near-tie selection may flip
    later), the three splits give the same bits, and every stored energy is the
    oracle's score of its stored genotype."""
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    bounds = [b for b, _, _ in dk.dock_search_shapes(ligs)]
    from tests._systems import assert_energies_match
    runs = []
    for split in (4, 2, 8):
        print("case: population 150, split", split, flush=True)
        dk.dock_search_set_shapes(ligs, [(b, split, 1) for b in bounds])
        if split == 4:
            gb, ob, first = _lockstep(dk, ora, pocket, ligs, grid, maps, ff, [lig], lo, hi, 13, 150, 30, 3)
            print("population 150: first diverging generation", int(first[0]), "gpu best", gb[0], "oracle best",
                  ob[0], flush=True)
            assert first[0] < 0 or first[0] >= 10, first
        r = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, pop_size=150, n_generations=30, seed=3), 1, 13)
        runs.append([x.cpu().numpy() for x in r[:4]])
    for other in runs[1:]:
        for x, y in zip(runs[0], other):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    ref = ora.score_poses(grid, maps, ff, [lig], runs[0][0][0])
    assert_energies_match(runs[0][1][0], ref)


def test_gen_reached(dk):
    import torch
    ff, rec, grid, maps = system(0)
    lig = synth.make_ligand(1, 0, 24, 6, 8)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    full = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=30), 1, 13)
    tgt = full[3].clone()
    r = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=30), 1, 13, target=tgt)
    gr = int(r[4].cpu()[0])
    assert 0 <= gr <= 30
    if gr > 0:
        part = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=gr - 1), 1, 13)
        assert float(part[3].cpu()[0]) > float(tgt.cpu()[0])
    r = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, n_generations=30), 1, 13, target=tgt - 1e4)
    assert int(r[4].cpu()[0]) == -1


def test_launch_shape_does_not_change_results(dk):
    """Splits of one, two, four and eight wavefronts per block, and every block
    count (including a block with no individual of its own), give the same
    search bit for bit (the energies sum the same partial sums in the same
    order); the autotuner fixes a valid shape per bucket and changes nothing.
    Population 75 ends each generation of a one-block workgroup with a half-block
    pass of 11 individuals (splits 2 and 4); population 178 with two blocks ends
    with a half-block pass of 50, over both blocks."""
    ff, rec, grid, maps = system(2, grid_n=48)
    atoms = [10, 14, 20, 31, 33, 40, 47, 52, 60, 70, 85, 96]
    ligands = [synth.make_ligand(1, 400 + i, n, min(12, n // 4), 8) for i, n in enumerate(atoms)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    bounds = [b for b, _, _ in dk.dock_search_shapes(ligs)]
    assert bounds == [16, 32, 48, 64, 96]
    for pop in (178, 75):
        print("case: launch shapes, population", pop, flush=True)
        params = _params(dk, lo, hi, pop_size=pop, n_generations=6)
        ref = None
        for lp in (1, 2, 4, 8):
            for w in (0, 1, 2, 3):
                if w * lp > 12:
                    continue   # at most twelve wavefronts per workgroup
                dk.dock_search_set_shapes(ligs, [(b, lp, w) for b in bounds])
                got = [x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs, params, len(ligands), stride)[:4]]
                if ref is None:
                    ref = got
                for x, y in zip(ref, got):
                    assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (pop, lp, w)
    dk.dock_search_autotune(pocket, ligs, params, stride, tune_generations=2)
    for b, lp, w in dk.dock_search_shapes(ligs):
        assert lp in (1, 2, 4, 8) and 1 <= w <= 12 // lp
    got = [x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs, params, len(ligands), stride)[:4]]
    for x, y in zip(ref, got):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    with pytest.raises(dk.DockError):
        dk.dock_search_set_shapes(ligs, [(b, 3, 0) for b in bounds])
    # stopping at a target: the same generations and bests with splits of one, two, four or eight
    import torch
    target = torch.from_numpy(ref[3] + 0.1).cuda()
    reached = []
    for lp in (1, 2, 4, 8):
        dk.dock_search_set_shapes(ligs, [(b, lp, 0) for b in bounds])
        stop = _params(dk, lo, hi, pop_size=75, n_generations=6, stop_at_target=1)
        r = _run_gpu_search(dk, pocket, ligs, stop, len(ligands), stride, target=target)
        reached.append((r[4].cpu().numpy(), r[3].cpu().numpy()))
    for k in (1, 2, 3):
        np.testing.assert_array_equal(reached[0][0], reached[k][0])
        np.testing.assert_array_equal(reached[0][1], reached[k][1])
    assert np.all((reached[0][0] >= 0) & (reached[0][0] <= 6))
    assert np.all(reached[0][1] <= ref[3] + 0.1)


def test_quad_line_and_pair_line_search_same_bits(dk):
    """A whole search reads its maps through either line layout with the same
    results bit for bit: populations, energies and bests."""
    ff, rec, grid, maps = system(2, grid_n=48)
    ligands = _ligs_cfg2(10)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    params = _params(dk, lo, hi, pop_size=50, n_generations=8)
    runs = []
    for layout in (dk.DOCK_LAYOUT_QUADLINE, dk.DOCK_LAYOUT_PAIRLINE):
        print("case: search with layout", layout, flush=True)
        pocket = dk.dock_create_pocket(grid, maps, ff, layout=layout)
        assert pocket.layout == layout
        ligs = dk.dock_create_ligands(pocket, ligands)
        runs.append([x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs, params, len(ligands), stride)[:4]])
    for x, y in zip(*runs):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_tune_cache_file_applies_to_new_handles(dk, tmp_path):
    """Tuned shapes saved to a file name this device's kind, pocket and buckets;
    loaded back (edited), they are what a new handle for the same ligands uses,
    and the search gives the same bits."""
    ff, rec, grid, maps = system(2, grid_n=48)
    atoms = [12, 20, 31, 40, 47, 60, 85]
    ligands = [synth.make_ligand(1, 500 + i, n, min(10, n // 4), 8) for i, n in enumerate(atoms)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    params = _params(dk, lo, hi, pop_size=75, n_generations=4)
    print("case: tune cache file, 7 ligands, pop 75", flush=True)
    dk.dock_search_autotune(pocket, ligs, params, stride, tune_generations=2)
    tuned = {b: (lp, w) for b, lp, w in dk.dock_search_shapes(ligs)}
    largest = {}
    for n in atoms:
        b = min(x for x in tuned if x >= n)
        largest[b] = max(largest.get(b, 0), n)
    path = tmp_path / "tune.txt"
    dk.dock_search_tune_save(path)
    mine = {}
    for line in path.read_text().splitlines()[1:]:
        f = line.split()
        key = [int(x) for x in f[1:10]]
        if key[1:6] == [pocket.layout, 48, 48, 48, 8] and key[8] == 75 and largest.get(key[6]) == key[7]:
            mine[key[6]] = (key[7], int(f[10]), int(f[11]))
    assert set(mine) == set(largest)
    for b, (lig_max, lp, w) in mine.items():
        assert lig_max == largest[b] and (lp, w) == tuned[b]
    # edit this pocket's lines to other shapes and load them
    edited, want = [], {}
    for line in path.read_text().splitlines()[1:]:
        f = line.split()
        b = int(f[7])
        if (b in mine and int(f[2]) == pocket.layout and int(f[3]) == 48 and int(f[9]) == 75
                and int(f[8]) == largest[b]):
            lp = {1: 2, 2: 4, 4: 8, 8: 1}[int(f[10])]
            f[10], f[11] = str(lp), "1"
            want[b] = (lp, 1)
        edited.append(" ".join(f))
    path.write_text("\n".join(edited) + "\n")
    dk.dock_search_tune_load(path)
    # a new handle: the autotuner finds every bucket in the cache and fixes the
    # loaded shapes without timing (timing would not have chosen the edits)
    ligs2 = dk.dock_create_ligands(pocket, ligands)
    dk.dock_search_autotune(pocket, ligs2, params, stride, tune_generations=2)
    for b, lp, w in dk.dock_search_shapes(ligs2):
        if b in want:
            assert (lp, w) == want[b]
    a = [x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs, params, len(ligands), stride)[:4]]
    c = [x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs2, params, len(ligands), stride)[:4]]
    for x, y in zip(a, c):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_search_plan_graph_replays(dk):
    """A search captured into a HIP graph gives, on every replay (with eager work
    and synchronisations between the replays), exactly dock_search's result --
    plain, learned, and stopping at targets."""
    import torch
    ff, rec, grid, maps = system(2, grid_n=48)
    atoms = [12, 20, 31, 40, 52, 70, 90]
    ligands = [synth.make_ligand(1, 500 + i, n, min(10, n // 4), 8) for i, n in enumerate(atoms)]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    nl = len(ligands)
    net = dk.dock_mlp_create(0, 5)
    cases = [dict(), dict(proposal=net, proposal_step=0.5, proposal_every=2, proposal_until=5)]
    for kw in cases:
        params = _params(dk, lo, hi, pop_size=75, n_generations=6, **kw)
        ref = [x.cpu().numpy() for x in _run_gpu_search(dk, pocket, ligs, params, nl, stride)[:4]]
        buf = [torch.zeros((nl, 75, stride), dtype=torch.float32, device="cuda"),
               torch.zeros((nl, 75), dtype=torch.float32, device="cuda"),
               torch.zeros((nl, stride), dtype=torch.float32, device="cuda"),
               torch.zeros(nl, dtype=torch.float32, device="cuda")]
        plan = dk.dock_search_plan_create(pocket, ligs, params, *buf)
        for rep in range(3):
            for b in buf:
                b.fill_(7.0)                       # eager work between replays
            dk.dock_search_plan_launch(plan)
            torch.cuda.synchronize()
            for x, y in zip(ref, buf):
                assert np.array_equal(x.view(np.uint32), y.cpu().numpy().view(np.uint32)), (kw.keys(), rep)
            _run_gpu_search(dk, pocket, ligs, params, nl, stride)   # an eager search in between
        del plan
    # stopping at targets
    params = _params(dk, lo, hi, pop_size=75, n_generations=6, stop_at_target=1)
    target = torch.from_numpy(ref[3] + 0.5).cuda()
    r = _run_gpu_search(dk, pocket, ligs, params, nl, stride, target=target)
    want = [x.cpu().numpy() for x in r[:4]] + [r[4].cpu().numpy()]
    buf = [torch.zeros((nl, 75, stride), dtype=torch.float32, device="cuda"),
           torch.zeros((nl, 75), dtype=torch.float32, device="cuda"),
           torch.zeros((nl, stride), dtype=torch.float32, device="cuda"),
           torch.zeros(nl, dtype=torch.float32, device="cuda"), target,
           torch.full((nl,), -5, dtype=torch.int32, device="cuda")]
    plan = dk.dock_search_plan_create(pocket, ligs, params, *buf)
    for rep in range(2):
        buf[5].fill_(-5)
        dk.dock_search_plan_launch(plan)
        torch.cuda.synchronize()
        for x, y in zip(want, buf[:4] + buf[5:]):
            assert np.array_equal(x.view(np.uint32), y.cpu().numpy().view(np.uint32)), rep


@pytest.mark.parametrize("pop", [4, 1000])
def test_search_population_extremes(dk, ora, pop):
    """The smallest population DE allows (4: every trial draws the three other
    members) and one far above a workgroup's lanes (1000), on ligands of 10, 40
    and 90 atoms: stored energies are the oracle's scores of the stored
    genotypes, the best is the first minimum, and a split-and-resumed search is
    the same bits as one call."""
    from tests._systems import assert_energies_match, near_face_mask
    ff, rec, grid, maps = system(2, grid_n=48)
    ligands = [synth.make_ligand(3, 600 + i, n, t, 8) for i, (n, t) in enumerate([(10, 2), (40, 10), (90, 15)])]
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    print("case: population", pop, flush=True)
    full = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, pop_size=pop, n_generations=8), 3, stride)
    half = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, pop_size=pop, n_generations=4), 3, stride)
    rest = _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, pop_size=pop, n_generations=4, init=0,
                                                     first_generation=4), 3, stride,
                           population=half[0], pop_energy=half[1])
    for x, y in zip(full[:4], rest[:4]):
        assert np.array_equal(x.cpu().numpy().view(np.uint32), y.cpu().numpy().view(np.uint32))
    pop_np, pe, bg, be = (x.cpu().numpy() for x in full[:4])
    np.testing.assert_array_equal(be, pe.min(axis=1))
    np.testing.assert_array_equal(bg, pop_np[np.arange(3), pe.argmin(axis=1)])
    rng = np.random.default_rng(pop)
    members = np.sort(rng.choice(pop, min(pop, 48), replace=False))
    geno = np.concatenate([pop_np[l, members] for l in range(3)])
    pl = np.repeat(np.arange(3, dtype=np.int32), len(members))
    ref = ora.score_poses(grid, maps, ff, ligands, geno, pose_ligand=pl)
    keep = near_face_mask(ora, grid, ligands, geno, pl)
    assert_energies_match(np.concatenate([pe[l, members] for l in range(3)]), ref, keep)
    with pytest.raises(dk.DockError):
        _run_gpu_search(dk, pocket, ligs, _params(dk, lo, hi, pop_size=3, n_generations=1), 3, stride)


def test_handles_release_device_memory(dk):
    """Pockets (with their packed map copy), ligand sets (with side streams),
    search plans and networks give back their device memory when destroyed:
    twenty create/use/destroy cycles leave free memory where one cycle left it."""
    import gc
    import torch
    ff, rec, grid, maps = system(2, grid_n=48)
    ligands = [synth.make_ligand(1, 800 + i, n, 5, 8) for i, n in enumerate([14, 30, 50])]
    lo, hi = synth.pocket_box(grid)
    params = _params(dk, lo, hi, pop_size=64, n_generations=2)

    def cycle():
        pocket = dk.dock_create_pocket(grid, maps, ff)
        ligs = dk.dock_create_ligands(pocket, ligands)
        out = _run_gpu_search(dk, pocket, ligs, params, 3, 12)
        plan = dk.dock_search_plan_create(pocket, ligs, params, *[x.clone() for x in out[:4]])
        dk.dock_search_plan_launch(plan)
        net = dk.dock_mlp_create(0, 3)
        torch.cuda.synchronize()
        del plan, net, ligs, pocket, out
        gc.collect()
        torch.cuda.synchronize()

    cycle()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        cycle()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    print("free device memory drift over 20 cycles:", (free0 - free1) / 2**20, "MiB", flush=True)
    assert free0 - free1 < 32 * 2**20


def test_config2_subset_best_scores_match_oracle(dk, ora):
    """The first 20 ligands of the 1000-ligand batch (10-60 atoms, 0-15
    torsions, ten 64^3 maps, population 128 x 200 generations), 8 seeds each,
    searched by the GPU and by the oracle on the oracle's maps.  The two draw the
    same random streams, so a ligand's search agrees exactly until a near-tie
    selection flips between FP32 and FP64; the first diverging generation of
    every (ligand, seed) is reported.  The 160 best scores must agree in
    distribution: medians within 0.1 kcal/mol and a two-sample KS p > 0.01."""
    from scipy.stats import ks_2samp
    c = synth.CONFIGS[2]
    ff, rec, grid, maps = system(2)
    ligands = synth.config_ligands(2, count=20)
    pocket = dk.dock_create_pocket(grid, maps, ff)
    ligs = dk.dock_create_ligands(pocket, ligands)
    lo, hi = synth.pocket_box(grid)
    stride = 7 + max(l.n_torsions for l in ligands)
    gpu_best, ora_best, firsts = [], [], []
    for seed in range(1, 9):
        print("case: config2 first 20 ligands, seed", seed, flush=True)
        gb, ob, first = _lockstep(dk, ora, pocket, ligs, grid, maps, ff, ligands, lo, hi, stride, c["pop"],
                                  c["gens"], seed)
        gpu_best += list(gb)
        ora_best += list(ob)
        firsts.append(first)
    gpu_best, ora_best, firsts = np.array(gpu_best), np.array(ora_best), np.array(firsts)
    div = firsts[firsts >= 0]
    print("config 2 subset: median best gpu", np.median(gpu_best), "oracle", np.median(ora_best), flush=True)
    print(f"config 2 subset: {int((firsts < 0).sum())} of {firsts.size} searches identical to the end; first "
          f"diverging generation of the others: min {div.min() if div.size else None}, median "
          f"{np.median(div) if div.size else None}", flush=True)
    print("config 2 subset: first diverging generation [seed][ligand] (-1: never)", firsts.tolist(), flush=True)
    assert abs(np.median(gpu_best) - np.median(ora_best)) < 0.1
    assert ks_2samp(gpu_best, ora_best).pvalue > 0.01
