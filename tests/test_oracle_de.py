"""Pins of the oracle's random stream (Philox4x64-10 against numpy's
implementation of the same generator) and of its differential-evolution search
(the paper's evolutionary search with the score as fitness, Sec. V)."""
import numpy as np
import pytest

import synth

NT = 8


def test_philox4x64_matches_numpy(ora):
    """numpy.random.Philox is Philox4x64-10; it increments the counter before
    producing each block of four 64-bit words."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2, dtype=np.uint64)]
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, 4, dtype=np.uint64)]
        ctr[0] |= 1   # no carry out of word 0 on the increment below
        bg = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
        expect = bg.random_raw(4).astype(np.uint64)
        got = ora.philox4x64([ctr[0] + 1] + ctr[1:], key)
        assert np.array_equal(got, expect)
    # all-zero and all-ones corners
    for fill in (0, 2 ** 64 - 1):
        key = [fill, fill]
        ctr = [fill] * 4
        bg = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
        expect = bg.random_raw(4).astype(np.uint64)
        nxt = [(ctr[0] + 1) % 2 ** 64, ctr[1] + (1 if fill else 0), ctr[2], ctr[3]]
        if fill:   # carry ripples through every word
            nxt = [0, 0, 0, 0]
        got = ora.philox4x64(nxt, key)
        assert np.array_equal(got, expect)


def _setup(n_lig=2, n_atoms=(24, 18), n_tor=(6, 4), grid_n=24):
    ff = synth.forcefield(NT)
    rec = synth.make_receptor(1, 600, NT)
    grid = synth.make_grid(grid_n, NT, spacing=0.5)
    maps = ora_maps_cache(ff, rec, grid)
    ligs = [synth.make_ligand(1, i, n_atoms[i], n_tor[i], NT) for i in range(n_lig)]
    lo, hi = synth.pocket_box(grid, half=3.0)
    return ff, grid, maps, ligs, lo, hi


_MAPS = {}


def ora_maps_cache(ff, rec, grid):
    import oracle
    key = (grid.dims, grid.spacing, ff.n_types, len(rec.type))
    if key not in _MAPS:
        _MAPS[key] = oracle.build_maps(ff, rec, grid)
    return _MAPS[key]


def _params(ora, lo, hi, **kw):
    base = dict(pop_size=24, n_generations=10, seed=1, box_lo=tuple(lo), box_hi=tuple(hi))
    base.update(kw)
    return ora.SearchParams(**base)


def test_init_population_in_domain(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    p = _params(ora, lo, hi, pop_size=500)
    pop = ora.de_init(ligs[0], p, 0, 16)
    assert np.all(pop[:, 0:3] >= np.float32(lo) - 0) and np.all(pop[:, 0:3] <= np.float32(hi))
    qn = (pop[:, 3:7].astype(np.float64) ** 2).sum(1)
    assert np.all(qn > 0) and np.all(qn <= 1.0 + 1e-6)
    th = pop[:, 7:13]
    assert np.all(th >= -np.pi - 1e-6) and np.all(th <= np.pi + 1e-6)
    assert np.all(pop[:, 13:] == 0)
    # orientations uniform on the rotation group: E[w^2] = 1/4 for each quaternion component
    qu = pop[:, 3:7] / np.sqrt(qn)[:, None]
    np.testing.assert_allclose((qu ** 2).mean(0), 0.25, atol=0.04)


def test_trial_partners_distinct(ora):
    """With F = 1/1024 and CR = 1 every gene is x_r1 + (x_r2 - x_r3)/1024; encoding
    the row index r as gene 3 = r and gene 4 = r^2 lets the test recover r1, r2, r3."""
    lig = synth.make_ligand(1, 0, 24, 6, NT)
    P = 40
    p = ora.SearchParams(pop_size=P, n_generations=1, seed=7, box_lo=(-1e3,) * 3, box_hi=(1e3,) * 3,
                         F=1 / 1024, CR=1.0)
    pop = np.zeros((P, 13), np.float32)
    pop[:, 3] = np.arange(P)
    pop[:, 4] = np.arange(P) ** 2
    for gen in range(5):
        tr = ora.de_trials(lig, p, 0, gen, pop)
        for i in range(P):
            v3, v4 = float(tr[i, 3]), float(tr[i, 4])
            r1 = int(round(v3))
            d = round((v3 - r1) * 1024)          # r2 - r3
            s = round((v4 - r1 * r1) * 1024)     # r2^2 - r3^2
            assert d != 0
            r2 = (s // d + d) // 2
            r3 = r2 - d
            assert len({i, r1, r2, r3}) == 4 and 0 <= min(r1, r2, r3) and max(r1, r2, r3) < P


def test_trial_crossover_rates(ora):
    lig = synth.make_ligand(1, 0, 24, 6, NT)
    P = 64
    rng = np.random.default_rng(2)
    pop = rng.uniform(-1, 1, (P, 13)).astype(np.float32)
    p0 = ora.SearchParams(pop_size=P, n_generations=1, seed=3, box_lo=(-5,) * 3, box_hi=(5,) * 3,
                          F=0.5, CR=0.0)
    tr = ora.de_trials(lig, p0, 0, 0, pop)
    changed = (tr != pop).sum(1)
    assert np.all(changed <= 1) and changed.mean() > 0.9   # only the forced gene j_rand
    p1 = ora.SearchParams(pop_size=P, n_generations=1, seed=3, box_lo=(-5,) * 3, box_hi=(5,) * 3,
                          F=0.0, CR=1.0)
    tr = ora.de_trials(lig, p1, 0, 0, pop)
    # F = 0: every trial equals some other member (the base vector r1), torsions wrapped
    for i in range(P):
        assert any(np.array_equal(tr[i], pop[r]) for r in range(P) if r != i)


def test_trial_wraps_torsions_and_clamps_translation(ora):
    lig = synth.make_ligand(1, 0, 24, 6, NT)
    P = 32
    rng = np.random.default_rng(4)
    pop = np.zeros((P, 13), np.float32)
    pop[:, 0:3] = rng.uniform(-2, 2, (P, 3))
    pop[:, 3:7] = rng.normal(size=(P, 4))
    pop[:, 7:] = rng.uniform(-np.pi, np.pi, (P, 6))
    p = ora.SearchParams(pop_size=P, n_generations=1, seed=5, box_lo=(-1.0,) * 3, box_hi=(1.5,) * 3,
                         F=0.9, CR=1.0)
    tr = ora.de_trials(lig, p, 0, 3, pop)
    assert np.all(tr[:, 0:3] >= -1.0) and np.all(tr[:, 0:3] <= 1.5)
    assert np.all(tr[:, 7:] > -np.pi - 1e-6) and np.all(tr[:, 7:] <= np.pi + 1e-6)


def test_search_reproducible_and_seed_dependent(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    p = _params(ora, lo, hi)
    a = ora.search(grid, maps, ff, ligs, p, 16)
    b = ora.search(grid, maps, ff, ligs, p, 16, n_threads=1)
    assert np.array_equal(a["population"], b["population"])
    assert np.array_equal(a["best_energy"], b["best_energy"])
    c = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, seed=2), 16)
    assert not np.array_equal(a["population"], c["population"])


def test_resume_is_bit_identical(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    full = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, n_generations=12), 16)
    part = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, n_generations=5), 16)
    rest = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, n_generations=7, init=0, first_generation=5),
                      16, population=part["population"], pop_energy=part["pop_energy"])
    assert np.array_equal(full["population"], rest["population"])
    assert np.array_equal(full["pop_energy"], rest["pop_energy"])
    assert np.array_equal(full["best_energy"], rest["best_energy"])


def test_best_monotone_and_improves(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    r = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, n_generations=0), 16)
    bests = [r["best_energy"].copy()]
    for g in range(15):
        r = ora.search(grid, maps, ff, ligs, _params(ora, lo, hi, n_generations=1, init=0, first_generation=g),
                       16, population=r["population"], pop_energy=r["pop_energy"])
        bests.append(r["best_energy"].copy())
    bests = np.array(bests)
    assert np.all(np.diff(bests, axis=0) <= 0)
    assert np.all(bests[-1] < bests[0])
    # the stored population energies are the scores of the stored genotypes
    for l, lig in enumerate(ligs):
        e = ora.score_poses(grid, maps, ff, [lig], r["population"][l])
        np.testing.assert_array_equal(e, r["pop_energy"][l])


def test_gen_reached_target(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    p = _params(ora, lo, hi, n_generations=20)
    r = ora.search(grid, maps, ff, ligs, p, 16)
    # target = the final best: reached exactly at the generation that first produced it
    r2 = ora.search(grid, maps, ff, ligs, p, 16, target=r["best_energy"])
    assert np.all(r2["gen_reached"] >= 0) and np.all(r2["gen_reached"] <= 20)
    r3 = ora.search(grid, maps, ff, ligs, p, 16, target=r["best_energy"] - 1e6)
    assert np.all(r3["gen_reached"] == -1)


def test_invalid_descriptors_rejected(ora):
    ff, grid, maps, ligs, lo, hi = _setup()
    lig = ligs[0]
    bad_tree = synth.Ligand(lig.xyz, lig.type, lig.charge, np.vstack([lig.bonds[:-1], [[1, 2]]]).astype(np.int32),
                            lig.torsion_bonds)
    with pytest.raises(ValueError):
        ora.score_poses(grid, maps, ff, [bad_tree], np.zeros((1, 16), np.float32))
    term = int(np.flatnonzero(np.bincount(lig.bonds.ravel(), minlength=lig.n_atoms) == 1)[0])
    tb = int(np.flatnonzero((lig.bonds == term).any(1))[0])
    bad_tor = synth.Ligand(lig.xyz, lig.type, lig.charge, lig.bonds, np.array([tb], np.int32))
    with pytest.raises(ValueError):
        ora.score_poses(grid, maps, ff, [bad_tor], np.zeros((1, 16), np.float32))
    bad_type = synth.Ligand(lig.xyz, lig.type + NT, lig.charge, lig.bonds, lig.torsion_bonds)
    with pytest.raises(ValueError):
        ora.score_poses(grid, maps, ff, [bad_type], np.zeros((1, 16), np.float32))
