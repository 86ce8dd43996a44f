"""Pins of the oracle's intra-energy term (ligand atom pairs, Sec. V, Algorithm 2):
closed-form properties of each pair term, the pair-list rule checked by an
independent enumeration, and invariances of the total."""
import math

import numpy as np
import pytest

import synth

NT = 8


def _ff(**over):
    ff = synth.forcefield(NT)
    for k, v in over.items():
        setattr(ff, k, v)
    return ff


def test_lj_12_6_minimum_is_minus_eps_at_req(ora):
    ff = _ff(qsolpar=0.0)
    for ti, tj in [(0, 0), (2, 5), (7, 1)]:
        req = 0.5 * (float(ff.Rii[ti]) + float(ff.Rii[tj]))
        eps = math.sqrt(float(ff.epsii[ti]) * float(ff.epsii[tj]))
        e0 = ora.pair_energy(ff, ti, tj, 0.0, 0.0, req)
        assert e0 == pytest.approx(-eps, rel=1e-12)
        h = 1e-5
        de = (ora.pair_energy(ff, ti, tj, 0, 0, req + h) - ora.pair_energy(ff, ti, tj, 0, 0, req - h)) / (2 * h)
        assert abs(de) < 1e-8
        # zero crossing of the 12-6 form at req / 2^(1/6)
        assert ora.pair_energy(ff, ti, tj, 0, 0, req / 2 ** (1 / 6)) == pytest.approx(0.0, abs=1e-12)
        # attractive tail falls as r^-6
        r1, r2 = 3 * req, 6 * req
        ratio = ora.pair_energy(ff, ti, tj, 0, 0, r1) / ora.pair_energy(ff, ti, tj, 0, 0, r2)
        assert ratio == pytest.approx(64.0, rel=1e-3)


def test_hbond_12_10_minimum_is_minus_eps_at_req(ora):
    ff = synth.forcefield(NT, hbond_pairs=[(1, 4)])
    ff.qsolpar = 0.0
    req = 0.5 * (float(ff.Rii[1]) + float(ff.Rii[4]))
    eps = math.sqrt(float(ff.epsii[1]) * float(ff.epsii[4]))
    assert ora.pair_energy(ff, 1, 4, 0, 0, req) == pytest.approx(-eps, rel=1e-12)
    assert ora.pair_energy(ff, 4, 1, 0, 0, req) == pytest.approx(-eps, rel=1e-12)
    h = 1e-5
    de = (ora.pair_energy(ff, 1, 4, 0, 0, req + h) - ora.pair_energy(ff, 1, 4, 0, 0, req - h)) / (2 * h)
    assert abs(de) < 1e-8
    # attractive tail of the hydrogen-bond form falls as r^-10
    ratio = ora.pair_energy(ff, 1, 4, 0, 0, 30 * req) / ora.pair_energy(ff, 1, 4, 0, 0, 60 * req)
    assert ratio == pytest.approx(1024.0, rel=1e-3)


def test_repulsion_capped(ora):
    ff = _ff(qsolpar=0.0)
    assert ora.pair_energy(ff, 0, 0, 0, 0, 0.5) == pytest.approx(ff.e_cap, abs=1e-12)
    assert ora.pair_energy(ff, 0, 0, 0, 0, 0.0) == pytest.approx(ff.e_cap, abs=1e-12)


def test_coulomb_limit_and_dielectric_shape(ora):
    """With van der Waals and desolvation switched off the pair energy is
    C q_i q_j / (eps(r) r): eps tends to eps0 far away, is A + B/(1+k) at contact,
    and grows monotonically."""
    ff = _ff(epsii=np.zeros(NT, np.float32), qsolpar=0.0, r_min=1e-12)
    qi, qj = 0.3, -0.45
    C = ff.coulomb

    def eps_of(r):
        return C * qi * qj / (ora.pair_energy(ff, 0, 1, qi, qj, r) * r)

    assert eps_of(1e5) == pytest.approx(ff.diel_eps0, rel=1e-9)
    B = ff.diel_eps0 - ff.diel_A
    assert eps_of(1e-9) == pytest.approx(ff.diel_A + B / (1 + ff.diel_k), rel=1e-6)
    rs = np.linspace(0.5, 40, 80)
    e = np.array([eps_of(r) for r in rs])
    assert np.all(np.diff(e) > 0)
    # bilinear in the charges, antisymmetric in the sign of one charge
    r = 4.2
    assert ora.pair_energy(ff, 0, 1, 2 * qi, qj, r) == pytest.approx(2 * ora.pair_energy(ff, 0, 1, qi, qj, r))
    assert ora.pair_energy(ff, 0, 1, -qi, qj, r) == pytest.approx(-ora.pair_energy(ff, 0, 1, qi, qj, r))


def test_desolvation_gaussian(ora):
    ff = _ff(epsii=np.zeros(NT, np.float32), solpar=np.full(NT, 0.002, np.float32), qsolpar=0.0,
             r_min=1e-12)
    s = ff.sigma
    e0 = ora.pair_energy(ff, 2, 3, 0, 0, 1e-9)
    assert e0 == pytest.approx(float(np.float32(0.002)) * (float(ff.vol[2]) + float(ff.vol[3])), rel=1e-9)
    assert ora.pair_energy(ff, 2, 3, 0, 0, s) / e0 == pytest.approx(math.exp(-0.5), rel=1e-9)
    assert ora.pair_energy(ff, 2, 3, 0, 0, 2 * s) / e0 == pytest.approx(math.exp(-2.0), rel=1e-9)


def test_pair_energy_symmetric(ora):
    ff = synth.forcefield(NT, solpar=-0.0007, hbond_pairs=[(0, 3)])
    rng = np.random.default_rng(0)
    for _ in range(50):
        ti, tj = rng.integers(0, NT, 2)
        qi, qj = rng.uniform(-0.5, 0.5, 2)
        r = rng.uniform(0.05, 12)
        assert ora.pair_energy(ff, ti, tj, qi, qj, r) == pytest.approx(ora.pair_energy(ff, tj, ti, qj, qi, r), rel=1e-14, abs=1e-15)


def _independent_pairs(lig):
    """Pair rule re-derived with Python sets: i<j, graph distance >= 4, and not
    joined by a path of non-rotatable bonds."""
    n = lig.n_atoms
    nbr = {i: set() for i in range(n)}
    rigid = {i: set() for i in range(n)}
    rot = {int(b) for b in lig.torsion_bonds}
    for k, (a, b) in enumerate(lig.bonds):
        nbr[int(a)].add(int(b))
        nbr[int(b)].add(int(a))
        if k not in rot:
            rigid[int(a)].add(int(b))
            rigid[int(b)].add(int(a))

    def reach(start, adj, limit=None):
        d = {start: 0}
        frontier = [start]
        while frontier:
            nxt = []
            for u in frontier:
                for v in adj[u]:
                    if v not in d:
                        d[v] = d[u] + 1
                        nxt.append(v)
            frontier = nxt
        return d

    out = set()
    for i in range(n):
        dist = reach(i, nbr)
        same = reach(i, rigid)
        for j in range(i + 1, n):
            if dist[j] >= 4 and j not in same:
                out.add((i, j))
    return out


@pytest.mark.parametrize("lig_id,n,nt", [(0, 24, 6), (1, 40, 10), (2, 60, 15), (3, 12, 0), (4, 96, 20)])
def test_pair_list_matches_independent_enumeration(ora, lig_id, n, nt):
    lig = synth.make_ligand(1, lig_id, n, nt, NT)
    pairs, _, _, _ = ora.ligand_info(lig, NT)
    got = {(int(a), int(b)) for a, b in pairs}
    assert got == _independent_pairs(lig)
    assert len(got) == len(pairs)


def test_intra_invariant_under_rigid_moves(ora):
    lig = synth.make_ligand(1, 1, 40, 10, NT)
    ff = synth.forcefield(NT, solpar=-0.0005)
    rng = np.random.default_rng(2)
    g = np.zeros((6, 17), np.float32)
    g[:, 7:] = rng.uniform(-np.pi, np.pi, 10)
    g[:, 3] = 1
    g[1:, 0:3] = rng.uniform(-5, 5, (5, 3))
    g[1:, 3:7] = rng.normal(size=(5, 4))
    grid = synth.make_grid(8, NT)
    maps = np.zeros((NT + 2, 8, 8, 8), np.float32)
    _, _, intra = ora.score_poses(grid, maps, ff, [lig], g, parts=True)
    np.testing.assert_allclose(intra, intra[0], rtol=1e-12)


def test_relabelling_atoms_keeps_energy(ora):
    """Renumbering atoms (root kept at index 0) builds the same molecule and the same
    pose, so every energy term is unchanged."""
    NTY = 8
    lig = synth.make_ligand(1, 5, 30, 8, NTY)
    ff = synth.forcefield(NTY, solpar=-0.0005)
    rec = synth.make_receptor(2, 300, NTY)
    grid = synth.make_grid(24, NTY, spacing=0.5)
    maps = ora.build_maps(ff, rec, grid)
    rng = np.random.default_rng(3)
    perm = np.concatenate([[0], 1 + rng.permutation(lig.n_atoms - 1)])   # new index -> old index
    inv = np.argsort(perm)                                                # old index -> new index
    lig2 = synth.Ligand(lig.xyz[perm], lig.type[perm], lig.charge[perm], inv[lig.bonds].astype(np.int32),
                        lig.torsion_bonds)
    lo, hi = synth.pocket_box(grid, half=2.0)
    g = synth.sample_genotypes(4, 20, lig.n_torsions, 15, lo, hi)
    e1, i1, a1 = ora.score_poses(grid, maps, ff, [lig], g, parts=True)
    e2, i2, a2 = ora.score_poses(grid, maps, ff, [lig2], g, parts=True)
    np.testing.assert_allclose(e2, e1, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(a2, a1, rtol=1e-11, atol=1e-11)


def test_other_root_changes_pose_by_a_rigid_motion(ora):
    """Choosing another root makes each torsion move the other side of its bond; the
    conformation differs only by a rigid motion, so the intra energy is unchanged."""
    lig = synth.make_ligand(1, 6, 30, 8, NT)
    ff = synth.forcefield(NT)
    n = lig.n_atoms
    r = n - 1
    perm = np.arange(n)
    perm[0], perm[r] = r, 0
    inv = np.argsort(perm)
    lig2 = synth.Ligand(lig.xyz[perm], lig.type[perm], lig.charge[perm], inv[lig.bonds].astype(np.int32),
                        lig.torsion_bonds)
    rng = np.random.default_rng(5)
    for _ in range(4):
        g = np.zeros(15, np.float32)
        g[3] = 1
        g[7:] = rng.uniform(-np.pi, np.pi, 8)
        X1 = ora.pose(lig, NT, g)
        X2 = ora.pose(lig2, NT, g)[inv]
        assert ora.intra_xyz(lig, ff, X1) == pytest.approx(ora.intra_xyz(lig, ff, X2), rel=1e-11, abs=1e-11)


def test_nonfinite_gene_gives_nan(ora):
    lig = synth.make_ligand(1, 0, 24, 6, NT)
    grid = synth.make_grid(8, NT)
    maps = np.zeros((NT + 2, 8, 8, 8), np.float32)
    g = np.zeros((3, 13), np.float32)
    g[:, 3] = 1
    g[1, 9] = np.nan
    g[2, 0] = np.inf
    e = ora.score_poses(grid, maps, synth.forcefield(NT), [lig], g)
    assert np.isfinite(e[0]) and np.isnan(e[1]) and np.isnan(e[2])
