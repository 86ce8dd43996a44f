"""Host checks of the seeded input generator: the ligand sets of the learned
proposal comparison (evaluation batch, training set, schedule-validation batch)
are disjoint and follow their size law, and generation does not depend on the
number of worker processes."""
import numpy as np

import synth


def _ids(cfg):
    c = synth.CONFIGS[cfg]
    first = c.get("first_id", 0)
    return set(range(first, first + c["n_ligands"]))


def test_learned_proposal_sets_are_disjoint():
    ev, tr, val = _ids(3), _ids(4), _ids(5)
    assert not (ev & tr) and not (ev & val) and not (tr & val)
    # the same size law, the same pocket recipe
    for cfg in (4, 5):
        for key in ("n_types", "grid_n", "atoms", "torsions", "pop", "gens"):
            assert synth.CONFIGS[cfg][key] == synth.CONFIGS[3][key], (cfg, key)


def test_size_law_of_the_uneven_batches():
    for cfg in (3, 4, 5):
        atoms, tors = synth.config_ligand_sizes(cfg)
        assert len(atoms) == synth.CONFIGS[cfg]["n_ligands"]
        assert atoms.min() >= 8 and atoms.max() <= 96
        assert tors.min() >= 0 and tors.max() <= 20
        # lognormal with median 32 (clipped): the sample median sits near 32
        assert 28 <= np.median(atoms) <= 36


def test_ligands_differ_across_sets_and_match_across_workers():
    a = synth.config_ligands(5, count=70, workers=1)
    b = synth.config_ligands(5, count=70, workers=2)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.xyz, y.xyz)
        np.testing.assert_array_equal(x.type, y.type)
        np.testing.assert_array_equal(x.charge, y.charge)
    ev = synth.config_ligands(3, count=3)
    tr = synth.config_ligands(4, count=3)
    for p, q, r in zip(ev, tr, a[:3]):
        assert not np.array_equal(p.charge[:8], q.charge[:8])
        assert not np.array_equal(p.charge[:8], r.charge[:8])
        assert not np.array_equal(q.charge[:8], r.charge[:8])
