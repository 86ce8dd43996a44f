"""Pins of the oracle's pose build (docking of one individual, Sec. V, Algorithm 1).

Each test checks the oracle against a fact fixed by geometry or by a library
routine, not against a re-typed copy of its own formula."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth

NT = 8


def _lig(n=24, nt=6, lig_id=0):
    return synth.make_ligand(1, lig_id, n, nt, NT)


def _geno(lig, t=(0, 0, 0), q=(1, 0, 0, 0), th=None, stride=None):
    stride = stride or 7 + lig.n_torsions
    g = np.zeros(stride, np.float32)
    g[0:3] = t
    g[3:7] = q
    if lig.n_torsions:
        g[7:7 + lig.n_torsions] = 0 if th is None else th
    return g


def _rand_geno(rng, lig):
    q = rng.normal(size=4)
    return _geno(lig, t=rng.uniform(-5, 5, 3), q=q, th=rng.uniform(-np.pi, np.pi, lig.n_torsions))


def test_identity_genotype_reproduces_centred_reference(ora):
    lig = _lig()
    X = ora.pose(lig, NT, _geno(lig))
    ref = lig.xyz.astype(np.float64)
    ref = ref - ref.mean(axis=0)
    np.testing.assert_allclose(X, ref, rtol=0, atol=1e-12)


def test_full_turn_torsion_gives_same_pose(ora):
    lig = _lig()
    rng = np.random.default_rng(3)
    g = _rand_geno(rng, lig)
    X0 = ora.pose(lig, NT, g)
    for k in range(lig.n_torsions):
        g2 = g.copy()
        g2[7 + k] = np.float32(g[7 + k] + 2 * np.pi)
        # the float32 gene cannot hold theta + 2 pi exactly: bound by that rounding times the lever arm
        dth = abs((float(g2[7 + k]) - 2 * np.pi) - float(g[7 + k]))
        X1 = ora.pose(lig, NT, g2)
        lever = np.linalg.norm(X0 - X0.mean(axis=0), axis=1).max() * 2
        assert np.abs(X1 - X0).max() <= dth * lever + 1e-12


def test_bond_lengths_and_angles_invariant(ora):
    lig = _lig(40, 10)
    ref = lig.xyz.astype(np.float64)
    rng = np.random.default_rng(4)
    nbr = {i: set() for i in range(lig.n_atoms)}
    for a, b in lig.bonds:
        nbr[a].add(b)
        nbr[b].add(a)
    pairs13 = {(min(a, c), max(a, c)) for b in nbr for a in nbr[b] for c in nbr[b] if a != c}
    for _ in range(5):
        X = ora.pose(lig, NT, _rand_geno(rng, lig))
        for a, b in lig.bonds:
            assert abs(np.linalg.norm(X[a] - X[b]) - np.linalg.norm(ref[a] - ref[b])) < 1e-9
        for a, c in pairs13:
            assert abs(np.linalg.norm(X[a] - X[c]) - np.linalg.norm(ref[a] - ref[c])) < 1e-9


def test_rigid_fragment_distances_invariant(ora):
    lig = _lig(40, 10)
    _, frag, _, _ = ora.ligand_info(lig, NT)
    ref = lig.xyz.astype(np.float64)
    rng = np.random.default_rng(5)
    X = ora.pose(lig, NT, _rand_geno(rng, lig))
    n = lig.n_atoms
    for i in range(n):
        for j in range(i + 1, n):
            if frag[i] == frag[j]:
                assert abs(np.linalg.norm(X[i] - X[j]) - np.linalg.norm(ref[i] - ref[j])) < 1e-9


def test_torsion_order_irrelevant(ora):
    lig = _lig(40, 10)
    rng = np.random.default_rng(6)
    g = _rand_geno(rng, lig)
    X0 = ora.pose(lig, NT, g)
    perm = rng.permutation(lig.n_torsions)
    lig2 = synth.Ligand(lig.xyz, lig.type, lig.charge, lig.bonds, lig.torsion_bonds[perm])
    g2 = g.copy()
    g2[7:] = g[7:][perm]
    X1 = ora.pose(lig2, NT, g2)
    np.testing.assert_allclose(X1, X0, rtol=0, atol=1e-10)


def _dihedral(p0, p1, p2, p3):
    """Textbook signed dihedral angle (IUPAC sign convention)."""
    b1, b2, b3 = p1 - p0, p2 - p1, p3 - p2
    return math.atan2(np.linalg.norm(b2) * np.dot(b1, np.cross(b2, b3)),
                      np.dot(np.cross(b1, b2), np.cross(b2, b3)))


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.9])
def test_chain_dihedral_changes_by_theta(ora, theta):
    xyz = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [2.0, 1.4, 0.0], [3.5, 1.5, 0.3]], np.float32)
    lig = synth.Ligand(xyz, np.zeros(4, np.int32), np.zeros(4, np.float32),
                       np.array([[0, 1], [1, 2], [2, 3]], np.int32), np.array([1], np.int32))
    X0 = ora.pose(lig, NT, _geno(lig, th=[0.0]))
    X1 = ora.pose(lig, NT, _geno(lig, th=[theta]))
    d0, d1 = _dihedral(*X0), _dihedral(*X1)
    delta = (d1 - d0 + np.pi) % (2 * np.pi) - np.pi
    assert abs(delta - np.float32(theta)) < 1e-12


def test_quaternion_sign_and_scale_invariance(ora):
    lig = _lig()
    rng = np.random.default_rng(7)
    g = _rand_geno(rng, lig)
    X0 = ora.pose(lig, NT, g)
    gneg = g.copy()
    gneg[3:7] = -g[3:7]
    np.testing.assert_allclose(ora.pose(lig, NT, gneg), X0, rtol=0, atol=1e-12)
    gs = g.copy()
    gs[3:7] = g[3:7] * np.float32(4.0)
    np.testing.assert_allclose(ora.pose(lig, NT, gs), X0, rtol=0, atol=1e-12)


def test_zero_quaternion_is_identity(ora):
    lig = _lig()
    g = _geno(lig, t=(1, 2, 3), q=(0, 0, 0, 0))
    ref = lig.xyz.astype(np.float64)
    ref = ref - ref.mean(axis=0) + np.array([1, 2, 3])
    np.testing.assert_allclose(ora.pose(lig, NT, g), ref, rtol=0, atol=1e-12)


def test_rotation_matches_scipy_axis_angle(ora):
    """Rigid part of the pose equals scipy's rotation of the centred reference plus t."""
    lig = _lig(30, 0)
    rng = np.random.default_rng(8)
    ref = lig.xyz.astype(np.float64)
    ref = ref - ref.mean(axis=0)
    for _ in range(5):
        q = rng.normal(size=4).astype(np.float32)   # (w, x, y, z)
        t = rng.uniform(-3, 3, 3).astype(np.float32)
        X = ora.pose(lig, NT, _geno(lig, t=t, q=q))
        rot = Rotation.from_quat(np.array([q[1], q[2], q[3], q[0]], np.float64))
        np.testing.assert_allclose(X, rot.apply(ref) + t.astype(np.float64), rtol=0, atol=1e-12)


def test_translation_only_shifts(ora):
    lig = _lig()
    rng = np.random.default_rng(9)
    g = _rand_geno(rng, lig)
    X0 = ora.pose(lig, NT, g)
    g2 = g.copy()
    g2[0:3] = g[0:3] + np.float32(1.0)
    np.testing.assert_allclose(ora.pose(lig, NT, g2) - X0, np.ones_like(X0) *
                               (g2[0:3].astype(np.float64) - g[0:3].astype(np.float64)), atol=1e-12)


def test_moving_sets_are_far_subtrees(ora):
    """Each torsion moves exactly the atoms on the far side of its bond from atom 0."""
    lig = _lig(40, 10)
    _, _, moving, axis = ora.ligand_info(lig, NT)
    n = lig.n_atoms
    nbr = {i: [] for i in range(n)}
    for a, b in lig.bonds:
        nbr[a].append(b)
        nbr[b].append(a)
    for k, bi in enumerate(lig.torsion_bonds):
        a, b = lig.bonds[bi]
        # atoms reachable from atom 0 without crossing bond (a, b)
        seen, stack = {0}, [0]
        while stack:
            u = stack.pop()
            for v in nbr[u]:
                if {u, v} == {int(a), int(b)} or v in seen:
                    continue
                seen.add(v)
                stack.append(v)
        expect = np.array([i not in seen for i in range(n)])
        assert (moving[k] == expect).all()
        assert axis[k][0] in seen and axis[k][1] not in seen
