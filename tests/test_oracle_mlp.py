"""Pins of the FP64 reference of the learned proposal (oracle/mlp.py).

The proposal network is this project's addition (the paper's search has no
learned component), so every pin here is mathematical: a library routine
(torch's bfloat16 conversion), finite differences, closed forms and round
trips."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp

RNG = np.random.default_rng(7)


def small_params(rng, scale=0.2):
    flat = rng.standard_normal(mlp.N_PARAMS) * scale
    return mlp.unpack(flat)


def test_bf16_matches_torch_conversion():
    x = np.concatenate([RNG.standard_normal(20000) * 10 ** RNG.uniform(-6, 6, 20000),
                        np.array([1.0, -1.0, 1.00390625, 1.01171875, 3.0e-3])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: the even one is 1 + 2^-6
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)


def test_backward_matches_finite_differences():
    """Unquantised back-propagation equals central differences of the loss."""
    rng = np.random.default_rng(3)
    P = small_params(rng, 0.15)
    X = rng.standard_normal((6, mlp.N_IN))
    T = rng.standard_normal((6, mlp.N_OUT))
    w = rng.uniform(0.5, 2.0, 6)
    y, cache = mlp.forward(P, X, quantize=False)
    g = mlp.backward(P, cache, y, T, w)
    h = 1e-6
    for name, shape in mlp.SHAPES:
        idx = [tuple(rng.integers(0, s) for s in shape) for _ in range(12)]
        for ix in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][ix] += h
            Pm[name][ix] -= h
            lp = mlp.loss(mlp.forward(Pp, X, False)[0], T, w)
            lm = mlp.loss(mlp.forward(Pm, X, False)[0], T, w)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][ix]) <= 1e-6 * max(1.0, abs(fd)), (name, ix, fd, g[name][ix])


def test_forward_single_path_closed_form():
    """One active path through the network: y_j = w3 relu(w2 relu(w1 x + b1) + b2) + b3."""
    P = {k: np.zeros(s) for k, s in mlp.SHAPES}
    P["W1"][5, 7] = 2.0
    P["b1"][7] = -1.0
    P["W2"][7, 3] = 0.5
    P["b2"][3] = 0.25
    P["W3"][3, 10] = -4.0
    P["b3"][10] = 1.0
    X = np.zeros((3, mlp.N_IN))
    X[:, 5] = [3.0, 0.25, 0.75]
    y, _ = mlp.forward(P, X, quantize=True)
    for r, x in enumerate([3.0, 0.25, 0.75]):
        hid = max(2.0 * x - 1.0, 0.0)
        expect = -4.0 * max(0.5 * hid + 0.25, 0.0) + 1.0
        assert y[r, 10] == expect
        assert np.count_nonzero(np.delete(y[r], 10)) == 0


def test_quantized_forward_near_exact():
    """Rounding to bfloat16 perturbs the output by about 2^-8 relative, never more than
    a few percent of the accumulated magnitudes."""
    rng = np.random.default_rng(11)
    P = small_params(rng, 0.1)
    X = rng.standard_normal((64, mlp.N_IN))
    yq, cq = mlp.forward(P, X, True)
    ye, _ = mlp.forward(P, X, False)
    scale = np.abs(cq["a2"]) @ np.abs(cq["W"]["W3"]) + 1e-3
    assert np.all(np.abs(yq - ye) <= 0.05 * scale)
    assert np.median(np.abs(yq - ye) / scale) < 2 ** -7


def test_adam_first_step_closed_form():
    """From zero moments the first step is -lr g / (|g| + eps) (bias corrections cancel)."""
    rng = np.random.default_rng(5)
    P = small_params(rng)
    G = {k: rng.standard_normal(v.shape) for k, v in P.items()}
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    P0 = {k: x.copy() for k, x in P.items()}
    mlp.adam(P, G, m, v, 1, 1e-3)
    for k in P:
        np.testing.assert_allclose(P[k] - P0[k], -1e-3 * G[k] / (np.abs(G[k]) + 1e-8), rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(m[k], 0.1 * G[k], rtol=1e-12)
        np.testing.assert_allclose(v[k], 0.001 * G[k] ** 2, rtol=1e-12)


def test_pack_roundtrip():
    flat = np.arange(mlp.N_PARAMS, dtype=np.float64)
    assert mlp.N_PARAMS == 96 * 256 + 256 + 256 * 256 + 256 + 256 * 32 + 32
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(flat)), flat)


@pytest.mark.parametrize("n_tor", [0, 3, 20, 28])
def test_move_then_decode_round_trip(n_tor):
    """decode(a, move(a, b), alpha=1) is b: same translation, same rotation, same
    torsions modulo 2 pi (for the first 25 torsions)."""
    rng = np.random.default_rng(n_tor)
    lo, hi = (-8.0, -7.0, -6.0), (8.0, 9.0, 10.0)
    for _ in range(20):
        a = synth.sample_genotypes(int(rng.integers(1 << 30)), 1, n_tor, 7 + n_tor, lo, hi)[0].astype(np.float64)
        b = synth.sample_genotypes(int(rng.integers(1 << 30)), 1, n_tor, 7 + n_tor, lo, hi)[0].astype(np.float64)
        f = mlp.move(a, b, n_tor, lo, hi)
        g = mlp.decode(a, f, n_tor, lo, hi, 1.0)
        np.testing.assert_allclose(g[:3], b[:3], atol=1e-12)
        qg, qb = mlp.canonical_q(g[3:7]), mlp.canonical_q(b[3:7])
        np.testing.assert_allclose(qg, qb, atol=1e-12)
        k = min(n_tor, mlp.MAX_ENCODED_TORSIONS)
        d = (g[7:7 + k] - b[7:7 + k] + np.pi) % (2 * np.pi) - np.pi
        np.testing.assert_allclose(d, 0.0, atol=1e-12)
        np.testing.assert_array_equal(g[7 + k:], a[7 + k:])
        assert np.all(np.abs(f[7:]) <= 1.0) and np.all(np.abs(f[:3]) <= 2.0)


def test_encode_ranges_and_sign():
    lo, hi = (-8.0, -8.0, -8.0), (8.0, 8.0, 8.0)
    g = np.array([8.0, -8.0, 0.0, -0.5, 0.5, 0.5, 0.5, np.pi, -np.pi / 2], np.float64)
    f = mlp.encode(g, 2, lo, hi)
    np.testing.assert_allclose(f[:3], [1.0, -1.0, 0.0])
    np.testing.assert_allclose(f[3:7], [0.5, -0.5, -0.5, -0.5])
    np.testing.assert_allclose(f[7:9], [1.0, -0.5])
    assert np.all(f[9:] == 0)
    # a zero quaternion encodes as the identity, a zero-width box axis as 0
    f = mlp.encode(np.zeros(9), 2, (0.0, -1.0, -1.0), (0.0, 1.0, 1.0))
    np.testing.assert_array_equal(f[:7], [0, 0, 0, 1, 0, 0, 0])


def test_descriptor_features():
    lig = synth.make_ligand(1, 3, 30, 7, 12)
    d = mlp.descriptor(lig, 200)
    counts = np.bincount(lig.type, minlength=32)
    np.testing.assert_allclose(d[:32], counts / 30)
    assert d[:32].sum() == pytest.approx(1.0)
    assert d[32] == lig.n_torsions / 20 and d[33] == 30 / 96
    x = lig.xyz.astype(np.float64)
    rg = np.sqrt(np.mean(np.sum((x - x.mean(0)) ** 2, axis=1)))
    assert d[36] == pytest.approx(rg / 10, rel=1e-12)
    assert d[37] == 200 / 4096
    assert np.all(d[38:] == 0)


def test_rank_weights_pins():
    """Rank weights: beta = 0 is uniform; the ranks are a permutation of 0..P-1
    (recovered from beta = 1, where w = 2 (1 - r / P)); ties go by index, NaNs
    last; the mean over a ligand tends to 1 (exactly (1 + beta) times a Riemann
    sum of (1 - x)^beta)."""
    rng = np.random.default_rng(2)
    e = rng.normal(0, 5, 50)
    e[[4, 9]] = e[17]
    e[[2, 30]] = np.nan
    assert np.all(mlp.rank_weights(e, 0.0) == 1.0)
    r = np.rint((1 - mlp.rank_weights(e, 1.0).astype(np.float64) / 2) * 50).astype(int)
    assert sorted(r) == list(range(50))
    assert r[30] == 49 and r[2] == 48                      # NaNs last, by index
    assert r[4] + 1 == r[9] and r[9] + 1 == r[17]         # three equal energies: consecutive ranks, by index
    order = sorted(range(50), key=lambda i: (np.isnan(e[i]), 0.0 if np.isnan(e[i]) else e[i], i))
    assert [r[i] for i in order] == list(range(50))
    for beta in (0.5, 2.0, -0.5):
        w = mlp.rank_weights(np.arange(1000.0), beta).astype(np.float64)
        assert abs(w.mean() - 1.0) < 0.05
        assert np.all(np.diff(w) < 0) if beta > 0 else np.all(np.diff(w) > 0)
