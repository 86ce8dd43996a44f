"""Plain FP64 reference of the learned proposal (numpy).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py`` may import this module; the product path never does and
shares no code with it.

The learned proposal is an addition to the method, not a part of the paper:
the paper's search is the plain evolutionary loop of Sec. V.  What it computes
is therefore this project's own definition, written out here step by step:

* a 64-feature ligand descriptor (type fractions, torsion and atom counts,
  charge statistics, radius of gyration, pair count);
* an encoding of a genotype (translation, orientation, torsions) into 32
  normalised features;
* a three-layer perceptron 96 -> 256 -> 256 -> 32 with ReLU hidden layers, whose
  matrix products take bfloat16 operands and accumulate in float32 on the GPU:
  ``forward``/``backward`` with ``quantize=True`` round to bfloat16 at exactly
  the points where the GPU does and are otherwise exact (binary64);
* a weighted squared-error loss, the Adam update (Kingma & Ba, ICLR 2015), the
  encoded move between two genotypes (the training target), the decoding of
  a network output into a proposal genotype, and per-individual training
  weights from the ranks of a population's energies.

Pins (tests/test_oracle_mlp.py): bfloat16 rounding against torch's conversion;
the unquantised backward against central finite differences of the forward;
Adam's first step against its closed form; decode(encode-move) round trips;
descriptor features against direct counts.  Parity of the descriptor's choice
of features with anything published is unpinned (no such reference exists).
"""
from __future__ import annotations

import numpy as np

N_GENES = 32          # encoded genotype features: t(3), q(4), up to 25 torsions
N_DESC = 64           # descriptor features
N_IN = N_GENES + N_DESC
N_HIDDEN = 256
N_OUT = N_GENES
MAX_TYPES = 32
MAX_ENCODED_TORSIONS = N_GENES - 7

# packed parameter order: W1 [96][256], b1 [256], W2 [256][256], b2, W3 [256][32], b3 [32]
SHAPES = (("W1", (N_IN, N_HIDDEN)), ("b1", (N_HIDDEN,)), ("W2", (N_HIDDEN, N_HIDDEN)), ("b2", (N_HIDDEN,)),
          ("W3", (N_HIDDEN, N_OUT)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape).copy()
        o += n
    return out


def pack(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even, as float64.

    x = m 2^e with 0.5 <= |m| < 1; the bfloat16 value is round(m 2^8) 2^(e-8).
    Normal range only (|x| >= 2^-126), which is all the network produces."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


# ----------------------------------------------------------------------- descriptor
def descriptor(ligand, n_pairs: int) -> np.ndarray:
    """64 features of a ligand: [0, 32) fraction of atoms of each type; 32 torsions / 20;
    33 atoms / 96; 34 mean |charge|; 35 mean charge; 36 radius of gyration / 10 A;
    37 non-bonded pair count / 4096; the rest 0."""
    n = int(ligand.n_atoms)
    d = np.zeros(N_DESC)
    for t in np.asarray(ligand.type):
        d[int(t)] += 1.0 / n
    d[32] = ligand.n_torsions / 20.0
    d[33] = n / 96.0
    q = np.asarray(ligand.charge, np.float64)
    d[34] = np.abs(q).sum() / n
    d[35] = q.sum() / n
    x = np.asarray(ligand.xyz, np.float64)
    c = x.mean(axis=0)
    d[36] = np.sqrt(((x - c) ** 2).sum() / n) / 10.0
    d[37] = n_pairs / 4096.0
    return d


# ------------------------------------------------------------------------ genotypes
def _half_box(lo, hi):
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    return (lo + hi) / 2.0, (hi - lo) / 2.0


def canonical_q(q) -> np.ndarray:
    """Unit quaternion with w >= 0 (the same rotation); identity for a zero quaternion."""
    q = np.asarray(q, np.float64)
    nn = float(q @ q)
    if nn < 1e-24:
        return np.array([1.0, 0.0, 0.0, 0.0])
    u = q / np.sqrt(nn)
    return -u if u[0] < 0 else u


def encode(genotype, n_tor: int, lo, hi) -> np.ndarray:
    """32 features: (t - centre) / half-width per axis (0 where the width is 0), the
    canonical unit quaternion, theta_k / pi for k < min(n_tor, 25), zeros."""
    g = np.asarray(genotype, np.float64)
    c, h = _half_box(lo, hi)
    f = np.zeros(N_GENES)
    for d in range(3):
        f[d] = (g[d] - c[d]) / h[d] if h[d] > 0 else 0.0
    f[3:7] = canonical_q(g[3:7])
    for k in range(min(n_tor, MAX_ENCODED_TORSIONS)):
        f[7 + k] = g[7 + k] / np.pi
    return f


def wrap(a: float) -> float:
    """Angle into (-pi, pi]."""
    a = float(np.fmod(a, 2 * np.pi))
    if a > np.pi:
        a -= 2 * np.pi
    elif a <= -np.pi:
        a += 2 * np.pi
    return a


def move(g_from, g_to, n_tor: int, lo, hi) -> np.ndarray:
    """Encoded move from one genotype to another (the training target): translation
    difference / half-width; q_to' - q_from' with both canonical and q_to' taken
    with the sign nearer q_from'; wrap(theta_to - theta_from) / pi; zeros."""
    a, b = np.asarray(g_from, np.float64), np.asarray(g_to, np.float64)
    c, h = _half_box(lo, hi)
    f = np.zeros(N_GENES)
    for d in range(3):
        f[d] = (b[d] - a[d]) / h[d] if h[d] > 0 else 0.0
    qa, qb = canonical_q(a[3:7]), canonical_q(b[3:7])
    if qa @ qb < 0:
        qb = -qb
    f[3:7] = qb - qa
    for k in range(min(n_tor, MAX_ENCODED_TORSIONS)):
        f[7 + k] = wrap(b[7 + k] - a[7 + k]) / np.pi
    return f


def decode(genotype, y, n_tor: int, lo, hi, alpha: float) -> np.ndarray:
    """Proposal genotype: t + alpha h y_t clamped to the box; canonical q + alpha y_q
    (left unnormalised, as every genotype's quaternion); wrap(theta_k + alpha pi y_k)
    for k < min(n_tor, 25), other genes unchanged."""
    g = np.asarray(genotype, np.float64).copy()
    y = np.asarray(y, np.float64)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    c, h = _half_box(lo, hi)
    for d in range(3):
        g[d] = min(max(g[d] + alpha * h[d] * y[d], lo[d]), hi[d])
    g[3:7] = canonical_q(g[3:7]) + alpha * y[3:7]
    for k in range(min(n_tor, MAX_ENCODED_TORSIONS)):
        g[7 + k] = wrap(g[7 + k] + alpha * np.pi * y[7 + k])
    return g


# -------------------------------------------------------------------------- network
def forward(params: dict, X, quantize: bool = True):
    """y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3 for every row x of X.

    With quantize, the matrix-product operands are rounded to bfloat16 (inputs,
    weights, hidden activations), everything else is exact."""
    q = bf16 if quantize else (lambda v: np.asarray(v, np.float64))
    a0 = q(X)
    W = {k: q(params[k]) for k in ("W1", "W2", "W3")}
    z1 = a0 @ W["W1"] + params["b1"]
    a1 = q(np.maximum(z1, 0.0))
    z2 = a1 @ W["W2"] + params["b2"]
    a2 = q(np.maximum(z2, 0.0))
    y = a2 @ W["W3"] + params["b3"]
    cache = dict(a0=a0, a1=a1, a2=a2, z1=z1, z2=z2, W=W, quantize=quantize)
    return y, cache


def rank_weights(energies, beta: float) -> np.ndarray:
    """Training weights of one ligand's population from its energies (one
    snapshot of the search's energy trace): individual i of rank r_i (0 = the
    lowest energy; equal energies ranked by index; a NaN after every number)
    among the P individuals gets (1 + beta) (1 - r_i / P) ** beta, computed in
    binary64 and rounded to float32.  A definition of this build: beta = 0 is
    uniform, beta > 0 favours the individuals nearer the ligand's best."""
    e = np.asarray(energies, np.float64)
    P = e.size
    nan = np.isnan(e)

    def before(j, i):
        if nan[j] != nan[i]:
            return not nan[j]           # every number before every NaN
        if not nan[i] and e[j] != e[i]:
            return e[j] < e[i]
        return j < i                    # equal energies (or two NaNs): by index

    out = np.empty(P, np.float32)
    for i in range(P):
        r = sum(1 for j in range(P) if j != i and before(j, i))
        out[i] = np.float32((1.0 + beta) * (1.0 - r / P) ** beta)
    return out


def loss(y, T, w=None) -> float:
    """(1/M) sum_m w_m sum_j (y_mj - t_mj)^2, w = 1 if absent."""
    M = y.shape[0]
    w = np.ones(M) if w is None else np.asarray(w, np.float64)
    return float((w[:, None] * (y - T) ** 2).sum() / M)


def backward(params: dict, cache: dict, y, T, w=None) -> dict:
    """Gradients of ``loss`` by back-propagation through ``forward``'s cache.

    With quantize, the back-propagated errors that enter a matrix product are
    rounded to bfloat16 first and the bias gradients sum those rounded values;
    the ReLU derivative is taken where the stored activation is > 0."""
    q = bf16 if cache["quantize"] else (lambda v: np.asarray(v, np.float64))
    M = y.shape[0]
    w = np.ones(M) if w is None else np.asarray(w, np.float64)
    W = cache["W"]
    g3 = q((2.0 / M) * w[:, None] * (y - T))
    grads = {"W3": cache["a2"].T @ g3, "b3": g3.sum(axis=0)}
    g2 = q((g3 @ W["W3"].T) * (cache["a2"] > 0))
    grads["W2"] = cache["a1"].T @ g2
    grads["b2"] = g2.sum(axis=0)
    g1 = q((g2 @ W["W2"].T) * (cache["a1"] > 0))
    grads["W1"] = cache["a0"].T @ g1
    grads["b1"] = g1.sum(axis=0)
    return grads


def adam(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1), in place on params, m and v."""
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
