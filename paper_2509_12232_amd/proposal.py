"""Training recipe of the learned proposal and the time-to-target comparison.

The learned proposal is an addition to the paper's method (its search, Sec. V,
is a plain evolutionary loop).  This module only sequences calls of the C ABI;
every computation runs in libdock's kernels, and torch tensors hold the device
buffers:

* ``plain_snapshots`` -- plain DE over a set of ligands, keeping the population
  at chosen generations and the final one;
* ``make_tuples`` -- for every individual of every snapshot, the network input
  (its genotype and its ligand's descriptor) and, as target, the encoded move
  from it to the converged pose the plain search reached for that ligand (or,
  optionally, to the same individual of the final population: the accepted
  moves of that individual from there on, composed), optionally weighted by
  the individual's energy rank at that snapshot;
* ``train`` -- Adam on minibatches of a seeded random sample of those tuples;
* ``time_to_target`` -- one search (plain or learned) in which every ligand
  stops once its population best reaches its target, timed with HIP events on
  the launching stream;
* ``anytime`` / ``time_to_level`` -- the median best energy of a batch against
  GPU time, and the time at which it first reaches a level.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import dock as dk


def _buffers(n_ligs: int, pop: int, stride: int):
    import torch
    f32 = dict(dtype=torch.float32, device="cuda")
    return dict(pop=torch.zeros((n_ligs, pop, stride), **f32), pe=torch.zeros((n_ligs, pop), **f32),
                bg=torch.zeros((n_ligs, stride), **f32), be=torch.zeros(n_ligs, **f32))


def plain_snapshots(pocket, ligs, params: dk.SearchParams, stride: int, snap_gens, energies: dict | None = None):
    """Plain search of params.n_generations generations from a fresh population.

    Returns ({g: population after g generations} for g in snap_gens below
    n_generations, buffers of the final state); with `energies` (a dict), also
    fills it with {g: the population's energies after g generations}.  The run
    is cut into resumed pieces at the snapshot generations, which gives exactly
    the uninterrupted run."""
    B = _buffers(ligs.n, params.pop_size, stride)
    snaps = {}
    marks = sorted({int(g) for g in snap_gens if 0 <= g < params.n_generations}) + [params.n_generations]
    g = 0
    for i, m in enumerate(marks):
        p = replace(params, init=1 if i == 0 else 0, first_generation=g, n_generations=m - g, proposal=None,
                    stop_at_target=0)
        dk.dock_search(pocket, ligs, p, B["pop"], B["pe"], B["bg"], B["be"])
        if m < params.n_generations:
            snaps[m] = B["pop"].clone()
            if energies is not None:
                energies[m] = B["pe"].clone()
        g = m
    return snaps, B


SNAPSHOT_GENERATIONS = (0, 5, 15, 40, 80)


def make_tuples(ligs, params: dk.SearchParams, snaps: dict, final_pop=None, final_best=None,
                snap_energies: dict | None = None, beta: float = 0.0):
    """(x [N, 96], target [N, 32], weight [N] or None) for every individual of
    every snapshot: the target is the encoded move to the ligand's converged
    pose (final_best [n_ligs][g_stride], the best member of the final
    population) or, given final_pop instead, to the same individual of the
    final population.  With beta != 0 and the snapshots' energies, each tuple
    is weighted by its individual's rank in its ligand's population at that
    snapshot (dock_mlp_rank_weights)."""
    import torch
    n = ligs.n * params.pop_size
    if final_best is not None:
        final_pop = final_best[:, None, :].expand(-1, params.pop_size, -1).contiguous()
    weighted = beta != 0.0
    if weighted and snap_energies is None:
        raise ValueError("rank weights need the snapshots' energies")
    xs, ts, ws = [], [], []
    for g in sorted(snaps):
        x = torch.empty((n, dk.DOCK_MLP_IN), dtype=torch.float32, device="cuda")
        t = torch.empty((n, dk.DOCK_MLP_OUT), dtype=torch.float32, device="cuda")
        dk.dock_mlp_features(ligs, params, snaps[g], x)
        dk.dock_mlp_moves(ligs, params, snaps[g], final_pop, t)
        xs.append(x)
        ts.append(t)
        if weighted:
            w = torch.empty(n, dtype=torch.float32, device="cuda")
            dk.dock_mlp_rank_weights(ligs, params, snap_energies[g], beta, w)
            ws.append(w)
    return torch.cat(xs), torch.cat(ts), (torch.cat(ws) if weighted else None)


@dataclass
class TrainConfig:
    n_tuples: int = 1_000_000   # size of the random sample trained on
    batch: int = 4096
    epochs: float = 8.0
    lr: float = 1e-3
    seed: int = 1


def train(x, t, cfg: TrainConfig, weight=None):
    """A new network trained on a seeded random sample of the tuples (rows
    weighted by `weight` if given); returns (network, per-step losses as a
    numpy array)."""
    import torch
    n_data = int(x.shape[0])
    n_rows = min(cfg.n_tuples, n_data) // cfg.batch * cfg.batch
    if n_rows < cfg.batch:
        raise ValueError("fewer tuples than one batch")
    rng = np.random.default_rng([cfg.seed, 0x7E41])
    order = torch.from_numpy(rng.permutation(n_data)[:n_rows].astype(np.int32)).cuda()
    steps = max(1, int(round(cfg.epochs * n_rows / cfg.batch)))
    net = dk.dock_mlp_create(0, cfg.seed)
    losses = torch.empty(steps, dtype=torch.float32, device="cuda")
    dk.dock_mlp_train(net, x, t, cfg.batch, steps, cfg.lr, weight=weight, order=order, losses=losses)
    return net, losses.cpu().numpy()


@dataclass
class ProposalConfig:
    """Round schedule of the learned proposal.  The defaults were chosen on a
    validation batch of 2000 ligands disjoint from the training set and from
    the batch the comparison is reported on (time to the plain search's final
    median + 0.1 kcal/mol, over six seeds)."""
    step: float = 1.0     # alpha_max
    every: int = 12       # learned round every this many generations (0: only after the initial population)
    until: int = 300      # no later rounds at or after this generation


def time_to_target(pocket, ligs, params: dk.SearchParams, stride: int, target, net=None,
                   prop: ProposalConfig | None = None):
    """One search from a fresh population in which each ligand stops once its
    best is <= target (a float32 device tensor, one value per ligand).  Returns
    GPU milliseconds (HIP events around the whole call on the current stream),
    the generation at which each ligand got there (-1: never) and the best
    energies."""
    import torch
    prop = prop or ProposalConfig()
    p = replace(params, init=1, first_generation=0, stop_at_target=1, proposal=net, proposal_step=prop.step,
                proposal_every=prop.every, proposal_until=prop.until)
    B = _buffers(ligs.n, params.pop_size, stride)
    gr = torch.zeros(ligs.n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    dk.dock_search(pocket, ligs, p, B["pop"], B["pe"], B["bg"], B["be"], target=target, gen_reached=gr)
    b.record()
    torch.cuda.synchronize()
    return dict(ms=a.elapsed_time(b), gen_reached=gr.cpu().numpy(), best=B["be"].cpu().numpy())


def anytime(pocket, ligs, params: dk.SearchParams, stride: int, net=None, prop: ProposalConfig | None = None,
            seg: int = 10, reference_best=None):
    """A search of params.n_generations generations from a fresh population, run
    as resumed pieces of `seg` generations (the same search as one call).  After
    each piece: (generations, cumulative GPU ms from HIP events on the current
    stream, median best energy over the ligands, fraction of ligands whose best
    is <= reference_best + 0.1 (a host array; None: nan))."""
    import torch
    prop = prop or ProposalConfig()
    B = _buffers(ligs.n, params.pop_size, stride)
    pts, cum = [], 0.0
    for g0 in range(0, params.n_generations, seg):
        n = min(seg, params.n_generations - g0)
        p = replace(params, init=int(g0 == 0), first_generation=g0, n_generations=n, proposal=net,
                    proposal_step=prop.step, proposal_every=prop.every, proposal_until=prop.until,
                    stop_at_target=0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        dk.dock_search(pocket, ligs, p, B["pop"], B["pe"], B["bg"], B["be"])
        b.record()
        torch.cuda.synchronize()
        cum += a.elapsed_time(b)
        be = B["be"].cpu().numpy()
        frac = float(np.mean(be <= reference_best + 0.1)) if reference_best is not None else float("nan")
        pts.append((g0 + n, cum, float(np.median(be)), frac))
    return pts, B


def time_to_level(pts, level: float):
    """(GPU ms, generations) at which the median best of an anytime curve first
    reaches `level`, interpolated linearly inside the piece; (None, None) if never."""
    prev = (0, 0.0, float("inf"))
    for g, ms, med, _ in pts:
        if med <= level:
            g0, ms0, m0 = prev
            f = (m0 - level) / (m0 - med) if np.isfinite(m0) and m0 > med else 1.0
            return ms0 + f * (ms - ms0), g0 + f * (g - g0)
        prev = (g, ms, med)
    return None, None
