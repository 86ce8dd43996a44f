"""Benchmark of the docking hot path on one MI355X.

Workload (one step): score 10^7 random poses of one 40-atom, 10-torsion ligand
(12 atom types) against 14 float32 grid maps of 100^3 nodes (56 MB) -- pose
build (Algorithm 1) + inter and intra energy (Algorithm 2) for every pose.
Genotypes (680 MB) and maps are resident in HBM before timing starts.

Prints one JSON line: throughput in poses/s, the scoring kernel against its
roofline (kernel time from HIP events on the launch stream), and the FP64 CPU
oracle timed on a bounded sample of the same workload.  Beside them (unless
--no-search): the persistent search's throughput on the 1000- and
10000-ligand batches, and time-to-target of the plain and the learned search
on the 10000-ligand batch, with the learned proposal trained first on plain
runs over 5000 other ligands.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "poses scored/sec (FP32, vs FP64 oracle) + time-to-target score, plain vs learned"
# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# FP32 vector FMA without packed instructions (the library is built without
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 78.6

# VALU lane-instruction issue: 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz
VALU_PEAK_T_PER_S = 256 * 64 * 2.4e9 / 1e12

# Algorithmic work per pose
BYTES_PER_ATOM = 96            # 3 maps x 8 corners x 4 B gathered per atom
FLOPS_PER_PAIR = 38            # one 12-6 pair term (FMA = 2, transcendental = 1)
# VALU lane-instructions the method needs per pose: per non-bonded pair (the
# pair term), per atom (pose build and interpolation), per torsion
VALU_PER_PAIR, VALU_PER_ATOM, VALU_PER_TORSION = 30, 60, 20


# The paper's own figures, as context (it prints no throughput or time for the
# docking path; its timing figures are not in the text).
PAPER_CONTEXT = {
    "throughput": None,
    "note": "the paper prints no poses/s or time for the docking path; its results are in figures",
    "hardware": ["GH200 Grace 72 cores 2.5 GHz", "Xeon Platinum 8470 2x52 cores 2.5 GHz",
                 "EPYC 9684X 96 cores 2.7 GHz", "A64FX FX700 48 cores 2.0 GHz", "Graviton 4 96 cores (AWS)"],
    "precision": "FP32; fast math changes scores by under 0.0002% on average (Sec. VII)",
    "run_to_run": "about 1% sigma/mean over 10 runs after 3 dropped (Sec. VIII)",
    "workload": "100 individuals x 1000 generations per ligand; ~2500 MEDIATE ligands; 1a30 replicated (Sec. VII)",
    "bound": "compute-bound on one core per its roofline analysis (Sec. VIII, Tables IV-V)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(n_poses: int, seed: int = 1):
    import torch

    from paper_2509_12232_amd import dock as dk
    c = synth.CONFIGS[1]
    nt = c["n_types"]
    ff = synth.forcefield(nt)
    rec = synth.make_receptor(seed, 2000, nt)
    grid = synth.make_grid(c["grid_n"], nt)
    lig = synth.make_ligand(seed, 0, c["atoms"], c["torsions"], nt)
    t0 = time.time()
    pocket = dk.dock_create_pocket_from_receptor(grid, ff, rec, device=0)
    log(f"maps built on GPU in {time.time() - t0:.2f} s")
    ligs = dk.dock_create_ligands(pocket, [lig])
    lo, hi = synth.pocket_box(grid)
    stride = 7 + lig.n_torsions
    t0 = time.time()
    g = synth.sample_genotypes(seed, n_poses, lig.n_torsions, stride, lo, hi)
    gt = torch.from_numpy(g).cuda()
    log(f"{n_poses} genotypes generated and uploaded in {time.time() - t0:.2f} s")
    e = torch.empty(n_poses, dtype=torch.float32, device="cuda")
    return dict(dk=dk, ff=ff, rec=rec, grid=grid, lig=lig, pocket=pocket, ligs=ligs, g=g, gt=gt, e=e,
                n_pairs=ligs.pair_count(0))


def _code_only(text: str) -> str:
    """C++ source without // comments, trailing blanks and empty lines (the
    kernel sources hold no string literal with //)."""
    lines = (line.split("//", 1)[0].rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash() -> str:
    """Hash of the scoring kernel's code (its sources less comments); HBM
    traffic figures recorded under profiles/ are used only while it matches."""
    h = hashlib.sha256()
    for f in ("score.hip", "score_pose.h", "dock_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_12232_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def read_record(name: str, n_poses: int):
    """The key = value lines of a committed counter summary under profiles/, or
    None if it is missing, was taken on other scoring-kernel code (its
    kernel_hash) or on another workload (its poses)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_source_hash() or int(kv.get("poses", "0")) != n_poses:
        return None
    return kv


def recorded_traffic(n_poses: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel has
    changed since it was taken or the workload differs."""
    kv = read_record("score_kernel_config1_traffic.txt", n_poses)
    return None if kv is None else float(kv["traffic_bytes"])


def recorded_valu(n_poses: int):
    """VALU activity of the scoring kernel from the committed rocprofv3 summary
    (VALUBusy: the share of SIMD cycles issuing vector instructions, and the
    same counter on the pair probe, a VALU-only kernel at full occupancy), or
    None as for the traffic record."""
    kv = read_record("score_kernel_config1_valu.txt", n_poses)
    if kv is None:
        return None
    return {"valu_busy": float(kv["valu_busy"]), "valu_busy_pair_probe": float(kv["valu_busy_pair_probe"]),
            "valu_share_of_probe": round(float(kv["valu_busy"]) / float(kv["valu_busy_pair_probe"]), 4),
            "valu_utilization": float(kv["valu_utilization"]),
            "valu_insts_per_pose": float(kv["valu_insts_per_pose"])}


def choose_bound(traffic_frac, valu):
    """The resource the counters say binds: HBM when the line traffic actually
    moved is the larger share of the HBM peak, VALU when the kernel's VALUBusy
    is the larger share of the pair probe's (a VALU-only kernel at full
    occupancy, taken as a saturated VALU).  None unless both records apply."""
    if traffic_frac is None or valu is None:
        return None
    return "alu" if valu["valu_busy"] / valu["valu_busy_pair_probe"] > traffic_frac else "hbm"


def roofline_record(kernel_ms: float, n: int, n_atoms: int, n_pairs: int, n_tors: int) -> dict:
    """The scoring kernel against its roofline for a launch of n poses of one
    ligand: the HBM leg (algorithmic map bytes), the ALU leg (algorithmic VALU
    lane-instructions, with the pair flops and the executed instructions beside
    them), the line traffic from the counter record, and the bound the counters
    name.  The top-level achieved / peak / frac are those of the bound's leg."""
    s = kernel_ms * 1e-3
    gather_gbs = BYTES_PER_ATOM * n_atoms * n / s / 1e9
    tflops = FLOPS_PER_PAIR * n_pairs * n / s / 1e12
    valu_per_pose = VALU_PER_PAIR * n_pairs + VALU_PER_ATOM * n_atoms + VALU_PER_TORSION * n_tors
    valu_rate = valu_per_pose * n / s / 1e12
    traffic = recorded_traffic(n)
    traffic_frac = None if traffic is None else traffic / s / 1e9 / HBM_PEAK_GBS
    valu = recorded_valu(n)
    bound = choose_bound(traffic_frac, valu)
    hbm_leg = {"achieved": round(gather_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gather_gbs / HBM_PEAK_GBS, 4)}
    alu_leg = {"achieved": round(valu_rate, 2), "peak": round(VALU_PEAK_T_PER_S, 2), "unit": "T VALU lane-instr/s",
               "frac": round(valu_rate / VALU_PEAK_T_PER_S, 4),
               "work": f"{valu_per_pose} algorithmic VALU lane-instructions per pose ({VALU_PER_PAIR} per pair, "
                       f"{VALU_PER_ATOM} per atom, {VALU_PER_TORSION} per torsion)",
               "flops": {"achieved": round(tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4)}}
    if valu is not None:
        # what the kernel issues, from the counters (64 lanes per wavefront instruction)
        ex = valu["valu_insts_per_pose"] * 64 * n / s / 1e12
        alu_leg["executed"] = {"lane_instr_per_pose": round(valu["valu_insts_per_pose"] * 64, 1),
                               "achieved": round(ex, 2), "frac": round(ex / VALU_PEAK_T_PER_S, 4)}
    return {"bound": bound or "hbm", **{k: v for k, v in (alu_leg if bound == "alu" else hbm_leg).items()
                                        if k in ("achieved", "peak", "unit", "frac")},
            "traffic": traffic,
            "bound_source": "counters (line traffic vs VALUBusy)" if bound else
                            "none: no counter record for this kernel code",
            # the measured line traffic as a rate: what the fabric actually moves
            "traffic_GBs": None if traffic is None else round(traffic / s / 1e9, 1),
            "traffic_frac": None if traffic_frac is None else round(traffic_frac, 4),
            "valu": valu, "kernel": "score_kernel", "kernel_ms": round(kernel_ms, 4),
            "hbm": hbm_leg, "alu": alu_leg}


def probes(S, kernel_ms: float, n_poses: int):
    """Measured ceilings at the same spatial distribution: map lookups alone
    (gather probe: random rigid placements of the whole ligand, translations in
    the pocket box, its atoms looked up in order) and pair terms alone (pair
    probe)."""
    import torch
    dk = S["dk"]
    lig = S["lig"]
    blo, bhi = synth.pocket_box(S["grid"])

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    # the ceiling is the fastest probe form: lookups in flight per lane x lanes
    lanes_max, per = 1 << 21, 128
    out = torch.empty(lanes_max, dtype=torch.float32, device="cuda")
    probe_lps, probe_form = 0.0, None
    for in_flight in (2, 4, 8):
        for lanes in (1 << 19, 1 << 21):
            o = out[:lanes]
            g_ms = timeit(lambda: dk.dock_gather_probe(S["pocket"], S["ligs"], 0, blo, bhi, o, per,
                                                       in_flight=in_flight))
            rate = lanes * per / (g_ms * 1e-3)
            if rate > probe_lps:
                probe_lps, probe_form = rate, {"in_flight": in_flight, "lanes": lanes}
    lanes, per = 1 << 20, 1024
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    p_ms = timeit(lambda: dk.dock_pair_probe(S["pocket"], out, per))
    probe_pps = lanes * per / (p_ms * 1e-3)
    kernel_lps = lig.n_atoms * n_poses / (kernel_ms * 1e-3)
    kernel_pps = S["n_pairs"] * n_poses / (kernel_ms * 1e-3)
    return {
        "gather": {"unit": "lookups/s", "kernel": round(kernel_lps, -6), "probe": round(probe_lps, -6),
                   "frac": round(kernel_lps / probe_lps, 4), "probe_form": probe_form,
                   "probe_kind": "rigid random placements of the whole ligand, its atoms looked up in order, "
                                 "translations in the pocket box"},
        "pairs": {"unit": "pair terms/s", "kernel": round(kernel_pps, -6), "probe": round(probe_pps, -6),
                  "frac": round(kernel_pps / probe_pps, 4)},
    }


def cpu_baseline(S, target_seconds: float, max_poses: int):
    """The FP64 oracle on the host cores, on a prefix of the same genotypes."""
    import oracle
    threads = oracle.default_threads()
    t0 = time.time()
    maps = oracle.build_maps(S["ff"], S["rec"], S["grid"], n_threads=threads)
    log(f"oracle maps built in {time.time() - t0:.1f} s on {threads} threads")
    n = 2000
    t = 0.0
    while True:
        g = S["g"][:n]
        t0 = time.perf_counter()
        e_ora = oracle.score_poses(S["grid"], maps, S["ff"], [S["lig"]], g, n_threads=threads)
        t = time.perf_counter() - t0
        if t >= target_seconds or n >= max_poses:
            break
        n = min(max_poses, int(n * max(2.0, 1.2 * target_seconds / max(t, 1e-3))))
    # the GPU's FP32 energies of the same poses (the last timed step) against the oracle's
    e_gpu = S["e"][:n].cpu().numpy().astype(np.float64)
    diff = np.abs(e_gpu - e_ora)
    rel = diff / np.maximum(np.abs(e_ora), 1e-12)
    tol = np.maximum(1e-4 * np.abs(e_ora), 1e-3)
    parity = {"poses": int(n), "mean_rel_diff": float(np.mean(rel)), "median_rel_diff": float(np.median(rel)),
              "max_abs_diff": float(diff.max()), "within_tolerance": float(np.mean(diff <= tol))}
    # one core, on a prefix sized to about a tenth of the threaded run's time
    n1 = max(200, int(n / threads / 10))
    t0 = time.perf_counter()
    oracle.score_poses(S["grid"], maps, S["ff"], [S["lig"]], S["g"][:n1], n_threads=1)
    t1 = time.perf_counter() - t0
    return {"value": n / t, "unit": "poses/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the 1e7 genotypes, scored in {t:.1f} s (FP64, {threads} threads)",
            "one_core": {"value": round(n1 / t1, 1), "unit": "poses/s", "sample": f"first {n1} genotypes, {t1:.1f} s"},
            "parity": parity,
            "host": host_info(),
            "search": cpu_search_baseline(threads)}


def host_info():
    """CPU model, logical CPUs and the current clock of the host (from /proc/cpuinfo)."""
    model, mhz = None, []
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k == "model name" and model is None:
                model = v.strip()
            elif k == "cpu MHz":
                mhz.append(float(v))
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "mean_mhz": round(float(np.mean(mhz)), 0) if mhz else None}


def cpu_search_baseline(threads: int):
    """The FP64 oracle's plain search (threads over ligands) on the single-ligand
    workload (pop 64 x 100 generations) and on the first 20 ligands of the
    1000-ligand batch (pop 128 x 200): poses scored per second."""
    import oracle
    out = {}
    for cid, count in ((0, 1), (2, 20)):
        c = synth.CONFIGS[cid]
        nt = c["n_types"]
        ff = synth.forcefield(nt)
        grid = synth.make_grid(c["grid_n"], nt)
        maps = oracle.build_maps(ff, synth.make_receptor(1, 2000, nt), grid, n_threads=threads)
        ligands = synth.config_ligands(cid, count=count)
        lo, hi = synth.pocket_box(grid)
        stride = 7 + max(lg.n_torsions for lg in ligands)
        p = oracle.SearchParams(pop_size=c["pop"], n_generations=c["gens"], seed=1, box_lo=tuple(lo),
                                box_hi=tuple(hi))
        t0 = time.perf_counter()
        r = oracle.search(grid, maps, ff, ligands, p, stride, n_threads=threads)
        dt = time.perf_counter() - t0
        n = count * c["pop"] * (c["gens"] + 1)
        out[f"{count}_ligands"] = {"poses_per_s": round(n / dt, 1), "seconds": round(dt, 2),
                                   "best_median": round(float(np.median(r["best_energy"])), 4)}
    return out


def batch_setup(cfg_id: int, extra_cfg: int | None = None):
    """Pocket (GPU-built maps) and ligand set(s) of a batch workload."""
    from paper_2509_12232_amd import dock as dk
    c = synth.CONFIGS[cfg_id]
    nt = c["n_types"]
    ff = synth.forcefield(nt)
    rec = synth.make_receptor(1, 2000, nt)
    grid = synth.make_grid(c["grid_n"], nt)
    pocket = dk.dock_create_pocket_from_receptor(grid, ff, rec, device=0)
    ligands = synth.config_ligands(cfg_id, workers=16)
    sets = [ligands] + ([synth.config_ligands(extra_cfg, workers=16)] if extra_cfg is not None else [])
    handles = [dk.dock_create_ligands(pocket, s) for s in sets]
    stride = 7 + max(lg.n_torsions for s in sets for lg in s)
    lo, hi = synth.pocket_box(grid)
    return dict(dk=dk, pocket=pocket, sets=sets, handles=handles, stride=stride, lo=tuple(lo), hi=tuple(hi), c=c)


def search_throughput(B, gens: int, pop: int):
    """One plain search over the whole batch (fresh population, `gens`
    generations) after the launch-shape autotuner and one untimed search of the
    same length (scratch pool sized, clocks up after the host-side legs): poses
    scored per second of wall time (pop x (gens + 1) poses per ligand)."""
    import torch
    from paper_2509_12232_amd import proposal as pr
    dk = B["dk"]
    L = B["handles"][0]
    buf = pr._buffers(L.n, pop, B["stride"])
    p = dk.SearchParams(pop_size=pop, n_generations=2, seed=1, box_lo=B["lo"], box_hi=B["hi"])
    t0 = time.perf_counter()
    dk.dock_search_autotune(B["pocket"], L, p, B["stride"], tune_generations=3)
    tune_s = time.perf_counter() - t0
    p = dk.SearchParams(pop_size=pop, n_generations=gens, seed=1, box_lo=B["lo"], box_hi=B["hi"])
    dk.dock_search(B["pocket"], L, p, buf["pop"], buf["pe"], buf["bg"], buf["be"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dk.dock_search(B["pocket"], L, p, buf["pop"], buf["pe"], buf["bg"], buf["be"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = L.n * pop * (gens + 1)
    # the same search captured once into a HIP graph and launched as one graph
    plan = dk.dock_search_plan_create(B["pocket"], L, p, buf["pop"], buf["pe"], buf["bg"], buf["be"])
    dk.dock_search_plan_launch(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dk.dock_search_plan_launch(plan)
    torch.cuda.synchronize()
    graph_dt = time.perf_counter() - t0
    del plan
    shapes = {f"<={b}": {"split": ws, "blocks": nb} for b, ws, nb in dk.dock_search_shapes(L)}
    return {"ligands": L.n, "pop": pop, "generations": gens, "seconds": round(dt, 4),
            "graph_seconds": round(graph_dt, 4), "graph_poses_per_s": round(n / graph_dt, 1),
            "poses_per_s": round(n / dt, 1), "best_median": round(float(buf["be"].median()), 4),
            "autotune_s": round(tune_s, 2), "shapes": shapes, "roofline": search_roofline(B, n / dt, pop, gens)}


def search_roofline(B, poses_per_s: float, pop: int, gens: int):
    """The search's map lookups and pair terms per second (every scored pose does
    all of its ligand's), against the two probes measured on the same pocket:
    the gather probe with a ligand of the batch's median size, and the pair
    probe.  The two fractions are shares of the time each ceiling alone would
    need; what they leave is DE work, synchronisation and idle lanes."""
    import torch
    dk = B["dk"]
    L = B["handles"][0]
    ligands = B["sets"][0]
    atoms = np.array([lg.n_atoms for lg in ligands], dtype=np.float64)
    pairs = np.array([L.pair_count(i) for i in range(L.n)], dtype=np.float64)
    per_pose = pop * (gens + 1)
    secs = L.n * per_pose / poses_per_s
    lookups_s = atoms.sum() * per_pose / secs
    pairs_s = pairs.sum() * per_pose / secs
    med = int(np.argsort(atoms)[len(atoms) // 2])
    timeit = _event_timer()
    lanes_max, per = 1 << 21, 128
    out = torch.empty(lanes_max, dtype=torch.float32, device="cuda")
    probe = 0.0
    for in_flight in (2, 4, 8):
        for lanes in (1 << 19, 1 << 21):
            o = out[:lanes]
            ms = timeit(lambda: dk.dock_gather_probe(B["pocket"], L, med, B["lo"], B["hi"], o, per,
                                                     in_flight=in_flight))
            probe = max(probe, lanes * per / (ms * 1e-3))
    lanes, per = 1 << 20, 1024
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    pair_probe = lanes * per / (timeit(lambda: dk.dock_pair_probe(B["pocket"], out, per)) * 1e-3)
    return {"lookups_per_s": round(lookups_s, -6), "gather_probe": round(probe, -6),
            "gather_frac": round(lookups_s / probe, 4), "pair_terms_per_s": round(pairs_s, -6),
            "pair_probe": round(pair_probe, -6), "pair_frac": round(pairs_s / pair_probe, 4),
            "probe_ligand_atoms": int(atoms[med])}


def _event_timer(reps: int = 5):
    """Median of `reps` timed calls (HIP events on the current stream), after one untimed call."""
    import torch

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))
    return timeit


def learned_vs_plain():
    """Time-to-target on the 10000-ligand batch, plain DE vs the learned proposal.

    The network is trained (on the GPU, by the library's kernels) on plain runs
    over 5000 other ligands.  A control runs the same proposal rounds from the
    untrained network (its seeded initial weights), so that what training
    itself buys is measured apart from what the extra exactly scored proposals
    buy.  Batch level: GPU time until the median best energy
    over the batch reaches the plain search's final median + 0.1 kcal/mol.
    Ligand level: the fraction of ligands whose best reaches the plain (seed 1)
    final best + 0.1, and the generations it took; a plain run with another
    seed is the baseline for that fraction (the seed-1 plain run reaches every
    target by construction)."""
    import torch
    from paper_2509_12232_amd import proposal as pr
    B = batch_setup(3, extra_cfg=4)
    dk = B["dk"]
    c4 = synth.CONFIGS[4]
    L_ev, L_tr = B["handles"]
    stride = B["stride"]
    P = dk.SearchParams(pop_size=c4["pop"], n_generations=c4["gens"], seed=1, box_lo=B["lo"], box_hi=B["hi"])
    for L in (L_ev, L_tr):
        dk.dock_search_autotune(B["pocket"], L, P, stride, tune_generations=3)
    # plain, seed 1: the reference bests and the plain batch-level curve
    plain_pts, buf = pr.anytime(B["pocket"], L_ev, P, stride)
    ref_best = buf["be"].cpu().numpy()
    level = float(np.median(ref_best)) + 0.1
    target = buf["be"] + 0.1
    # training data and training
    t0 = time.perf_counter()
    snaps, fin = pr.plain_snapshots(B["pocket"], L_tr, P, stride, pr.SNAPSHOT_GENERATIONS)
    x, t, _ = pr.make_tuples(L_tr, P, snaps, final_best=fin["bg"])
    del snaps
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    cfg = pr.TrainConfig(n_tuples=c4["tuples"])
    net, losses = pr.train(x, t, cfg)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    n_tuples_avail = int(x.shape[0])
    del x, t
    prop = pr.ProposalConfig()
    learned_pts, lbuf = pr.anytime(B["pocket"], L_ev, P, stride, net, prop, reference_best=ref_best)
    # the control: the same proposal rounds from the same network before training
    # (its initial weights, seeded as the trained one's were)
    net0 = dk.dock_mlp_create(0, cfg.seed)
    untrained_pts, _ = pr.anytime(B["pocket"], L_ev, P, stride, net0, prop, reference_best=ref_best)
    from dataclasses import replace
    plain2_pts, buf2 = pr.anytime(B["pocket"], L_ev, replace(P, seed=2), stride, reference_best=ref_best)
    # the same comparison with seed 2 on both sides (its own plain level)
    level2 = float(np.median(buf2["be"].cpu().numpy())) + 0.1
    learned2_pts, _ = pr.anytime(B["pocket"], L_ev, replace(P, seed=2), stride, net, prop, reference_best=ref_best)
    untrained2_pts, _ = pr.anytime(B["pocket"], L_ev, replace(P, seed=2), stride, net0, prop,
                                   reference_best=ref_best)
    # ligand level, with every ligand stopping at its target
    stops = {"plain_seed1": pr.time_to_target(B["pocket"], L_ev, P, stride, target),
             "plain_seed2": pr.time_to_target(B["pocket"], L_ev, replace(P, seed=2), stride, target),
             "learned_seed1": pr.time_to_target(B["pocket"], L_ev, P, stride, target, net, prop),
             "untrained_seed1": pr.time_to_target(B["pocket"], L_ev, P, stride, target, net0, prop)}

    def lig_stats(r):
        g = r["gen_reached"]
        ok = g >= 0
        return {"gpu_ms": round(r["ms"], 1), "reached": round(float(ok.mean()), 4),
                "gen_median": float(np.median(g[ok])) if ok.any() else None,
                "gen_p90": float(np.percentile(g[ok], 90)) if ok.any() else None}

    tp_ms, tp_gen = pr.time_to_level(plain_pts, level)
    tl_ms, tl_gen = pr.time_to_level(learned_pts, level)
    t2_ms, t2_gen = pr.time_to_level(plain2_pts, level)
    s2_plain, _ = pr.time_to_level(plain2_pts, level2)
    s2_learned, s2_gen = pr.time_to_level(learned2_pts, level2)
    tu_ms, tu_gen = pr.time_to_level(untrained_pts, level)
    s2_untrained, _ = pr.time_to_level(untrained2_pts, level2)
    rnd = (lambda v: None if v is None else round(v, 1))
    ratio = (lambda a, b: round(a / b, 3) if a and b else None)
    return {
        "workload": f"{L_ev.n} ligands (atoms lognormal median 32, 8-96; 0-20 torsions), 14 fp32 maps at 80^3, "
                    f"DE pop {P.pop_size} x {P.n_generations} generations",
        "level": round(level, 4),
        "batch_time_to_level_ms": {"plain_seed1": rnd(tp_ms), "plain_seed2": rnd(t2_ms), "learned_seed1": rnd(tl_ms),
                                   "untrained_seed1": rnd(tu_ms)},
        "batch_generations_to_level": {"plain_seed1": rnd(tp_gen), "plain_seed2": rnd(t2_gen),
                                       "learned_seed1": rnd(tl_gen), "untrained_seed1": rnd(tu_gen)},
        "speedup_vs_plain_seed1": ratio(tp_ms, tl_ms),
        # what training buys: the same rounds from the untrained network against the trained one
        "speedup_trained_vs_untrained": {"seed1": ratio(tu_ms, tl_ms), "seed2": ratio(s2_untrained, s2_learned)},
        "seed2": {"level": round(level2, 4), "plain_ms": rnd(s2_plain), "learned_ms": rnd(s2_learned),
                  "untrained_ms": rnd(s2_untrained), "learned_generations": rnd(s2_gen),
                  "speedup": ratio(s2_plain, s2_learned)},
        "median_best_at_end": {"plain_seed1": round(plain_pts[-1][2], 4), "plain_seed2": round(plain2_pts[-1][2], 4),
                               "learned_seed1": round(learned_pts[-1][2], 4),
                               "untrained_seed1": round(untrained_pts[-1][2], 4)},
        "gpu_ms_at_end": {"plain_seed1": round(plain_pts[-1][1], 1), "plain_seed2": round(plain2_pts[-1][1], 1),
                          "learned_seed1": round(learned_pts[-1][1], 1),
                          "untrained_seed1": round(untrained_pts[-1][1], 1)},
        "ligand_targets": {k: lig_stats(v) for k, v in stops.items()},
        "proposal": {"step": prop.step, "every": prop.every, "until": prop.until},
        "training": {"ligands": L_tr.n, "tuples_available": n_tuples_avail, "tuples": cfg.n_tuples,
                     "steps": int(len(losses)), "batch": cfg.batch, "lr": cfg.lr,
                     "loss_first": round(float(losses[:10].mean()), 4), "loss_last": round(float(losses[-50:].mean()), 4),
                     "data_s": round(data_s, 2), "train_s": round(train_s, 2)},
    }


def schedule_sweep(seeds=(1, 2)):
    """Chooses the learned proposal's round schedule on the validation batch
    (2000 ligands disjoint from the training set and from the batch the
    comparison is reported on): the network is trained as in learned_vs_plain,
    then every schedule of a grid is run from a fresh population and timed to
    the plain search's final median + 0.1 kcal/mol on the same seed.  Prints one
    JSON line per (schedule, seed) and the ranking by mean speedup."""
    import torch
    from dataclasses import replace
    from paper_2509_12232_amd import proposal as pr
    B = batch_setup(5, extra_cfg=4)
    dk = B["dk"]
    L_val, L_tr = B["handles"]
    stride = B["stride"]
    c4 = synth.CONFIGS[4]
    P = dk.SearchParams(pop_size=c4["pop"], n_generations=c4["gens"], seed=1, box_lo=B["lo"], box_hi=B["hi"])
    for L in (L_val, L_tr):
        dk.dock_search_autotune(B["pocket"], L, P, stride, tune_generations=3)
    snaps, fin = pr.plain_snapshots(B["pocket"], L_tr, P, stride, pr.SNAPSHOT_GENERATIONS)
    x, t, _ = pr.make_tuples(L_tr, P, snaps, final_best=fin["bg"])
    del snaps
    net, _ = pr.train(x, t, pr.TrainConfig(n_tuples=c4["tuples"]))
    del x, t
    torch.cuda.synchronize()
    grid = [(a, e, u) for a in (0.5, 1.0, 1.5) for e in (3, 5, 8, 12) for u in (50, 100, 150, 300)]
    speed = {k: [] for k in grid}
    for seed in seeds:
        Ps = replace(P, seed=seed)
        pts, buf = pr.anytime(B["pocket"], L_val, Ps, stride)
        level = float(np.median(buf["be"].cpu().numpy())) + 0.1
        t_plain, _ = pr.time_to_level(pts, level)
        for a, e, u in grid:
            lp, _ = pr.anytime(B["pocket"], L_val, Ps, stride, net, pr.ProposalConfig(a, e, u))
            t_l, g_l = pr.time_to_level(lp, level)
            sp = t_plain / t_l if t_l else 0.0
            speed[(a, e, u)].append(sp)
            print(json.dumps({"seed": seed, "alpha_max": a, "every": e, "until": u,
                              "ms": None if t_l is None else round(t_l, 1), "plain_ms": round(t_plain, 1),
                              "speedup": round(sp, 3)}), flush=True)
    rank = sorted(speed.items(), key=lambda kv: -float(np.mean(kv[1])))
    print(json.dumps({"ranking": [{"alpha_max": a, "every": e, "until": u, "mean_speedup": round(float(np.mean(v)), 3)}
                                  for (a, e, u), v in rank[:10]]}), flush=True)


def weight_sweep(betas=(0.0, 1.0, 3.0, -0.5), seeds=(1, 2, 3, 4)):
    """Chooses the training tuples' energy weighting on the validation batch:
    tuples weighted by their individual's energy rank at the snapshot,
    (1 + beta)(1 - rank / pop)^beta (beta = 0: uniform).  For each beta a network
    is trained as in learned_vs_plain on the same tuples, then the learned search
    with the default schedule runs from a fresh population on the validation
    batch and is timed to the plain search's final median + 0.1 kcal/mol on the
    same seed; an untrained network on the same schedule is the control.  Prints
    one JSON line per (beta, seed) and the mean speedups."""
    import torch
    from dataclasses import replace
    from paper_2509_12232_amd import proposal as pr
    B = batch_setup(5, extra_cfg=4)
    dk = B["dk"]
    L_val, L_tr = B["handles"]
    stride = B["stride"]
    c4 = synth.CONFIGS[4]
    P = dk.SearchParams(pop_size=c4["pop"], n_generations=c4["gens"], seed=1, box_lo=B["lo"], box_hi=B["hi"])
    for L in (L_val, L_tr):
        dk.dock_search_autotune(B["pocket"], L, P, stride, tune_generations=3)
    energies = {}
    snaps, fin = pr.plain_snapshots(B["pocket"], L_tr, P, stride, pr.SNAPSHOT_GENERATIONS, energies=energies)
    cfg = pr.TrainConfig(n_tuples=c4["tuples"])
    nets = {}
    for beta in betas:
        x, t, w = pr.make_tuples(L_tr, P, snaps, final_best=fin["bg"], snap_energies=energies, beta=beta)
        nets[beta], losses = pr.train(x, t, cfg, weight=w)
        print(json.dumps({"beta": beta, "loss_first": round(float(losses[:10].mean()), 4),
                          "loss_last": round(float(losses[-50:].mean()), 4)}), flush=True)
        del x, t, w
    nets["untrained"] = dk.dock_mlp_create(0, cfg.seed)
    del snaps
    torch.cuda.synchronize()
    speed = {k: [] for k in nets}
    for seed in seeds:
        Ps = replace(P, seed=seed)
        pts, buf = pr.anytime(B["pocket"], L_val, Ps, stride)
        level = float(np.median(buf["be"].cpu().numpy())) + 0.1
        t_plain, _ = pr.time_to_level(pts, level)
        for k, net in nets.items():
            lp, _ = pr.anytime(B["pocket"], L_val, Ps, stride, net, pr.ProposalConfig())
            t_l, _ = pr.time_to_level(lp, level)
            sp = t_plain / t_l if t_l else 0.0
            speed[k].append(sp)
            print(json.dumps({"seed": seed, "beta": k, "ms": None if t_l is None else round(t_l, 1),
                              "plain_ms": round(t_plain, 1), "speedup": round(sp, 3)}), flush=True)
    print(json.dumps({"mean_speedup": {str(k): round(float(np.mean(v)), 3) for k, v in speed.items()},
                      "min_speedup": {str(k): round(float(np.min(v)), 3) for k, v in speed.items()}}), flush=True)


def profile_search(gens: int = 30):
    """Short searches over the 10000-ligand batch for counter runs: the
    autotuner, then two plain searches of `gens` generations from a fresh
    population (the second one is the one to read)."""
    import torch
    from paper_2509_12232_amd import proposal as pr
    B = batch_setup(3)
    dk = B["dk"]
    L = B["handles"][0]
    c = B["c"]
    buf = pr._buffers(L.n, c["pop"], B["stride"])
    p = dk.SearchParams(pop_size=c["pop"], n_generations=gens, seed=1, box_lo=B["lo"], box_hi=B["hi"])
    dk.dock_search_autotune(B["pocket"], L, p, B["stride"], tune_generations=3)
    shapes = {f"<={b}": (lp, w) for b, lp, w in dk.dock_search_shapes(L)}
    for k in range(2):
        t0 = time.perf_counter()
        dk.dock_search(B["pocket"], L, p, buf["pop"], buf["pe"], buf["bg"], buf["be"])
        torch.cuda.synchronize()
        log(f"search {k}: {gens} generations in {time.perf_counter() - t0:.3f} s, shapes {shapes}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)   # the paper times 10 runs after dropping 3
    ap.add_argument("--poses", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-search", action="store_true", help="skip the search and learned-proposal legs")
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3 counter runs: one 1 GiB device copy (calibration of the "
                         "FETCH_SIZE/WRITE_SIZE counters) and two scoring steps, nothing else")
    ap.add_argument("--profile-search", action="store_true",
                    help="for rocprofv3 runs of the search kernel: the 10000-ligand batch, the launch-shape "
                         "autotuner, then two plain searches of 30 generations, nothing else")
    ap.add_argument("--schedule-sweep", action="store_true",
                    help="choose the learned proposal's round schedule on the validation batch, nothing else")
    ap.add_argument("--weight-sweep", action="store_true",
                    help="choose the energy-rank weighting of the training tuples on the validation batch, "
                         "nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the scoring workload would shard by "
              "pose range and the searches by ligand, with no communication inside the timed work",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.schedule_sweep:
        schedule_sweep()
        return
    if args.weight_sweep:
        weight_sweep()
        return
    if args.profile_search:
        profile_search()
        return
    S = setup(args.poses)
    dk = S["dk"]
    stream = torch.cuda.current_stream()

    def step():
        dk.dock_score_poses(S["pocket"], S["ligs"], S["gt"], S["e"])

    if args.profile:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        step()
        step()
        # the two probes once each, as counter references
        out = torch.empty(1 << 20, dtype=torch.float32, device="cuda")
        dk.dock_pair_probe(S["pocket"], out, 1024)
        blo, bhi = synth.pocket_box(S["grid"])
        dk.dock_gather_probe(S["pocket"], S["ligs"], 0, blo, bhi, out[:1 << 19], 128, in_flight=4)
        torch.cuda.synchronize()
        log("profile run: 1 GiB copy, 2 scoring steps, pair probe, gather probe")
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    kernel_ms = float(np.mean(step_ms))
    ms_per_step = wall * 1e3 / args.steps
    n = args.poses
    value = n / (wall / args.steps)
    e = S["e"].cpu().numpy()
    log(f"energies: finite {np.isfinite(e).mean():.4f}, median {np.median(e):.3f}, min {e.min():.3f}")

    n_atoms = S["lig"].n_atoms
    measured = probes(S, kernel_ms, n)
    roofline = roofline_record(kernel_ms, n, n_atoms, S["n_pairs"], S["lig"].n_torsions)
    roofline.update({"gather_probe_frac": measured["gather"]["frac"], "layout": S["pocket"].layout,
                     "split": S["dk"].dock_score_split(S["ligs"]),
                     "kernel_ms_sd": round(float(np.std(step_ms)), 4),
                     "kernel_ms_min": round(float(np.min(step_ms)), 4), "measured": measured})
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "poses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"scoring microbench: {n} random poses of one {n_atoms}-atom "
                               f"{S['lig'].n_torsions}-torsion ligand, {S['grid'].n_maps} fp32 maps at "
                               f"{S['grid'].dims[0]}^3, {S['n_pairs']} intra pairs",
                   "poses_per_step": n},
        "roofline": roofline,
    }
    out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(S, args.cpu_seconds, n)
    if not args.no_search:
        del S
        torch.cuda.empty_cache()
        searches = {}
        for cid in (2, 3):
            c = synth.CONFIGS[cid]
            log(f"search throughput on the {c['n_ligands']}-ligand batch")
            searches[f"{c['n_ligands']}_ligands"] = search_throughput(batch_setup(cid), c["gens"], c["pop"])
        out["search"] = searches
        log("learned proposal vs plain DE")
        out["time_to_target"] = learned_vs_plain()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
