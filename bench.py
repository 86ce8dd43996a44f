"""Benchmark of the docking hot path on one MI355X.

Workload (one step): score 10^7 random poses of one 40-atom, 10-torsion ligand
(12 atom types) against 14 float32 grid maps of 100^3 nodes (56 MB) -- pose
build (Algorithm 1) + inter and intra energy (Algorithm 2) for every pose.
Genotypes (680 MB) and maps are resident in HBM before timing starts.

Prints one JSON line: throughput in poses/s, the scoring kernel against its
roofline (kernel time from HIP events on the launch stream), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
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
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic work per pose, see the design doc (measurement section)
BYTES_PER_ATOM = 96            # 3 maps x 8 corners x 4 B gathered per atom
FLOPS_PER_PAIR = 38            # one 12-6 pair term (FMA = 2, transcendental = 1)


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


def kernel_source_hash() -> str:
    """Hash of the scoring kernel's sources; HBM traffic figures recorded under
    profiles/ are used only while it matches."""
    h = hashlib.sha256()
    for f in ("score.hip", "score_pose.h", "dock_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_12232_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(n_poses: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel has
    changed since it was taken or the workload differs."""
    path = os.path.join(ROOT, "profiles", "score_kernel_config1_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_source_hash() or int(kv.get("poses", "0")) != n_poses:
        return None
    return float(kv["traffic_bytes"])


def probes(S, kernel_ms: float, n_poses: int):
    """Measured ceilings at the same spatial distribution: map lookups alone
    (gather probe: random rigid placements of the ligand's atoms with
    translations in the pocket box) and pair terms alone (pair probe)."""
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

    lanes, per = 1 << 21, 128
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    g_ms = timeit(lambda: dk.dock_gather_probe(S["pocket"], S["ligs"], 0, blo, bhi, out, per))
    probe_lps = lanes * per / (g_ms * 1e-3)
    lanes, per = 1 << 20, 1024
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    p_ms = timeit(lambda: dk.dock_pair_probe(S["pocket"], out, per))
    probe_pps = lanes * per / (p_ms * 1e-3)
    kernel_lps = lig.n_atoms * n_poses / (kernel_ms * 1e-3)
    kernel_pps = S["n_pairs"] * n_poses / (kernel_ms * 1e-3)
    return {
        "gather": {"unit": "lookups/s", "kernel": round(kernel_lps, -6), "probe": round(probe_lps, -6),
                   "frac": round(kernel_lps / probe_lps, 4),
                   "probe_kind": "rigid random placements of the ligand's atoms, translations in the pocket box"},
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
        oracle.score_poses(S["grid"], maps, S["ff"], [S["lig"]], g, n_threads=threads)
        t = time.perf_counter() - t0
        if t >= target_seconds or n >= max_poses:
            break
        n = min(max_poses, int(n * max(2.0, 1.2 * target_seconds / max(t, 1e-3))))
    return {"value": n / t, "unit": "poses/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the 1e7 genotypes, scored in {t:.1f} s (FP64, {threads} threads)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--poses", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3 counter runs: one 1 GiB device copy (calibration of the "
                         "FETCH_SIZE/WRITE_SIZE counters) and two scoring steps, nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the workload shards by pose range "
              "across GPUs with no communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench needs a HIP device"
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
        torch.cuda.synchronize()
        log("profile run: 1 GiB copy, 2 scoring steps")
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
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    n = args.poses
    value = n / (wall / args.steps)
    e = S["e"].cpu().numpy()
    log(f"energies: finite {np.isfinite(e).mean():.4f}, median {np.median(e):.3f}, min {e.min():.3f}")

    n_atoms = S["lig"].n_atoms
    bytes_per_launch = BYTES_PER_ATOM * n_atoms * n
    gather_gbs = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    flops_per_launch = FLOPS_PER_PAIR * S["n_pairs"] * n
    tflops = flops_per_launch / (kernel_ms * 1e-3) / 1e12
    traffic = recorded_traffic(n)
    roofline = {"bound": "hbm", "achieved": round(gather_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gather_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "score_kernel", "kernel_ms": round(kernel_ms, 4), "layout": S["pocket"].layout,
                "alu": {"achieved": round(tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4)},
                "measured": probes(S, kernel_ms, n)}
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
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(S, args.cpu_seconds, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
