"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
every entry point on small inputs (edge-case ligands included) in a
subprocess that preloads the sanitizer runtime; any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SANITIZE = ["-fsanitize=address,undefined"]   # gcc, host code only

WORKLOAD = r"""
import numpy as np, synth, oracle
ff = synth.forcefield(8, solpar=-0.001, hbond_pairs=[(0, 1)])
rec = synth.make_receptor(3, 120, 8)
grid = synth.make_grid((12, 9, 7), 8, spacing=0.9)
maps = oracle.build_maps(ff, rec, grid, n_threads=2)
one = synth.Ligand(np.array([[0.3, -0.2, 0.1]], np.float32), np.array([3], np.int32),
                   np.array([0.25], np.float32), np.zeros((0, 2), np.int32), np.zeros(0, np.int32))
ligs = [one, synth.make_ligand(1, 3, 12, 0, 8), synth.make_ligand(1, 4, 40, 10, 8), synth.make_ligand(1, 5, 96, 20, 8)]
lo = np.asarray(grid.origin) - 1.0
hi = np.asarray(grid.upper()) + 1.0
g = synth.sample_genotypes(2, 64, 20, 27, lo, hi)
pl = np.arange(64, dtype=np.int32) % 4
for p in range(64):
    g[p, 7 + ligs[pl[p]].n_torsions:] = 0
g[6, 9] = np.nan                    # a torsion gene of the 10-torsion ligand
e = oracle.score_poses(grid, maps, ff, ligs, g, pose_ligand=pl, n_threads=2)
assert np.isnan(e[6]) and np.isfinite(np.delete(e, 6)).all()
oracle.score_poses(grid, maps, ff, ligs, g[:8], pose_ligand=pl[:8], parts=True)
for lig in ligs:
    oracle.ligand_info(lig, 8)
    oracle.pose(lig, 8, g[3])
P = oracle.SearchParams(pop_size=8, n_generations=3, seed=1, box_lo=tuple(lo), box_hi=tuple(hi))
r = oracle.search(grid, maps, ff, ligs, P, 27, n_threads=2)
oracle.philox4x64([1, 2, 3, 4], [5, 6])
print("sanitized workload ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    try:
        libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                                 check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("gcc not available")
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("no AddressSanitizer runtime")
    lib = oracle.build(out=str(tmp_path / "liboracle_san.so"),
                       extra_flags=SANITIZE + ["-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"])
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=libasan, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", WORKLOAD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "sanitized workload ok" in r.stdout, r.stderr[-4000:]


def test_sanitizer_harness_reports_a_planted_overflow(tmp_path):
    """The harness above would notice a bug: a throwaway library with a heap
    read one past its allocation, built and loaded the same way, is reported."""
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "int planted(int n) { int *a = malloc(n * sizeof(int)); for (int i = 0; i < n; ++i) a[i] = i;\n"
                   "  int s = a[n]; free(a); return s; }\n")
    try:
        libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                                 check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("gcc not available")
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("no AddressSanitizer runtime")
    so = tmp_path / "libplanted.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", *SANITIZE, "-fno-omit-frame-pointer", str(src), "-o", str(so)],
                   check=True)
    code = f"import ctypes; print(ctypes.CDLL({str(so)!r}).planted(8))"
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
