"""The C-ABI library loads and exports every entry point include/dock.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dock.h")


def declared_entry_points():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dock_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_entry_points()
    for must in ("dock_create_pocket", "dock_score_poses", "dock_search", "dock_create_ligands",
                 "dock_last_error", "dock_destroy_pocket", "dock_destroy_ligands"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2509_12232_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libdock.so is not built")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_abi():
    from paper_2509_12232_amd import dock
    for n in declared_entry_points():
        if n in ("dock_last_error", "dock_destroy_pocket", "dock_destroy_ligands", "dock_ligand_pair_count",
                 "dock_pocket_layout", "dock_mlp_destroy", "dock_search_plan_destroy"):
            continue
        assert hasattr(dock, n), n


def test_host_only_calls():
    from paper_2509_12232_amd import dock
    assert dock.dock_version() == 2
    lib = dock._lib
    # a null out-pointer is rejected on the host before any device work
    st = lib.dock_create_pocket(None, None, 0, None, -1, 0, None)
    assert st == dock.DOCK_E_INVALID
    assert b"null" in lib.dock_last_error()
    assert lib.dock_destroy_pocket(None) == dock.DOCK_OK
    assert lib.dock_destroy_ligands(None) == dock.DOCK_OK


def test_search_params_layout_matches_binding(tmp_path):
    """The ctypes mirror of dock_search_params has the C struct's field offsets."""
    import subprocess
    from paper_2509_12232_amd import dock
    fields = [f for f, _ in dock._Params._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("{f} %zu\\n", offsetof(dock_search_params, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "dock.h"\nint main(void) {\n' + body +
                   '  printf("sizeof %zu\\n", sizeof(dock_search_params));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(dock._Params, f).offset, f
    assert int(out["sizeof"]) == ctypes.sizeof(dock._Params)


def test_tune_cache_file_roundtrip(tmp_path):
    """The autotuner's cache file (host-only calls): a saved file loads back to
    the same entries, and a malformed or out-of-range line loads nothing."""
    from paper_2509_12232_amd import dock
    good = tmp_path / "shapes.txt"
    rows = ["gfx950 256 3 80 80 80 12 32 32 150 2 1", "gfx950 256 3 80 80 80 12 96 96 150 4 3",
            "gfx942 304 2 64 64 64 8 48 47 128 1 3"]
    good.write_text("# a comment\n" + "\n".join(rows) + "\n")
    dock.dock_search_tune_load(good)
    out = tmp_path / "out.txt"
    dock.dock_search_tune_save(out)
    lines = out.read_text().splitlines()
    assert lines[0].startswith("#")
    assert set(rows) <= set(lines[1:])
    # the same key again replaces the entry
    (tmp_path / "upd.txt").write_text("gfx950 256 3 80 80 80 12 32 32 150 4 2\n")
    dock.dock_search_tune_load(tmp_path / "upd.txt")
    dock.dock_search_tune_save(out)
    lines = set(out.read_text().splitlines()[1:])
    assert "gfx950 256 3 80 80 80 12 32 32 150 4 2" in lines and rows[0] not in lines
    for bad in ("gfx950 256 3 80 80 80 12 32 32 150 3 1",     # split 3
                "gfx950 256 3 80 80 80 12 32 32 150 4 4",     # 16 wavefronts per workgroup
                "gfx950 256 3 80 80 80 12 32 32 150 8 2",     # 16 wavefronts per workgroup
                "gfx950 256 3 80 80 80 12 32 40 150 2 1",     # largest ligand above the bucket
                "gfx950 256 7 80 80 80 12 32 32 150 2 1",     # unknown layout
                "gfx950 256 3 80 80 80 12 32 32 150 2",       # a field missing
                "gfx950 256 3 80 80 80 12 32 32 150 2 1 9"):  # a field too many
        f = tmp_path / "bad.txt"
        f.write_text("gfx950 256 3 80 80 80 12 96 96 151 4 3\n" + bad + "\n")   # a new key, then the bad line
        before = out.read_text()
        with pytest.raises(dock.DockError):
            dock.dock_search_tune_load(f)
        dock.dock_search_tune_save(out)
        assert out.read_text() == before      # nothing of the bad file was loaded
    with pytest.raises(dock.DockError):
        dock.dock_search_tune_load(tmp_path / "missing.txt")


def _fake_handles(dock, n_ligs=3, device=0):
    """Handle objects that never reach the library: every call below is rejected
    by the binding's own checks first (they hold no library handle)."""
    import synth
    pocket = object.__new__(dock.Pocket)
    pocket.handle, pocket.device, pocket.grid = None, device, synth.make_grid(8, 4)
    ligs = object.__new__(dock.Ligands)
    ligs.handle, ligs.n, ligs.max_torsions, ligs.pocket = None, n_ligs, 5, pocket
    net = object.__new__(dock.Mlp)
    net.handle, net.device = None, device
    return pocket, ligs, net


def test_binding_rejects_short_buffers_before_the_library():
    """Every buffer a kernel writes through is checked for its element count (and
    dtype) before its pointer reaches the library; a long enough buffer that is
    not on the device is rejected too.  CPU tensors only: nothing is launched."""
    import torch
    from paper_2509_12232_amd import dock
    pocket, ligs, net = _fake_handles(dock)
    P = dock.SearchParams(pop_size=10, n_generations=1, seed=1, box_lo=(0, 0, 0), box_hi=(1, 1, 1))
    f = lambda *s: torch.zeros(*s, dtype=torch.float32)   # noqa: E731
    i = lambda *s: torch.zeros(*s, dtype=torch.int32)     # noqa: E731
    G = 12
    pop, pe, bg, be = f(3, 10, G), f(3, 10), f(3, G), f(3)
    short = {
        "population": lambda: dock.dock_search(pocket, ligs, P, f(3, 9, G), pe, bg, be),
        "pop_energy": lambda: dock.dock_search(pocket, ligs, P, pop, f(29), bg, be),
        "best_genotypes": lambda: dock.dock_search(pocket, ligs, P, pop, pe, f(3 * G - 1), be),
        "best_energies": lambda: dock.dock_search(pocket, ligs, P, pop, pe, bg, f(2)),
        "target": lambda: dock.dock_search(pocket, ligs, P, pop, pe, bg, be, target=f(2), gen_reached=i(3)),
        "gen_reached": lambda: dock.dock_search(pocket, ligs, P, pop, pe, bg, be, target=f(3), gen_reached=i(2)),
        "plan population": lambda: dock.dock_search_plan_create(pocket, ligs, P, f(3, 9, G), pe, bg, be),
        "de_init": lambda: dock.dock_de_init(ligs, P, f(2, 10, G)),
        "de_trials": lambda: dock.dock_de_trials(ligs, P, 0, pop, f(3, 10, G - 1)),
        "energies": lambda: dock.dock_score_poses(pocket, ligs, f(100, G), f(99)),
        "pose_ligand": lambda: dock.dock_score_poses(pocket, ligs, f(100, G), f(100), pose_ligand=i(50)),
        "maps_out": lambda: dock.dock_pocket_maps(pocket, f(6 * 8 ** 3 - 1)),
        "mlp y": lambda: dock.dock_mlp_forward(net, f(10, 96), f(10, 31)),
        "mlp grads": lambda: dock.dock_mlp_gradients(net, f(10, 96), f(10, 32), f(dock.DOCK_MLP_PARAMS - 1), f(1)),
        "mlp target": lambda: dock.dock_mlp_gradients(net, f(10, 96), f(9, 32), f(dock.DOCK_MLP_PARAMS), f(1)),
        "mlp losses": lambda: dock.dock_mlp_train(net, f(64, 96), f(64, 32), 16, 4, 1e-3, losses=f(3)),
        "descriptors": lambda: dock.dock_ligand_descriptors(ligs, f(3 * 64 - 1)),
        "features": lambda: dock.dock_mlp_features(ligs, P, pop, f(30, 95)),
        "moves": lambda: dock.dock_mlp_moves(ligs, P, pop, pop, f(30 * 32 - 1)),
        "proposals": lambda: dock.dock_propose(ligs, net, P, 0, 1.0, pop, f(3, 10, G - 1)),
    }
    for what, call in short.items():
        with pytest.raises(ValueError, match="at least"):
            call()
    # long enough, but host memory: still rejected before the library is called
    with pytest.raises(TypeError, match="device tensor"):
        dock.dock_search(pocket, ligs, P, pop, pe, bg, be)
    with pytest.raises(TypeError, match="float32"):
        dock.dock_search(pocket, ligs, P, pop.double(), pe, bg, be)


def test_force_field_needs_a_positive_cap():
    """The pair term's caps compare float bit patterns as integers, which orders
    them like floats only for a positive bound: a cap <= 0 (or not finite) is
    rejected on the host, before anything touches a device."""
    import dataclasses
    import numpy as np
    import synth
    from paper_2509_12232_amd import dock
    nt = 4
    grid = synth.make_grid(8, nt)
    maps = np.zeros((nt + 2, 8, 8, 8), np.float32)
    for cap in (0.0, -10.0, float("inf"), float("nan")):
        ff = dataclasses.replace(synth.forcefield(nt), e_cap=cap)
        with pytest.raises(dock.DockError) as ei:
            dock.dock_create_pocket(grid, maps, ff)
        assert ei.value.status == dock.DOCK_E_INVALID, cap
