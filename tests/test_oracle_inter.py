"""Pins of the oracle's inter-energy term (grid-map lookup, Sec. V, Algorithm 2)
and of its AutoGrid-style maps (Sec. V), against closed forms, scipy's
RegularGridInterpolator and brute-force ligand-receptor pair sums."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import synth

NT = 3


def _grid(dims=(6, 5, 7), origin=(-1.25, 0.5, 2.0), h=0.375, nt=NT):
    return synth.Grid(dims=dims, origin=origin, spacing=h, n_types=nt)


def _node(grid, i, j, k):
    return np.array(grid.origin) + np.array([i, j, k]) * grid.spacing


def _maps_from(fn_list, grid):
    nx, ny, nz = grid.dims
    x = grid.origin[0] + np.arange(nx) * grid.spacing
    y = grid.origin[1] + np.arange(ny) * grid.spacing
    z = grid.origin[2] + np.arange(nz) * grid.spacing
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([fn(X, Y, Z) for fn in fn_list]).astype(np.float32)


def _random_maps(grid, seed=0):
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid.dims
    return rng.uniform(-5, 5, size=(grid.n_maps, nz, ny, nx)).astype(np.float32)


def test_exact_at_nodes(ora):
    grid = _grid()
    maps = _random_maps(grid)
    nx, ny, nz = grid.dims
    pts, types = [], []
    for (i, j, k) in [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (2, 3, 4), (nx - 1, 0, 3), (1, ny - 1, nz - 1)]:
        for t in range(NT):
            pts.append(_node(grid, i, j, k))
            types.append(t)
    pts = np.array(pts)
    q = np.zeros(len(pts))
    e = ora.inter_atoms(grid, maps, pts, types, q)
    for n, p in enumerate(pts):
        i, j, k = np.rint((p - np.array(grid.origin)) / grid.spacing).astype(int)
        assert e[n] == float(maps[types[n], k, j, i])


def test_charge_scaling_of_elec_and_desolv(ora):
    """e = T_t + q E + |q| D: with constant maps the three pieces separate."""
    grid = _grid()
    maps = np.zeros((grid.n_maps,) + tuple(reversed(grid.dims)), np.float32)
    maps[0] = 1.5
    maps[NT] = 2.0      # electrostatic
    maps[NT + 1] = 0.25  # desolvation
    p = np.array([_node(grid, 2, 2, 2) + 0.1])
    for q in (-0.4, 0.0, 0.3):
        e = ora.inter_atoms(grid, maps, p, [0], [q])[0]
        assert e == pytest.approx(1.5 + q * 2.0 + abs(q) * 0.25, abs=1e-14)


def test_trilinear_polynomial_reproduced(ora):
    """Any a+bx+cy+dz+exy+fxz+gyz+hxyz sampled at the nodes is interpolated exactly."""
    grid = _grid(origin=(0.0, 0.0, 0.0), h=0.5)
    co = [0.5, 1.25, -0.75, 2.0, 0.5, -1.0, 0.25, 0.125]

    def poly(X, Y, Z):
        a, b, c, d, e, f, g, h = co
        return a + b * X + c * Y + d * Z + e * X * Y + f * X * Z + g * Y * Z + h * X * Y * Z

    maps = _maps_from([poly] * grid.n_maps, grid)
    assert np.array_equal(maps.astype(np.float64), _maps_from([poly] * grid.n_maps, grid).astype(np.float64))
    rng = np.random.default_rng(1)
    up = grid.upper()
    pts = rng.uniform(np.array(grid.origin), up, size=(200, 3))
    e = ora.inter_atoms(grid, maps, pts, np.zeros(200, np.int32), np.zeros(200))
    ref = poly(pts[:, 0], pts[:, 1], pts[:, 2])
    np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-12)


def test_linear_along_cell_edge(ora):
    grid = _grid()
    maps = _random_maps(grid, 2)
    base = _node(grid, 1, 2, 3)
    for axis in range(3):
        s = np.linspace(0.0, 1.0, 9) * grid.spacing
        pts = np.repeat(base[None], len(s), axis=0)
        pts[:, axis] += s
        e = ora.inter_atoms(grid, maps, pts, np.ones(len(s), np.int32), np.zeros(len(s)))
        np.testing.assert_allclose(np.diff(e, 2), 0.0, atol=1e-12)


def test_matches_scipy_regular_grid_interpolator(ora):
    grid = _grid(dims=(9, 8, 10))
    maps = _random_maps(grid, 3)
    nx, ny, nz = grid.dims
    axes = [grid.origin[d] + np.arange(grid.dims[d]) * grid.spacing for d in range(3)]
    rng = np.random.default_rng(4)
    pts = rng.uniform(np.array(grid.origin) + 1e-9, grid.upper() - 1e-9, size=(300, 3))
    types = rng.integers(0, NT, 300).astype(np.int32)
    q = rng.uniform(-0.5, 0.5, 300)
    e = ora.inter_atoms(grid, maps, pts, types, q)
    ref = np.zeros(300)
    for m in range(grid.n_maps):
        # maps are [z][y][x]; scipy wants values[x][y][z]
        f = RegularGridInterpolator(axes, maps[m].astype(np.float64).transpose(2, 1, 0), method="linear")
        v = f(pts)
        if m < NT:
            ref += np.where(types == m, v, 0.0)
        elif m == NT:
            ref += q * v
        else:
            ref += np.abs(q) * v
    np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-12)


def test_outside_box_contributes_zero(ora):
    grid = _grid()
    maps = _random_maps(grid, 5) + np.float32(7.0)
    up = grid.upper()
    lo = np.array(grid.origin)
    mid = (lo + up) / 2
    pts = []
    for d in range(3):
        for side, val in ((0, lo[d] - 1e-9), (1, up[d] + 1e-9), (2, lo[d] - 5.0)):
            p = mid.copy()
            p[d] = val
            pts.append(p)
    pts = np.array(pts)
    e = ora.inter_atoms(grid, maps, pts, np.zeros(len(pts), np.int32), np.full(len(pts), 0.3))
    assert np.all(e == 0.0)
    # on the closed faces the atom is inside and takes the face value
    on = np.array([lo, up])
    e = ora.inter_atoms(grid, maps, on, np.zeros(2, np.int32), np.zeros(2))
    nx, ny, nz = grid.dims
    assert e[0] == float(maps[0, 0, 0, 0]) and e[1] == float(maps[0, nz - 1, ny - 1, nx - 1])


# ------------------------------------------------------------------------------ maps
def _tiny_system(seed=0, n_rec=8):
    """Receptor atoms on a shell 5-6 A from the grid centre so no clamp is active
    near the centre."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_rec, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz = (d * rng.uniform(5.0, 6.0, (n_rec, 1))).astype(np.float32)
    return synth.Receptor(xyz=xyz, type=rng.integers(0, NT, n_rec).astype(np.int32),
                          charge=rng.uniform(-0.5, 0.5, n_rec).astype(np.float32))


def _ff_with_solvation():
    ff = synth.forcefield(NT, solpar=-0.001, hbond_pairs=[(0, 2)])
    return ff


def test_maps_equal_brute_force_at_nodes(ora):
    """At grid nodes, map-based inter energy equals the brute-force ligand-receptor
    pair sum up to the float32 rounding of the stored map values."""
    ff = _ff_with_solvation()
    rec = _tiny_system()
    grid = synth.Grid(dims=(9, 9, 9), origin=(-1.5, -1.5, -1.5), spacing=0.375, n_types=NT)
    maps = ora.build_maps(ff, rec, grid)
    assert np.abs(maps).max() < ff.map_cap     # no clamp active
    rng = np.random.default_rng(1)
    for _ in range(20):
        ijk = rng.integers(0, 9, (4, 3))
        pts = np.array([_node(grid, *v) for v in ijk])
        types = rng.integers(0, NT, 4).astype(np.int32)
        q = rng.uniform(-0.5, 0.5, 4)
        e_map = ora.inter_atoms(grid, maps, pts, types, q).sum()
        e_bf = ora.brute_inter(ff, pts, types, q, rec)
        # each stored value carries <= 2^-24 relative rounding
        bound = 3 * 2.0 ** -24 * (np.abs(maps).max() * 4) * 4
        assert abs(e_map - e_bf) <= bound, (e_map, e_bf)


def test_map_interpolation_error_is_second_order(ora):
    """Off the nodes the error against the brute-force sum falls ~4x per halving of h
    (mean over many points, so the in-cell position averages out)."""
    ff = _ff_with_solvation()
    rec = _tiny_system(2)
    rng = np.random.default_rng(3)
    npts = 400
    pts = rng.uniform(-0.7, 0.7, size=(npts, 3))
    types = rng.integers(0, NT, npts).astype(np.int32)
    q = rng.uniform(-0.5, 0.5, npts)
    errs = []
    for h, n in ((0.375, 9), (0.1875, 17), (0.09375, 33)):
        grid = synth.Grid(dims=(n, n, n), origin=(-1.5, -1.5, -1.5), spacing=h, n_types=NT)
        maps = ora.build_maps(ff, rec, grid)
        e_map = ora.inter_atoms(grid, maps, pts, types, q)
        e_bf = np.array([ora.brute_inter(ff, pts[i:i + 1], types[i:i + 1], q[i:i + 1], rec) for i in range(npts)])
        errs.append(np.abs(e_map - e_bf).sum())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_elec_map_clamped_symmetrically(ora):
    ff = synth.forcefield(NT)
    rec = synth.Receptor(xyz=np.array([[0, 0, 0], [3.0, 0, 0]], np.float32), type=np.zeros(2, np.int32),
                         charge=np.array([0.5, -0.5], np.float32))
    grid = synth.Grid(dims=(9, 2, 2), origin=(0.0, 0.0, 0.0), spacing=0.375, n_types=NT)
    maps = ora.build_maps(ff, rec, grid)
    e = maps[NT, 0, 0, :]
    assert e[0] == pytest.approx(ff.map_cap) and e[8] == pytest.approx(-ff.map_cap)
    assert np.all(maps[:NT] <= ff.map_cap) and np.all(maps[NT + 1] <= ff.map_cap)
