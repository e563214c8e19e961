"""Pins for the oracle's cell-by-cell stepping (section 2.4: each step reaches the next
x, y or z cell boundary).

Checked against a brute-force slab intersection of the ray with every cell box, and
against special cases with known answers."""
import math

import numpy as np
import pytest

import oracle


def brute_force(shape, xs, d, t0, t_end):
    """All cells whose box meets x(t) = xs + t d, t in [t0, t_end), in a segment of
    positive length, sorted by entry; along an axis with d = 0 a cell is the half-open
    interval [c, c + 1)."""
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    segs = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = (x, y, z)
                lo, hi = t0, t_end
                ok = True
                for i in range(3):
                    if d[i] == 0:
                        if not (c[i] <= xs[i] < c[i] + 1):
                            ok = False
                            break
                        continue
                    ta = (c[i] - xs[i]) / d[i]
                    tb = (c[i] + 1 - xs[i]) / d[i]
                    lo = max(lo, min(ta, tb))
                    hi = min(hi, max(ta, tb))
                if ok and hi - lo > 1e-12:
                    segs.append((lo, x + nx * (y + ny * z), hi - lo))
    segs.sort()
    assert all(0 <= c < math.prod(dims) for _, c, _ in segs)
    return [s[1] for s in segs], np.array([s[2] for s in segs])


def f32(v):
    return np.asarray(v, np.float32).astype(np.float64)


def lattice(rng, shape):
    nz, ny, nx = shape
    return (rng.integers(0, [nx, ny, nz]) + rng.integers(0, 4096, 3) / 4096).astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (5, 5, 5), (8, 8, 8), (3, 7, 2)])
def test_brute_force_random_rays(shape):
    rng = np.random.default_rng(sum(shape))
    nz, ny, nx = shape
    for trial in range(60):
        xs = lattice(rng, shape)
        d = rng.standard_normal(3)
        d = f32(d / np.linalg.norm(d))
        t0 = float(rng.choice([0.0, 0.25, 1.0 + rng.random()]))
        t_end = float(rng.choice([-1.0, t0 + 0.5 + 3 * rng.random()]))
        cells, ds, how = oracle.walk(shape, xs, d, t0, t_end)
        ref_cells, ref_ds = brute_force(shape, xs, d, t0, t_end if t_end > 0 else np.inf)
        assert list(cells) == ref_cells, (trial, xs, d, t0, t_end)
        np.testing.assert_allclose(ds, ref_ds, atol=1e-12)


def test_brute_force_healpix_directions_from_lattice_points():
    shape = (6, 6, 6)
    rng = np.random.default_rng(3)
    for level in (0, 1, 2):
        dirs = f32(oracle.healpix_vec(level, np.arange(oracle.npix(level))).astype(np.float32))
        for q in range(0, len(dirs), max(1, len(dirs) // 24)):
            for xs in (np.array([3.0, 3.0, 3.0]), np.array([2.5, 3.0, 1.25]), lattice(rng, shape)):
                cells, ds, _ = oracle.walk(shape, xs, dirs[q], 0.0, -1.0)
                ref_cells, ref_ds = brute_force(shape, xs, dirs[q], 0.0, np.inf)
                assert list(cells) == ref_cells
                np.testing.assert_allclose(ds, ref_ds, atol=1e-12)


def test_axis_ray_unit_steps():
    cells, ds, how = oracle.walk((8, 8, 8), [3.5, 2.5, 4.5], [1.0, 0.0, 0.0])
    assert how == 0
    assert list(cells) == [x + 8 * (2 + 8 * 4) for x in range(3, 8)]
    np.testing.assert_array_equal(ds, [0.5, 1, 1, 1, 1])


def test_diagonal_ray_exact_corner_steps():
    """(1,1,0)/sqrt(2) from a cell centre passes through cell corners: x and y advance
    together, so no zero-length segment appears."""
    d = f32([1 / math.sqrt(2), 1 / math.sqrt(2), 0.0])
    cells, ds, how = oracle.walk((8, 8, 8), [0.5, 0.5, 0.5], d)
    assert list(cells) == [i + 8 * i for i in range(8)]
    np.testing.assert_allclose(ds[1:], 1.0 / d[0], rtol=1e-15)
    np.testing.assert_allclose(ds[0], 0.5 / d[0], rtol=1e-15)


def test_ray_in_grid_plane_belongs_to_upper_cell():
    cells, ds, how = oracle.walk((4, 4, 4), [0.5, 2.0, 1.0], [1.0, 0.0, 0.0])
    assert list(cells) == [x + 4 * (2 + 4 * 1) for x in range(4)]


def test_start_on_boundary_moving_down():
    # starts on the plane x = 2 moving to -x: the first cell is x = 1
    cells, ds, how = oracle.walk((4, 4, 4), [2.0, 0.5, 0.5], [-1.0, 0.0, 0.0])
    assert list(cells) == [1 + 4 * (0 + 4 * 0), 0]
    np.testing.assert_array_equal(ds, [1.0, 1.0])
    cells, ds, how = oracle.walk((4, 4, 4), [0.0, 0.5, 0.5], [-1.0, 0.0, 0.0])
    assert how == 2 and len(cells) == 0


@pytest.mark.parametrize("seed", range(5))
def test_in_box_length(seed):
    """Sum of segment lengths = distance from the origin to the box surface."""
    rng = np.random.default_rng(seed)
    shape = (9, 13, 11)
    nz, ny, nx = shape
    for _ in range(50):
        xs = lattice(rng, shape)
        d = rng.standard_normal(3)
        d = f32(d / np.linalg.norm(d))
        cells, ds, how = oracle.walk(shape, xs, d)
        exit_t = min(((nx, ny, nz)[i] - xs[i]) / d[i] if d[i] > 0 else -xs[i] / d[i] for i in range(3))
        assert how == 0
        assert ds.sum() == pytest.approx(exit_t, rel=1e-13)


def test_split_end_inside_cell():
    cells, ds, how = oracle.walk((8, 8, 8), [0.5, 0.5, 0.5], [1.0, 0.0, 0.0], 0.0, 2.25)
    assert how == 1
    np.testing.assert_array_equal(ds, [0.5, 1.0, 0.75])
