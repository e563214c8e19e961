"""Pins for the oracle tracer (section 2.1 steps iii a-d, section 2.4, eq:ion).

Each pin is fixed by something other than the tracer's own code: a closed-form
attenuation series, photon conservation, an independent enumeration of the ray tree
and its in-box path lengths, the 1/r^2 flux of a point source, and the flux the paper
prints for its Test 3 geometry."""
import math

import numpy as np
import pytest

import oracle
from paper_1807_07094_amd import workload as W


def uniform_grid(shape, cell_cm, n_h=1e-3, x_hi=1.0, y_he=0.0):
    g = {"n_h": np.full(shape, n_h, np.float32), "x_hi": np.full(shape, x_hi, np.float32),
         "x_hei": np.zeros(shape, np.float32), "x_heii": np.zeros(shape, np.float32),
         "cell_cm": cell_cm, "y_he": y_he}
    return g


def params(level0=0, phi=4.0, max_level=-1, eps_term=0.0):
    return {"level0": level0, "rays_per_cell": phi, "max_level": max_level, "eps_term": eps_term}


def test_single_ray_geometric_attenuation():
    """Uniform kappa per cell: along the +x root ray the deposit in the k-th cell beyond
    the source cell is P e^{-kappa (k - 1/2)} g(kappa); the escaping fraction of every
    root ray is e^{-kappa len}."""
    n = 64
    L = 3.0e20
    sigma = 6.3e-18
    kappa = 0.1
    n_h = kappa / (L * sigma)
    g = uniform_grid((n, n, n), L, n_h=n_h)
    kap32 = float(np.float32(n_h)) * L * sigma  # the grid stores n_H as float32
    bins = W.bins_monochromatic(13.6, sigma)
    S = 5e48
    src = {"pos": np.array([[32.5, 32.5, 32.5]]), "ndot": np.array([S])}
    r = oracle.trace(g, src, bins, params(level0=0, max_level=0))
    J = r["J"][0]
    P = S / 12
    gk = -math.expm1(-kap32) / kap32
    for k in range(1, 31):
        expect = P * math.exp(-kap32 * (k - 0.5)) * gk
        assert J[32, 32, 32 + k] == pytest.approx(expect, rel=1e-13)
    dirs = oracle.healpix_vec(0, np.arange(12)).astype(np.float32).astype(np.float64)
    esc = 0.0
    for d in dirs:
        t = min((n - 32.5) / c if c > 0 else (-32.5 / c if c < 0 else np.inf) for c in d)
        esc += P * math.exp(-kap32 * t)
    assert r["ledger"]["escaped"] == pytest.approx(esc, rel=1e-13)


def tree_path_integral(shape, xs, S, level0, phi, lmax):
    """Independent enumeration of the ray tree for a transparent grid: sum of
    P_ray * (in-box length of the ray between its start and split radii), and the set
    of rays traced. No cell stepping is involved."""
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    total = 0.0
    rays = []
    stack = [(level0, p) for p in range(12 * 4 ** level0)]
    while stack:
        level, p = stack.pop()
        d = oracle.healpix_vec(level, [p])[0].astype(np.float32).astype(np.float64)
        t0 = 0.0 if level == level0 else oracle.t_split(phi, level - 1)
        t_end = oracle.t_split(phi, level) if level < lmax else np.inf
        exit_t = min((dims[i] - xs[i]) / d[i] if d[i] > 0 else (-xs[i] / d[i] if d[i] < 0 else np.inf)
                     for i in range(3))
        rays.append((level, p))
        if t0 >= exit_t:
            continue
        total += S / (12 * 4 ** level) * (min(t_end, exit_t) - t0)
        if t_end < exit_t:
            stack += [(level + 1, 4 * p + k) for k in range(4)]
    return total, rays


@pytest.mark.parametrize("shape,xs,level0,phi", [
    ((16, 16, 16), (8.0, 8.0, 8.0), 0, 4.0),
    ((12, 20, 16), (5.25, 9.5, 3.75), 1, 4.0),
    ((10, 10, 10), (2.125, 7.0625, 4.5), 0, 1.0),
])
def test_transparent_tree_and_path_integral(shape, xs, level0, phi):
    g = uniform_grid(shape, 1e20, x_hi=0.0)
    bins = W.bins_monochromatic()
    S = 1e48
    src = {"pos": np.array([xs]), "ndot": np.array([S])}
    r = oracle.trace(g, src, bins, params(level0=level0, phi=phi), tree_cap=10 ** 6)
    lmax = oracle.auto_max_level(shape, phi)
    total, rays = tree_path_integral(shape, np.array(xs), S, level0, phi, lmax)
    assert r["J"].sum() == pytest.approx(total, rel=1e-12)
    got = {((int(t) >> 28) & 15, int(t) & ((1 << 28) - 1)) for t in r["tree"]}
    assert got == set(rays)
    L = r["ledger"]
    assert L["escaped"] == pytest.approx(S, rel=1e-12)
    assert L["rays"] == 12 * 4 ** level0 + 4 * L["splits"]
    assert L["rays"] == L["splits"] + L["escaped_rays"] + L["terminated"]


def test_point_source_flux_falls_as_inverse_square():
    """Transparent grid: J_c 4 pi r_c^2 / S -> 1 in radial shells."""
    n = 48
    g = uniform_grid((n, n, n), 1e20, x_hi=0.0)
    S = 1e48
    src = {"pos": np.array([[24.0, 24.0, 24.0]]), "ndot": np.array([S])}
    r = oracle.trace(g, src, W.bins_monochromatic(), params(level0=1, phi=4.0))
    J = r["J"][0]
    z, y, x = np.indices(J.shape) + 0.5
    rr = np.sqrt((x - 24) ** 2 + (y - 24) ** 2 + (z - 24) ** 2)
    q = J * 4 * np.pi * rr ** 2 / S
    for lo in (4, 8, 12, 16, 20):
        m = (rr >= lo) & (rr < lo + 4)
        assert q[m].mean() == pytest.approx(1.0, abs=0.01), lo


def test_paper_test3_flux(golden):
    """Section 3, Test 3: 3e51 photons/s from the face centre at cell x = 0 give
    1e6 photons/s/cm^2 at the clump centre 97 cells away (6.6 kpc on 128 cells).
    Transparent narrow box around the axis, Phi = 16, 3x3x3 average."""
    t3 = golden["test3"]
    L = t3["box_kpc"] * W.KPC_CM / t3["n"]
    shape = (9, 9, 100)
    g = uniform_grid(shape, L, x_hi=0.0)
    src = {"pos": np.array([[0.0, 4.5, 4.5]]), "ndot": np.array([t3["ndot"]])}
    r = oracle.trace(g, src, W.bins_monochromatic(), params(level0=1, phi=16.0))
    flux = r["J"][0] / L ** 2
    cx = t3["clump_cell"][0]
    avg = flux[3:6, 3:6, cx - 1:cx + 2].mean()
    assert avg == pytest.approx(t3["flux"], rel=0.05)


@pytest.mark.parametrize("eps_term", [0.0, 1e-6])
def test_conservation_and_species_routes(eps_term):
    w = W.lognormal(20, 3, seed=11, source_cells="uniform", eps_term=eps_term)
    # give the helium something to absorb in every band
    w.grid["x_heii"][...] = 0.3
    w.grid["x_hei"][...] = 0.6
    r = oracle.trace(w.grid, w.sources, w.bins, w.trace, direct=True)
    L = r["ledger"]
    gamma, heat, absorbed = oracle.finalize(w.grid, w.bins, r["J"])
    assert L["emitted"] == pytest.approx(w.sources["ndot"].sum(), rel=1e-15)
    assert abs(L["emitted"] - absorbed - L["escaped"]) <= 1e-10 * L["emitted"]
    assert absorbed == pytest.approx(L["absorbed_trace"], rel=1e-12)
    for sp in range(3):
        m = r["gdir"][sp] > 0
        assert m.sum() > 100
        np.testing.assert_allclose(r["gdir"][sp][m], gamma[sp][m], rtol=1e-12)
    assert L["rays"] == L["splits"] + L["escaped_rays"] + L["terminated"]
    if eps_term == 0:
        assert L["terminated"] == 0


def test_heating_rate_definition():
    """H_S = sum_b sigma_bS (E_b - E_S)^+ J_b / L^2, zero for bins below threshold."""
    w = W.lognormal(12, 2, seed=5, source_cells="uniform")
    r = oracle.trace(w.grid, w.sources, w.bins, w.trace)
    gamma, heat, _ = oracle.finalize(w.grid, w.bins, r["J"])
    L2 = w.grid["cell_cm"] ** 2
    b = w.bins
    for sp in range(3):
        expect = sum(b["sigma"][k, sp] * max(b["e_erg"][k] - b["e_thr"][sp], 0) * r["J"][k] for k in range(3)) / L2
        np.testing.assert_allclose(heat[sp], expect, rtol=1e-13)
    # HeI cannot absorb below 24.6 eV and HeII below 54.4 eV
    assert b["sigma"][0, 1] == 0 and b["sigma"][0, 2] == 0 and b["sigma"][1, 2] == 0


def test_linear_in_sources():
    """J is a sum over sources: two disjoint halves add up to the whole."""
    w = W.lognormal(16, 4, seed=9, source_cells="uniform")
    full = oracle.trace(w.grid, w.sources, w.bins, w.trace)["J"]
    a = oracle.trace(w.grid, w.subset([0, 2]).sources, w.bins, w.trace)["J"]
    b = oracle.trace(w.grid, w.subset([1, 3]).sources, w.bins, w.trace)["J"]
    np.testing.assert_allclose(a + b, full, rtol=1e-12, atol=1e-300)


@pytest.fixture(scope="module")
def golden():
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_oracle_equals_single_thread(threads):
    """The oracle on several host threads (used to time it on every core): the same field
    and ledger up to the order of the floating-point additions."""
    w = W.lognormal(24, 7, seed=13, source_cells="uniform")
    w.sources["r_thin"] = np.array([0.0, 2.5, 0.0, 0.7, 4.0, 0.0, 1.25])
    one = oracle.trace(w.grid, w.sources, w.bins, dict(w.trace, correction=2))
    many = oracle.trace_mt(w.grid, w.sources, w.bins, dict(w.trace, correction=2), threads)
    np.testing.assert_allclose(many["J"], one["J"], rtol=1e-13, atol=1e-300)
    np.testing.assert_array_equal(many["r_thin_out"], one["r_thin_out"])
    for k in ("crossings", "rays", "splits", "terminated", "escaped_rays"):
        assert many["ledger"][k] == one["ledger"][k], k
    for k in ("emitted", "absorbed_trace", "escaped", "absorbed_thin"):
        assert many["ledger"][k] == pytest.approx(one["ledger"][k], rel=1e-10), k  # sums of ~1e6 terms
