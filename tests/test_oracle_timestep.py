"""Pins for the oracle's adaptive RT time step (section 2.9).

The two limits are plain definitions; what pins their code is what they promise, checked
with the oracle's independent chemistry integrator: over dt_n the limiting cell's neutral
density changes by the fraction eps, and over dt_I its optical depth (hence the intensity
behind it) changes by eps, both to first order in eps. Also: the tau > 0.5 restriction of
dt_n (and its absence for dt_I), and +inf when no cell changes."""
import numpy as np
import pytest

import oracle

SIGMA = 6.3e-18
CP = {"isothermal": 1, "rates": 0, "collisional": 0, "alpha_hii": 2.59e-13, "eps": 0.1}


def cells(x_hi, n_h=1e-3, L=3.0e20):
    x = np.asarray(x_hi, np.float32).reshape(1, 1, -1)
    grid = {"n_h": np.full(x.shape, n_h, np.float32), "cell_cm": L, "y_he": 0.0}
    state = {"x_hi": x, "x_hei": np.zeros_like(x), "x_heii": np.zeros_like(x), "temp": np.full(x.shape, 1e4, np.float32)}
    return grid, state


def gamma_of(shape, g):
    out = np.zeros((3,) + shape)
    out[0] = g
    return out


@pytest.mark.parametrize("eps", [0.01, 0.003])
def test_neutral_limit_is_the_fractional_change_eps(eps):
    grid, state = cells([0.9])
    gam = gamma_of(state["x_hi"].shape, 3e-13)
    dt_n, dt_i = oracle.timestep(grid, state, gam, CP, SIGMA, eps)
    assert np.isfinite(dt_n) and np.isfinite(dt_i)
    out = oracle.chem(grid, state, gam, gam * 0, dt_n, dict(CP, eps=1e-3))
    x0, x1 = float(state["x_hi"][0, 0, 0]), float(out["x_hi"][0, 0, 0])
    assert abs(x1 - x0) / x0 == pytest.approx(eps, rel=5 * eps)


@pytest.mark.parametrize("eps", [0.01, 0.003])
def test_intensity_limit_is_the_optical_depth_change_eps(eps):
    grid, state = cells([0.3])
    gam = gamma_of(state["x_hi"].shape, 1e-13)
    _, dt_i = oracle.timestep(grid, state, gam, CP, SIGMA, eps)
    out = oracle.chem(grid, state, gam, gam * 0, dt_i, dict(CP, eps=1e-3))
    dtau = SIGMA * grid["cell_cm"] * grid["n_h"][0, 0, 0] * abs(float(out["x_hi"][0, 0, 0]) - float(state["x_hi"][0, 0, 0]))
    assert dtau == pytest.approx(eps, rel=5 * eps)


def test_neutral_limit_ignores_optically_thin_cells():
    """A nearly ionised cell changes fastest in relative terms, but its tau is below 0.5:
    it limits dt_I, not dt_n."""
    grid, state = cells([0.9, 1e-4])
    gam = gamma_of(state["x_hi"].shape, 3e-13)
    dt_n, dt_i = oracle.timestep(grid, state, gam, CP, SIGMA, 0.1)
    g1, s1 = cells([0.9])
    dt_n1, dt_i1 = oracle.timestep(g1, s1, gamma_of(s1["x_hi"].shape, 3e-13), CP, SIGMA, 0.1)
    assert dt_n == dt_n1
    assert SIGMA * grid["cell_cm"] * 1e-3 * 1e-4 < 0.5
    # the thin cell's own intensity limit is smaller only if its |ndot| is larger
    assert dt_i <= dt_i1


def test_no_change_means_no_limit():
    grid, state = cells([1.0, 1.0])
    dt_n, dt_i = oracle.timestep(grid, state, gamma_of(state["x_hi"].shape, 0.0), CP, SIGMA, 0.1)
    assert dt_n == np.inf and dt_i == np.inf
