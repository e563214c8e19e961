"""Input-generator checks: cross sections against textbook values, band tables,
lattice positions, seeding."""
import math

import numpy as np
import pytest

from paper_1807_07094_amd import workload as W


def test_threshold_cross_sections():
    # hydrogenic threshold value and Z^-2 scaling (Osterbrock & Ferland)
    assert W.sigma_hydrogenic(W.E_THR_EV[0], 1) == pytest.approx(6.30e-18, rel=1e-3)
    assert W.sigma_hydrogenic(W.E_THR_EV[2], 2) == pytest.approx(6.30e-18 / 4, rel=1e-3)
    # He I ground state at threshold, Verner et al. (1996) fit: 7.4e-18 cm^2
    assert W.sigma_hei(W.E_THR_EV[1]) == pytest.approx(7.43e-18, rel=5e-3)
    assert W.sigma_hei(24.0) == 0.0 and W.sigma_hydrogenic(13.0, 1) == 0.0
    # far above threshold the hydrogenic cross section falls roughly as nu^-3
    r = W.sigma_hydrogenic(400.0, 1) / W.sigma_hydrogenic(200.0, 1)
    assert 2 ** -3.3 < r < 2 ** -2.7


def test_blackbody_bands():
    b = W.bins_blackbody()
    assert b["frac"].sum() == pytest.approx(1.0, abs=1e-12)
    e = b["e_erg"] / W.EV_ERG
    assert 13.6 < e[0] < 24.6 < e[1] < 54.4 < e[2]
    # photon-weighted averages of a 1e5 K blackbody with edges 13.6, 24.6, 54.4 eV
    np.testing.assert_allclose(b["frac"], [0.4474, 0.4940, 0.0586], rtol=3e-3)
    np.testing.assert_allclose(e, [18.86, 35.08, 65.64], rtol=3e-3)
    np.testing.assert_allclose(b["sigma"][:, 0], [3.000e-18, 5.698e-19, 7.886e-20], rtol=5e-3)
    assert b["sigma"][2, 2] == pytest.approx(1.051e-18, rel=5e-3)
    assert b["sigma"][0, 1] == 0 and b["sigma"][0, 2] == 0 and b["sigma"][1, 2] == 0


def test_lognormal_workload():
    w = W.lognormal(32, 40, seed=3)
    assert w.grid["n_h"].dtype == np.float32 and w.shape == (32, 32, 32)
    assert np.mean(w.grid["n_h"]) == pytest.approx(1e-3, rel=0.05)
    ln = np.log(w.grid["n_h"].astype(np.float64))
    assert np.std(ln) == pytest.approx(1.0, rel=0.03)
    pos = w.sources["pos"]
    assert np.all(pos * W.LATTICE == np.round(pos * W.LATTICE))
    cells = np.floor(pos).astype(int)
    dens = w.grid["n_h"][cells[:, 2], cells[:, 1], cells[:, 0]]
    assert np.all(dens >= np.quantile(w.grid["n_h"], 0.99) * (1 - 1e-6))
    nd = w.sources["ndot"]
    assert np.all((nd >= 1e48) & (nd <= 1e51))
    w2 = W.lognormal(32, 40, seed=3)
    assert np.array_equal(w.grid["n_h"], w2.grid["n_h"]) and np.array_equal(pos, w2.sources["pos"])
    assert not np.array_equal(W.lognormal(32, 40, seed=4).grid["n_h"], w.grid["n_h"])


def test_power_law_luminosities():
    nd = W.power_law_ndot(200000, seed=1)
    # dN/dNdot ~ Ndot^-2 on [a, b]: P(Ndot > x) = (1/x - 1/b) / (1/a - 1/b)
    for x in (2e48, 1e49, 1e50):
        expect = (1 / x - 1e-51) / (1e-48 - 1e-51)
        assert np.mean(nd > x) == pytest.approx(expect, abs=0.005)


def test_grf_workload_small():
    w = W.grf(32, 8, seed=5)
    d = np.log(w.grid["n_h"].astype(np.float64) / 1e-3) + 0.125
    assert np.std(d) == pytest.approx(0.5, rel=0.01)
    # smoothed: neighbouring cells are strongly correlated
    c = np.corrcoef(d[:, :, :-1].ravel(), d[:, :, 1:].ravel())[0, 1]
    assert c > 0.8


def test_c1():
    w = W.c1()
    assert w.shape == (64, 64, 64)
    assert w.grid["cell_cm"] == pytest.approx(3.18213e20, rel=1e-5)
    assert w.trace["level0"] == 0 and w.trace["rays_per_cell"] == 4.0
    kappa = w.grid["cell_cm"] * 1e-3 * 6.30e-18 * 0.9988
    assert kappa == pytest.approx(2.00, abs=0.01)
