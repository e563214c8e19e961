"""GPU parity of the optically thin approximation (section 2.6) against the oracle: sources
with thin radii from zero to several split radii (rays of the levels below split at once),
the analytic fill, the measured R_tau<0.1 of every source, the ledger (the rays still
conserve photons; the fill's absorption is booked apart), plain = batched bitwise, split
trees bit-exact in geometry mode, the combination with the conserving correction, and the
argument checks."""
import numpy as np
import pytest

from helpers import CONSERVATION_TOL, GAMMA_REL_TOL, rate_errors, run_gpu_trace, run_oracle
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu

THIN_R_TOL = 1e-5  # measured radius: FP32 compensated depth against FP64


@pytest.fixture(scope="module")
def ctx(arc):
    c = arc.Context(0)
    yield c
    c.close()


def thin_workload(seed=41, shape=(40, 44, 36), n_src=5, radii=(0.0, 0.3, 2.75, 6.5, 13.0)):
    w = W.lognormal(0, n_src, seed, source_cells="uniform", shape=shape)
    # a partly ionised grid, as after a few steps: thin gas within 8 cells of the sources
    z, y, x = np.indices(w.shape) + 0.5
    ion = np.zeros(w.shape, bool)
    for p in w.sources["pos"]:
        ion |= (x - p[0]) ** 2 + (y - p[1]) ** 2 + (z - p[2]) ** 2 < 64.0
    w.grid["x_hi"] = np.where(ion, np.float32(1e-4), w.grid["x_hi"]).astype(np.float32)
    w.grid["x_hei"] = np.where(ion, np.float32(1e-3), w.grid["x_hei"]).astype(np.float32)
    w.grid["x_heii"] = np.where(ion, np.float32(0.5), w.grid["x_heii"]).astype(np.float32)
    w.sources["r_thin"] = np.array(radii[:n_src], np.float64)
    return w


def ledger_check(led):
    # rays: emitted = absorbed by the rays + escaped
    rays = led["absorbed"] - led["absorbed_thin"]
    return abs(led["emitted"] - rays - led["escaped"]) / led["emitted"]


@pytest.mark.parametrize("schedule", ["plain", "batched"])
def test_thin_parity(arc, ctx, schedule):
    w = thin_workload()
    print(f"[thin] {schedule} {w.shape} radii {w.sources['r_thin']}", flush=True)
    w.sources["r_thin_out"] = np.empty(len(w.sources["ndot"]))
    g = run_gpu_trace(arc, ctx, w, schedule=schedule)
    o = run_oracle(w)
    errs = rate_errors(g, o)
    assert max(errs) <= GAMMA_REL_TOL, errs
    assert max(rate_errors(g, o, "heat")) <= GAMMA_REL_TOL
    np.testing.assert_allclose(w.sources["r_thin_out"], o["r_thin_out"], rtol=THIN_R_TOL)
    assert g["ledger"]["crossings"] == pytest.approx(o["ledger"]["crossings"], rel=1e-5, abs=50)
    led = g["ledger"]
    assert ledger_check(led) <= CONSERVATION_TOL
    dt = w.dt
    assert led["absorbed_thin"] == pytest.approx(o["ledger"]["absorbed_thin"] * dt, rel=1e-6)


def test_thin_plain_equals_batched_and_trees_bit_exact(arc, ctx):
    w = thin_workload(seed=43, radii=(0.0, 1.5, 4.0, 9.25, 20.0))
    a = run_gpu_trace(arc, ctx, w, schedule="plain", eps_term=0.0, tree_cap=1 << 22)
    b = run_gpu_trace(arc, ctx, w, schedule="batched", eps_term=0.0, tree_cap=1 << 22)
    c = run_gpu_trace(arc, ctx, w, schedule="batched", eps_term=0.0, tune_waves=2, tune_refill=1, tune_blocks=29)
    assert np.array_equal(a["J"], b["J"]) and np.array_equal(b["J"], c["J"])
    o = run_oracle(w, tree_cap=1 << 22, eps_term=0.0)
    assert np.array_equal(b["tree"], o["tree"])
    assert b["ledger"]["crossings"] == o["ledger"]["crossings"]
    assert b["ledger"]["splits"] == o["ledger"]["splits"]
    assert max(rate_errors(b, o)) <= GAMMA_REL_TOL


def test_thin_with_the_conserving_correction(arc, ctx):
    w = thin_workload(seed=45, radii=(0.0, 3.5, 7.0, 0.0, 11.0))
    w.sources["r_thin_out"] = np.empty(len(w.sources["ndot"]))
    w.trace["correction"] = 2
    try:
        o = run_oracle(w)
    finally:
        w.trace.pop("correction")
    g = run_gpu_trace(arc, ctx, w, correction="conserving")
    assert max(rate_errors(g, o)) <= GAMMA_REL_TOL
    np.testing.assert_allclose(w.sources["r_thin_out"], o["r_thin_out"], rtol=THIN_R_TOL)
    assert ledger_check(g["ledger"]) <= CONSERVATION_TOL


def test_thin_radius_grows_over_steps(arc, ctx):
    """Feeding each trace the radius the previous one measured: the GPU and the oracle reach
    the same radii, and a radius fed back reproduces the oracle's field. Rays start at the
    radius fed in, so a measured radius never falls below it (a source near a face of the
    box may keep a radius below one cell: the shortest way out)."""
    w = thin_workload(seed=47, radii=(0.0,) * 5)
    r = np.zeros(5)
    radii = []
    for step in range(2):
        w.sources["r_thin"] = r.copy()
        w.sources["r_thin_out"] = np.empty(5)
        g = run_gpu_trace(arc, ctx, w)
        o = run_oracle(w)
        np.testing.assert_allclose(w.sources["r_thin_out"], o["r_thin_out"], rtol=THIN_R_TOL)
        assert max(rate_errors(g, o)) <= GAMMA_REL_TOL, step
        r = o["r_thin_out"].copy()
        radii.append(r)
    assert np.all(radii[0] > 0.0)
    assert np.all(radii[1] >= radii[0].astype(np.float32).astype(np.float64))


def test_thin_argument_checks(arc, ctx):
    w = thin_workload(shape=(12, 12, 12), n_src=2)
    w.sources["r_thin_out"] = np.empty(2)
    with pytest.raises(arc.ArcError) as e:
        run_gpu_trace(arc, ctx, w, precision="fp32_plain")
    assert e.value.status == -7
    w.sources.pop("r_thin_out")
    for bad in (-1.0, np.inf, 2e6):
        w.sources["r_thin"] = np.array([1.0, bad])
        with pytest.raises(arc.ArcError) as e:
            run_gpu_trace(arc, ctx, w)
        assert e.value.status == -2


def test_thin_graph_replays_equal_eager(arc, ctx):
    """Recorded graphs with thin spheres: the radii are read from device memory at every
    replay, so a replay with new radii (the same fill shape) equals an eager trace with them,
    and the measured radii too."""
    w = thin_workload(seed=49, radii=(0.0, 2.0, 5.5, 8.0, 3.0))
    out = []
    for radii in ((0.0, 2.0, 5.5, 8.0, 3.0), (1.0, 2.5, 5.0, 7.5, 3.5), (0.0, 2.0, 5.5, 8.0, 3.0)):
        w.sources["r_thin"] = np.array(radii)
        res = {}
        for graph in (True, False):
            w.sources["r_thin_out"] = np.empty(5)
            g = run_gpu_trace(arc, ctx, w, graph=graph)
            res[graph] = (g["J"], w.sources["r_thin_out"].copy(), g["ledger"]["absorbed_thin"])
        assert np.array_equal(res[True][0], res[False][0])
        assert np.array_equal(res[True][1], res[False][1])
        assert res[True][2] == pytest.approx(res[False][2], rel=1e-12)
        out.append(res[True][0])
    assert np.array_equal(out[0], out[2]) and not np.array_equal(out[0], out[1])
