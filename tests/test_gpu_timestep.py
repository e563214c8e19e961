"""GPU parity of the adaptive RT time step (section 2.9): the two grid minima from the HIP
reduction against the oracle's, each side from its own trace of the same seeded workload
(the oracle's rates from the oracle's tracer), for the hydrogen gas with a fixed alpha_B and
for the H + He gas with the Hui & Gnedin coefficients. Bar: 1e-3 relative (per-cell rates
agree to 1e-4; FP32 rate fits add ~1e-5). Edge cases: no changing cell gives +inf, bad
arguments are rejected."""
import numpy as np
import pytest

import oracle
from helpers import run_oracle
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(arc):
    c = arc.Context(0)
    yield c
    c.close()


def gpu_rates(arc, ctx, w):
    import torch

    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    ctx.trace(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
              rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"])
    return g, gamma


@pytest.mark.parametrize("which", ["c1", "lognormal"])
def test_timestep_parity(arc, ctx, which):
    if which == "c1":
        w = W.c1(n=32)
        w.grid["x_hi"] = np.full(w.shape, 0.5, np.float32)  # partly ionised: both limits act
    else:
        w = W.lognormal(0, 4, 13, source_cells="uniform", shape=(40, 36, 44))
    cp = w.chem
    sigma0 = float(np.asarray(w.bins["sigma"]).reshape(-1, 3)[0, 0])
    o = run_oracle(w)
    ref = oracle.timestep(w.grid, w.state(), o["gamma"], cp, sigma0, 0.1)
    g, gamma = gpu_rates(arc, ctx, w)
    got = ctx.rt_timestep(g, gamma, w.bins, eps=0.1, rates=cp.get("rates", 1), collisional=cp.get("collisional", 1),
                          alpha_hii=cp.get("alpha_hii", 2.59e-13))
    print(f"[timestep] {which} gpu {got} oracle {ref}", flush=True)
    for a, b in zip(got, ref):
        assert np.isfinite(b)
        assert a == pytest.approx(b, rel=1e-3)


def test_timestep_without_change_is_infinite(arc, ctx):
    import torch

    w = W.c1(n=16)
    w.grid["x_hi"] = np.ones(w.shape, np.float32)  # fully neutral and unlit: nothing changes
    g = arc.device_grid(w.grid)
    gamma = torch.zeros((3,) + w.shape, dtype=torch.float32, device="cuda")
    dn, di = ctx.rt_timestep(g, gamma, w.bins, eps=0.1, rates=0, collisional=0)
    assert dn == np.inf and di == np.inf


def test_timestep_rejects_bad_arguments(arc, ctx):
    import torch

    w = W.c1(n=8)
    g = arc.device_grid(w.grid)
    gamma = torch.zeros((3,) + w.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(arc.ArcError):
        ctx.rt_timestep(g, gamma, w.bins, eps=0.0)
    with pytest.raises(arc.ArcError):
        ctx.rt_timestep(g, gamma, w.bins, eps=0.1, rates=2)
