"""GPU checks on the 256^3 lognormal workload with 1024 sources (power-law luminosities,
positions in the densest 1% of the cells), traced as one persistent batched launch with the
autotuned launch shape and recorded HIP graphs.

* A sample of the sources (every 64th) against the FP64 oracle on the whole grid: per-cell
  Gamma within the parity bar, crossing counts equal up to the few tau-termination decisions
  that FP32 tau may take differently.
* All sources: photon conservation; the autotuned shape, the default shape and the plain
  per-level schedule give the same fixed-point field bit for bit; graph replay = eager.
"""
import os

import numpy as np
import pytest

import oracle
from helpers import CONSERVATION_TOL, GAMMA_REL_TOL, conservation, rate_errors
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3(arc):
    import torch

    w = W.config(2)
    ctx = arc.Context(0)
    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    yield w, ctx, g, gamma, heat
    ctx.close()


def trace(w, ctx, g, gamma, heat, sources, schedule="batched_tuned", graph=True):
    return ctx.trace(g, sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                     rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"],
                     precision="fp32_comp", schedule=schedule, graph=graph and schedule != "plain")


def field(ctx, nb, ncell):
    import torch

    J = torch.empty(nb * ncell, dtype=torch.int64, device="cuda")
    ctx.get_field(J)
    return J


def test_c3_sample_against_oracle(c3):
    w, ctx, g, gamma, heat = c3
    nsrc = len(w.sources["ndot"])
    sub = w.subset(np.arange(0, nsrc, 64))
    print(f"[c3] {len(sub.sources['ndot'])} sources on {w.shape}", flush=True)
    led = trace(w, ctx, g, gamma, heat, sub.sources)
    gpu = {"gamma": gamma.cpu().numpy(), "heat": heat.cpu().numpy()}
    threads = max(1, min(16, os.cpu_count() or 1))
    r = oracle.trace_mt(w.grid, sub.sources, w.bins, w.trace, threads)
    oc = r["ledger"]["crossings"]
    og, oh, _ = oracle.finalize(w.grid, w.bins, r["J"])
    ora = {"gamma": og, "heat": oh}
    assert max(rate_errors(gpu, ora)) <= GAMMA_REL_TOL
    assert max(rate_errors(gpu, ora, "heat")) <= GAMMA_REL_TOL
    assert conservation(led) <= CONSERVATION_TOL
    assert abs(led["crossings"] - oc) <= max(8, oc // 1_000_000), (led["crossings"], oc)


def test_c3_all_sources_tuned_default_plain_and_graph_bitwise(c3):
    import torch

    w, ctx, g, gamma, heat = c3
    nb = len(w.bins["frac"])
    ncell = int(np.prod(w.shape))
    lt = trace(w, ctx, g, gamma, heat, w.sources, schedule="batched_tuned", graph=True)
    ref = field(ctx, nb, ncell)
    ld = trace(w, ctx, g, gamma, heat, w.sources, schedule="batched", graph=False)
    assert torch.equal(ref, field(ctx, nb, ncell))
    lp = trace(w, ctx, g, gamma, heat, w.sources, schedule="plain")
    assert torch.equal(ref, field(ctx, nb, ncell))
    lg = trace(w, ctx, g, gamma, heat, w.sources, schedule="batched_tuned", graph=True)
    assert torch.equal(ref, field(ctx, nb, ncell))
    for led in (lt, ld, lp, lg):
        assert conservation(led) <= CONSERVATION_TOL
        assert led["crossings"] == lt["crossings"]
    assert lt["crossings"] > 2e9  # the whole workload
