"""GPU checks on the 512^3 lognormal workload with 4096 sources, the configuration of the
learned chemistry step (BF16 MLP on MFMA, the plain solver as the fallback beyond the gate):

* a sample of the sources (every 1024th) against the FP64 oracle on the whole grid: per-cell
  Gamma and H within the parity bar, crossing counts equal up to the few tau-termination
  decisions that FP32 tau may take differently;
* all sources: photon conservation, and the autotuned, default and plain schedules give the
  same fixed-point field bit for bit;
* the learned step from the grid as generated and the oracle's rates of the sample (rounded to
  FP32 for both sides), judged cell by cell by the oracle's chemistry on cells drawn half among
  the irradiated ones and half uniformly: fractions within 1e-3 absolute, T within 1e-2.
"""
import os

import numpy as np
import pytest

import oracle
from helpers import CONSERVATION_TOL, GAMMA_REL_TOL, conservation, rate_errors
from paper_1807_07094_amd import learned
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4(arc):
    import torch

    w = W.config(3, device="cuda")
    ctx = arc.Context(0)
    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    yield w, ctx, g, gamma, heat
    ctx.close()
    del g, gamma, heat
    torch.cuda.empty_cache()


def trace(w, ctx, g, gamma, heat, sources, schedule="batched_tuned", graph=True):
    return ctx.trace(g, sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                     rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"],
                     precision="fp32_comp", schedule=schedule, graph=graph and schedule != "plain")


def field(ctx, nb, ncell):
    import torch

    J = torch.empty(nb * ncell, dtype=torch.int64, device="cuda")
    ctx.get_field(J)
    return J


@pytest.fixture(scope="module")
def sample(c4):
    """The oracle's trace of every 1024th source, on the grid as generated."""
    w = c4[0]
    sub = w.subset(np.arange(0, len(w.sources["ndot"]), 1024))
    threads = max(1, min(16, os.cpu_count() or 1))
    r = oracle.trace_mt(w.grid, sub.sources, w.bins, w.trace, threads)
    og, oh, _ = oracle.finalize(w.grid, w.bins, r["J"])
    return sub, r["ledger"]["crossings"], og, oh


def test_c4_sample_against_oracle(c4, sample):
    w, ctx, g, gamma, heat = c4
    sub, oc, og, oh = sample
    print(f"[c4] {len(sub.sources['ndot'])} sources on {w.shape}", flush=True)
    led = trace(w, ctx, g, gamma, heat, sub.sources)
    gpu = {"gamma": gamma.cpu().numpy(), "heat": heat.cpu().numpy()}
    ora = {"gamma": og, "heat": oh}
    assert max(rate_errors(gpu, ora)) <= GAMMA_REL_TOL
    assert max(rate_errors(gpu, ora, "heat")) <= GAMMA_REL_TOL
    assert conservation(led) <= CONSERVATION_TOL
    assert abs(led["crossings"] - oc) <= max(8, oc // 1_000_000), (led["crossings"], oc)


def test_c4_all_sources_tuned_default_plain_bitwise(c4):
    import torch

    w, ctx, g, gamma, heat = c4
    nb = len(w.bins["frac"])
    ncell = int(np.prod(w.shape))
    lt = trace(w, ctx, g, gamma, heat, w.sources, schedule="batched_tuned", graph=True)
    ref = field(ctx, nb, ncell)
    ld = trace(w, ctx, g, gamma, heat, w.sources, schedule="batched", graph=False)
    assert torch.equal(ref, field(ctx, nb, ncell))
    lp = trace(w, ctx, g, gamma, heat, w.sources, schedule="plain")
    assert torch.equal(ref, field(ctx, nb, ncell))
    del ref
    for led in (lt, ld, lp):
        assert conservation(led) <= CONSERVATION_TOL
    assert lt["crossings"] == ld["crossings"] == lp["crossings"]


def test_c4_learned_step_judged_by_the_oracle(arc, c4, sample):
    import torch

    w, ctx, g, gamma, heat = c4
    _, _, og, oh = sample
    X, Y = learned.training_set(ctx, arc, n=400_000, seed=5, sizes=(48, 64), n_src=(32, 48))
    net = arc.MLP(ctx)
    net.train(X, Y, epochs=10, batch=1024, lr=2e-3, seed=3)
    del X, Y
    g32, h32 = og.astype(np.float32), oh.astype(np.float32)
    gamma.copy_(torch.from_numpy(g32))
    heat.copy_(torch.from_numpy(h32))
    st = ctx.chem_step(g, gamma, heat, w.dt, mode="mlp_gated", mlp=net, gate_tol=1e-3, **w.chem)
    accepted = st["cells"] - st["fallback"]
    print(f"[c4 judge] accepted {accepted} of {st['cells']} cells", flush=True)
    assert accepted > 0
    rng = np.random.default_rng(41)
    ncell = int(np.prod(w.shape))
    lit = np.flatnonzero(g32[0].reshape(-1) > 0)
    idx = np.unique(np.concatenate([rng.choice(lit, min(lit.size, 1 << 14), replace=False),
                                    rng.integers(0, ncell, 1 << 14)]))
    sub_grid = {"n_h": w.grid["n_h"].reshape(-1)[idx], "y_he": w.grid["y_he"]}
    sub_state = {k: w.grid[k].reshape(-1)[idx] for k in ("x_hi", "x_hei", "x_heii", "temp")}
    ref = oracle.chem(sub_grid, sub_state, g32.reshape(3, -1)[:, idx].astype(np.float64),
                      h32.reshape(3, -1)[:, idx].astype(np.float64), w.dt, w.chem)
    tid = torch.from_numpy(idx).cuda()
    for k in ("x_hi", "x_hei", "x_heii"):
        err = float(np.abs(g[k].reshape(-1)[tid].cpu().numpy() - ref[k]).max())
        assert err <= 1e-3, (k, err)
    t_err = float(np.abs(g["temp"].reshape(-1)[tid].cpu().numpy() / ref["temp"] - 1.0).max())
    assert t_err <= 1e-2, t_err
