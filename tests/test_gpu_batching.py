"""Batched schedule extras: graph replay and the autotuner.

* replaying the recorded graphs gives the eager result bit for bit, on every replay,
  with other GPU work and synchronisations between the replays, and a change of the
  sources' luminosities (new fixed-point scales) is recorded afresh;
* the autotuner's chosen shape, and the tuned schedule (tuned on first use), reach the
  plain schedule's fixed-point field exactly;
* rays moved from a wave's on-chip stack to its spill area in memory and back (deep
  subtrees: work items at the first level) give the plain schedule's field bit for bit
  and the oracle's rates; a spill area too small for them fails with ARC_E_QUEUE and
  leaves the context usable.
"""
import numpy as np
import pytest

from helpers import CONSERVATION_TOL, GAMMA_REL_TOL, conservation, rate_errors, run_gpu_trace, run_oracle
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(arc):
    c = arc.Context(0)
    yield c
    c.close()


def test_graph_replays_equal_eager(arc, ctx):
    import torch

    w = W.lognormal(40, 12, 21)
    eager = run_gpu_trace(arc, ctx, w, schedule="batched")
    other = arc.Context(0)
    try:
        for rep in range(3):
            got = run_gpu_trace(arc, ctx, w, schedule="batched", graph=True)
            assert np.array_equal(got["J"], eager["J"]), rep
            assert np.array_equal(got["gamma"], eager["gamma"]), rep
            assert got["ledger"]["crossings"] == eager["ledger"]["crossings"]
            # FP64 atomics of the ledger sum in a run-dependent order
            assert abs(got["ledger"]["absorbed"] / eager["ledger"]["absorbed"] - 1) <= 1e-12
            # unrelated eager work between replays
            a = torch.randn(512, 512, device="cuda")
            float((a @ a).sum())
            run_gpu_trace(arc, other, W.lognormal(24, 3, 100 + rep), schedule="batched")
            torch.cuda.synchronize()
        # other luminosities: new fixed-point scales, recorded again
        w2 = w.subset(np.arange(12))
        w2.sources["ndot"] = w2.sources["ndot"] * np.linspace(0.5, 2.0, 12)
        e2 = run_gpu_trace(arc, ctx, w2, schedule="batched")
        g2 = run_gpu_trace(arc, ctx, w2, schedule="batched", graph=True)
        assert np.array_equal(g2["J"], e2["J"])
        assert not np.array_equal(e2["J"], eager["J"])
    finally:
        other.close()


def test_autotuner_shape_matches_plain_bitwise(arc, ctx):
    import torch

    w = W.lognormal(40, 12, 22)
    plain = run_gpu_trace(arc, ctx, w, schedule="plain")
    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, device="cuda")
    heat = torch.empty_like(gamma)
    res = ctx.autotune(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                       rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"])
    assert res["candidates"] >= 10
    assert res["waves"] in (2, 4, 8) and res["waves_per_cu"] in (8, 12, 16)
    assert res["refill"] in (16, 32, 48, 56, 64) and 5 <= res["item_delta"] <= 7
    assert res["stack"] in (64, 128, 256)
    assert 0 < res["ms_best"] <= res["ms_default"]
    tuned = run_gpu_trace(arc, ctx, w, schedule="batched_tuned")
    assert np.array_equal(tuned["J"], plain["J"])
    tuned_graph = run_gpu_trace(arc, ctx, w, schedule="batched_tuned", graph=True)
    assert np.array_equal(tuned_graph["J"], plain["J"])


def test_tuned_schedule_tunes_on_first_use(arc):
    w = W.lognormal(32, 9, 23)
    fresh = arc.Context(0)
    try:
        plain = run_gpu_trace(arc, fresh, w, schedule="plain")
        tuned = run_gpu_trace(arc, fresh, w, schedule="batched_tuned")
        assert np.array_equal(tuned["J"], plain["J"])
        assert tuned["ledger"]["crossings"] == plain["ledger"]["crossings"]
    finally:
        fresh.close()


def test_chemistry_graph_replays_equal_eager(arc, ctx):
    """The plain chemistry step recorded and replayed: every replay from the same state
    equals the eager step bit for bit, with other GPU work between replays."""
    import torch

    w = W.lognormal(32, 6, 24)
    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, device="cuda")
    heat = torch.empty_like(gamma)
    ctx.trace(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"], eps_term=w.trace["eps_term"])
    fields = ("x_hi", "x_hei", "x_heii", "temp")
    start = {k: g[k].clone() for k in fields}
    eager_stats = ctx.chem_step(g, gamma, heat, w.dt, **w.chem)
    eager = {k: g[k].clone() for k in fields}
    for rep in range(3):
        for k in fields:
            g[k].copy_(start[k])
        torch.cuda.synchronize()
        st = ctx.chem_step(g, gamma, heat, w.dt, graph=True, **w.chem)
        for k in fields:
            assert bool((g[k] == eager[k]).all()), (rep, k)
        assert st["sub_total"] == eager_stats["sub_total"]
        a = torch.randn(256, 256, device="cuda")
        float((a @ a).sum())
        torch.cuda.synchronize()


def deep_subtrees():
    # level-1 work items on a 96^3 grid: every item is a whole subtree of up to 8 levels,
    # far more than a wave's LDS stack (64 split rays' families) holds
    return W.lognormal(96, 8, 25, source_cells="uniform")


def test_spilled_rays_match_plain_and_oracle(arc, ctx):
    w = deep_subtrees()
    print(f"[spill] {w.shape} {len(w.sources['ndot'])} sources, item level {w.trace['level0']}", flush=True)
    b = run_gpu_trace(arc, ctx, w, schedule="batched", tune_item_level=w.trace["level0"], tune_waves=1)
    assert b["ledger"]["spills"] > 0, b["ledger"]
    p = run_gpu_trace(arc, ctx, w, schedule="plain")
    assert np.array_equal(b["J"], p["J"])
    assert b["ledger"]["crossings"] == p["ledger"]["crossings"]
    o = run_oracle(w)
    assert max(rate_errors(b, o)) <= GAMMA_REL_TOL
    assert conservation(b["ledger"]) <= CONSERVATION_TOL


def test_spill_area_overflow_is_reported_and_context_reused(arc, ctx):
    w = deep_subtrees()
    with pytest.raises(arc.ArcError) as e:
        run_gpu_trace(arc, ctx, w, schedule="batched", tune_item_level=w.trace["level0"], tune_waves=1, spill_cap=2)
    assert e.value.status == -6, e.value
    # the same context traces correctly afterwards
    again = run_gpu_trace(arc, ctx, w, schedule="batched", tune_item_level=w.trace["level0"], tune_waves=1)
    p = run_gpu_trace(arc, ctx, w, schedule="plain")
    assert np.array_equal(again["J"], p["J"])
    with pytest.raises(arc.ArcError) as e:
        run_gpu_trace(arc, ctx, w, schedule="batched", spill_cap=-1)
    assert e.value.status == -1
    with pytest.raises(arc.ArcError) as e:
        run_gpu_trace(arc, ctx, w, schedule="batched", tune_stack=96)
    assert e.value.status == -1


@pytest.mark.parametrize("delta", [0, 1, 3, 5, 6])
def test_every_work_item_level_equals_plain_bitwise(arc, ctx, delta):
    """The persistent launch's work items are the first level's rays (delta 0) or the family
    records the level-synchronous stage leaves (four rays each): every item level gives the
    plain schedule's field, rays and crossings."""
    w = W.lognormal(40, 12, 22)
    p = run_gpu_trace(arc, ctx, w, schedule="plain")
    b = run_gpu_trace(arc, ctx, w, schedule="batched", tune_item_level=w.trace["level0"] + delta)
    assert np.array_equal(b["J"], p["J"])
    assert b["ledger"]["rays"] == p["ledger"]["rays"]
    assert b["ledger"]["crossings"] == p["ledger"]["crossings"]


@pytest.mark.parametrize("delta", [1, 3])
def test_family_work_items_with_the_correction_equal_plain_bitwise(arc, ctx, delta):
    """The family records between the two stages, in the geometric correction's kernels: the
    field and both limbs of the moved-photon field as the plain schedule's."""
    w = W.lognormal(40, 12, 23)
    p = run_gpu_trace(arc, ctx, w, schedule="plain", correction="conserving")
    b = run_gpu_trace(arc, ctx, w, schedule="batched", correction="conserving",
                      tune_item_level=w.trace["level0"] + delta)
    for k in ("J", "moved_lo", "moved_hi"):
        assert np.array_equal(b[k], p[k]), k
    assert b["ledger"]["rays"] == p["ledger"]["rays"]


@pytest.mark.parametrize("delta", [1, 3])
def test_family_work_items_with_thin_spheres_equal_plain_bitwise(arc, ctx, delta):
    """The family records between the two stages, in the thin-sphere kernels: rays of sources
    whose thin radius lies beyond a level's split radius split at once."""
    w = W.lognormal(40, 6, 24, source_cells="uniform")
    w.sources["r_thin"] = np.array([0.0, 0.4, 1.5, 3.0, 6.0, 12.0])
    p = run_gpu_trace(arc, ctx, w, schedule="plain")
    b = run_gpu_trace(arc, ctx, w, schedule="batched", tune_item_level=w.trace["level0"] + delta)
    assert np.array_equal(b["J"], p["J"])
    assert b["ledger"]["rays"] == p["ledger"]["rays"]
    assert b["ledger"]["crossings"] == p["ledger"]["crossings"]
