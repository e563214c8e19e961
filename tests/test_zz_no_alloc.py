"""The allocation-free time-step entry point (arc_rt_timestep_noalloc) against arc_rt_timestep
on the same inputs: the same minima bit for bit (the same kernels, min-reductions in any
order), on two calls in a row, the second on a smaller grid, with other GPU work between."""
import numpy as np
import pytest

from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu


def _state(arc, w, seed):
    import torch

    g = arc.device_grid(w.grid)
    rng = np.random.default_rng(seed)
    gamma = torch.from_numpy(
        np.ascontiguousarray(10.0 ** rng.uniform(-16, -11, (3,) + w.shape)).astype(np.float32)).cuda()
    return g, gamma


def test_noalloc_timestep_equals_the_allocating_entry_point(arc):
    import torch

    ctx = arc.Context(0)
    try:
        for n, seed in ((40, 3), (24, 5)):
            w = W.lognormal(n, 2, seed)
            g, gamma = _state(arc, w, seed)
            print(f"[noalloc] grid {w.shape}", flush=True)
            ref = ctx.rt_timestep(g, gamma, w.bins, eps=0.1)
            out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
            ctx.rt_timestep_noalloc(g, gamma, w.bins, out, eps=0.1)
            torch.cuda.synchronize()
            got = tuple(float(v) for v in out.cpu())
            assert np.isfinite(ref[0]) and np.isfinite(ref[1])
            assert got == ref, (got, ref)
            # other work between the calls, then the same call again: the array starts afresh
            a = torch.randn(512, 512, device="cuda")
            float((a @ a).sum())
            out.fill_(-1.0)
            ctx.rt_timestep_noalloc(g, gamma, w.bins, out, eps=0.1)
            torch.cuda.synchronize()
            assert tuple(float(v) for v in out.cpu()) == ref
    finally:
        ctx.close()


def test_noalloc_timestep_argument_checks(arc):
    import torch

    ctx = arc.Context(0)
    try:
        w = W.lognormal(16, 1, 7)
        g, gamma = _state(arc, w, 7)
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        with pytest.raises(arc.ArcError) as e:
            ctx.rt_timestep_noalloc(g, gamma, w.bins, out, eps=0.0)
        assert e.value.status == -2
        with pytest.raises(ValueError):
            ctx.rt_timestep_noalloc(g, gamma, w.bins, torch.zeros(2, dtype=torch.float32, device="cuda"))
    finally:
        ctx.close()
