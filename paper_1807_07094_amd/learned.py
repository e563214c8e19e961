"""Training samples for the learned chemistry step.

Samples are cell states met in real runs: a few trace + chemistry steps of the He
workloads are run through the library, cells are drawn from the traced grids (half
uniformly, half among cells that receive radiation), each with a time step drawn
log-uniformly, and the plain solver of the library gives the targets. Only sampling
choices live here; tracing and the chemistry run in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import workload as W

N_DT = 32  # time steps are drawn from this many log-spaced values


def sample_states(ctx, arc_mod, w: W.Workload, n: int, seed: int, steps: int = 3,
                  dt_range_myr=(1e-3, 10.0)):
    """Draw n (inputs, targets) pairs from the states of workload w over `steps` RT steps.

    Returns device tensors X [n, 8] = (n_H, x_HI, T, Gamma_HI, dt, h, x_HeII, x_HeI), with h
    the photoheating per H atom, and Y [n, 2] = (x_HI', T')."""
    import torch

    rng = np.random.Generator(np.random.Philox(key=int(seed) | (7 << 64)))
    g = arc_mod.device_grid(w.grid)
    shape = w.shape
    ncell = int(np.prod(shape))
    gamma = torch.empty((3,) + shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    per_step = n // steps
    xs, ys = [], []
    dts = np.logspace(np.log10(dt_range_myr[0]), np.log10(dt_range_myr[1]), N_DT) * W.MYR_S
    for step in range(steps):
        m = per_step if step < steps - 1 else n - per_step * (steps - 1)
        ctx.trace(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                  rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"])
        lit = torch.nonzero(gamma[0].reshape(-1) > 1e-6 * float(gamma[0].max())).flatten().cpu().numpy()
        half = m // 2
        cells = np.concatenate([rng.integers(0, ncell, m - half),
                                lit[rng.integers(0, max(1, lit.size), half)] if lit.size else
                                rng.integers(0, ncell, half)])
        which = rng.integers(0, N_DT, m)
        cells_t = torch.from_numpy(cells).cuda()
        flat = {k: g[k].reshape(-1)[cells_t] for k in ("n_h", "x_hi", "x_hei", "x_heii", "temp")}
        gam = gamma.reshape(3, -1)[:, cells_t].contiguous()
        hea = heat.reshape(3, -1)[:, cells_t].contiguous()
        out = {k: flat[k].clone() for k in ("x_hi", "x_hei", "x_heii", "temp")}
        for j in range(N_DT):
            sel = np.flatnonzero(which == j)
            if sel.size == 0:
                continue
            # the selected cells as a grid of rows of at most 1024 (padded with copies of
            # the last cell; the padding is dropped afterwards)
            rows = -(-sel.size // 1024)
            width = min(1024, sel.size)
            pad = np.concatenate([sel, np.full(rows * width - sel.size, sel[-1])])
            sel_t = torch.from_numpy(pad).cuda()
            sub = {"n_h": flat["n_h"][sel_t].contiguous().reshape(1, rows, width), "cell_cm": w.grid["cell_cm"],
                   "y_he": w.grid["y_he"]}
            for k in ("x_hi", "x_hei", "x_heii", "temp"):
                sub[k] = flat[k][sel_t].contiguous().reshape(1, rows, width)
            ctx.chem_step(sub, gam[:, sel_t].contiguous(), hea[:, sel_t].contiguous(), float(dts[j]), **w.chem)
            keep = torch.from_numpy(sel).cuda()
            for k in ("x_hi", "x_hei", "x_heii", "temp"):
                out[k][keep] = sub[k].reshape(-1)[: sel.size]
        dt_col = torch.from_numpy(dts[which].astype(np.float32)).cuda()
        y = float(w.grid["y_he"])
        h = hea[0] * flat["x_hi"] + y * (hea[1] * flat["x_hei"] + hea[2] * flat["x_heii"])
        xs.append(torch.stack([flat["n_h"], flat["x_hi"], flat["temp"], gam[0], dt_col, h, flat["x_heii"],
                               flat["x_hei"]], dim=1))
        ys.append(torch.stack([out["x_hi"], out["temp"]], dim=1))
        # advance the run itself by one RT step so that later samples see evolved states
        ctx.chem_step(g, gamma, heat, w.dt, **w.chem)
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def training_set(ctx, arc_mod, n: int = 1_000_000, seed: int = 11, sizes=(64, 96), n_src=(64, 128)):
    """Samples from lognormal He workloads of the given sizes (the shapes of the benchmark
    configurations at a scale that generates quickly)."""
    import torch

    X, Y = [], []
    for i, (size, ns) in enumerate(zip(sizes, n_src)):
        w = W.lognormal(size, ns, seed + i)
        x, y = sample_states(ctx, arc_mod, w, n // len(sizes), seed + 100 + i)
        X.append(x)
        Y.append(y)
    return torch.cat(X).contiguous(), torch.cat(Y).contiguous()
