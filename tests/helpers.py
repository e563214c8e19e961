"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on the same
seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

import oracle

GAMMA_REL_TOL = 1e-4      # per-cell rate, relative, where rate > 1e-6 * max
GAMMA_FLOOR = 1e-6
CONSERVATION_TOL = 1e-6   # GPU photon ledger
FRACTION_TOL = 1e-3       # ionised fractions after the chemistry step, absolute


def run_gpu_trace(arc_mod, ctx, w, schedule="batched", precision="fp32_comp", tree_cap=0, eps_term=None,
                  max_level=None, **kw):
    import torch

    g = arc_mod.device_grid(w.grid)
    shape = (3,) + w.shape
    gamma = torch.empty(shape, dtype=torch.float32, device="cuda")
    heat = torch.empty(shape, dtype=torch.float32, device="cuda")
    tree = torch.zeros(tree_cap, dtype=torch.int64, device="cuda") if tree_cap else None
    led = ctx.trace(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                    rays_per_cell=w.trace["rays_per_cell"],
                    max_level=w.trace["max_level"] if max_level is None else max_level,
                    eps_term=w.trace["eps_term"] if eps_term is None else eps_term, precision=precision,
                    schedule=schedule, tree=tree, **kw)
    nb = len(w.bins["frac"])
    # with the conserving correction the moved-photon field's two limbs follow the field
    parts = 3 if kw.get("correction") in ("conserving", 2) else 1
    J = torch.empty((parts, nb) + w.shape, dtype=torch.int64, device="cuda")
    ctx.get_field(J)
    Jh = J.cpu().numpy()
    out = {"gamma": gamma.cpu().numpy(), "heat": heat.cpu().numpy(), "J": Jh[0], "ledger": led}
    if parts == 3:
        out["moved_lo"], out["moved_hi"] = Jh[1], Jh[2]
    if tree is not None:
        n = min(led["tree_count"], tree_cap)
        out["tree"] = np.sort(tree[:n].cpu().numpy().view(np.uint64))
    return out


def run_oracle(w, tree_cap=0, eps_term=None, max_level=None):
    params = dict(w.trace)
    if eps_term is not None:
        params["eps_term"] = eps_term
    if max_level is not None:
        params["max_level"] = max_level
    r = oracle.trace(w.grid, w.sources, w.bins, params, tree_cap=tree_cap)
    gamma, heat, absorbed = oracle.finalize(w.grid, w.bins, r["J"])
    r.update(gamma=gamma, heat=heat, absorbed=absorbed)
    if tree_cap:
        r["tree"] = np.sort(r["tree"])
    return r


def rate_errors(gpu, ora, key="gamma"):
    """Max relative error per species over cells above 1e-6 of that species' maximum. A cell
    below that floor in the oracle must stay below twice the floor on the GPU (a spurious
    deposit there would otherwise go unseen); if one does not, the species' error is inf."""
    errs = []
    for sp in range(3):
        ref = ora[key][sp]
        got = gpu[key][sp]
        top = ref.max()
        if top <= 0:
            errs.append(0.0 if np.abs(got).max() == 0 else np.inf)
            continue
        m = ref > GAMMA_FLOOR * top
        if np.any(np.abs(got[~m]) > 2.0 * GAMMA_FLOOR * top):
            errs.append(np.inf)
            continue
        errs.append(float(np.max(np.abs(got[m] / ref[m] - 1.0))))
    return errs


def conservation(led):
    return abs(led["emitted"] - led["absorbed"] - led["escaped"]) / led["emitted"]
