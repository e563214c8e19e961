"""Learned chemistry step (BF16 network on the matrix cores, gated, plain-solver fallback).

* the MFMA forward pass equals a NumPy forward pass of the same BF16 weights;
* a gate that accepts nothing reproduces the plain solver bitwise;
* with the gate on, every accepted cell stays within the tolerance of the plain solver
  (the plain solver is the judge; it is itself parity-checked against the oracle);
* the gated step judged by the FP64 oracle's chemistry directly: from the same state and
  the same rates (the oracle's own, rounded to FP32), every cell's fractions within 1e-3
  and temperature within 1e-2 relative, accepted cells and fallback cells alike;
* save / load round trip.
"""
import struct

import numpy as np
import pytest

from paper_1807_07094_amd import learned
from paper_1807_07094_amd import workload as W

pytestmark = pytest.mark.gpu

HID, K1, OUTP, NIN = 64, 32, 16, 8


@pytest.fixture(scope="module")
def ctx(arc):
    c = arc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def trained(arc, ctx):
    X, Y = learned.training_set(ctx, arc, n=400_000, seed=5, sizes=(48, 64), n_src=(32, 48))
    net = arc.MLP(ctx)
    rep = net.train(X, Y, epochs=10, batch=1024, lr=2e-3, seed=3)
    return net, rep, X, Y


def bf16_to_f32(u16: np.ndarray) -> np.ndarray:
    return (u16.astype(np.uint32) << 16).view(np.float32)


def f32_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round to nearest even BF16, returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return bf16_to_f32(u.astype(np.uint16))


def parse_model(blob: bytes):
    """Fields of the saved network: standardisation, biases and the BF16 weight images."""
    off = 16  # magic, version, nparams, pad
    f = lambda n: (np.frombuffer(blob, np.float32, n, off), n * 4)
    out = {}
    for name, n in (("in_mu", NIN), ("in_sd", NIN), ("lo", NIN), ("hi", NIN), ("out_mu", 2), ("out_sd", 2),
                    ("base_y", 1), ("base_coll", 1), ("b1", HID), ("b2", HID), ("b3", 2)):
        a, nb = f(n)
        out[name] = a.copy()
        off += nb
    out["base_coll"] = out["base_coll"].view(np.int32)
    for name, shape in (("w1t", (HID, K1)), ("w2t", (HID, HID)), ("w3t", (OUTP, HID))):
        n = shape[0] * shape[1]
        out[name] = bf16_to_f32(np.frombuffer(blob, np.uint16, n, off)).reshape(shape)
        off += 2 * n
    return out


def x_baseline(m, X):
    """The network's x_HI baseline in FP32: exact relaxation with the start-of-step recombination
    (case-B fit), collisional and photoionisation rates (Hui & Gnedin 1997 fits)."""
    f32 = np.float32
    nh, x, T, gam, dt, xheii, xhei = (X[:, i].astype(f32) for i in (0, 1, 2, 3, 4, 6, 7))
    lhi = f32(2.0 * 157807.0) / T
    a_hii = f32(2.753e-14) * lhi ** f32(1.5) / (f32(1) + (lhi / f32(2.740)) ** f32(0.407)) ** f32(2.242)
    k_hi = (f32(21.11) * T ** f32(-1.5) * np.exp(-lhi / f32(2)) * lhi ** f32(-1.089)
            / (f32(1) + (lhi / f32(0.354)) ** f32(0.874)) ** f32(1.101))
    y = m["base_y"][0]
    ne = nh * ((f32(1) - x) + y * (xheii + f32(2) * np.maximum(f32(0), f32(1) - xhei - xheii)))
    a = a_hii * ne
    b = gam + (k_hi * ne if m["base_coll"][0] else f32(0))
    lam = a + b
    with np.errstate(divide="ignore", invalid="ignore"):
        xeq = a / lam
        xb = xeq + (x - xeq) * np.exp(-lam * dt)
    return np.where(lam > 0, xb, x).astype(f32)


def reference_forward(m, X):
    """NumPy forward pass in the network's arithmetic: BF16 inputs, weights and hidden
    activations (ReLU), FP32 sums; outputs are corrections of the x_HI baseline and the change
    of log10 T. Returns (x_HI', log10 T')."""
    f = np.stack([np.log10(X[:, 0]), X[:, 1], np.log10(X[:, 2]), np.log10(np.maximum(X[:, 3], 1e-30)),
                  np.log10(X[:, 4]), np.log10(np.maximum(X[:, 5], 1e-35)), X[:, 6], X[:, 7]],
                 axis=1).astype(np.float32)
    x = f32_to_bf16((f - m["in_mu"]) / m["in_sd"])
    h1 = f32_to_bf16(np.maximum(x @ m["w1t"][:, :NIN].T + m["b1"], 0.0))
    h2 = f32_to_bf16(np.maximum(h1 @ m["w2t"].T + m["b2"], 0.0))
    o = h2 @ m["w3t"][:2].T + m["b3"]
    x_new = np.clip(x_baseline(m, X) + (o[:, 0] * m["out_sd"][0] + m["out_mu"][0]), 0.0, 1.0)
    return x_new, np.log10(X[:, 2]) + (o[:, 1] * m["out_sd"][1] + m["out_mu"][1])


def test_training_report(trained):
    net, rep, X, Y = trained
    assert rep["n_train"] + rep["n_val"] == X.shape[0]
    assert rep["val_rmse_x"] < 0.05
    assert rep["val_rmse_logt"] < 0.05
    assert rep["bins_used"] > 50


def test_mfma_forward_matches_numpy(arc, ctx, trained):
    import torch

    net, _, X, _ = trained
    m = parse_model(net.save())
    Xs = X[:: max(1, X.shape[0] // 4000)].contiguous()
    P = torch.empty((Xs.shape[0], 2), dtype=torch.float32, device="cuda")
    net.predict(Xs, P)
    got = P.cpu().numpy()
    x_ref, lt_ref = reference_forward(m, Xs.cpu().numpy().astype(np.float32))
    assert np.max(np.abs(got[:, 0] - x_ref)) < 3e-3
    assert np.max(np.abs(np.log10(got[:, 1]) - lt_ref)) < 3e-3
    # a wrong lane layout gives errors of order one, not of order the BF16 rounding
    assert np.median(np.abs(got[:, 0] - x_ref)) < 2e-4


def chem_copies(arc, ctx, w):
    import torch

    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    ctx.trace(g, w.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"], eps_term=w.trace["eps_term"])
    copy = lambda: {k: (v.clone() if hasattr(v, "clone") else v) for k, v in g.items()}
    return copy, gamma, heat


def test_closed_gate_equals_plain_bitwise(arc, ctx, trained):
    net = trained[0]
    w = W.lognormal(40, 16, 77)
    copy, gamma, heat = chem_copies(arc, ctx, w)
    a, b = copy(), copy()
    ctx.chem_step(a, gamma, heat, w.dt, **w.chem)
    st = ctx.chem_step(b, gamma, heat, w.dt, mode="mlp_gated", mlp=net, gate_tol=1.0, gate_min_count=2 ** 30,
                       **w.chem)
    assert st["fallback"] == a["x_hi"].numel()
    for k in ("x_hi", "x_hei", "x_heii", "temp"):
        assert bool((a[k] == b[k]).all()), k


def test_gated_step_within_tolerance_of_plain(arc, ctx, trained):
    net = trained[0]
    w = W.lognormal(48, 32, 78)
    copy, gamma, heat = chem_copies(arc, ctx, w)
    plain, gated = copy(), copy()
    ctx.chem_step(plain, gamma, heat, w.dt, **w.chem)
    st = ctx.chem_step(gated, gamma, heat, w.dt, mode="mlp_gated", mlp=net, gate_tol=1e-3, **w.chem)
    accepted = st["cells"] - st["fallback"]
    assert accepted > 0
    dx = (gated["x_hi"] - plain["x_hi"]).abs()
    dt = ((gated["temp"] - plain["temp"]) / plain["temp"]).abs()
    # judge run: the plain solver on every cell; the accepted cells stay within the gate
    # (fractions to gate_tol absolute, temperature to 10 gate_tol relative)
    assert float(dx.max()) <= 1e-3
    assert float(dt.max()) <= 1e-2
    # helium is untouched by the network and equal to the plain solver where it fell back
    assert float((gated["x_heii"] - plain["x_heii"]).abs().max()) <= 1e-3


def test_gated_step_judged_by_the_oracle(arc, ctx, trained):
    import torch

    import oracle

    net = trained[0]
    w = W.lognormal(48, 32, 79)
    # rates from the oracle's trace of the grid as generated, rounded to FP32 for both sides
    r = oracle.trace(w.grid, w.sources, w.bins, w.trace)
    og, oh, _ = oracle.finalize(w.grid, w.bins, r["J"])
    g32, h32 = og.astype(np.float32), oh.astype(np.float32)
    g = arc.device_grid(w.grid)
    gamma = torch.from_numpy(g32).cuda()
    heat = torch.from_numpy(h32).cuda()
    st = ctx.chem_step(g, gamma, heat, w.dt, mode="mlp_gated", mlp=net, gate_tol=1e-3, **w.chem)
    accepted = st["cells"] - st["fallback"]
    print(f"[mlp judge] accepted {accepted} of {st['cells']} cells", flush=True)
    assert accepted > 0
    ref = oracle.chem(w.grid, w.state(), g32.astype(np.float64), h32.astype(np.float64), w.dt, w.chem)
    for k in ("x_hi", "x_hei", "x_heii"):
        err = float(np.abs(g[k].cpu().numpy() - ref[k]).max())
        assert err <= 1e-3, (k, err)
    t_err = float(np.abs(g["temp"].cpu().numpy() / ref["temp"] - 1).max())
    assert t_err <= 1e-2, t_err


def test_save_load_round_trip(arc, ctx, trained):
    import torch

    net, _, X, _ = trained
    blob = net.save()
    other = arc.MLP(ctx)
    other.load(blob)
    Xs = X[:2048].contiguous()
    P1 = torch.empty((Xs.shape[0], 2), device="cuda")
    P2 = torch.empty_like(P1)
    net.predict(Xs, P1)
    other.predict(Xs, P2)
    assert bool((P1 == P2).all())
    with pytest.raises(arc.ArcError):
        other.load(blob[:100])
    other.close()


def test_mlp_modes_need_a_network(arc, ctx):
    import torch

    w = W.lognormal(8, 2, 3)
    g = arc.device_grid(w.grid)
    gamma = torch.zeros((3,) + w.shape, device="cuda")
    heat = torch.zeros_like(gamma)
    untrained = arc.MLP(ctx)
    with pytest.raises(arc.ArcError):
        ctx.chem_step(g, gamma, heat, w.dt, mode="mlp_gated", mlp=untrained, **w.chem)
    untrained.close()
