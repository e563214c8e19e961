"""Benchmark: cell crossings per second of one full radiative-transfer step (trace +
chemistry) on one MI355X, with the batched FP32 tracer.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4]

Prints one JSON line. Default workload: the 1024^3 Gaussian-random-field grid with
16384 sources (H + He, three bands); smaller configurations with --config 0..3.
The CPU baseline is the FP64 oracle timed on a bounded sample of the same workload
(a subset of the sources on the full grid).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Counters of the trace kernel on this workload (rocprofv3, one launch from the generated state):
# HBM bytes per crossing from FETCH_SIZE (x2.0, calibrated on a copy) and WRITE_SIZE (x1.0), VALU
# wave-instructions per crossing (SQ_INSTS_VALU) and the L2 hit rate (TCC_HIT_sum, TCC_MISS_sum).
# Valid for the kernel sources with these digests; with any other sources they are stale and
# reported as null.
MEASURED_COUNTERS = {
    "bytes_per_crossing": 15.47,
    "valu_per_crossing": 5.924,
    "l2_hit_rate": 0.0803,
    "sha256": {
        "paper_1807_07094_amd/csrc/arc_device.h": "e391af014143268c460e533da8fb189835cb8300db2c07f183a9defa19897767",
        "paper_1807_07094_amd/csrc/arc_kernels.hip": "25d63b65c69587935ee0fbd9f93d932980bec682d193fdaac6f984ae9fbc878e",
    },
    "profile": "profiles/hbm_l2_sq_k_trace_persistent_grf1024_16384src.md",
}
# VALU issue of the whole chip: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every four
# cycles (16 lanes wide), at 2.4 GHz: 6.14e11 wave-instructions per second.
VALU_PEAK_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def measured_counters():
    """The profiled counter figures if the kernel sources are the profiled ones, else None."""
    import hashlib

    for rel, digest in MEASURED_COUNTERS["sha256"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return MEASURED_COUNTERS


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def field_checksum(ctx, buf):
    """Two 64-bit sums of the last trace's fixed-point field (sum J_i and sum J_i (2i + 1), mod
    2^64) read with arc_get_field into the device int64 buffer `buf`: equal fields give equal
    sums bit for bit."""
    import torch

    ctx.get_field(buf)
    flat = buf.view(-1)
    s0 = torch.zeros((), dtype=torch.int64, device=flat.device)
    s1 = torch.zeros((), dtype=torch.int64, device=flat.device)
    chunk = 1 << 27
    for i0 in range(0, flat.numel(), chunk):
        part = flat[i0:i0 + chunk]
        w = torch.arange(i0, i0 + part.numel(), dtype=torch.int64, device=flat.device) * 2 + 1
        s0 += part.sum()
        s1 += (part * w).sum()
    return int(s0), int(s1)


def measure_ceilings(ctx):
    """Random-request ceilings of the device on the trace's own buffers (the library's probe:
    deposits, each an int64 atomic add to the bins of a random cell issued by adjacent lanes
    as the trace issues them, and 16-byte opacity gathers of random cells), and the device
    copy bandwidth (torch copy_ of 4 GiB, timed with events)."""
    import torch

    items = 1 << 27
    dep, gat = ctx.probe_requests(items=items, seed=12345)
    out = {"deposits_per_s": dep, "gathers_per_s": gat,
           "method": f"arc_probe_requests: {items} random cells of the last trace's buffers, best of 3"}
    # the same requests confined to 2^16 cells (2 MB of field, 1 MB of opacity: cache-resident)
    dep_s, gat_s = ctx.probe_requests(items=items, cells=1 << 16, seed=54321)
    out["cached"] = {"cells": 1 << 16, "deposits_per_s": dep_s, "gathers_per_s": gat_s}
    n = 1 << 30
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    best = float("inf")
    for _ in range(3):
        ev0.record()
        b.copy_(a)
        ev1.record()
        ev1.synchronize()
        best = min(best, ev0.elapsed_time(ev1) * 1e-3)
    out["copy_gbs"] = 2 * 4 * n / best / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4, help="benchmark configuration 0..4 (4 = 1024^3, 16384 sources)")
    ap.add_argument("--schedule", default="batched", choices=["batched", "plain"])
    ap.add_argument("--precision", default="fp32_comp", choices=["fp32_comp", "fp32_plain"])
    ap.add_argument("--chem", default=None, choices=["mlp_gated", "plain", "none"],
                    help="chemistry of the step: learned step with the plain fallback, plain solver, or none "
                         "(default: the learned step for configurations 3 and 4, the plain solver otherwise)")
    ap.add_argument("--mlp-samples", type=int, default=1_000_000, help="training samples of the learned step")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--gate-tol", type=float, default=1e-3, help="gate: largest held-out error of a bin")
    ap.add_argument("--cpu-sample", type=int, default=16, help="sources in the oracle's timed sample (0 = skip)")
    ap.add_argument("--plain-sample", type=int, default=256, help="sources traced by the plain schedule (0 = skip)")
    ap.add_argument("--plain-full", type=int, default=1,
                    help="1: also trace every source with the plain schedule once (bitwise field check, extra)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle's all-core leg (0: OMP_NUM_THREADS, else every core)")
    ap.add_argument("--cpu-sample-mt", type=int, default=64, help="sources in the all-core oracle sample (0 = skip)")
    ap.add_argument("--thin-run", type=int, default=1,
                    help="1: trace an evolved state (ionised bubbles around the sources, volume-filling ionised "
                         "fraction ~0.2) with and without the optically thin approximation (extra)")
    ap.add_argument("--ceilings", type=int, default=1,
                    help="1: measure the random-request ceilings (int64 atomics, 16-byte gathers) at the end")
    ap.add_argument("--correction-run", type=int, default=1,
                    help="1: also trace the workload once with the conserving geometric correction (extra)")
    ap.add_argument("--tune-waves", type=int, default=0)
    ap.add_argument("--tune-blocks", type=int, default=0)
    ap.add_argument("--tune-refill", type=int, default=0)
    ap.add_argument("--tune-item-level", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true",
                    help="default launch shape instead of the autotuned one (tuned before warm-up)")
    ap.add_argument("--graph", type=int, default=1, help="1: replay the trace's recorded HIP graphs")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only copy this many GiB device to device (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.chem is None:
        args.chem = "mlp_gated" if args.config >= 3 else "plain"

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the tracer runs on a single MI355X; sharding the sources over "
              "several GPUs (an integer sum of their fields) is not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1807_07094_amd import arc
    from paper_1807_07094_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_gib > 0:
        n = int(args.copy_gib * 2**30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return
    t0 = time.time()
    w = W.config(args.config, device="cuda")
    log(f"workload {w.name}: {w.shape} cells, {len(w.sources['ndot'])} sources, generated in {time.time() - t0:.1f}s")
    ctx = arc.Context(0)
    g = arc.device_grid(w.grid)
    gamma = torch.empty((3,) + w.shape, dtype=torch.float32, device="cuda")
    heat = torch.empty_like(gamma)
    nb = len(w.bins["frac"])
    tune = dict(tune_waves=args.tune_waves, tune_blocks=args.tune_blocks, tune_refill=args.tune_refill,
                tune_item_level=args.tune_item_level)

    def trace(grid, sources, schedule, **kw):
        return ctx.trace(grid, sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                         rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"],
                         precision=args.precision, schedule=schedule, **kw)

    net, mlp_info = None, None
    if args.chem == "mlp_gated":
        from paper_1807_07094_amd import learned

        tt = time.perf_counter()
        # half from small lognormal runs (broad coverage), half from two steps of this
        # workload itself (on a copy of its grid)
        X1, Y1 = learned.training_set(ctx, arc, n=args.mlp_samples // 2)
        X2, Y2 = learned.sample_states(ctx, arc, w, args.mlp_samples - args.mlp_samples // 2, seed=17, steps=2)
        X, Y = torch.cat([X1, X2]).contiguous(), torch.cat([Y1, Y2]).contiguous()
        del X1, Y1, X2, Y2
        torch.cuda.empty_cache()
        ts = time.perf_counter() - tt
        net = arc.MLP(ctx)
        rep = net.train(X, Y, epochs=args.mlp_epochs, batch=1024, lr=2e-3, seed=3, y_he=w.grid["y_he"],
                        collisional=w.chem.get("collisional", 1))
        del X, Y
        mlp_info = {"samples": args.mlp_samples, "sampling_s": round(ts, 2), "train_ms": round(rep["ms"], 1),
                    "val_rmse_x": rep["val_rmse_x"], "val_rmse_logt": rep["val_rmse_logt"],
                    "bins_used": rep["bins_used"], "gate_tol": args.gate_tol}
        log(f"learned chemistry: {mlp_info}")
    chem_kw = dict(w.chem, graph=bool(args.graph))
    if net is not None:
        chem_kw.update(mode="mlp_gated", mlp=net, gate_tol=args.gate_tol)

    schedule = args.schedule
    tune_info = None
    if not args.no_tune and args.schedule == "batched" and not any(tune.values()):
        nsrc_all = len(w.sources["ndot"])
        sub = w.subset(np.arange(0, nsrc_all, max(1, nsrc_all // 256)))
        tt = time.perf_counter()
        tune_info = ctx.autotune(g, sub.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                                 rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"],
                                 precision=args.precision)
        tune_info["tuning_s"] = round(time.perf_counter() - tt, 2)
        tune_info["tuning_sources"] = len(sub.sources["ndot"])
        log(f"autotuned shape: {tune_info}")
        schedule = "batched_tuned"
        tune = {}
    if schedule != "plain":
        tune["graph"] = bool(args.graph)

    def step():
        led = trace(g, w.sources, schedule, **tune)
        cs = None if args.chem == "none" else ctx.chem_step(g, gamma, heat, w.dt, **chem_kw)
        return led, cs

    for i in range(args.warmup):
        led, cs = step()
        log(f"warmup {i}: crossings={led['crossings']} trace {led['ms_total']:.1f} ms, kernel {led['ms_kernel']:.1f} ms"
            + (f", chem {cs['ms']:.1f} ms" if cs else ""))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    leds, chems = [], []
    for i in range(args.steps):
        led, cs = step()
        leds.append(led)
        chems.append(cs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    crossings = sum(l["crossings"] for l in leds)
    value = crossings / elapsed
    ms_step = 1e3 * elapsed / args.steps
    cons = max(abs(l["emitted"] - l["absorbed"] - l["escaped"]) / l["emitted"] for l in leds)
    for i, (l, c) in enumerate(zip(leds, chems)):
        log(f"step {i}: crossings={l['crossings']} rays={l['rays']} spills={l['spills']} trace {l['ms_total']:.1f} ms "
            f"(kernel {l['ms_kernel']:.1f} ms)" + (f", chem {c['ms']:.1f} ms, substeps {c['sub_total']}" if c else ""))

    # Roofline of the dominant kernel (the persistent trace kernel): algorithmic bytes per
    # crossing = per bin one 4-byte opacity read and one 8-byte read + 8-byte write of the
    # fixed-point field; the crossings are the launch's own (the ledger's count minus those of
    # the levels traced before it).
    bpc = 20 * nb
    batched = args.schedule == "batched"
    kms = float(np.mean([l["ms_kernel"] for l in leds])) if batched else float(
        np.mean([l["ms_trace"] for l in leds]))
    per_launch = float(np.mean([l["kernel_crossings"] if batched else l["crossings"] for l in leds]))
    deposits_per_launch = float(np.mean([l["kernel_deposits"] if batched else l["deposits"] for l in leds]))
    achieved = per_launch * bpc / (kms * 1e-3) / 1e9
    mc = measured_counters() if args.config == 4 and args.schedule == "batched" and args.precision == "fp32_comp" \
        else None
    tpc = mc["bytes_per_crossing"] if mc else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(tpc * per_launch) if tpc is not None else None,
                "traffic_unit": "bytes per launch", "traffic_bytes_per_crossing": tpc,
                "kernel": "k_trace_persistent" if args.schedule == "batched" else "k_trace_rays",
                "kernel_ms": round(kms, 3), "bytes_per_crossing": bpc}
    if mc:
        # what the counters say limits the kernel: the HBM traffic it really moves, and its VALU
        # issue against the chip's (profiled instructions per crossing at this launch's rate)
        valu_rate = mc["valu_per_crossing"] * per_launch / (kms * 1e-3)
        roofline["counters"] = {
            "hbm_traffic_gbs": round(tpc * per_launch / (kms * 1e-3) / 1e9, 1),
            "hbm_traffic_frac": round(tpc * per_launch / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "valu_wave_instr_per_crossing": mc["valu_per_crossing"],
            "valu_issue_frac": round(valu_rate / VALU_PEAK_WAVE_INSTR_PER_S, 4),
            "l2_hit_rate": mc["l2_hit_rate"], "profile": mc["profile"]}

    crossings_step = float(np.mean([l["crossings"] for l in leds]))
    extra = {"trace_crossings_per_s": round(crossings_step / (float(np.mean([l["ms_total"] for l in leds])) * 1e-3), 1),
             "kernel_crossings_per_s": round(per_launch / (kms * 1e-3), 1),
             "conservation": cons, "crossings_per_step": crossings_step, "kernel_crossings_per_launch": per_launch,
             "kernel_deposits_per_launch": deposits_per_launch,
             "deposits_per_crossing": round(deposits_per_launch / max(per_launch, 1.0), 4)}
    if tune_info is not None:
        extra["autotune"] = tune_info
    if chems[0] is not None:
        extra["chem_ms"] = round(float(np.mean([c["ms"] for c in chems])), 2)
    if net is not None:
        # the plain solver judges the learned step: both from the same state and rates
        fields = ("x_hi", "x_hei", "x_heii", "temp")
        keep = {k: g[k].clone() for k in fields}
        cg = ctx.chem_step(g, gamma, heat, w.dt, **chem_kw)
        got = {k: g[k].clone() for k in fields}
        for k in fields:
            g[k].copy_(keep[k])
        cp = ctx.chem_step(g, gamma, heat, w.dt, **w.chem)
        dx = float((got["x_hi"] - g["x_hi"]).abs().max())
        dT = float(((got["temp"] - g["temp"]) / g["temp"]).abs().max())
        mlp_info.update(accepted_frac=round(1.0 - cg["fallback"] / cg["cells"], 4), max_abs_dx_hi=dx,
                        max_rel_dT=dT, ms_gated=round(cg["ms"], 2), ms_mlp=round(cg["ms_mlp"], 2),
                        ms_plain=round(cp["ms"], 2))
        del keep, got
        extra["learned_chem"] = mlp_info
        log(f"learned chemistry vs plain: {mlp_info}")

    # Plain (per source, per level) schedule on a source subset: crossings/s of the paper's loop.
    nsrc = len(w.sources["ndot"])
    if args.plain_sample and args.schedule == "batched":
        idx = np.arange(0, nsrc, max(1, nsrc // args.plain_sample))[: args.plain_sample]
        sub = w.subset(idx)
        lb = trace(g, sub.sources, schedule, **tune)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        lp = trace(g, sub.sources, "plain")
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        tb = time.perf_counter()
        lb = trace(g, sub.sources, schedule, **tune)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb
        extra["plain_sample"] = {"sources": int(idx.size), "plain_crossings_per_s": round(lp["crossings"] / tp, 1),
                                 "batched_crossings_per_s": round(lb["crossings"] / tb, 1),
                                 "batched_over_plain": round(tp / tb, 2), "same_crossings": lp["crossings"] == lb["crossings"]}
        log(f"plain sample: {extra['plain_sample']}")

    # Plain schedule over every source: the paper's loop on the whole workload, with the
    # fixed-point field checked against the batched schedule's bit for bit.
    if args.plain_full and args.schedule == "batched":
        ncell = int(np.prod(w.shape))
        buf = torch.empty(nb * ncell, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        tb = time.perf_counter()
        lb = trace(g, w.sources, schedule, **tune)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb
        sum_b = field_checksum(ctx, buf)
        tp = time.perf_counter()
        lp = trace(g, w.sources, "plain")
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        sum_p = field_checksum(ctx, buf)
        del buf
        torch.cuda.empty_cache()
        extra["plain_full"] = {"sources": nsrc, "crossings": lp["crossings"],
                               "plain_crossings_per_s": round(lp["crossings"] / tp, 1),
                               "batched_crossings_per_s": round(lb["crossings"] / tb, 1),
                               "plain_s": round(tp, 3), "batched_s": round(tb, 3),
                               "batched_over_plain": round(tp / tb, 2),
                               "same_crossings": lp["crossings"] == lb["crossings"],
                               "field_bitwise_equal": sum_b == sum_p}
        log(f"plain schedule, all sources: {extra['plain_full']}")

    # The adaptive RT time step (section 2.9) on the state and rates the timed steps left.
    if args.chem != "none":
        t0 = time.perf_counter()
        dt_n, dt_i = ctx.rt_timestep(g, gamma, w.bins, eps=0.1, rates=w.chem.get("rates", 1),
                                     collisional=w.chem.get("collisional", 1),
                                     alpha_hii=w.chem.get("alpha_hii", 2.59e-13))
        extra["rt_timestep"] = {"eps": 0.1, "dt_n_myr": dt_n / W.MYR_S, "dt_i_myr": dt_i / W.MYR_S,
                                "ms": round(1e3 * (time.perf_counter() - t0), 2)}
        log(f"adaptive time step: {extra['rt_timestep']}")

    # The geometric correction (section 2.5, f_c with the conserving secondary deposit) on
    # the whole workload: one untimed and one timed trace, next to the uncorrected kernel.
    if args.correction_run and args.schedule == "batched" and args.precision == "fp32_comp":
        trace(g, w.sources, schedule, correction="conserving", **tune)
        lc = trace(g, w.sources, schedule, correction="conserving", **tune)
        extra["correction"] = {"mode": "conserving", "kernel_ms": round(lc["ms_kernel"], 1),
                               "trace_ms": round(lc["ms_total"], 1), "crossings": lc["crossings"],
                               "kernel_crossings_per_s": round(lc["crossings"] / (lc["ms_kernel"] * 1e-3), 1),
                               "over_uncorrected_kernel": round(lc["ms_kernel"] / kms, 3),
                               "conservation": abs(lc["emitted"] - lc["absorbed"] - lc["escaped"]) / lc["emitted"]}
        log(f"geometric correction: {extra['correction']}")

    cpu = None
    if args.cpu_sample:
        import oracle

        idx = np.arange(0, nsrc, max(1, nsrc // args.cpu_sample))[: args.cpu_sample]
        sub = w.subset(idx)
        # the oracle takes the workload as generated (nothing the library computed); the
        # device grid, evolved by the chemistry steps above, goes back to that state for the
        # GPU side of the sample
        state = w.grid
        for k in ("x_hi", "x_hei", "x_heii", "temp"):
            g[k].copy_(torch.from_numpy(np.ascontiguousarray(w.grid[k], np.float32)))
        log(f"oracle sample: {idx.size} sources on the full {w.shape} grid")
        tc = time.perf_counter()
        r = oracle.trace(state, sub.sources, w.bins, w.trace)
        tc = time.perf_counter() - tc
        cpu = {"value": round(r["ledger"]["crossings"] / tc, 1), "unit": "cell-crossings/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{idx.size} of {nsrc} sources (every {max(1, nsrc // args.cpu_sample)}th) on the full grid; "
                         f"{r['ledger']['crossings']} crossings in {tc:.1f}s including the FP64 opacity pass"}
        if args.cpu_sample_mt:
            # the same oracle on every host core: sources spread over threads, one shared field
            threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
            idx_mt = np.arange(0, nsrc, max(1, nsrc // args.cpu_sample_mt))[: args.cpu_sample_mt]
            sub_mt = w.subset(idx_mt)
            log(f"oracle all-core sample: {idx_mt.size} sources on {threads} threads")
            tm = time.perf_counter()
            rm = oracle.trace_mt(state, sub_mt.sources, w.bins, w.trace, threads)
            tm = time.perf_counter() - tm
            single = dict(cpu)
            cpu = {"value": round(rm["ledger"]["crossings"] / tm, 1), "unit": "cell-crossings/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"{idx_mt.size} of {nsrc} sources (every {max(1, nsrc // args.cpu_sample_mt)}th) on the "
                             f"full grid, split over {threads} threads; {rm['ledger']['crossings']} crossings in "
                             f"{tm:.1f}s including the FP64 opacity pass",
                   "single_core": {k: single[k] for k in ("value", "sample")},
                   "host_cpu": host_cpu_model()}
            del rm
        # the same sample on the GPU, checked against the oracle, in both traversal precisions
        og, oh, _ = oracle.finalize(state, w.bins, r["J"])

        def sample_error(precision):
            led = ctx.trace(g, sub.sources, w.bins, w.dt, gamma, heat, level0=w.trace["level0"],
                            rays_per_cell=w.trace["rays_per_cell"], eps_term=w.trace["eps_term"],
                            precision=precision, schedule="batched")
            gg = gamma.cpu().numpy()
            errs = []
            for sp in range(3):
                m = og[sp] > 1e-6 * og[sp].max()
                errs.append(float(np.max(np.abs(gg[sp][m] / og[sp][m] - 1))) if m.any() else 0.0)
            return max(errs), led["crossings"]

        e_comp, x_comp = sample_error("fp32_comp")
        e_plain, x_plain = sample_error("fp32_plain")
        extra["sample_parity"] = {"max_gamma_rel_err": e_comp, "max_gamma_rel_err_fp32_plain": e_plain,
                                  "crossings_gpu": x_comp, "crossings_gpu_fp32_plain": x_plain,
                                  "crossings_oracle": r["ledger"]["crossings"]}
        log(f"sample parity: {extra['sample_parity']}")

        if net is not None:
            # the learned step judged by the FP64 oracle's chemistry: both sides from the grid as
            # generated and the oracle's rates of the sample (rounded to FP32 for both), compared on
            # cells drawn half among the irradiated ones and half uniformly
            g32, h32 = og.astype(np.float32), oh.astype(np.float32)
            gamma.copy_(torch.from_numpy(g32))
            heat.copy_(torch.from_numpy(h32))
            cs = ctx.chem_step(g, gamma, heat, w.dt, **chem_kw)
            rng = np.random.default_rng(99)
            ncell = int(np.prod(w.shape))
            lit = np.flatnonzero(g32[0].reshape(-1) > 0)
            idx = np.unique(np.concatenate([rng.choice(lit, min(lit.size, 1 << 15), replace=False),
                                            rng.integers(0, ncell, 1 << 15)]))
            sub_grid = {"n_h": w.grid["n_h"].reshape(-1)[idx], "y_he": w.grid["y_he"]}
            sub_state = {k: w.grid[k].reshape(-1)[idx] for k in ("x_hi", "x_hei", "x_heii", "temp")}
            ref = oracle.chem(sub_grid, sub_state, g32.reshape(3, -1)[:, idx].astype(np.float64),
                              h32.reshape(3, -1)[:, idx].astype(np.float64), w.dt, w.chem)
            tid = torch.from_numpy(idx).cuda()
            judge = {"cells": int(idx.size), "accepted_frac_grid": round(1.0 - cs["fallback"] / cs["cells"], 4)}
            for k in ("x_hi", "x_hei", "x_heii"):
                judge[f"max_abs_d{k}"] = float(np.abs(g[k].reshape(-1)[tid].cpu().numpy() - ref[k]).max())
            judge["max_rel_dT"] = float(np.abs(g["temp"].reshape(-1)[tid].cpu().numpy() / ref["temp"] - 1.0).max())
            extra["learned_chem_vs_oracle"] = judge
            log(f"learned chemistry vs the oracle: {judge}")
            for k in ("x_hi", "x_hei", "x_heii", "temp"):
                g[k].copy_(torch.from_numpy(np.ascontiguousarray(w.grid[k], np.float32)))

    # The optically thin approximation (section 2.6) on an evolved state: ionised bubbles of
    # radius k Ndot^(1/3) around the sources (H and He ionised to x_HI = 1e-4), k such that the
    # bubbles' volumes add up to a fifth of the box; one trace measures every source's
    # R_tau<0.1 without the approximation, the next starts the rays there and fills the
    # spheres analytically.
    if args.thin_run and args.schedule == "batched" and args.precision == "fp32_comp":
        ncell = int(np.prod(w.shape))
        pos = np.asarray(w.sources["pos"], np.float64).reshape(-1, 3)
        nd = np.asarray(w.sources["ndot"], np.float64)
        kr = (0.2 * ncell / (4.0 * np.pi / 3.0 * nd.sum())) ** (1.0 / 3.0)
        rb = kr * np.cbrt(nd)
        ion = torch.zeros(w.shape, dtype=torch.bool, device="cuda")
        nz, ny, nx = w.shape
        for (x, y, z), r in zip(pos, rb):
            lo = [max(0, int(np.floor(c - r))) for c in (x, y, z)]
            hi = [min(n, int(np.ceil(c + r)) + 1) for c, n in zip((x, y, z), (nx, ny, nz))]
            zz = torch.arange(lo[2], hi[2], device="cuda", dtype=torch.float64).view(-1, 1, 1) + 0.5 - z
            yy = torch.arange(lo[1], hi[1], device="cuda", dtype=torch.float64).view(1, -1, 1) + 0.5 - y
            xx = torch.arange(lo[0], hi[0], device="cuda", dtype=torch.float64).view(1, 1, -1) + 0.5 - x
            ion[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= (xx * xx + yy * yy + zz * zz) < r * r
        filled = float(ion.float().mean())
        g["x_hi"].masked_fill_(ion, 1e-4)
        g["x_hei"].masked_fill_(ion, 1e-4)
        g["x_heii"].masked_fill_(ion, 1e-2)
        del ion
        src = dict(w.sources)
        src["r_thin_out"] = np.empty(nsrc)
        trace(g, src, schedule, **tune)  # warm-up of this state
        l0 = trace(g, src, schedule, **tune)
        r1 = src["r_thin_out"].copy()
        src_thin = dict(w.sources)
        src_thin["r_thin"] = r1
        src_thin["r_thin_out"] = np.empty(nsrc)
        trace(g, src_thin, schedule, **tune)
        l1 = trace(g, src_thin, schedule, **tune)
        extra["thin"] = {"ionised_fraction": round(filled, 4), "bubble_radius_median": round(float(np.median(rb)), 2),
                         "r_thin_median": round(float(np.median(r1)), 2), "r_thin_max": round(float(np.max(r1)), 2),
                         "crossings_traced": l0["crossings"], "crossings_thin": l1["crossings"],
                         "trace_ms": round(l0["ms_total"], 1), "trace_ms_thin": round(l1["ms_total"], 1),
                         "kernel_ms": round(l0["ms_kernel"], 1), "kernel_ms_thin": round(l1["ms_kernel"], 1),
                         "speedup": round(l0["ms_total"] / l1["ms_total"], 3),
                         "conservation_thin": abs(l1["emitted"] - (l1["absorbed"] - l1["absorbed_thin"]) - l1["escaped"])
                         / l1["emitted"]}
        log(f"optically thin approximation: {extra['thin']}")

    # Second ceiling: the trace kernel issues, per crossing, one random 16-byte opacity gather
    # and (after merging crossings of one cell on chip) deposits.../crossing random int64 atomic
    # deposits. At the device's measured random-request rates that work alone takes
    # deposits / R_dep + crossings / R_gather; frac is that time over the kernel's.
    ceil = None
    if args.ceilings and nb >= 2:
        try:
            ceil = measure_ceilings(ctx)
            t_req = deposits_per_launch / ceil["deposits_per_s"] + per_launch / ceil["gathers_per_s"]
            ceil["trace_kernel"] = {"deposits_per_s": round(deposits_per_launch / (kms * 1e-3), 1),
                                    "gathers_per_s": round(per_launch / (kms * 1e-3), 1),
                                    "request_bound_ms": round(1e3 * t_req, 2),
                                    "frac": round(1e3 * t_req / kms, 4)}
        except Exception as e:  # a probe failure must not cost the benchmark line
            ceil = {"error": repr(e)[:300]}
        log(f"ceilings: {ceil}")
    roofline["requests"] = ceil

    names = {0: "64^3 uniform H, 1 source (Test 1 gas)", 1: "128^3 lognormal H+He, 16 sources",
             2: "256^3 lognormal H+He, 1024 sources", 3: "512^3 lognormal H+He, 4096 sources",
             4: "1024^3 GRF H+He, 16384 sources"}
    out = {
        "metric": "cell-crossings/s per RT step at 1024^3 x 16k sources",
        "value": round(value, 1),
        "unit": "cell-crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": names[args.config], "grid": list(w.shape), "sources": nsrc, "bins": nb,
                   "schedule": schedule, "graph": bool(args.graph) and schedule != "plain",
                   "precision": args.precision, "chemistry": args.chem,
                   "dt_myr": w.dt / W.MYR_S},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()
    ctx.close()


if __name__ == "__main__":
    main()
