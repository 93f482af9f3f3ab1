#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the paper-scale workload
(800,000 trials x 1,000 events, one layer of 16 XELTs, secondary uncertainty):
ara_run_layer (stream the YET, look up the XELTs, draw every loss, apply the
XELT / occurrence / aggregate terms, write the YLT) followed by
ara_risk_measures (PML and TVaR at 10/50/100/250 years).  Inputs are
resident in HBM before timing starts.

Printed: one JSON line with the metric (trial-events/s of the plain form),
the roofline of the dominant kernel, the streaming-phase (mean mode)
roofline, the surrogate form (speed and PML/TVaR difference), optional
portfolio-batch and serving legs, and the FP64 oracle timed on this host on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0                 # MI355X HBM3E
# VALU issue peak in lane-instructions/s: MI355X's FP32 vector rate of
# 157.3 TFLOP/s counts an FMA as two flops, i.e. 78.6e12 FP32 lane-instructions
# per second (256 CUs x 128 lanes x 2.4 GHz).  SQ_INSTS_VALU x 64 counts every
# VALU instruction once, so FP64 and transcendental instructions, which issue
# at lower rates, make the achieved figure an underestimate, never an overcount.
PEAK_VALU_TOPS = 157.3 / 2
# VALU lane-instructions per draw of the plain layer kernel on this workload,
# SQ_INSTS_VALU x 64 / draws from rocprofv3 (profiles/k_layer_plain_*_counters.md).
VALU_OPS_PER_DRAW = 746.2
# Bytes per launch of the plain layer kernel at 800,000 trials between L2 and
# the memory fabric: FETCH_SIZE (x2, copy-kernel calibration) + WRITE_SIZE,
# measured on the 100,000-trial slice and scaled by 8.
TRAFFIC_BYTES = 8 * (2.0 * 25379206.7 + 1.0 * 344259.3) * 1024
# The same for one 800,000-trial mean-mode pass (k_mean_slice + k_mean_finish,
# profiles/k_mean_slice_paper800k_trace.md).
MEAN_TRAFFIC_BYTES = (2.0 * (1669229.0 + 28132.0) + 1.0 * (56297.0 + 3125.0)) * 1024


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def count_draws(yet, layer, catalog_size) -> int:
    """Number of (trial, slot, XELT) hits: the draws one pass makes."""
    cnt = np.zeros(catalog_size, dtype=np.int64)
    for e in layer.elts:
        cnt[e.event_id] += 1
    total = 0
    for lo in range(0, yet.shape[0], 65536):
        total += int(cnt[yet[lo:lo + 65536]].sum())
    return total


def cpu_baseline(wl, seconds: float, threads: int):
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    lay = wl.layers[0]
    done, t_used, chunk = 0, 0.0, 256
    while t_used < seconds and done < wl.n_trials:
        trials = np.arange(done, min(done + chunk, wl.n_trials))
        rows = wl.yet_rows(trials)
        t0 = time.perf_counter()
        oracle.run_layer(lay, rows, trials, wl.catalog_size, wl.seed, threads=threads)
        t_used += time.perf_counter() - t0
        done += trials.size
    return {"value": done * wl.events_per_trial / t_used, "unit": "trial-events/s", "cores": threads,
            "kind": "oracle",
            "sample": f"trials 0..{done - 1} of the {wl.n_trials}-trial YET ({done * wl.events_per_trial} "
                      f"trial-events, {t_used:.1f} s, FP64 C oracle, OpenMP over trials)"}


def autotune(P, eng, yh, desc, mode, n_trials):
    """Pick the trial tile (wavefronts per workgroup) for this layer and mode on
    a slice of the YET, outside the timed region."""
    h = P.ara_prepare_layer(eng.ctx, desc, mode)
    try:
        best, ms = P.ara_autotune(eng.ctx, yh, [h], n_trials)
    finally:
        P.ara_free_layer(eng.ctx, h)
    return {"waves_per_workgroup": int(best), "candidates": [1, 2, 4, 8],
            "slice_ms": [None if not np.isfinite(m) else round(float(m), 3) for m in ms], "slice_trials": n_trials}


def timed_steps(P, torch, eng, yh, desc, mode, seed, out, rps, steps, warmup):
    for _ in range(warmup):
        P.ara_run_layer(eng.ctx, yh, desc, mode, seed, out)
        P.ara_risk_measures(eng.ctx, out, rps)
    torch.cuda.synchronize()
    P.ara_set_profiling(eng.ctx, True)
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        P.ara_run_layer(eng.ctx, yh, desc, mode, seed, out)
        pml, tvar = P.ara_risk_measures(eng.ctx, out, rps)
        kms.append(P.ara_last_kernel_ms(eng.ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P.ara_set_profiling(eng.ctx, False)
    return dt / steps, float(np.mean(kms)), pml, tvar


def surrogate_leg(P, torch, eng, yh, desc, wl, out, rps, steps, warmup, plain_step_s, plain_pml, plain_tvar,
                  n_tuples, epochs, ckpt):
    t0 = time.perf_counter()
    losses = P.ara_surrogate_train(eng.ctx, n_tuples, epochs=epochs, batch=4096, lr=3e-3, seed=11)
    t_train = time.perf_counter() - t0
    cmax, cbias, marked = P.ara_surrogate_calibrate(eng.ctx, 4_000_000, seed=12, tol=1e-3)
    log(f"surrogate trained in {t_train:.1f} s (loss {losses[0]:.2e} -> {losses[-1]:.2e}), "
        f"{marked}/{P.SUR_CELLS} cells fall back")
    if ckpt:
        P.save_surrogate(eng.ctx, ckpt)
    tile = autotune(P, eng, yh, desc, P.MODE_SURROGATE, min(wl.n_trials, 100_000))["waves_per_workgroup"]
    step_s, kms, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_SURROGATE, wl.seed, out, rps, steps, warmup)
    rel_p = np.abs(pml - plain_pml) / np.abs(plain_pml)
    rel_t = np.abs(tvar - plain_tvar) / np.abs(plain_tvar)
    return {"trial_events_per_s": wl.trial_events / step_s, "ms_per_step": step_s * 1e3, "kernel_ms": kms,
            "speedup_vs_plain": plain_step_s / step_s, "pml": pml.tolist(), "tvar": tvar.tolist(),
            "pml_rel_diff_vs_plain": rel_p.tolist(), "tvar_rel_diff_vs_plain": rel_t.tolist(),
            "train": {"tuples": n_tuples, "epochs": epochs, "seconds": t_train, "final_mse": float(losses[-1])},
            "fallback_cells": int(marked), "cells": P.SUR_CELLS, "waves_per_workgroup": tile,
            "note": "PML/TVaR differences are against the plain GPU path, which matches the FP64 oracle per "
                    "trial far inside 1e-5 of the gross loss (tests/test_gpu_parity.py)"}


def table_leg(P, torch, eng, yh, desc, wl, out, rps, steps, warmup, plain_step_s, plain_pml, plain_tvar):
    """The table mode (per-entry tabulated inverse, no iteration) on the same
    workload and draws as the plain path."""
    t0 = time.perf_counter()
    P.ara_run_layer(eng.ctx, yh, desc, P.MODE_TABLE, wl.seed, out)      # builds the XELTs' tables once
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    step_s, kms, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_TABLE, wl.seed, out, rps, steps, warmup)
    rel_p = np.abs(pml - plain_pml) / np.abs(plain_pml)
    rel_t = np.abs(tvar - plain_tvar) / np.abs(plain_tvar)
    return {"trial_events_per_s": wl.trial_events / step_s, "ms_per_step": step_s * 1e3, "kernel_ms": kms,
            "speedup_vs_plain": plain_step_s / step_s, "pml_rel_diff_vs_plain": rel_p.tolist(),
            "tvar_rel_diff_vs_plain": rel_t.tolist(), "first_run_with_table_build_s": t_build,
            "note": "per-draw error against the FP64 inverse below 2e-4 relative and 2e-5 of max_l "
                    "(tests/test_gpu_table.py)"}


def portfolio_leg(P, torch, synth, steps):
    wl = synth.portfolio()
    eng = P.Engine(0)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    descs = [eng.load_layer(l, wl.catalog_size) for l in wl.layers]
    outs = [torch.empty(wl.n_trials, device="cuda") for _ in descs]
    res = {"waves_per_workgroup": autotune(P, eng, yh, descs[0], P.MODE_PLAIN, 50_000)["waves_per_workgroup"]}
    for name, mode in (("plain", P.MODE_PLAIN), ("surrogate", P.MODE_SURROGATE)):
        if mode == P.MODE_SURROGATE:
            P.ara_surrogate_train(eng.ctx, 4_000_000, epochs=10, batch=4096, lr=3e-3, seed=11)
            P.ara_surrogate_calibrate(eng.ctx, 2_000_000, seed=12, tol=1e-3)
        P.ara_run_layers(eng.ctx, yh, descs, mode, wl.seed, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            P.ara_run_layers(eng.ctx, yh, descs, mode, wl.seed, outs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms_per_step": dt * 1e3,
                     "trial_events_per_s": len(descs) * wl.trial_events / dt}
        log(f"portfolio {name}: {dt * 1e3:.1f} ms for {len(descs)} layers")
    eng.close()
    res["workload"] = f"{wl.n_trials} trials x {wl.events_per_trial} events, {len(wl.layers)} layers " \
                      f"({sum(len(l.elts) for l in wl.layers)} XELTs), one launch per step"
    return res


def correlated_leg(P, torch, synth, steps):
    """10 programs x 2 layers sharing ELTs with correlated std (sigma_C > 0),
    program and portfolio totals and their PML/TVaR; the same portfolio with
    sigma_C = 0 beside it."""
    res = {}
    rps = P.DEFAULT_RETURN_PERIODS
    for name, frac in (("correlated", 0.6), ("independent", 0.0)):
        wl = synth.correlated_portfolio(n_programs=10, layers_per_program=2, n_trials=200_000, sigma_c_frac=frac)
        eng = P.Engine(0)
        yh = eng.load_yet(wl.yet(), wl.catalog_size)
        descs = [eng.load_layer(l, wl.catalog_size) for l in wl.layers]
        N = wl.n_trials
        tile = autotune(P, eng, yh, descs[0], P.MODE_PLAIN, min(N, 50_000))["waves_per_workgroup"]
        outs = [torch.empty(N, device="cuda") for _ in descs]
        progs = sorted({l.program_id for l in wl.layers})
        ptot = [torch.empty(N, device="cuda") for _ in progs]
        total = torch.empty(N, device="cuda")

        def step():
            P.ara_run_layers(eng.ctx, yh, descs, P.MODE_PLAIN, wl.seed, outs)
            for k, p in enumerate(progs):
                P.ara_sum_ylts(eng.ctx, [outs[l] for l, lay in enumerate(wl.layers) if lay.program_id == p], ptot[k])
            P.ara_sum_ylts(eng.ctx, ptot, total)
            return P.ara_risk_measures(eng.ctx, total, rps)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pml, tvar = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms_per_step": dt * 1e3, "trial_events_per_s": len(descs) * wl.trial_events / dt,
                     "portfolio_pml": [float(v) for v in pml], "portfolio_tvar": [float(v) for v in tvar],
                     "waves_per_workgroup": tile}
        log(f"correlated portfolio ({name}): {dt * 1e3:.1f} ms for {len(descs)} layers + totals")
        eng.close()
    res["workload"] = (f"200000 trials x 1000 events, 10 programs x 2 layers over a shared pool of 24 ELTs "
                       f"(10k-40k entries), sigma_C share U(0, 0.6) of each std; one launch for all layers, "
                       f"program and portfolio totals, portfolio PML/TVaR")
    return res


def serving_leg(P, torch, synth, rate, n_warm, n_meas, mode_name):
    from paper_1310_2274_amd import serving
    wl = synth.serving_yet()
    eng = P.Engine(0)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    mode = P.MODE_SURROGATE if mode_name == "surrogate" else P.MODE_PLAIN
    if mode == P.MODE_SURROGATE:
        P.ara_surrogate_train(eng.ctx, 4_000_000, epochs=10, batch=4096, lr=3e-3, seed=11)
        P.ara_surrogate_calibrate(eng.ctx, 2_000_000, seed=12, tol=1e-3)
    n = n_warm + n_meas
    arr = serving.poisson_arrivals(rate, n, seed=4)
    reqs = [serving.Request(i, synth.pricing_request(i), seed=1000 + i, arrival=float(arr[i])) for i in range(n)]
    srv = serving.PricingServer(eng, yh, wl.n_trials, wl.events_per_trial, wl.catalog_size, mode,
                                hbm_budget_bytes=64 << 30, tile=65536)
    t0 = time.perf_counter()
    done = srv.run_open_loop(reqs)
    wall = time.perf_counter() - t0
    meas = [r for r in done if r.req_id >= n_warm]
    st = serving.latency_stats(meas)
    eng.close()
    st.update({"rate_req_per_s": rate, "mode": mode_name, "requests": n_meas, "warmup_requests": n_warm,
               "trial_events_per_s": len(done) * wl.trial_events / wall, "wall_s": wall, "ticks": srv.ticks,
               "budget_refusals": srv.refusals,
               "workload": f"resident YET {wl.n_trials} x {wl.events_per_trial}, catalog {wl.catalog_size}; "
                           f"requests of log-uniform 1-32 XELTs x 10k-60k entries"})
    log(f"serving {mode_name} @ {rate}/s: p50 {st['p50_s'] * 1e3:.0f} ms, p99 {st['p99_s'] * 1e3:.0f} ms")
    return st


def copy_probe():
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    readings give the factors that turn those counters into bytes."""
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trials", type=int, default=800_000)
    ap.add_argument("--no-mean-leg", action="store_true", help="skip the streaming-phase (mean mode) leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-table", action="store_true", help="skip the table-mode leg")
    ap.add_argument("--sur-tuples", type=int, default=10_000_000)
    ap.add_argument("--sur-epochs", type=int, default=20)
    ap.add_argument("--sur-ckpt", default="")
    ap.add_argument("--portfolio", action="store_true", help="add the 64-layer portfolio-batch leg")
    ap.add_argument("--correlated", action="store_true",
                    help="add the correlated multi-program portfolio leg (sigma_C > 0, program totals)")
    ap.add_argument("--serve", default="", help="serving leg: comma-separated request rates, e.g. 5,20")
    ap.add_argument("--serve-mode", default="plain", choices=["plain", "surrogate"])
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=60)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU baseline budget (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default trial tile (1 wavefront per workgroup for the plain mode, 4 for the surrogate)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB three times (FETCH_SIZE/WRITE_SIZE calibration under rocprofv3)")
    args = ap.parse_args()

    if args.copy_probe:
        copy_probe()
        return

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the path has no multi-GPU mode, run with --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1310_2274_amd as P
    from paper_1310_2274_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    wl = synth.paper_scale(n_trials=args.trials)
    lay = wl.layers[0]
    N, K = wl.n_trials, wl.events_per_trial
    log(f"generating {N}x{K} YET")
    yet = wl.yet()
    draws = count_draws(yet, lay, wl.catalog_size)
    eng = P.Engine(0)
    yh = eng.load_yet(yet, wl.catalog_size)
    desc = eng.load_layer(lay, wl.catalog_size)
    out = torch.empty(N, dtype=torch.float32, device="cuda")
    rps = P.DEFAULT_RETURN_PERIODS
    log(f"setup {time.perf_counter() - t_setup:.1f} s, {draws} draws/pass")

    tune = {}
    if not args.no_autotune:
        # on the whole YET (two passes per candidate, about 1.5 s): on a 100,000-trial slice two
        # wavefronts per workgroup come out ~3% faster, on the full 800,000-trial grid ~2% slower
        tune["plain"] = autotune(P, eng, yh, desc, P.MODE_PLAIN, N)
        log(f"trial tile (plain): {tune['plain']['waves_per_workgroup']} waves/workgroup, "
            f"slice ms {tune['plain']['slice_ms']}")
    step_s, kernel_ms, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_PLAIN, wl.seed, out, rps,
                                               args.steps, args.warmup)
    value = N * K / step_s
    log(f"plain: {step_s * 1e3:.2f} ms/step, layer kernel {kernel_ms:.2f} ms")
    # occurrence exceedance beside the aggregate: PML/TVaR of the largest occurrence loss per trial (untimed)
    om = torch.empty(N, dtype=torch.float32, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, P.MODE_PLAIN, wl.seed, 0, N, out, om)
    oep_pml, oep_tvar = P.ara_risk_measures(eng.ctx, om, rps)
    del om
    ach = VALU_OPS_PER_DRAW * draws / (kernel_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s", "frac": ach / PEAK_VALU_TOPS,
            "traffic": TRAFFIC_BYTES if N == 800_000 else None, "kernel": "k_layer_plain", "kernel_ms": kernel_ms,
            "draws_per_launch": draws, "draws_per_s": draws / (kernel_ms * 1e-3),
            "ops_per_draw": VALU_OPS_PER_DRAW}

    mean_leg = None
    if not args.no_mean_leg:
        if not args.no_autotune:
            tune["mean"] = autotune(P, eng, yh, desc, P.MODE_MEAN, min(N, 200_000))
        mstep, mk, _, _ = timed_steps(P, torch, eng, yh, desc, P.MODE_MEAN, wl.seed, out, rps, max(3, args.steps), 2)
        gbs = (N * K * 4 + N * 4) / (mk * 1e-3) / 1e9
        mean_leg = {"bound": "hbm", "kernel": "k_mean_slice + k_mean_finish", "kernel_ms": mk, "achieved": gbs,
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                    "algorithmic_bytes": N * K * 4 + N * 4, "ms_per_step": mstep * 1e3,
                    "trial_events_per_s": N * K / mstep,
                    "traffic": MEAN_TRAFFIC_BYTES if N == 800_000 else None}
        log(f"mean mode: kernel {mk:.3f} ms = {gbs:.0f} GB/s")

    tab = None
    if not args.no_table:
        tab = table_leg(P, torch, eng, yh, desc, wl, out, rps, args.steps, args.warmup, step_s, pml, tvar)
        log(f"table mode: {tab['ms_per_step']:.2f} ms/step, x{tab['speedup_vs_plain']:.2f} vs plain, "
            f"max PML/TVaR rel diff {max(tab['pml_rel_diff_vs_plain'] + tab['tvar_rel_diff_vs_plain']):.2e} "
            f"(first run with the table build {tab['first_run_with_table_build_s']:.2f} s)")

    sur = None
    if not args.no_surrogate:
        sur = surrogate_leg(P, torch, eng, yh, desc, wl, out, rps, args.steps, args.warmup, step_s, pml, tvar,
                            args.sur_tuples, args.sur_epochs, args.sur_ckpt)
        log(f"surrogate: {sur['ms_per_step']:.2f} ms/step, x{sur['speedup_vs_plain']:.2f} vs plain, "
            f"max PML/TVaR rel diff {max(sur['pml_rel_diff_vs_plain'] + sur['tvar_rel_diff_vs_plain']):.2e}")
    eng.close()

    port = portfolio_leg(P, torch, synth, max(1, args.steps // 2)) if args.portfolio else None
    corr = correlated_leg(P, torch, synth, max(1, args.steps // 2)) if args.correlated else None
    serve = None
    if args.serve:
        serve = [serving_leg(P, torch, synth, float(r), args.serve_warmup, args.serve_requests, args.serve_mode)
                 for r in args.serve.split(",")]

    cpu = None
    if args.cpu_seconds > 0:
        threads = len(os.sched_getaffinity(0))
        log(f"CPU oracle baseline on {threads} threads")
        cpu = cpu_baseline(wl, args.cpu_seconds, threads)

    rec = {
        "metric": "trial-events/s", "value": value, "unit": "trial-events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{N} trials x {K} events/trial, 100,000-event catalog, 1 layer of 16 XELTs "
                               f"(20k-50k entries), plain inverse-Beta sampling, PML/TVaR at 10/50/100/250 yr",
                   "n_trials": N, "events_per_trial": K, "n_elts": len(lay.elts), "draws_per_step": draws},
        "roofline": roof,
        "roofline_streaming": mean_leg,
        "trial_tile": tune or None,
        "table_mode": tab,
        "surrogate": sur,
        "portfolio": port,
        "correlated_portfolio": corr,
        "serving": serve,
        "cpu_baseline": cpu,
        "pml": [float(v) for v in pml], "tvar": [float(v) for v in tvar],
        "oep": {"pml": [float(v) for v in oep_pml], "tvar": [float(v) for v in oep_tvar],
                "note": "PML/TVaR of the largest occurrence loss per trial (occurrence exceedance)"},
        "context": {"paper_c2075_trial_events_per_s": 8e8 / 41.0,
                    "note": "paper: 800k x 1,000 in 41 s on a Tesla C2075 with ~0.3 draws per trial-event; "
                            "this workload has ~5.3 draws per trial-event"},
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
