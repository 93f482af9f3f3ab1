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
roofline, the PML/TVaR error of each sampling form against the FP64
oracle's measures of the same workload (tests/golden/, written by a script
that runs only the oracle), the surrogate and table forms, the 64-layer
portfolio batch and the serving loop (plain and surrogate), and the FP64
oracle timed on this host on fixed slices of the same YET (all cores and one
core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0                 # MI355X HBM3E
# VALU issue ceiling in lane-instructions/s: each SIMD issues one wave64 VALU
# instruction every 4 cycles (16 lanes per cycle), so 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.32e12.  The FP32 vector peak of 157.3 TFLOP/s is this
# rate x 2 (an FMA counts two flops) x 2 (packed FP32, not used here).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_800k_oracle.json")
PROFILE_PLAIN = os.path.join(ROOT, "profiles", "k_layer_plain_paper800k_counters.md")
PROFILE_MEAN = os.path.join(ROOT, "profiles", "k_mean_slice_paper800k_trace.md")
# the sources that define the layer and mean kernels: counters taken on other
# sources do not describe the kernels this run times
KERNEL_SOURCES = ("ara_kernels.hip", "ara_math.hpp", "ara_wave.hpp", "ara_internal.hpp")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1310_2274_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_constants(path: str) -> dict:
    """`key: value` lines of a profile summary's constants block, and whether
    they were taken on the current kernel sources."""
    if not os.path.exists(path):
        return {"current": False}
    text = open(path).read()
    m = re.search(r"<!-- bench constants(.*?)-->", text, re.S)
    vals = {}
    for line in (m.group(1).splitlines() if m else []):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    vals["current"] = vals.get("sources_sha256") == kernel_sources_sha256()
    return vals


def event_counts(yet, catalog_size) -> np.ndarray:
    """Occurrences of each event in the YET (each is one draw per XELT holding it)."""
    cnt = np.zeros(catalog_size, dtype=np.int64)
    for lo in range(0, yet.shape[0], 65536):
        cnt += np.bincount(yet[lo:lo + 65536].ravel(), minlength=catalog_size)
    return cnt


def count_draws(occ, layer) -> int:
    """Number of (trial, slot, XELT) hits: the draws one pass makes."""
    return int(sum(int(occ[e.event_id].sum()) for e in layer.elts))


def cpu_baseline(wl, seconds_all: float, seconds_one: float):
    """The FP64 oracle (C, OpenMP over trials) on fixed leading slices of the
    YET: trials 0..7,999 on every core this process may use, and a slice sized
    to about `seconds_one` on one core (the sequential run), each extrapolated
    linearly to all trials (trials are independent)."""
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    lay = wl.layers[0]
    K, N = wl.events_per_trial, wl.n_trials

    def run(n_trials, threads, budget):
        done, t_used, chunk = 0, 0.0, 250
        while done < n_trials and t_used < budget:
            trials = np.arange(done, min(done + chunk, n_trials))
            rows = wl.yet_rows(trials)
            t0 = time.perf_counter()
            oracle.run_layer(lay, rows, trials, wl.catalog_size, wl.seed, threads=threads)
            t_used += time.perf_counter() - t0
            done += trials.size
        return done, t_used

    cores = len(os.sched_getaffinity(0))
    n_all, t_all = run(min(8000, N), cores, 4 * seconds_all)
    rate = n_all * K / t_all
    n_one, t_one = run(min(8000, N), 1, seconds_one)
    rate1 = n_one * K / t_one
    return {"value": rate, "unit": "trial-events/s", "cores": cores, "kind": "oracle",
            "sample": f"trials 0..{n_all - 1} of the {N}-trial YET ({n_all * K} trial-events) in {t_all:.1f} s, "
                      f"FP64 C oracle, OpenMP over trials on {cores} threads",
            "extrapolated_full_pass_s": N * K / rate,
            "single_core": {"value": rate1, "unit": "trial-events/s", "cores": 1,
                            "sample": f"trials 0..{n_one - 1} ({n_one * K} trial-events) in {t_one:.1f} s",
                            "extrapolated_full_pass_s": N * K / rate1}}


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
    """Wall time per step (run + risk measures), mean layer-kernel time, time of
    the run alone, and the last step's PML/TVaR."""
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
    # the run alone (no risk measures), back to back
    t1 = time.perf_counter()
    for _ in range(steps):
        P.ara_run_layer(eng.ctx, yh, desc, mode, seed, out)
    torch.cuda.synchronize()
    dt_run = time.perf_counter() - t1
    return dt / steps, float(np.mean(kms)), dt_run / steps, pml, tvar


def oracle_errors(wl, pml, tvar):
    """Relative PML/TVaR errors against the FP64 oracle's measures of the same
    workload over all its trials (tests/golden/), when they are there."""
    if not os.path.exists(GOLDEN):
        return None
    g = json.load(open(GOLDEN))
    if g.get("workload") != wl.name or g.get("n_trials") != wl.n_trials or g.get("seed") != wl.seed:
        return None
    po, to = np.array(g["pml"]), np.array(g["tvar"])
    return {"pml_rel_err_vs_oracle": (np.abs(pml - po) / po).tolist(),
            "tvar_rel_err_vs_oracle": (np.abs(tvar - to) / to).tolist(),
            "oracle_pml": g["pml"], "oracle_tvar": g["tvar"],
            "oracle": "tests/golden/paper_800k_oracle.json (FP64 oracle over every trial)"}


def surrogate_share(P, eng, handles, layer, occ, n=1_000_000, seed=5):
    """Share of draws the network answers (the rest fall back to the exact
    inverse): draws sampled in proportion to their entries' occurrence counts,
    u uniform on the 2^-24 grid, answered by ara_surrogate_eval.  The layer
    pass gives draws whose XELT term is fixed their term without a quantile;
    they are counted here like any other draw."""
    rng = np.random.default_rng(seed)
    a_all, b_all, w_all = [], [], []
    for h, e in zip(handles, layer.elts):
        a, b = P.ara_elt_params(eng.ctx, h, e.n)
        a_all.append(a)
        b_all.append(b)
        w_all.append(occ[e.event_id].astype(np.float64))
    a, b, w = np.concatenate(a_all), np.concatenate(b_all), np.concatenate(w_all)
    pick = rng.choice(a.size, size=n, p=w / w.sum())
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    ok = a[pick] > 0                                   # degenerate entries take no quantile
    _, used = P.ara_surrogate_eval(eng.ctx, a[pick][ok], b[pick][ok], u[ok])
    return float(used.sum()) / n


def surrogate_leg(P, torch, eng, yh, desc, wl, out, rps, steps, warmup, plain_step_s, plain_pml, plain_tvar,
                  n_tuples, epochs, ckpt, occ, load=""):
    if load:
        # a checkpoint of an earlier run (for profiling the layer kernel without thousands of training launches)
        P.load_surrogate(eng.ctx, load)
        marked = int(P.ara_surrogate_export(eng.ctx)["mask"].sum())
        losses, t_train = np.array([math.nan]), math.nan
        log(f"surrogate loaded from {load}, {marked}/{P.SUR_CELLS} cells fall back")
    else:
        t0 = time.perf_counter()
        losses = P.ara_surrogate_train(eng.ctx, n_tuples, epochs=epochs, batch=4096, lr=3e-3, seed=11)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        cmax, cbias, marked = P.ara_surrogate_calibrate(eng.ctx, 4_000_000, seed=12, tol=1e-3)
        log(f"surrogate trained in {t_train:.1f} s (loss {losses[0]:.2e} -> {losses[-1]:.2e}), "
            f"{marked}/{P.SUR_CELLS} cells fall back")
    if ckpt:
        P.save_surrogate(eng.ctx, ckpt)
    share = surrogate_share(P, eng, list(desc._keep), wl.layers[0], occ)
    tile = autotune(P, eng, yh, desc, P.MODE_SURROGATE, min(wl.n_trials, 100_000))["waves_per_workgroup"]
    step_s, kms, run_s, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_SURROGATE, wl.seed, out, rps,
                                                steps, warmup)
    rel_p = np.abs(pml - plain_pml) / np.abs(plain_pml)
    rel_t = np.abs(tvar - plain_tvar) / np.abs(plain_tvar)
    res = {"trial_events_per_s": wl.trial_events / step_s, "ms_per_step": step_s * 1e3, "kernel_ms": kms,
           "speedup_vs_plain": plain_step_s / step_s, "pml": pml.tolist(), "tvar": tvar.tolist(),
           "pml_rel_diff_vs_plain": rel_p.tolist(), "tvar_rel_diff_vs_plain": rel_t.tolist(),
           "train": {"tuples": n_tuples, "epochs": epochs, "seconds": t_train, "final_mse": float(losses[-1])},
           "fallback_cells": int(marked), "cells": P.SUR_CELLS, "share_of_draws_answered_by_network": share,
           "waves_per_workgroup": tile}
    res.update(oracle_errors(wl, pml, tvar) or {})
    return res


def table_leg(P, torch, eng, yh, desc, wl, out, rps, steps, warmup, plain_step_s, plain_pml, plain_tvar):
    """The table mode (per-entry tabulated inverse, no iteration) on the same
    workload and draws as the plain path."""
    t0 = time.perf_counter()
    P.ara_run_layer(eng.ctx, yh, desc, P.MODE_TABLE, wl.seed, out)      # builds the XELTs' tables once
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    step_s, kms, _, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_TABLE, wl.seed, out, rps, steps, warmup)
    rel_p = np.abs(pml - plain_pml) / np.abs(plain_pml)
    rel_t = np.abs(tvar - plain_tvar) / np.abs(plain_tvar)
    res = {"trial_events_per_s": wl.trial_events / step_s, "ms_per_step": step_s * 1e3, "kernel_ms": kms,
           "speedup_vs_plain": plain_step_s / step_s, "pml_rel_diff_vs_plain": rel_p.tolist(),
           "tvar_rel_diff_vs_plain": rel_t.tolist(), "first_run_with_table_build_s": t_build}
    res.update(oracle_errors(wl, pml, tvar) or {})
    return res


def layout_leg(P, torch, synth, eng, yh, desc, wl, out, rps, steps, plain_kernel_ms, plain_ylt):
    """The hashed layer table against the direct one: on the paper workload
    (the layer holds 99.6% of the catalog's events) and on a 20M-event catalog
    that the layer covers sparsely (about 5%)."""
    res = {}
    P.ara_set_table_kind(eng.ctx, P.TABLE_HASHED)
    try:
        _, kms, _, _, _ = timed_steps(P, torch, eng, yh, desc, P.MODE_PLAIN, wl.seed, out, rps, steps, 1)
        same = bool(torch.equal(out, plain_ylt))
    finally:
        P.ara_set_table_kind(eng.ctx, P.TABLE_DIRECT)
    res["paper"] = {"direct_kernel_ms": plain_kernel_ms, "hashed_kernel_ms": kms, "ylt_identical": same}
    log(f"layer table on the paper workload: direct {plain_kernel_ms:.2f} ms, hashed {kms:.2f} ms, "
        f"identical YLT {same}")
    sw = synth.sparse_catalog()
    e2 = P.Engine(0)
    try:
        yh2 = e2.load_yet(sw.yet(), sw.catalog_size)
        d2 = e2.load_layer(sw.layers[0], sw.catalog_size)
        o2 = torch.empty(sw.n_trials, device="cuda")
        ylts, row = {}, {}
        for name, kind in (("direct", P.TABLE_DIRECT), ("hashed", P.TABLE_HASHED)):
            P.ara_set_table_kind(e2.ctx, kind)
            _, kms, run_s, _, _ = timed_steps(P, torch, e2, yh2, d2, P.MODE_PLAIN, sw.seed, o2, rps, steps, 1)
            ylts[name] = o2.clone()
            row[f"{name}_kernel_ms"] = kms
            row[f"{name}_trial_events_per_s"] = sw.trial_events / run_s
        row["ylt_identical"] = bool(torch.equal(ylts["direct"], ylts["hashed"]))
        row["workload"] = (f"{sw.n_trials} trials x {sw.events_per_trial} events over a {sw.catalog_size}-event "
                           f"catalog, 16 XELTs of 20k-60k entries ({sum(e.n for e in sw.layers[0].elts)} in all)")
        res["sparse_catalog"] = row
        log(f"layer table on the sparse 20M catalog: direct {row['direct_kernel_ms']:.2f} ms, "
            f"hashed {row['hashed_kernel_ms']:.2f} ms, identical YLT {row['ylt_identical']}")
    finally:
        e2.close()
    return res


def variable_leg(P, torch, synth, steps, fixed_trial_events_per_s):
    """The paper layer over 800,000 trials of U{800..1,500} events (CSR)."""
    wl, ev, offs = synth.paper_variable()
    eng = P.Engine(0)
    try:
        yh = eng.load_yet(ev, wl.catalog_size, trial_offsets=offs)
        desc = eng.load_layer(wl.layers[0], wl.catalog_size)
        out = torch.empty(wl.n_trials, device="cuda")
        _, kms, run_s, _, _ = timed_steps(P, torch, eng, yh, desc, P.MODE_PLAIN, wl.seed, out,
                                          P.DEFAULT_RETURN_PERIODS, steps, 1)
    finally:
        eng.close()
    te = int(offs[-1])
    res = {"workload": f"{wl.n_trials} trials of U{{800..1500}} events ({te} trial-events, CSR), the paper layer",
           "kernel_ms": kms, "ms_per_run": run_s * 1e3, "trial_events_per_s": te / run_s,
           "vs_fixed_length_trial_events_per_s": (te / run_s) / fixed_trial_events_per_s}
    log(f"variable-length trials: {kms:.2f} ms kernel, {te / run_s:.3e} trial-events/s "
        f"({res['vs_fixed_length_trial_events_per_s']:.3f} of the fixed-length rate)")
    return res


def portfolio_leg(P, torch, synth, steps, sur_state):
    """64 layers over one 200,000-trial YET in one launch per step, plain and
    surrogate (the surrogate trained on the paper workload, imported)."""
    wl = synth.portfolio()
    eng = P.Engine(0)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    descs = [eng.load_layer(l, wl.catalog_size) for l in wl.layers]
    outs = [torch.empty(wl.n_trials, device="cuda") for _ in descs]
    res = {"waves_per_workgroup": autotune(P, eng, yh, descs[0], P.MODE_PLAIN, 50_000)["waves_per_workgroup"]}
    modes = [("plain", P.MODE_PLAIN)] + ([("surrogate", P.MODE_SURROGATE)] if sur_state is not None else [])
    for name, mode in modes:
        if mode == P.MODE_SURROGATE:
            s = sur_state
            P.ara_surrogate_import(eng.ctx, s["params"], s["adam_m"], s["adam_v"], s["step"], s["mask"], s["bias"])
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
    if "surrogate" in res:
        res["surrogate"]["speedup_vs_plain"] = res["plain"]["ms_per_step"] / res["surrogate"]["ms_per_step"]
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


def serving_leg(P, torch, synth, runs, sur_state):
    """The serving loop on a resident 1,000,000-trial YET: a Poisson stream of
    pricing requests per (mode, rate, warm-up, measured) run; p50/p99 latency
    from arrival to PML/TVaR and the sustained trial-event rate."""
    from paper_1310_2274_amd import serving
    wl = synth.serving_yet()
    eng = P.Engine(0)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    out = []
    for mode_name, rate, n_warm, n_meas in runs:
        mode = P.MODE_SURROGATE if mode_name == "surrogate" else P.MODE_PLAIN
        if mode == P.MODE_SURROGATE:
            if sur_state is None:
                continue
            s = sur_state
            P.ara_surrogate_import(eng.ctx, s["params"], s["adam_m"], s["adam_v"], s["step"], s["mask"], s["bias"])
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
        st.update({"rate_req_per_s": rate, "mode": mode_name, "requests": n_meas, "warmup_requests": n_warm,
                   "completed_req_per_s": len(done) / wall,
                   "trial_events_per_s": len(done) * wl.trial_events / wall, "wall_s": wall, "ticks": srv.ticks,
                   "budget_refusals": srv.refusals, "hbm_budget_bytes": 64 << 30})
        log(f"serving {mode_name} @ {rate}/s: p50 {st['p50_s'] * 1e3:.0f} ms, p99 {st['p99_s'] * 1e3:.0f} ms, "
            f"{st['completed_req_per_s']:.1f} req/s completed")
        out.append(st)
    eng.close()
    return {"runs": out,
            "workload": f"resident YET {wl.n_trials} x {wl.events_per_trial}, catalog {wl.catalog_size}; Poisson "
                        f"requests of log-uniform 1-32 XELTs x 10k-60k entries, 64 GiB admission budget"}


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


def parse_serve(spec: str, default_meas: int, default_warm: int):
    """'plain:20,surrogate:20:100' -> [(mode, rate, warm-up, measured)]."""
    runs = []
    for item in [s for s in spec.split(",") if s]:
        parts = item.split(":")
        mode, rate = parts[0], float(parts[1])
        meas = int(parts[2]) if len(parts) > 2 else default_meas
        warm = int(parts[3]) if len(parts) > 3 else default_warm
        runs.append((mode, rate, warm, meas))
    return runs


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
    ap.add_argument("--sur-ckpt", default="", help="save the trained surrogate here (.npz)")
    ap.add_argument("--sur-load", default="", help="load the surrogate from this checkpoint instead of training")
    ap.add_argument("--no-portfolio", action="store_true", help="skip the 64-layer portfolio-batch leg")
    ap.add_argument("--no-layouts", action="store_true", help="skip the hashed-against-direct layer-table leg")
    ap.add_argument("--no-variable", action="store_true", help="skip the variable-length (CSR) trials leg")
    ap.add_argument("--no-correlated", action="store_true",
                    help="skip the correlated multi-program portfolio leg (sigma_C > 0, program totals)")
    ap.add_argument("--serve", default="plain:20:300:30,surrogate:20:100:20,surrogate:5:60:10",
                    help="serving runs, comma-separated mode:rate[:measured[:warm-up]] ('' = none)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU baseline: about this many seconds per slice, all cores and one core (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default trial tile (1 wavefront per workgroup for the plain mode, 4 for the "
                         "surrogate)")
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
    occ = event_counts(yet, wl.catalog_size)
    draws = count_draws(occ, lay)
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
    step_s, kernel_ms, run_s, pml, tvar = timed_steps(P, torch, eng, yh, desc, P.MODE_PLAIN, wl.seed, out, rps,
                                                      args.steps, args.warmup)
    value = N * K / step_s
    log(f"plain: {step_s * 1e3:.2f} ms/step, layer kernel {kernel_ms:.2f} ms")
    plain_vs_oracle = oracle_errors(wl, pml, tvar)
    if plain_vs_oracle:
        log(f"plain PML/TVaR vs FP64 oracle: max rel err "
            f"{max(plain_vs_oracle['pml_rel_err_vs_oracle'] + plain_vs_oracle['tvar_rel_err_vs_oracle']):.2e}")
    # occurrence exceedance beside the aggregate: PML/TVaR of the largest occurrence loss per trial
    # (untimed), for the layer as priced and with its occurrence limit lifted: the limit binds in
    # nearly every trial of this workload, so only the second varies with the return period
    om = torch.empty(N, dtype=torch.float32, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, P.MODE_PLAIN, wl.seed, 0, N, out, om)
    oep_pml, oep_tvar = P.ara_risk_measures(eng.ctx, om, rps)
    desc_nl = P.layer_desc([desc.elt_handles[i] for i in range(desc.n_elts)], desc.occ_retention, math.inf,
                           desc.agg_retention, desc.agg_limit, desc.program_id)
    scratch = torch.empty(N, dtype=torch.float32, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc_nl, P.MODE_PLAIN, wl.seed, 0, N, scratch, om)
    oep_nl_pml, oep_nl_tvar = P.ara_risk_measures(eng.ctx, om, rps)
    del om, scratch

    pc = profile_constants(PROFILE_PLAIN)
    opd = float(pc["valu_lane_instructions_per_draw"]) if "valu_lane_instructions_per_draw" in pc else None
    ach = opd * draws / (kernel_ms * 1e-3) / 1e12 if opd else None
    traffic = None
    if pc["current"] and N == 800_000 and "fetch_kib_per_launch" in pc:
        traffic = (float(pc["fetch_scale"]) * float(pc["fetch_kib_per_launch"]) +
                   float(pc["write_scale"]) * float(pc["write_kib_per_launch"])) * 1024
    # Algorithmic bytes per launch (the units of the plain path's gathers): the
    # YET's 4-byte ids, one 16-byte layer-table row per trial-event, the
    # entry's 16 bytes of Beta parameters per draw, and the 4-byte YLT.
    te = float(N) * float(wl.events_per_trial)
    alg_bytes = 4.0 * te + 16.0 * te + 16.0 * draws + 4.0 * N
    ach_gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": ach_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach_gbs / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": "k_layer_plain", "kernel_ms": kernel_ms, "draws_per_launch": draws,
            "draws_per_s": draws / (kernel_ms * 1e-3), "algorithmic_bytes": alg_bytes,
            "counters_match_kernel_sources": pc["current"],
            "alu_view": {"ops_per_draw": opd, "ops_unit": "VALU lane-instructions (SQ_INSTS_VALU x 64 / draws)",
                         "achieved_TOPs": ach, "peak_TOPs": PEAK_VALU_TOPS,
                         "valu_busy": float(pc["valu_busy"]) if "valu_busy" in pc else None},
            "note": "algorithmic bytes: 4 B (YET id) + 16 B (layer row) per trial-event, 16 B (Beta parameters) "
                    "per draw, 4 B per trial; traffic: L2 <-> fabric bytes from FETCH_SIZE/WRITE_SIZE. The "
                    "launch is bound by L1 misses in flight (about 62 per CU, 410-cycle average L2 latency, "
                    "texture data unit busy 0.98: profiles/k_layer_plain_paper800k_memory.md), not by VALU "
                    "issue: removing the solve arithmetic or 6 of the 10 Philox rounds saves little"}

    mean_leg = None
    if not args.no_mean_leg:
        before = P.lib().ara_bytes_in_use(eng.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.ara_run_layer(eng.ctx, yh, desc, P.MODE_MEAN, wl.seed, out)     # builds the slice-major YET copy
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t0
        copy_bytes = P.lib().ara_bytes_in_use(eng.ctx) - before
        if not args.no_autotune:
            tune["mean"] = autotune(P, eng, yh, desc, P.MODE_MEAN, min(N, 200_000))
        mstep, mk, _, _, _ = timed_steps(P, torch, eng, yh, desc, P.MODE_MEAN, wl.seed, out, rps,
                                         max(3, args.steps), 2)
        gbs = (N * K * 4 + N * 4) / (mk * 1e-3) / 1e9
        mc = profile_constants(PROFILE_MEAN)
        mtraffic = None
        if mc["current"] and N == 800_000 and "fetch_kib_per_launch" in mc:
            mtraffic = (float(mc["fetch_scale"]) * float(mc["fetch_kib_per_launch"]) +
                        float(mc["write_scale"]) * float(mc["write_kib_per_launch"])) * 1024
        mean_leg = {"bound": "hbm", "kernel": "k_mean_slice + k_mean_finish", "kernel_ms": mk, "achieved": gbs,
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                    "algorithmic_bytes": N * K * 4 + N * 4,
                    "note": "algorithmic bytes: 4 B per int32 trial-event of the YET + 4 B per trial; the kernel "
                            "reads the slice-major copy of the YET, 2 B per trial-event (16-bit ids within a "
                            "catalog slice), so it moves about half of them (traffic)",
                    "ms_per_step": mstep * 1e3,
                    "trial_events_per_s": N * K / mstep, "traffic": mtraffic,
                    "counters_match_kernel_sources": mc["current"],
                    "first_run_with_slice_copy_s": first_s, "slice_copy_device_bytes": int(copy_bytes)}
        log(f"mean mode: kernel {mk:.3f} ms = {gbs:.0f} GB/s (first run with the slice-major copy "
            f"{first_s * 1e3:.0f} ms, {copy_bytes / 1e9:.2f} GB)")

    tab = None
    if not args.no_table:
        tab = table_leg(P, torch, eng, yh, desc, wl, out, rps, args.steps, args.warmup, step_s, pml, tvar)
        log(f"table mode: {tab['ms_per_step']:.2f} ms/step, x{tab['speedup_vs_plain']:.2f} vs plain, "
            f"max PML/TVaR rel diff {max(tab['pml_rel_diff_vs_plain'] + tab['tvar_rel_diff_vs_plain']):.2e} "
            f"(first run with the table build {tab['first_run_with_table_build_s']:.2f} s)")

    layouts = None
    if not args.no_layouts:
        plain_ylt = out.clone()
        P.ara_run_layer(eng.ctx, yh, desc, P.MODE_PLAIN, wl.seed, plain_ylt)
        layouts = layout_leg(P, torch, synth, eng, yh, desc, wl, out, rps, max(2, args.steps // 2), kernel_ms,
                             plain_ylt)
        del plain_ylt

    sur, sur_state = None, None
    if not args.no_surrogate:
        sur = surrogate_leg(P, torch, eng, yh, desc, wl, out, rps, args.steps, args.warmup, step_s, pml, tvar,
                            args.sur_tuples, args.sur_epochs, args.sur_ckpt, occ, args.sur_load)
        sur_state = P.ara_surrogate_export(eng.ctx)
        err = sur.get("pml_rel_err_vs_oracle")
        log(f"surrogate: {sur['ms_per_step']:.2f} ms/step, x{sur['speedup_vs_plain']:.2f} vs plain, "
            f"{sur['share_of_draws_answered_by_network']:.3f} of draws answered by the network, "
            f"max PML/TVaR rel diff vs plain {max(sur['pml_rel_diff_vs_plain'] + sur['tvar_rel_diff_vs_plain']):.2e}"
            + (f", vs oracle {max(err + sur['tvar_rel_err_vs_oracle']):.2e}" if err else ""))
    eng.close()
    del yet

    var = None if args.no_variable else variable_leg(P, torch, synth, max(2, args.steps // 2), N * K / run_s)
    port = None if args.no_portfolio else portfolio_leg(P, torch, synth, max(1, args.steps // 2), sur_state)
    corr = None if args.no_correlated else correlated_leg(P, torch, synth, max(1, args.steps // 2))
    serve = None
    runs = parse_serve(args.serve, 300, 30)
    if runs:
        serve = serving_leg(P, torch, synth, runs, sur_state)

    cpu = None
    if args.cpu_seconds > 0:
        log(f"CPU oracle baseline on {len(os.sched_getaffinity(0))} threads and on one")
        cpu = cpu_baseline(wl, args.cpu_seconds, args.cpu_seconds)

    rec = {
        "metric": "trial-events/s", "value": value, "unit": "trial-events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{N} trials x {K} events/trial, 100,000-event catalog, 1 layer of 16 XELTs "
                               f"(20k-50k entries), plain inverse-Beta sampling, PML/TVaR at 10/50/100/250 yr",
                   "n_trials": N, "events_per_trial": K, "n_elts": len(lay.elts), "draws_per_step": draws},
        "run_only": {"ms": run_s * 1e3, "trial_events_per_s": N * K / run_s, "draws_per_s": draws / run_s,
                     "note": "ara_run_layer alone, without ara_risk_measures"},
        "roofline": roof,
        "roofline_streaming": mean_leg,
        "trial_tile": tune or None,
        "plain_vs_oracle": plain_vs_oracle,
        "table_mode": tab,
        "layer_table_layouts": layouts,
        "variable_length_trials": var,
        "surrogate": sur,
        "portfolio": port,
        "correlated_portfolio": corr,
        "serving": serve,
        "cpu_baseline": cpu,
        "pml": [float(v) for v in pml], "tvar": [float(v) for v in tvar],
        "oep": {"pml": [float(v) for v in oep_pml], "tvar": [float(v) for v in oep_tvar],
                "without_occurrence_limit": {"pml": [float(v) for v in oep_nl_pml],
                                             "tvar": [float(v) for v in oep_nl_tvar]},
                "note": "PML/TVaR of the largest occurrence loss per trial (occurrence exceedance), for the "
                        "layer as priced (its occurrence limit binds in nearly every trial) and with the "
                        "occurrence limit lifted"},
        "context": {"paper_c2075_trial_events_per_s": 8e8 / 41.0,
                    "note": "paper: 800k x 1,000 in 41 s on a Tesla C2075 with ~0.3 draws per trial-event; "
                            "this workload has ~5.3 draws per trial-event"},
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
