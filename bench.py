#!/usr/bin/env python3
"""Throughput of the residue-based ACT matching-pursuit hot path on one GPU.

One step = one act_decompose call: every order of the pursuit (search,
certified FP64 rescoring, refinement, coefficient, update) over one batch of
seeded synthetic signals already resident in HBM.  The default run measures
the metric "GMAC/s + MP iters/s, BF16+rescore vs plain FP32":
  * value: the plain FP32 search of one 2048-sample channel against the
    2,097,152-atom dictionary streamed from an HBM table (10 orders);
  * companions in the same line: the same workload with the dictionary
    synthesised on the device; 64 channels (20 orders) with the BF16 table +
    FP64 rescoring and with FP16 factor-table synthesis + FP64 rescoring; and
    the uneven batch of 1000 signals of 256..16384 samples (15 orders, FP16
    synthesis, one launch per pass over a tile queue).
GMAC/s counts the dense correlation work atoms x samples x orders x channels.
The roofline object of each leg uses its search kernel's mean launch time,
measured with HIP events that the library records on the launch stream.  The
FP64 CPU oracle is timed on a bounded sample of the primary workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-companions]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "residual-chirplet GMAC/s + MP iters/s, BF16+rescore vs plain FP32, 1 GPU"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32_mfma": 157.3, "bf16_mfma": 2500.0, "f16_mfma": 2500.0, "f64_vector": 78.6}

# name -> (workload factory, plan kwargs, roofline kind, table element bytes)
WORKLOADS = {
    "fp32-1x2048": ("fp32_1x2048", dict(dict_="table", prec="f32"), "hbm", 4),
    "fp32-1x2048-synth": ("fp32_1x2048", dict(dict_="synth", prec="f32"), "mfma_f32", 0),
    "bf16-64x2048": ("batched_64x2048", dict(dict_="table", prec="bf16"), "hbm", 2),
    "f16-64x2048-synth": ("batched_64x2048", dict(dict_="synth", prec="f16"), "mfma_f16", 0),
    # support-truncated: GMAC/s still counts the dense work (dense-equivalent rate)
    "f16-64x2048-synth-cut": ("batched_64x2048", dict(dict_="synth", prec="f16", support_cut=True), "mfma_f16", 0),
    "plain-1x512": ("plain_1x512", dict(dict_="synth", prec="f64"), "f64", 0),
    # FP16 lag table of one time centre: the dense correlation as one matrix product
    "lag-f16-64x2048": ("batched_64x2048", dict(dict_="lag", prec="f16"), "mfma_f16", 0),
    "lag-f16-1x2048": ("fp32_1x2048", dict(dict_="lag", prec="f16"), "mfma_f16", 0),
    # the same lag table in BF16 (BF16 x BF16 -> FP32 MFMA)
    "lag-bf16-64x2048": ("batched_64x2048", dict(dict_="lag", prec="bf16"), "mfma_bf16", 0),
    # complex (analytic) atoms: two correlations per atom (real and imaginary part)
    "complex-f32-64x2048-synth": ("batched_64x2048", dict(dict_="synth", prec="f32", complex_atoms=True),
                                  "mfma_f32", 0),
    "complex-lag-f16-64x2048": ("batched_64x2048", dict(dict_="lag", prec="f16", complex_atoms=True),
                                "mfma_f16", 0),
}
KERNELS = {("table", "f32"): ("k_search_f32_table", "act_search_f32t.hip"),
           ("table", "bf16"): ("k_search_bf16_table", "act_search_bf16.hip"),
           ("synth", "f32"): ("k_search_synth_f32", "act_search_synth.hip"),
           ("synth", "f16"): ("k_search_h16", "act_search_h16.hip"),
           ("synth", "f64"): ("k_search_f64", "act_search_f64.hip"),
           ("lag", "f16"): ("k_search_lag", "act_search_lag.hip"),
           ("lag", "bf16"): ("k_search_lag", "act_search_lag.hip")}


def source_sha(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2607_16629_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(workload: str, kernel_sha: str):
    """HBM bytes per search launch from the committed rocprofv3 PMC summary,
    or None when there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_search_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_sha") != kernel_sha:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(wl, seconds: float):
    """FP64 oracle correlation of the first order on a bounded prefix of the
    dictionary, scaled to GMAC/s (the search dominates the oracle's time)."""
    import oracle
    g = wl.grid
    r = wl.signals[0]
    t0 = time.perf_counter()
    oracle.correlate(g, r, 0, 512)
    per_atom = (time.perf_counter() - t0) / 512
    count = int(min(g.size, max(1024, seconds / per_atom)))
    t0 = time.perf_counter()
    oracle.correlate(g, r, 0, count)
    dt = time.perf_counter() - t0
    return {"value": round(count * g.n / dt / 1e9, 4), "unit": "GMAC/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"order-1 FP64 correlation of channel 0 of {wl.name} against atoms "
                      f"[0, {count}) of {g.size} ({dt:.1f} s, OpenMP over atoms)"}


TUNE = True  # pick the search's launch shape with act_tune before timing (--no-tune: built-in defaults)


def run_workload(name: str, steps: int, warmup: int):
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W

    factory, plan_kw, kind, elt = WORKLOADS[name]
    wl = getattr(W, factory)()
    g = wl.grid
    B, order = wl.signals.shape[0], wl.order
    plan = act.Plan(g, max_batch=B, refine_steps=wl.refine_steps, **plan_kw)
    sig = torch.from_numpy(wl.signals).cuda()
    resid = torch.empty_like(sig)
    out = plan.alloc_outputs(B, order)

    def step():
        resid.copy_(sig)
        plan.act_decompose(resid, order, out)

    shape = plan.act_tune(sig, reps=2) if TUNE else None  # untimed: shape choice on the input
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.act_timing_enable(True)
    plan.act_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = plan.act_timing_read()
    plan.act_timing_enable(False)
    flags = out["flags"].cpu().numpy()
    lag_flops = plan.search_flops(B) if plan_kw.get("dict_") == "lag" else None
    plan.close()

    s_ms, s_n = phases["search"]
    search_ms = s_ms / max(s_n, 1)
    res = {
        "workload": name, "value": round(g.size * g.n * order * B * steps / wall / 1e9, 3),
        "unit": "GMAC/s", "ms_per_step": round(wall * 1e3 / steps, 4),
        "mp_iters_per_s": round(order * steps / wall, 3),
        "channel_iters_per_s": round(order * B * steps / wall, 3),
        "search_only_gmac_per_s": round(g.size * g.n * B / (search_ms * 1e-3) / 1e9, 3),
        "dtype": plan_kw["prec"],
        "config": {"workload": wl.name, "atoms": g.size, "n_samples": g.n, "channels": B,
                   "order": order, "dict": plan_kw["dict_"], "refine_steps": wl.refine_steps,
                   "support_cut": bool(plan_kw.get("support_cut", False)),
                   "complex_atoms": bool(plan_kw.get("complex_atoms", False)), "parallelism": "single-gpu"},
        "phases_ms_per_order": {k: round(v[0] / max(v[1], 1), 5) for k, v in phases.items()},
        "candidate_overflow_channels": int(((flags & act.FLAG_CAND_OVERFLOW) != 0).sum()),
        "launch_shape": shape,
    }
    kname, ksrc = KERNELS[(plan_kw["dict_"], plan_kw["prec"])]
    if kind == "hbm":
        algo_bytes = g.size * g.n * elt + B * g.n * elt
        achieved = algo_bytes / (search_ms * 1e-3) / 1e9
        traffic = committed_traffic(wl.name, source_sha(ksrc, "act_emit.h"))
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": traffic, "kernel": kname,
                           "algorithmic_bytes_per_launch": algo_bytes,
                           "avg_launch_ms": round(search_ms, 5)}
        if plan_kw["prec"] == "bf16":
            flops = 2.0 * g.size * g.n * B
            res["roofline"]["mfma_frac_of_bf16_peak"] = round(
                flops / (search_ms * 1e-3) / (PEAK_TFLOPS["bf16_mfma"] * 1e12), 4)
    elif kind in ("mfma_f32", "mfma_f16", "mfma_bf16"):
        # factored synthesis: the matrix cores execute 2 x (atoms x N x B)
        # multiply-adds; the roofline counts the dense correlation's flops
        # (complex atoms: both parts, 2 x atoms x N x B multiply-adds)
        algo = 2.0 * g.size * g.n * B * (2 if plan_kw.get("complex_atoms") else 1)
        lag = plan_kw["dict_"] == "lag"
        achieved = algo / (search_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[kind[5:] + "_mfma"]
        # the factored synthesis runs two products per sample; the lag table
        # only its tiles' nonzero lag bands (counted by the library)
        executed = lag_flops if lag else 2 * algo
        # lag table: HBM bytes per launch from the committed counter summary
        # (the table's re-reads by row tiles are served by L2 or not)
        traffic = committed_traffic(name, source_sha(ksrc, "act_emit.h")) if lag else None
        res["roofline"] = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                           "kernel": kname, "avg_launch_ms": round(search_ms, 5),
                           "algorithmic_flops_per_launch": algo,
                           "executed_mfma_flops_per_launch": executed,
                           "executed_frac": round(executed / (search_ms * 1e-3) / (peak * 1e12), 4)}
        if lag:
            # the lag table skips exact zeros: frac is a dense-equivalent rate
            res["roofline"]["dense_equivalent"] = True
    else:
        # FP64 on-the-fly synthesis, ~60 FP64 operations per atom sample
        ops = g.size * g.n * B * 60
        achieved = ops / (search_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS["f64_vector"]
        res["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                           "kernel": kname, "avg_launch_ms": round(search_ms, 5)}
    return res, wl


def run_ragged(steps: int, warmup: int, prec: str = "f16", cut: bool = False, dict_: str = "synth"):
    """Uneven batch: 1000 signals of log-uniform length 256..16384 in one
    act_decompose call, each with its own grid (floor(N/32) time centres,
    64 f_c x 32 c x 16 dt), 15 orders, synthesised search (or the FP16 lag
    table) + FP64 rescoring."""
    import numpy as np
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W
    wl = W.ragged_batch()
    lens = wl.lengths
    B, order = len(lens), wl.order
    per_tc = 64 * 32 * 16
    plan = act.Plan(W.ragged_grid(int(lens.max()), 32, 64, 32, 16), dict_=dict_, prec=prec, max_batch=B,
                    refine_steps=wl.refine_steps, ragged=True, ragged_tc_div=32, support_cut=cut)
    sig = torch.from_numpy(wl.signals).cuda()
    resid = torch.empty_like(sig)
    lt = torch.from_numpy(lens.astype(np.int32)).cuda()
    ot = torch.from_numpy(wl.offsets.astype(np.int64)).cuda()
    out = plan.alloc_outputs(B, order, approx=False)
    out["approx"] = torch.empty_like(sig)

    def step():
        resid.copy_(sig)
        plan.act_decompose_ragged(resid, lt, ot, order, out)

    shape = plan.act_tune(sig, reps=1, lengths=lt, offsets=ot) if TUNE else None
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.act_timing_enable(True)
    plan.act_timing_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = plan.act_timing_read()
    plan.act_timing_enable(False)
    flags = out["flags"].cpu().numpy()
    plan.close()
    macs = float(sum((int(n) // 32) * per_tc * int(n) for n in lens))  # dense MACs of one order
    s_ms, s_n = phases["search"]
    search_ms = s_ms / max(s_n, 1)
    algo = 2.0 * macs
    achieved = algo / (search_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec + "_mfma"]
    kname, _ = KERNELS[(dict_, prec)]
    lag = dict_ == "lag"
    return {"workload": wl.name + "-" + prec + ("-cut" if cut else "") + ("-lag" if lag else ""),
            "value": round(macs * order * steps / wall / 1e9, 3),
            "unit": "GMAC/s", "ms_per_step": round(wall * 1e3 / steps, 3),
            "mp_iters_per_s": round(order * steps / wall, 3),
            "channel_iters_per_s": round(order * B * steps / wall, 3),
            "search_only_gmac_per_s": round(macs / (search_ms * 1e-3) / 1e9, 3),
            "dtype": prec,
            "config": {"workload": wl.name, "signals": B, "n_min": int(lens.min()), "n_max": int(lens.max()),
                       "dense_macs_per_order": macs, "order": order, "dict": dict_, "support_cut": cut,
                       "refine_steps": wl.refine_steps, "parallelism": "single-gpu"},
            "phases_ms_per_order": {k: round(v[0] / max(v[1], 1), 5) for k, v in phases.items()},
            "candidate_overflow_channels": int(((flags & act.FLAG_CAND_OVERFLOW) != 0).sum()),
            "launch_shape": shape,
            "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(achieved / peak, 4), "traffic": None,
                         "kernel": kname + ("" if lag else "_ragged"), "avg_launch_ms": round(search_ms, 5),
                         "algorithmic_flops_per_launch": algo,
                         # the lag table runs its tiles' nonzero bands (counted per call on the device only)
                         "executed_mfma_flops_per_launch": None if lag else 2 * algo,
                         "dense_equivalent": lag}}


def run_sweep(steps: int, warmup: int):
    """The paper's EEG protocol on synthetic windows (Sec. III-B/III-C): 50
    one-second windows on its 185,600-atom EEG grid, the residue-based ACT to
    order 200 (FP32 synthesis + FP64 rescoring) and the prior ACT to order 10
    (contrast mode, FP64); normalised residues E_k/|s|^2 per order."""
    import numpy as np
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W
    wl = W.eeg_sweep()
    g = wl.grid
    B, order = wl.signals.shape[0], wl.order
    sig = torch.from_numpy(wl.signals).cuda()

    def timed_run(plan, orders, reps, warm):
        resid = torch.empty_like(sig)
        out = plan.alloc_outputs(B, orders)
        for _ in range(warm):
            resid.copy_(sig)
            plan.act_decompose(resid, orders, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            resid.copy_(sig)
            plan.act_decompose(resid, orders, out)
        torch.cuda.synchronize()
        e = out["energy"].cpu().numpy()
        return (time.perf_counter() - t0) / reps, e / e[:, :1]

    new_plan = act.Plan(g, dict_="synth", prec="f32", max_batch=B, refine_steps=wl.refine_steps)
    if TUNE:
        new_plan.act_tune(sig, reps=2)
    t_new, e_new = timed_run(new_plan, order, steps, warmup)
    new_plan.close()
    old_plan = act.Plan(g, dict_="synth", prec="f64", max_batch=B, refine_steps=wl.refine_steps, prior_act=True)
    t_old, e_old = timed_run(old_plan, 10, 1, 0)
    old_plan.close()

    def stat(e, k):
        return [round(float(e[:, k].mean()), 5), round(float(e[:, k].std()), 5)]

    return {"workload": "eeg-sweep", "value": round(g.size * g.n * order * B / t_new / 1e9, 3),
            "unit": "GMAC/s", "ms_per_step": round(t_new * 1e3, 3),
            "mp_iters_per_s": round(order / t_new, 3), "channel_iters_per_s": round(order * B / t_new, 3),
            "dtype": "f32",
            "config": {"workload": "eeg-sweep", "atoms": g.size, "n_samples": g.n, "windows": B, "order": order,
                       "dict": "synth", "refine_steps": wl.refine_steps, "parallelism": "single-gpu"},
            "normalised_residue_mean_std": {f"order_{k}": stat(e_new, k) for k in (5, 10, 50, 100, 200)},
            "prior_act_normalised_residue_mean_std": {f"order_{k}": stat(e_old, k) for k in (5, 10)},
            "prior_act_windows_above_1_at_order_10": int((e_old[:, 10] > 1.0).sum()),
            "residue_act_monotone": bool(np.all(np.diff(e_new, axis=1) <= 1e-12)),
            "prior_act_ms_for_10_orders": round(t_old * 1e3, 3)}


def run_lem(steps: int, warmup: int):
    """The paper's LEM study on synthetic windows (Sec. VII): 19 windows of
    2 s on its EEG ranges, order 10, the hierarchical search with the paper's
    settings (512 LHS samples) against the dense FP64 and FP32-synthesised
    searches; per-window times and normalised residues."""
    import numpy as np
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W
    wl = W.lem_eeg()
    g = wl.grid
    B, order = wl.signals.shape[0], wl.order
    cfg = W.paper_lem_config(samples=512)
    lhs = torch.from_numpy(W.lem_lhs(70, B, order, cfg.samples)).cuda()
    sig = torch.from_numpy(wl.signals).cuda()
    res = {}

    def run(kind, plan):
        resid = torch.empty_like(sig)
        out = plan.alloc_outputs(B, order)
        ts = []
        for rep in range(warmup + steps):
            resid.copy_(sig)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "lem":
                plan.act_lem_decompose(resid, lhs, cfg, order, out)
            else:
                plan.act_decompose(resid, order, out)
            torch.cuda.synchronize()
            if rep >= warmup:
                ts.append(time.perf_counter() - t0)
        e = out["energy"].cpu().numpy()
        nr = e[:, -1] / e[:, 0]
        return {"ms_per_window": round(float(np.mean(ts)) * 1e3 / B, 4),
                "normalised_residue": [round(float(nr.mean()), 5), round(float(nr.std()), 5)],
                "plan_workspace_bytes": int(plan.query(act.Q_WORKSPACE_BYTES))}

    for kind, kw in (("lem", dict(dict_="synth", prec="f64")), ("dense-f64", dict(dict_="synth", prec="f64")),
                     ("dense-f32-synth", dict(dict_="synth", prec="f32"))):
        plan = act.Plan(g, max_batch=B, refine_steps=wl.refine_steps, **kw)
        res[kind] = run(kind, plan)
        plan.close()
    t = res["lem"]["ms_per_window"] * 1e-3
    return {"workload": "lem-eeg", "value": round(order / t, 3), "unit": "MP iters/s per window",
            "ms_per_step": round(res["lem"]["ms_per_window"] * B, 3), "dtype": "f64",
            "config": {"workload": "lem-eeg", "windows": B, "n_samples": g.n, "grid_atoms": g.size, "order": order,
                       "lhs_samples": cfg.samples, "levels": cfg.levels, "topk": cfg.topk,
                       "parallelism": "single-gpu"},
            "modes": res}


def run_refine(steps: int, warmup: int):
    """act_refine on 4096 (residual, start) pairs, 30 L-BFGS iterations each."""
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W
    wl = W.refine_pairs()
    plan = act.Plan(wl.grid, dict_="synth", prec="f64")
    r = torch.from_numpy(wl.signals).cuda()
    th0 = torch.from_numpy(wl.theta0).cuda()
    for _ in range(warmup):
        plan.act_refine(r, th0, wl.refine_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.act_refine(r, th0, wl.refine_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"workload": wl.name, "value": round(r.shape[0] * steps / wall, 2),
            "unit": "refinements/s", "ms_per_step": round(wall * 1e3 / steps, 4),
            "config": {"workload": wl.name, "pairs": r.shape[0], "n_samples": wl.grid.n,
                       "lbfgs_steps": wl.refine_steps}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp32-1x2048",
                    choices=sorted(WORKLOADS) + ["refine-4096", "ragged-1000-f16", "ragged-1000-f32",
                                                 "ragged-1000-f16-cut", "ragged-1000-f16-lag", "eeg-sweep", "lem-eeg"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companions", action="store_true")
    ap.add_argument("--companions", default="fp32-1x2048-synth,lag-f16-1x2048,bf16-64x2048,lag-f16-64x2048,lag-bf16-64x2048,"
                                            "f16-64x2048-synth,f16-64x2048-synth-cut,complex-f32-64x2048-synth,complex-lag-f16-64x2048,"
                                            "ragged-1000-f16,ragged-1000-f16-cut,ragged-1000-f16-lag",
                    help="comma-separated companion workloads of the default run")
    ap.add_argument("--no-tune", action="store_true", help="time the built-in launch shapes (no act_tune)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "refine-4096":
        res = run_refine(args.steps, args.warmup)
        line = {"metric": "refinements/s (4096 pairs x 30 L-BFGS iterations, FP64)", **res,
                "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64", "data": "synthetic"}
        print(json.dumps(line), flush=True)
        return

    if args.workload in ("eeg-sweep", "lem-eeg"):
        res = run_sweep(args.steps, args.warmup) if args.workload == "eeg-sweep" else run_lem(args.steps, args.warmup)
        line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": res.pop("dtype"), "data": "synthetic", "config": res.pop("config")}
        line.update(res)
        print(json.dumps(line), flush=True)
        return
    if args.workload.startswith("ragged-1000"):
        parts = args.workload.split("-")
        res = run_ragged(args.steps, args.warmup, parts[2], parts[-1] == "cut", "lag" if parts[-1] == "lag" else "synth")
        line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": res.pop("dtype"), "data": "synthetic", "config": res.pop("config")}
        line.update(res)
        print(json.dumps(line), flush=True)
        return

    res, wl = run_workload(args.workload, args.steps, args.warmup)
    line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": res.pop("dtype"), "data": "synthetic", "config": res.pop("config")}
    line.update(res)
    if args.workload == "fp32-1x2048" and not args.no_companions:
        comp = {}
        for name in [c for c in args.companions.split(",") if c]:
            if name.startswith("ragged-1000"):
                # the uneven batch (15 orders of 1000 signals, ~3.3e13 MACs per
                # order) takes seconds per step: one timed step after one warm-up
                parts = name.split("-")
                comp[name] = run_ragged(1, 1, parts[2], parts[-1] == "cut", "lag" if parts[-1] == "lag" else "synth")
            else:
                comp[name], _ = run_workload(name, args.steps, args.warmup)
        line["companions"] = comp
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
