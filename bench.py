#!/usr/bin/env python3
"""Throughput of the residue-based ACT matching-pursuit hot path on one GPU.

One step = one act_decompose call: every order of the pursuit (search,
certified FP64 rescoring, refinement, coefficient, update) over one batch of
seeded synthetic signals already resident in HBM.  The default run measures
the metric "GMAC/s + MP iters/s, BF16+rescore vs plain FP32":
  * value: the plain FP32 search of one 2048-sample channel against the
    2,097,152-atom dictionary streamed from an HBM table (10 orders);
  * companions in the same line: the same workload synthesised and on the
    FP16 lag table; 64 channels (20 orders) with the BF16 table, the BF16 and
    FP16 lag tables and the FP16 synthesis (+ FP64 rescoring); complex atoms;
    the uneven batch of 1000 signals of 256..16384 samples (15 orders, lag
    table and support-cut synthesis); the 1x512 FP64 pursuit; 4096
    refinements in FP64 and FP32.

Timing.  The timed steps replay each call's captured hipGraph with phase
timing off: the path the library ships.  A second, untimed pass of direct
launches with the library's phase timing on (HIP events on the launch
stream) gives the per-order phase split and the search kernel's mean launch
time, from which each roofline object is computed.  GMAC/s counts the dense
correlation work atoms x samples x orders x channels (the uneven batch sums
K_i N_i).

Rooflines.  HBM kinds: algorithmic bytes per launch / mean launch time
against 8 TB/s.  Matrix-core kinds: `frac` is the executed MFMA work (counted
by the device for the lag-table and FP16 searches, act_search_executed;
exactly twice the dense work for the factored FP32 synthesis) over the
launch time against the dtype's peak; the dense-equivalent rate, which
counts skipped exact zeros and support cuts as done, sits in its own keys.
Every object also carries the fraction of the peak the repository's own
probes measure on this GPU (streaming read, MFMA loop).

The FP64 CPU oracle is timed on a bounded sample of the primary workload (one
full order) in the cpu_baseline leg, which also reports each form's error
against the oracle on sampled results (scores, selected atoms, energies).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-companions]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "residual-chirplet GMAC/s + MP iters/s, BF16+rescore vs plain FP32, 1 GPU"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32_mfma": 157.3, "bf16_mfma": 2500.0, "f16_mfma": 2500.0, "f64_vector": 78.6}

# The paper's reported speedups, quoted with their hardware as context only
# (other GPUs, CPUs and recorded datasets; not a target for this workload).
PAPER_CONTEXT = {
    "per_epoch_speedup_hybrid_vs_cpu": "6.6x-7.38x: NVIDIA RTX 5070 desktop GPU (CuPy/PyTorch hybrid) vs "
                                       "Intel i9-14900K CPU, EEG epochs, order 10 (abstract; Table "
                                       "'tab:benchmark'; Table 'tab:hardware')",
    "channel_scaling_speedup": "3.94x (1 channel) to 8.22x (10 channels): RTX 5070 vs i9-14900K, CHB-MIT EEG, "
                               "order 10 (Table 'tab:channel_scaling')",
    "note": "the paper reports wall time per epoch only (no GMAC/s, bandwidth or roofline figures); "
            "its numbers are for other hardware and recorded datasets",
}

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
RAGGED = ("ragged-1000-f16-lag", "ragged-1000-f16-cut", "ragged-1000-f16", "ragged-1000-f32")
REFINE = ("refine-4096", "refine-4096-f32")
DEFAULT_COMPANIONS = ("fp32-1x2048-synth,lag-f16-1x2048,bf16-64x2048,lag-f16-64x2048,lag-bf16-64x2048,"
                      "f16-64x2048-synth,f16-64x2048-synth-cut,complex-f32-64x2048-synth,complex-lag-f16-64x2048,"
                      "ragged-1000-f16-lag,ragged-1000-f16-cut,plain-1x512,refine-4096,refine-4096-f32")

TUNE = True  # pick the search's launch shape with act_tune before timing (--no-tune: built-in defaults)
MEASURED_PEAKS = {}  # filled by measure_peaks(): achievable rates of this GPU from the library's probes


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


def _timed_launches(fn, reps: int):
    """Median milliseconds of `reps` launches of fn() on the current stream."""
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def measure_peaks():
    """Achievable peaks of this GPU from the library's probes: a streaming read
    of a 4 GiB buffer (16x the last-level cache) and dependent-free MFMA loops."""
    import torch
    from paper_2607_16629_amd import act
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    buf = torch.zeros(1 << 30, dtype=torch.float32, device="cuda")
    nbytes = buf.numel() * 4
    best, shape = 0.0, None
    for bpc in (2, 4, 8, 16, 32):  # launch shapes: the best one is the achievable rate
        act.probe_read(buf, bpc, sink)
        ms = _timed_launches(lambda: act.probe_read(buf, bpc, sink), 7)
        if nbytes / (ms * 1e-3) / 1e9 > best:
            best, shape = nbytes / (ms * 1e-3) / 1e9, bpc
    peaks = {"hbm_read_gbs": round(best, 1), "hbm_read_blocks_per_cu": shape}
    # a library reduction over the same buffer, as a cross-check of the probe
    ms = _timed_launches(lambda: buf.sum(), 5)
    peaks["torch_sum_read_gbs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    del buf
    for prec, iters in (("bf16", 6000), ("f16", 6000), ("f32", 3000)):
        best = 0.0
        for bpc in (1, 2, 4):
            flops = act.probe_mfma(prec, iters, bpc, sink)
            ms = _timed_launches(lambda: act.probe_mfma(prec, iters, bpc, sink), 5)
            best = max(best, flops / (ms * 1e-3) / 1e12)
        peaks[f"{prec}_mfma_tflops"] = round(best, 1)
    torch.cuda.synchronize()
    return peaks


def _measured(kind: str):
    key = {"hbm": "hbm_read_gbs", "mfma_f32": "f32_mfma_tflops", "mfma_f16": "f16_mfma_tflops",
           "mfma_bf16": "bf16_mfma_tflops"}.get(kind)
    return MEASURED_PEAKS.get(key) if key else None


def _phase_pass(plan, step, steps: int):
    """Direct launches with the library's phase timing on: (per-order phase
    milliseconds, mean search launch ms, executed MFMA flops per launch)."""
    import torch
    counts = plan.dict in ("lag",) or (plan.dict == "synth" and plan.prec == "f16")
    if counts:
        plan.search_executed()  # discard the timed region's counts
    plan.act_timing_enable(True)
    plan.act_timing_read()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    phases = plan.act_timing_read()
    plan.act_timing_enable(False)
    executed = None
    if counts:
        f, n = plan.search_executed()
        executed = f / max(n, 1)
    s_ms, s_n = phases["search"]
    per_order = {k: round(v[0] / max(v[1], 1), 5) for k, v in phases.items()}
    return per_order, s_ms / max(s_n, 1), executed


def _mfma_roofline(kind, algo, executed, source, search_ms, kname, traffic=None):
    peak = PEAK_TFLOPS[kind[5:] + "_mfma"]
    ach = executed / (search_ms * 1e-3) / 1e12
    dense = algo / (search_ms * 1e-3) / 1e12
    meas = _measured(kind)
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "traffic": traffic, "kernel": kname, "avg_launch_ms": round(search_ms, 5),
            "executed_mfma_flops_per_launch": executed, "executed_source": source,
            "algorithmic_flops_per_launch": algo,
            "dense_equivalent_tflops": round(dense, 3), "dense_equivalent_frac": round(dense / peak, 4),
            "measured_peak": meas, "frac_of_measured_peak": round(ach / meas, 4) if meas else None}


def _keep_results(plan, out, channels, order, sig_np, grid, complex_atoms, corr=True):
    """Small copies of the GPU's results for the oracle report: the pursuit of
    the given channels and (plain plans) scores of three atom ranges."""
    import numpy as np
    keep = {"grid": grid, "channels": list(channels), "order": order, "complex": complex_atoms,
            "signals": sig_np[list(channels)].copy()}
    for k in ("index", "theta", "coef", "energy"):
        keep[k] = out[k].cpu().numpy()[list(channels)].copy()
    if corr:
        K = grid.size
        keep["ranges"] = [(0, 1024), (K // 2 - 333, 1024), (K - 1024, 1024)]
        keep["scores"] = [plan.act_correlate(sig_np[list(channels)], b, c).cpu().numpy() for b, c in keep["ranges"]]
    return keep


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
    for _ in range(max(warmup, 1)):  # the first call captures the graph that the timed steps replay
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags = out["flags"].cpu().numpy()
    phases, search_ms, executed = _phase_pass(plan, step, min(steps, 3))
    chans = [0] if B == 1 else [0, B - 1]
    keep = _keep_results(plan, out, chans, order, wl.signals, g, bool(plan_kw.get("complex_atoms")))
    # the lag-table search of 32+ channels keeps the residual copies in LDS
    # unless the tuner chose the staged tiles (launch-shape form 1)
    resident = (plan_kw["dict_"] == "lag" and B >= 32
                and plan.query(act.Q_LAG_RESIDENT) == 1 and (shape is None or shape.get("form", 0) == 0))
    plan.close()

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
        "timing": "hipGraph replays, phase timing off; phases and launch times from a separate pass",
        "phases_ms_per_order": phases,
        "candidate_overflow_channels": int(((flags & act.FLAG_CAND_OVERFLOW) != 0).sum()),
        "launch_shape": shape,
        "_keep": keep,
    }
    kname, ksrc = KERNELS[(plan_kw["dict_"], plan_kw["prec"])]
    if resident:
        kname = "k_search_lag_rs"
        res["phases_note"] = "rerun: the emission pass of the resident form (flagged units scored again)"
    if kind == "hbm":
        algo_bytes = g.size * g.n * elt + B * g.n * elt
        achieved = algo_bytes / (search_ms * 1e-3) / 1e9
        traffic = committed_traffic(wl.name, source_sha(ksrc, "act_emit.h"))
        meas = _measured("hbm")
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": traffic, "kernel": kname,
                           "algorithmic_bytes_per_launch": algo_bytes,
                           "avg_launch_ms": round(search_ms, 5),
                           "measured_peak": meas, "frac_of_measured_peak": round(achieved / meas, 4) if meas else None}
        if plan_kw["prec"] == "bf16":
            flops = 2.0 * g.size * g.n * B
            res["roofline"]["mfma_frac_of_bf16_peak"] = round(
                flops / (search_ms * 1e-3) / (PEAK_TFLOPS["bf16_mfma"] * 1e12), 4)
    elif kind in ("mfma_f32", "mfma_f16", "mfma_bf16"):
        # dense correlation flops (complex atoms: both parts)
        algo = 2.0 * g.size * g.n * B * (2 if plan_kw.get("complex_atoms") else 1)
        if executed is not None:
            source = "device count (act_search_executed)"
        else:
            # the factored FP32 synthesis runs both products of every sample
            executed, source = 2.0 * algo, "factored synthesis: 2 x dense (every stage runs)"
        lag = plan_kw["dict_"] == "lag"
        traffic = committed_traffic(name, source_sha(ksrc, "act_emit.h")) if lag else None
        res["roofline"] = _mfma_roofline(kind, algo, executed, source, search_ms, kname, traffic)
    else:
        # FP64 on-the-fly synthesis, ~60 FP64 operations per atom sample
        ops = g.size * g.n * B * 60
        achieved = ops / (search_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS["f64_vector"]
        res["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                           "kernel": kname, "avg_launch_ms": round(search_ms, 5),
                           "ops_per_atom_sample": 60}
    return res, wl


def run_ragged(steps: int, warmup: int, prec: str = "f16", cut: bool = False, dict_: str = "synth"):
    """Uneven batch: 1000 signals of log-uniform length 256..16384 in one
    act_decompose call, each with its own grid (floor(N/32) time centres,
    64 f_c x 32 c x 16 dt), 15 orders, FP16 lag table or synthesised search
    + FP64 rescoring."""
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
    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags = out["flags"].cpu().numpy()
    srt = np.argsort(lens, kind="stable")
    pick = [int(srt[0]), int(srt[len(srt) // 2])]
    keep = {"ragged": True, "picks": []}
    for b in pick:
        n, o = int(lens[b]), int(wl.offsets[b])
        keep["picks"].append({"b": b, "grid": wl.grids[b], "signal": wl.signals[o:o + n].copy(),
                              **{k: out[k][b].cpu().numpy().copy() for k in ("index", "theta", "coef", "energy")}})
    keep["order"] = order
    phases, search_ms, executed = _phase_pass(plan, step, 1)
    plan.close()
    macs = float(sum((int(n) // 32) * per_tc * int(n) for n in lens))  # dense MACs of one order
    algo = 2.0 * macs
    kind = prec + "_mfma"
    kname, _ = KERNELS[(dict_, prec)]
    lag = dict_ == "lag"
    if executed is not None:
        source = "device count (act_search_executed)"
    else:
        executed, source = 2.0 * algo, "factored synthesis: 2 x dense (every stage runs)"
    roof = _mfma_roofline("mfma_" + prec, algo, executed, source, search_ms, kname + ("" if lag else "_ragged"))
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
            "timing": "hipGraph replays, phase timing off; phases and launch times from a separate pass",
            "phases_ms_per_order": phases,
            "candidate_overflow_channels": int(((flags & act.FLAG_CAND_OVERFLOW) != 0).sum()),
            "launch_shape": shape, "roofline": roof, "_keep": keep}


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
        for _ in range(max(warm, 1)):
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


def run_refine(steps: int, warmup: int, dtype: str = "f64"):
    """act_refine on 4096 (residual, start) pairs, 30 L-BFGS iterations each,
    with FP64 or FP32 arithmetic."""
    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W
    wl = W.refine_pairs()
    plan = act.Plan(wl.grid, dict_="synth", prec="f64")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = torch.from_numpy(wl.signals).cuda().to(tdt)
    th0 = torch.from_numpy(wl.theta0).cuda()
    for _ in range(max(warmup, 1)):
        th, J, fl = plan.act_refine(r, th0, wl.refine_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        th, J, fl = plan.act_refine(r, th0, wl.refine_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pick = list(range(0, r.shape[0], 256))
    import numpy as np
    sig_in = wl.signals if dtype == "f64" else wl.signals.astype(np.float32).astype(np.float64)
    keep = {"refine": True, "grid": wl.grid, "pick": pick, "signals": sig_in[pick].copy(),
            "theta0": wl.theta0[pick].copy(), "theta": th.cpu().numpy()[pick].copy(), "J": J.cpu().numpy()[pick].copy(),
            "steps": wl.refine_steps, "dtype": dtype}
    plan.close()
    return {"workload": wl.name + ("" if dtype == "f64" else "-f32"), "value": round(r.shape[0] * steps / wall, 2),
            "unit": "refinements/s", "ms_per_step": round(wall * 1e3 / steps, 4), "dtype": dtype,
            "config": {"workload": wl.name, "pairs": r.shape[0], "n_samples": wl.grid.n,
                       "lbfgs_steps": wl.refine_steps, "dtype": dtype},
            "_keep": keep}


# --------------------------------------------------------------------------
# cpu_baseline leg: the FP64 oracle (test infrastructure) on the host cores
# --------------------------------------------------------------------------

def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _gpu_chain(oracle, grid, s, keep_row, order, complex_atoms):
    """The GPU's residual before each order, rebuilt in FP64 from its atoms."""
    import numpy as np
    r = np.array(s, dtype=np.float64)
    rs = [r.copy()]
    for k in range(order):
        th = keep_row["theta"][k]
        if complex_atoms:
            u, v = oracle.atom_complex(grid.fs, grid.n, th)
            r = r - (keep_row["coef"][k][0] * u + keep_row["coef"][k][1] * v)
        else:
            gu, _ = oracle.atom_unit(grid.fs, grid.n, th)
            r = r - keep_row["coef"][k] * gu
        rs.append(r.copy())
    return rs


def oracle_report(results: dict, exhaustive_orders: int = 2):
    """Error of each form against the FP64 oracle on sampled results: scores
    of 3 x 1024 atoms per kept channel (max |p_gpu - p_oracle| / |r|), the
    selected atoms of the first orders of channel 0 against the oracle's
    exhaustive arg-max on the GPU's own residual (identical rows scored
    once), and every order's energy against the GPU chain rebuilt in FP64."""
    import numpy as np
    import oracle
    rep = {}
    pending = {}  # (grid, complex) -> list of (workload, order, residual, gpu index)
    for name, res in results.items():
        keep = res.get("_keep")
        if not keep:
            continue
        if keep.get("refine"):
            # matched by optimum: the runs may end in different local maxima of J
            g = keep["grid"]
            th_o, J_o, _ = oracle.refine_many(g, keep["signals"], keep["theta0"], keep["steps"])
            h = np.array([oracle.refine_scales(g, t) for t in keep["theta0"]])
            du = np.max(np.abs(keep["theta"] - th_o) / np.where(h > 0, h, 1.0), axis=1)
            J_at = np.array([oracle.objective(g.fs, t, r)[0] for t, r in zip(keep["theta"], keep["signals"])])
            same = du <= 0.05
            rel = np.abs(J_at - J_o) / np.maximum(J_o, 1e-300)
            rep[name] = {"pairs_checked": len(keep["pick"]), "at_oracle_optimum": int(same.sum()),
                         "J_rel_err_max_at_oracle_optimum": float(rel[same].max()) if same.any() else None,
                         "J_over_oracle_J_other_pairs": [float((J_at / J_o)[~same].min()),
                                                         float((J_at / J_o)[~same].max())] if (~same).any() else None,
                         "reported_J_rel_err_max": float(np.max(np.abs(keep["J"] - J_at) / np.maximum(J_at, 1e-300)))}
            continue
        if keep.get("ragged"):
            e_err = 0.0
            for pk in keep["picks"]:
                rs = _gpu_chain(oracle, pk["grid"], pk["signal"], pk, keep["order"], False)
                for k in range(keep["order"]):
                    e = float(rs[k + 1] @ rs[k + 1])
                    e_err = max(e_err, abs(pk["energy"][k + 1] - e) / max(e, 1e-300))
            rep[name] = {"signals_checked": [int(p["b"]) for p in keep["picks"]], "energy_rel_err_max": e_err}
            continue
        g, cplx, order = keep["grid"], keep["complex"], keep["order"]
        entry = {}
        # scores against the oracle on three atom ranges, every kept channel
        worst = 0.0
        for (b0, cnt), p in zip(keep["ranges"], keep["scores"]):
            ref = oracle.correlate_many(g, keep["signals"], b0, cnt, complex_atoms=cplx)
            for c in range(ref.shape[0]):
                worst = max(worst, float(np.max(np.abs(p[c] - ref[c]))) / float(np.linalg.norm(keep["signals"][c])))
        entry["score_err_max_over_rnorm"] = worst
        entry["score_atoms_checked_per_channel"] = int(sum(c for _, c in keep["ranges"]))
        # energies of every order of every kept channel against the rebuilt chain
        e_err = 0.0
        for c in range(len(keep["channels"])):
            row = {k: keep[k][c] for k in ("theta", "coef", "energy")}
            rs = _gpu_chain(oracle, g, keep["signals"][c], row, order, cplx)
            for k in range(order):
                e = float(rs[k + 1] @ rs[k + 1])
                e_err = max(e_err, abs(keep["energy"][c][k + 1] - e) / max(e, 1e-300))
            if c == 0:
                kk = min(exhaustive_orders, order) if g.size > 100000 else order
                for k in range(kk):
                    pending.setdefault((g, cplx), []).append((name, k, rs[k], int(keep["index"][0][k])))
        entry["energy_rel_err_max"] = e_err
        rep[name] = entry
    # exhaustive arg-max, one oracle pass per (grid, atom kind)
    t_exh = 0.0
    for (g, cplx), rows in pending.items():
        t0 = time.perf_counter()
        uniq, where = [], []
        for _, _, r, _ in rows:
            for j, u in enumerate(uniq):
                if np.array_equal(u, r):
                    where.append(j)
                    break
            else:
                where.append(len(uniq))
                uniq.append(r)
        idx, gap, _ = oracle.argmax_many(g, np.array(uniq), complex_atoms=cplx)
        t_exh += time.perf_counter() - t0
        for (name, k, _, gi), j in zip(rows, where):
            e = rep[name].setdefault("index_agreement", {"orders_checked": 0, "identical": 0, "gap_excused": 0})
            e["orders_checked"] += 1
            if gi == int(idx[j]):
                e["identical"] += 1
            elif gap[j] <= 1e-6:
                e["gap_excused"] += 1
    return rep, t_exh


def cpu_baseline(wl, results: dict):
    """The FP64 oracle on the host cores: one full order of the primary
    workload's pursuit (exhaustive correlation of every atom, arg-max,
    refinement, update), scaled to the metric's GMAC/s, plus the error of each
    benchmarked form against the oracle."""
    import oracle
    g = wl.grid
    t0 = time.perf_counter()
    oracle.decompose(g, wl.signals[:1], 1, refine_steps=wl.refine_steps)
    dt = time.perf_counter() - t0
    errors, t_exh = oracle_report(results)
    return {"value": round(g.size * g.n / dt / 1e9, 4), "unit": "GMAC/s",
            "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"one full order (exhaustive FP64 correlation of {g.size} atoms x {g.n} samples, arg-max, "
                      f"{wl.refine_steps}-step refinement, update) of the {wl.order} orders of {wl.name} "
                      f"channel 0: {dt:.1f} s, OpenMP over atoms",
            "oracle_seconds": round(dt, 2),
            "errors_vs_oracle": errors,
            "errors_vs_oracle_note": "score error: max |p_gpu - p_oracle| / |r| over 3 x 1024 atoms per kept "
                                     "channel; selection: the GPU's atom vs the oracle's exhaustive arg-max on the "
                                     "GPU's own residual (orders 0-1 of channel 0 on 2M-atom grids, all orders on "
                                     "the 65,536-atom grid); energies: every order of the kept channels vs the GPU "
                                     "chain rebuilt in FP64; refinement: J and theta of 16 pairs vs the oracle's "
                                     f"L-BFGS; exhaustive passes took {t_exh:.1f} s"}


def _strip(res):
    return {k: v for k, v in res.items() if not k.startswith("_")}


def _run_named(name, steps, warmup):
    if name in RAGGED:
        parts = name.split("-")
        # the uneven batch (~3.3e13 dense MACs per order) takes 0.2-2 s per step:
        # one timed step after one warm-up
        return run_ragged(1, 1, parts[2], parts[-1] == "cut", "lag" if parts[-1] == "lag" else "synth")
    if name in REFINE:
        return run_refine(steps, warmup, "f32" if name.endswith("f32") else "f64")
    return run_workload(name, steps, warmup)[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp32-1x2048",
                    choices=sorted(WORKLOADS) + list(REFINE) + list(RAGGED) + ["eeg-sweep", "lem-eeg"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companions", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the achievable-peak probes")
    ap.add_argument("--companions", default=DEFAULT_COMPANIONS,
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
    if not args.no_peaks:
        MEASURED_PEAKS.update(measure_peaks())

    base = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload in REFINE:
        res = _strip(run_refine(args.steps, args.warmup, "f32" if args.workload.endswith("f32") else "f64"))
        line = {"metric": f"refinements/s (4096 pairs x 30 L-BFGS iterations, {res['dtype'].upper()})", **res,
                **base}
        print(json.dumps(line), flush=True)
        return
    if args.workload in ("eeg-sweep", "lem-eeg") or args.workload in RAGGED:
        if args.workload == "eeg-sweep":
            res = run_sweep(args.steps, args.warmup)
        elif args.workload == "lem-eeg":
            res = run_lem(args.steps, args.warmup)
        else:
            parts = args.workload.split("-")
            res = _strip(run_ragged(args.steps, args.warmup, parts[2], parts[-1] == "cut",
                                    "lag" if parts[-1] == "lag" else "synth"))
        line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), **base,
                "ms_per_step": res.pop("ms_per_step"), "dtype": res.pop("dtype"), "config": res.pop("config")}
        line.update(res)
        print(json.dumps(line), flush=True)
        return

    res, wl = run_workload(args.workload, args.steps, args.warmup)
    kept = {args.workload: res}
    line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), **base,
            "ms_per_step": res.pop("ms_per_step"), "dtype": res.pop("dtype"), "config": res.pop("config")}
    line.update(_strip(res))
    if MEASURED_PEAKS:
        line["measured_peaks"] = dict(MEASURED_PEAKS, note="the library's own probes on this GPU "
                                                           "(act_probe_read, act_probe_mfma)")
    line["paper_context"] = PAPER_CONTEXT
    if args.workload == "fp32-1x2048" and not args.no_companions:
        comp = {}
        for name in [c for c in args.companions.split(",") if c]:
            r = _run_named(name, args.steps, args.warmup)
            kept[name] = r
            comp[name] = _strip(r)
        line["companions"] = comp
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, kept)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
