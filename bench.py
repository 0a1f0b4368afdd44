#!/usr/bin/env python3
"""Throughput of the residue-based ACT matching-pursuit hot path on one GPU.

One step = one act_decompose call: every order of the pursuit (search,
certified FP64 rescoring, refinement, coefficient, update) over one batch of
seeded synthetic signals that are already resident in HBM.  Prints one JSON
line: GMAC/s of the dense correlation work (atoms x samples x orders x
channels per second), MP iterations/s, a roofline object for the search
kernel measured live with HIP events on the launch stream, and the FP64 CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "residual-chirplet GMAC/s + MP iters/s, BF16+rescore vs plain FP32, 1 GPU"
HBM_PEAK_GBS = 8000.0

# name -> (workload factory, plan kwargs, bound, element bytes of the streamed table)
WORKLOADS = {
    "fp32-1x2048": ("fp32_1x2048", dict(dict_="table", prec="f32"), "hbm", 4),
    "plain-1x512": ("plain_1x512", dict(dict_="synth", prec="f64"), "alu", 0),
    "bf16-64x2048": ("batched_64x2048", dict(dict_="table", prec="bf16"), "hbm", 2),
}


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
    return {"value": count * g.n / dt / 1e9, "unit": "GMAC/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"order-1 correlation of channel 0 against atoms [0, {count}) of {g.size} "
                      f"({dt:.1f} s, FP64, OpenMP over atoms)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp32-1x2048", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_2607_16629_amd import act
    from paper_2607_16629_amd import workloads as W

    factory, plan_kw, bound, elt = WORKLOADS[args.workload]
    wl = getattr(W, factory)()
    g = wl.grid
    B, order = wl.signals.shape[0], wl.order
    torch.cuda.set_device(0)
    plan = act.Plan(g, max_batch=B, refine_steps=wl.refine_steps, **plan_kw)
    sig = torch.from_numpy(wl.signals).cuda()
    resid = torch.empty_like(sig)
    out = plan.alloc_outputs(B, order)

    def step():
        resid.copy_(sig)
        plan.act_decompose(resid, order, out)

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.act_timing_enable(True)
    plan.act_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = plan.act_timing_read()
    plan.act_timing_enable(False)

    macs_per_step = g.size * g.n * order * B
    ms_step = wall * 1e3 / args.steps
    value = macs_per_step * args.steps / wall / 1e9
    s_ms, s_n = phases["search"]
    search_ms = s_ms / max(s_n, 1)
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "GMAC/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": plan_kw["prec"], "data": "synthetic",
        "config": {"workload": wl.name, "atoms": g.size, "n_samples": g.n, "channels": B,
                   "order": order, "dict": plan_kw["dict_"], "refine_steps": wl.refine_steps,
                   "parallelism": "single-gpu"},
        "mp_iters_per_s": round(order * args.steps / wall, 3),
        "channel_iters_per_s": round(order * B * args.steps / wall, 3),
        "search_only_gmac_per_s": round(g.size * g.n * B / (search_ms * 1e-3) / 1e9, 3),
        "phases_ms_per_order": {k: round(v[0] / max(v[1], 1), 5) for k, v in phases.items()},
    }
    if bound == "hbm":
        algo_bytes = g.size * g.n * elt + B * g.n * elt
        achieved = algo_bytes / (search_ms * 1e-3) / 1e9
        sha = source_sha({"f32": "act_search_f32t.hip", "bf16": "act_search_bf16.hip"}[plan_kw["prec"]],
                         "act_emit.h")
        traffic = committed_traffic(wl.name, sha)
        kern = {"f32": "k_search_f32_table", "bf16": "k_search_bf16_table"}[plan_kw["prec"]]
        line["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                            "traffic": traffic, "kernel": kern,
                            "algorithmic_bytes_per_launch": algo_bytes,
                            "avg_launch_ms": round(search_ms, 5)}
        if plan_kw["prec"] == "bf16":
            flops = 2.0 * g.size * g.n * B
            line["roofline"]["mfma_frac_of_bf16_peak"] = round(flops / (search_ms * 1e-3) / 2.5e15, 4)
    else:
        # FP64 on-the-fly synthesis: counted as FP64 ALU work per sample
        # (exp + cospi + the dot products ~ 60 FP64 ops); reported against
        # the FP64 vector peak.
        ops = g.size * g.n * B * 60
        achieved = ops / (search_ms * 1e-3) / 1e12
        line["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": 78.6,
                            "unit": "TFLOP/s", "frac": round(achieved / 78.6, 4), "traffic": None,
                            "kernel": "k_search_f64", "avg_launch_ms": round(search_ms, 5)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
