#!/usr/bin/env python3
"""Benchmark of the MI355X AMR lattice Boltzmann path (one JSON line on stdout).

Workload: the D3Q19 BGK lid-driven cube cavity, 64^3 root cells (16^3 blocks of
4^3 cells), 3 grid levels, Re 400, lid speed 0.05, vorticity-threshold
refinement (theta = 0.1) every 50 coarse steps, seeded +-1e-4 velocity noise.
One benchmark "step" is one pass of the whole hot path: 50 coarse time steps
(recursive sub-cycled collide/stream, interpolation, averaging) followed by one
adaptation cycle (pre-adaptation sync, criterion, tagging, refine/coarsen,
connectivity rebuild).  It runs with FP32 shifted storage (the reported value)
and with FP16 shifted storage.

value = million lattice-node updates per second of the advancement, counted with
the paper's AMR weighting (Sec. "Solver Performance"), adaptation excluded as
in the paper; the adaptation time is reported per cycle next to it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "AMR-LBM MLUPS (FP32 vs FP16-storage) + adapt ms/cycle; % HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_storage(case, storage, steps, warmup, theta, profile_periods=2):
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    g = abi.AmrLbm(case, storage=storage)
    g.set_root_rho_u(case.initial_rho_u())
    period = case.adapt_every
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def one_period(profile=False):
        counts = g.counts().copy()
        ev0.record(g.stream)
        g.step(period, profile=profile)
        ev1.record(g.stream)
        t0 = time.perf_counter()
        g.tag(abi.TAG_VORTICITY_REL, theta=theta)
        g.adapt()
        t_adapt = time.perf_counter() - t0
        adv_ms = ev0.elapsed_time(ev1)
        return period * W.mlups_updates(counts, case.dim), adv_ms, t_adapt * 1e3, counts

    for i in range(warmup):
        u, ms, ams, counts = one_period()
        log("[%s] warmup %d/%d: %.1f MLUPS, adapt %.2f ms, blocks/level %s" %
            (storage, i + 1, warmup, u / ms / 1e3, ams, counts.tolist()))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    tot_u = tot_ms = tot_adapt = 0.0
    for i in range(steps):
        u, ms, ams, counts = one_period()
        tot_u += u
        tot_ms += ms
        tot_adapt += ams
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log("[%s] timed %d steps: %.1f MLUPS (advance), %.2f ms adapt/cycle, wall %.3f s, blocks/level %s" %
        (storage, steps, tot_u / tot_ms / 1e3, tot_adapt / steps, wall, g.counts().tolist()))
    # kernel event timing of the dominant kernel, on the handle's stream
    g.kernel_stats(reset=True)
    for _ in range(profile_periods):
        one_period(profile=True)
    ks = g.kernel_stats()
    out = {
        "mlups": tot_u / tot_ms / 1e3,
        "mlups_wall": tot_u / wall / 1e6,
        "adv_ms_per_step": tot_ms / steps,
        "adapt_ms_per_cycle": tot_adapt / steps,
        "wall_s": wall,
        "level_blocks": g.counts().tolist(),
        "kernels": {k: {"launches": int(v[0]), "ms": v[1], "blocks": v[2], "bytes": v[3]} for k, v in ks.items()},
    }
    g.close()
    del g
    torch.cuda.empty_cache()
    return out


def roofline(res):
    k = res["kernels"]["collide_stream"]
    gbs = k["bytes"] / (k["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_collide_stream<19, F32S>",
            "avg_launch_us": round(k["ms"] * 1e3 / max(k["launches"], 1), 2),
            "bytes_per_launch": round(k["bytes"] / max(k["launches"], 1))}


def error_leg(theta):
    """velocity L2 error of the GPU storages against the FP64 oracle on a reduced cavity"""
    import oracle
    from paper_2308_08085_amd import abi, workloads as W

    case = W.cavity(3, 19, 32, 3, 400.0, storage="f32s", seed=2308087, cap=8 * 8 * 8 * 24)
    out = {"case": "D3Q19 cavity 32^3 root cells, 3 levels, Re 400, 100 coarse steps, oracle tags at steps "
                   "50 and 100 replayed into the GPU runs"}
    ru = case.initial_rho_u()
    o = oracle.Oracle(case)
    o.set_root_rho_u(ru)
    tags = []
    for _ in range(2):
        o.step(50)
        tags.append(o.tag(kind=0, theta=theta))
        o.adapt()
    oo = o.output()
    for storage in ("f32s", "f16s", "bf16s"):
        g = abi.AmrLbm(case, storage=storage)
        g.set_root_rho_u(ru)
        for t in tags:
            g.step(50)
            g.tag(tags_in=t)
            g.adapt()
        og = g.output()
        g.close()
        if not (np.array_equal(oo["blk"], og["blk"]) and np.array_equal(oo["cell"], og["cell"])):
            out[storage] = "output cells differ"
            continue
        du = np.linalg.norm(og["u"] - oo["u"]) / np.linalg.norm(oo["u"])
        out[storage] = {"u_l2_rel": float(du), "rho_max_abs": float(np.abs(og["rho"] - oo["rho"]).max())}
    return out


def cpu_baseline(theta, seconds=20.0):
    """the FP64 oracle on a bounded sample of the same workload, one host thread"""
    import oracle
    from paper_2308_08085_amd import workloads as W

    case = W.config2()
    o = oracle.Oracle(case)
    o.set_root_rho_u(case.initial_rho_u())
    tot_u = tot_s = 0.0
    n = 0
    adapt_s = None

    def counts():
        return [len(x) for x in o.mesh()["ids"]]

    t_begin = time.perf_counter()
    while time.perf_counter() - t_begin < seconds:
        c = counts()
        t0 = time.perf_counter()
        o.step(1)
        dt = time.perf_counter() - t0
        tot_u += W.mlups_updates(c, case.dim)
        tot_s += dt
        n += 1
        if n == 10 and adapt_s is None:
            t0 = time.perf_counter()
            o.tag(kind=0, theta=theta)
            o.adapt()
            adapt_s = time.perf_counter() - t0
    return {"value": round(tot_u / tot_s / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "adapt_ms_per_cycle": round(adapt_s * 1e3, 1) if adapt_s else None,
            "sample": "same cavity set-up, FP64 oracle, one thread: %d coarse steps from the initial field "
                      "with one vorticity adaptation after step 10 (%.1f s of stepping)" % (n, tot_s)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (adaptation periods)")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-leg", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    abi.load()
    case = W.config2()
    theta = case.theta
    log("device:", torch.cuda.get_device_name(0))
    r32 = run_storage(case, "f32s", args.steps, args.warmup, theta)
    r16 = None if args.no_fp16 else run_storage(case, "f16s", args.steps, args.warmup, theta)
    err = None if args.no_error_leg else error_leg(theta)
    cpu = None if args.no_cpu_baseline else cpu_baseline(theta)
    line = {
        "metric": METRIC,
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["wall_s"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "D3Q19 BGK lid-driven cube cavity, 64^3 root cells (16^3 blocks of 4^3), 3 levels, "
                        "Re 400, lid u 0.05, vorticity tagging theta 0.1 every 50 coarse steps; FP32 shifted storage",
            "step": "50 coarse steps + 1 adaptation cycle",
            "level_blocks_end": r32["level_blocks"],
        },
        "adapt_ms_per_cycle": round(r32["adapt_ms_per_cycle"], 3),
        "mlups_incl_adapt": round(r32["mlups_wall"], 1),
        "roofline": roofline(r32),
        "cpu_baseline": cpu,
    }
    if r16 is not None:
        line["fp16s"] = {"mlups": round(r16["mlups"], 1), "adapt_ms_per_cycle": round(r16["adapt_ms_per_cycle"], 3),
                         "speedup_vs_fp32": round(r16["mlups"] / r32["mlups"], 3),
                         "roofline_frac": roofline(r16)["frac"], "level_blocks_end": r16["level_blocks"]}
    if err is not None:
        line["error_vs_fp64_oracle"] = err
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
