#!/usr/bin/env python3
"""Benchmark of the MI355X AMR lattice Boltzmann path (one JSON line on stdout).

Main workload: D3Q27 BGK flow past a square-section cylinder, 256x128x128 root
cells (64x32x32 blocks of 4^3 cells), cylinder side 16 spanning z at x = 64,
inlet u = 0.05, Re 200, 3 levels; static near-wall refinement at t = 0 (frozen)
and vorticity-threshold refinement (theta = 0.1) every 32 coarse steps.  It runs
with FP32 shifted storage (the reported value) and with FP16 shifted storage.
Also reported: the D3Q19 lid-driven cube cavity (64^3 root cells, 3 levels,
Re 400, adaptation every 50 coarse steps).

One benchmark "step" is one pass of the whole hot path: one adaptation period of
coarse time steps (recursive sub-cycled collide/stream, interpolation,
averaging) followed by one adaptation cycle (pre-adaptation sync, criterion,
tagging, refine/coarsen, connectivity rebuild).

value = million lattice-node updates per second of the advancement, counted with
the paper's AMR weighting (Sec. "Solver Performance"), adaptation excluded as
in the paper; the adaptation time is reported per cycle next to it.
"""
from __future__ import annotations

import argparse
import dataclasses
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
# HBM bytes per launch of a kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE, per dispatch), each scaled by what the counter reads for a
# copy of known size: the committed summaries under profiles/ carry one
# "TRAFFIC_JSON {...}" line per kernel and workload, with the hash of the
# kernel sources the counters were taken on.  A summary taken on other sources
# gives no traffic figure (null).
KERNEL_SOURCES = ("paper_2308_08085_amd/csrc/lbm_kernels.hip", "paper_2308_08085_amd/csrc/common.h")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """{key: bytes per launch} from profiles/*.md, for the current kernel sources"""
    out, cur = {}, source_hash()
    pdir = os.path.join(HERE, "profiles")
    for name in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for ln in fh:
                if ln.startswith("TRAFFIC_JSON "):
                    d = json.loads(ln[len("TRAFFIC_JSON "):])
                    if d.get("source_sha") == cur:
                        out[d["key"]] = (d["fetch_kib"] * d["fetch_scale"] + d["write_kib"] * d["write_scale"]) * 1024
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_storage(case, storage, steps, warmup, theta, profile_periods=2, graph=True, tag_kind=None,
                keep_state=False, collision=None):
    """keep_state: also return the tags of every adaptation and the final rho/u
    of the output cells (for the error leg); collision: (kind, s_high) for
    amr_set_collision, else BGK"""
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    g = abi.AmrLbm(case, storage=storage)
    g.set_root_rho_u(case.initial_rho_u())
    if case.interp == 0:
        # sweeps leave out refined blocks none of whose children has an N_SKIP
        # link: leaf results are unchanged bit for bit (the paper's MLUPS count
        # excludes refined blocks anyway)
        g.skip_parents(True)
    if collision is not None:
        g.set_collision(*collision)
    for _ in range(case.dist_levels):  # static near-wall refinement at t = 0
        g.tag(abi.TAG_DISTANCE, d_spec=case.d_spec, freeze=1)
        g.adapt()
    period = case.adapt_every
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    refused = [0]
    steps_ms = {k: 0.0 for k in abi.ADAPT_STEPS}  # device time per adaptation step, summed
    tags_seq = []

    def one_period(profile=False, check=False):
        counts = g.counts().copy()
        ev0.record(g.stream)
        g.step(period, profile=profile, graph=graph and not profile, check_finite=check)
        ev1.record(g.stream)
        g.synchronize()  # the adaptation clock starts once the advancement has finished
        t0 = time.perf_counter()
        if tag_kind == abi.TAG_LADDER:
            tg = g.tag(abi.TAG_LADDER, n_start=-2.0, n_inc=1.0)
        else:
            tg = g.tag(abi.TAG_VORTICITY_REL, theta=theta)
        if keep_state:
            tags_seq.append(tg)
        try:
            st = g.adapt()
            for k, v in st["step_ms"].items():
                steps_ms[k] += v
        except abi.AmrError as e:  # atomic refusal: the mesh is unchanged
            if e.code != abi.AMR_ERR_CAPACITY:
                raise
            refused[0] += 1
        t_adapt = time.perf_counter() - t0
        adv_ms = ev0.elapsed_time(ev1)
        return period * W.mlups_updates(counts, case.dim), adv_ms, t_adapt * 1e3, counts

    for i in range(warmup):
        u, ms, ams, counts = one_period(check=(i == warmup - 1))
        log("[%s] warmup %d/%d: %.1f MLUPS, adapt %.2f ms, blocks/level %s" %
            (storage, i + 1, warmup, u / ms / 1e3, ams, counts.tolist()))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    tot_u = tot_ms = tot_adapt = 0.0
    for k in steps_ms:
        steps_ms[k] = 0.0
    for i in range(steps):
        u, ms, ams, counts = one_period()
        tot_u += u
        tot_ms += ms
        tot_adapt += ams
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    adapt_steps = {k: round(v / steps, 3) for k, v in steps_ms.items()}
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
        "adapt_steps_device_ms": adapt_steps,
        "wall_s": wall,
        "level_blocks": g.counts().tolist(),
        "kernels": {k: {"launches": int(v[0]), "ms": v[1], "blocks": v[2], "bytes": v[3]} for k, v in ks.items()},
        "adaptations_refused_for_capacity": refused[0],
    }
    if keep_state:
        out["tags_seq"] = tags_seq
        out["rho_u"] = g.rho_u_out()
    g.close()
    del g
    torch.cuda.empty_cache()
    return out


def run_batch(steps, warmup, theta, trial_steps=2):
    """the batched set-up: 64 cavities advanced by fused level sweeps"""
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    cases = W.config5_cases()
    stream = torch.cuda.Stream()
    sims = []
    for c in cases:
        g = abi.AmrLbm(c, stream=stream)
        g.set_root_rho_u(c.initial_rho_u())
        sims.append(g)
    b = abi.AmrBatch(sims)
    best, best_ms = b.autotune(trial_steps=trial_steps)
    log("[batch] %d simulations, autotuned shape %s (%.3f ms per coarse step)" % (len(sims), best, best_ms))
    period = cases[0].adapt_every
    live = [True] * len(sims)
    refused = [0]
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def updates():
        return [period * W.mlups_updates(g.counts(), c.dim) for g, c in zip(sims, cases)]

    def one_period():
        u = updates()
        ev0.record(stream)
        b.step(period, graph=True)
        ev1.record(stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for i, g in enumerate(sims):
            if not live[i]:
                continue
            if not np.all(np.isfinite(g.mass_mom())):
                live[i] = False
                continue
            g.tag(abi.TAG_VORTICITY_REL, theta=theta)
            try:
                g.adapt()
            except abi.AmrError as e:  # atomic refusal: the mesh is unchanged
                if e.code != abi.AMR_ERR_CAPACITY:
                    raise
                refused[0] += 1
        t_adapt = time.perf_counter() - t0
        return sum(x for x, ok in zip(u, live) if ok), ev0.elapsed_time(ev1), t_adapt * 1e3

    for i in range(warmup):
        u, ms, ams = one_period()
        log("[batch] warmup %d/%d: %.1f MLUPS, adapt %.1f ms (all members)" % (i + 1, warmup, u / ms / 1e3, ams))
    tot_u = tot_ms = tot_a = 0.0
    for i in range(steps):
        u, ms, ams = one_period()
        tot_u += u
        tot_ms += ms
        tot_a += ams
    # the same members one after another, each replaying its own graph
    u = updates()
    for g in sims:  # capture outside the timed region
        g.step(2, graph=True)
    b.step(0)
    ev0.record(stream)
    for g in sims:
        g.step(period, graph=True)
    ev1.record(stream)
    stream.synchronize()
    seq_ms = ev0.elapsed_time(ev1)
    seq_mlups = sum(x for x, ok in zip(u, live) if ok) / seq_ms / 1e3
    mlups = tot_u / tot_ms / 1e3
    unstable = [cases[i].name for i in range(len(sims)) if not live[i]]
    log("[batch] timed %d periods: %.1f MLUPS fused vs %.1f one by one; %d members non-finite" %
        (steps, mlups, seq_mlups, len(unstable)))
    out = {"workload": "64 lid-driven cavities (32 D2Q9 sides 32-256, 32 D3Q19 sides 32-64), Re log-uniform "
                       "100-3200, 2-4 levels, FP16 shifted storage, adaptation every 50 coarse steps",
           "mlups": round(mlups, 1), "mlups_members_one_by_one": round(seq_mlups, 1),
           "speedup_vs_one_by_one": round(mlups / seq_mlups, 3),
           "adapt_ms_per_cycle_all_members": round(tot_a / steps, 2),
           "tuning": best, "non_finite_members": unstable, "adaptations_refused_for_capacity": refused[0],
           "blocks": int(sum(int(g.counts().sum()) for g in sims))}
    b.close()
    for g in sims:
        g.close()
    del b, sims
    torch.cuda.empty_cache()
    return out


# The paper's drag coefficients (linear / cubic interpolation) and Strouhal
# numbers of the square cylinder at Re 100 with 256 root cells along x, by
# effective finest resolution 256 * 2^(L_max - 1) (Sec. "Flow Past a Square
# Cylinder", table of results).
PAPER_FPSC_256 = {512: (1.581, 1.5010, 0.1469), 1024: (1.584, 1.503, 0.1472),
                  2048: (1.553, 1.500, 0.1473), 4096: (1.508, 1.498, 0.1472)}
# the same table's uniform-grid column: C_D, St
PAPER_FPSC_UNIFORM = {512: (1.513, 0.1470), 1024: (1.501, 0.1473), 2048: (1.501, 0.1473), 4096: (1.499, 0.1472)}


def run_physics(n_x, lmax, interp, storage="f64", t_end=150.0, t_avg=140.0, height=32):
    """C_D and St of the paper's square-cylinder run (n_x root cells along x,
    L_max levels) against the paper's table"""
    from paper_2308_08085_amd import physics, workloads as W

    case = W.fpsc(n_x, lmax, interp, storage=storage, height=height)
    r = physics.run_fpsc(case, n_x, t_end, t_avg, log=log)
    n_eff = n_x * 2 ** (lmax - 1)
    if lmax == 1:
        ref = PAPER_FPSC_UNIFORM.get(n_eff)
        ref = (ref[0], ref[0], ref[1]) if ref else None
    else:
        ref = PAPER_FPSC_256.get(n_eff) if n_x == 256 else None
    return {"workload": case.name, "storage": storage, "n_eff": n_eff, "root_steps": r["root_steps"],
            "wall_s": r["wall_s"], "adapt_s": r["adapt_s"], "samples": r["samples"],
            "C_D_mean": round(r["C_D_mean"], 4),
            "C_L_amplitude": round(r["C_L_amplitude"], 4), "St": round(r["St"], 4),
            "paper": {"C_D": ref[interp], "St": ref[2]} if ref else None,
            "level_blocks_end": r["level_blocks_end"]}


def kernel_rates(res):
    """event-timed rate of each solver kernel over the profiled periods"""
    out = {}
    for k, v in res["kernels"].items():
        if v["launches"] and v["ms"] > 0:
            out[k] = {"launches": v["launches"], "avg_us": round(v["ms"] * 1e3 / v["launches"], 2),
                      "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)}
    return out


def copy_bandwidth(gib=1, reps=10):
    """GB/s (read + write) of a device-to-device copy of `gib` GiB, the practical
    bandwidth ceiling on this machine"""
    import torch
    a = torch.empty(gib << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


COPY_GBS = [None]  # measured once per run
TRAFFIC = {}  # measured_traffic(), read once per run


def uniform_sweep(steps=20):
    """the collide-stream kernel on one uniform periodic level of 384^3 cells
    (D3Q19, FP32 shifted: 4.3 GB per buffer, over 4 x the 256 MB Infinity Cache)"""
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    case = dataclasses.replace(W.cavity(3, 19, 384, 1, 1000.0, storage="f32s", seed=2308092, cap=96 ** 3),
                               periodic=(1, 1, 1))
    g = abi.AmrLbm(case)
    g.set_root_rho_u(case.initial_rho_u())
    g.step(3, graph=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(steps, graph=True)
    e1.record(g.stream)
    g.synchronize()
    mlups = steps * case.nroot * 64 / (e0.elapsed_time(e1) * 1e-3) / 1e6
    g.kernel_stats(reset=True)
    g.step(steps, profile=True)
    n, ms, blocks, byts = g.kernel_stats()["collide_stream"]
    g.close()
    del g
    torch.cuda.empty_cache()
    res = {"kernels": {"collide_stream": {"launches": n, "ms": ms, "blocks": blocks, "bytes": byts}}}
    return {"workload": "uniform periodic D3Q19 level, 384^3 cells (96^3 blocks), FP32 shifted storage",
            "mlups": round(mlups, 1), "roofline": roofline(res, "k_collide_stream<19, F32S, uniform 384^3>")}


def roofline(res, kernel):
    k = res["kernels"]["collide_stream"]
    gbs = k["bytes"] / (k["ms"] * 1e-3) / 1e9
    traffic = TRAFFIC.get(kernel)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": round(traffic) if traffic else None,
            "copy_GBs": round(COPY_GBS[0], 1) if COPY_GBS[0] else None,
            "frac_of_copy": round(gbs / COPY_GBS[0], 4) if COPY_GBS[0] else None,
            "traffic_over_algorithmic": round(traffic * max(k["launches"], 1) / k["bytes"], 3) if traffic else None,
            "kernel": kernel,
            "avg_launch_us": round(k["ms"] * 1e3 / max(k["launches"], 1), 2),
            "bytes_per_launch": round(k["bytes"] / max(k["launches"], 1))}


def replay_error(case, res, storage_ref="f64"):
    """velocity error of a run (res from run_storage with keep_state) against
    the same schedule with FP64 storage and the same tags (the FP64 storage is
    held to the FP64 oracle within 1e-12 by the parity tests)"""
    from paper_2308_08085_amd import abi

    t0 = time.perf_counter()
    g = abi.AmrLbm(case, storage=storage_ref)
    g.set_root_rho_u(case.initial_rho_u())
    for _ in range(case.dist_levels):
        g.tag(abi.TAG_DISTANCE, d_spec=case.d_spec, freeze=1)
        g.adapt()
    for t in res["tags_seq"]:
        g.step(case.adapt_every, graph=True)
        g.tag(tags_in=t)
        try:
            g.adapt()
        except abi.AmrError as e:
            if e.code != abi.AMR_ERR_CAPACITY:
                raise
    ref = g.rho_u_out()
    g.close()
    got = res["rho_u"]
    if ref.shape != got.shape:
        return {"error": "output cells differ"}
    U = float(np.abs(np.asarray(case.face_u)).max())
    du = got[:, 1:4] - ref[:, 1:4]
    out = {"u_l2_rel": float(np.linalg.norm(du) / np.linalg.norm(ref[:, 1:4])),
           "u_max_abs_over_U": float(np.abs(du).max() / U),
           "rho_max_abs": float(np.abs(got[:, 0] - ref[:, 0]).max()),
           "coarse_steps": len(res["tags_seq"]) * case.adapt_every, "reference": "FP64 storage, same tags",
           "seconds": round(time.perf_counter() - t0, 1)}
    log("[error] %s" % out)
    return out


def error_leg(theta):
    """velocity L2 error of the 32- and 16-bit storages on a reduced cavity,
    against the FP64 storage of the same library (which the parity tests hold
    to the FP64 oracle within 1e-12)"""
    from paper_2308_08085_amd import abi, workloads as W

    case = W.cavity(3, 19, 32, 3, 400.0, storage="f32s", seed=2308087, cap=8 * 8 * 8 * 24)
    out = {"case": "D3Q19 cavity 32^3 root cells, 3 levels, Re 400, 100 coarse steps, FP64-storage tags at "
                   "steps 50 and 100 replayed into the other runs; reference: FP64 storage"}
    ru = case.initial_rho_u()
    ref = abi.AmrLbm(case, storage="f64")
    ref.set_root_rho_u(ru)
    tags = []
    for _ in range(2):
        ref.step(50)
        tags.append(ref.tag(abi.TAG_VORTICITY_REL, theta=theta))
        ref.adapt()
    oo = ref.output()
    ref.close()
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


def cpu_baseline(case):
    """The FP64 oracle on the main workload's own mesh (the same near-wall
    refinement at t = 0 as the GPU run, so the same 9.3e5 blocks), on the
    host cores: one collide-stream sweep of levels 0 and 1 on one thread
    pinned to one core, then one whole coarse step on every core the process
    may use"""
    import oracle

    cores = sorted(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    oracle.set_threads(len(cores))
    o = oracle.Oracle(case)
    o.set_root_rho_u(case.initial_rho_u())
    for _ in range(case.dist_levels):
        o.tag(kind=1, d_spec=case.d_spec, freeze=1)
        o.adapt()
    counts = [len(x) for x in o.mesh()["ids"]]
    setup_s = time.perf_counter() - t0
    log("[cpu] oracle set up on the main mesh %s in %.1f s" % (counts, setup_s))
    # one thread on one core: the level-0 and level-1 sweeps
    os.sched_setaffinity(0, {cores[0]})
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.sweep(0)
    o.sweep(1)
    one_s = time.perf_counter() - t0
    os.sched_setaffinity(0, set(cores))
    one_cells = (counts[0] + counts[1]) * case.mb
    log("[cpu] one core: %d cell updates in %.1f s" % (one_cells, one_s))
    # every core: a whole coarse step (every level, interpolation, averaging)
    n = oracle.set_threads(len(cores))
    from paper_2308_08085_amd import workloads as W
    t0 = time.perf_counter()
    o.step(1)
    all_s = time.perf_counter() - t0
    upd = W.mlups_updates(counts, case.dim)
    log("[cpu] %d threads: one coarse step (%.0f M updates) in %.1f s" % (n, upd / 1e6, all_s))
    del o
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(upd / all_s / 1e6, 2), "unit": "MLUPS", "cores": n, "kind": "oracle", "cpu": model,
            "sample": "FP64 oracle on the main workload's mesh after its near-wall refinement (blocks per level %s): "
                      "one coarse step (all levels, interpolation, averaging) on %d threads, %.1f s; MLUPS by the "
                      "paper's leaf-weighted count" % (counts, n, all_s),
            "one_core": {"value": round(one_cells / one_s / 1e6, 3), "unit": "MLUPS", "cores": 1,
                         "sample": "one collide-stream sweep each of levels 0 and 1 (%d cell updates), one thread "
                                   "pinned to one core, %.1f s" % (one_cells, one_s)},
            "setup_s": round(setup_s, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (adaptation periods)")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-leg", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-cavity", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-uniform", action="store_true")
    ap.add_argument("--no-d2q9", action="store_true", help="skip the D2Q9 cavity and cylinder legs")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--physics", action="store_true",
                    help="only the paper's square-cylinder runs: C_D and St against its table")
    ap.add_argument("--physics-nx", type=int, default=256, help="root cells along x")
    ap.add_argument("--physics-levels", default="2,3,4,5", help="L_max values, comma-separated")
    ap.add_argument("--physics-interp", default="linear,cubic")
    ap.add_argument("--physics-storage", default="f64")
    ap.add_argument("--physics-height", type=int, default=32, help="channel height in cylinder diameters")
    ap.add_argument("--physics-uniform", type=int, default=2048,
                    help="also run the uniform grid at each effective resolution up to this one (0: none)")
    ap.add_argument("--physics-t-end", type=float, default=150.0,
                    help="end time in domain-length units; C_D and St come from its last 10 units")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device three times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.physics:
        import torch  # noqa: F401
        from paper_2308_08085_amd import abi
        abi.load()
        for lm in [int(x) for x in args.physics_levels.split(",")]:
            for name in args.physics_interp.split(","):
                r = run_physics(args.physics_nx, lm, {"linear": 0, "cubic": 1}[name], args.physics_storage,
                                args.physics_t_end, args.physics_t_end - 10.0, args.physics_height)
                print(json.dumps({"physics": r}), flush=True)
            if lm > 1 and args.physics_nx * 2 ** (lm - 1) <= args.physics_uniform:
                # the uniform grid at the same effective resolution, for C_D, St and the AMR speedup
                r = run_physics(args.physics_nx * 2 ** (lm - 1), 1, 0, args.physics_storage,
                                args.physics_t_end, args.physics_t_end - 10.0, args.physics_height)
                print(json.dumps({"physics": r}), flush=True)
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2308_08085_amd import abi, workloads as W

    abi.load()
    log("device:", torch.cuda.get_device_name(0))
    TRAFFIC.update(measured_traffic())
    COPY_GBS[0] = copy_bandwidth()
    log("[copy] 1 GiB device-to-device: %.1f GB/s" % COPY_GBS[0])
    main_case = W.config4(cap=W.config4().nroot * 16)
    cav = W.config2()
    theta = main_case.theta
    keep = not args.no_error_leg
    r32 = run_storage(main_case, "f32s", args.steps, args.warmup, theta, keep_state=keep)
    e32 = replay_error(main_case, r32) if keep else None
    r16 = None if args.no_fp16 else run_storage(main_case, "f16s", args.steps, args.warmup, theta, keep_state=keep)
    e16 = replay_error(main_case, r16) if (keep and r16 is not None) else None
    for r in (r32, r16):
        if r is not None:
            r.pop("rho_u", None)
            r.pop("tags_seq", None)
    d2 = None
    if not args.no_d2q9:
        # set-up 1 (D2Q9 FP64 cavity) and set-up 3 (D2Q9 cylinder, FP32 against FP16)
        c1 = W.config1()
        c3 = W.config3(cap=W.config3().nroot * 12)
        d2 = {"cfg1": run_storage(c1, "f64", max(2, args.steps // 2), 2, theta),
              "cfg3_f32s": run_storage(c3, "f32s", args.steps, args.warmup, theta),
              "cfg3_f16s": None if args.no_fp16 else run_storage(c3, "f16s", args.steps, args.warmup, theta)}
    c32 = None if args.no_cavity else run_storage(cav, "f32s", args.steps, args.warmup, theta)
    c16 = None if (args.no_cavity or args.no_fp16) else run_storage(cav, "f16s", args.steps, args.warmup, theta)
    ext = None
    if not args.no_extensions:
        # cubic coarse-to-fine interpolation and the log2 criterion ladder on the same set-up
        cub = dataclasses.replace(main_case, interp=1)
        rc = run_storage(cub, "f32s", max(2, args.steps // 4), 1, theta)
        rl = run_storage(main_case, "f32s", max(2, args.steps // 4), 1, theta, tag_kind=abi.TAG_LADDER)
        ext = {"cubic_interp_f32s": {"mlups": round(rc["mlups"], 1), "kernels": kernel_rates(rc),
                                     "level_blocks_end": rc["level_blocks"]},
               "ladder_criterion_f32s": {"n_start": -2.0, "n_inc": 1.0, "mlups": round(rl["mlups"], 1),
                                         "adapt_ms_per_cycle": round(rl["adapt_ms_per_cycle"], 3),
                                         "adaptations_refused_for_capacity": rl["adaptations_refused_for_capacity"],
                                         "level_blocks_end": rl["level_blocks"]}}
        # moment-space collision (D3Q27; higher moments at 1.2): vector ALU and
        # matrix-core transforms against the BGK runs above, same set-up
        mrt = {"s_high": 1.2}
        for st, base in (("f32s", r32), ("f16s", r16)):
            if base is None:
                continue
            for name, kind in (("vector_alu", abi.COLLIDE_MRT), ("matrix_cores", abi.COLLIDE_MRT_MFMA)):
                rm = run_storage(main_case, st, max(2, args.steps // 4), 1, theta, collision=(kind, 1.2))
                k = rm["kernels"]["collide_stream"]
                mrt["%s_%s" % (name, st)] = {
                    "mlups": round(rm["mlups"], 1), "vs_bgk": round(rm["mlups"] / base["mlups"], 3),
                    "collide_avg_us": round(k["ms"] * 1e3 / max(k["launches"], 1), 1)}
        ext["moment_space_collision"] = mrt
    uni = None if args.no_uniform else uniform_sweep()
    if uni:
        log("[uniform] %s: %.1f MLUPS, collide %.1f GB/s" % (uni["workload"], uni["mlups"], uni["roofline"]["achieved"]))
    bat = None if args.no_batch else run_batch(max(2, args.steps // 2), 2, theta)
    err = None if args.no_error_leg else error_leg(theta)
    cpu = None if args.no_cpu_baseline else cpu_baseline(main_case)
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
            "workload": "D3Q27 BGK flow past a square cylinder, 256x128x128 root cells (64x32x32 blocks of 4^3), "
                        "cylinder side 16 at x = 64 spanning z, inlet u 0.05, Re 200, 3 levels, near-wall "
                        "refinement at t = 0 + vorticity tagging theta 0.1 every 32 coarse steps; FP32 shifted storage",
            "step": "32 coarse steps + 1 adaptation cycle",
            "sweeps": "every leaf and every refined block with an N_SKIP child (AMR_FIELD_SKIP_PARENTS); "
                      "leaf results identical to sweeping every block",
            "level_blocks_end": r32["level_blocks"],
        },
        "adapt_ms_per_cycle": round(r32["adapt_ms_per_cycle"], 3),
        "adapt_steps_device_ms": r32["adapt_steps_device_ms"],
        "mlups_incl_adapt": round(r32["mlups_wall"], 1),
        "roofline": roofline(r32, "k_collide_stream<27, F32S>"),
        "kernels_f32s": kernel_rates(r32),
        "error_f32s_vs_fp64_storage": e32,
        "cpu_baseline": cpu,
    }
    if r16 is not None:
        line["fp16s"] = {"mlups": round(r16["mlups"], 1), "adapt_ms_per_cycle": round(r16["adapt_ms_per_cycle"], 3),
                         "speedup_vs_fp32": round(r16["mlups"] / r32["mlups"], 3),
                         "roofline": roofline(r16, "k_collide_stream<27, F16S>"),
                         "kernels": kernel_rates(r16),
                         "error_vs_fp64_storage": e16,
                         "level_blocks_end": r16["level_blocks"]}
    if c32 is not None:
        line["cavity_d3q19"] = {
            "workload": "D3Q19 lid-driven cube cavity, 64^3 root cells, 3 levels, Re 400, adapt every 50",
            "mlups_f32s": round(c32["mlups"], 1), "adapt_ms_per_cycle_f32s": round(c32["adapt_ms_per_cycle"], 3),
            "roofline_f32s": roofline(c32, "k_collide_stream<19, F32S>"), "level_blocks_end": c32["level_blocks"]}
        if c16 is not None:
            line["cavity_d3q19"]["mlups_f16s"] = round(c16["mlups"], 1)
            line["cavity_d3q19"]["speedup_f16s_vs_f32s"] = round(c16["mlups"] / c32["mlups"], 3)
    if d2 is not None:
        r1, a3, b3 = d2["cfg1"], d2["cfg3_f32s"], d2["cfg3_f16s"]
        line["cavity_d2q9_fp64"] = {
            "workload": "D2Q9 lid-driven cavity, 64^2 root cells, 3 levels, Re 100, FP64, adapt every 100",
            "mlups": round(r1["mlups"], 1), "adapt_ms_per_cycle": round(r1["adapt_ms_per_cycle"], 3),
            "roofline": roofline(r1, "k_collide_stream<9, F64>"), "kernels": kernel_rates(r1),
            "level_blocks_end": r1["level_blocks"]}
        line["cylinder_d2q9"] = {
            "workload": "D2Q9 flow past a square cylinder, 1024x256 root cells, side 32 at x = 256, Re 100, "
                        "4 levels, near-wall refinement at t = 0 + vorticity tagging every 32 coarse steps",
            "mlups_f32s": round(a3["mlups"], 1), "adapt_ms_per_cycle_f32s": round(a3["adapt_ms_per_cycle"], 3),
            "roofline_f32s": roofline(a3, "k_collide_stream<9, F32S>"), "kernels_f32s": kernel_rates(a3),
            "level_blocks_end": a3["level_blocks"]}
        if b3 is not None:
            line["cylinder_d2q9"].update({
                "mlups_f16s": round(b3["mlups"], 1), "adapt_ms_per_cycle_f16s": round(b3["adapt_ms_per_cycle"], 3),
                "speedup_f16s_vs_f32s": round(b3["mlups"] / a3["mlups"], 3),
                "roofline_f16s": roofline(b3, "k_collide_stream<9, F16S>"), "kernels_f16s": kernel_rates(b3)})
    if ext is not None:
        line["extensions"] = ext
    if uni is not None:
        line["uniform_d3q19"] = uni
    if bat is not None:
        line["batched_cfg5"] = bat
    if err is not None:
        line["error_vs_fp64"] = err
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
