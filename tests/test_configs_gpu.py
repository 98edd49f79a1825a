"""Benchmark set-ups over their whole schedules against the oracle: adaptation
after coarse step k when k is a multiple of the adaptation period and below the
total, vorticity tagging with theta = 0.1.

Set-up 1 runs next to the oracle in the test.  The longer schedules (set-up 2's
2000 coarse steps; set-ups 3 and 4 at half their root size, through the
near-wall refinement and the vorticity adaptations) replay the oracle's stored
run (tests/golden/make_golden.py): the tags its criterion chose, mesh digests
after every adaptation, mass and momentum after every period, and a seeded
sample of output cells at the end.  FP32 runs write every level with
non-temporal stores, the store path of the full-size benchmark."""
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_2308_08085_amd import abi, workloads as W
from parity_util import Pair, assert_cells, velocity_scale

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import goldens as G  # noqa: E402

pytestmark = pytest.mark.gpu


def run_schedule(p, steps, period, theta):
    done = 0
    while done < steps:
        n = min(period, steps - done)
        p.step(n, graph=True)
        done += n
        if done < steps:
            p.tag_vorticity(theta, require_equal=False)
            p.adapt()
            p.check_mesh("after coarse step %d" % done)


def test_config1_full_schedule_fp64():
    """D2Q9 FP64 cavity, 64^2 cells, 3 levels, Re 100: all 1000 coarse steps,
    adaptation every 100 -> every cell within 1e-12 of the oracle."""
    case = W.config1()
    t0 = time.perf_counter()
    p = Pair(case)
    run_schedule(p, case.steps, case.adapt_every, case.theta)
    print("config 1: %d coarse steps, blocks per level %s, tag mismatches %d, %.1f s" %
          (case.steps, p.g.counts().tolist(), p.tag_mismatches, time.perf_counter() - t0), flush=True)
    assert p.tag_mismatches == 0
    assert len(p.g.mesh()["ids"][1]) > 0
    p.assert_parity(1e-12, "config 1 after 1000 coarse steps")


def replay(name, storage, all_streaming, skip_parents=False):
    """Run the stored schedule `name` on the GPU with the oracle's tags; check
    tags, adaptation counts and mesh digests on the way, return the errors of
    the sampled output cells and of mass and momentum.  skip_parents: sweeps
    leave out the refined blocks none of whose children has an N_SKIP link."""
    gd = G.load(name)
    meta = json.loads(str(gd["meta"]))
    setup, freeze = G.CASES[name]
    case = getattr(W, setup)(storage=storage)
    cap, U = case.cap, velocity_scale(case)
    t0 = time.perf_counter()
    g = abi.AmrLbm(case)
    if all_streaming:
        g.stream_bytes(0)
    if skip_parents:
        g.skip_parents(True)
    g.set_root_rho_u(case.initial_rho_u())
    k = 0

    def adapt(tags):
        nonlocal k
        want = G.unpack_tags(gd, k, cap)
        assert np.array_equal(tags, want), "%s adaptation %d: tags differ at %s" % (
            name, k, np.flatnonzero(tags != want)[:8].tolist())
        st = g.adapt()
        assert (st["n_refine"], st["n_coarsen"], st["n_reverted"]) == tuple(gd["stats"][k]), (k, st, gd["stats"][k])
        assert G.mesh_digest(g.mesh(), cap) == str(gd["digests"][k]), "%s: mesh differs after adaptation %d" % (name, k)
        k += 1

    for _ in range(case.dist_levels):
        adapt(g.tag(abi.TAG_DISTANCE, d_spec=case.d_spec, freeze=freeze))
    periods = G.schedule(case)
    e = {"mass": 0.0, "momentum": 0.0, "U": U}
    for i, n in enumerate(periods):
        g.step(n, graph=True)
        m, mo = g.mass_mom(), gd["mass_after"][i]
        e["mass"] = max(e["mass"], abs(m[0] - mo[0]) / mo[0])
        e["momentum"] = max(e["momentum"], float(np.abs(m[1:] - mo[1:]).max() / (mo[0] * U)))
        if i < len(periods) - 1:
            adapt(g.tag(tags_in=G.unpack_tags(gd, k, cap)))
    assert k == len(gd["stats"])
    assert np.array_equal(g.counts(), gd["counts"]) and G.mesh_digest(g.mesh(), cap) == str(gd["final_digest"])
    n_out = g.n_out()
    assert n_out == meta["n_out"]
    sel, nf = gd["sample"], len(gd["f"])
    cells = g._fields(abi.AMR_GET, abi.F_CELLS, np.zeros((n_out, 2), np.int32))[sel]
    assert np.array_equal(cells[:, 0], gd["blk"]) and np.array_equal(cells[:, 1], gd["cell"]), "output cells differ"
    ru = g.rho_u_out()[sel]
    f = g.get_block_f_all()[gd["blk"][:nf], gd["cell"][:nf]]
    g.close()
    du = ru[:, 1: 1 + case.dim] - gd["u"]
    e.update({
        "f_cell": float((np.abs(f - gd["f"]) / np.abs(gd["f"])).max()),
        "rho_cell": float(np.abs(ru[:, 0] - gd["rho"]).max()),
        "u_cell": float(np.abs(du).max() / U),
        "u": float(np.linalg.norm(du) / np.linalg.norm(gd["u"])),
        "f": float(np.linalg.norm(f - gd["f"]) / np.linalg.norm(gd["f"])),
    })
    print("%s %s%s: %d coarse steps, %d adaptations, blocks per level %s, %d output cells (%d sampled): %s, %.1f s"
          % (name, storage, " (non-temporal stores)" if all_streaming else "", case.steps, k,
             gd["counts"].tolist(), n_out, len(sel), {a: float("%.3g" % b) for a, b in e.items()},
             time.perf_counter() - t0), flush=True)
    return e


SCHEDULES = list(G.CASES)


@pytest.mark.parametrize("name", SCHEDULES)
def test_schedule_fp32_storage(name):
    """FP32 shifted storage, every level streamed: sampled cells within 1e-5
    (per cell, parity_util), mass within 1e-7 after every period"""
    e = replay(name, "f32s", all_streaming=True)
    assert_cells(e, 1e-5, name, e["U"])
    assert e["mass"] < 1e-7 and e["momentum"] < 1e-5, e


@pytest.mark.parametrize("name", SCHEDULES)
def test_schedule_fp64_storage(name):
    """FP64 storage: sampled cells within 1e-12 (per cell, parity_util), mass and
    momentum within 1e-12 after every period (FP64 sums of ~1e6 cells in another
    order differ by ~1e-13)"""
    e = replay(name, "f64", all_streaming=False)
    assert_cells(e, 1e-12, name, e["U"])
    assert e["mass"] < 1e-12 and e["momentum"] < 1e-12, e


@pytest.mark.parametrize("name", [n for n in SCHEDULES if "unfrozen" not in n])
def test_schedule_fp16_storage_error(name):
    """FP16 shifted storage (FP32 arithmetic), every level streamed: the
    velocity error against the FP64 oracle on the same mesh, stated per run
    (norm-wise and per cell against the velocity scale)"""
    e = replay(name, "f16s", all_streaming=True)
    assert e["u"] < 2e-2 and e["u_cell"] < 2e-2 and e["f_cell"] < 5e-3 and e["mass"] < 1e-4, e


@pytest.mark.parametrize("name", [n for n in SCHEDULES if "cylinder" in n])
@pytest.mark.parametrize("storage,tol,mass_tol", [("f64", 1e-12, 1e-12), ("f32s", 1e-5, 1e-7)])
def test_schedule_skipping_deep_parents(name, storage, tol, mass_tol):
    """sweeps that leave out the refined blocks none of whose children has an
    N_SKIP link (AMR_FIELD_SKIP_PARENTS) against the oracle's run, which sweeps
    every block: tags, adaptation counts and mesh digests on the way, sampled
    output cells, mass and momentum after every period, at the same bars"""
    e = replay(name, storage, all_streaming=storage != "f64", skip_parents=True)
    assert_cells(e, tol, name, e["U"])
    assert e["mass"] < mass_tol and e["momentum"] < (1e-12 if storage == "f64" else 1e-5), e
