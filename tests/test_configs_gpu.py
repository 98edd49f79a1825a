"""Benchmark set-ups on their stated schedules against the oracle: adaptation
after coarse step k when k is a multiple of the adaptation period and k is
below the total, vorticity tagging with theta = 0.1."""
import time

import pytest

from paper_2308_08085_amd import workloads as W
from parity_util import Pair

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
    adaptation every 100 -> FP64 fields within 1e-12 of the oracle."""
    case = W.config1()
    t0 = time.perf_counter()
    p = Pair(case)
    run_schedule(p, case.steps, case.adapt_every, case.theta)
    e = p.errors()
    print("config 1: %d coarse steps, blocks per level %s, errors %s, tag mismatches %d, %.1f s" %
          (case.steps, p.g.counts().tolist(), e, p.tag_mismatches, time.perf_counter() - t0), flush=True)
    assert p.tag_mismatches == 0
    assert len(p.g.mesh()["ids"][1]) > 0
    assert e["f"] < 1e-12 and e["rho"] < 1e-12 and e["u"] < 1e-12, e


def test_config2_fp32_storage_first_100_steps():
    """D3Q19 cavity, 64^3 cells, 3 levels, Re 400, FP32 shifted storage: the
    first 100 of its 2000 coarse steps (adaptation after step 50; the FP64
    oracle needs about 0.4 s per coarse step here) -> within 1e-5."""
    case = W.config2()
    t0 = time.perf_counter()
    p = Pair(case)
    run_schedule(p, 100, case.adapt_every, case.theta)
    e = p.errors()
    print("config 2 (100 steps): blocks per level %s, errors %s, tag mismatches %d, %.1f s" %
          (p.g.counts().tolist(), e, p.tag_mismatches, time.perf_counter() - t0), flush=True)
    assert e["f"] < 1e-5 and e["rho"] < 1e-5 and e["u"] < 1e-5, e
