#!/usr/bin/env python3
"""Write the stored oracle results of the long benchmark schedules.

Runs each set-up through the FP64 CPU oracle only (``oracle/``; the inputs come
from the seeded set-ups of ``paper_2308_08085_amd.workloads``) and writes
``tests/golden/<name>.npz``; see ``goldens.py`` for what is stored.  The
oracle's results do not depend on its thread count.

    python tests/golden/make_golden.py [names...] [--threads N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle  # noqa: E402
import goldens as G  # noqa: E402
from paper_2308_08085_amd import workloads as W  # noqa: E402


def run(name: str, log=print):
    setup, freeze = G.CASES[name]
    case = getattr(W, setup)()
    t0 = time.perf_counter()
    o = oracle.Oracle(case)
    o.set_root_rho_u(case.initial_rho_u())
    kinds, tag_idx, tag_val, tag_ptr, stats, digests, mass_after = [], [], [], [0], [], [], []

    def record(kind, tags):
        st = o.adapt()
        nz = np.flatnonzero(tags)
        kinds.append(kind)
        tag_idx.append(nz.astype(np.int32))
        tag_val.append(tags[nz].astype(np.int8))
        tag_ptr.append(tag_ptr[-1] + len(nz))
        stats.append((st["n_refine"], st["n_coarsen"], st["n_reverted"]))
        digests.append(G.mesh_digest(o.mesh(), case.cap))

    for _ in range(case.dist_levels):
        record(1, o.tag(kind=1, d_spec=case.d_spec, freeze=freeze))
    periods = G.schedule(case)
    for i, n in enumerate(periods):
        o.step(n)
        mass_after.append(o.mass_mom())
        if i < len(periods) - 1:
            record(0, o.tag(kind=0, theta=case.theta))
        log("%s: period %d/%d, blocks per level %s, adaptations %s, %.0f s" %
            (name, i + 1, len(periods), [len(x) for x in o.mesh()["ids"]], stats[-1:], time.perf_counter() - t0),
            flush=True)
    out = o.output()
    mesh = o.mesh()
    sel = G.sample_cells(out["blk"], mesh["level"].astype(np.int64), seed=2308085)
    selF = sel[: G.N_SAMPLE_F]
    meta = {"name": name, "case": case.name, "freeze": freeze, "steps": case.steps, "adapt_every": case.adapt_every,
            "theta": case.theta, "dist_levels": case.dist_levels, "d_spec": case.d_spec,
            "n_out": int(len(out["blk"])), "oracle_seconds": round(time.perf_counter() - t0, 1),
            "threads": oracle.set_threads(0)}
    np.savez_compressed(
        G.path(name), meta=np.array(json.dumps(meta)), kinds=np.array(kinds, np.int8),
        tag_idx=np.concatenate(tag_idx) if tag_idx else np.zeros(0, np.int32),
        tag_val=np.concatenate(tag_val) if tag_val else np.zeros(0, np.int8),
        tag_ptr=np.array(tag_ptr, np.int64), stats=np.array(stats, np.int32).reshape(-1, 3),
        digests=np.array(digests), mass_after=np.array(mass_after, np.float64),
        counts=np.array([len(x) for x in mesh["ids"]], np.int32),
        final_digest=np.array(G.mesh_digest(mesh, case.cap)), mass_mom=o.mass_mom(),
        sample=sel.astype(np.int64), blk=out["blk"][sel], cell=out["cell"][sel], rho=out["rho"][sel],
        u=out["u"][sel], f=out["f"][selF])
    log("%s: wrote %s (%d output cells, %.0f s)" % (name, G.path(name), len(out["blk"]), time.perf_counter() - t0))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("names", nargs="*", default=list(G.CASES))
    ap.add_argument("--threads", type=int, default=0, help="oracle host threads (0: all)")
    a = ap.parse_args()
    oracle.build(force=False)
    oracle.set_threads(a.threads)
    for n in a.names:
        run(n)


if __name__ == "__main__":
    main()
