"""Stored oracle results of the long benchmark schedules (test helper).

The set-ups of the benchmark run for hundreds to thousands of coarse steps,
longer than the FP64 oracle can follow inside a GPU test.  ``make_golden.py``
runs each of them once through the oracle (and nothing else) and stores, per
adaptation, the tags the oracle's criterion chose and a digest of the oracle's
mesh tables, and at the end a seeded sample of output cells (rho, u, and f for
a subset), the mass and momentum and the block counts.  The GPU tests replay
the stored tags and compare against the stored values.

The schedule is the benchmark's: coarse steps in periods of ``adapt_every``,
an adaptation after every period that ends before ``steps``.  Set-ups with a
static near-wall refinement apply it at t = 0 first.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

# stored schedules: name -> (set-up function of paper_2308_08085_amd.workloads,
# freeze flag of the near-wall refinement at t = 0)
CASES = {
    # D3Q19 lid-driven cube cavity, 64^3 root cells, 3 levels, Re 400: all 2000 coarse steps
    "cfg2_d3q19_cavity": ("config2", 1),
    # the D2Q9 and D3Q27 cylinder set-ups at half the root size, through the
    # frozen near-wall refinement and the vorticity adaptations of their schedule
    "cfg3r_d2q9_cylinder": ("config3_reduced", 1),
    "cfg4r_d3q27_cylinder": ("config4_reduced", 1),
    # the same without freezing the near-wall refinement, so that the vorticity
    # adaptations coarsen and refine around the cylinder and in the wake
    "cfg3r_d2q9_cylinder_unfrozen": ("config3_reduced", 0),
    "cfg4r_d3q27_cylinder_unfrozen": ("config4_reduced", 0),
}

# output cells sampled for rho/u, and for f (a subset of the first)
N_SAMPLE = 6144
N_SAMPLE_F = 2048


def path(name: str) -> str:
    return os.path.join(HERE, name + ".npz")


def mesh_digest(m, cap: int) -> str:
    """SHA-256 over the mesh tables of the active blocks (level, status, origin,
    neighbour and neighbour-child links), the ID sets and the gap stack"""
    h = hashlib.sha256()
    act = np.asarray(m["status"]) != 8
    h.update(np.ascontiguousarray(np.flatnonzero(act).astype(np.int32)).tobytes())
    for k, dt in (("level", np.int8), ("status", np.int8), ("X", np.int32), ("nbr", np.int32), ("nbrc", np.int32)):
        h.update(np.ascontiguousarray(np.asarray(m[k])[act].astype(dt)).tobytes())
    for ids in m["ids"]:
        h.update(np.int64(len(ids)).tobytes())
        h.update(np.ascontiguousarray(np.asarray(ids, np.int32)).tobytes())
    h.update(np.ascontiguousarray(np.asarray(m["gap"], np.int32)).tobytes())
    return h.hexdigest()


def schedule(case):
    """coarse-step counts of the periods; an adaptation follows every period but the last"""
    out, done = [], 0
    while done < case.steps:
        n = min(case.adapt_every, case.steps - done)
        out.append(n)
        done += n
    return out


def sample_cells(blk, level_of_block, seed: int):
    """indices into the output cells: a seeded sample stratified by level (every
    level gets at least a share of N_SAMPLE / (2 L_max)); the first N_SAMPLE_F
    of them also carry f"""
    rng = np.random.default_rng(seed)
    lv = level_of_block[blk]
    levels = sorted(set(lv.tolist()))
    floor = N_SAMPLE // (2 * max(len(levels), 1))
    picked = []
    for L in levels:
        idx = np.flatnonzero(lv == L)
        k = min(len(idx), floor)
        picked.append(rng.choice(idx, k, replace=False))
    rest = np.setdiff1d(np.arange(len(blk)), np.concatenate(picked))
    k = min(len(rest), N_SAMPLE - sum(len(p) for p in picked))
    picked.append(rng.choice(rest, k, replace=False))
    sel = np.concatenate(picked)
    rng.shuffle(sel)
    return sel


def load(name: str):
    with np.load(path(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def unpack_tags(g, k: int, cap: int) -> np.ndarray:
    """effective tags of adaptation k (stored sparse)"""
    t = np.zeros(cap, np.int8)
    a, b = g["tag_ptr"][k], g["tag_ptr"][k + 1]
    t[g["tag_idx"][a:b]] = g["tag_val"][a:b]
    return t
