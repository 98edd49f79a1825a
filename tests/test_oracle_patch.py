"""The block-patch check of the full-size GPU tests (patchcheck.py), validated
on the oracle itself: for every eligible leaf of a refined cylinder mesh, the
patch's single-level run reproduces the oracle's own coarse step to rounding
(the patch's relaxation time comes from a viscosity scaled by 2^L, which can
differ from the forest's tau*_L = 1/2 + 2^L (tau*_0 - 1/2) in the last bit)."""
import numpy as np
import pytest

import oracle
from paper_2308_08085_amd import workloads as W
from patchcheck import Geometry, block_class, patch, patch_expected


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_reproduces_a_coarse_step(dim):
    if dim == 2:
        case = W.cylinder(2, 9, (96, 48), 8, 24, 4, 100.0, storage="f64", cap=12000, seed=21)
    else:
        case = W.cylinder(3, 19, (32, 16, 16), 4, 8, 3, 100.0, storage="f64", cap=4000, seed=22)
    o = oracle.Oracle(case)
    o.set_root_rho_u(case.initial_rho_u())
    for _ in range(case.dist_levels):
        o.tag(kind=1, d_spec=case.d_spec, freeze=1)
        o.adapt()
    o.step(3)
    m = o.mesh()
    fpre = o.get_f_all()
    o.step(1)
    fpost = o.get_f_all()
    geo = Geometry(case, m)
    seen = {}
    leaves = np.flatnonzero((m["status"] == 0))
    np.random.default_rng(5).shuffle(leaves)
    for B in leaves:
        L = int(m["level"][B])
        key = (L, block_class(m, B))
        if seen.get(key, 0) >= 12:
            continue
        n = 2 ** L
        p = patch(geo, int(B), n)
        if p is None:
            continue
        want = patch_expected(*p, fpre, n)
        assert np.abs(want - fpost[B]).max() <= 1e-14, (B, L, key, np.abs(want - fpost[B]).max())
        seen[key] = seen.get(key, 0) + 1
    print(sorted(seen.items()))
    # every level, and faces and solid neighbours on the finest level
    assert {L for L, _ in seen} == set(range(case.lmax))
    assert (case.lmax - 1, "solid") in seen and (case.lmax - 1, "face") in seen and (0, "face") in seen
