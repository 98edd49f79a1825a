"""Pins of the oracle's refinement and coarsening (Sec. "Refinement and
Coarsening", Algs. 1-2): after random tag sequences on tiny forests every link
equals a brute-force geometric search, the forest stays 2:1 balanced and the ID
and gap sets stay consistent; refining and then coarsening the same blocks
restores every table."""
import numpy as np
import pytest

import oracle
from paper_2308_08085_amd import workloads as W

from meshcheck import check_forest, random_tags


def _small_cases():
    out = []
    out.append(W.cavity(2, 9, 16, 4, 100.0, cap=600, name="2d_walls"))
    c = W.cavity(2, 9, 12, 3, 100.0, cap=400, name="2d_periodic_x")
    c.periodic = (1, 0, 0)
    out.append(c)
    out.append(W.cylinder(2, 9, (32, 16), 4, 8, 3, 100.0, cap=500, name="2d_solid"))
    out.append(W.cavity(3, 19, 8, 3, 100.0, cap=400, name="3d_walls"))
    c = W.cavity(3, 27, 12, 3, 100.0, cap=1200, name="3d_periodic_xz")
    c.periodic = (1, 0, 1)
    out.append(c)
    out.append(W.cylinder(3, 27, (16, 12, 8), 4, 4, 3, 100.0, cap=900, name="3d_solid"))
    return out


@pytest.mark.parametrize("case", _small_cases(), ids=lambda c: c.name)
def test_random_adaptation_matches_geometry(case):
    o = oracle.Oracle(case)
    rng = np.random.default_rng(11)
    check_forest(case, o.mesh())
    grew = False
    for it in range(8):
        m = o.mesh()
        tags = random_tags(case, m, rng, 0.35 if it < 5 else 0.1, 0.25 if it < 5 else 0.6)
        eff = o.tag(tags_in=tags)
        # effective tags are a subset of the requested ones
        assert np.all((eff == 0) | (eff == tags))
        st = o.adapt()
        m2 = o.mesh()
        n = check_forest(case, m2)
        grew = grew or len(m2["ids"][-1]) > 0
        o.step(1)
    assert grew


@pytest.mark.parametrize("dim,q", [(2, 9), (3, 19)])
def test_refine_then_coarsen_restores_tables(dim, q):
    case = W.cavity(dim, q, 16 if dim == 2 else 8, 3, 100.0, cap=500)
    o = oracle.Oracle(case)
    rng = np.random.default_rng(5)
    # one level of refinement first, so that the round trip also runs on level 1
    o.tag(tags_in=random_tags(case, o.mesh(), rng, 0.5, 0.0))
    o.adapt()
    before = o.mesh()
    lvl1 = before["ids"][1]
    tags = np.zeros(case.cap, np.int8)
    pick = rng.choice(lvl1, size=min(6, len(lvl1)), replace=False)
    tags[pick] = 1
    eff = o.tag(tags_in=tags)
    st = o.adapt()
    assert st["n_refine"] > 0
    mid = o.mesh()
    refined = np.where(eff == 1)[0]
    tags2 = np.zeros(case.cap, np.int8)
    tags2[refined] = -1
    eff2 = o.tag(tags_in=tags2)
    assert np.array_equal(np.where(eff2 == -1)[0], refined)
    o.adapt()
    after = o.mesh()
    act = before["status"] != 8
    for key in ("level", "status", "X", "nbr", "nbrc"):
        assert np.array_equal(before[key][act], after[key][act]), key
    assert np.array_equal(before["status"] != 8, after["status"] != 8)
    for L in range(case.lmax):
        assert np.array_equal(before["ids"][L], after["ids"][L])
    assert np.array_equal(before["gap"], after["gap"])
    assert len(mid["gap"]) == len(before["gap"]) - st["n_refine"] * (4 if dim == 2 else 8)


def test_capacity_error_leaves_mesh_unchanged():
    case = W.cavity(2, 9, 16, 3, 100.0, cap=16 + 12)
    o = oracle.Oracle(case)
    before = o.mesh()
    tags = np.ones(case.cap, np.int8)
    o.tag(tags_in=tags)
    with pytest.raises(RuntimeError):
        o.adapt()
    after = o.mesh()
    for key in ("level", "status", "nbr", "nbrc"):
        assert np.array_equal(before[key], after[key])
    assert np.array_equal(before["gap"], after["gap"])
