"""Pins of the oracle's cell classes (Sec. "Grid Communication") for fine
blocks whose coarser neighbour touches them only along an edge or at a corner,
with the ghost and interface cells enumerated by hand; the oracle's threads do
not change its results."""
import numpy as np
import pytest

import oracle
from paper_2308_08085_amd import workloads as W

GHOST, INTERFACE, INTERIOR = 2, 1, 0


def _all_but(case, keep):
    """refine every root block except those in `keep` (structured (i, j, k))"""
    o = oracle.Oracle(case)
    o.set_root_rho_u(case.initial_rho_u())
    r = case.root
    tags = np.zeros(case.cap, np.int8)
    for k in range(r[2] if case.dim == 3 else 1):
        for j in range(r[1]):
            for i in range(r[0]):
                if (i, j, k) not in keep:
                    tags[i + r[0] * (j + r[1] * k)] = 1
    o.tag(tags_in=tags)
    st = o.adapt()
    assert st["n_refine"] == case.nroot - len(keep)
    return o


def _child(o, case, root_ijk, c):
    i, j, k = root_ijk
    R = i + case.root[0] * (j + case.root[1] * k)
    return int(o.mesh()["nbrc"][R, 0]) + c


def _cells(dim, pred):
    out = set()
    for l in range(16 if dim == 2 else 64):
        if pred(l & 3, (l >> 2) & 3, l >> 4):
            out.add(l)
    return out


def _classes_by_hand(o, B, dim, ghost):
    cls = o.cell_classes(B)
    assert set(np.flatnonzero(cls == GHOST).tolist()) == ghost
    # every other cell is within Chebyshev distance 4 of the one coarse region
    assert set(np.flatnonzero(cls == INTERFACE).tolist()) == _cells(dim, lambda i, j, k: True) - ghost
    assert not np.any(cls == INTERIOR)


def test_corner_only_coarse_neighbour_2d():
    """3x3 root blocks, all but (2, 2) refined: child (1, 1) of root (1, 1)
    sees the coarse block only through its +x+y corner.  Ghost cells: the
    2x2 cells with i, j >= 2; the other 12 are interface cells."""
    case = W.cavity(2, 9, 12, 2, 100.0, cap=64)
    o = _all_but(case, {(2, 2, 0)})
    B = _child(o, case, (1, 1, 0), 3)
    links = o.mesh()["nbr"][B]
    assert [p for p in range(1, 9) if links[p] == oracle.N_SKIP] == [5]  # direction (1, 1)
    _classes_by_hand(o, B, 2, _cells(2, lambda i, j, k: i >= 2 and j >= 2))


def test_corner_only_coarse_neighbour_3d():
    """3x3x3 root blocks, all but (2, 2, 2) refined: child (1, 1, 1) of root
    (1, 1, 1) touches the coarse block only at its +x+y+z corner.  Ghost: the
    2x2x2 cells with i, j, k >= 2; interface: the other 56."""
    case = W.cavity(3, 19, 12, 2, 100.0, cap=256)
    o = _all_but(case, {(2, 2, 2)})
    B = _child(o, case, (1, 1, 1), 7)
    links = o.mesh()["nbr"][B]
    assert [p for p in range(1, 27) if links[p] == oracle.N_SKIP] == [19]  # direction (1, 1, 1)
    _classes_by_hand(o, B, 3, _cells(3, lambda i, j, k: i >= 2 and j >= 2 and k >= 2))


def test_edge_only_coarse_neighbour_3d():
    """3x3x3 root blocks, all but (2, 2, 1) refined: child (1, 1, 0) of root
    (1, 1, 1) touches the coarse block along its +x+y edge (regions (1, 1, 0)
    and (1, 1, 1)), through no face.  Ghost: i, j >= 2 for every k (16 cells);
    interface: the other 48."""
    case = W.cavity(3, 19, 12, 2, 100.0, cap=256)
    o = _all_but(case, {(2, 2, 1)})
    B = _child(o, case, (1, 1, 1), 3)
    links = o.mesh()["nbr"][B]
    # regions (1, 1, 0) and (1, 1, 1) both lie in root (2, 2, 1)
    assert [p for p in range(1, 27) if links[p] == oracle.N_SKIP] == [7, 19]
    _classes_by_hand(o, B, 3, _cells(3, lambda i, j, k: i >= 2 and j >= 2))


@pytest.mark.parametrize("dim,q", [(2, 9), (3, 27)])
def test_oracle_threads_do_not_change_results(dim, q):
    case = W.cavity(dim, q, 32 if dim == 2 else 16, 3, 100.0, seed=11)
    runs = []
    for nt in (1, 3):
        oracle.set_threads(nt)
        o = oracle.Oracle(case)
        o.set_root_rho_u(case.initial_rho_u())
        for _ in range(2):
            o.step(10)
            o.tag(kind=0, theta=0.1)
            o.adapt()
        o.step(3)
        runs.append((o.get_f_all(), o.crit(), o.mass_mom()))
    oracle.set_threads(0)
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
