"""Pins of the oracle's lattice, equilibrium and collision against what the paper
and the mathematics fix (velocity-set figure; moment constraints of the
second-order equilibrium; BGK fixed point and conservation)."""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "velocity_set_figure.txt")
LATTICES = [(2, 9), (3, 19), (3, 27)]


def _figure_labels():
    out = {"D2Q9": {}, "D3Q27": {}}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lat, lab, x, y = line.split()
            out[lat][int(lab)] = (float(x), float(y))
    return out


def _direction_from_figure_2d(pos):
    # square centre (199,137), half width 50; y grows downwards in the drawing
    cx, cy = 199.0, 137.0
    best = None
    for v in itertools.product((-1, 0, 1), repeat=2):
        px, py = cx + 50 * v[0], cy - 50 * v[1]
        d = (pos[0] - px) ** 2 + (pos[1] - py) ** 2
        if best is None or d < best[0]:
            best = (d, v)
    return (best[1][0], best[1][1], 0)


def _direction_from_figure_3d(pos):
    # cube centre (469,132); x -> (+50,0), y -> (0,-50), z -> (-10,+20) per unit
    cx, cy = 469.0, 132.0
    best = None
    for v in itertools.product((-1, 0, 1), repeat=3):
        px = cx + 50 * v[0] - 10 * v[2]
        py = cy - 50 * v[1] + 20 * v[2]
        d = (pos[0] - px) ** 2 + (pos[1] - py) ** 2
        if best is None or d < best[0]:
            best = (d, v)
    return tuple(best[1])


def test_direction_numbering_matches_figure():
    labels = _figure_labels()
    c, _, _ = oracle.lattice(2, 9)
    for p in range(9):
        assert tuple(c[p]) == _direction_from_figure_2d(labels["D2Q9"][p]), p
    c27, _, _ = oracle.lattice(3, 27)
    for p in range(27):
        assert tuple(c27[p]) == _direction_from_figure_3d(labels["D3Q27"][p]), p
    c19, _, _ = oracle.lattice(3, 19)
    assert np.array_equal(c19, c27[:19])
    # every direction appears once
    assert len({tuple(v) for v in c27}) == 27


@pytest.mark.parametrize("dim,q", LATTICES)
def test_lattice_isotropy(dim, q):
    c, w, opp = oracle.lattice(dim, q)
    c = c[:, :dim].astype(np.float64)
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-15
    M2 = np.einsum("p,pa,pb->ab", w, c, c)
    assert np.abs(M2 - cs2 * np.eye(dim)).max() < 1e-15
    M3 = np.einsum("p,pa,pb,pc->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-15
    M4 = np.einsum("p,pa,pb,pc,pd->abcd", w, c, c, c, c)
    d = np.eye(dim)
    iso = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.abs(M4 - iso).max() < 1e-15
    # opposite table is an involution with c_opp = -c
    assert np.array_equal(opp[opp], np.arange(q))
    assert np.array_equal(c[opp], -c)
    assert opp[0] == 0


@pytest.mark.parametrize("dim,q", LATTICES)
def test_equilibrium_moments(dim, q):
    """sum feq = rho, sum feq c = rho u, sum feq c c = rho cs^2 I + rho u u (pins the signs)."""
    c, w, _ = oracle.lattice(dim, q)
    c = c[:, :dim].astype(np.float64)
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = 1.0 + rng.uniform(-0.1, 0.1)
        u = rng.uniform(-0.08, 0.08, size=dim)
        f = oracle.feq(dim, q, rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.abs((f[:, None] * c).sum(0) - rho * u).max() < 1e-15
        P = np.einsum("p,pa,pb->ab", f, c, c)
        assert np.abs(P - (rho / 3.0 * np.eye(dim) + rho * np.outer(u, u))).max() < 1e-15


@pytest.mark.parametrize("dim,q", LATTICES)
def test_collision_fixed_point_and_conservation(dim, q):
    c, w, _ = oracle.lattice(dim, q)
    rng = np.random.default_rng(2)
    rho, u = 1.02, rng.uniform(-0.05, 0.05, size=dim)
    f = oracle.feq(dim, q, rho, u)
    out = oracle.collide(dim, q, 1.7, f)
    assert np.abs(out - f).max() <= 1e-15 * np.abs(f).max() * 4
    g = f + rng.uniform(-1e-3, 1e-3, size=q)
    for omega in (0.3, 1.0, 1.9):
        h = oracle.collide(dim, q, omega, g)
        assert abs(h.sum() - g.sum()) < 1e-15
        assert np.abs(((h - g)[:, None] * c[:, :dim]).sum(0)).max() < 1e-16
    # omega = 0 leaves f unchanged; omega = 1 gives the equilibrium
    assert np.array_equal(oracle.collide(dim, q, 0.0, g), g)
    rg = g.sum()
    ug = (g[:, None] * c[:, :dim]).sum(0) / rg
    assert np.abs(oracle.collide(dim, q, 1.0, g) - oracle.feq(dim, q, rg, ug)).max() < 1e-16
