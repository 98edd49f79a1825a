"""Pins of the oracle's moment-space (multiple-relaxation-time) collision, the
reference for the library's optional moment-space collision (D3Q27).  The
paper's method is BGK; it names moment-space operators as the alternative
(Sec. "Lattice Boltzmann Method").  Checked against what the definition fixes:
the basis rows are the stated polynomial products and orthogonal under the
lattice weights, equal rates give BGK, mass and momentum are conserved for any
rate, and each moment's non-equilibrium part relaxes at the rate of its order."""
import numpy as np
import pytest

import oracle
from paper_2308_08085_amd import workloads as W

C, Wt, _ = oracle.lattice(3, 27)


def phi(a, c):
    return np.ones_like(c, dtype=float) if a == 0 else (c.astype(float) if a == 1 else 3.0 * c * c - 1.0)


def order(k):
    return sum(k // 3 ** d % 3 for d in range(3))


def random_cell(rng, rho=1.0, u=(0.04, -0.03, 0.02), noise=0.02):
    f = oracle.feq(3, 27, rho, u)
    return f * (1.0 + noise * rng.standard_normal(27))


def test_basis_rows_are_the_stated_products():
    M = oracle.mrt_matrix()
    for k in range(27):
        a, b, c = k % 3, k // 3 % 3, k // 9
        want = phi(a, C[:, 0]) * phi(b, C[:, 1]) * phi(c, C[:, 2])
        assert np.array_equal(M[k], want), k
    # spot values written out by hand: density row, x-momentum row, phi_2(c_z) row
    assert np.all(M[0] == 1.0)
    assert np.array_equal(M[1], C[:, 0].astype(float))
    assert np.array_equal(M[18], np.where(C[:, 2] != 0, 2.0, -1.0))


def test_basis_is_orthogonal_under_the_weights():
    M = oracle.mrt_matrix()
    G = M @ np.diag(Wt) @ M.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-15
    # norms: products of the 1-D norms 1, 1/3, 2 of phi_0, phi_1, phi_2
    n1 = [1.0, 1.0 / 3.0, 2.0]
    for k in range(27):
        want = n1[k % 3] * n1[k // 3 % 3] * n1[k // 9]
        assert abs(G[k, k] - want) < 1e-15 * want


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.7, 1.98])
def test_equal_rates_give_bgk(omega):
    rng = np.random.default_rng(int(omega * 100))
    for _ in range(20):
        f = random_cell(rng, rho=1.0 + 0.02 * rng.standard_normal(), u=0.05 * rng.standard_normal(3))
        a = oracle.mrt_collide(omega, omega, f)
        b = oracle.collide(3, 27, omega, f)
        assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("s_high", [0.3, 1.0, 1.6, 1.99])
def test_mass_and_momentum_conserved(s_high):
    rng = np.random.default_rng(7)
    for _ in range(20):
        f = random_cell(rng, rho=1.0 + 0.02 * rng.standard_normal(), u=0.05 * rng.standard_normal(3), noise=0.05)
        out = oracle.mrt_collide(1.4, s_high, f)
        assert abs(out.sum() - f.sum()) < 1e-15
        assert np.abs(out @ C - f @ C).max() < 1e-15


@pytest.mark.parametrize("k", [4, 5, 8, 12, 13, 18, 22, 26])
def test_each_moment_relaxes_at_the_rate_of_its_order(k):
    """f = f_eq + eps M^-1 e_k keeps rho and u (k is not a conserved moment),
    so after the collision the moment k of f - f_eq is (1 - s) eps with s =
    omega for order <= 2 and s_high above, and every other moment stays 0."""
    M = oracle.mrt_matrix()
    omega, s_high, eps = 1.3, 0.7, 1e-3
    feq = oracle.feq(3, 27, 1.02, [0.03, 0.01, -0.02])
    e = np.zeros(27)
    e[k] = 1.0
    f = feq + eps * np.linalg.solve(M, e)
    out = oracle.mrt_collide(omega, s_high, f)
    dm = M @ (out - feq)
    s = omega if order(k) <= 2 else s_high
    want = np.zeros(27)
    want[k] = (1.0 - s) * eps
    assert np.abs(dm - want).max() < 1e-14, (k, order(k), dm[k], want[k])


def test_forest_run_with_equal_rates_matches_bgk():
    """a one-level D3Q27 cavity: the moment-space collision with s_high equal
    to the level's omega reproduces the BGK run over 20 steps (only rounding
    differs)"""
    case = W.cavity(3, 27, 16, 1, 100.0, storage="f64", seed=3, cap=64)
    a, b = oracle.Oracle(case), oracle.Oracle(case)
    for o in (a, b):
        o.set_root_rho_u(case.initial_rho_u())
    a.set_collision(1, 1.0 / (0.5 + 3.0 * case.nu0))
    a.step(20)
    b.step(20)
    assert np.abs(a.get_f_all() - b.get_f_all()).max() < 1e-13


def test_only_d3q27_accepts_the_moment_space_collision():
    o = oracle.Oracle(W.cavity(3, 19, 8, 1, 100.0, storage="f64", cap=8))
    with pytest.raises(ValueError):
        o.set_collision(1, 1.0)
