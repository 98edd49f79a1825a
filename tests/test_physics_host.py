"""Host-side conversion of the momentum-exchange force to the paper's
dimensionless coefficients (Sec. "Flow Past a Square Cylinder")."""
import numpy as np

from paper_2308_08085_amd import physics


def test_level0_force_scaling():
    # a force G (level-0 units) acting on level L's cells is F = G * 2^(L (d-1)) per level-L sweep
    G = np.array([0.3, -0.1, 0.05])
    for dim in (2, 3):
        F = np.zeros((3, 4))
        for L, sweeps in ((0, 5), (1, 10), (2, 20)):
            F[L, :3] = G / 3 * 2.0 ** (L * (dim - 1)) * sweeps
            F[L, 3] = sweeps
        assert np.allclose(physics.level0_force(F, dim), G, rtol=1e-14)
    # a level with no sweeps contributes nothing
    F = np.zeros((2, 4))
    F[0] = [1.0, 2.0, 3.0, 4.0]
    assert np.allclose(physics.level0_force(F, 2), [0.25, 0.5, 0.75])


def test_sine_fit_recovers_frequency_and_amplitude():
    rng = np.random.default_rng(5)
    t = np.arange(140, 150, 16 / 256) + 8 / 256
    for f, a in ((0.2355, 0.27), (0.41, 0.05), (0.12, 1.3)):
        y = 0.01 + a * np.sin(2 * np.pi * f * t + 1.1) + 1e-3 * rng.standard_normal(len(t))
        fit_f, fit_a = physics.sine_fit(t, y)
        assert abs(fit_f / f - 1) < 2e-3 and abs(fit_a / a - 1) < 2e-2, (f, fit_f, a, fit_a)
