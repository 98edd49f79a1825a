"""The paper's flow past a square cylinder at Re 100 (Sec. "Flow Past a Square
Cylinder"): a 32 D x 32 D domain, FP64, run to t = 150 with drag and shedding
frequency taken over the last 10 time units, as in the paper.

At effective resolution 512 the paper prints C_D = 1.513 and St = 0.1470 for
the uniform grid (its table of results).  Two-level AMR from 256 x 256 root
cells (D = 8), linear and cubic interpolation, must agree with our own uniform
512 x 512 grid, and both with the paper's values.  This checks the whole
solver -- open boundaries, solid blocks, sub-cycled levels, ladder adaptation
and the momentum exchange -- against printed numbers."""
import pytest

from paper_2308_08085_amd import physics, workloads as W

pytestmark = pytest.mark.gpu

PAPER_UNIFORM_512 = {"C_D": 1.513, "St": 0.1470}


@pytest.fixture(scope="module")
def uniform512():
    case = W.fpsc(512, 1, storage="f64")
    print("case", case.name, flush=True)
    r = physics.run_fpsc(case, 512)
    print(case.name, r, flush=True)
    return r


@pytest.mark.parametrize("interp", [0, 1])
def test_square_cylinder_amr_matches_uniform_grid_and_the_paper(uniform512, interp):
    case = W.fpsc(256, 2, interp, storage="f64")
    print("case", case.name, flush=True)
    r = physics.run_fpsc(case, 256)
    print(case.name, r, flush=True)
    assert r["samples"] == 160 and uniform512["samples"] == 320
    for k in ("C_D_mean", "St"):
        assert abs(r[k] / uniform512[k] - 1) < 2e-3, (k, r[k], uniform512[k])
    for res in (r, uniform512):
        assert abs(res["C_D_mean"] / PAPER_UNIFORM_512["C_D"] - 1) < 0.02, res
        assert abs(res["St"] / PAPER_UNIFORM_512["St"] - 1) < 0.02, res
        assert 0.2 < res["C_L_amplitude"] < 0.35, res  # periodic shedding is established
