"""Seeded synthetic workloads (problem set-ups and initial fields).

This module describes inputs only: domain shape, boundary kinds, viscosity from
the Reynolds number, the seeded velocity noise.  It holds none of the method's
arithmetic and is shared by the HIP binding, the CPU oracle's tests and the
benchmark.  The set-ups follow the paper's two test problems (lid-driven cavity,
flow past a square cylinder; Sec. "Validation and Case Studies").
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FACE_VELOCITY, FACE_OUTFLOW = 0, 1
# face order: -x, +x, -y, +y, -z, +z
PRIO_WALL, PRIO_INLET, PRIO_OUTFLOW, PRIO_LID = 1, 2, 3, 4


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    q: int
    root: tuple            # root blocks per axis (4^d cells each); root[2] = 1 in 2-D
    lmax: int              # number of grid levels
    nu0: float             # lattice viscosity on level 0
    cap: int               # block capacity
    face_kind: tuple = (FACE_VELOCITY,) * 6
    face_u: tuple = ((0.0, 0.0, 0.0),) * 6
    face_prio: tuple = (PRIO_WALL,) * 6
    periodic: tuple = (0, 0, 0)
    solid: np.ndarray | None = None   # uint8 per root block, structured order
    storage: str = "f64"
    seed: int = 0
    noise: float = 1e-4
    u_init: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    adapt_every: int = 0
    theta: float = 0.1
    dist_levels: int = 0    # static distance refinement passes at t = 0
    d_spec: float = 0.0     # distance criterion, root cells
    interp: int = 0         # coarse-to-fine interpolation: 0 linear, 1 cubic
    ladder: tuple | None = None  # (N_start, N_inc) of the log2 criterion ladder, else the relative threshold

    @property
    def mb(self) -> int:
        return 16 if self.dim == 2 else 64

    @property
    def nroot(self) -> int:
        return int(self.root[0] * self.root[1] * (self.root[2] if self.dim == 3 else 1))

    @property
    def root_cells(self) -> tuple:
        return tuple(4 * r for r in self.root[: self.dim])

    def initial_rho_u(self) -> np.ndarray:
        """rho = 1 and u = u_init + seeded uniform noise, per root cell in (root block ID, cell) order.

        Returns float64 [nroot * Mb, 4] = (rho, ux, uy, uz).
        """
        rng = np.random.default_rng(self.seed)
        n = self.nroot * self.mb
        out = np.zeros((n, 4), np.float64)
        out[:, 0] = 1.0
        out[:, 1 : 1 + self.dim] = rng.uniform(-self.noise, self.noise, size=(n, self.dim))
        out[:, 1:4] += np.asarray(self.u_init, np.float64)[None, :]
        return out


def _root3(root):
    r = tuple(int(v) for v in root)
    return r + (1,) * (3 - len(r))


def cavity(dim: int, q: int, side_cells: int, lmax: int, re: float, u_lid: float = 0.05,
           storage: str = "f64", seed: int = 0, cap: int | None = None, name: str = "cavity",
           steps: int = 0, adapt_every: int = 0, theta: float = 0.1) -> Case:
    """Lid-driven cavity: lid on +y (2-D) / +z (3-D) moving along +x; nu = U N / Re."""
    nb = side_cells // 4
    root = (nb, nb, nb if dim == 3 else 1)
    lid = 3 if dim == 2 else 5
    face_u = [[0.0, 0.0, 0.0] for _ in range(6)]
    face_u[lid] = [u_lid, 0.0, 0.0]
    prio = [PRIO_WALL] * 6
    prio[lid] = PRIO_LID
    nroot = nb ** dim
    if cap is None:
        cap = nroot * 24
    return Case(name=name, dim=dim, q=q, root=root, lmax=lmax, nu0=u_lid * side_cells / re, cap=cap,
                face_kind=(FACE_VELOCITY,) * 6, face_u=tuple(tuple(v) for v in face_u),
                face_prio=tuple(prio), storage=storage, seed=seed, steps=steps,
                adapt_every=adapt_every, theta=theta)


def cylinder(dim: int, q: int, cells: tuple, side: int, x0: int, lmax: int, re: float,
             u_in: float = 0.05, storage: str = "f32s", seed: int = 0, cap: int | None = None,
             name: str = "cylinder", steps: int = 0, adapt_every: int = 32, theta: float = 0.1) -> Case:
    """Channel flow past a block-aligned square cylinder.

    Inlet (-x) and far-field faces are known-velocity faces at u = (U, 0, 0); +x is
    the outflow.  The cylinder occupies [x0, x0+side) along x, is centred in y and
    spans z in 3-D.  nu = U D / Re.
    """
    root = tuple(c // 4 for c in cells)
    root3 = _root3(root)
    face_kind = [FACE_VELOCITY] * 6
    face_kind[1] = FACE_OUTFLOW
    face_u = [[u_in, 0.0, 0.0] for _ in range(6)]
    face_u[1] = [0.0, 0.0, 0.0]
    prio = [PRIO_INLET] * 6
    prio[1] = PRIO_OUTFLOW
    solid = np.zeros(root3[0] * root3[1] * root3[2], np.uint8)
    y0 = (cells[1] - side) // 2
    for bk in range(root3[2]):
        for bj in range(root3[1]):
            for bi in range(root3[0]):
                x, y = bi * 4, bj * 4
                if x0 <= x < x0 + side and y0 <= y < y0 + side:
                    solid[bi + root3[0] * (bj + root3[1] * bk)] = 1
    nroot = root3[0] * root3[1] * root3[2]
    if cap is None:
        cap = nroot * 4
    return Case(name=name, dim=dim, q=q, root=root3, lmax=lmax, nu0=u_in * side / re, cap=cap,
                face_kind=tuple(face_kind), face_u=tuple(tuple(v) for v in face_u), face_prio=tuple(prio),
                solid=solid, storage=storage, seed=seed, u_init=(u_in, 0.0, 0.0), steps=steps,
                adapt_every=adapt_every, theta=theta, dist_levels=lmax - 1,
                d_spec=0.15 * cells[0])


def fpsc(n_x: int = 256, lmax: int = 4, interp: int = 0, storage: str = "f64", seed: int = 2308091,
         cap: int | None = None, height: int = 32) -> Case:
    """The paper's flow past a square cylinder at Re 100 (Sec. "Flow Past a Square
    Cylinder", runs F-A to F-C of its parameter table).

    Channel 32 D long and `height` D high (the text's square domain by default)
    with n_x root cells along x, so
    D = n_x / 32; the cylinder's upstream face 10 D from the inlet, centred in y.  Inlet and far field at U = 0.05, outflow at +x, nu from Re 100.
    Static near-wall refinement with freeze at t = 0, then the log2 ladder with
    N_start = -3, N_inc = 1 every 32 root steps.  One time unit of the paper
    (domain length 1) is n_x root steps.
    """
    d = n_x // 32
    ny = height * d
    case = cylinder(2, 9, (n_x, ny), d, 10 * d, lmax, 100.0, storage=storage, seed=seed,
                    name="fpsc_nx%d_h%d_l%d_%s" % (n_x, height, lmax, "cubic" if interp else "linear"),
                    steps=150 * n_x, adapt_every=32,
                    cap=cap if cap is not None else (n_x // 4) * (ny // 4) * (12 * 2 ** lmax if lmax > 1 else 1))
    case.interp = interp
    case.ladder = (-3.0, 1.0)
    return case


# The five set-ups of the benchmark (seed 2308085 + i for set-up i).
def config1(**kw) -> Case:
    """D2Q9 FP64 lid-driven cavity, 64^2 cells (16^2 blocks), 3 levels, Re 100."""
    args = dict(storage="f64", seed=2308086, steps=1000, adapt_every=100, name="cfg1_d2q9_cavity")
    args.update(kw)
    return cavity(2, 9, 64, 3, 100.0, **args)


def config2(**kw) -> Case:
    """D3Q19 FP32 lid-driven cube cavity, 64^3 cells (16^3 blocks), 3 levels, Re 400."""
    args = dict(storage="f32s", seed=2308087, steps=2000, adapt_every=50, name="cfg2_d3q19_cavity")
    args.update(kw)
    return cavity(3, 19, 64, 3, 400.0, **args)


def config3(**kw) -> Case:
    """D2Q9 channel 1024x256 cells past a 32-cell square cylinder at x = 256, 4 levels, Re 100."""
    args = dict(storage="f32s", seed=2308088, steps=2500, adapt_every=32, name="cfg3_d2q9_cylinder")
    args.update(kw)
    return cylinder(2, 9, (1024, 256), 32, 256, 4, 100.0, **args)


def config4(**kw) -> Case:
    """D3Q27 channel 256x128x128 cells past a 16-cell square cylinder at x = 64, 3 levels, Re 200."""
    args = dict(storage="f32s", seed=2308089, steps=1000, adapt_every=32, name="cfg4_d3q27_cylinder")
    args.update(kw)
    return cylinder(3, 27, (256, 128, 128), 16, 64, 3, 200.0, **args)


def config3_reduced(**kw) -> Case:
    """Set-up 3 at half the root size along each axis: D2Q9 channel 512x128 cells
    past a 16-cell square cylinder at x = 128, 4 levels, Re 100 (same side
    ratio, levels, boundaries and schedule)."""
    args = dict(storage="f32s", seed=2308088, steps=160, adapt_every=32, name="cfg3r_d2q9_cylinder",
                cap=128 * 32 * 16)
    args.update(kw)
    return cylinder(2, 9, (512, 128), 16, 128, 4, 100.0, **args)


def config4_reduced(**kw) -> Case:
    """Set-up 4 at half the root size along each axis: D3Q27 channel 128x64x64
    cells past an 8-cell square cylinder at x = 32 spanning z, 3 levels, Re 200
    (same side ratio, levels, boundaries and schedule)."""
    args = dict(storage="f32s", seed=2308089, steps=128, adapt_every=32, name="cfg4r_d3q27_cylinder",
                cap=32 * 16 * 16 * 16)
    args.update(kw)
    return cylinder(3, 27, (128, 64, 64), 8, 32, 3, 200.0, **args)


def config5_cases(n: int = 64, seed: int = 2308090):
    """Batched set-up: n independent cavities, half D2Q9 and half D3Q19, FP16 storage.

    Root sides from {32,64,128,256} (2-D) / {32,48,64} (3-D), Re log-uniform in
    [100, 3200], 2-4 levels, adaptation every 50 coarse steps.
    """
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        if s < n // 2:
            dim, q, side = 2, 9, int(rng.choice([32, 64, 128, 256]))
        else:
            dim, q, side = 3, 19, int(rng.choice([32, 48, 64]))
        re = float(math.exp(rng.uniform(math.log(100.0), math.log(3200.0))))
        lmax = int(rng.integers(2, 5))
        nroot = (side // 4) ** dim
        out.append(cavity(dim, q, side, lmax, re, storage="f16s", seed=seed + 1 + s, cap=nroot * 48,
                          name="cfg5_sim%02d" % s, steps=1000, adapt_every=50))
    return out


def mlups_updates(level_counts, dim: int) -> float:
    """Lattice-node updates per coarse step by the paper's AMR-weighted count
    (Sec. "Solver Performance"): sum_L 2^L (N_L - N_{L+1}/N_c [L < L_max-1]), in cells."""
    nc = 4 if dim == 2 else 8
    mb = 16 if dim == 2 else 64
    lmax = len(level_counts)
    tot = 0.0
    for L in range(lmax):
        n = level_counts[L] * mb
        if L < lmax - 1:
            n -= level_counts[L + 1] * mb / nc
        tot += (2 ** L) * n
    return tot
