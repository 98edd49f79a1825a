"""Drag, lift and shedding frequency of the flow past a square cylinder
(Sec. "Flow Past a Square Cylinder").

The force comes from the library's momentum exchange with the solid blocks
(`AmrLbm.force`); this module only converts it to the dimensionless
coefficients C_D = 2 F_x / (rho_0 U^2 D), C_L = 2 F_y / (rho_0 U^2 D) and
St = f_s D / U, and drives the paper's run.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import abi


def level0_force(F, dim: int) -> np.ndarray:
    """Mean force per sweep in level-0 lattice units from the per-level sums of
    `AmrLbm.force` (rows: F_x, F_y, F_z summed over that level's sweeps in its own
    lattice units, sweep count).  On level L momentum scales by 2^(-L d) and
    time by 2^(-L), so a force scales by 2^(-L (d - 1))."""
    out = np.zeros(3)
    for L in range(F.shape[0]):
        if F[L, 3] > 0:
            out += F[L, :3] * (2.0 ** (-L * (dim - 1)) / F[L, 3])
    return out


def sine_fit(t, y):
    """Least-squares fit of y ~ a + b sin(2 pi f t) + c cos(2 pi f t) over a grid of
    frequencies, then golden-section refinement.  Returns (f, amplitude)."""
    t, y = np.asarray(t, float), np.asarray(y, float)

    def resid(f):
        A = np.stack([np.ones_like(t), np.sin(2 * np.pi * f * t), np.cos(2 * np.pi * f * t)], 1)
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        return float(np.sum((A @ coef - y) ** 2)), coef

    span = t[-1] - t[0]
    fs = np.linspace(0.5 / span, 0.5 / (t[1] - t[0]), 4000)
    f = fs[int(np.argmin([resid(x)[0] for x in fs]))]
    lo, hi = f - (fs[1] - fs[0]), f + (fs[1] - fs[0])
    g = (math.sqrt(5) - 1) / 2
    for _ in range(60):
        a, b = hi - g * (hi - lo), lo + g * (hi - lo)
        if resid(a)[0] < resid(b)[0]:
            hi = b
        else:
            lo = a
    f = (lo + hi) / 2
    coef = resid(f)[1]
    return f, float(math.hypot(coef[1], coef[2]))


def run_fpsc(case, n_x: int, t_end: float = 150.0, t_avg: float = 140.0, sample: int = 16, log=None):
    """Advance a square-cylinder case (`workloads.fpsc`) to t_end domain-length
    time units (n_x root steps each) with the paper's schedule: static near-wall
    refinement with freeze at t = 0, the log2 ladder every `case.adapt_every`
    root steps (a single-level case is a uniform grid and never adapts).
    C_D is averaged and C_L fitted by a sinusoid over
    [t_avg, t_end], sampled every `sample` root steps (each sample the mean over
    those steps).  A capacity refusal raises: the run would no longer be the
    paper's."""
    U, D = float(case.face_u[0][0]), float(n_x // 32)
    g = abi.AmrLbm(case)
    try:
        g.force_accumulation(False)  # until the sampling window opens
        g.set_root_rho_u(case.initial_rho_u())
        for _ in range(case.dist_levels):
            g.tag(abi.TAG_DISTANCE, d_spec=case.d_spec, freeze=1)
            g.adapt()
        period = case.adapt_every
        if period % sample:
            raise ValueError("the sampling interval must divide the adaptation period")
        n_end, n_avg = int(round(t_end * n_x)), int(round(t_avg * n_x))
        n_start, n_inc = case.ladder
        t, cd, cl = [], [], []
        t0 = time.perf_counter()
        t_adapt = 0.0
        done = 0
        while done < n_end:
            if done < n_avg:
                g.step(period, graph=True)
                done += period
                if done == n_avg:
                    g.force_accumulation(True)
                    g.force(reset=True)
            else:
                for _ in range(period // sample):
                    g.step(sample, graph=True)
                    done += sample
                    fx, fy, _ = level0_force(g.force(reset=True), case.dim)
                    t.append((done - sample / 2) / n_x)
                    cd.append(2 * fx / (U * U * D))
                    cl.append(2 * fy / (U * U * D))
            if not np.all(np.isfinite(g.mass_mom())):
                raise RuntimeError("%s went non-finite at root step %d" % (case.name, done))
            if done < n_end and case.lmax > 1:
                ta = time.perf_counter()  # the stream has drained (mass_mom above)
                g.tag(abi.TAG_LADDER, n_start=n_start, n_inc=n_inc)
                g.adapt()
                t_adapt += time.perf_counter() - ta
            if log is not None and done % (20 * n_x) == 0:
                log("[%s] t = %.0f, blocks/level %s (%.0f s)" % (case.name, done / n_x, g.counts().tolist(),
                                                              time.perf_counter() - t0))
        if len(t) < 8:
            raise ValueError("too few samples in [t_avg, t_end]")
        t, cd, cl = np.array(t), np.array(cd), np.array(cl)
        f_s, amp = sine_fit(t, cl)  # per time unit of the domain length
        return {"root_steps": done, "wall_s": round(time.perf_counter() - t0, 1),
                "adapt_s": round(t_adapt, 1), "samples": len(t),
                "C_D_mean": float(cd.mean()), "C_L_amplitude": amp, "St": f_s * (D / n_x) / U,
                "level_blocks_end": g.counts().tolist()}
    finally:
        g.close()
