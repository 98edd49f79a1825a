"""Helpers of the GPU-vs-oracle parity tests: run one schedule on both, compare
mesh tables bit for bit and fields by norm-wise relative error."""
import numpy as np

import oracle
from paper_2308_08085_amd import abi

MESH_KEYS = ("level", "status", "X", "nbr", "nbrc")


def compare_mesh(mo, mg, where=""):
    act = mo["status"] != 8
    assert np.array_equal(act, mg["status"] != 8), "active sets differ " + where
    for k in MESH_KEYS:
        a, b = mo[k][act], mg[k][act]
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)[:5]
            raise AssertionError("%s differs %s at %s: oracle %s gpu %s" % (k, where, bad.tolist(),
                                                                               a[tuple(bad[0])], b[tuple(bad[0])]))
    for L, (x, y) in enumerate(zip(mo["ids"], mg["ids"])):
        assert np.array_equal(x, y), "id_set %d differs %s" % (L, where)
    assert np.array_equal(mo["gap"], mg["gap"]), "gap stack differs " + where


def field_errors(oo, og, u_scale=0.0):
    """Norm-wise relative L2 errors of rho, u, f over the output cells, plus max |d rho|.

    The velocity norm is floored at u_scale * sqrt(n) (u_scale = the case's lid or
    inlet speed): while the flow is still at the level of the initial noise, the
    rounding of u is set by the populations, not by |u|.
    """
    assert np.array_equal(oo["blk"], og["blk"]) and np.array_equal(oo["cell"], og["cell"]), "output cells differ"
    out = {}
    for k in ("rho", "u", "f"):
        a, b = oo[k], og[k]
        ref = np.linalg.norm(a)
        if k == "u":
            ref = max(ref, u_scale * np.sqrt(a.size / max(a.shape[1], 1)))
        out[k] = float(np.linalg.norm(b - a) / max(ref, 1e-300))
    out["max_drho"] = float(np.abs(og["rho"] - oo["rho"]).max()) if len(oo["rho"]) else 0.0
    return out


def velocity_scale(case):
    return float(max(np.abs(np.asarray(case.face_u)).max(), np.abs(np.asarray(case.u_init)).max()))


class Pair:
    """The same simulation on the oracle and on the GPU."""

    def __init__(self, case, storage=None, init=True):
        self.case = case
        self.o = oracle.Oracle(case)
        self.g = abi.AmrLbm(case, storage=storage)
        if init:
            ru = case.initial_rho_u()
            self.o.set_root_rho_u(ru)
            self.g.set_root_rho_u(ru)
        self.tag_mismatches = 0

    def step(self, n, graph=False):
        self.o.step(n)
        self.g.step(n, graph=graph)

    def tag_vorticity(self, theta=0.1, require_equal=True):
        tg = self.g.tag(abi.TAG_VORTICITY_REL, theta=theta)
        to = self.o.tag(kind=0, theta=theta)
        if not np.array_equal(tg, to):
            self.tag_mismatches += int((tg != to).sum())
            if require_equal:
                raise AssertionError("tags differ at %s" % np.where(tg != to)[0][:10].tolist())
            self.o.tag(tags_in=tg)  # replay the GPU's tags so the meshes stay identical
        return tg

    def tag_distance(self, d_spec, freeze=1):
        tg = self.g.tag(abi.TAG_DISTANCE, d_spec=d_spec, freeze=freeze)
        to = self.o.tag(kind=1, d_spec=d_spec, freeze=freeze)
        assert np.array_equal(tg, to), "distance tags differ"
        return tg

    def tag_replay(self, tags):
        tg = self.g.tag(tags_in=tags)
        to = self.o.tag(tags_in=tags)
        assert np.array_equal(tg, to), "effective tags differ"
        return tg

    def adapt(self):
        so = self.o.adapt()
        sg = self.g.adapt()
        assert so["n_refine"] == sg["n_refine"] and so["n_coarsen"] == sg["n_coarsen"], (so, sg)
        assert so["n_reverted"] == sg["n_reverted"], (so, sg)
        return sg

    def check_mesh(self, where=""):
        compare_mesh(self.o.mesh(), self.g.mesh(), where)

    def errors(self):
        return field_errors(self.o.output(), self.g.output(), velocity_scale(self.case))
