"""Helpers of the GPU-vs-oracle parity tests: run one schedule on both, compare
mesh tables bit for bit and fields cell by cell.

Per-cell bar (asserted), for tolerance tol (1e-12 FP64 storage, 1e-5 FP32):
  - every population of every compared cell: |f_gpu - f_oracle| <= tol |f_oracle|;
  - every output cell: |rho_gpu - rho_oracle| <= tol (rho is about 1) and
    max_a |u_gpu,a - u_oracle,a| <= tol / 3 in lattice units.  u is a
    difference of populations, rho u_a = sum_p f_p c_pa: populations each
    within tol |f_p| move it by at most tol sum_p f_p |c_pa|, which is tol/3
    near rest for every lattice here (sum_p w_p |c_pa| = sum_p w_p c_pa^2 =
    c_s^2 = 1/3).  u itself is near 0 in parts of every flow, so it is not
    measured against itself; u_cell reports max |du| / U with U the set-up's
    lid or inlet speed (the bar is then tol / (3 U)).
The norm-wise relative L2 errors ||d||/||ref|| of f, rho and u (u against ||u||,
with no floor) are reported beside them.
"""
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


def _norm_rel(d, ref):
    r = np.linalg.norm(ref)
    return float(np.linalg.norm(d) / r) if r > 0 else float(np.linalg.norm(d))


def field_errors(oo, og, u_scale):
    """Per-cell and norm-wise errors of the output cells (leaf, non-ghost).

    f_cell = max |df| / |f| over cells and populations, rho_cell = max |d rho|,
    u_cell = max |du| / u_scale; f, rho, u = norm-wise relative L2 errors."""
    assert np.array_equal(oo["blk"], og["blk"]) and np.array_equal(oo["cell"], og["cell"]), "output cells differ"
    out = {"n": int(len(oo["rho"]))}
    if not len(oo["rho"]):
        return dict(out, f=0.0, rho=0.0, u=0.0, f_cell=0.0, rho_cell=0.0, u_cell=0.0, max_drho=0.0)
    df = og["f"] - oo["f"]
    du = og["u"] - oo["u"]
    drho = og["rho"] - oo["rho"]
    out["f"] = _norm_rel(df, oo["f"])
    out["rho"] = _norm_rel(drho, oo["rho"])
    out["u"] = _norm_rel(du, oo["u"])
    out["f_cell"] = float((np.abs(df) / np.abs(oo["f"])).max())
    out["rho_cell"] = out["max_drho"] = float(np.abs(drho).max())
    out["u_cell"] = float(np.abs(du).max() / u_scale)
    # where the worst cell is, for the message
    k = int(np.argmax(np.abs(du).max(axis=1)))
    out["u_cell_at"] = (int(oo["blk"][k]), int(oo["cell"][k]))
    return out


def block_errors(fo, fg, status):
    """Every stored population of every cell of every active block (leaves,
    parents, ghost cells): max |df| / |f|, and where."""
    act = np.asarray(status) != 8
    a, b = fo[act], fg[act]
    rel = np.abs(b - a) / np.abs(a)
    k = np.unravel_index(int(np.argmax(rel)), rel.shape)
    return {"block_f_cell": float(rel[k]), "block_f_cell_at": (int(np.flatnonzero(act)[k[0]]), int(k[1]), int(k[2]))}


def assert_cells(e, tol, what="", u_scale=0.05):
    """the per-cell bar (module docstring) on a result of field_errors (+
    block_errors); u_scale = the U that u_cell was divided by"""
    bars = {"f_cell": tol, "rho_cell": tol, "u_cell": tol / (3.0 * u_scale), "block_f_cell": tol}
    bad = [k for k, b in bars.items() if k in e and not e[k] <= b]
    assert not bad, "%s: %s above the bar (tol %g): %s" % (what, bad, tol, e)


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

    def errors(self, blocks=True):
        """field_errors of the output cells, plus block_errors of every active
        block's cells unless blocks=False"""
        e = field_errors(self.o.output(), self.g.output(), velocity_scale(self.case))
        if blocks:
            e.update(block_errors(self.o.get_f_all(), self.g.get_block_f_all(), self.o.mesh()["status"]))
        return e

    def assert_parity(self, tol, what=""):
        e = self.errors()
        print("%s: %s" % (what or self.case.name, {k: (round(v, 16) if isinstance(v, float) else v)
                                                    for k, v in e.items()}), flush=True)
        assert_cells(e, tol, what or self.case.name, velocity_scale(self.case))
        return e
