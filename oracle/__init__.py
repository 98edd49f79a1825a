"""FP64 CPU oracle of the block-based AMR lattice Boltzmann method (arXiv 2308.08085).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2308_08085_amd``) and never imports it.

The arithmetic lives in ``amr_oracle.c`` (plain C, FP64, naive loops); this file
only compiles it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_NONE, TAG_REFINE, TAG_COARSEN, TAG_REFINE_PERM = 0, 1, -1, 2
ST_UNREFINED, ST_REFINED, ST_REFINED_CHILD, ST_REFINED_PERM = 0, 1, 2, 3
ST_INACTIVE = 8
NONE_ID, N_SKIP, SOLID_CODE = -1, -2, -9


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (``-O2``, plain C99, FP64; OpenMP over the
    per-block loops, which does not change any result)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("q", C.c_int32), ("root", C.c_int32 * 3), ("lmax", C.c_int32),
        ("cap", C.c_int32), ("nu0", C.c_double), ("periodic", C.c_int32 * 3),
        ("face_kind", C.c_int32 * 6), ("face_u", (C.c_double * 3) * 6), ("face_prio", C.c_int32 * 6),
        ("solid", C.POINTER(C.c_uint8)), ("rescale_mode", C.c_int32), ("interp", C.c_int32),
    ]


class _TagParams(C.Structure):
    _fields_ = [("kind", C.c_int32), ("theta", C.c_double), ("d_spec", C.c_double), ("freeze", C.c_int32),
                ("n_start", C.c_double), ("n_inc", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Config)]
        L.orc_destroy.argtypes = [P]
        L.orc_n_out.restype = C.c_int64
        L.orc_n_out.argtypes = [P]
        for name in ("orc_set_root_rho_u", "orc_get_block_f", "orc_set_block_f", "orc_step", "orc_sync",
                     "orc_tag", "orc_adapt", "orc_get_crit", "orc_get_out", "orc_mass_mom", "orc_get_mesh",
                     "orc_lattice", "orc_feq", "orc_collide", "orc_interp_child", "orc_interp_child_cubic",
                     "orc_average_parent",
                     "orc_parity", "orc_force", "orc_get_f_all", "orc_cell_classes", "orc_set_threads",
                     "orc_ratios", "orc_sweep", "orc_mrt_collide", "orc_mrt_matrix", "orc_set_collision"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- primitives
def lattice(dim: int, q: int):
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    if lib().orc_lattice(dim, q, _ip(c), _dp(w), _ip(opp)) != 0:
        raise ValueError("unknown lattice")
    return c, w, opp


def feq(dim: int, q: int, rho: float, u) -> np.ndarray:
    uu = np.zeros(3, np.float64)
    uu[: len(u)] = u
    out = np.zeros(q, np.float64)
    lib().orc_feq(dim, q, C.c_double(rho), _dp(uu), _dp(out))
    return out


def collide(dim: int, q: int, omega: float, f) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(q, np.float64)
    lib().orc_collide(dim, q, C.c_double(omega), _dp(f), _dp(out))
    return out


def mrt_collide(omega: float, s_high: float, f) -> np.ndarray:
    """moment-space collision of one D3Q27 cell (moments above second order at s_high)"""
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(27, np.float64)
    if lib().orc_mrt_collide(C.c_double(omega), C.c_double(s_high), _dp(f), _dp(out)) != 0:
        raise RuntimeError("moment matrix is singular")
    return out


def mrt_matrix() -> np.ndarray:
    """the D3Q27 moment matrix M[k][p] of the moment-space collision"""
    m = np.zeros((27, 27), np.float64)
    if lib().orc_mrt_matrix(_dp(m)) != 0:
        raise RuntimeError("moment matrix is singular")
    return m


def interp_child(dim: int, q: int, r: float, parent, child: int, cubic: bool = False) -> np.ndarray:
    parent = np.ascontiguousarray(parent, np.float64)
    out = np.zeros_like(parent)
    fn = lib().orc_interp_child_cubic if cubic else lib().orc_interp_child
    fn(dim, q, C.c_double(r), _dp(parent), child, _dp(out))
    return out


def average_parent(dim: int, q: int, r: float, children) -> np.ndarray:
    children = np.ascontiguousarray(children, np.float64)
    mb = 16 if dim == 2 else 64
    out = np.zeros((mb, q), np.float64)
    lib().orc_average_parent(dim, q, C.c_double(r), _dp(children), _dp(out))
    return out


def set_threads(n: int = 0) -> int:
    """host threads of the oracle's per-block loops (0: leave unchanged); returns the count in use"""
    return int(lib().orc_set_threads(int(n)))


# ---------------------------------------------------------------- forest
class Oracle:
    """One simulation on the CPU, FP64, following the paper's algorithm step by step.

    ``case`` is any object with the attributes dim, q, root, lmax, cap, nu0,
    periodic, face_kind, face_u, face_prio, solid (see
    ``paper_2308_08085_amd.workloads.Case``).
    """

    def __init__(self, case, rescale_mode: int = 0):
        self.case = case
        self.dim, self.q, self.lmax, self.cap = case.dim, case.q, case.lmax, case.cap
        self.mb = 16 if self.dim == 2 else 64
        self.nb = 9 if self.dim == 2 else 27
        cfg = _Config()
        cfg.dim, cfg.q, cfg.lmax, cfg.cap = case.dim, case.q, case.lmax, case.cap
        for a in range(3):
            cfg.root[a] = int(case.root[a]) if a < len(case.root) else 1
            cfg.periodic[a] = int(case.periodic[a])
        cfg.nu0 = float(case.nu0)
        for fc in range(6):
            cfg.face_kind[fc] = int(case.face_kind[fc])
            cfg.face_prio[fc] = int(case.face_prio[fc])
            for a in range(3):
                cfg.face_u[fc][a] = float(case.face_u[fc][a])
        self._solid = None
        if case.solid is not None:
            self._solid = np.ascontiguousarray(case.solid, np.uint8)
            cfg.solid = self._solid.ctypes.data_as(C.POINTER(C.c_uint8))
        cfg.rescale_mode = rescale_mode
        cfg.interp = int(getattr(case, "interp", 0))
        self._h = lib().orc_create(C.byref(cfg))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.nroot = int(np.prod([cfg.root[a] for a in range(3)]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(C.c_void_p(h))
            self._h = None

    @property
    def h(self):
        return C.c_void_p(self._h)

    def set_root_rho_u(self, ru: np.ndarray):
        ru = np.ascontiguousarray(ru, np.float64).reshape(self.nroot * self.mb, 4)
        lib().orc_set_root_rho_u(self.h, _dp(ru))

    def get_block_f(self, B: int) -> np.ndarray:
        out = np.zeros((self.mb, self.q), np.float64)
        lib().orc_get_block_f(self.h, int(B), _dp(out))
        return out

    def set_block_f(self, B: int, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        lib().orc_set_block_f(self.h, int(B), _dp(f))

    def get_f_all(self) -> np.ndarray:
        """[cap][Mb][q]: every active block's current data (zeros for inactive IDs)"""
        out = np.zeros((self.cap, self.mb, self.q), np.float64)
        lib().orc_get_f_all(self.h, _dp(out))
        return out

    def cell_classes(self, B: int) -> np.ndarray:
        """[Mb]: 0 interior, 1 interface, 2 ghost (Sec. "Grid Communication")"""
        out = np.zeros(self.mb, np.int32)
        if lib().orc_cell_classes(self.h, int(B), _ip(out)) != 0:
            raise ValueError("block %d is not active" % B)
        return out

    def step(self, n: int = 1):
        lib().orc_step(self.h, int(n))

    def set_collision(self, kind: int, s_high: float = 1.0):
        """0 = BGK; 1 = moment-space collision (D3Q27), higher moments at s_high"""
        if lib().orc_set_collision(self.h, int(kind), C.c_double(s_high)) != 0:
            raise ValueError("collision kind %d with s_high %g is not available here" % (kind, s_high))

    def sweep(self, L: int):
        """one collide-stream sweep of level L alone (timing only: the forest is
        left mid-step)"""
        if lib().orc_sweep(self.h, int(L)) != 0:
            raise ValueError("no level %d" % L)

    def sync(self):
        lib().orc_sync(self.h)

    def tag(self, kind: int = 0, theta: float = 0.1, d_spec: float = 0.0, freeze: int = 0,
            tags_in: np.ndarray | None = None, n_start: float = -2.0, n_inc: float = 1.0) -> np.ndarray:
        p = _TagParams(kind, theta, d_spec, freeze, n_start, n_inc)
        out = np.zeros(self.cap, np.int8)
        tin = None
        if tags_in is not None:
            tin = np.ascontiguousarray(tags_in, np.int8)
            assert tin.shape == (self.cap,)
        lib().orc_tag(self.h, C.byref(p), _ip(tin) if tin is not None else None, _ip(out))
        return out

    def force(self, reset: bool = False) -> np.ndarray:
        """[lmax][4]: force on the solid blocks per level (x, y, z) summed over the
        level's sweeps since the last reset, and the number of sweeps"""
        out = np.zeros((self.lmax, 4), np.float64)
        lib().orc_force(self.h, _dp(out), int(reset))
        return out

    def adapt(self):
        st = np.zeros(4, np.int32)
        rc = lib().orc_adapt(self.h, _ip(st))
        if rc != 0:
            raise RuntimeError("oracle adapt failed (capacity)" if rc == -2 else "oracle adapt failed")
        return {"n_refine": int(st[0]), "n_coarsen": int(st[1]), "n_reverted": int(st[2])}

    def crit(self) -> np.ndarray:
        out = np.zeros(self.cap, np.float64)
        lib().orc_get_crit(self.h, _dp(out))
        return out

    def ratios(self, L: int):
        """(coarse-to-fine, fine-to-coarse) rescaling ratios between levels L and L+1"""
        out = np.zeros(2, np.float64)
        if lib().orc_ratios(self.h, int(L), _dp(out)) != 0:
            raise ValueError("no level %d -> %d" % (L, L + 1))
        return float(out[0]), float(out[1])

    def parity(self, L: int) -> int:
        return int(lib().orc_parity(self.h, L))

    def output(self):
        n = int(lib().orc_n_out(self.h))
        blk = np.zeros(n, np.int32)
        cell = np.zeros(n, np.int32)
        rho = np.zeros(n, np.float64)
        u = np.zeros((n, 3), np.float64)
        f = np.zeros((n, self.q), np.float64)
        lib().orc_get_out(self.h, _ip(blk), _ip(cell), _dp(rho), _dp(u), _dp(f))
        return {"blk": blk, "cell": cell, "rho": rho, "u": u[:, : self.dim], "f": f}

    def mass_mom(self) -> np.ndarray:
        out = np.zeros(4, np.float64)
        lib().orc_mass_mom(self.h, _dp(out))
        return out

    def mesh(self):
        cap, nb, lmax = self.cap, self.nb, self.lmax
        level = np.zeros(cap, np.int8)
        status = np.zeros(cap, np.int8)
        X = np.zeros((cap, 3), np.int32)
        nbr = np.zeros((cap, nb), np.int32)
        nbrc = np.zeros((cap, nb), np.int32)
        nids = np.zeros(lmax, np.int32)
        ids = np.zeros((lmax, cap), np.int32)
        gtop = np.zeros(1, np.int32)
        gap = np.zeros(cap, np.int32)
        lib().orc_get_mesh(self.h, _ip(level), _ip(status), _ip(X), _ip(nbr), _ip(nbrc), _ip(nids),
                           _ip(ids), _ip(gtop), _ip(gap))
        return {
            "level": level, "status": status, "X": X, "nbr": nbr, "nbrc": nbrc,
            "ids": [ids[L, : nids[L]].copy() for L in range(lmax)],
            "gap": gap[: gtop[0]].copy(),
        }
