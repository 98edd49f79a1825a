"""Thin Python binding of the C ABI in ``include/amr_lbm.h``.

Argument marshalling only: every step of the method runs in the HIP library
``libamrlbm.so``.  PyTorch supplies the device arena and a HIP stream.  There is
no CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrlbm.so")

AMR_OK = 0
AMR_ERR_ARG, AMR_ERR_CAPACITY, AMR_ERR_STATE, AMR_ERR_DEVICE, AMR_ERR_UNSTABLE = -1, -2, -3, -4, -5
STORAGE = {"f64": 0, "f32": 1, "f32s": 2, "f16s": 3, "bf16s": 4}
AMR_GET, AMR_SET = 0, 1
(F_N_OUT, F_CELLS, F_RHO_U, F_F, F_BLOCK_F, F_LEVEL, F_STATUS, F_COORD, F_NBR, F_NBR_CHILD, F_IDSET, F_GAP,
 F_COUNTS, F_MASS_MOM, F_CRIT, F_PARITY, F_KERNEL_STATS, F_FORCE, F_FORCE_ON, F_STREAM_BYTES,
 F_SYNC_VELOCITY, F_SKIP_PARENTS) = range(22)
AMR_CHECK_FINITE, AMR_USE_GRAPH, AMR_PROFILE = 1, 2, 4
TAG_VORTICITY_REL, TAG_DISTANCE, TAG_LADDER = 0, 1, 2
COLLIDE_BGK, COLLIDE_MRT, COLLIDE_MRT_MFMA = 0, 1, 2

# every symbol the header declares
EXPORTS = ("amr_query_bytes", "amr_create", "amr_tag", "amr_adapt", "lbm_step", "amr_fields", "amr_destroy",
           "amr_batch_query_bytes", "amr_batch_create", "amr_batch_step", "amr_batch_set_tuning",
           "amr_batch_get_tuning", "amr_batch_autotune", "amr_batch_destroy", "amr_mass_mom_static",
           "amr_set_collision", "amr_last_error")


class AmrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("amr error %d: %s" % (code, msg))
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("q", C.c_int32), ("root", C.c_int32 * 3), ("max_levels", C.c_int32),
        ("max_blocks", C.c_int32), ("storage", C.c_int32), ("nu0", C.c_double), ("periodic", C.c_int32 * 3),
        ("face_kind", C.c_int32 * 6), ("face_u", (C.c_double * 3) * 6), ("face_prio", C.c_int32 * 6),
        ("solid_root", C.POINTER(C.c_uint8)), ("interp", C.c_int32),
    ]


class TagParams(C.Structure):
    _fields_ = [("kind", C.c_int32), ("theta", C.c_double), ("d_spec", C.c_double), ("freeze", C.c_int32),
                ("n_start", C.c_double), ("n_inc", C.c_double)]


class AdaptStats(C.Structure):
    _fields_ = [("n_refine", C.c_int32), ("n_coarsen", C.c_int32), ("n_reverted", C.c_int32),
                ("n_free", C.c_int32), ("level_blocks", C.c_int32 * 8), ("step_ms", C.c_double * 8)]


ADAPT_STEPS = ("sync_average", "sync_interp", "criterion", "prep", "assign", "build", "connect", "fill")


class BatchTuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("wg_per_cu", C.c_int32), ("schedule", C.c_int32)]


_lib = None


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run paper_2308_08085_amd.build.build()" % LIB_PATH)
        # torch first: the library must bind to the HIP runtime torch already
        # loaded (the arenas are torch allocations); loaded the other way round
        # a process can end up with two runtimes and no shared device pointers
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.amr_query_bytes.argtypes = [C.POINTER(Config), C.POINTER(C.c_uint64)]
        L.amr_create.argtypes = [C.POINTER(Config), P, C.c_uint64, P, C.POINTER(P)]
        L.amr_tag.argtypes = [P, C.POINTER(TagParams), P, P]
        L.amr_adapt.argtypes = [P, C.POINTER(AdaptStats)]
        L.lbm_step.argtypes = [P, C.c_int32, C.c_uint32]
        L.amr_fields.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, C.c_uint64]
        L.amr_destroy.argtypes = [P]
        L.amr_batch_query_bytes.argtypes = [C.POINTER(P), C.c_int32, C.POINTER(C.c_uint64)]
        L.amr_batch_create.argtypes = [C.POINTER(P), C.c_int32, P, C.c_uint64, P, C.POINTER(P)]
        L.amr_batch_step.argtypes = [P, C.c_int32, C.c_uint32]
        L.amr_batch_set_tuning.argtypes = [P, C.POINTER(BatchTuning)]
        L.amr_batch_get_tuning.argtypes = [P, C.POINTER(BatchTuning)]
        L.amr_batch_autotune.argtypes = [P, C.c_int32, C.POINTER(BatchTuning), C.POINTER(C.c_double)]
        L.amr_batch_destroy.argtypes = [P]
        L.amr_mass_mom_static.argtypes = [P, P]
        L.amr_set_collision.argtypes = [P, C.c_int32, C.c_double]
        L.amr_last_error.restype = C.c_char_p
        for n in EXPORTS[:-1]:
            getattr(L, n).restype = C.c_int32
        _lib = L
    return _lib


def _check(rc):
    if rc != AMR_OK:
        raise AmrError(rc, load().amr_last_error().decode())


def make_config(case, storage=None):
    cfg = Config()
    cfg.dim, cfg.q = case.dim, case.q
    for a in range(3):
        cfg.root[a] = int(case.root[a]) if a < len(case.root) else 1
        cfg.periodic[a] = int(case.periodic[a])
    if case.dim == 2:
        cfg.root[2] = 1
    cfg.max_levels, cfg.max_blocks = case.lmax, case.cap
    cfg.storage = STORAGE[storage or case.storage]
    cfg.nu0 = float(case.nu0)
    cfg.interp = int(getattr(case, "interp", 0))
    for f in range(6):
        cfg.face_kind[f] = int(case.face_kind[f])
        cfg.face_prio[f] = int(case.face_prio[f])
        for a in range(3):
            cfg.face_u[f][a] = float(case.face_u[f][a])
    return cfg


def query_bytes(case, storage=None) -> int:
    cfg = make_config(case, storage)
    out = C.c_uint64(0)
    _check(load().amr_query_bytes(C.byref(cfg), C.byref(out)))
    return int(out.value)


class AmrLbm:
    """One simulation on the GPU behind the C ABI."""

    def __init__(self, case, storage=None, device="cuda", stream=None):
        import torch
        self.case = case
        self.storage = storage or case.storage
        self.dim, self.q, self.lmax, self.cap = case.dim, case.q, case.lmax, case.cap
        self.mb = 16 if self.dim == 2 else 64
        self.nb = 9 if self.dim == 2 else 27
        lib = load()
        cfg = make_config(case, self.storage)
        self._solid = None
        if case.solid is not None:
            self._solid = np.ascontiguousarray(case.solid, np.uint8)
            cfg.solid_root = self._solid.ctypes.data_as(C.POINTER(C.c_uint8))
        nbytes = C.c_uint64(0)
        _check(lib.amr_query_bytes(C.byref(cfg), C.byref(nbytes)))
        self.arena_bytes = int(nbytes.value)
        self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        # the arena comes from torch's caching allocator on the current stream:
        # order the library stream after work pending there (a recycled block)
        self.stream.wait_stream(torch.cuda.current_stream(device))
        h = C.c_void_p(0)
        _check(lib.amr_create(C.byref(cfg), C.c_void_p(aligned), C.c_uint64(self.arena_bytes),
                              C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.nroot = int(np.prod([cfg.root[a] for a in range(3)]))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            load().amr_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ calls
    def _fields(self, op, kind, arr):
        _check(load().amr_fields(self._h, op, kind, 0, arr.ctypes.data_as(C.c_void_p), arr.nbytes))
        return arr

    def set_root_rho_u(self, ru):
        ru = np.ascontiguousarray(ru, np.float64).reshape(self.nroot * self.mb, 4)
        self._fields(AMR_SET, F_RHO_U, ru)

    def step(self, n=1, check_finite=False, graph=False, profile=False):
        flags = ((AMR_CHECK_FINITE if check_finite else 0) | (AMR_USE_GRAPH if graph else 0)
                 | (AMR_PROFILE if profile else 0))
        _check(load().lbm_step(self._h, int(n), flags))

    def kernel_stats(self, reset=False):
        """{kernel: (launches, ms, blocks, bytes)} of the lbm_step calls made with profile=True"""
        a = self._fields(AMR_GET, F_KERNEL_STATS, np.zeros((3, 4), np.float64))
        if reset:
            self._fields(AMR_SET, F_KERNEL_STATS, np.zeros((3, 4), np.float64))
        return {k: tuple(a[i]) for i, k in enumerate(("collide_stream", "interp", "average"))}

    def tag(self, kind=TAG_VORTICITY_REL, theta=0.1, d_spec=0.0, freeze=0, tags_in=None, n_start=-2.0, n_inc=1.0):
        p = TagParams(kind, theta, d_spec, freeze, n_start, n_inc)
        out = np.zeros(self.cap, np.int8)
        tin = None
        if tags_in is not None:
            tin = np.ascontiguousarray(tags_in, np.int8)
            assert tin.shape == (self.cap,)
        _check(load().amr_tag(self._h, C.byref(p), tin.ctypes.data_as(C.c_void_p) if tin is not None else None,
                              out.ctypes.data_as(C.c_void_p)))
        return out

    def adapt(self):
        st = AdaptStats()
        _check(load().amr_adapt(self._h, C.byref(st)))
        return {"n_refine": st.n_refine, "n_coarsen": st.n_coarsen, "n_reverted": st.n_reverted,
                "n_free": st.n_free, "level_blocks": list(st.level_blocks)[: self.lmax],
                "step_ms": dict(zip(ADAPT_STEPS, list(st.step_ms)))}

    def n_out(self) -> int:
        return int(self._fields(AMR_GET, F_N_OUT, np.zeros(1, np.int64))[0])

    def output(self):
        n = self.n_out()
        cells = self._fields(AMR_GET, F_CELLS, np.zeros((n, 2), np.int32))
        ru = self._fields(AMR_GET, F_RHO_U, np.zeros((n, 4), np.float64))
        f = self._fields(AMR_GET, F_F, np.zeros((n, self.q), np.float64))
        return {"blk": cells[:, 0].copy(), "cell": cells[:, 1].copy(), "rho": ru[:, 0].copy(),
                "u": ru[:, 1: 1 + self.dim].copy(), "f": f}

    def rho_u_out(self):
        """rho, ux, uy, uz of every output cell (no populations: for large meshes)"""
        n = self.n_out()
        return self._fields(AMR_GET, F_RHO_U, np.zeros((n, 4), np.float64))

    def get_block_f_all(self):
        return self._fields(AMR_GET, F_BLOCK_F, np.zeros((self.cap, self.mb, self.q), np.float64))

    def set_block_f_all(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(self.cap, self.mb, self.q)
        self._fields(AMR_SET, F_BLOCK_F, f)

    def force(self, reset=False):
        """[lmax][4]: momentum exchange with solid blocks per level (x, y, z) summed over
        the level's sweeps since the last reset, and the number of sweeps"""
        out = self._fields(AMR_GET, F_FORCE, np.zeros((self.lmax, 4), np.float64))
        if reset:
            self._fields(AMR_SET, F_FORCE, np.zeros(1, np.float64))
        return out

    def force_accumulation(self, on=None):
        """whether steps accumulate the momentum exchange; with `on`, switch it first"""
        if on is not None:
            self._fields(AMR_SET, F_FORCE_ON, np.array([1 if on else 0], np.int32))
        return bool(self._fields(AMR_GET, F_FORCE_ON, np.zeros(1, np.int32))[0])

    def sync_velocity(self, on=None):
        """whether the synchronisation's averaging also computes the criterion
        velocities; with `on`, switch it first"""
        if on is not None:
            self._fields(AMR_SET, F_SYNC_VELOCITY, np.array([1 if on else 0], np.int32))
        return bool(self._fields(AMR_GET, F_SYNC_VELOCITY, np.zeros(1, np.int32))[0])

    def skip_parents(self, on=None):
        """whether sweeps leave out refined blocks none of whose children has an
        N_SKIP link (linear interpolation); with `on`, switch it first"""
        if on is not None:
            self._fields(AMR_SET, F_SKIP_PARENTS, np.array([1 if on else 0], np.int32))
        return bool(self._fields(AMR_GET, F_SKIP_PARENTS, np.zeros(1, np.int32))[0])

    def stream_bytes(self, value=None):
        """store policy: sweeps writing more than this many bytes use non-temporal
        stores; with `value`, set it first (0 = every level)"""
        if value is not None:
            self._fields(AMR_SET, F_STREAM_BYTES, np.array([int(value)], np.int64))
        return int(self._fields(AMR_GET, F_STREAM_BYTES, np.zeros(1, np.int64))[0])

    def set_collision(self, kind, s_high=1.0):
        """amr_set_collision: COLLIDE_BGK, COLLIDE_MRT or COLLIDE_MRT_MFMA (D3Q27),
        the moments above second order relaxing at s_high"""
        _check(load().amr_set_collision(self._h, int(kind), C.c_double(s_high)))

    def mass_mom_static(self, out_dev):
        """amr_mass_mom_static: enqueue the mass/momentum sums into the caller's
        device buffer `out_dev` (a float64 CUDA tensor of 4 elements)"""
        import torch
        assert out_dev.dtype == torch.float64 and out_dev.is_cuda and out_dev.numel() >= 4
        _check(load().amr_mass_mom_static(self._h, C.c_void_p(out_dev.data_ptr())))
        return out_dev

    def mass_mom(self):
        return self._fields(AMR_GET, F_MASS_MOM, np.zeros(4, np.float64))

    def crit(self):
        return self._fields(AMR_GET, F_CRIT, np.zeros(self.cap, np.float64))

    def counts(self):
        return self._fields(AMR_GET, F_COUNTS, np.zeros(self.lmax, np.int32))

    def parity(self):
        return self._fields(AMR_GET, F_PARITY, np.zeros(self.lmax, np.int32))

    def mesh(self):
        cap, nb, lmax = self.cap, self.nb, self.lmax
        level = self._fields(AMR_GET, F_LEVEL, np.zeros(cap, np.int8))
        status = self._fields(AMR_GET, F_STATUS, np.zeros(cap, np.int8))
        X = self._fields(AMR_GET, F_COORD, np.zeros((3, cap), np.int32))
        nbr = self._fields(AMR_GET, F_NBR, np.zeros((nb, cap), np.int32))
        nbrc = self._fields(AMR_GET, F_NBR_CHILD, np.zeros((nb, cap), np.int32))
        ids = self._fields(AMR_GET, F_IDSET, np.zeros(lmax + lmax * cap, np.int32))
        gap = self._fields(AMR_GET, F_GAP, np.zeros(1 + cap, np.int32))
        lists = ids[lmax:].reshape(lmax, cap)
        return {"level": level, "status": status, "X": np.ascontiguousarray(X.T),
                "nbr": np.ascontiguousarray(nbr.T), "nbrc": np.ascontiguousarray(nbrc.T),
                "ids": [lists[L, : ids[L]].copy() for L in range(lmax)], "gap": gap[1: 1 + gap[0]].copy()}

    def synchronize(self):
        self.stream.synchronize()


class AmrBatch:
    """Several AmrLbm simulations (created on one shared stream) advanced together."""

    def __init__(self, sims, device="cuda"):
        import torch
        self.sims = list(sims)
        lib = load()
        handles = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        self._handles = handles
        nbytes = C.c_uint64(0)
        _check(lib.amr_batch_query_bytes(handles, len(self.sims), C.byref(nbytes)))
        self.arena_bytes = int(nbytes.value)
        self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.arena.data_ptr() + 255) & ~255
        self.stream = self.sims[0].stream
        self.stream.wait_stream(torch.cuda.current_stream(device))  # as in AmrLbm: the arena may be recycled
        h = C.c_void_p(0)
        _check(lib.amr_batch_create(handles, len(self.sims), C.c_void_p(aligned), C.c_uint64(self.arena_bytes),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def step(self, n=1, graph=True, check_finite=False):
        flags = (AMR_USE_GRAPH if graph else 0) | (AMR_CHECK_FINITE if check_finite else 0)
        _check(load().amr_batch_step(self._h, int(n), flags))

    def set_tuning(self, threads=256, wg_per_cu=8, schedule=0):
        t = BatchTuning(int(threads), int(wg_per_cu), int(schedule))
        _check(load().amr_batch_set_tuning(self._h, C.byref(t)))

    def tuning(self):
        t = BatchTuning()
        _check(load().amr_batch_get_tuning(self._h, C.byref(t)))
        return {"threads": t.threads, "wg_per_cu": t.wg_per_cu, "schedule": t.schedule}

    def autotune(self, trial_steps=4):
        t = BatchTuning()
        ms = C.c_double(0)
        _check(load().amr_batch_autotune(self._h, int(trial_steps), C.byref(t), C.byref(ms)))
        return {"threads": t.threads, "wg_per_cu": t.wg_per_cu, "schedule": t.schedule}, float(ms.value)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            load().amr_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
