"""Oracle checks of single blocks of a mesh of any size (test helper).

A leaf block of level L advances by 2^L collide-stream sweeps of its level per
coarse step (Sec. "Grid Advancement").  A sweep moves information by one cell,
so after n <= 4 R sweeps the block's cells depend only on the blocks within R
block widths of it.  When those blocks are same-level leaves without a coarser
neighbour (no ghost cells, nothing interpolated or averaged into them during
the step), the block's new state is that of a small single-level oracle run on
this patch: the patch's pre-step populations, its solid blocks, the domain
faces it touches with their conditions, n sweeps at the level's relaxation
time.  Patch sides inside the domain are cut; whatever the oracle does there
stays more than n cells away from the checked block.  On level 0 (one sweep)
neighbours may be refined blocks, which the level's sweep advances too.

The ghost fill and the averaging of the pre-adaptation synchronisation are
checked cell by cell with the oracle's interpolation and averaging of the
GPU's own data.
"""
import numpy as np

import oracle
from paper_2308_08085_amd import workloads as W

CUT_PRIO = 0  # a cut side never wins an edge or corner against a domain face


class Geometry:
    """same-level block lookup by position on a fetched mesh"""

    def __init__(self, case, mesh):
        assert not any(case.periodic), "periodic axes are not handled"
        self.case, self.m = case, mesh
        self.dim = case.dim
        self.W0 = 4 << (case.lmax - 1)
        root = list(case.root) + [1] * (3 - len(case.root))
        self.root = root
        self.dom = [root[a] * self.W0 if a < case.dim else 1 for a in range(3)]
        act = np.flatnonzero(mesh["status"] != 8)
        X = mesh["X"][act].astype(np.int64)
        L = mesh["level"][act].astype(np.int64)
        key = ((L << 60) | (X[:, 2] << 40) | (X[:, 1] << 20) | X[:, 0])
        self.index = dict(zip(key.tolist(), act.tolist()))

    def width(self, L):
        return 4 << (self.case.lmax - 1 - L)

    def at(self, L, x):
        """('block', id) | ('solid',) | ('missing',) for an in-domain position"""
        r = [x[a] // self.W0 if a < self.dim else 0 for a in range(3)]
        rid = r[0] + self.root[0] * (r[1] + self.root[1] * r[2])
        if self.case.solid is not None and self.case.solid[rid]:
            return ("solid",)
        B = self.index.get((L << 60) | (x[2] << 40) | (x[1] << 20) | x[0])
        return ("block", B) if B is not None else ("missing",)


def patch(geo, B, nsweeps):
    """The single-level oracle set-up of the patch around leaf B: (tiny case,
    {tiny root index: block id}, tiny index of B) or None when the patch holds
    a position covered by a coarser or finer block, or (nsweeps > 1) a block
    that is not a leaf or has a coarser neighbour."""
    case, m, dim = geo.case, geo.m, geo.dim
    L = int(m["level"][B])
    w = geo.width(L)
    R = (nsweeps + 3) // 4
    X = [int(v) for v in m["X"][B]]
    lo, hi = [0, 0, 0], [0, 0, 0]
    for a in range(dim):
        lo[a] = max(-R, -(X[a] // w))
        hi[a] = min(R, (geo.dom[a] - X[a]) // w - 1)
    n = [hi[a] - lo[a] + 1 for a in range(3)]
    kind, fu, prio = [0] * 6, [(0.0, 0.0, 0.0)] * 6, [CUT_PRIO] * 6
    for a in range(dim):
        if X[a] + lo[a] * w == 0:
            kind[2 * a], fu[2 * a], prio[2 * a] = case.face_kind[2 * a], case.face_u[2 * a], case.face_prio[2 * a]
        if X[a] + (hi[a] + 1) * w == geo.dom[a]:
            kind[2 * a + 1], fu[2 * a + 1], prio[2 * a + 1] = (case.face_kind[2 * a + 1], case.face_u[2 * a + 1],
                                                             case.face_prio[2 * a + 1])
    solid = np.zeros(n[0] * n[1] * n[2], np.uint8)
    blocks = {}
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                v = (lo[0] + i, lo[1] + j, lo[2] + k)
                x = [X[a] + v[a] * w for a in range(3)]
                t = i + n[0] * (j + n[1] * k)
                where = geo.at(L, x)
                if where[0] == "missing":
                    return None
                if where[0] == "solid":
                    solid[t] = 1
                    continue
                N = where[1]
                if nsweeps > 1 and (m["status"][N] != 0 or np.any(m["nbr"][N] == -2)):
                    return None
                blocks[t] = N
    tiny = W.Case(name="patch", dim=dim, q=case.q, root=(n[0], n[1], n[2]), lmax=1, nu0=case.nu0 * 2 ** L,
                  cap=n[0] * n[1] * n[2], face_kind=tuple(kind), face_u=tuple(tuple(u) for u in fu),
                  face_prio=tuple(prio), solid=solid if solid.any() else None)
    return tiny, blocks, (-lo[0]) + n[0] * ((-lo[1]) + n[1] * (-lo[2]))


def patch_expected(tiny, blocks, centre, fpre, nsweeps):
    """the oracle's state of the centre block after nsweeps sweeps of the patch;
    fpre[id] = pre-step populations [Mb][q] of block id"""
    o = oracle.Oracle(tiny)
    for t, N in blocks.items():
        o.set_block_f(t, fpre[N])
    o.step(nsweeps)
    return o.get_block_f(centre)


def block_class(m, B):
    codes = m["nbr"][B]
    if np.any(codes == -9):
        return "solid"
    if np.any((codes <= -3) & (codes >= -8)):
        return "face"
    if m["level"][B] == 0 and np.any([m["status"][N] != 0 for N in codes if N >= 0]):
        return "next to refined"
    return "interior"
