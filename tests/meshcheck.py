"""Brute-force geometric checks of a forest's tables (test helper).

Given only the block origins, levels and statuses, finds every block's
neighbours by searching all active blocks (O(N^2)), and checks the invariants a
2:1-balanced forest of quad/octrees must satisfy.  Independent of how either
implementation computes its links.
"""
import itertools

import numpy as np

ST_INACTIVE = 8
REFINED = (1, 2, 3)


def block_vectors(dim):
    """neighbour direction vectors in the numbering of the paper's velocity-set figure"""
    if dim == 2:
        return [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0), (1, 1, 0), (-1, 1, 0),
                (-1, -1, 0), (1, -1, 0)]
    return [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
            (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
            (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1),
            (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1), (1, -1, 1), (-1, 1, -1),
            (-1, 1, 1), (1, -1, -1)]


def expected_links(case, mesh):
    """Geometric neighbour table for every active block."""
    dim, lmax = case.dim, case.lmax
    root = list(case.root) + [1] * (3 - len(case.root))
    W0 = 4 << (lmax - 1)
    dom = [root[a] * W0 for a in range(3)]
    vec = block_vectors(dim)
    level, status, X = mesh["level"], mesh["status"], mesh["X"]
    active = [B for B in range(case.cap) if status[B] != ST_INACTIVE]
    index = {}
    for B in active:
        index[(int(level[B]), int(X[B, 0]), int(X[B, 1]), int(X[B, 2]))] = B
    solid = case.solid
    out = {}
    for B in active:
        L = int(level[B])
        Wl = 4 << (lmax - 1 - L)
        row = []
        for p, v in enumerate(vec):
            r = [int(X[B, a]) + v[a] * Wl for a in range(3)]
            crossed = []
            for a in range(dim):
                if r[a] < 0:
                    if case.periodic[a]:
                        r[a] += dom[a]
                    else:
                        crossed.append(2 * a)
                elif r[a] >= dom[a]:
                    if case.periodic[a]:
                        r[a] -= dom[a]
                    else:
                        crossed.append(2 * a + 1)
            if crossed:
                best = crossed[0]
                for fc in crossed[1:]:
                    if case.face_prio[fc] > case.face_prio[best]:
                        best = fc
                row.append(-3 - best)
                continue
            rb = [r[a] // W0 for a in range(3)]
            rid = rb[0] + root[0] * (rb[1] + root[1] * rb[2])
            if solid is not None and solid[rid]:
                row.append(-9)
                continue
            row.append(index.get((L, r[0], r[1], r[2]), -2))
        out[B] = row
    return out


def check_forest(case, mesh):
    """Assert every invariant of a valid forest; returns the number of active blocks."""
    dim, lmax, cap = case.dim, case.lmax, case.cap
    nc = 4 if dim == 2 else 8
    level, status, X, nbr, nbrc = mesh["level"], mesh["status"], mesh["X"], mesh["nbr"], mesh["nbrc"]
    W0 = 4 << (lmax - 1)
    root = list(case.root) + [1] * (3 - len(case.root))
    active = [B for B in range(cap) if status[B] != ST_INACTIVE]
    exp = expected_links(case, mesh)
    # (1) links equal the geometric search
    for B in active:
        assert list(nbr[B]) == exp[B], (B, list(nbr[B]), exp[B])
    # (2) neighbour-children: first child of a refined neighbour, NONE for a leaf, the code if negative
    for B in active:
        for p in range(len(exp[B])):
            n = nbr[B, p]
            if n < 0:
                want = n
            elif status[n] in REFINED:
                want = nbrc[n, 0]
            else:
                want = -1
            assert nbrc[B, p] == want, (B, p)
    # (3) children contiguous, one level down, tiling the parent
    for B in active:
        if status[B] in REFINED:
            c0 = nbrc[B, 0]
            Wc = 4 << (lmax - 2 - int(level[B]))
            for c in range(nc):
                ch = c0 + c
                assert status[ch] != ST_INACTIVE and level[ch] == level[B] + 1
                cv = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
                for a in range(3):
                    assert X[ch, a] == X[B, a] + cv[a] * Wc
        else:
            assert status[B] == 0, (B, status[B])
    # (4) leaves partition the fluid domain; 2:1 balance including edges and corners
    leaves = [B for B in active if status[B] == 0]
    vol = sum((4 << (lmax - 1 - int(level[B]))) ** dim for B in leaves)
    nsolid = 0 if case.solid is None else int(case.solid.sum())
    dom_vol = int(np.prod([root[a] * W0 for a in range(dim)])) - nsolid * W0 ** dim
    assert vol == dom_vol
    fine = {}
    for B in leaves:
        W = 4 << (lmax - 1 - int(level[B]))
        fine[B] = (np.array(X[B, :dim]), W)
    for B in leaves:
        for p, n in enumerate(nbr[B]):
            if n == -2:  # region covered by a coarser leaf: the parent's neighbour must be a leaf
                assert level[B] > 0
    # 2:1 across any touching pair of leaves
    lv = np.array([int(level[B]) for B in leaves])
    lo = np.array([fine[B][0] for B in leaves])
    wd = np.array([fine[B][1] for B in leaves])
    dom = np.array([root[a] * W0 for a in range(dim)])
    for i, B in enumerate(leaves):
        gap = np.zeros((len(leaves), dim))
        for a in range(dim):
            d1 = lo[:, a] - (lo[i, a] + wd[i])
            d2 = lo[i, a] - (lo[:, a] + wd)
            g = np.maximum(np.maximum(d1, d2), 0)
            if case.periodic[a]:
                d1p = (lo[:, a] + dom[a]) - (lo[i, a] + wd[i])
                d2p = lo[i, a] - (lo[:, a] + dom[a] + wd)
                g = np.minimum(g, np.maximum(np.maximum(d1p, d2p), 0))
                d1m = (lo[:, a] - dom[a]) - (lo[i, a] + wd[i])
                d2m = lo[i, a] - (lo[:, a] - dom[a] + wd)
                g = np.minimum(g, np.maximum(np.maximum(d1m, d2m), 0))
            gap[:, a] = g
        touch = (gap.max(1) == 0)
        assert np.all(np.abs(lv[touch] - lv[i]) <= 1), B
    # (5) ID sets hold exactly the active blocks of each level; with the gap stack and
    #     the solid roots they cover [0, cap) once
    seen = np.zeros(cap, np.int32)
    for L in range(lmax):
        for B in mesh["ids"][L]:
            assert level[B] == L and status[B] != ST_INACTIVE
            seen[B] += 1
    for B in mesh["gap"]:
        seen[B] += 1
    if case.solid is not None:
        seen[: case.nroot][case.solid.astype(bool)] += 1
    assert np.all(seen == 1)
    # (6) link symmetry between same-level blocks
    vec = block_vectors(dim)
    opp = [vec.index(tuple(-x for x in v)) for v in vec]
    for B in active:
        for p, n in enumerate(nbr[B]):
            if n >= 0:
                assert nbr[n, opp[p]] == B
    return len(active)


def random_tags(case, mesh, rng, p_ref=0.3, p_coa=0.3):
    tags = np.zeros(case.cap, np.int8)
    for B in range(case.cap):
        if mesh["status"][B] == ST_INACTIVE:
            continue
        r = rng.random()
        if r < p_ref:
            tags[B] = 1
        elif r < p_ref + p_coa:
            tags[B] = -1
    return tags


def all_offsets(dim):
    return list(itertools.product((-1, 0, 1), repeat=dim))
