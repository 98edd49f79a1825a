"""The main benchmark set-ups at their full size (D3Q27, 256x128x128 root
cells, near-wall refinement to ~9.3e5 blocks; D2Q9, 1024x256 root cells, 4
levels), in the launch configuration the benchmark times: sampled blocks of
every level and boundary class against the oracle run on their patch, the
synchronisation's interpolation and averaging against the oracle's, and
properties that hold at any size (a uniform flow is a fixed point of the whole
step, the tables satisfy the forest invariants, graph replay equals eager
launches)."""
import time

import numpy as np
import pytest

import oracle
from paper_2308_08085_amd import abi, workloads as W
from meshcheck import block_vectors
from patchcheck import Geometry, block_class, patch, patch_expected

pytestmark = pytest.mark.gpu

U = 0.05


def full_case(solid=True, storage="f32s"):
    case = W.config4(cap=W.config4().nroot * 16, storage=storage)
    if not solid:
        case.solid = None
        case.noise = 0.0
    return case


def refine_near_walls(g, case):
    for _ in range(case.dist_levels):
        g.tag(abi.TAG_DISTANCE, d_spec=case.d_spec, freeze=1)
        g.adapt()


def test_uniform_flow_is_a_fixed_point_at_full_size():
    """no cylinder: inlet and far field at u = (U, 0, 0), outflow at +x; the
    near-outflow refinement still gives three levels"""
    case = full_case(solid=False)
    t0 = time.perf_counter()
    g = abi.AmrLbm(case)
    g.set_root_rho_u(case.initial_rho_u())
    refine_near_walls(g, case)
    counts = g.counts().tolist()
    print("full-size uniform flow: blocks per level", counts, flush=True)
    assert counts[2] > 100000
    g.step(32, graph=True, check_finite=True)
    ru = g.rho_u_out()
    drho = np.abs(ru[:, 0] - 1.0).max()
    du = max(np.abs(ru[:, 1] - U).max(), np.abs(ru[:, 2:]).max())
    print("  %d output cells, max |rho - 1| %.2e, max |u - U| %.2e, %.1f s" %
          (len(ru), drho, du, time.perf_counter() - t0), flush=True)
    assert drho < 1e-5 and du < 1e-6
    g.close()


def _check_forest_invariants(case, m):
    cap, lmax = case.cap, case.lmax
    status, level, X, nbr = m["status"], m["level"], m["X"], m["nbr"]
    active = status != 8
    # the ID sets, the gap stack and the solid root blocks (never used) hold
    # every ID exactly once
    ids = np.concatenate(m["ids"])
    solid = np.flatnonzero(case.solid) if case.solid is not None else np.zeros(0, np.int64)
    every = np.concatenate([ids, m["gap"], solid])
    assert len(every) == cap and np.array_equal(np.sort(every), np.arange(cap)), "IDs not partitioned"
    on = np.zeros(cap, bool)
    on[ids] = True
    assert np.array_equal(on, active), "ID sets differ from the active blocks"
    for L in range(lmax):
        assert np.all(level[m["ids"][L]] == L), "level %d list holds other levels" % L
    # same-level links: reciprocal and geometric (no periodic axes here)
    vec = np.array(block_vectors(case.dim))
    opp = np.array([next(k for k in range(len(vec)) if np.all(vec[k] == -vec[p])) for p in range(len(vec))])
    W0 = 4 << (lmax - 1)
    act = np.flatnonzero(active)
    for p in range(1, len(vec)):
        B = act
        N = nbr[B, p]
        ok = N >= 0
        B, N = B[ok], N[ok]
        assert np.all(active[N]), "link to an inactive block"
        assert np.all(level[N] == level[B]), "link between levels"
        assert np.all(nbr[N, opp[p]] == B), "link %d not reciprocal" % p
        width = (W0 >> level[B].astype(np.int64))[:, None]
        assert np.array_equal(X[N].astype(np.int64), X[B].astype(np.int64) + vec[p][None, :] * width), \
            "link %d not at the neighbouring position" % p
    # children tile their parents
    refined = act[np.isin(status[act], (1, 2, 3))]
    first = m["nbrc"][refined, 0]
    assert np.all(first >= 0)
    for c in range(8):
        ch = first + c
        off = np.array([c & 1, (c >> 1) & 1, c >> 2])
        half = ((W0 >> level[refined].astype(np.int64)) // 2)[:, None]
        assert np.all(level[ch] == level[refined] + 1)
        assert np.array_equal(X[ch].astype(np.int64), X[refined].astype(np.int64) + off[None, :] * half)


def test_forest_invariants_at_full_size_after_adaptation():
    case = full_case()
    g = abi.AmrLbm(case)
    g.set_root_rho_u(case.initial_rho_u())
    refine_near_walls(g, case)
    _check_forest_invariants(case, g.mesh())
    # the wake needs a few adaptation periods before the criterion changes the mesh
    for period in range(4):
        g.step(case.adapt_every, graph=True)
        g.tag(abi.TAG_VORTICITY_REL, theta=case.theta)
        st = g.adapt()
        print("full-size adaptation after period %d:" % (period + 1), st, flush=True)
        if st["n_refine"] + st["n_coarsen"] > 0:
            break
    assert st["n_refine"] + st["n_coarsen"] > 0
    _check_forest_invariants(case, g.mesh())
    g.close()


def test_graph_replay_equals_eager_at_full_size():
    case = full_case()
    runs = []
    for graph in (True, False):
        g = abi.AmrLbm(case)
        g.set_root_rho_u(case.initial_rho_u())
        refine_near_walls(g, case)
        g.step(8, graph=graph)
        runs.append(g.mass_mom())
        g.close()
        del g
    print("mass/momentum graph %s eager %s" % (runs[0], runs[1]), flush=True)
    assert np.array_equal(runs[0], runs[1])


def _tolerance(storage, g_scale, n):
    """n sweeps, each rounding the stored shifted values (half an ulp: 2^-24
    relative in FP32, 2^-11 in FP16) plus the FP32 arithmetic (2e-7)"""
    ulp = 2.0 ** -11 if storage == "f16s" else 2.0 ** -24
    return n * (ulp * g_scale + 2e-7)


def _patch_check(case, g, m, per_class=16):
    """leaf blocks of every level and class (interior, domain faces, solid
    neighbours, refined neighbours), one coarse step against the oracle run on
    the block's patch (patchcheck.py)"""
    geo = Geometry(case, m)
    rng = np.random.default_rng(20230808)
    leaves = np.flatnonzero(m["status"] == 0)
    rng.shuffle(leaves)
    picked, counts = [], {}
    for B in leaves:
        L = int(m["level"][B])
        key = (L, block_class(m, B))
        if counts.get(key, 0) >= per_class:
            continue
        p = patch(geo, int(B), 2 ** L)
        if p is None:
            continue
        picked.append((int(B), L, key, p))
        counts[key] = counts.get(key, 0) + 1
    need = sorted({N for _, _, _, p in picked for N in p[1].values()})
    fall = g.get_block_f_all()
    fpre = {N: fall[N].copy() for N in need}
    del fall
    g.step(1, graph=True)
    fall = g.get_block_f_all()
    got = {B: fall[B].copy() for B, _, _, _ in picked}
    del fall
    _, w, _ = oracle.lattice(case.dim, case.q)
    worst = {}
    for B, L, key, p in picked:
        want = patch_expected(*p, fpre, 2 ** L)
        g_scale = np.abs(want - w).max(axis=1, keepdims=True)
        r = (np.abs(got[B] - want) / _tolerance(case.storage, g_scale, 2 ** L)).max()
        worst[key] = max(worst.get(key, 0.0), float(r))
    print("  patch check, blocks per (level, class): %s" % sorted(counts.items()), flush=True)
    print("  max error / tolerance per (level, class): %s" % {k: round(v, 3) for k, v in sorted(worst.items())},
          flush=True)
    assert max(worst.values()) <= 1.0, worst
    return counts


def _sync_check(case, g, m, per_level=24):
    """pre-adaptation synchronisation at full size: ghost cells of sampled
    children equal the oracle's interpolation of their parent's final cells,
    and parent cells whose fine cells are not ghosts the oracle's average of
    the children (Secs. "Linear Interpolation", "Averaging")"""
    d, q = case.dim, case.q
    mb, nc = (16, 4) if d == 2 else (64, 8)
    g.tag(tags_in=np.zeros(case.cap, np.int8))  # the synchronisation only
    n_out = g.n_out()
    cells = g._fields(abi.AMR_GET, abi.F_CELLS, np.zeros((n_out, 2), np.int32))
    out = np.zeros((case.cap, mb), bool)
    out[cells[:, 0], cells[:, 1]] = True
    del cells
    f = g.get_block_f_all()
    ro = oracle.Oracle(W.Case(name="ratios", dim=d, q=q, root=(1, 1, 1), lmax=case.lmax, nu0=case.nu0, cap=1))
    _, w, _ = oracle.lattice(d, q)
    geo = Geometry(case, m)
    rng = np.random.default_rng(7)
    worst_i = worst_a = 0.0
    n_i = n_a = 0
    for L in range(case.lmax - 1):
        r_cf, r_fc = ro.ratios(L)
        parents = np.flatnonzero((m["level"] == L) & np.isin(m["status"], (1, 2, 3)))
        # children with ghost cells (a coarser neighbour) and their parents
        kids = np.flatnonzero((m["level"] == L + 1) & (m["status"] == 0) & np.any(m["nbr"] == -2, axis=1))
        for C in rng.choice(kids, min(per_level, len(kids)), replace=False):
            wc = geo.width(L + 1)
            xp = [int(v) - int(v) % (2 * wc) for v in m["X"][C]]
            where = geo.at(L, xp)
            assert where[0] == "block", (C, where)
            P = where[1]
            c = sum(((int(m["X"][C][a]) - xp[a]) // wc) << a for a in range(d))
            want = oracle.interp_child(d, q, r_cf, f[P], c)
            ghost = ~out[C]
            assert ghost.any()
            gs = np.abs(want[ghost] - w).max(axis=1, keepdims=True)
            r = (np.abs(f[C][ghost] - want[ghost]) / _tolerance(case.storage, gs, 1)).max()
            worst_i, n_i = max(worst_i, float(r)), n_i + 1
        for P in rng.choice(parents, min(per_level, len(parents)), replace=False):
            first = int(m["nbrc"][P, 0])
            kids_f = f[first: first + nc]
            kid_ok = [out[first + c] if m["status"][first + c] == 0 else np.ones(mb, bool) for c in range(nc)]
            want = oracle.average_parent(d, q, r_fc, kids_f)
            for l in range(mb):
                i, j, k = l & 3, (l >> 2) & 3, l >> 4
                c = (i >> 1) + 2 * (j >> 1) + 4 * (k >> 1)
                fine = [(2 * (i & 1) + a) + 4 * (2 * (j & 1) + b) + 16 * (2 * (k & 1) + e)
                        for e in range(2 if d == 3 else 1) for b in range(2) for a in range(2)]
                if not all(kid_ok[c][x] for x in fine):
                    continue
                gs = np.abs(want[l] - w).max()
                r = (np.abs(f[P][l] - want[l]) / _tolerance(case.storage, gs, 1)).max()
                worst_a, n_a = max(worst_a, float(r)), n_a + 1
    del f
    print("  sync: %d children's ghost cells, %d parent cells; max error / tolerance %.3f (interpolation), "
          "%.3f (averaging)" % (n_i, n_a, worst_i, worst_a), flush=True)
    assert n_i > 0 and n_a > 0
    assert worst_i <= 1.0 and worst_a <= 1.0


def _full_size_check(case):
    """the benchmark's launch configuration (graph replay, non-temporal stores
    on every level above 128 MiB): one coarse step of sampled leaves against
    the patch oracle, then the synchronisation's interpolation and averaging"""
    t0 = time.perf_counter()
    g = abi.AmrLbm(case)
    g.set_root_rho_u(case.initial_rho_u())
    refine_near_walls(g, case)
    g.step(6, graph=True)  # a developing flow near the cylinder
    m = g.mesh()
    print("full-size %s %s: blocks per level %s" % (case.name, case.storage, g.counts().tolist()), flush=True)
    counts = _patch_check(case, g, m)
    levels = {L for L, _ in counts}
    assert levels == set(range(case.lmax)), counts
    assert (case.lmax - 1, "solid") in counts and (case.lmax - 1, "face") in counts and (0, "face") in counts
    _sync_check(case, g, g.mesh())
    print("  %.1f s" % (time.perf_counter() - t0), flush=True)
    g.close()


@pytest.mark.parametrize("storage", ["f32s", "f16s"])
def test_sampled_blocks_match_the_oracle_at_full_size(storage):
    """the D3Q27 cylinder of the benchmark"""
    _full_size_check(full_case(storage=storage))


@pytest.mark.parametrize("storage", ["f32s", "f16s"])
def test_sampled_blocks_match_the_oracle_d2q9_cylinder(storage):
    """the D2Q9 square cylinder: 1024 x 256 root cells, D = 32, 4 levels"""
    case = W.config3(cap=W.config3().nroot * 12, storage=storage)
    _full_size_check(case)
