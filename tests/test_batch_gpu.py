"""Batches of independent simulations (fused persistent launches per level
sweep): every member must end exactly where the same calls on it alone end,
and a member with FP64 storage must still match the oracle."""
import numpy as np
import pytest
import torch

from paper_2308_08085_amd import abi, workloads as W
from parity_util import Pair, assert_cells, block_errors, compare_mesh, field_errors, velocity_scale

pytestmark = pytest.mark.gpu


def mixed_cases():
    """Uneven sizes, depths, lattices and storages, as in a batch of parameter runs."""
    return [
        W.cavity(2, 9, 32, 3, 400.0, storage="f32s", seed=11),
        W.cavity(2, 9, 64, 2, 1000.0, storage="f32s", seed=12),
        W.cavity(3, 19, 16, 3, 200.0, storage="f32s", seed=13),
        W.cavity(3, 19, 32, 2, 400.0, storage="f16s", seed=14),
        W.cavity(2, 9, 16, 4, 100.0, storage="f64", seed=15),
        W.cylinder(3, 27, (32, 16, 16), 4, 8, 3, 100.0, storage="f32s", seed=16, cap=8 * 4 * 4 * 24),
        _cubic(W.cavity(3, 19, 16, 3, 300.0, storage="f32s", seed=17)),
    ]


def _cubic(case):
    case.interp = 1
    return case


def make(cases, stream=None):
    sims = []
    for c in cases:
        g = abi.AmrLbm(c, stream=stream)
        g.set_root_rho_u(c.initial_rho_u())
        sims.append(g)
    return sims


def adapt_all(sims, theta=0.1):
    tags = []
    for g in sims:
        tags.append(g.tag(abi.TAG_VORTICITY_REL, theta=theta))
        g.adapt()
    return tags


def assert_same(a, b, what):
    ma, mb = a.mesh(), b.mesh()
    act = ma["status"] != 8
    for k in ("level", "status", "X", "nbr", "nbrc"):
        assert np.array_equal(ma[k][act], mb[k][act]), "%s: %s differs" % (what, k)
    assert np.array_equal(a.parity(), b.parity()), what + ": parity differs"
    fa, fb = a.get_block_f_all()[act], b.get_block_f_all()[act]
    if not np.array_equal(fa, fb):
        bad = np.argwhere(fa != fb)
        raise AssertionError("%s: %d block populations differ, first %s: %r vs %r" %
                             (what, len(bad), bad[0].tolist(), fa[tuple(bad[0])], fb[tuple(bad[0])]))


def test_batch_equals_members_alone_across_adaptation():
    cases = mixed_cases()
    shared = torch.cuda.Stream()
    batched = make(cases, stream=shared)
    alone = make(cases)
    b = abi.AmrBatch(batched)
    print("batch of", len(cases), "simulations, groups by (q, storage)", flush=True)
    b.step(6, graph=True)
    for g in alone:
        g.step(6)
    t1, t2 = adapt_all(batched), adapt_all(alone)
    for x, y in zip(t1, t2):
        assert np.array_equal(x, y), "tags differ between batched and lone runs"
    # graphs captured before the adaptation are replayed after it
    b.step(5, graph=True)
    b.step(2, graph=False)
    for g in alone:
        g.step(7)
    for i, (x, y) in enumerate(zip(batched, alone)):
        assert_same(x, y, "member %d (%s)" % (i, cases[i].name))
    b.close()


def test_batch_member_matches_oracle_fp64():
    cases = mixed_cases()
    shared = torch.cuda.Stream()
    others = make(cases[:2], stream=shared)
    c = cases[4]
    p = Pair(c, init=False)
    p.g.close()
    p.g = abi.AmrLbm(c, stream=shared)
    ru = c.initial_rho_u()
    p.o.set_root_rho_u(ru)
    p.g.set_root_rho_u(ru)
    b = abi.AmrBatch(others + [p.g])
    for _ in range(2):
        b.step(8)
        p.o.step(8)
        for g in others:
            g.tag(abi.TAG_VORTICITY_REL, theta=0.1)
            g.adapt()
        p.tag_vorticity()
        p.o.adapt()
        p.g.adapt()
    b.step(4)
    p.o.step(4)
    compare_mesh(p.o.mesh(), p.g.mesh(), "after batched steps")
    err = field_errors(p.o.output(), p.g.output(), velocity_scale(c))
    err.update(block_errors(p.o.get_f_all(), p.g.get_block_f_all(), p.o.mesh()["status"]))
    assert_cells(err, 1e-12, "batch member " + c.name, velocity_scale(c))
    b.close()


def test_autotune_keeps_results_and_picks_a_valid_shape():
    cases = [mixed_cases()[i] for i in (0, 2, 3)]
    shared = torch.cuda.Stream()
    batched = make(cases, stream=shared)
    alone = make(cases)
    b = abi.AmrBatch(batched)
    best, ms = b.autotune(trial_steps=1)
    print("autotune:", best, "%.3f ms per coarse step" % ms, flush=True)
    assert best["threads"] in (64, 128, 256) and 1 <= best["wg_per_cu"] <= 64 and best["schedule"] in (0, 1)
    assert ms > 0 and b.tuning() == best
    # every tried shape advanced the members 2 + 1 coarse steps: 2 schedules x 3 x 4 shapes
    n_steps = 2 * 3 * 4 * 3
    for g in alone:
        g.step(n_steps)
    for i, (x, y) in enumerate(zip(batched, alone)):
        assert_same(x, y, "member %d after autotune" % i)
    b.close()


def test_batch_refuses_bad_members():
    c = W.cavity(2, 9, 16, 2, 100.0, storage="f32s", seed=1)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a, d = abi.AmrLbm(c, stream=s1), abi.AmrLbm(c, stream=s2)
    with pytest.raises(abi.AmrError) as e:
        abi.AmrBatch([a, d])
    assert e.value.code == abi.AMR_ERR_ARG
    e2 = abi.AmrLbm(c, stream=s1)
    e2.step(1)
    with pytest.raises(abi.AmrError) as e:
        abi.AmrBatch([a, e2])
    assert e.value.code == abi.AMR_ERR_STATE
    e2.step(1)
    b = abi.AmrBatch([a, e2])
    b.step(2)
    a.step(1)  # stepped outside the batch by an odd number of steps
    with pytest.raises(abi.AmrError) as e:
        b.step(1)
    assert e.value.code == abi.AMR_ERR_STATE
    b.close()


def test_benchmark_batch_sampled_cells_match_the_oracle():
    """The 64-member batch of the benchmark (FP16 shifted storage), one fused
    graph-replayed coarse step in the concurrent-groups schedule: before any
    adaptation every member is one level, so an interior block's new f_p(x) is
    population p of the oracle's BGK collision of the pre-step populations at
    x - c_p.  Two 2-D and two 3-D members, 16 blocks each, every cell."""
    import oracle
    from meshcheck import block_vectors

    cases = W.config5_cases()
    shared = torch.cuda.Stream()
    sims = make(cases, stream=shared)
    b = abi.AmrBatch(sims)
    b.set_tuning(256, 8, 1)
    picks = [0, 1, 32, 33]
    rng = np.random.default_rng(20230808)
    pre = {}
    for i in picks:
        c, g = cases[i], sims[i]
        nbr = g.mesh()["nbr"]
        blocks = np.flatnonzero(np.all(nbr[: c.nroot] >= 0, axis=1))
        sample = rng.choice(blocks, min(16, len(blocks)), replace=False)
        pre[i] = (sample, g.get_block_f_all(), nbr)
    b.step(1, graph=True)
    for i in picks:
        c, g = cases[i], sims[i]
        sample, f, nbr = pre[i]
        d, q = c.dim, c.q
        cv, w, _ = oracle.lattice(d, q)
        vec = np.array(block_vectors(d))
        omega = 1.0 / (3.0 * c.nu0 + 0.5)
        got = g.get_block_f_all()[sample]
        n = 12 if d == 3 else 1
        for s_, B in enumerate(sample):
            # the block and its neighbours as a 12^d region, cell-major
            region = np.zeros((n, 12, 12, q))
            for r in range(len(vec)):
                ox, oy, oz = 4 * (vec[r] + 1)
                blk = f[nbr[B, r]].reshape((4, 4, 4, q) if d == 3 else (1, 4, 4, q))
                region[(oz if d == 3 else 0):(oz + 4 if d == 3 else 1), oy:oy + 4, ox:ox + 4] = blk
            post = {}
            for l in range(c.mb):
                i_, j_, k_ = l & 3, (l >> 2) & 3, l >> 4
                for p in range(q):
                    y = ((4 + k_ - cv[p, 2]) if d == 3 else 0, 4 + j_ - cv[p, 1], 4 + i_ - cv[p, 0])
                    if y not in post:
                        post[y] = oracle.collide(d, q, omega, region[y])
                    want = post[y][p]
                    tol = 2.0 ** -11 * abs(want - w[p]) + 2e-7
                    assert abs(got[s_, l, p] - want) <= tol, (c.name, int(B), l, p, got[s_, l, p], want)
        print("%s: %d sampled blocks match" % (c.name, len(sample)), flush=True)
    b.close()
