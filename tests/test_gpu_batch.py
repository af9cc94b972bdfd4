"""Batched persistent launch (many REV samples in one cooperative kernel).

Every domain of a batch must evolve exactly as the same domain stepped alone
by the single-domain sweep (same cell arithmetic), for every launch shape;
run-to-steady must agree with the FP64 oracle's steady permeability.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1507_06565_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _lbm():
    from paper_1507_06565_amd import lbm
    return lbm


def small_rev(i, edge, seed0=500):
    """Small periodic REV cube with a few spheres (seeded)."""
    rng = np.random.default_rng(seed0 + i)
    n = 3 + i % 3
    S = W.quantise(np.column_stack([rng.uniform(0, edge, n), rng.uniform(0, edge, n), rng.uniform(0, edge, n),
                                    rng.uniform(2.0, edge / 4.0, n)]))
    return W.Domain(edge, edge, edge, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), spheres=S, bc="cli")


def batch_domains():
    edges = [16, 24, 20, 32, 12, 28, 16]
    return [small_rev(i, e) for i, e in enumerate(edges)]


PARAMS = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3 / 16, force=(1e-5, 0.0, 0.0), layout="aa")
LAYOUTS = ["aa", "brick"]  # AA in place, or 4x4x4 bricks with two grids per domain


def params(layout):
    return W.Params(**{**PARAMS.__dict__, "layout": layout})


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_equals_single_domain_runs_bitwise(layout):
    say("test_batch_equals_single_domain_runs_bitwise", layout)
    lbm = _lbm()
    doms = batch_domains()
    ctx = lbm.Context(lbm.Geometry(doms), params(layout))
    ctx.step(37)
    ctx.step(20)
    for i, d in enumerate(doms):
        single = lbm.Context(lbm.Geometry(d), params(layout))
        single.step(57)
        _, u1 = single.fields()
        _, u2 = ctx.fields(i)
        assert np.array_equal(u1, u2), i


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_mixed_step_parities_bitwise(layout):
    """Domains that stopped at different step counts (check every 7 steps, so
    some stop on odd counts) and are then stepped together: each domain's
    state is in the grid of its own parity, and every field still equals a
    single-domain run of the same number of steps bit for bit."""
    say("test_batch_mixed_step_parities_bitwise", layout)
    lbm = _lbm()
    doms = batch_domains()
    ctx = lbm.Context(lbm.Geometry(doms), params(layout))
    steps = ctx.run_to_steady(rel_tol=1e-4, check_every=7, max_steps=700)
    say("steps", steps)
    assert len(set(int(v) % 2 for v in steps)) == 2  # both parities present
    ctx.step(5)
    for i, d in enumerate(doms):
        single = lbm.Context(lbm.Geometry(d), params(layout))
        single.step(int(steps[i]) + 5)
        assert np.array_equal(single.fields()[1], ctx.fields(i)[1]), i


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_launch_shapes_bitwise(layout):
    say("test_batch_launch_shapes_bitwise", layout)
    lbm = _lbm()
    doms = batch_domains()
    base = None
    # AA: workgroups per domain; brick: cells per thread
    shapes = [(256, 1), (512, 2), (1024, 4), (256, 3), (512, 16)] if layout == "aa" else \
        [(256, 1), (512, 2), (1024, 4), (64, 4), (128, 2)]
    for block, w in shapes:
        ctx = lbm.Context(lbm.Geometry(doms), params(layout))
        ctx.batch_set_launch(block, w)
        steps = ctx.run_to_steady(rel_tol=1e-6, check_every=50, max_steps=3000)
        us = [ctx.fields(i)[1] for i in range(len(doms))]
        if base is None:
            base = (steps, us)
        assert np.array_equal(steps, base[0]), (block, w)
        for a, b in zip(us, base[1]):
            assert np.array_equal(a, b), (block, w)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_fixed_steps_parity_with_oracle(layout):
    say("test_batch_fixed_steps_parity_with_oracle", layout)
    lbm = _lbm()
    doms = batch_domains()[:4]
    ctx = lbm.Context(lbm.Geometry(doms), params(layout))
    ctx.step(150)
    for i, d in enumerate(doms):
        ref = oracle.Sim(d, PARAMS)
        ref.step(150)
        _, u = ctx.fields(i)
        fl = np.broadcast_to(ref.fluid(), u.shape)
        e = np.linalg.norm((u - ref.velocity())[fl]) / np.linalg.norm(ref.velocity()[fl])
        say("domain", i, "rel L2", e)
        assert e <= 1e-4


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_run_to_steady_permeability(layout):
    """Steady-state test (relative change of the mean velocity over
    check_every steps) and Darcy permeability (eq. (1)) per sample against
    the oracle run to its own steady state."""
    say("test_batch_run_to_steady_permeability", layout)
    lbm = _lbm()
    doms = [small_rev(0, 16), small_rev(1, 20), small_rev(2, 12)]
    ctx = lbm.Context(lbm.Geometry(doms), params(layout))
    steps = ctx.run_to_steady(rel_tol=1e-7, check_every=100, max_steps=200000)
    say("steps", steps)
    assert np.all(steps < 200000)
    for i, d in enumerate(doms):
        k = ctx.permeability(i, 0)
        ref = oracle.Sim(d, PARAMS)
        prev = None
        for _ in range(2000):
            ref.step(100)
            U = ref.velocity()[0][ref.fluid()].sum()
            if prev is not None and abs(U - prev) <= 1e-10 * abs(U):
                break
            prev = U
        sup, _, _ = oracle.plane_profile(ref.velocity(), ref.fluid(), 2, 0)
        kref = oracle.permeability(sup, 0, d.nz, 1.0 / 6.0, 1.0, 1e-5)
        say("domain", i, "K", k, "oracle", kref)
        assert abs(k / kref - 1) <= 2e-4


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_restart_bitwise(layout):
    say("test_batch_restart_bitwise", layout)
    lbm = _lbm()
    doms = batch_domains()[:3]
    g = lbm.Geometry(doms)
    a = lbm.Context(g, params(layout))
    a.step(21)
    img = a.save()
    a.step(10)
    b = lbm.Context(g, params(layout))
    b.load(img)
    b.step(10)
    for i in range(3):
        assert np.array_equal(a.fields(i)[1], b.fields(i)[1])


def test_rev_workload_samples_permeability():
    """Two cubes of the batched REV workload (edge 32, radii U[3,10]) run to
    steady state in one batched launch; K against the oracle run to its own
    steady state within 1e-4."""
    say("test_rev_workload_samples_permeability")
    lbm = _lbm()
    picks = [0, 7]  # the edge-32 samples among the first indices (porosity 0.69 and 0.80)
    gen = [W.rev_sample_c3(i) for i in picks]
    doms = [g[0] for g in gen]
    params = gen[0][1]
    assert all(d.nx == 32 for d in doms)
    p = W.Params(**{**params.__dict__, "layout": "aa"})
    ctx = lbm.Context(lbm.Geometry(doms), p)
    steps = ctx.run_to_steady(rel_tol=1e-7, check_every=100, max_steps=200000)
    say("steps", steps)
    nu = (params.tau_plus - 0.5) / 3.0
    for i, d in enumerate(doms):
        k = ctx.permeability(i, 0)
        ref = oracle.Sim(d, params)
        prev = None
        for _ in range(3000):
            ref.step(100)
            U = ref.velocity()[0][ref.fluid()].sum()
            if prev is not None and abs(U - prev) <= 1e-10 * abs(U):
                break
            prev = U
        sup, _, _ = oracle.plane_profile(ref.velocity(), ref.fluid(), 2, 0)
        kref = oracle.permeability(sup, 0, d.nz, nu, 1.0, params.force[0])
        say("sample", picks[i], "K", k, "oracle", kref)
        assert abs(k / kref - 1) <= 1e-4


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_steady_in_chunks_matches_one_call(layout):
    """run_to_steady in short launches (samples that converged earlier are
    skipped by the later launches) ends exactly where one long launch ends:
    same steps per sample, same fields bit for bit."""
    say("test_batch_steady_in_chunks_matches_one_call", layout)
    lbm = _lbm()
    doms = batch_domains()
    one = lbm.Context(lbm.Geometry(doms), params(layout))
    s1 = one.run_to_steady(rel_tol=1e-7, check_every=100, max_steps=200000)
    chunked = lbm.Context(lbm.Geometry(doms), params(layout))
    prev = np.zeros(len(doms), np.int64)
    for _ in range(2000):
        s2 = chunked.run_to_steady(rel_tol=1e-7, check_every=100, max_steps=300)
        adv = s2 - prev
        prev = s2
        if np.all(adv < 300):
            break
    say("steps", s1, s2)
    assert np.array_equal(s1, s2)
    for i in range(len(doms)):
        assert np.array_equal(one.fields(i)[1], chunked.fields(i)[1]), i


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rev_workload_representative_permeability(layout):
    """Lowest- and highest-porosity cubes of the smallest (32) and largest (96)
    edge of the batched REV workload, run to steady state together in one
    batched launch; K against the oracle's steady permeability stored in
    golden/rev_k.json (written by golden/make_rev_k.py) within 1e-4."""
    import json
    import os
    say("test_rev_workload_representative_permeability", layout)
    lbm = _lbm()
    with open(os.path.join(os.path.dirname(__file__), "golden", "rev_k.json")) as f:
        gold = json.load(f)
    assert len(gold) == 8 and {g["edge"] for g in gold} == {32, 96}
    gen = [W.rev_sample_c3(g["index"]) for g in gold]
    doms = [x[0] for x in gen]
    p = W.Params(**{**gen[0][1].__dict__, "layout": layout})
    ctx = lbm.Context(lbm.Geometry(doms), p)
    steps = ctx.run_to_steady(rel_tol=1e-7, check_every=100, max_steps=400000)
    say("steps", steps)
    assert np.all(steps < 400000)
    for i, g in enumerate(gold):
        assert doms[i].nx == g["edge"] and abs(gen[i][3] - g["porosity"]) < 1e-12
        k = ctx.permeability(i, 0)
        say("sample", g["index"], "edge", g["edge"], "porosity", round(g["porosity"], 4), "K", k, "oracle", g["K"])
        assert abs(k / g["K"] - 1) <= 1e-4, (g["index"], k, g["K"])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_walled_bouzidi_and_moving_lid_bitwise(layout):
    """Batches of walled domains: spheres between wall layers with Bouzidi
    links, and Couette cells under a moving lid (the lid's partial values are
    seeded per domain); every domain equals its single-domain run bit for bit."""
    say("test_batch_walled_bouzidi_and_moving_lid_bitwise", layout)
    lbm = _lbm()
    rng = np.random.default_rng(77)
    walled = []
    for i, (nx, ny, nz) in enumerate([(16, 12, 20), (24, 8, 16), (12, 16, 24)]):
        S = W.quantise(np.column_stack([rng.uniform(0, nx, 4), rng.uniform(0, ny, 4), rng.uniform(2, nz - 2, 4),
                                        rng.uniform(2.0, 4.5, 4)]))
        walled.append(W.Domain(nx, ny, nz, spheres=S, bc="bouzidi"))
    lids = [W.Domain(8, 4, 20, wall_hi_velocity=(2e-3, 0.0, 0.0), bc="cli"),
            W.Domain(4, 8, 16, wall_hi_velocity=(2e-3, 0.0, 0.0), bc="cli")]
    pw = W.Params(**{**params(layout).__dict__, "force": (1e-5, 0.0, 0.0)})
    pl = W.Params(**{**params(layout).__dict__, "force": (0.0, 0.0, 0.0)})
    for doms, p in ((walled, pw), (lids, pl)):
        ctx = lbm.Context(lbm.Geometry(doms), p)
        ctx.step(33)
        for i, d in enumerate(doms):
            single = lbm.Context(lbm.Geometry(d), p)
            single.step(33)
            assert np.array_equal(single.fields()[1], ctx.fields(i)[1]), (i, d.bc)
