"""Brick layout (4x4x4 bricks, bricks without fluid cells not stored) through
the C ABI.

The brick layout streams like the two-grid layout (pull from x - e_k, store at
x) with the same cell arithmetic, so its fields must equal the two-grid
layout's bit for bit, for every boundary scheme, periodic and walled axes, a
moving lid, dropped (all-solid) bricks and every launch shape; the reductions
read it through the brick map, so profiles, totals, permeability and the
steady-state test must agree bit for bit too.  Parity with the FP64 oracle
then follows, and is checked directly as well.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1507_06565_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
P = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3 / 16, force=(2e-5, 0, 0))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _lbm():
    from paper_1507_06565_amd import lbm
    return lbm


def ctx_for(d, p, layout, block=None, flags=0):
    lbm = _lbm()
    ctx = lbm.Context(lbm.Geometry(d), W.Params(**{**p.__dict__, "layout": layout}))
    if block is not None:
        ctx.set_launch(block, flags)
    return ctx


def spheres(seed, shape, bc, periodic=False, n=14, r=(2.5, 6.5)):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    zlo, zhi = (0, nz) if periodic else (1, nz - 1)
    S = W.quantise(np.column_stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(zlo, zhi, n),
                                    rng.uniform(r[0], r[1], n)]))
    if periodic:
        return W.Domain(nx, ny, nz, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), spheres=S, bc=bc)
    return W.Domain(nx, ny, nz, spheres=S, bc=bc)


def solid_bricks(d):
    """Number of 4x4x4 bricks without a fluid cell (dropped by the layout)."""
    f = oracle.flags(d) == 0
    b = f.reshape(d.nz // 4, 4, d.ny // 4, 4, d.nx // 4, 4).any(axis=(1, 3, 5))
    return int((~b).sum())


CASES = {
    "cli-walls": lambda: spheres(3, (48, 40, 36), "cli"),
    "bouzidi-periodic": lambda: spheres(4, (32, 32, 32), "bouzidi", periodic=True, n=10),
    "sbb-walls": lambda: spheres(5, (40, 24, 28), "sbb"),
    "cli-large-grains": lambda: spheres(6, (48, 48, 48), "cli", periodic=True, n=10, r=(8.0, 13.0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_brick_equals_twogrid_bitwise(case):
    say("test_brick_equals_twogrid_bitwise", case)
    d = CASES[case]()
    if case == "cli-large-grains":
        assert solid_bricks(d) > 20  # the case drops bricks
    for n in (1, 2, 57):
        a = ctx_for(d, P, "twogrid")
        b = ctx_for(d, P, "brick")
        a.step(n)
        b.step(n)
        ra, ua = a.fields()
        rb, ub = b.fields()
        assert np.array_equal(ua, ub) and np.array_equal(ra, rb), (case, n)


def test_brick_moving_lid():
    """Couette flow between a resting wall and a moving lid (the lid's partial
    values are seeded in storage order): bitwise equal to two-grid and exact."""
    say("test_brick_moving_lid")
    d = W.Domain(8, 4, 20, wall_hi_velocity=(2e-3, 0.0, 0.0), bc="cli")
    p = W.Params(collision="trt", tau_plus=0.8, magic_lambda=0.25, force=(0, 0, 0))
    a = ctx_for(d, p, "twogrid")
    b = ctx_for(d, p, "brick")
    a.step(8000)  # about 2.5 diffusion times of the 18-cell gap
    b.step(8000)
    ua, ub = a.fields()[1], b.fields()[1]
    assert np.array_equal(ua, ub)
    z = np.arange(20)
    exact = 2e-3 * (z - 0.5) / 18
    fl = slice(1, 19)
    assert np.max(np.abs(ub[0, fl, 0, 0] - exact[fl])) <= 1e-6 * 2e-3 * 10


def test_brick_launch_shapes_bitwise():
    say("test_brick_launch_shapes_bitwise")
    d = spheres(7, (64, 20, 32), "bouzidi")
    a = ctx_for(d, P, "twogrid")
    a.step(41)
    base = a.fields()[1]
    # flags: XCD remap 1, non-temporal 2, two / four cells per thread 4 / 8
    for block in (64, 128, 256, 512, 1024):
        for flags in (0, 1, 2, 3, 4, 8, 4 | 2, 8 | 1):
            b = ctx_for(d, P, "brick", block, flags)
            b.step(41)
            assert np.array_equal(b.fields()[1], base), (block, flags)


def test_brick_oracle_parity():
    say("test_brick_oracle_parity")
    d = spheres(8, (48, 40, 36), "cli")
    b = ctx_for(d, P, "brick")
    b.step(300)
    ref = oracle.Sim(d, P)
    ref.step(300)
    u = b.fields()[1]
    m = np.broadcast_to(ref.fluid(), u.shape)
    e = float(np.linalg.norm((u - ref.velocity())[m]) / np.linalg.norm(ref.velocity()[m]))
    say("brick vs oracle rel L2", e)
    assert e <= REL_L2


def test_brick_reductions_and_steady_state_bitwise():
    say("test_brick_reductions_and_steady_state_bitwise")
    d = spheres(9, (32, 32, 32), "cli", periodic=True, n=10)
    p = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3 / 16, force=(1e-5, 0, 0))
    a = ctx_for(d, p, "twogrid")
    b = ctx_for(d, p, "brick")
    sa = a.run_to_steady(1e-7, 100, 100000)
    sb = b.run_to_steady(1e-7, 100, 100000)
    assert np.array_equal(sa, sb) and sa[0] < 100000
    for axis in (0, 1, 2):
        for comp in (0, 1, 2):
            pa, pb = a.average_profile(0, axis, comp), b.average_profile(0, axis, comp)
            for x, y in zip(pa, pb):
                assert np.array_equal(x, y), (axis, comp)
    assert a.totals()[0] == b.totals()[0] and np.array_equal(a.totals()[1], b.totals()[1])
    assert a.permeability() == b.permeability()


def test_brick_split_runs_and_restart_bitwise():
    say("test_brick_split_runs_and_restart_bitwise")
    d = spheres(10, (48, 40, 36), "cli")
    a = ctx_for(d, P, "brick")
    a.step(37)
    a.step(26)
    b = ctx_for(d, P, "brick")
    b.step(63)
    assert np.array_equal(a.fields()[1], b.fields()[1])
    img = a.save()
    a.step(15)
    c = ctx_for(d, P, "brick")
    c.load(img)
    assert c.steps_done() == 63
    c.step(15)
    assert np.array_equal(a.fields()[1], c.fields()[1])


def test_brick_all_solid_domain():
    """No brick is stored: steps and reductions still work and report no flow."""
    lbm = _lbm()
    d = W.Domain(8, 8, 8, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0),
                 spheres=np.array([[4.0, 4.0, 4.0, 7.9375]]))
    p = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3 / 16, force=(1e-5, 0, 0), layout="brick")
    ctx = lbm.Context(lbm.Geometry(d), p)
    ctx.step(5)
    rho, u = ctx.fields()
    assert np.all(u == 0) and np.all(rho == 0)
    m, j = ctx.totals()
    assert m == 0 and np.all(j == 0)
    assert ctx.permeability() == 0
    assert ctx.run_to_steady(1e-7, 10, 1000)[0] <= 1000
