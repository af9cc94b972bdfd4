"""The layout autotuner (lbm_autotune_layout): it times the candidate
layouts of a geometry and returns one of them; the choice is cached per
shape; a context built with layout "auto" uses it and gives the same fields
as every fixed layout, bit for bit."""
import sys

import numpy as np
import pytest

from paper_1507_06565_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bed(seed=5):
    S, _ = W.porous_bed(seed, 64, 32, 64, 32, (3.0, 5.0), 0.6)
    return W.Domain(64, 32, 64, spheres=S, bc="cli", name="bed-64x32x64")


def test_layout_autotuner_single_domain():
    import torch

    from paper_1507_06565_amd import lbm

    dom = _bed()
    p = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3 / 16, force=(1e-5, 0, 0), layout="auto")
    geo = lbm.Geometry(dom)
    name, ms = lbm.autotune_layout(geo, p, steps_per_trial=6)
    say("chosen layout", name, ms)
    assert name in ("twogrid", "aa", "brick") and ms > 0
    # cached: the same answer without a buffer
    assert lbm.autotune_layout(geo, p)[0] == name
    # the caches travel as text: the layout choice and the tuned launch of
    # every candidate are in the export, and importing it back changes nothing
    text = lbm.tuning_export()
    lay_id = {"twogrid": 0, "aa": 1, "brick": 2}[name]
    assert any(l.startswith("layout ") and l.split()[3:6] == [str(dom.nx), str(dom.ny), str(dom.nz)]
               and l.split()[9] == str(lay_id) for l in text.splitlines()), text
    assert sum(l.startswith("sweep ") and l.split()[2:5] == [str(dom.nx), str(dom.ny), str(dom.nz)]
               for l in text.splitlines()) >= 2, text
    lbm.tuning_import(text)
    assert lbm.tuning_export() == text
    # a context with layout "auto" runs the chosen layout; fields equal every fixed layout's
    out = {}
    for lay in ("auto", "twogrid", "aa", "brick"):
        ctx = lbm.Context(geo, W.Params(**{**p.__dict__, "layout": lay}))
        ctx.step(40)
        out[lay] = ctx.fields()
        del ctx
        torch.cuda.synchronize()
    for lay in ("twogrid", "aa", "brick"):
        assert np.array_equal(out[lay][0], out["auto"][0]) and np.array_equal(out[lay][1], out["auto"][1]), lay


def test_layout_autotuner_batch():
    from paper_1507_06565_amd import lbm

    doms = []
    for i, (edge, eps) in enumerate(((32, 0.5), (48, 0.7), (32, 0.8))):
        S, _ = W.rev_cube(700 + i, edge, (3.0, 6.0), eps)
        doms.append(W.Domain(edge, edge, edge, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0),
                             spheres=S, bc="cli", name=f"rev-{i}"))
    p = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3 / 16, force=(1e-6, 0, 0), layout="auto")
    geo = lbm.Geometry(doms)
    name, ms = lbm.autotune_layout(geo, p, steps_per_trial=6)
    say("batch layout", name, ms)
    assert name in ("aa", "brick")
    ctx = lbm.Context(geo, p)
    ctx.step(30)
    ref = lbm.Context(geo, W.Params(**{**p.__dict__, "layout": "aa" if name == "brick" else "brick"}))
    ref.step(30)
    for d in range(3):
        a, b = ctx.fields(d), ref.fields(d)
        assert np.array_equal(a[1], b[1]), d
