"""Host-side checks of the library (no GPU): exported symbols, the host
geometry build against the oracle bit for bit, and argument validation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1507_06565_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:lbm_status|void|const char\*|int32_t|int64_t)\s+\**\s*(\w+)\s*\(", txt, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    from paper_1507_06565_amd import _lib
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(_lib.lib, n), n
        assert n in _lib.EXPORTS, f"{n} has no ctypes signature in the binding"


@pytest.mark.parametrize("which", ["c0", "small", "periodic", "c1", "c3"])
def test_geometry_bitwise_equal_to_oracle(which):
    """Flags, link set, directions and q of the library's host geometry equal
    the oracle's bit for bit (exact dyadic arithmetic + one IEEE sqrt)."""
    from paper_1507_06565_amd import lbm
    if which == "c0":
        d, _ = W.channel_c0()
    elif which == "small":
        rng = np.random.default_rng(9)
        S = W.quantise(np.column_stack([rng.uniform(0, 40, 12), rng.uniform(0, 30, 12),
                                        rng.uniform(-3, 30, 12), rng.uniform(2, 7, 12)]))
        d = W.Domain(40, 30, 27, spheres=S, bc="bouzidi")
    elif which == "periodic":
        rng = np.random.default_rng(10)
        S = W.quantise(np.column_stack([rng.uniform(0, 33, 10), rng.uniform(0, 21, 10),
                                        rng.uniform(0, 25, 10), rng.uniform(1.5, 9.5, 10)]))
        d = W.Domain(33, 21, 25, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), spheres=S)
    elif which == "c1":
        d, _, _ = W.coupled_c1()
    else:
        d, _, _, _ = W.rev_sample_c3(2)
    g = lbm.Geometry(d)
    fo = oracle.flags(d)
    co, ko, qo, so = oracle.links(d, fo)
    assert np.array_equal(g.flags(), fo)
    c, k, q = g.links()
    assert np.array_equal(c, co)
    assert np.array_equal(k, ko)
    assert np.array_equal(q.view(np.uint64), qo.view(np.uint64))
    nd, nf, nl = g.info()
    assert nf == int((fo == 0).sum()) and nl == len(co)


def _status(fn):
    from paper_1507_06565_amd import _lib
    try:
        fn()
    except _lib.LbmError as e:
        return e.status
    return 0


def test_invalid_inputs_are_rejected():
    from paper_1507_06565_amd import lbm
    E_INVAL = -1
    # non-periodic axis without walls
    assert _status(lambda: lbm.Geometry(W.Domain(8, 8, 8, periodic=(1, 1, 0), wall_lo=(0, 0, 0),
                                                  wall_hi=(0, 0, 0)))) == E_INVAL
    # non-dyadic sphere
    assert _status(lambda: lbm.Geometry(W.Domain(16, 16, 16, spheres=np.array([[4.1, 4, 4, 2.0]])))) == E_INVAL
    # centre outside a periodic axis
    assert _status(lambda: lbm.Geometry(W.Domain(16, 16, 16, spheres=np.array([[17.0, 4, 4, 2.0]])))) == E_INVAL
    g = lbm.Geometry(W.Domain(16, 16, 16))
    # tau+ <= 1/2 and omega- outside (0, 2)
    assert _status(lambda: lbm.required_bytes(g, W.Params(tau_plus=0.5))) == E_INVAL
    assert _status(lambda: lbm.required_bytes(g, W.Params(tau_plus=0.8, magic_lambda=-0.1))) == E_INVAL
    assert lbm.required_bytes(g, W.Params(tau_plus=0.8)) > 19 * 4 * 16 ** 3


def test_domain_size_limits():
    """A domain above 2^30 cells (32-bit byte offsets of the sweep) is
    rejected before anything is allocated; so is a walled axis of fewer
    than 3 cells."""
    from paper_1507_06565_amd import lbm
    E_INVAL = -1
    assert _status(lambda: lbm.Geometry(W.Domain(1024, 1024, 1025))) == E_INVAL
    assert _status(lambda: lbm.Geometry(W.Domain(16, 16, 2))) == E_INVAL
    g = lbm.Geometry(W.Domain(1024, 1024, 1024, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0)))
    assert g.info()[1] == 1 << 30


def test_required_bytes_layouts():
    from paper_1507_06565_amd import lbm
    g = lbm.Geometry(W.Domain(64, 32, 40))
    two = lbm.required_bytes(g, W.Params(layout="twogrid"))
    aa = lbm.required_bytes(g, W.Params(layout="aa"))
    nl = g.info()[2]
    # the AA layout drops one population grid and adds one float per link
    assert two - aa >= 19 * 4 * 64 * 32 * 40 - 4 * nl - 4096


def test_brick_layout_plan():
    """The brick layout stores only 4x4x4 bricks that hold fluid (two grids of
    them), and rejects sizes not divisible by 4."""
    import numpy as np

    import oracle
    from paper_1507_06565_amd import lbm
    E_INVAL = -1
    S = np.array([[16.0, 16.0, 16.0, 11.0], [40.0, 20.0, 30.0, 9.0]])
    d = W.Domain(48, 32, 40, spheres=S)
    g = lbm.Geometry(d)
    two = lbm.required_bytes(g, W.Params(layout="twogrid"))
    brick = lbm.required_bytes(g, W.Params(layout="brick"))
    f = oracle.flags(d) == 0
    stored = int(f.reshape(10, 4, 8, 4, 12, 4).any(axis=(1, 3, 5)).sum())
    assert stored < 12 * 8 * 10
    dropped = (12 * 8 * 10 - stored) * 64
    # two grids of 19 arrays lose the dropped cells; 27 neighbours per stored
    # brick and one map entry per brick are added
    assert two - brick >= 2 * 19 * 4 * dropped - 27 * 4 * stored - 4 * 12 * 8 * 10 - 8192
    assert two - brick <= 2 * 19 * 4 * dropped + 8192
    for shape in ((30, 32, 40), (48, 34, 40), (48, 32, 42)):
        gb = lbm.Geometry(W.Domain(*shape))
        assert _status(lambda: lbm.required_bytes(gb, W.Params(layout="brick"))) == E_INVAL
        assert lbm.required_bytes(gb, W.Params(layout="twogrid")) > 0
    # batches: every domain's bricks in one array (two grids), each domain's range
    # padded to a multiple of 8 bricks; a domain not divisible by 4 is rejected
    per = lambda dd: W.Domain(dd, dd, dd, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0))
    gbatch = lbm.Geometry([per(16), per(12), per(20)])
    nb = sum(-(-(e // 4) ** 3 // 8) * 8 for e in (16, 12, 20))  # all fluid: every brick stored, padded
    assert lbm.required_bytes(gbatch, W.Params(layout="brick", force=(1e-5, 0, 0))) >= 2 * 19 * 4 * 64 * nb
    gbad = lbm.Geometry([per(16), per(18)])
    assert _status(lambda: lbm.required_bytes(gbad, W.Params(layout="brick", force=(1e-5, 0, 0)))) == E_INVAL
    assert lbm.required_bytes(gbad, W.Params(layout="aa", force=(1e-5, 0, 0))) > 0


def test_closure_and_gray_argument_validation():
    """Size and pointer checks of the gray and network entry points, which
    return before any device work."""
    from paper_1507_06565_amd._lib import lib
    E_INVAL = -1
    n = C.c_int64(0)
    assert lib.gray_required_bytes(1, 705, C.byref(n)) == E_INVAL
    assert lib.gray_required_bytes(1, 2, C.byref(n)) == E_INVAL
    assert lib.gray_required_bytes(0, 64, C.byref(n)) == E_INVAL
    assert lib.gray_required_bytes(3, 512, C.byref(n)) == 0 and n.value >= 3 * 19 * 512 * 4
    assert lib.mlp_workspace_bytes(100, C.byref(n)) == E_INVAL
    assert lib.mlp_workspace_bytes(0, C.byref(n)) == E_INVAL
    assert lib.mlp_workspace_bytes(128, C.byref(n)) == 0 and n.value > 0
    # null pointers and sizes out of range are rejected up front
    assert lib.mlp_profile_loss(None, None, None, 1, 64, 0.1, 1e-6, 1.0, None, None, None) == E_INVAL
    assert lib.mlp_closure(None, None, 10, 0.1, None, None, None) == E_INVAL


def test_link_count_limit(monkeypatch):
    """Link records and partial values are addressed by 32-bit byte offsets:
    a domain or a brick-layout batch with more links than the limit is
    refused with LBM_E_INVAL (the limit is lowered through the environment so
    that a small geometry can cross it)."""
    from paper_1507_06565_amd import lbm
    d, _, _ = W.coupled_c1()
    g = lbm.Geometry(d)
    nl = g.info()[2]
    for layout in ("twogrid", "aa", "brick"):
        p = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3 / 16, layout=layout)
        monkeypatch.setenv("MI355LBM_MAX_LINKS", str(nl))
        assert lbm.required_bytes(g, p) > 0
        monkeypatch.setenv("MI355LBM_MAX_LINKS", str(nl - 1))
        with pytest.raises(lbm.LbmError, match="too many boundary links"):
            lbm.required_bytes(g, p)
    cubes = [W.rev_sample_c3(i)[0] for i in (0, 1)]
    gb = lbm.Geometry(cubes)
    nlb = sum(gb.info(i)[2] for i in range(2))
    p = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3 / 16, layout="brick")
    monkeypatch.setenv("MI355LBM_MAX_LINKS", str(nlb))
    assert lbm.required_bytes(gb, p) > 0
    monkeypatch.setenv("MI355LBM_MAX_LINKS", str(nlb - 1))
    with pytest.raises(lbm.LbmError, match="too many boundary links"):
        lbm.required_bytes(gb, p)


def test_tuning_cache_round_trip():
    """lbm_tuning_export / lbm_tuning_import carry every autotuner's cached
    choices to another process as text: entries of all four kinds come back
    out exactly; a malformed or unknown line fails the whole import, names
    the line, and changes nothing."""
    from paper_1507_06565_amd import lbm
    entries = [
        "sweep test-arch-a 512 256 1024 2 1 1024 2",
        "sweep test-arch-a 128 64 256 1 2 256 1",
        "layout test-arch-a 1 128 64 256 1 1 2097152 1 0.0562",
        "brick-batch test-arch-a 512 2437120 512 1 1",
        "aa-batch test-arch-a 48 8093696 512 4",
    ]
    lbm.tuning_import("# saved\n" + "\n".join(entries) + "\n")
    out = lbm.tuning_export()
    lines = set(out.splitlines())
    for e in entries:
        assert e in lines, e
    lbm.tuning_import(out)  # its own export imports cleanly and changes nothing
    assert lbm.tuning_export() == out
    for bad, why in [("sweep test-arch-b 64 64 64 2 1 100 0", "malformed"),      # block 100
                     ("sweep test-arch-b 64 64 64 0 1 256 4", "malformed"),      # cells per thread on a dense layout
                     ("brick-batch test-arch-b 1 10 256 0 3", "malformed"),      # 3 cells per thread
                     ("layout test-arch-b 1 8 8 8 1 1 512 2", "malformed"),      # missing time
                     ("autotune test-arch-b 1 2 3", "unknown")]:
        text = "sweep test-arch-b 32 32 32 0 0 128 0\n" + bad + "\n"
        with pytest.raises(lbm.LbmError, match=f"line 2: {why}"):
            lbm.tuning_import(text)
        assert "test-arch-b" not in lbm.tuning_export()
