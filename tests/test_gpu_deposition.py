"""Grid study on a deposited packing (Sec. 3.1) through the C ABI: the same
unit packing at D = 4, 8 and 16 cells per mean diameter, driven to
Re_D = U_max D / nu = 2 and run to steady state; the plane-averaged profile
normalised by its maximum and the channel height converges with D."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(300)
def test_grid_study_converges():
    from paper_1507_06565_amd import deposition as Dp

    out = Dp.grid_study(Ds=(4, 8, 16), seed=11, n=64, log=say)
    runs = out["runs"]
    for r in runs:
        say(f"D {r['D']}: Re_D {r['Re_D']:.3f}, {r['steps']} steps, vs D=16 {r['diff_finest']:.4%}")
        assert abs(r["Re_D"] / 2.0 - 1.0) <= 0.1
        assert r["nz"] == Dp.channel_height(out["unit_packing"], 3.0) * r["D"] + 2
        u = np.asarray(r["u"])
        assert u[0] == 0.0 and u[-1] == 0.0 and np.all(u[1:-1] > 0)
        # the maximum lies in the free channel above the bed
        assert np.argmax(u) > out["bed_height"] * r["D"]
    d4, d8 = runs[0]["diff_finest"], runs[1]["diff_finest"]
    # the coarsest grid is the furthest from the finest, the error shrinks
    # faster than linearly with D, and D = 8 is within one per cent
    assert d4 > 2.5 * d8 and d8 < 0.01
