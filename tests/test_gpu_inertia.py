"""Inertial regime (Sec. 3.1, Reynolds-number effect; eq. (PorousForce),
Forchheimer term) on the GPU: the scaled-down closure experiment trained at
tau+ = 0.56 in the Stokes regime, then one held-out bed (porosity 0.65) run to
steady state at Re_D = 0.5 and 30 (force raised at fixed viscosity), each
compared with the gray column under the learned closure with and without the
Forchheimer term."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(600)
def test_reynolds_sweep_and_forchheimer_closure():
    from paper_1507_06565_amd import closure as CL
    from paper_1507_06565_amd import inertia as IN

    s = CL.small_setup()
    nu0 = s.nu
    s.tau = 0.56
    s.force = s.force * (s.nu / nu0) ** 2
    res = CL.experiment(s)
    for r in res["held_out"]:
        say(f"held-out eps {r['porosity']}: learned {r['learned_err']:.4f}")
        assert r["learned_err"] <= 0.02
    lo, hi = IN.reynolds_sweep(s, res["params"], [(0.65, 32)], re_targets=(0.5, 30.0), tau=0.56)
    for r in (lo, hi):
        say(f"Re_D {r['Re_D']:.2f}: gray {r['err_gray']:.4f}, Forchheimer {r['err_forchheimer']:.4f}, "
            f"surface/max pore {r['shape_pore'][1]:.4f} gray {r['shape_gray'][1]:.4f} "
            f"Forchheimer {r['shape_forchheimer'][1]:.4f}")
    assert 0.4 < lo["Re_D"] < 0.7 and 25.0 < hi["Re_D"] < 35.0
    # slow flow: the Forchheimer term changes nothing
    assert lo["gray_forchheimer_diff"] < 1e-3
    assert lo["err_gray"] <= 0.02
    # faster flow penetrates the bed less relative to the channel maximum
    # (Sec. 3.1); the Stokes gray model is linear and cannot follow, the
    # Forchheimer drag does
    assert hi["shape_pore"][1] < 0.98 * lo["shape_pore"][1]
    assert abs(hi["shape_gray"][1] / lo["shape_gray"][1] - 1.0) < 2e-3
    assert hi["shape_forchheimer"][1] < 0.98 * lo["shape_forchheimer"][1]
    assert hi["err_forchheimer"] < hi["err_gray"]
    u = np.asarray(hi["u_pore"])
    assert np.all(u[1:-1] > 0)
