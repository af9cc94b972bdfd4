"""Host tests of the seeded sphere-packing generator (the stand-in for the
rigid-body deposition of Sec. 3.1): determinism, exact non-overlap with
periodic images, porosity within the workload's tolerance (measured on the
oracle's own voxelisation), the radius range and distribution, and a loud
failure when no packing meets the tolerance."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1507_06565_amd import workloads as W


def _bed_porosity_by_oracle(dom, bed_top):
    fl = oracle.flags(dom)
    return float((fl[1:bed_top] == oracle.FLUID).mean())


def _check_radii(S, r_range):
    r = S[:, 3]
    a, b = r_range
    assert r.min() >= W.R_SHRINK_MIN * a and r.max() <= b
    # drawn uniform in [a, b]; the jam shrink moves radii by a few percent at most
    D = stats.kstest((r - a) / (b - a), "uniform").statistic
    assert D <= 1.63 / math.sqrt(len(r)) + 0.03, D


def _check_bed_heights(S, bed_top, r_range):
    rbar = 0.5 * sum(r_range)
    assert np.all(S[:, 2] + S[:, 3] <= bed_top)
    assert np.all(S[:, 2] - S[:, 3] >= 0.5 - 2 * rbar)


@pytest.fixture(scope="module")
def c1():
    return W.coupled_c1()


def test_c1_bed(c1):
    d, _, eps = c1
    assert abs(eps - 0.6) <= 0.01
    assert _bed_porosity_by_oracle(d, 128) == pytest.approx(eps, abs=1e-15)
    assert W.check_non_overlap(d.spheres, (d.nx, d.ny, 128), (1, 1, 0))
    _check_radii(d.spheres, (6.0, 10.0))
    _check_bed_heights(d.spheres, 128, (6.0, 10.0))
    # dyadic: every value a multiple of 2^-12
    assert np.array_equal(W.quantise(d.spheres), d.spheres)
    assert np.all((d.spheres[:, 0] >= 0) & (d.spheres[:, 0] < d.nx))
    assert np.all((d.spheres[:, 1] >= 0) & (d.spheres[:, 1] < d.ny))


def test_c1_deterministic(c1):
    d, _, eps = c1
    d2, _, eps2 = W.coupled_c1()
    assert np.array_equal(d.spheres, d2.spheres) and eps == eps2
    d3, _, _ = W.coupled_c1(seed=7)
    assert not np.array_equal(d.spheres[:5], d3.spheres[:5])


def test_c2_bed():
    """512 x 256 x 1024 bed of radii U[8,16] at porosity 0.45 +- 0.01."""
    d, _, eps = W.large_c2()
    assert abs(eps - 0.45) <= 0.01
    assert len(d.spheres) > 4000
    assert W.check_non_overlap(d.spheres, (d.nx, d.ny, 512), (1, 1, 0))
    _check_radii(d.spheres, (8.0, 16.0))
    _check_bed_heights(d.spheres, 512, (8.0, 16.0))


@pytest.mark.parametrize("i", [0, 35, 60, 79, 128, 200, 287, 300, 437, 511])
def test_c3_cube(i):
    """Sampled REV cubes (including ones that need reseeding): porosity within
    0.02 of the cube's target (checked on the oracle's voxelisation), exact
    non-overlap across the periodic images, radii in range, deterministic."""
    d, _, target, eps = W.rev_sample_c3(i)
    assert d.nx in (32, 48, 64, 96) and d.nx == d.ny == d.nz
    assert 0.35 <= target <= 0.9
    assert abs(eps - target) <= 0.02
    fl = oracle.flags(d)
    assert float((fl == oracle.FLUID).mean()) == pytest.approx(eps, abs=1e-15)
    assert W.check_non_overlap(d.spheres, (d.nx,) * 3, (1, 1, 1))
    r = d.spheres[:, 3]
    assert r.min() >= W.R_SHRINK_MIN * 3.0 and r.max() <= 10.0
    assert np.all((d.spheres[:, :3] >= 0) & (d.spheres[:, :3] < d.nx))
    d2, _, _, eps2 = W.rev_sample_c3(i)
    assert np.array_equal(d.spheres, d2.spheres) and eps == eps2


def test_c3_radius_distribution():
    rs = [W.rev_sample_c3(i)[0].spheres for i in range(0, 512, 16)]
    _check_radii(np.concatenate(rs), (3.0, 10.0))


def test_check_non_overlap_sees_periodic_images():
    """Two spheres that only touch across the periodic boundary."""
    S = np.array([[0.5, 5.0, 5.0, 2.0], [18.0, 5.0, 5.0, 2.0]])
    assert not W.check_non_overlap(S, (20, 20, 20), (1, 1, 1))
    assert W.check_non_overlap(S, (20, 20, 20), (0, 1, 1))
    T = np.array([[0.5, 5.0, 5.0, 2.0], [16.5, 5.0, 5.0, 2.0]])  # exactly touching: allowed
    assert W.check_non_overlap(T, (20, 20, 20), (1, 1, 1))


def test_impossible_target_raises():
    """A porosity below random close packing cannot be reached."""
    with pytest.raises(W.PackingError):
        W.rev_cube(5, 16, (3.0, 4.0), 0.05, max_tries=2, reseeds=1)
    with pytest.raises(W.PackingError):
        W.porous_bed(5, 16, 16, 32, 16, (3.0, 4.0), 0.05, max_tries=2, reseeds=1)
