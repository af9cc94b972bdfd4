"""Deposited packings (Sec. 3.1: spheres of diameters 50-150 % of the mean,
dropped one after another until they rest): the generator's output is
deterministic, non-overlapping, and mechanically settled (no sphere can be
lowered without overlapping another or the floor), with the solid fraction of
random sequential deposition; scaled to a lattice it is exactly
non-overlapping and inside the domain."""
import numpy as np
import pytest

from paper_1507_06565_amd import deposition as Dp
from paper_1507_06565_amd import workloads as W

LX, LY = 4.0, 4.0


@pytest.fixture(scope="module")
def packing():
    return Dp.deposit(5, LX, LY, 48)


def _pair_gaps(S, L):
    g = []
    for i in range(len(S)):
        d = S[i + 1:, :3] - S[i, :3]
        d[:, :2] -= L * np.round(d[:, :2] / L)
        s = S[i + 1:, 3] + S[i, 3]
        g.append((np.sqrt((d * d).sum(1)) - s) / s)
    return np.concatenate(g)


def test_deterministic(packing):
    assert np.array_equal(Dp.deposit(5, LX, LY, 48), packing)
    assert not np.array_equal(Dp.deposit(6, LX, LY, 48), packing)


def test_diameters_and_box(packing):
    d = 2 * packing[:, 3]
    assert d.min() >= 0.5 and d.max() <= 1.5
    assert np.all((packing[:, 0] >= 0) & (packing[:, 0] < LX) & (packing[:, 1] >= 0) & (packing[:, 1] < LY))
    assert np.all(packing[:, 2] - packing[:, 3] >= -1e-12)  # above the floor


def test_non_overlapping_with_periodic_images(packing):
    assert _pair_gaps(packing, np.array([LX, LY])).min() > -1e-12


def test_every_sphere_is_settled(packing):
    """Static equilibrium under gravity: with all of its contacts (spheres
    deposited before and after it, and the floor), no direction lowers a
    sphere's centre without moving into a contact; and each one rests on the
    floor or on at least one sphere."""
    L = np.array([LX, LY])
    assert Dp.supported(packing, LX, LY).all()
    for i, (x, y, z, r) in enumerate(packing):
        d = packing[:, :3] - np.array([x, y, z])
        d = -d
        d[:, :2] -= L * np.round(d[:, :2] / L)
        dist = np.sqrt((d * d).sum(1))
        touch = (dist <= (packing[:, 3] + r) * (1 + 1e-7)) & (np.arange(len(packing)) != i)
        N = d[touch] / dist[touch][:, None]
        if z <= r * (1 + 1e-7):
            N = np.vstack([N, [0.0, 0.0, 1.0]])
        assert len(N) > 0, i
        dv, _ = Dp._descent(N)
        assert np.linalg.norm(dv) < 1e-6, (i, dv)


def test_solid_fraction_of_random_deposition(packing):
    """Random sequential deposition packs to a solid fraction near 0.58;
    sampled over the bed interior (half a diameter above the floor up to
    two below the top) it lies between 0.5 and 0.66."""
    rng = np.random.default_rng(0)
    h = Dp.bed_height(packing)
    P = rng.uniform(0, 1, (100000, 3)) * [LX, LY, 1.0]
    P[:, 2] = 0.5 + P[:, 2] * (h - 2.5)
    inside = np.zeros(len(P), bool)
    for x, y, z, r in packing:
        d = P - [x, y, z]
        d[:, :2] -= np.array([LX, LY]) * np.round(d[:, :2] / np.array([LX, LY]))
        inside |= (d * d).sum(1) <= r * r
    assert 0.5 < inside.mean() < 0.66, inside.mean()


def test_narrow_box_is_refused():
    with pytest.raises(ValueError):
        Dp.deposit(1, 2.0, 4.0, 10)


@pytest.mark.parametrize("D", [4, 12, 48])
def test_lattice_packing_exact(packing, D):
    """Scaled to D cells per mean diameter and quantised: dyadic, exactly
    non-overlapping with periodic images, centres inside the periodic box,
    resting on the bottom wall plane z = 0.5; the study domain's fluid height
    is the same whole number of mean diameters at every D."""
    S, nx, ny = Dp.lattice_packing(packing, D, LX, LY)
    assert (nx, ny) == (4 * D, 4 * D)
    assert np.array_equal(S, W.quantise(S))
    assert W.check_non_overlap(S, np.array([nx, ny, 1e9]), np.array([True, True, False]))
    assert np.all((S[:, 0] >= 0) & (S[:, 0] < nx) & (S[:, 1] >= 0) & (S[:, 1] < ny))
    assert np.all(S[:, 2] - S[:, 3] >= 0.5 - 2.0 ** -11)
    d = Dp.study_domain(packing, D, LX, LY, 3.0)
    T = Dp.channel_height(packing, 3.0)
    assert d.nz == T * D + 2 and T >= Dp.bed_height(packing) + 3.0


def test_normalised_profile():
    u = np.zeros(12)
    H = 10.0
    zc = (np.arange(1, 11) - 0.5) / H
    u[1:11] = zc * (1 - zc)
    s, un = Dp.normalised_profile(u, 101)
    assert un.max() <= 1.0 + 1e-15 and abs(un.max() - 1.0) < 1e-15
    assert un[0] == 0.0 and un[-1] == 0.0
    ref = s * (1 - s) / (zc * (1 - zc)).max()
    assert np.max(np.abs(un - ref)) < 0.02
