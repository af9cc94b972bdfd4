"""Pins of the FP64 reference of the closure's training signal: the steady
1-D Brinkman column against closed forms and against the gray lattice
Boltzmann column itself, and its adjoint gradient against central
differences."""
import numpy as np

import oracle
from oracle import closure as CL


def test_channel_parabola_exact():
    """Free fluid between half-way walls: the plane Poiseuille parabola with
    zero velocity on the wall planes, exactly (the wall closure is exact for
    quadratics)."""
    nz, nu, G = 40, 1.0 / 6.0, 1e-6
    U = CL.steady_profile(np.ones(nz), np.full(nz, nu), np.zeros(nz), G)
    s = np.arange(nz) - 0.5
    H = nz - 2
    ref = G / (2 * nu) * s * (H - s)
    assert np.max(np.abs(U[1:-1] - ref[1:-1])) <= 1e-12 * ref.max()
    assert U[0] == 0 and U[-1] == 0


def test_darcy_limit():
    """Uniform porous column far from the walls: drag balances the force,
    U = eps G / drag (the Darcy velocity K G / nu for drag = eps nu / K)."""
    nz, nu, G, eps, K = 200, 1.0 / 6.0, 1e-6, 0.4, 0.5
    drag = eps * nu / K
    U = CL.steady_profile(np.full(nz, eps), np.full(nz, nu / eps), np.full(nz, drag), G)
    assert abs(U[nz // 2] / (K * G / nu) - 1) <= 1e-10


def test_brinkman_half_space_decay():
    """Free channel over a uniform porous layer: inside the layer the excess
    over the Darcy velocity decays geometrically with the rate of the
    three-point recurrence, acosh(1 + drag / (2 nu_eff)) per cell, which tends
    to the continuum Brinkman rate sqrt(drag / nu_eff)."""
    nz, nu, G = 400, 1.0 / 6.0, 1e-6
    eps = np.ones(nz)
    eps[:200] = 0.5
    nue = np.where(eps < 1, 0.3, nu)
    drag = np.where(eps < 1, 0.01, 0.0)
    U = CL.steady_profile(eps, nue, drag, G)
    ud = 0.5 * G / 0.01
    z = np.arange(150, 190)
    ex = U[z] - ud
    rate = np.polyfit(z, np.log(ex), 1)[0]
    assert abs(rate - np.arccosh(1 + 0.01 / 0.6)) <= 1e-9
    assert abs(rate - np.sqrt(0.01 / 0.3)) <= 2e-3 * np.sqrt(0.01 / 0.3)


def test_matches_gray_lattice_steady_state():
    """The surrogate is the steady state of the gray column to second order:
    on a smoothed-step porosity with matching closure it agrees with the
    lattice scheme run to steady state within 1e-3."""
    nz, nu, G = 96, 1.0 / 6.0, 1e-6
    z = np.arange(nz)
    s = np.clip((z - 48 + 6) / 12.0, 0, 1)
    S = 3 * s * s - 2 * s ** 3
    eps = 0.5 + 0.5 * S
    eps[0] = eps[-1] = 1.0
    nue = nu / eps
    drag = (1 - S) * eps * nu / 1.5
    U = CL.steady_profile(eps, nue, drag, G)
    u, _ = oracle.gray_to_steady(nz, eps, nue, drag, G=(G, 0, 0), rel_tol=1e-13, check=2000)
    e = np.linalg.norm(U - u[:, 0]) / np.linalg.norm(u[:, 0])
    assert e <= 1e-3, e


def test_gradient_against_central_differences():
    rng = np.random.default_rng(7)
    nprof, nz, nu, G = 2, 12, 1.0 / 6.0, 1e-6
    eps = rng.uniform(0.4, 1.0, nprof * nz)
    eps[::nz] = 0.0
    eps[nz - 1::nz] = 0.0
    Y = rng.normal(0, 0.5, (nprof * nz, 16))
    ut = rng.uniform(0.0, 1e-4, nprof * nz)
    L, dY = CL.profile_loss(Y, eps, ut, nprof, nz, nu, G, 0.7)
    h = 1e-6
    for r in range(nprof * nz):
        for c in (0, 1, 5):
            E = np.zeros_like(Y)
            E[r, c] = h
            fd = (CL.profile_loss(Y + E, eps, ut, nprof, nz, nu, G, 0.7)[0].sum()
                  - CL.profile_loss(Y - E, eps, ut, nprof, nz, nu, G, 0.7)[0].sum()) / (2 * h)
            assert abs(fd - dY[r, c]) <= 1e-6 * abs(fd) + 1e-7 * np.abs(dY).max(), (r, c, fd, dY[r, c])
