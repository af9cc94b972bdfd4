"""Two-domain interface evaluation (host FP64): the fits recover the slip and
jump coefficients of profiles built from the sharp-interface conditions
themselves, and the analytic two-domain profiles satisfy their equations."""
import math

import numpy as np

from paper_1507_06565_amd import interface as I

NU, G = 1.0 / 6.0, 1e-6


def synthetic(alpha, beta, zi=120.5, nz=256, K=2.0, eps_b=0.5, J=2.0, b=1.0):
    """Free side: the BJ parabola; porous side: Um + A exp(b (z - zi)) with A
    fixed by continuity and b chosen; beta follows from the slopes."""
    Um = K * G / NU
    top = nz - 1.5
    f = I.stokes_bj(zi, top, G, NU, K, Um, alpha)
    z = np.arange(nz, dtype=np.float64)
    Us = f(0.0)
    A = Us - Um
    u = np.where(z >= zi, f(z - zi), Um + A * np.exp(b * (z - zi)))
    u[0] = u[-1] = 0.0
    eps = np.where(z < zi, eps_b, 1.0)
    eps[0] = eps[-1] = 0.0
    return u, eps, Um, Us


def test_fits_recover_beavers_joseph_alpha():
    for alpha in (0.1, 0.5, 2.0):
        u, eps, Um, Us = synthetic(alpha, 0.0)
        f = I.fit_interface(u, eps, 120.5, 128, NU, G)
        assert abs(f.K / 2.0 - 1) < 1e-9 and abs(f.Um / Um - 1) < 1e-9
        assert abs(f.Us / Us - 1) < 1e-9
        assert abs(f.alpha / alpha - 1) < 1e-7, (alpha, f.alpha)
        assert f.rms_free < 1e-12 and f.rms_porous < 1e-8
        # beta from the definition with the fitted slopes
        beta = math.sqrt(f.K) / (NU * f.Us) * (f.J * NU * f.dU_minus - NU * f.dU_plus)
        assert abs(f.beta - beta) <= 1e-12 * abs(beta)


def test_porosity_limit_position():
    eps = np.ones(40)
    eps[0] = eps[-1] = 0.0
    eps[1:20] = 0.5
    eps[20] = 0.97
    assert I.porosity_limit(eps, 39) == 20.5


def test_two_domain_brinkman_solution_satisfies_its_equations():
    zi, top, bottom, K, eps, J = 100.5, 198.5, 0.5, 1.5, 0.45, 2.2
    for beta in (0.0, -1.3, 0.7):
        U = I.stokes_brinkman(zi, top, bottom, G, NU, K, eps, J, beta)
        h = 1e-2
        # free side: nu U'' + G = 0; porous side: J nu U'' - eps nu / K U + eps G = 0
        for z in (130.0, 180.0):
            hf = 0.05  # the free-side profile is quadratic: second differences are exact
            d2 = (U(z + hf) - 2 * U(z) + U(z - hf)) / hf ** 2
            assert abs(NU * d2 + G) < 1e-6 * G
        for z in (30.0, 95.0):
            hp = 2e-3
            d2 = (U(z + hp) - 2 * U(z) + U(z - hp)) / hp ** 2
            assert abs(J * NU * d2 - eps * NU / K * U(z) + eps * G) < 1e-5 * eps * G
        assert abs(U(top)) < 1e-15 and abs(U(bottom)) < 1e-15
        # continuity and the stress jump at the interface
        # one-sided second-order slopes on each side of the interface
        up = (-3 * U(zi) + 4 * U(zi + h) - U(zi + 2 * h)) / (2 * h)
        um = (3 * U(zi - 1e-13) - 4 * U(zi - h) + U(zi - 2 * h)) / (2 * h)
        assert abs(U(zi + 1e-12) - U(zi - 1e-12)) < 1e-12
        jump = J * NU * um - NU * up
        assert abs(jump - NU * beta / math.sqrt(K) * U(zi)) < 1e-4 * NU * abs(up) + 1e-12


def test_brinkman_far_field_is_darcy():
    U = I.stokes_brinkman(150.5, 254.5, 0.5, G, NU, 2.0, 0.5, 2.0, 0.0)
    assert abs(U(60.0) / (2.0 * G / NU) - 1) < 1e-9


def test_saffman_profile_is_beavers_joseph_without_seepage():
    """eq. (BJS): sqrt(K)/alpha U'(zi+) = U_s, i.e. BJ with U_m = 0."""
    zi, top, K, alpha = 120.5, 254.5, 1.7, 0.4
    f = I.stokes_bjs(zi, top, G, NU, K, alpha)
    g = I.stokes_bj(zi, top, G, NU, K, 0.0, alpha)
    s = np.linspace(0.0, top - zi, 101)
    assert np.array_equal(f(s), g(s))
    h = 1e-3  # the profile is quadratic: the centred difference of f at h is exact up to rounding
    slope = (-3 * f(0.0) + 4 * f(h) - f(2 * h)) / (2 * h)
    assert abs(math.sqrt(K) / alpha * slope - f(0.0)) < 1e-9 * f(0.0)
    assert abs(f(top - zi)) < 1e-15


def test_sensitivity_reproduces_the_parameter_study():
    """Sec. 3.2's observations on the analytic two-domain profiles: raising the
    viscosity ratio J of Br lowers the maximum velocity and makes the shear
    rate jump by 1/J across the interface; negative OTW jump coefficients
    change the profile little, positive ones strongly; BJ and BJS are nearly
    the same at low Re; the maximum falls as alpha grows and a small alpha
    gives a much larger maximum.  Also: the profile-misfit search returns the
    alpha a BJ profile was built with."""
    u, eps, Um, Us = synthetic(0.5, 0.0)
    r = I.sensitivity(u, eps, 120.5, 128, NU, G)
    br = r["Br"]
    assert [e["J"] for e in br] == sorted(e["J"] for e in br)
    mx = [e["u_max"] for e in br]
    assert all(a > b for a, b in zip(mx, mx[1:])), mx
    for e in br:
        assert abs(e["slope_ratio"] * e["J"] - 1) < 1e-4, e
    otw = {e["beta"]: e["u_max"] for e in r["OTW"]}
    neg = abs(otw[-4.0] - otw[0.0])
    pos = abs(otw[0.5] - otw[0.0])
    assert pos > 0.8 * neg and pos / 0.5 > 4 * neg / 4.0, (neg, pos)
    # near the pole the profile grows without bound
    bs = r["otw_pole_beta"]
    assert 0 < bs < 5
    U = I.stokes_brinkman(120.5, 254.5, 0.5, G, NU, r["K"], r["eps_bed"], 1 / r["eps_bed"], bs * (1 - 1e-6))
    assert abs(U(200.0)) > 1e3 * r["umax"]
    bj = [e["u_max"] for e in r["BJ"]]
    bjs = [e["u_max"] for e in r["BJS"]]
    assert all(a > b for a, b in zip(bj, bj[1:])), bj
    assert bj[0] > 1.5 * bj[-1]
    assert max(abs(a / b - 1) for a, b in zip(bj, bjs)) < 1e-3
    assert abs(r["best"]["BJ"]["alpha"] / 0.5 - 1) < 1e-6
    assert r["best"]["Br"]["err"] <= min(e["err"] for e in br) + 1e-12
