"""Two-domain (sharp-interface) evaluation of a steady coupled-flow profile.

Sec. 3.2 of the paper takes the plane-averaged velocity of a pore-scale run of
a free channel over a porous bed and asks which sharp-interface conditions,
with which parameters, reproduce it:

  (BJ)   dU/dz(0+) = alpha / sqrt(K) (U_s - U_m)                 Beavers-Joseph
  (BJS)  sqrt(K) / alpha dU/dz(0+) = U_s  (+ O(K), U_m dropped)    Saffman
  (OTW)  nu_eff dU/dz(0-) - nu dU/dz(0+) = nu beta / sqrt(K) U_s   Ochoa-Tapia & Whitaker
  (Br)   Brinkman in the porous layer, continuous velocity and stress

with U_s the velocity at the interface, U_m the Darcy (seepage) velocity far
inside the bed and K the permeability from eq. (Darcy).  As in the paper, the
free-side profile near the interface is fitted by a second-order polynomial
and the porous side by an exponential; the interface is placed either where
the planar porosity reaches one or at the highest plane down to which the
exponential still fits.  This module is host-side FP64 post-processing of a
profile the GPU produced (lbm_average_profile); the parameters follow from
the fits and the definitions above, and the analytic two-domain profiles of
each condition are compared with the pore-scale one.

Geometry convention: cells z = 0 .. nz-1, wall layers at 0 and nz-1, so the
top wall plane is at nz - 1.5; the interface position zi is a real number
(a plane between or through cells).
"""
from __future__ import annotations

import json
import math
import sys
from dataclasses import dataclass

import numpy as np


@dataclass
class Fit:
    zi: float          # interface position
    K: float           # far-field permeability
    Um: float          # Darcy velocity far inside the bed
    Us: float          # interface velocity (free-side polynomial at zi)
    dU_plus: float     # free-side slope at zi
    dU_minus: float    # porous-side slope at zi (exponential fit)
    decay: float       # exponential rate of the porous-side fit
    alpha: float       # Beavers-Joseph / Saffman slip coefficient
    beta: float        # Ochoa-Tapia-Whitaker jump coefficient (nu_eff = nu / eps_bed)
    J: float           # nu_eff / nu used for beta
    poly: tuple        # (c0, c1, c2) of the free-side fit in (z - zi)
    rms_free: float    # fit residuals (relative to max U)
    rms_porous: float


def porosity_limit(eps, top):
    """Lowest plane boundary above which the planar porosity is one up to the
    top wall layer `top` (exclusive)."""
    z = top - 1
    while z > 0 and eps[z] >= 1.0:
        z -= 1
    return z + 0.5


def far_field(u, eps, bed_top, nu, G):
    """Darcy velocity and permeability (eq. (Darcy)) over the bed interior
    band [bed_top/4, 3 bed_top/4)."""
    z0, z1 = bed_top // 4, 3 * bed_top // 4
    Um = float(np.mean(u[z0:z1]))
    return Um, nu * Um / G


def exp_fit(z, y):
    """y = A exp(b z) by least squares on log y (y > 0)."""
    b, logA = np.polyfit(z, np.log(y), 1)
    return math.exp(logA), b


def fit_interface(u, eps, zi, bed_top, nu, G, free_cells=24, porous_cells=12, J=None):
    """Polynomial and exponential fits around the interface zi and the
    resulting slip (alpha) and jump (beta) coefficients."""
    nz = len(u)
    Um, K = far_field(u, eps, bed_top, nu, G)
    zc = np.arange(nz, dtype=np.float64)
    # free side: cells whose centre lies above zi, up to free_cells of them
    free = (zc > zi) & (zc <= zi + free_cells) & (zc < nz - 1)
    c2, c1, c0 = np.polyfit(zc[free] - zi, u[free], 2)
    Us = c0
    dplus = c1
    rfree = u[free] - (c0 + c1 * (zc[free] - zi) + c2 * (zc[free] - zi) ** 2)
    # porous side: excess over the Darcy velocity decays into the bed
    por = (zc < zi) & (zc >= zi - porous_cells) & (zc >= 1)
    ex = u[por] - Um
    ok = ex > 0
    A, b = exp_fit(zc[por][ok] - zi, ex[ok])
    dminus = A * b
    rpor = ex[ok] - A * np.exp(b * (zc[por][ok] - zi))
    umax = float(np.max(np.abs(u)))
    if J is None:
        eb = float(np.mean(eps[bed_top // 4:3 * bed_top // 4]))
        J = 1.0 / eb
    sk = math.sqrt(K)
    alpha = sk * dplus / (Us - Um)
    beta = sk / (nu * Us) * (J * nu * dminus - nu * dplus)
    return Fit(zi=zi, K=K, Um=Um, Us=Us, dU_plus=dplus, dU_minus=dminus, decay=b, alpha=alpha, beta=beta, J=J,
               poly=(c0, c1, c2), rms_free=float(np.sqrt(np.mean(rfree ** 2))) / umax,
               rms_porous=float(np.sqrt(np.mean(rpor ** 2))) / umax)


def apparent_interface(u, eps, bed_top, nu, G, tol=1e-3, porous_cells=12):
    """Highest cell boundary at or below the porosity limit down to which the
    porous-side exponential fits within tol (relative RMS, as the paper's
    criterion of a good exponential fit)."""
    z_lim = porosity_limit(eps, len(u) - 1)
    best = z_lim
    for k in range(0, 16):
        zi = z_lim - k
        f = fit_interface(u, eps, zi, bed_top, nu, G, porous_cells=porous_cells)
        if f.rms_porous <= tol:
            best = zi
            break
    return best


# ---------------------------------------------------------------- analytic --

def stokes_bj(zi, top, G, nu, K, Um, alpha):
    """Free region zi..top (no slip at top): nu U'' = -G with the BJ slip
    U'(zi) = alpha/sqrt(K) (U(zi) - Um); returns U(s), s = z - zi."""
    H = top - zi
    s_ = alpha / math.sqrt(K)
    # U = -G/(2 nu) s^2 + a s + c;  U(H) = 0;  a = s_ (c - Um)
    # -G H^2/(2nu) + s_ (c - Um) H + c = 0
    c = (G * H * H / (2 * nu) + s_ * Um * H) / (1 + s_ * H)
    a = s_ * (c - Um)
    return lambda s: -G / (2 * nu) * s * s + a * s + c


def stokes_bjs(zi, top, G, nu, K, alpha):
    """Saffman's form of the slip condition (eq. (BJS)), U_s = sqrt(K)/alpha
    U'(zi+): the seepage velocity is of order K and is absorbed by the O(k)
    term, so this is the BJ profile with U_m = 0.  Returns U(s), s = z - zi."""
    return stokes_bj(zi, top, G, nu, K, 0.0, alpha)


def _brinkman_system(zi, top, bottom, G, nu, K, eps, J, beta):
    H = top - zi
    d = bottom - zi  # negative
    r = math.sqrt(eps / (J * K))  # Brinkman rate: J nu U'' = eps nu/K U - eps G
    Ud = K * G / nu               # Darcy velocity
    # porous: U = Ud + P e^{r s} + M e^{-r s}, s = z - zi in [d, 0]; U(d) = 0
    # free:   U = -G/(2 nu) s^2 + a s + c, U(H) = 0
    # unknowns P, M, a, c: linear system
    Amat = np.array([
        [math.exp(r * d), math.exp(-r * d), 0.0, 0.0],              # U(d) = 0
        [0.0, 0.0, H, 1.0],                                          # U(H) = 0 (plus the -G/(2nu)H^2 term)
        [1.0, 1.0, 0.0, -1.0],                                       # continuity at s = 0
        [J * r, -J * r, -1.0, -beta / math.sqrt(K)],                 # stress jump at s = 0
    ])
    # continuity: Ud + P + M = c  ->  P + M - c = -Ud
    # jump: J (r P - r M) - a - beta/sqrt(K) c = 0
    rhs = np.array([-Ud, G * H * H / (2 * nu), -Ud, 0.0])
    return Amat, rhs, r, Ud


def otw_pole(zi, top, bottom, G, nu, K, eps, J):
    """The jump coefficient beta* > 0 at which the two-domain Stokes/Brinkman
    system with the OTW condition becomes singular: the determinant is linear
    in beta (beta enters one matrix entry), so beta* = det(0)/(det(0) - det(1)).
    Profiles with beta approaching beta* grow without bound."""
    d0 = np.linalg.det(_brinkman_system(zi, top, bottom, G, nu, K, eps, J, 0.0)[0])
    d1 = np.linalg.det(_brinkman_system(zi, top, bottom, G, nu, K, eps, J, 1.0)[0])
    return float(d0 / (d0 - d1))


def stokes_brinkman(zi, top, bottom, G, nu, K, eps, J, beta=0.0):
    """Stokes above zi (no slip at top), Brinkman below (nu_eff = J nu, drag
    eps nu / K, force eps G, no slip at bottom); continuous velocity and the
    stress jump nu_eff U'(zi-) - nu U'(zi+) = nu beta / sqrt(K) U(zi)
    (beta = 0: the Brinkman (Br) model with continuous stress).  Returns a
    function of z."""
    Amat, rhs, r, Ud = _brinkman_system(zi, top, bottom, G, nu, K, eps, J, beta)
    P, M, a, c = np.linalg.solve(Amat, rhs)

    def U(z):
        s = np.asarray(z, dtype=np.float64) - zi
        free = -G / (2 * nu) * s * s + a * s + c
        porous = Ud + P * np.exp(r * s) + M * np.exp(-r * s)
        return np.where(s >= 0, free, porous)
    return U


def _profile_stats(z, U, zi, umax_ref):
    """Maximum and interface velocity of a profile sampled on z, normalised by
    umax_ref (the maximum of the pore-scale profile, as in the paper's
    figures of the analytic parameter study)."""
    i = int(np.searchsorted(z, zi))
    return float(np.max(U) / umax_ref), float(U[i] / umax_ref)


def _rel_err(U, u, inner):
    return float(np.linalg.norm((U - u)[inner]) / np.linalg.norm(u[inner]))


def sensitivity(u, eps, zi, bed_top, nu, G, Js=(1.0, 2.0, 4.0, 8.0), betas=(-4.0, -2.0, -1.0, 0.0, 0.25, 0.5),
                alphas=(0.01, 0.1, 0.3, 1.0, 5.0)):
    """How the free parameter of each two-domain condition shapes its analytic
    profile (Sec. 3.2, the parameter study of the analytic solutions: Stokes
    above the interface zi, Brinkman below with nu_eff = J nu and the
    permeability K of the bed interior): for Br the viscosity ratio J (and
    J = 1/eps_bed), for OTW the jump coefficient beta at J = 1/eps_bed, for BJ
    and BJS the slip coefficient alpha.  Each entry gives the profile's
    maximum and interface velocity normalised by the pore-scale maximum, and
    its relative L2 difference from the pore-scale profile u; Br also gives the
    ratio of the porous-side to the free-side slope at zi (1/J: the stress is
    continuous, the shear rate jumps).  Also returned: the OTW pole beta*
    (profiles blow up as beta approaches it from below) and, per condition,
    the parameter that minimises the profile difference (bounded scalar
    search)."""
    from scipy.optimize import minimize_scalar

    nz = len(u)
    top, bottom = nz - 1.5, 0.5
    Um, K = far_field(u, eps, bed_top, nu, G)
    eb = float(np.mean(eps[bed_top // 4:3 * bed_top // 4]))
    umax = float(np.max(u))
    zc = np.arange(nz, dtype=np.float64)
    inner = slice(1, nz - 1)
    zf = np.linspace(bottom, top, 20001)
    zf = np.union1d(zf, [zi])
    out = {"zi": zi, "K": K, "Um": Um, "eps_bed": eb, "umax": umax, "Br": [], "OTW": [], "BJ": [], "BJS": []}

    def two_domain_bj(alpha, um):
        f = stokes_bj(zi, top, G, nu, K, um, alpha)
        return (lambda z: np.where(np.asarray(z) >= zi, f(np.asarray(z) - zi), Um))

    h = 1e-6
    for J in sorted(set(list(Js) + [1.0 / eb])):
        U = lambda z, J=J: stokes_brinkman(zi, top, bottom, G, nu, K, eb, J, 0.0)(z)
        mx, us = _profile_stats(zf, U(zf), zi, umax)
        up = (U(zi + h) - U(zi)) / h
        um = (U(zi) - U(zi - h)) / h
        out["Br"].append({"J": J, "u_max": mx, "u_s": us, "slope_ratio": float(um / up), "err": _rel_err(U(zc), u, inner)})
    beta_star = otw_pole(zi, top, bottom, G, nu, K, eb, 1.0 / eb)
    out["otw_pole_beta"] = beta_star
    for b in betas:
        if b >= beta_star:
            continue
        U = stokes_brinkman(zi, top, bottom, G, nu, K, eb, 1.0 / eb, b)
        mx, us = _profile_stats(zf, U(zf), zi, umax)
        out["OTW"].append({"beta": b, "u_max": mx, "u_s": us, "err": _rel_err(U(zc), u, inner)})
    for a in alphas:
        for name, um in (("BJ", Um), ("BJS", 0.0)):
            U = two_domain_bj(a, um)
            mx, us = _profile_stats(zf, U(zf), zi, umax)
            out[name].append({"alpha": a, "u_max": mx, "u_s": us, "err": _rel_err(U(zc), u, inner)})

    best = {}
    r = minimize_scalar(lambda J: _rel_err(stokes_brinkman(zi, top, bottom, G, nu, K, eb, J, 0.0)(zc), u, inner),
                        bounds=(0.05, 50.0), method="bounded", options={"xatol": 1e-6})
    best["Br"] = {"J": float(r.x), "err": float(r.fun)}
    r = minimize_scalar(lambda b: _rel_err(stokes_brinkman(zi, top, bottom, G, nu, K, eb, 1.0 / eb, b)(zc), u, inner),
                        bounds=(-50.0, beta_star - 1e-3 * abs(beta_star)), method="bounded", options={"xatol": 1e-6})
    best["OTW"] = {"beta": float(r.x), "err": float(r.fun)}
    for name, um in (("BJ", Um), ("BJS", 0.0)):
        r = minimize_scalar(lambda la: _rel_err(two_domain_bj(10.0 ** la, um)(zc), u, inner),
                            bounds=(-3.0, 3.0), method="bounded", options={"xatol": 1e-8})
        best[name] = {"alpha": float(10.0 ** r.x), "err": float(r.fun)}
    out["best"] = best
    return out


def evaluate(u, eps, bed_top, nu, G):
    """Fits at the porosity-limit and the apparent interface positions, and the
    relative L2 error of the analytic two-domain profiles (BJ, Br, OTW)
    against the pore-scale one over the fluid layers."""
    nz = len(u)
    top = nz - 1.5
    zc = np.arange(nz, dtype=np.float64)
    inner = slice(1, nz - 1)
    out = {}
    for name, zi in (("porosity_limit", porosity_limit(eps, nz - 1)),
                     ("apparent", apparent_interface(u, eps, bed_top, nu, G))):
        f = fit_interface(u, eps, zi, bed_top, nu, G)
        eb = float(np.mean(eps[bed_top // 4:3 * bed_top // 4]))
        bj = stokes_bj(zi, top, G, nu, f.K, f.Um, f.alpha)
        ubj = np.where(zc >= zi, bj(zc - zi), f.Um)
        br = stokes_brinkman(zi, top, 0.5, G, nu, f.K, eb, f.J, 0.0)(zc)
        otw = stokes_brinkman(zi, top, 0.5, G, nu, f.K, eb, f.J, f.beta)(zc)
        nrm = np.linalg.norm(u[inner])
        out[name] = {"zi": zi, "K": f.K, "Um": f.Um, "Us": f.Us, "dU_plus": f.dU_plus, "dU_minus": f.dU_minus,
                     "alpha": f.alpha, "beta": f.beta, "J": f.J, "poly": list(f.poly), "decay": f.decay,
                     "rms_free": f.rms_free, "rms_porous": f.rms_porous,
                     "err_BJ": float(np.linalg.norm((ubj - u)[inner]) / nrm),
                     "err_Br": float(np.linalg.norm((br - u)[inner]) / nrm),
                     "err_OTW": float(np.linalg.norm((otw - u)[inner]) / nrm)}
    return out


def steady_profile(dom, p, bed_top, tol=1e-7, check=100, chunk=20000, max_steps=2_000_000):
    """Run a coupled bed from rest to steady state on the GPU (the steady test
    of lbm_run_to_steady, in chunks) and return its plane-averaged superficial
    x-velocity, planar porosity, step count and seconds."""
    import time

    import torch

    from . import lbm

    ctx = lbm.Context(lbm.Geometry(dom), p)
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        n = int(ctx.run_to_steady(tol, check, chunk)[0])
        steps += n
        print(f"  {steps} steps", file=sys.stderr, flush=True)
        if n < chunk:
            break
    torch.cuda.synchronize()
    u, _, por = ctx.average_profile()
    return u, por, steps, time.perf_counter() - t0


def study(u, eps, bed_top, nu, G):
    """evaluate() plus the parameter study of every condition at both
    interface positions."""
    res = evaluate(u, eps, bed_top, nu, G)
    for name in ("porosity_limit", "apparent"):
        res[name]["sensitivity"] = sensitivity(u, eps, res[name]["zi"], bed_top, nu, G)
    return res


def main():
    """Steady coupled bed (128x64x256, radii U[6,10], porosity 0.6, tau+ 1.0) on
    the GPU, then the two-domain evaluation and parameter study; prints one
    JSON line."""
    from . import workloads as W

    dom, _, eps_bed = W.coupled_c1(seed=1, bc="cli")
    p = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3.0 / 16.0, force=(1e-6, 0.0, 0.0), layout="aa")
    nu = (p.tau_plus - 0.5) / 3.0
    u, por, steps, sec = steady_profile(dom, p, 128)
    res = study(u, por, 128, nu, p.force[0])
    res["bed_porosity"] = eps_bed
    res["steps"] = steps
    res["seconds"] = sec
    res["u"] = u.tolist()
    res["eps"] = por.tolist()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
