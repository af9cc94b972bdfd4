"""Two-domain (sharp-interface) evaluation of a steady coupled-flow profile.

Sec. 3.2 of the paper takes the plane-averaged velocity of a pore-scale run of
a free channel over a porous bed and asks which sharp-interface conditions,
with which parameters, reproduce it:

  (BJ)   dU/dz(0+) = alpha / sqrt(K) (U_s - U_m)                 Beavers-Joseph
  (BJS)  sqrt(K) / alpha dU/dz(0+) = U_s - U_m                    Saffman
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


def stokes_brinkman(zi, top, bottom, G, nu, K, eps, J, beta=0.0):
    """Stokes above zi (no slip at top), Brinkman below (nu_eff = J nu, drag
    eps nu / K, force eps G, no slip at bottom); continuous velocity and the
    stress jump nu_eff U'(zi-) - nu U'(zi+) = nu beta / sqrt(K) U(zi)
    (beta = 0: the Brinkman (Br) model with continuous stress).  Returns a
    function of z."""
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
    P, M, a, c = np.linalg.solve(Amat, rhs)

    def U(z):
        s = np.asarray(z, dtype=np.float64) - zi
        free = -G / (2 * nu) * s * s + a * s + c
        porous = Ud + P * np.exp(r * s) + M * np.exp(-r * s)
        return np.where(s >= 0, free, porous)
    return U


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


def main():
    """Steady coupled bed (128x64x256, radii U[6,10], porosity 0.6, tau+ 1.0) on
    the GPU, then the two-domain evaluation; prints one JSON line."""
    import time

    import torch

    from . import lbm
    from . import workloads as W

    dom, _, eps_bed = W.coupled_c1(seed=1, bc="cli")
    p = W.Params(collision="trt", tau_plus=1.0, magic_lambda=3.0 / 16.0, force=(1e-6, 0.0, 0.0), layout="aa")
    nu = (p.tau_plus - 0.5) / 3.0
    ctx = lbm.Context(lbm.Geometry(dom), p)
    t0 = time.perf_counter()
    steps = 0
    while True:
        n = int(ctx.run_to_steady(1e-7, 100, 20000)[0])
        steps += n
        print(f"  {steps} steps", file=sys.stderr, flush=True)
        if n < 20000:
            break
    torch.cuda.synchronize()
    u, _, por = ctx.average_profile()
    res = evaluate(u, por, 128, nu, p.force[0])
    res["bed_porosity"] = eps_bed
    res["steps"] = steps
    res["seconds"] = time.perf_counter() - t0
    res["u"] = u.tolist()
    res["eps"] = por.tolist()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
