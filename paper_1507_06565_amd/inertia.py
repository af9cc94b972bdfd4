"""Inertial regime of the coupled flow: a Reynolds-number sweep of pore-scale
beds and the learned closure with and without the Forchheimer term.

Sec. 3.1 of the paper varies the Reynolds number of the coupled flow by the
driving pressure gradient at fixed viscosity and grain size, and reports that
at higher Re the flow penetrates the bed less (relative to the free channel)
and the maximum of the plane-averaged velocity moves towards the top wall.
Sec. 4 writes the porous force of the Brinkman-Forchheimer model (eq.
(PorousForce)) with a quadratic Forchheimer drag, negligible in slow flow.

This module runs steady pore-scale beds at increasing body force G (fixed
nu, so Re_D = U_max D / nu grows with G), each run starting from the previous
steady state scaled by the force ratio (the Stokes scaling, which leaves only
the inertial correction to relax), and at each Re evaluates the gray column
with the closure learned in the Stokes regime:
  * Stokes closure: nu_eff and the Darcy drag eps nu / K from the network;
  * plus Forchheimer: phi = eps F_eps / sqrt(K) per cell with K from the
    network's drag and Ergun's F_eps = 1.75 / sqrt(150 eps^3).
Both are compared with the pore-scale U(z) (relative L2), together with the
shape measures of the paper's observation: the height of the maximum and the
velocity at the bed surface relative to the maximum.
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np

from . import closure as CL
from . import workloads as W


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ergun_phi(eps, nu, drag):
    """Forchheimer coefficient phi = eps F_eps / sqrt(K) of eq. (PorousForce)
    per cell, with K = eps nu / drag from the closure's Darcy drag and Ergun's
    F_eps = 1.75 / sqrt(150 eps^3); 0 where the cell is free fluid."""
    eps = np.asarray(eps, dtype=np.float64)
    drag = np.asarray(drag, dtype=np.float64)
    out = np.zeros_like(eps)
    por = (eps > 0.0) & (eps < 1.0) & (drag > 0.0)  # wall layers (eps 0) and free fluid get 0
    K = eps[por] * nu / drag[por]
    F = 1.75 / np.sqrt(150.0 * eps[por] ** 3)
    out[por] = eps[por] * F / np.sqrt(K)
    return out


def shape(u, eps):
    """(height of the maximum of U, U at the bed surface / U_max, mean U over
    the bed interior / U_max): the bed surface is the porosity-limit plane,
    the interior the layers of the lower half of the bed."""
    nz = len(u)
    zmax = float(np.argmax(u))
    top = nz - 2
    while top > 0 and eps[top] >= 1.0:
        top -= 1
    um = float(np.max(u))
    lo, hi = max(1, top // 4), max(2, top // 2)
    return zmax, float(u[top]) / um, float(np.mean(u[lo:hi])) / um


def steady(ctx, tol, check, chunk, max_steps):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        n = int(ctx.run_to_steady(tol, check, chunk)[0])
        steps += n
        if n < chunk:
            break
    torch.cuda.synchronize()
    return steps, time.perf_counter() - t0


def reynolds_sweep(s: CL.Setup, params, beds, re_targets=(0.5, 5.0, 15.0, 30.0), tau=0.56, tol=1e-7, check=100,
                   chunk=100_000, max_steps=6_000_000):
    """Pore-scale beds of the setup's family at the target Reynolds numbers
    (fixed tau, force scaled), each compared with the gray column under the
    learned closure (network parameters `params`) with and without the
    Forchheimer term.  beds: (porosity, seed) pairs.  Returns one record per
    bed and Re."""
    from . import gray, lbm, mlp

    net = mlp.ClosureNet(params)
    nu = (tau - 0.5) / 3.0
    D = float(s.r_range[0] + s.r_range[1])  # mean grain diameter
    out = []
    for porosity, seed in beds:
        dom, eps_bed = CL.bed_domain(s, porosity, seed)
        geo = lbm.Geometry(dom)
        prev, G_prev, k_lin = None, None, None
        for re in re_targets:
            if k_lin is None:
                # first run: plane-channel estimate over the free height
                Hf = s.nz - 2 - s.bed_top
                G = 8.0 * nu * (re * nu / D) / (Hf * Hf)
            else:
                G = re * nu / (D * k_lin)
            p = W.Params(collision="trt", tau_plus=tau, magic_lambda=3.0 / 16.0, force=(G, 0.0, 0.0),
                         layout=s.layout)
            ctx = lbm.Context(geo, p)
            if prev is not None:
                img = prev.copy()
                img[32:].view(np.float32)[:] *= np.float32(G / G_prev)
                ctx.load(img)
            steps, sec = steady(ctx, tol, check, chunk, max_steps)
            u, _, por = ctx.average_profile()
            prev, G_prev = ctx.save(), G
            del ctx
            umax = float(np.max(u))
            if k_lin is None:
                k_lin = umax / G
            re_act = umax * D / nu
            nue, drag = net.closure(por, nu)
            nue, drag = nue.ravel(), drag.ravel()
            ug, _, _ = CL.gray_steady(por, nue, drag, G, s)
            uf, _, _ = gray_steady_forchheimer(por, nue, drag, ergun_phi(por, nu, drag), G, s)
            rec = {"porosity": porosity, "seed": seed, "eps_bed": eps_bed, "Re_target": re, "Re_D": re_act, "G": G,
                   "nu": nu, "steps": steps, "seconds": sec, "u_max": umax,
                   "shape_pore": shape(u, por), "shape_gray": shape(ug, por), "shape_forchheimer": shape(uf, por),
                   "err_gray": CL.rel_err(ug, u), "err_forchheimer": CL.rel_err(uf, u),
                   "gray_forchheimer_diff": CL.rel_err(uf, ug),
                   "u_pore": u.tolist(), "u_gray": ug.tolist(), "u_forchheimer": uf.tolist(), "eps": por.tolist()}
            log(f"bed {porosity}/{seed} Re_D {re_act:.2f} (G {G:.3e}, {steps} steps, {sec:.1f} s): "
                f"gray {rec['err_gray']:.4f}, +Forchheimer {rec['err_forchheimer']:.4f}; "
                f"z_max pore {rec['shape_pore'][0]:.0f} gray {rec['shape_gray'][0]:.0f}; "
                f"U_surface/U_max pore {rec['shape_pore'][1]:.4f} gray {rec['shape_gray'][1]:.4f} "
                f"Forchheimer {rec['shape_forchheimer'][1]:.4f}")
            out.append(rec)
    return out


def gray_steady_forchheimer(eps, nue, drag, phi, G, s: CL.Setup):
    """CL.gray_steady with the per-cell Forchheimer coefficients phi."""
    import torch

    from . import gray

    e, nue, drag = CL.wall_free_fluid(eps, nue, drag, s.nu)
    ph = np.array(phi, dtype=np.float64)
    ph[0] = ph[-1] = 0.0
    col = gray.GrayColumns(e, nue, drag, G=(G, 0.0, 0.0), walls=True)
    col.set_forchheimer(ph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = int(col.run_to_steady(s.tol, s.check, s.max_steps)[0])
    torch.cuda.synchronize()
    return col.profile()[:, 0], steps, time.perf_counter() - t0


def main():
    import argparse
    import json

    ap = argparse.ArgumentParser(description="Reynolds-number sweep of coupled beds against the learned closure")
    ap.add_argument("--small", action="store_true", help="the scaled-down bed family (64x32x128, radii U[3,5])")
    ap.add_argument("--re", default="0.5,5,15,30", help="target Re_D values")
    ap.add_argument("--tau", type=float, default=0.56)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    s = CL.small_setup() if args.small else CL.Setup()
    # train the closure at the sweep's viscosity, with the force scaled by
    # (nu / nu_setup)^2 so that the training runs keep the setup's (Stokes)
    # Reynolds number
    nu0 = s.nu
    s.tau = args.tau
    s.force = s.force * (s.nu / nu0) ** 2
    res = CL.experiment(s)
    log(f"closure trained: held-out errors {[round(r['learned_err'], 4) for r in res['held_out']]}")
    rs = tuple(float(v) for v in args.re.split(","))
    sweep = reynolds_sweep(s, res["params"], s.test, rs, tau=args.tau)
    line = [{k: v for k, v in r.items() if not k.startswith("u_") and k != "eps"} for r in sweep]
    print(json.dumps({"setup": "small" if args.small else "bed 128x64x256", "tau": args.tau, "runs": line},
                     default=float), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(sweep, f, default=float)


if __name__ == "__main__":
    main()
