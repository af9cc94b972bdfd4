"""Deposited sphere packings and the grid-resolution study of Sec. 3.1.

The paper builds its porous beds with a rigid-body simulation: spheres whose
diameters vary by up to 50 % around a mean fall into the domain from the top
one after another and come to rest on the floor or on spheres below; their
final positions define the solid matrix.  This module generates such
packings by sequential deposition in units of the mean diameter, periodic in
x and y:

  * each sphere starts at a random (x, y) above the bed, falls vertically to
    its first contact (floor or a sphere), then settles: repeated small
    downward steps, each followed by projection out of every overlap (the
    sphere slides or rolls over its supports), until it no longer descends,
    i.e. it rests on the floor or in a pocket of three supports;
  * the packing is then scaled to a lattice resolution D (cells per mean
    diameter), quantised to 2^-12 and made exactly non-overlapping.

The same unit packing scaled to several D is the input of the grid study
(D = 4 ... 48 at Re_D = U_max D / nu of about 2: the plane-averaged profile,
normalised by its maximum and the channel height, converges with D).  The
packings are input preparation on the host, not part of the timed path.
"""
from __future__ import annotations

import math

import numpy as np

from . import workloads as W


def _min_image_xy(d, L):
    d[..., 0] -= L[0] * np.round(d[..., 0] / L[0])
    d[..., 1] -= L[1] * np.round(d[..., 1] / L[1])
    return d


def _drop_height(x, y, r, C, R, L, z_from=np.inf):
    """Height of the centre of a sphere (radius r) falling vertically at
    (x, y) from z_from when it first touches the floor (centre at z = r) or a
    sphere of C/R (only contacts at or below z_from count)."""
    z = r
    if len(C):
        d = _min_image_xy(C[:, :2] - np.array([x, y]), L)
        h2 = (d * d).sum(1)
        s = R + r
        m = h2 < s * s
        if m.any():
            zc = C[m, 2] + np.sqrt(s[m] * s[m] - h2[m])
            zc = zc[zc <= z_from + 1e-12 * max(1.0, abs(z_from) if np.isfinite(z_from) else 1.0)]
            if len(zc):
                z = max(z, float(np.max(zc)))
    return z


_G = np.array([0.0, 0.0, -1.0])  # gravity


def _overlapping(c, r, C, s, L):
    if not len(C):
        return False
    d = _min_image_xy(c - C, L)
    return bool(np.any(np.sqrt((d * d).sum(1)) < s * (1.0 - 1e-9)))


def _descent(N):
    """Direction of steepest descent of the height that keeps every contact
    (rows of N: outward unit normals of the active contacts, n.d >= 0): the
    projection of gravity onto that cone, found by trying every active set of
    up to three contacts and keeping the one that satisfies the optimality
    conditions (non-negative multipliers, feasible direction).  Returns the
    direction and the contacts that stay closed along it."""
    from itertools import combinations

    m = len(N)
    gn = N @ _G
    if np.all(gn >= 0.0):
        return _G.copy(), ()
    if m == 1:
        return _G - gn[0] * N[0], (0,)
    best, bestd, bestS = None, np.inf, ()
    for k in range(0, min(m, 3) + 1):
        for S in combinations(range(m), k):
            if k == 0:
                d, lam = _G.copy(), np.zeros(0)
            else:
                A = N[list(S)]
                M = A @ A.T
                if abs(np.linalg.det(M)) < 1e-14:
                    continue
                lam = -np.linalg.solve(M, A @ _G)
                d = _G + A.T @ lam
            if np.any(lam < -1e-12) or np.any(N @ d < -1e-10):
                continue
            dist = float(np.linalg.norm(d - _G))
            if dist < bestd:
                best, bestd, bestS = d, dist, S
    if best is None:
        return np.zeros(3), ()
    return best, bestS


def _newton_contacts(p, r, Cc, sc, L, eq, floor, iters=30):
    """Nearest point to p (Gauss-Newton on the squared distances) at which
    the sphere touches exactly the spheres eq (indices into Cc) and, if floor,
    the floor; None if that fails to converge."""
    if not eq and not floor:
        return p
    for _ in range(iters):
        rows, res = [], []
        for j in eq:
            d = _min_image_xy((p - Cc[j])[None, :], L)[0]
            rows.append(2.0 * d)
            res.append(float(d @ d) - sc[j] * sc[j])
        if floor:
            rows.append(np.array([0.0, 0.0, 1.0]))
            res.append(p[2] - r)
        J = np.array(rows)
        res = np.array(res)
        if np.max(np.abs(res)) <= 1e-13 * (1.0 + r * r):
            return p
        M = J @ J.T
        try:
            p = p - J.T @ np.linalg.solve(M, res)
        except np.linalg.LinAlgError:
            return None
    return None


def _settle(c, r, C, R, L, rng, step, max_iter=20000, tol=1e-9):
    """Roll from c to a resting position.  Without a contact the sphere falls
    to its next contact; otherwise it moves along the steepest feasible
    descent over its contacts (sliding and rolling over its supports) by at
    most `step`, and Newton's method puts it back on the contacts that stay
    closed along that direction and on any sphere the step reaches.  It rests
    when no descent remains with the floor or three spheres as supports; a
    balance on one or two spheres alone (unstable) is broken by a small random
    horizontal nudge.  Only spheres within reach of the current position take
    part (the candidate set is renewed as the sphere moves)."""
    c = c.copy()
    rmax = float(R.max()) if len(R) else r
    reach = r + rmax + 4.0 * step + 0.5
    anchor = None

    def candidates(c):
        if not len(C):
            return C, R
        d = _min_image_xy(C[:, :2] - c[:2], L)
        m = (d * d).sum(1) < reach * reach
        return C[m], R[m]

    h = step
    for _ in range(max_iter):
        if anchor is None or float(np.hypot(*_min_image_xy((c[:2] - anchor)[None, :], L)[0])) > 0.25:
            anchor = c[:2].copy()
            Cc, Rc = candidates(c)
            sc = Rc + r
        if len(Cc):
            d = _min_image_xy(c - Cc, L)
            dist = np.sqrt((d * d).sum(1))
            act = np.nonzero(dist <= sc * (1.0 + 100.0 * tol))[0]
            N = d[act] / dist[act][:, None]
        else:
            act = np.zeros(0, int)
            N = np.zeros((0, 3))
        on_floor = c[2] <= r * (1.0 + 100.0 * tol)
        if on_floor:
            N = np.vstack([N, [0.0, 0.0, 1.0]])
        if len(N) == 0:
            c[2] = _drop_height(c[0], c[1], r, C, R, L, c[2])
            anchor = None
            continue
        dv, keep = _descent(N)
        if float(np.linalg.norm(dv)) < 1e-9:
            if on_floor or len(act) >= 3:
                break
            cn = c.copy()
            cn[:2] += rng.normal(0.0, 1e-3 * r, 2)
            cn = _newton_contacts(cn, r, Cc, sc, L, list(act), False)
            if cn is not None and not _overlapping(cn, r, Cc, sc, L):
                c = cn
            continue
        eq = [int(act[i]) for i in keep if i < len(act)]
        fl = on_floor and any(i == len(act) for i in keep)
        trial = c + h * dv
        ok = False
        for _add in range(3):
            cn = _newton_contacts(trial, r, Cc, sc, L, eq, fl)
            if cn is None:
                break
            dd = _min_image_xy(cn - Cc, L) if len(Cc) else np.zeros((0, 3))
            dist2 = np.sqrt((dd * dd).sum(1)) if len(Cc) else np.zeros(0)
            hit = [int(j) for j in np.nonzero(dist2 < sc * (1.0 - 1e-12))[0] if int(j) not in eq]
            below_floor = cn[2] < r * (1.0 - 1e-12)
            if not hit and not below_floor:
                ok = True
                break
            eq += hit
            fl = fl or below_floor
            if len(eq) + fl > 3:
                break
        if not ok or cn[2] >= c[2] - 1e-13:
            h *= 0.5
            if h < 1e-7 * r:
                break
            continue
        c = cn
        h = min(step, 2.0 * h)
    c[0] %= L[0]
    c[1] %= L[1]
    return c


def deposit(seed, Lx, Ly, n, d_spread=0.5, step=0.05):
    """n spheres of diameters uniform in [1 - d_spread, 1 + d_spread] (units of
    the mean diameter) deposited one after another in a box periodic in x
    and y (extent Lx, Ly) onto the floor z = 0.  Returns an (n, 4) array
    (cx, cy, cz, r) in those units, non-overlapping to rounding."""
    if min(Lx, Ly) <= 2.0 * (1.0 + d_spread):
        # a sphere could touch two periodic images of one neighbour, which the
        # minimum-image contacts cannot represent
        raise ValueError("deposit: Lx and Ly must exceed twice the largest diameter")
    rng = np.random.default_rng(seed)
    L = np.array([Lx, Ly], dtype=np.float64)
    C = np.zeros((0, 3))
    R = np.zeros(0)
    for _ in range(n):
        r = 0.5 * rng.uniform(1.0 - d_spread, 1.0 + d_spread)
        x, y = rng.uniform(0.0, Lx), rng.uniform(0.0, Ly)
        z = _drop_height(x, y, r, C, R, L)
        c = _settle(np.array([x, y, z]), r, C, R, L, rng, step * 2 * r)
        C = np.vstack([C, c])
        R = np.append(R, r)
    return np.column_stack([C, R])


def bed_height(S_unit):
    """Top of the deposited bed: the highest sphere top."""
    return float(np.max(S_unit[:, 2] + S_unit[:, 3]))


def supported(S, Lx, Ly, tol=1e-6):
    """Per sphere: resting on the floor, or touching at least one sphere
    below its centre (a settled sphere always has a support)."""
    L = np.array([Lx, Ly])
    ok = np.zeros(len(S), bool)
    for i, (x, y, z, r) in enumerate(S):
        if z <= r * (1 + tol):
            ok[i] = True
            continue
        d = _min_image_xy(S[:, :3] - np.array([x, y, z]), L)
        dist = np.sqrt((d * d).sum(1))
        s = S[:, 3] + r
        below = (d[:, 2] < 0) & (dist <= s * (1 + tol)) & (np.arange(len(S)) != i)
        ok[i] = bool(below.any())
    return ok


def lattice_packing(S_unit, D, Lx, Ly):
    """The unit packing at D cells per mean diameter: centres and radii scaled
    by D, the floor at the bottom wall plane z = 0.5 (wall layer z = 0),
    quantised to 2^-12 and made exactly non-overlapping (shrinking radii by
    2^-12 where quantisation created an overlap).  Returns (spheres, nx, ny)."""
    nx, ny = int(round(Lx * D)), int(round(Ly * D))
    S = np.array(S_unit, dtype=np.float64) * D
    S[:, 0] *= nx / (Lx * D)
    S[:, 1] *= ny / (Ly * D)
    S[:, 2] += 0.5
    S = W.quantise(S)
    S[:, 0] = np.mod(S[:, 0], nx)
    S[:, 1] = np.mod(S[:, 1], ny)
    S = W._fix_exact(S, np.array([nx, ny, 1e9]), np.array([True, True, False]), None)
    return S, nx, ny


def channel_height(S_unit, free_height):
    """Height between the wall planes in mean diameters: the bed top plus the
    free channel, rounded up to a whole number so that every resolution D
    has the same height H = T D cells."""
    return int(math.ceil(bed_height(S_unit) + free_height))


def study_domain(S_unit, D, Lx, Ly, free_height, bc="cli"):
    """Channel over the deposited bed at resolution D: periodic x and y, wall
    layers at z = 0 and z = T D + 1 (T = channel_height), so the fluid height
    between the wall planes is exactly T D cells at every D."""
    S, nx, ny = lattice_packing(S_unit, D, Lx, Ly)
    nz = channel_height(S_unit, free_height) * D + 2
    return W.Domain(nx, ny, nz, spheres=S, bc=bc, name=f"deposit-D{D}")


# ----------------------------------------------------------------------------
# grid study (Sec. 3.1): one packing at several resolutions, Re_D about 2
# ----------------------------------------------------------------------------

def normalised_profile(u, npts=401):
    """U(z)/U_max on npts points of z/H in [0, 1], H the fluid height between
    the wall planes (cell z of the fluid layers 1..nz-2 sits at (z - 0.5)/H),
    by linear interpolation with U = 0 at both walls."""
    nz = len(u)
    H = nz - 2.0
    zc = np.concatenate([[0.0], (np.arange(1, nz - 1) - 0.5) / H, [1.0]])
    uc = np.concatenate([[0.0], u[1:-1], [0.0]])
    s = np.linspace(0.0, 1.0, npts)
    return s, np.interp(s, zc, uc) / float(np.max(u))


def run_resolution(S_unit, D, Lx, Ly, free_height, re_target=2.0, tau=1.0, tol=1e-7, check=100,
                   chunk=50_000, max_steps=4_000_000, layout="auto", G=None, log=None):
    """One resolution of the study: the channel over the unit packing at D
    cells per mean diameter, driven by a body force G along x chosen for
    Re_D = U_max D / nu = re_target (from a plane-channel estimate over the
    free height unless given), run from rest to steady state on the GPU.
    Returns the plane-averaged profile and the achieved Re_D."""
    import time

    import torch

    from . import lbm

    dom = study_domain(S_unit, D, Lx, Ly, free_height)
    nu = (tau - 0.5) / 3.0
    if G is None:
        Hf = free_height * D
        G = 8.0 * nu * (re_target * nu / D) / (Hf * Hf)
    p = W.Params(collision="trt", tau_plus=tau, magic_lambda=3.0 / 16.0, force=(G, 0.0, 0.0), layout=layout)
    ctx = lbm.Context(lbm.Geometry(dom), p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        n = int(ctx.run_to_steady(tol, check, chunk)[0])
        steps += n
        if n < chunk:
            break
        if log:
            log(f"  D = {D}: {steps} steps ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    u, _, por = ctx.average_profile()
    re = float(np.max(u)) * D / nu
    return {"D": D, "nx": dom.nx, "ny": dom.ny, "nz": dom.nz, "cells": dom.ncells, "G": G, "nu": nu,
            "Re_D": re, "steps": steps, "seconds": sec, "u": u, "eps": por}


def grid_study(Ds=(4, 8, 16, 24, 32, 48), seed=11, Lx=4.0, Ly=4.0, n=64, free_height=3.0, re_target=2.0,
               tau=1.5, re_tol=0.1, log=None):
    """The grid study: one deposited packing (n spheres, diameters 50-150 %
    of the mean, in an Lx x Ly box of mean diameters) at each resolution D,
    at Re_D within re_tol of re_target (a second run with the force rescaled
    by the first run's Re_D if needed; Stokes flow scales linearly).  Returns
    per D the normalised profile and its relative L2 distance from the finest
    resolution's and from the next finer one's.  TRT with Lambda = 3/16 gives
    steady Stokes fields independent of nu (Sec. 2.1), so a large tau (fast
    diffusion to the steady state) changes only the run time."""
    S_unit = deposit(seed, Lx, Ly, n)
    res = []
    G_next = None
    for D in Ds:
        r = run_resolution(S_unit, D, Lx, Ly, free_height, re_target, tau, G=G_next, log=log)
        if abs(r["Re_D"] / re_target - 1.0) > re_tol:
            if log:
                log(f"D = {D}: Re_D {r['Re_D']:.3f}, rerun with the force rescaled")
            r = run_resolution(S_unit, D, Lx, Ly, free_height, re_target, tau, G=r["G"] * re_target / r["Re_D"],
                               log=log)
        # at fixed nu and geometry in units of D, Re_D grows as G D^3: the next
        # resolution's force
        G_next = None
        if D != Ds[-1]:
            G_next = r["G"] * (re_target / r["Re_D"]) * (D / Ds[Ds.index(D) + 1]) ** 3
        s, un = normalised_profile(r["u"])
        r["s"], r["u_norm"] = s, un
        if log:
            log(f"D = {D}: {r['nx']}x{r['ny']}x{r['nz']}, Re_D {r['Re_D']:.3f}, {r['steps']} steps, "
                f"{r['seconds']:.1f} s")
        res.append(r)
    fine = res[-1]["u_norm"]
    for i, r in enumerate(res):
        r["diff_finest"] = float(np.linalg.norm(r["u_norm"] - fine) / np.linalg.norm(fine))
        nxt = res[i + 1]["u_norm"] if i + 1 < len(res) else None
        r["diff_next"] = None if nxt is None else float(np.linalg.norm(r["u_norm"] - nxt) / np.linalg.norm(nxt))
    return {"unit_packing": S_unit, "bed_height": bed_height(S_unit), "runs": res}


def main():
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="grid study on a deposited packing (Sec. 3.1)")
    ap.add_argument("--D", default="4,8,16,24,32,48", help="resolutions, cells per mean diameter")
    ap.add_argument("--n", type=int, default=64, help="spheres in the unit packing")
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args()
    Ds = tuple(int(v) for v in args.D.split(","))
    out = grid_study(Ds, seed=args.seed, n=args.n, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    line = {"bed_height": out["bed_height"], "spheres": len(out["unit_packing"]),
            "runs": [{k: (v.tolist() if isinstance(v, np.ndarray) and k in ("u",) else v)
                      for k, v in r.items() if k not in ("s", "u_norm", "eps")} for r in out["runs"]]}
    print(json.dumps(line, default=float), flush=True)


if __name__ == "__main__":
    main()
