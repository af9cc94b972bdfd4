"""Learned closure of the gray (Brinkman) model of Sec. 4, end to end on the GPU.

Data.  Steady pore-scale runs of a free channel over a sphere bed (the
coupled configuration of Sec. 3.1) give the superficial velocity U(z) and the
planar porosity eps(z) of each bed; periodic REV cubes of the same grain
size, run together in one batched launch, give the Darcy permeability K of
eq. (Darcy) over a range of porosities.

Training.  The network maps the 33 planar porosities around a cell to
(nu_eff, drag) of the gray model.  Its loss has two parts, both evaluated on
the GPU by this library's kernels:
  * bed profiles: the relative L2 misfit between the steady gray column and
    the pore-scale U(z) (mlp_profile_loss, an adjoint through the steady
    column);
  * REV cubes: squared error of o2 against the value that reproduces K in
    every plane (mlp_loss), which pins the drag deep inside porous layers
    where the bed profiles carry little signal.
Both gradients flow back through mlp_backward; Adam updates the FP32 master
weights.

Evaluation.  For a bed that was not trained on, the closure sets the cells of
a gray column, which runs to steady state (gray LBM kernel), and its U(z) is
compared with the pore-scale U(z).  The reference model is the one the paper
evaluates: nu_eff = nu / eps with a drag eps nu / K(eps) from a Kozeny-Carman
fit K = C eps^3 / (1 - eps)^2 to the REV permeabilities.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import gray, lbm, mlp
from . import workloads as W


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@dataclass
class Setup:
    """Shapes and physics of one closure experiment."""
    nx: int = 128
    ny: int = 64
    nz: int = 256
    bed_top: int = 128
    r_range: tuple = (6.0, 10.0)
    tau: float = 1.0
    force: float = 1e-6
    bc: str = "cli"
    # layout of the pore-scale runs and the REV batch: "auto" lets the
    # library's layout autotuner time the candidates once per shape (every
    # layout gives the same fields bit for bit)
    layout: str = "auto"
    train: list = field(default_factory=lambda: [(e, 21 + i) for i, e in
                                                 enumerate((0.40, 0.45, 0.50, 0.55, 0.60, 0.65, 0.70, 0.75, 0.80))])
    test: list = field(default_factory=lambda: [(0.425, 31), (0.575, 32), (0.725, 33)])
    rev_edges: tuple = (48, 64)
    rev_count: int = 48
    rev_porosity: tuple = (0.35, 0.85)
    rev_seed: int = 3000
    tol: float = 1e-7
    check: int = 100
    max_steps: int = 2_000_000
    chunk: int = 20_000
    # Adam steps: over six initialisation seeds the worst held-out error was
    # 0.6-2.5 % (mean 1.2 %) after 3000 steps and 0.3-1.7 % (mean 0.9 %) after
    # 10000, at 3.5 s of training
    train_steps: int = 10000
    lr: float = 2e-3
    w_rev: float = 0.003
    seed: int = 0

    @property
    def nu(self):
        return (self.tau - 0.5) / 3.0

    def params(self):
        return W.Params(collision="trt", tau_plus=self.tau, magic_lambda=3.0 / 16.0,
                        force=(self.force, 0.0, 0.0), layout=self.layout)


def small_setup():
    """A scaled-down experiment (64 x 32 x 128 beds, radii U[3,5]) that runs in
    seconds."""
    return Setup(nx=64, ny=32, nz=128, bed_top=64, r_range=(3.0, 5.0),
                 train=[(e, 21 + i) for i, e in enumerate((0.40, 0.50, 0.60, 0.70, 0.80))],
                 test=[(0.45, 31), (0.65, 32)], rev_edges=(32,), rev_count=24, chunk=10_000,
                 train_steps=1500)


# ----------------------------------------------------------------------------
# pore-scale data
# ----------------------------------------------------------------------------

def bed_domain(s: Setup, porosity, seed):
    S, eps = W.porous_bed(seed, s.nx, s.ny, s.nz, s.bed_top, s.r_range, porosity)
    return W.Domain(s.nx, s.ny, s.nz, spheres=S, bc=s.bc, name=f"bed-{porosity}-{seed}"), eps


def run_bed(s: Setup, porosity, seed):
    """Steady pore-scale run of one bed; returns its planar porosity, the
    superficial velocity profile and the GPU time to steady state."""
    dom, eps_bed = bed_domain(s, porosity, seed)
    geo = lbm.Geometry(dom)
    ctx = lbm.Context(geo, s.params())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while steps < s.max_steps:
        # one call per chunk keeps the host informed; the steady test restarts
        # its reference value at each call, which costs one check interval
        n = int(ctx.run_to_steady(s.tol, s.check, s.chunk)[0])
        steps += n
        if n < s.chunk:
            break
        log(f"  bed eps {porosity} seed {seed}: {steps} steps")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    u_sup, _, por = ctx.average_profile()
    K = ctx.permeability(z0=s.bed_top // 4, z1=3 * s.bed_top // 4)
    layout = ctx.params.layout
    del ctx
    return {"porosity": porosity, "seed": seed, "eps_bed": eps_bed, "eps": por, "u": u_sup, "steps": steps,
            "seconds": sec, "K_bed": K, "cells": s.nx * s.ny * s.nz, "layout": layout}


def run_revs(s: Setup):
    """Periodic REV cubes of the bed's grain size in one batched launch;
    returns (planar porosity profile, K, mean porosity) per cube."""
    rng = np.random.default_rng(s.rev_seed)
    doms = []
    for i in range(s.rev_count):
        edge = int(rng.choice(s.rev_edges))
        target = float(rng.uniform(*s.rev_porosity))
        S, _ = W.rev_cube(s.rev_seed + i, edge, s.r_range, target)
        d = W.Domain(edge, edge, edge, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), spheres=S,
                     bc=s.bc, name=f"rev-{i}")
        doms.append(d)
    geo = lbm.Geometry(doms)
    ctx = lbm.Context(geo, s.params())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = ctx.run_to_steady(s.tol, s.check, 200_000)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out = []
    for i in range(len(doms)):
        _, _, por = ctx.average_profile(dom=i)
        K = ctx.permeability(dom=i)
        out.append({"eps": por, "K": K, "eps_mean": float(por.mean()), "steps": int(steps[i])})
    del ctx
    log(f"  {len(doms)} REV cubes in {sec:.2f} s, steps {int(steps.min())}..{int(steps.max())}")
    return out, sec


def kozeny_carman(revs):
    """C of K = C eps^3 / (1 - eps)^2, least squares in log K."""
    e = np.array([r["eps_mean"] for r in revs])
    K = np.array([r["K"] for r in revs])
    ok = K > 0
    return float(np.exp(np.mean(np.log(K[ok]) - np.log(e[ok] ** 3 / (1 - e[ok]) ** 2))))


# ----------------------------------------------------------------------------
# training
# ----------------------------------------------------------------------------

def _pad_rows(x):
    n = x.shape[0]
    npad = (n + mlp.ROWS - 1) // mlp.ROWS * mlp.ROWS
    if npad == n:
        return x
    return torch.cat([x, torch.zeros((npad - n, x.shape[1]), dtype=x.dtype, device=x.device)])


def training_set(net: mlp.ClosureNet, beds, revs, nu):
    """Inputs, REV targets and masks: rows [0, P*nz) are the bed profiles (in
    the order of beds), the REV rows follow."""
    P, nz = len(beds), len(beds[0]["eps"])
    eb = np.stack([b["eps"] for b in beds])
    xb, nb = net.windows(eb)
    xs, ts, ms = [xb[:nb]], [np.zeros((nb, 2))], [np.zeros((nb, 2))]
    for r in revs:
        e = r["eps"]
        L = len(e)
        ext = np.concatenate([e[L - 16:], e, e[:16]])  # periodic windows
        xw, n = net.windows(ext)
        xs.append(xw[16:16 + L])
        t = np.zeros((L, 2))
        m = np.zeros((L, 2))
        drag = e * nu / r["K"]
        s = 1.0 - e
        ok = s > 1e-6
        t[ok, 1] = np.log(np.expm1(drag[ok] / s[ok]))
        m[ok, 1] = 1.0
        ts.append(t)
        ms.append(m)
    x = _pad_rows(torch.cat(xs))
    B = x.shape[0]
    T = np.zeros((B, 2))
    M = np.zeros((B, 2))
    T[:sum(len(a) for a in ts)] = np.concatenate(ts)
    M[:sum(len(a) for a in ms)] = np.concatenate(ms)
    dev = net.dev
    return {"x": x, "t": torch.tensor(T, dtype=torch.float32, device=dev),
            "m": torch.tensor(M, dtype=torch.float32, device=dev), "msum": float(M.sum()),
            "eps": torch.tensor(eb.ravel(), dtype=torch.float64, device=dev),
            "u": torch.tensor(np.stack([b["u"] for b in beds]).ravel(), dtype=torch.float64, device=dev),
            "P": P, "nz": nz}


def train(net: mlp.ClosureNet, data, nu, G, steps, lr, w_rev, log_every=500):
    """Adam on profile loss + w_rev * REV loss; returns the loss history."""
    hist = []
    P, nz = data["P"], data["nz"]
    for it in range(steps):
        lr_it = lr * (0.1 ** (it / max(steps, 1)))  # decays to lr/10
        y = net.forward(data["x"], train=True)
        Lr, dy = net.loss(y, data["t"], data["m"], max(data["msum"], 1.0) / w_rev)
        Lp, _ = net.profile_loss(y, data["eps"], data["u"], P, nz, nu, G, 1.0, dy=dy)
        net.backward(data["x"], dy)
        net.adam(lr_it)
        hist.append((float(Lp.sum()), Lr))
        if log_every and (it % log_every == 0 or it == steps - 1):
            log(f"  train {it}: profile {Lp.sum():.3e}  rev {Lr:.3e}")
    return hist


# ----------------------------------------------------------------------------
# evaluation
# ----------------------------------------------------------------------------

def wall_free_fluid(eps, nue, drag, nu):
    """Copies of a column's coefficients whose wall layers (z = 0 and nz-1,
    solid in the gray model: bounce-back, their coefficients unused) carry
    free-fluid values, porosity clipped to [1e-3, 1].  The closure network
    never sees wall layers in training, so its outputs there are arbitrary
    and may lie outside what the collision accepts."""
    e = np.array(eps, dtype=np.float64)
    n = np.array(nue, dtype=np.float64)
    d = np.array(drag, dtype=np.float64)
    e[0] = e[-1] = 1.0
    n[0] = n[-1] = nu
    d[0] = d[-1] = 0.0
    return np.clip(e, 1e-3, 1.0), n, d


def gray_steady(eps, nue, drag, G, s: Setup):
    """Gray column to steady state on the GPU; wall layers are given free-fluid
    values (they are solid in the model)."""
    e, nue, drag = wall_free_fluid(eps, nue, drag, s.nu)
    col = gray.GrayColumns(e, nue, drag, G=(G, 0.0, 0.0), walls=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = int(col.run_to_steady(s.tol, s.check, s.max_steps)[0])
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    u = col.profile()[:, 0]
    return u, steps, sec


def rel_err(u, ref):
    return float(np.linalg.norm(u[1:-1] - ref[1:-1]) / np.linalg.norm(ref[1:-1]))


def evaluate(net: mlp.ClosureNet, bed, s: Setup, C_kc):
    """Learned closure and the reference models on one bed."""
    nu, G, eps = s.nu, s.force, bed["eps"]
    res = {"porosity": bed["porosity"], "seed": bed["seed"], "pore_scale_seconds": bed["seconds"],
           "pore_scale_steps": bed["steps"], "pore_scale_layout": bed["layout"]}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nue, drag = net.closure(eps, nu)
    torch.cuda.synchronize()
    t_mlp = time.perf_counter() - t0
    u, steps, sec = gray_steady(eps, nue.ravel(), drag.ravel(), G, s)
    res.update({"learned_err": rel_err(u, bed["u"]), "gray_steps": steps, "gray_seconds": sec,
                "mlp_seconds": t_mlp, "cost_ratio": bed["seconds"] / (sec + t_mlp)})
    # reference: nu/eps and Kozeny-Carman drag (porous cells only)
    e = np.clip(eps, 1e-3, 1.0)
    porous = e < 1.0
    Kkc = np.where(porous, C_kc * e ** 3 / np.maximum(1 - e, 1e-12) ** 2, np.inf)
    drag_kc = np.where(porous, e * nu / Kkc, 0.0)
    u1, _, _ = gray_steady(eps, nu / e, drag_kc, G, s)
    u2, _, _ = gray_steady(eps, np.full_like(e, nu), drag_kc, G, s)
    res["baseline_nu_over_eps_err"] = rel_err(u1, bed["u"])
    res["baseline_nu_err"] = rel_err(u2, bed["u"])
    res["u_pore"] = bed["u"].tolist()
    res["u_learned"] = u.tolist()
    res["u_baseline"] = u1.tolist()
    return res


def experiment(s: Setup, init_seed=0, extra_seeds=()):
    """Data, training and evaluation; returns a summary dict.  extra_seeds:
    further initialisation seeds, each trained on the same data and scored
    on the held-out beds (the spread over initialisations)."""
    t_all = time.perf_counter()
    log(f"REV batch: {s.rev_count} cubes, edges {s.rev_edges}, radii {s.r_range}")
    revs, t_rev = run_revs(s)
    C_kc = kozeny_carman(revs)
    log(f"Kozeny-Carman constant {C_kc:.4g}")
    beds = []
    for e, seed in s.train + s.test:
        b = run_bed(s, e, seed)
        log(f"bed eps {e} seed {seed}: bed porosity {b['eps_bed']:.4f}, {b['steps']} steps, {b['seconds']:.2f} s "
            f"({b['layout']} layout)")
        beds.append(b)
    train_beds, test_beds = beds[:len(s.train)], beds[len(s.train):]
    nu, G = s.nu, s.force
    net = mlp.ClosureNet(mlp.init_params(init_seed))
    data = training_set(net, train_beds, revs, nu)
    log(f"training: {data['x'].shape[0]} rows ({data['P']} profiles of {data['nz']} cells + REV cells), "
        f"{s.train_steps} Adam steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, data, nu, G, s.train_steps, s.lr, s.w_rev)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    results = []
    for b in test_beds:
        r = evaluate(net, b, s, C_kc)
        log(f"held-out bed eps {b['porosity']} seed {b['seed']}: learned {r['learned_err']:.4f}, "
            f"nu/eps {r['baseline_nu_over_eps_err']:.4f}, nu {r['baseline_nu_err']:.4f}; "
            f"pore scale {r['pore_scale_seconds']:.2f} s vs gray+MLP {r['gray_seconds'] + r['mlp_seconds']:.4f} s "
            f"(x{r['cost_ratio']:.0f})")
        results.append(r)
    train_fit = [evaluate(net, b, s, C_kc) for b in train_beds]
    spread = [{"seed": init_seed, "held_out_err": [r["learned_err"] for r in results]}]
    for k in extra_seeds:
        other = mlp.ClosureNet(mlp.init_params(k))
        train(other, training_set(other, train_beds, revs, nu), nu, G, s.train_steps, s.lr, s.w_rev, log_every=0)
        errs = []
        for b in test_beds:
            nue, drag = other.closure(b["eps"], nu)
            u, _, _ = gray_steady(b["eps"], nue.ravel(), drag.ravel(), G, s)
            errs.append(rel_err(u, b["u"]))
        log(f"initialisation seed {k}: held-out errors {[round(e, 4) for e in errs]}")
        spread.append({"seed": k, "held_out_err": errs})
    return {"setup": {k: v for k, v in s.__dict__.items()}, "kozeny_carman_C": C_kc, "rev_seconds": t_rev,
            "train_seconds": t_train, "final_loss": hist[-1], "initial_loss": hist[0], "held_out": results,
            "train_fit": [{k: v for k, v in r.items() if not k.startswith("u_")} for r in train_fit],
            "rev": [{"eps_mean": r["eps_mean"], "K": r["K"], "steps": r["steps"]} for r in revs],
            "seed_spread": spread, "params": net.params.cpu().numpy(), "total_seconds": time.perf_counter() - t_all}


def evaluate_at_height(params, s: Setup, nz, C_kc, beds=None):
    """The trained closure (network parameters `params`) on held-out beds of
    another height: the same lateral size, grain sizes and physics, nz layers
    with the bed in the lower half, so the gray column is 1 x 1 x nz.  The
    network is local (33-cell porosity windows), so a closure trained on one
    bed height applies to any."""
    import dataclasses

    se = dataclasses.replace(s, nz=nz, bed_top=nz // 2)
    net = mlp.ClosureNet(params)
    out = []
    for e, seed in (beds or s.test):
        b = run_bed(se, e, seed)
        r = evaluate(net, b, se, C_kc)
        log(f"bed {se.nx}x{se.ny}x{nz} eps {e} seed {seed}: learned {r['learned_err']:.4f}, "
            f"nu/eps {r['baseline_nu_over_eps_err']:.4f}, nu {r['baseline_nu_err']:.4f}; "
            f"pore scale {r['pore_scale_seconds']:.2f} s ({r['pore_scale_steps']} steps) vs gray+MLP "
            f"{r['gray_seconds'] + r['mlp_seconds']:.4f} s (x{r['cost_ratio']:.0f})")
        out.append(r)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--small", action="store_true", help="the scaled-down experiment")
    ap.add_argument("--seeds", type=int, default=1,
                    help="also train networks from initialisation seeds 1 .. N-1 on the same data and report "
                         "their held-out errors")
    ap.add_argument("--eval-nz", type=int, default=0,
                    help="also evaluate the trained closure on held-out beds of this height (1 x 1 x nz columns)")
    ap.add_argument("--out", default=None, help="write the summary JSON here")
    args = ap.parse_args()
    s = small_setup() if args.small else Setup()
    res = experiment(s, extra_seeds=range(1, args.seeds))
    if args.eval_nz:
        hs = evaluate_at_height(res["params"], s, args.eval_nz, res["kozeny_carman_C"])
        res["held_out_nz"] = [{k: v for k, v in r.items() if not k.startswith("u_")} for r in hs]
        res["eval_nz"] = args.eval_nz
    res.pop("params")
    line = {k: v for k, v in res.items() if k != "held_out"}
    line["held_out"] = [{k: v for k, v in r.items() if not k.startswith("u_")} for r in res["held_out"]]
    print(json.dumps(line, default=float), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, default=float)


if __name__ == "__main__":
    main()
