"""Writes rev_k.json: the FP64 oracle's steady Darcy permeability of eight
cubes of the batched REV workload -- the lowest- and highest-porosity cubes
of the smallest (32) and largest (96) edge -- run from rest until the sum of
u_x over the fluid changes by at most 1e-9 of itself over 100 steps, or for
40000 steps.  Past the physical transient only a weak drift of about 1e-9 per
100 steps remains (worth below 1e-6 of K in total); each entry records its
last relative change.  Calls only oracle/ (and the input generator).  Entries
already in the file are kept, so an interrupted run resumes.  About an hour
on 8 cores.

    python tests/golden/make_rev_k.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1507_06565_amd import workloads as W  # noqa: E402

SAMPLES = [287, 432, 437, 67, 162, 104, 169, 133]


def main():
    path = os.path.join(HERE, "rev_k.json")
    out = []
    if os.path.exists(path):
        with open(path) as f:
            out = [e for e in json.load(f) if e["index"] in SAMPLES]
    done = {e["index"] for e in out}
    for i in SAMPLES:
        if i in done:
            continue
        d, p, target, eps = W.rev_sample_c3(i)
        nu = (p.tau_plus - 0.5) / 3.0
        sim = oracle.Sim(d, p)
        t = time.perf_counter()
        prev = None
        rel = None
        steps = 0
        while steps < 40000:
            sim.step(100)
            steps += 100
            U = float(sim.velocity()[0][sim.fluid()].sum())
            if prev is not None:
                rel = abs(U - prev) / abs(U)
                if rel <= 1e-9:
                    break
            prev = U
        sup, _, _ = oracle.plane_profile(sim.velocity(), sim.fluid(), 2, 0)
        K = oracle.permeability(sup, 0, d.nz, nu, p.rho0, p.force[0])
        out.append({"index": i, "edge": d.nx, "porosity": eps, "K": K, "steps": steps, "last_rel_change": rel})
        print(f"sample {i}: edge {d.nx}, porosity {eps:.4f}, K {K:.6g}, {steps} steps, last change {rel:.2e}, "
              f"{time.perf_counter() - t:.0f} s", flush=True)
        out.sort(key=lambda e: SAMPLES.index(e["index"]))
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
