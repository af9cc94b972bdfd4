"""Writes c1_20000.json: the FP64 oracle's state of the coupled 128x64x256
bed (Bouzidi, TRT Lambda 3/16, tau+ 0.7, force 1e-6) after 20000 steps from
rest -- the plane-averaged superficial velocity profile and the velocity of
4096 fluid cells drawn with a fixed seed.  Calls only oracle/ (and the input
generator).  About 15 minutes on 8 cores.

    python tests/golden/make_c1_drift.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1507_06565_amd import workloads as W  # noqa: E402

STEPS = 20000


def main():
    dom, params, eps = W.coupled_c1()
    sim = oracle.Sim(dom, params)
    t = time.perf_counter()
    for k in range(STEPS // 1000):
        sim.step(1000)
        print(f"{(k + 1) * 1000} steps, {time.perf_counter() - t:.0f} s", flush=True)
    u = sim.velocity()
    fl = sim.fluid()
    prof = oracle.plane_profile(u, fl, 2, 0)
    rng = np.random.default_rng(20000)
    idx = np.flatnonzero(fl.ravel())
    pick = np.sort(rng.choice(idx, 4096, replace=False))
    ur = u.reshape(3, -1)
    out = {"steps": STEPS, "bed_porosity": eps, "u_sup": list(map(float, prof[0])),
           "cells": pick.tolist(), "u": ur[:, pick].T.tolist()}
    with open(os.path.join(HERE, "c1_20000.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
