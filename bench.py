"""Benchmark of the pore-scale hot path on one MI355X.

Workload (default): the large coupled free-channel / porous-bed domain,
512 x 256 x 1024 cells, sphere bed (radii U[8,16], porosity 0.45) in the lower
half, TRT with Lambda = 3/16, tau+ = 0.7, body force 5e-7, CLI bounce-back at
the spheres, FP32 shifted populations in the brick layout (4x4x4 bricks, the
all-solid ones not stored, pull streaming between two grids; --layout aa or
twogrid selects the dense layouts).  One step is one full time step of the hot
path: the fused stream + collide sweep with the interpolated bounce-back of
every boundary link.  Inputs are resident in HBM before the timed region
starts.

Prints ONE JSON line (rank 0) with MLUPS as `value`, plus the roofline of the
sweep kernel and the CPU oracle's rate on a bounded sample of the workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-check] [--layout L]
    python bench.py --workload rev-batch [--samples 512] [--out profiles.json]

The second form times the batched REV workload (512 periodic cubes to steady
state in persistent launches) and reports its aggregate MLUPS instead.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
CHECK_STEPS = 20  # steps of the sampled-window FP32-vs-FP64 check (short horizon, from rest)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n_fluid, n_cells, n_links):
    """Minimal HBM bytes of one sweep step: 19 FP32 loads + 19 FP32 stores per
    fluid cell, the 4 B cell word of every cell and, per boundary link, its
    4 B coefficient and the 4 B partial bounce-back value read and the new
    partial value stored (12 B)."""
    return 152 * n_fluid + 4 * n_cells + 12 * n_links


def sampled_window_check(dom, params, ctx_factory, geo, nsteps=20, nwin=16, seed=0):
    """FP32 GPU vs FP64 oracle on sampled cells of the full-size domain: the
    oracle runs a window of edge 2 (nsteps + 2) + 6 around each sample and the
    6^3 cells at its centre, more than nsteps + 1 cells from its edge (one
    cell of light cone per step), are compared with the GPU's full-domain
    run."""
    import numpy as np

    import oracle

    ctx = ctx_factory()
    ctx.step(nsteps)
    _, u = ctx.fields()
    rng = np.random.default_rng(seed)
    h = nsteps + 2
    w = 2 * h + 6
    num = den = 0.0
    for _ in range(nwin):
        cz = int(rng.integers(h + 1, dom.nz - h - 5))
        org = (int(rng.integers(0, dom.nx)), int(rng.integers(0, dom.ny)), cz - h)
        sim = oracle.Sim(dom, params, window=(org, (w, w, w)), geometry=geo)
        sim.step(nsteps)
        uw = sim.velocity()
        fw = sim.fluid()
        for zz in range(h, w - h):
            for yy in range(h, w - h):
                for xx in range(h, w - h):
                    if not fw[zz, yy, xx]:
                        continue
                    gx, gy, gz = (org[0] + xx) % dom.nx, (org[1] + yy) % dom.ny, org[2] + zz
                    ref = uw[:, zz, yy, xx]
                    got = u[:, gz, gy, gx]
                    num += float(((got - ref) ** 2).sum())
                    den += float((ref ** 2).sum())
    del ctx
    return (num / den) ** 0.5 if den > 0 else float("nan")


def host_cpu():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of this thread's later parallel regions
    (the oracle's); returns False if no OpenMP runtime is loaded."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(dom, params, geo_oracle, z0, nz_win, budget_s=15.0, single_s=4.0):
    """The FP64 oracle, as it is, on a slab of the workload straddling the
    bed surface; after one untimed step (threads and pages warm up), two
    timed steps calibrate the step count to about budget_s.  Then the same
    on one thread for about single_s (the single-core rate)."""
    import oracle

    sim = oracle.Sim(dom, params, window=((0, 0, z0), (dom.nx, dom.ny, nz_win)), geometry=geo_oracle)
    sim.step(1)
    t = time.perf_counter()
    sim.step(2)
    t1 = (time.perf_counter() - t) / 2
    nsteps = int(max(1, min(400, budget_s / max(t1, 1e-3))))
    t = time.perf_counter()
    sim.step(nsteps)
    dt = time.perf_counter() - t
    cells = dom.nx * dom.ny * nz_win
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    single = None
    if _omp_threads(1):
        t = time.perf_counter()
        sim.step(1)
        t1s = time.perf_counter() - t
        n1 = int(max(1, min(50, single_s / max(t1s, 1e-3))))
        t = time.perf_counter()
        sim.step(n1)
        single = round(cells * n1 / (time.perf_counter() - t) / 1e6, 2)
        _omp_threads(threads)
    return {"value": cells * nsteps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{dom.nx}x{dom.ny}x{nz_win} slab (z {z0}..{z0 + nz_win - 1}) of the workload, "
                      f"{nsteps} steps, FP64 two-grid, {dt:.1f} s",
            "single_core_mlups": single, "cpu": host_cpu()}


def gpu_runtime_loaded():
    """True if the HIP or HSA runtime is mapped into this process (then the
    GPU may already be initialised, and the process must not fork)."""
    try:
        with open("/proc/self/maps") as f:
            maps = f.read()
    except OSError:
        return True
    return "libamdhip64" in maps or "libhsa-runtime64" in maps


def _gen_rev(i):
    from paper_1507_06565_amd import workloads as W
    d, p, target, eps = W.rev_sample_c3(i)
    return i, d, p, target, eps


def rev_batch(args):
    """512 periodic REV cubes (edge in {32,48,64,96}, porosity U[0.35,0.9],
    radii U[3,10]) to steady state in chunks of steps.  Brick layout: all
    cubes in one brick array, one brick-sweep launch per step over the
    running cubes; AA layout: one persistent launch per chunk, whose team
    size grows as samples converge.  The launch shape is autotuned once
    (every shape gives the same result bit for bit)."""
    import multiprocessing as mp

    import numpy as np

    n = args.samples
    t0 = time.perf_counter()
    # sphere packings on the host.  Worker processes are forked only while no
    # GPU runtime is mapped into this process: a profiler's preload library
    # initialises the GPU before main(), and a child forked from such a
    # process inherits GPU state and the profiler's signal handlers (it has
    # crashed at exit, and hung, under rocprofv3).
    workers = args.gen_workers
    if workers > 1 and gpu_runtime_loaded():
        log("a GPU runtime is already loaded in this process (profiler preload?): generating in-process")
        workers = 1
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            gen = sorted(pool.map(_gen_rev, range(n), chunksize=4), key=lambda r: r[0])
    else:
        gen = []
        for i in range(n):
            gen.append(_gen_rev(i))
            if (i + 1) % 32 == 0:
                log(f"  {i + 1} of {n} samples generated ({time.perf_counter() - t0:.0f} s)")
    doms = [g[1] for g in gen]
    from paper_1507_06565_amd import workloads as W
    # a batch runs AA (persistent launch) or bricks (brick-list launches)
    layout = {"twogrid": "aa"}.get(args.layout, args.layout)
    params = W.Params(**{**gen[0][2].__dict__, "layout": layout})
    log(f"{n} REV samples generated ({time.perf_counter() - t0:.1f} s); edges "
        f"{dict(zip(*np.unique([d.nx for d in doms], return_counts=True)))}")

    import torch

    from paper_1507_06565_amd import lbm

    t0 = time.perf_counter()
    geo = lbm.Geometry(doms)
    info = np.array([geo.info(i)[1:] for i in range(n)], dtype=np.int64)  # fluid, links
    cells = np.array([d.nx * d.ny * d.nz for d in doms], dtype=np.int64)
    log(f"geometry: {cells.sum()} cells, {info[:, 0].sum()} fluid, {info[:, 1].sum()} links "
        f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.set_device(0)
    if layout == "auto":
        t1 = time.perf_counter()
        layout, ms_tuned = lbm.autotune_layout(geo, params, steps_per_trial=10)
        params = W.Params(**{**params.__dict__, "layout": layout})
        torch.cuda.empty_cache()
        log(f"layout autotuner: {layout} ({ms_tuned:.3f} ms per step with every cube active; "
            f"{time.perf_counter() - t1:.1f} s)")
    ctx = lbm.Context(geo, params)
    if args.launch:
        block, W0 = (int(v) for v in args.launch.split(","))
        ctx.batch_set_launch(block, W0)
    else:
        block, W0 = ctx.autotune(10) if not args.no_autotune else ctx.batch_get_launch()
    log(f"batched launch (block, workgroups per sample): ({block}, {W0})")
    if args.fixed_steps > 0:
        # every cube active: the batched kernel's steady throughput and bytes per step
        if args.copy_probe:
            a = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            del a, b
            torch.cuda.empty_cache()
        ctx.step(20)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.step(args.fixed_steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / args.fixed_steps
        alg = float((152 * info[:, 0] + 4 * cells + 12 * info[:, 1]).sum())
        print(json.dumps({"workload": f"{n} REV cubes, every cube active", "layout": layout, "block": block,
                          "workgroups_per_sample": W0, "steps": args.fixed_steps, "ms_per_step": round(ms, 3),
                          "cell_updates_per_s": round(float(cells.sum()) / (ms * 1e-3), 1),
                          "algorithmic_bytes_per_step": alg,
                          "algorithmic_gbs": round(alg / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return
    resident = 256 * 1024 // block  # workgroups of this size resident on 256 CUs at 4 waves per SIMD
    chunk = args.chunk
    prev = np.zeros(n, dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W = W0
    while True:
        steps = ctx.run_to_steady(1e-7, 100, chunk)
        adv = steps - prev
        prev = steps
        running = int((adv == chunk).sum())
        log(f"  {time.perf_counter() - t0:7.1f} s: {n - running} of {n} samples steady, "
            f"steps up to {int(steps.max())}" + ("" if layout == "brick" else f", team size {W}"))
        if running == 0 or steps.max() >= args.max_steps:
            break
        if layout == "brick":
            continue  # one launch per step over the running cubes' bricks: no teams to resize
        # fewer samples left: give each more workgroups (next power of two
        # of resident workgroups per running sample)
        want = 1 << max(0, int(np.ceil(np.log2(max(1.0, resident / running)))))
        Wn = int(min(64, max(W0, want)))
        if Wn != W:
            W = Wn
            ctx.batch_set_launch(block, W)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = prev
    converged = int((steps < args.max_steps).sum())
    updates = int((cells * steps).sum())
    alg = float(((152 * info[:, 0] + 4 * cells + 12 * info[:, 1]) * steps).sum())
    mlups = updates / wall / 1e6
    K = np.array([ctx.permeability(dom=i) for i in range(n)])
    eps = np.array([g[4] for g in gen])
    log(f"batch: {wall:.1f} s, {updates / 1e9:.1f} G cell updates, {mlups:.0f} MLUPS, "
        f"{alg / wall / 1e9:.0f} GB/s algorithmic")
    if args.out:
        prof = []
        for i in range(n):
            sup, _, por = ctx.average_profile(dom=i)
            prof.append({"edge": doms[i].nx, "porosity": float(eps[i]), "K": float(K[i]), "steps": int(steps[i]),
                         "eps_z": por.tolist(), "u_z": sup.tolist()})
        with open(args.out, "w") as f:
            json.dump(prof, f)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = rev_cpu_baseline(doms, params)
        log("cpu baseline:", cpu)
    out = {
        "metric": "MLUPS + HBM GB/s (% peak) at stated FP32 error; closure vs pore-scale speed/err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": int(steps.max()),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n} periodic REV cubes, edge in {{32,48,64,96}}, porosity U[0.35,0.9], radii "
                               f"U[3,10], TRT Lambda 3/16 tau 1.0, force 1e-6, CLI, {layout}, FP32 shifted, to steady "
                               f"state (relative change <= 1e-7 per 100 steps)",
                   "samples": n, "cells": int(cells.sum()), "fluid_cells": int(info[:, 0].sum()),
                   "links": int(info[:, 1].sum()), "layout": layout, "block": block,
                   "workgroups_per_sample": W0},
        "batch": {"wall_s": round(wall, 2), "converged": converged, "cell_updates": updates,
                  "steps_min": int(steps.min()), "steps_median": int(np.median(steps)),
                  "steps_max": int(steps.max()), "K_min": float(K.min()), "K_max": float(K.max())},
        "effective_gbs": round(alg / wall / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(alg / wall / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / wall / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_total": alg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def rev_cpu_baseline(doms, params, budget_s=15.0):
    """The FP64 oracle, as it is, on one 48^3 sample of the batch."""
    import oracle

    d = next(x for x in doms if x.nx == 48)
    sim = oracle.Sim(d, params)
    sim.step(1)
    t = time.perf_counter()
    sim.step(20)
    t1 = (time.perf_counter() - t) / 20
    nsteps = int(max(1, min(100000, budget_s / max(t1, 1e-6))))
    t = time.perf_counter()
    sim.step(nsteps)
    dt = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": d.nx ** 3 * nsteps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"one 48^3 REV cube of the batch ({d.name}), {nsteps} steps, FP64 two-grid, {dt:.1f} s",
            "cpu": host_cpu()}


def copy_ceiling(args):
    """The streaming ceiling for the sweep's working set.  (1) lbm_stream_probe:
    exactly the population bytes of the large bed's brick sweep (1,778,143
    bricks x 19 x 64 FP32, read once and written once, 17.3 GB), in the
    sweep's layout and grouped per brick, with nothing else.  (2) Plain
    torch device copies from 64 MiB to 8 GiB per buffer: a working set inside
    the 256 MB last-level cache shows the fabric's rate, larger ones HBM."""
    import torch

    from paper_1507_06565_amd import lbm

    torch.cuda.set_device(0)
    nb = 1778143
    probe = {}
    for grouped in (False, True):
        ms = lbm.stream_probe(nb, grouped=grouped, passes=20)
        tbs = 2 * nb * 64 * 19 * 4 / (ms * 1e-3) / 1e12
        name = "grouped" if grouped else "sweep_layout"
        log(f"stream probe ({name}): {nb} bricks, {ms:.4f} ms per pass, {tbs:.2f} TB/s read + write")
        probe[name] = {"ms": round(ms, 4), "tb_per_s": round(tbs, 3)}
        torch.cuda.empty_cache()
    rows = []
    for mib in (64, 128, 256, 512, 1024, 2048, 4096, 8192):
        n = mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        reps = max(10, int(40 * 1024 / mib))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tbs = 2 * mib * (1 << 20) / (ms * 1e-3) / 1e12
        log(f"copy {mib} MiB each way: {ms:.4f} ms, {tbs:.2f} TB/s read + write")
        rows.append({"mib_each_way": mib, "ms": round(ms, 5), "tb_per_s": round(tbs, 3)})
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "streaming ceiling", "stream_probe_bricks": nb, "stream_probe": probe,
                      "torch_copies": rows}), flush=True)


def weak_block(args):
    """The paper's weak-scaling block shape on one GPU (Sec. 3, the MLUPS-per-
    core figure: one 151^3 block with one sphere of diameter 90 per core, TRT):
    4 x 4 x 4 such blocks, 604^3 cells, periodic on every axis, body force
    along x, brick layout; the same run with simple and with central linear
    interpolated bounce-back, for the cost of CLI over SBB (the paper reports
    about 10 % on its CPU cluster)."""
    import numpy as np
    import torch

    from paper_1507_06565_amd import lbm, workloads as W

    n, B = 4, 151
    L = n * B
    c = np.array([(i + 0.5) * B for i in range(n)])
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    # centres off the lattice points by dyadic fractions, radius 45
    S = W.quantise(np.column_stack([X.ravel() + 0.25, Y.ravel() + 0.125, Z.ravel() + 0.375,
                                    np.full(X.size, 45.0)]))
    torch.cuda.set_device(0)
    out = {}
    for bc in ("sbb", "cli"):
        d = W.Domain(L, L, L, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), spheres=S, bc=bc,
                     name=f"weak-block-{bc}")
        p = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3.0 / 16.0, force=(1e-6, 0.0, 0.0),
                     layout="brick")
        t0 = time.perf_counter()
        geo = lbm.Geometry(d)
        _, n_fluid, n_links = geo.info()
        ctx = lbm.Context(geo, p)
        block, flags = ctx.autotune(6)
        log(f"{bc}: {L}^3, {n_fluid} fluid cells, {n_links} links, launch ({block}, {flags}) "
            f"({time.perf_counter() - t0:.1f} s)")
        ctx.step(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.step(args.steps)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out[bc] = {"ms_per_step": round(ms, 4), "mlups": round(L ** 3 / (ms * 1e-3) / 1e6, 1),
                   "fluid_cells": n_fluid, "links": n_links, "block": block, "flags": flags}
        log(f"{bc}: {ms:.4f} ms per step")
        del ctx, geo
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "4x4x4 blocks of 151^3, one sphere of diameter 90 each (604^3), TRT "
                      "Lambda 3/16 tau 0.7, periodic, brick layout", "steps": args.steps, "warmup": args.warmup,
                      "sbb": out["sbb"], "cli": out["cli"],
                      "cli_over_sbb": round(out["cli"]["ms_per_step"] / out["sbb"]["ms_per_step"], 4)}),
          flush=True)


def closure_kernels(args):
    """Speed of the learned-closure kernels: BF16 MFMA forward and backward of
    the closure network on B rows, the closure map, and the gray column (one
    1x1x512 column of the smoothed-step workload to steady state, and 4096
    columns for a fixed number of steps)."""
    import numpy as np
    import torch

    from paper_1507_06565_amd import gray, mlp, workloads as W

    torch.cuda.set_device(0)
    B = 1 << 16
    net = mlp.ClosureNet(mlp.init_params(0))
    rng = np.random.default_rng(0)
    X = np.zeros((B, 64), np.float32)
    X[:, :33] = rng.uniform(0.35, 1.0, (B, 33))
    x = torch.tensor(X).to(torch.bfloat16).cuda()
    dy = torch.tensor(rng.normal(0, 1e-3, (B, 16)).astype(np.float32)).cuda()
    s = net.stream

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    used = 2 * (33 * 128 + 128 * 128 * 2 + 128 * 2)  # multiply-adds x 2 of the weights in use, per row
    padded = 2 * (64 * 128 + 128 * 128 * 2 + 128 * 16)  # what the 16x16x32 tiles execute
    t_inf = timed(lambda: net.forward(x))
    t_fwd = timed(lambda: net.forward(x, train=True))
    t_bwd = timed(lambda: net.backward(x, dy))
    res = {"mlp_rows": B,
           "forward_ms": round(t_inf, 4), "forward_tflops_used": round(used * B / t_inf / 1e9, 2),
           "forward_tflops_executed": round(padded * B / t_inf / 1e9, 2),
           "train_forward_ms": round(t_fwd, 4), "backward_ms": round(t_bwd, 4),
           "backward_tflops_used": round(2 * used * B / t_bwd / 1e9, 2)}
    log("mlp:", res)
    eps, _, _ = W.smoothed_step_porosity(512, 0)
    nu = 1.0 / 6.0
    col = gray.GrayColumns(eps, nu / eps, np.where(eps < 1, eps * nu / 2.0, 0.0), G=(1e-6, 0, 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = int(col.run_to_steady(1e-7, 100, 2_000_000)[0])
    dt = time.perf_counter() - t0
    res.update({"gray_column_nz": 512, "gray_steps_to_steady": steps, "gray_seconds": round(dt, 4),
                "gray_us_per_step": round(dt / steps * 1e6, 3)})
    res["gray_precision"] = 64
    ncol = 4096
    for bits in (64, 32):
        cols = gray.GrayColumns(np.tile(eps, (ncol, 1)), np.tile(nu / eps, (ncol, 1)),
                                np.tile(np.where(eps < 1, eps * nu / 2.0, 0.0), (ncol, 1)), G=(1e-6, 0, 0),
                                precision=bits)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cols.run(10000)
        dt = time.perf_counter() - t0
        res.update({"gray_columns": ncol, f"gray_fp{bits}_cell_updates_per_s": round(ncol * 512 * 10000 / dt / 1e9, 2)})
    log("gray:", res)
    out = {"metric": "closure kernels: MLP TFLOP/s (BF16 MFMA) and gray-column steps/s", "value": res["forward_tflops_used"],
           "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "closure network 33-128-128-128-2 on 65536 windows; gray column 1x1x512"},
           "detail": res,
           "roofline": {"bound": "mfma", "achieved": res["forward_tflops_executed"], "peak": 2500.0,
                        "unit": "TFLOP/s", "frac": round(res["forward_tflops_executed"] / 2500.0, 5),
                        "traffic": None}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-closure", action="store_true",
                    help="bed: skip the learned-closure half of the metric (about 95 s of GPU work after the sweep)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--layout", choices=("auto", "aa", "twogrid", "brick"), default="auto",
                    help="bed: population layout of the sweep (auto: the library's layout autotuner)")
    ap.add_argument("--launch", default=None, metavar="BLOCK,FLAGS",
                    help="fixed launch shape instead of the autotuner: bed BLOCK,FLAGS (e.g. 1024,2); "
                         "rev-batch BLOCK,WORKGROUPS_PER_SAMPLE")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 2 GiB device copy (reference for HBM counter scaling)")
    ap.add_argument("--workload", choices=("bed", "rev-batch", "closure-kernels", "weak-block", "copy-ceiling"),
                    default="bed",
                    help="bed: the large coupled domain (default); rev-batch: the batched REV cubes; "
                         "closure-kernels: closure network and gray column speed; weak-block: the paper's "
                         "weak-scaling block shape, SBB against CLI; copy-ceiling: device-copy rate against "
                         "buffer size (the practical streaming ceiling)")
    ap.add_argument("--samples", type=int, default=512, help="rev-batch: number of cubes")
    ap.add_argument("--chunk", type=int, default=2000, help="rev-batch: steps per persistent launch")
    ap.add_argument("--max-steps", type=int, default=2_000_000, help="rev-batch: cap per sample")
    ap.add_argument("--out", default=None, help="rev-batch: write per-sample K and profiles (JSON)")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="rev-batch: host processes generating the cubes (1: in this process)")
    ap.add_argument("--fixed-steps", type=int, default=0,
                    help="rev-batch: time this many steps with every cube active (after 20 warm-up steps) "
                         "instead of the run to steady state")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the z-slab decomposition is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "rev-batch":
        rev_batch(args)
        return
    if args.workload == "closure-kernels":
        closure_kernels(args)
        return
    if args.workload == "weak-block":
        weak_block(args)
        return
    if args.workload == "copy-ceiling":
        copy_ceiling(args)
        return

    import numpy as np
    import torch

    from paper_1507_06565_amd import lbm, workloads as W

    t0 = time.perf_counter()
    dom, params, eps = W.large_c2()
    params = W.Params(**{**params.__dict__, "layout": args.layout})
    log(f"workload: {dom.nx}x{dom.ny}x{dom.nz}, {len(dom.spheres)} spheres, bed porosity {eps:.4f} "
        f"({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    geo = lbm.Geometry(dom)
    _, n_fluid, n_links = geo.info()
    log(f"geometry: {n_fluid} fluid cells, {n_links} links "
        f"({time.perf_counter() - t0:.1f} s)")
    n_cells = dom.nx * dom.ny * dom.nz

    torch.cuda.set_device(0)
    layout_tuned = None
    if params.layout == "auto":
        t0 = time.perf_counter()
        name, ms_tuned = lbm.autotune_layout(geo, params, steps_per_trial=10)
        params = W.Params(**{**params.__dict__, "layout": name})
        layout_tuned = {"chosen": name, "trial_ms_per_step": round(ms_tuned, 4)}
        torch.cuda.empty_cache()
        log(f"layout autotuner: {name} ({ms_tuned:.3f} ms per step in its trial; {time.perf_counter() - t0:.1f} s)")
    check = None
    geo_oracle = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        fl = oracle.flags(dom)
        geo_oracle = (fl,) + oracle.links(dom, fl)
        log(f"oracle geometry ({time.perf_counter() - t0:.1f} s)")
    if not args.no_check:
        t0 = time.perf_counter()
        check = sampled_window_check(dom, params, lambda: lbm.Context(geo, params), geo_oracle,
                                     nsteps=CHECK_STEPS, nwin=16)
        torch.cuda.empty_cache()
        log(f"sampled-window FP32 vs FP64 rel L2 after {CHECK_STEPS} steps: {check:.3e} "
            f"({time.perf_counter() - t0:.1f} s)")

    if args.copy_probe:
        a = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 3 x copy of 2 GiB (2 GiB read + 2 GiB written per launch)")
        del a, b
        torch.cuda.empty_cache()

    ctx = lbm.Context(geo, params)
    if args.launch:
        blk, fl = (int(v) for v in args.launch.split(","))
        ctx.set_launch(blk, fl)
    elif not args.no_autotune:
        log("autotuned launch (block, flags):", ctx.autotune(10))
    block, flags = ctx.get_launch()
    stream = ctx.stream
    ctx.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    mass, mom = ctx.totals()
    log(f"timed {args.steps} steps: {ms:.1f} ms; mass sum {mass:.3e}; momentum x {mom[0]:.4e}")

    alg = algorithmic_bytes(n_fluid, n_cells, n_links)
    achieved = alg / (ms_per_step * 1e-3) / 1e9
    mlups = n_cells / (ms_per_step * 1e-3) / 1e6
    mflups = n_fluid / (ms_per_step * 1e-3) / 1e6
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"sweep_{params.layout}_512x256x1024_traffic.json")
    if os.path.exists(tf):
        with open(tf) as f:
            tr = json.load(f)
        # counted bytes apply only to the same kernel sources and launch shape
        if tr.get("kernel_source_hash") == _sweep_hash() and tr.get("launch") == f"{block},{flags}":
            traffic = tr.get("bytes_per_launch")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(dom, params, geo_oracle, 480, 64)
        log("cpu baseline:", cpu)
    closure = None
    if not args.no_closure:
        del ctx
        torch.cuda.empty_cache()
        try:
            closure = closure_half()
        except Exception as e:  # the sweep's line is still printed, with the failure named
            closure = {"error": f"{type(e).__name__}: {e}"}
        log("closure:", closure)

    out = {
        "metric": "MLUPS + HBM GB/s (% peak) at stated FP32 error; closure vs pore-scale speed/err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "coupled channel over sphere bed 512x256x1024, radii U[8,16], "
                               f"bed porosity 0.45, TRT Lambda 3/16 tau 0.7, force 5e-7, CLI, {params.layout}, "
                               "FP32 shifted",
                   "nx": dom.nx, "ny": dom.ny, "nz": dom.nz, "cells": n_cells, "fluid_cells": n_fluid,
                   "links": n_links, "layout": params.layout, "layout_autotuner": layout_tuned,
                   "block": block, "launch_flags": flags},
        "mflups": round(mflups, 1),
        "effective_gbs": round(achieved, 1),
        "fp32_rel_l2_vs_fp64_oracle": check,
        "fp32_check": f"sampled windows, {CHECK_STEPS} steps from rest (short horizon)" if check is not None else None,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg,
                     # counted bytes (read and write requests by size at the L2-fabric interface)
                     # over this run's time per launch
                     "traffic_gbs": round(traffic / (ms_per_step * 1e-3) / 1e9, 1) if traffic else None},
        "cpu_baseline": cpu,
        "closure": closure,
    }
    print(json.dumps(out), flush=True)


def closure_half():
    """The closure half of the metric, measured after the sweep: the learned
    closure's whole experiment at the coupled-bed shape (128x64x256 beds,
    radii U[6,10], nine training beds, three held-out beds of porosities and
    packings never trained on; REV data, BF16 training and evaluation all on
    this GPU).  Per held-out bed: relative L2 error of the gray column's U(z)
    against the averaged pore-scale U(z), the same for the nu_eff = nu/eps
    reference model, and the cost ratio (pore-scale GPU time to steady state
    over closure inference plus gray column to the same tolerance)."""
    from paper_1507_06565_amd import closure as CL

    t0 = time.perf_counter()
    s = CL.Setup()
    res = CL.experiment(s)
    rows = [{"porosity": r["porosity"], "seed": r["seed"], "learned_err": round(r["learned_err"], 5),
             "nu_over_eps_err": round(r["baseline_nu_over_eps_err"], 5), "cost_ratio": round(r["cost_ratio"], 1),
             "pore_scale_s": round(r["pore_scale_seconds"], 3),
             "gray_plus_mlp_s": round(r["gray_seconds"] + r["mlp_seconds"], 4)} for r in res["held_out"]]
    worst = max(r["learned_err"] for r in rows)
    cheapest = min(r["cost_ratio"] for r in rows)
    return {"workload": f"beds {s.nx}x{s.ny}x{s.nz}, bed layers [1,{s.bed_top}), radii U[{s.r_range[0]:g},"
                        f"{s.r_range[1]:g}], tau {s.tau:g}, force {s.force:g}, {len(s.train)} training and "
                        f"{len(s.test)} held-out beds",
            "held_out": rows, "max_learned_err": worst, "min_cost_ratio": cheapest,
            "criterion": "learned error <= 0.02 at cost ratio >= 50", "met": bool(worst <= 0.02 and cheapest >= 50.0),
            "seconds": round(time.perf_counter() - t0, 1)}


def _sweep_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("sweep.hip", "cell.hpp", "internal.hpp", "lattice.hpp"):
        with open(os.path.join(ROOT, "paper_1507_06565_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
