#!/usr/bin/env python3
"""Throughput of the optimized Schwarz time loop on one MI355X.

Default workload (the largest configuration that fits one GPU): the rotating
GPE solved in the rotating frame (Section 5.2.1), V = -(x^2 + 1.2 y^2)/2,
f(u) = -500|u|^2, c = 1/2 on (-16,16)^2 with 2048 x 2048 cells (4,198,401
nodes), 64 uneven x-strips, Robin p = 5, dt = 5e-4, a vortex Gaussian u0,
preconditioned algorithm with GMRES on P = I - L_h, complex-FP32 factors
with FP64 refinement.  The step potential W_n changes every step, so every
step refactors all strip lines before its Schwarz iterations.  Synthetic,
seeded inputs.

A "step" is one time step: factor(W_n) plus the stationary nonlinear
problem of the step, solved by preconditioned Schwarz iterations (strip
fixed points: residual stencil + block-tridiagonal substitution, then GMRES
on the interface).  The timed region covers --steps steps with the inputs
resident in HBM; L_h is built once at setup (outside, its time reported).

Printed: one JSON line with dof-steps/s, iterations, the roofline of the
dominant kernel (the factor's sweep update on the matrix cores, live HIP
event timing of every launch in the timed region), the strip solve's HBM
roofline, the plain FP64 GPU path over the first steps (with the relative
L2 difference of the two), the first step checked against the discrete
equation the FP64 oracle solves, and the oracle's throughput on a bounded
sample of the same workload.  Other workloads: --workload gpe512 | batch64 |
learned1024 | paper-e5 | paper-e6.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dof-steps/s at 1e-10 rel L2 vs FP64 oracle; Schwarz/GMRES iters per step"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_FP64_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch), each scaled by the counter's reading for a 1 GiB device copy in
# the same run (fetch x2.0, write x1.0).  A record holds only while the
# source files of its kernel hash to source_sha256: any edit to them turns the
# reported traffic back to null until the counters are taken again.
TRAFFIC = {
    ("rot2048", "c32", "sweep_update"): {
        "bytes": 4.0256e+09,
        "source_sha256": "0188a515ae068128f803335738cdd412be490495c3eb45af7f1614408e1640bd",
        "summary": "profiles/sweep_update_c32_rot2048_hbm_counters.md"},
    ("rot2048", "c32", "ysolve"): {
        "bytes": 3.0766e+09,
        "source_sha256": "714329e0631c309012d2a5008703b3df51364cde2008881c307a75fbfab17483",
        "summary": "profiles/ysolve_yfactor_c32_rot2048_hbm_counters.md"},
    ("rot2048", "c32", "yfactor"): {
        "bytes": 1.8161e+09,
        "source_sha256": "714329e0631c309012d2a5008703b3df51364cde2008881c307a75fbfab17483",
        "summary": "profiles/ysolve_yfactor_c32_rot2048_hbm_counters.md"},
}

TRAFFIC_SOURCES = {"strip_solve": "kernels_solve.hip", "sweep_update": "kernels_factor.hip",
                   "ysolve": "kernels_yorder.hip", "yfactor": "kernels_yorder.hip"}


def kernel_source_sha256(kernel):
    """sha256 over the kernel's source file and the device part of the
    shared header (its text before the launcher declarations)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1603_05110_amd", "csrc")
    try:
        with open(os.path.join(csrc, TRAFFIC_SOURCES[kernel]), "rb") as fh:
            src = fh.read()
        with open(os.path.join(csrc, "osm_internal.h"), "rb") as fh:
            hdr = fh.read()
    except OSError:
        return None
    cut = hdr.find(b"// ---------------------------------------------------------------- launchers")
    if cut < 0:
        return None
    return hashlib.sha256(src + hdr[:cut]).hexdigest()


def measured_traffic(workload, prec, kernel, shape=None):
    """Counted HBM bytes per launch, or None when no record matches the
    current sources (and, for the strip solve, the tile shape the
    autotuner picked)."""
    rec = TRAFFIC.get((workload, prec, kernel))
    if rec is None or kernel_source_sha256(kernel) != rec["source_sha256"]:
        return None
    if shape is not None and rec.get("shape") not in (None, shape):
        return None
    return rec["bytes"]


def solver_opts(prec):
    return dict(algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True, max_k=500,
                tol_q=1e-13, max_q=200, warm_start=True, tol_gmres=3e-2,
                gmres_restart=50, max_gmres=2000, eta_q=3e-2, q_estimate=1)


def run_gpu(pb, u0, V, prec, steps, warmup, dev, measure=True, **extra):
    import torch
    from paper_1603_05110_amd import osm
    t = time.perf_counter()
    s = osm.OsmSolver(pb, dev, **solver_opts(prec), **extra)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    W = torch.from_numpy(V).to(dev)
    u = torch.from_numpy(u0).to(dev)
    if warmup > 0:
        s.factor(W)
        for _ in range(warmup):
            s.step(u)
    torch.cuda.synchronize()
    if measure:
        s.kernel_timing(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.factor(W)
    t_fac = time.perf_counter() - t0
    for _ in range(steps):
        stats.append(s.step(u))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = s.kernel_timing(False) if measure else (0.0, 0)
    work = s.kernel_work() if measure else 0.0
    team = s.solve_team()
    shape = s.solve_shape()
    order = s.strip_order()
    s.close()
    return dict(seconds=t1 - t0, factor_s=t_fac, setup_s=t_setup, stats=stats, u=u,
                solve_ms=kern[0], solve_launches=kern[1], solve_work=work, team=team, shape=shape,
                order=order)


def profile_solve(pb, V, prec, launches, dev, team=0, solve_shape=0):
    """Kernel-level measurement mode for profilers: factor once, then run
    `launches` strip solves on a seeded right-hand side, then one
    device-to-device copy of 1 GiB (the calibration kernel for the HBM byte
    counters: its algorithmic traffic is 1 GiB read + 1 GiB written)."""
    import torch
    from paper_1603_05110_amd import osm
    s = osm.OsmSolver(pb, dev, **dict(solver_opts(prec), team=team, solve_shape=solve_shape))
    s.factor(torch.from_numpy(V).to(dev))
    gen = torch.Generator(device="cpu").manual_seed(1603)
    b = torch.randn((s.lt, s.ny), dtype=torch.complex128, generator=gen).to(dev)
    s.strip_solve(b)
    torch.cuda.synchronize()
    s.kernel_timing(True)
    for _ in range(launches):
        s.strip_solve(b)
    torch.cuda.synchronize()
    ms, n = s.kernel_timing(False)
    nbytes = s.kernel_work() / max(n, 1)
    team, shape = s.solve_team(), s.solve_shape()
    s.close()
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    avg = ms / max(n, 1)
    print(json.dumps({"mode": "profile-solve", "prec": prec, "launches": n, "avg_launch_ms": avg,
                      "bytes_per_launch": nbytes, "achieved_GBs": nbytes / (avg * 1e-3) / 1e9,
                      "workgroups_per_strip": team, "tile_shape": shape,
                      "source_sha256": kernel_source_sha256("strip_solve"),
                      "copy_bytes": 2 * src.numel() * 8}),
          flush=True)


def run_batch(args, dev):
    """Batch of 64 independent cubic-NLS instances (grids 256..768 squared,
    8-32 uneven strips, seeded p and potentials), classical algorithm.  The
    timed region is the refactorisation of every instance plus K steps, each
    step replaying the captured graph of a chunk of Schwarz iterations; the
    solve roofline comes from one more step run launch by launch with HIP
    events around every batched solve.  Beside it (--sequential, on by
    default): the same instances run one by one on the single-instance path,
    complex FP32 and FP64, with the same timed work."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import osm
    from workloads import c3

    wl = c3()
    pbs = wl.problems
    dofs = [(pb.ncx + 1) * (pb.ncy + 1) for pb in pbs]
    dof = sum(dofs)
    opts = dict(prec=args.prec, tol_k=1e-12, tol_k_relative=True, tol_q=1e-13, max_k=5000,
                max_q=200, algo=args.batch_algo)
    if args.batch_algo == "precond":
        opts.update(tol_gmres=3e-2, gmres_restart=50, max_gmres=2000)
    print(f"bench: C3 batch {len(pbs)} instances, {dof} dofs, prec={args.prec}, "
          f"{args.batch_algo}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    b = osm.OsmBatch(pbs, dev, **opts)
    Ws = [torch.from_numpy(V).to(dev) for V in wl.V]
    us = [torch.from_numpy(u).to(dev) for u in wl.u0]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    b.factor(Ws)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t
    tuning = b.tuning()
    for _ in range(args.warmup):
        b.step(us)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    b.factor(Ws)
    for n in range(args.steps):
        stats.append(b.step(us))
        print(f"bench: step {n}: k max {max(s['k'] for s in stats[-1])}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = dof * args.steps / T
    b.kernel_timing(True)
    b.step(us)
    ms, launches = b.kernel_timing(False)
    nbytes = b.kernel_work()
    b.close()
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    print(f"bench: C3 {value:.4g} dof-steps/s, solve {achieved:.0f} GB/s", file=sys.stderr,
          flush=True)
    ks = np.array([[s["k"] for s in st] for st in stats])
    qs = np.array([[s["q_total"] for s in st] for st in stats])
    # the same instances one by one on the single-instance path, with the
    # same options and the same timed work (factor + steps), in both
    # precisions; the first factorisation of each (with its solve autotune)
    # is outside the timed region, as the batch's is
    sequential = {}
    if args.sequential:
        del us
        torch.cuda.empty_cache()
        for prec in ("c32", "fp64"):
            t_run, t_first, kk, gm = 0.0, 0.0, [], []
            for i, pb in enumerate(pbs):
                ta = time.perf_counter()
                s1 = osm.OsmSolver(pb, dev, **dict(opts, prec=prec))
                u1 = torch.from_numpy(wl.u0[i]).to(dev)
                s1.factor(Ws[i])
                torch.cuda.synchronize()
                tb = time.perf_counter()
                s1.factor(Ws[i])
                for _ in range(args.steps):
                    kk.append(s1.step(u1)["k"])
                torch.cuda.synchronize()
                tc = time.perf_counter()
                s1.close()
                t_first += tb - ta
                t_run += tc - tb
                del u1
            sequential[prec] = {"value": dof * args.steps / t_run,
                                "ms_per_step": 1e3 * t_run / args.steps,
                                "setup_and_first_factor_s": t_first,
                                "k_mean": float(np.mean(kk)), "k_max": int(np.max(kk))}
            print(f"bench: one by one, {prec}: {sequential[prec]['value']:.4g} dof-steps/s",
                  file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle.step import MonolithicStepper
        small = sorted(range(len(pbs)), key=lambda i: dofs[i])[:2]
        work = 0.0
        dsum = 0
        with threadpool_limits(1):
            for i in small:
                t0 = time.perf_counter()
                ost = MonolithicStepper(pbs[i], wl.V[i], form="B", tol_q=1e-14)
                tf = time.perf_counter() - t0
                t1 = time.perf_counter()
                ost.step(np.array(wl.u0[i], dtype=complex))
                ts = time.perf_counter() - t1
                work += tf + args.steps * ts
                dsum += dofs[i]
        cpu = {"value": dsum * args.steps / work, "unit": "dof-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": (f"FP64 monolithic oracle (SciPy splu, form B) on the 2 smallest "
                          f"instances ({dsum} dofs): factor + 1 step each, extrapolated to "
                          f"{args.steps} steps; larger instances would be slower per dof")}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "dof-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64-refine" if args.prec == "c32" else "c128",
        "data": "synthetic",
        "config": {"workload": "batch of 64 independent cubic-NLS instances, grids "
                               "{256,384,512,768}^2 seeded, 8-32 uneven strips, Robin p~U[1,10], "
                               f"V = 8 seeded Gaussians (max|V|=5), dt=0.01, {args.batch_algo}, "
                               "graph-replayed chunks, autotuned solve tiles",
                   "dof": dof, "instances": len(pbs), "strips": sum(pb.nsub for pb in pbs),
                   "algo": args.batch_algo, "prec": args.prec, "timed": "factor(W) + steps"},
        "iters": {"k_mean": float(ks.mean()), "k_max": int(ks.max()),
                  "q_total": int(qs.sum()),
                  "gmres_total": int(sum(x["gmres_total"] for st in stats for x in st))},
        "roofline": {"kernel": "batch_solve", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_timed": nbytes, "launches": launches,
                     "avg_launch_ms": ms / max(launches, 1),
                     "measured_on": "one extra step, launch by launch"},
        "tuning": tuning,
        "setup_s": t_setup,
        "first_factor_and_autotune_s": t_tune,
        "one_by_one": sequential or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_learned(args, dev):
    """Learned interface guess: interface traces from seeded runs of the GPE
    family V = -(x^2+y^2)/(2 w^2), w ~ U[0.5, 2], beta ~ -U[10, 200]
    (512^2 cells, 16 strips, 200 steps each), the network trained on them by
    the library's kernels, then a held-out 1024^2-cell, 32-strip member run
    from the previous converged vector (the paper's start), from linear
    extrapolation and from the learned prediction."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import learned, osm
    from workloads import c4, c4_family, net_init, rng_for

    opts = dict(solver_opts("c32"), strip_order=args.strip_order, lh_form=args.lh_form)
    t0 = time.perf_counter()
    Xs, Ts = [], []
    rng = rng_for(4, salt=1)
    for r in range(args.train_runs):
        pb, u0, V = c4_family(rng, ncells=512, nsub=16, steps=200)
        s = osm.OsmSolver(pb, dev, **opts)
        s.factor(torch.from_numpy(V).to(dev))
        X, T, _ = learned.collect_traces(s, torch.from_numpy(u0).to(dev), pb.steps)
        s.close()
        Xs.append(X)
        Ts.append(T)
        print(f"bench: training run {r}: {pb.name}, {X.shape[0]} traces", file=sys.stderr, flush=True)
    X, T = torch.cat(Xs), torch.cat(Ts)
    del Xs, Ts
    t_data = time.perf_counter() - t0
    net = osm.OsmNet(args.batch, dev)
    net.set_params(torch.from_numpy(net_init(0)))
    t0 = time.perf_counter()
    losses = learned.train(net, X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=0,
                           log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ntr = int(X.shape[0])
    del X, T
    wl = c4(steps=args.steps)
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    runs = {}
    for name, guess in [("previous", 0), ("extrapolated", 3), ("learned", 2)]:
        s = osm.OsmSolver(pb, dev, **dict(opts, guess=guess))
        if guess == 2:
            s.set_guess_net(net)
        Wd = torch.from_numpy(V).to(dev)
        u = torch.from_numpy(u0).to(dev)
        s.factor(Wd)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        s.factor(Wd)
        st = [s.step(u) for _ in range(args.steps)]
        torch.cuda.synchronize()
        T_run = time.perf_counter() - ta
        s.close()
        runs[name] = {"value": dof * args.steps / T_run, "ms_per_step": 1e3 * T_run / args.steps,
                      "k_total": int(sum(x["k"] for x in st)),
                      "k_after_step2": int(sum(x["k"] for x in st[2:])),
                      "q_total": int(sum(x["q_total"] for x in st)),
                      "gmres_total": int(sum(x["gmres_total"] for x in st)),
                      "fallbacks": int(sum(x["fallback_used"] > 0 for x in st)),
                      "restarts": int(sum(x["fallback_used"] == 2 for x in st)),
                      # ||g_n - prediction|| / ||g_n - g_{n-1}|| over the steps that
                      # formed a prediction (the fallback's judge)
                      "guess_ratio": ({"mean": float(np.mean(gr)), "median": float(np.median(gr)),
                                       "steps": len(gr)}
                                      if (gr := [x["guess_ratio"] for x in st
                                                 if x["guess_ratio"] > 0]) else None),
                      "u": u.cpu().numpy()}
        print(f"bench: {name}: {runs[name]['value']:.4g} dof-steps/s, k {runs[name]['k_total']}, "
              f"gmres {runs[name]['gmres_total']}, guess ratio {runs[name]['guess_ratio']}",
              file=sys.stderr, flush=True)
    ref = runs["previous"].pop("u")
    for name in ("extrapolated", "learned"):
        u = runs[name].pop("u")
        runs[name]["rel_l2_vs_previous_start"] = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    net.close()
    out = {
        "metric": METRIC,
        "value": runs["learned"]["value"],
        "unit": "dof-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 0,
        "ms_per_step": runs["learned"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64-refine; network bf16/f32",
        "data": "synthetic",
        "config": {"workload": "learned interface guess: GPE family V=-(x^2+y^2)/(2w^2), "
                               "w~U[0.5,2], beta~-U[10,200]; inference on (-8,8)^2, 1024^2 cells, "
                               "32 strips, p=5, dt=1e-3, preconditioned",
                   "dof": dof, "strips": pb.nsub, "training_traces": ntr,
                   "training_runs": args.train_runs, "epochs": args.epochs,
                   "timed": "factor(W) + steps, per start"},
        "starts": runs,
        "training": {"data_s": t_data, "train_s": t_train, "loss_first": losses[0],
                     "loss_last": losses[-1]},
    }
    print(json.dumps(out), flush=True)


def cpu_sample_rotating(pb, W1, u0, k_per_step, nsample=40):
    """The FP64 oracle's throughput estimated on a bounded sample of the same
    workload: the first `nsample` strips of the rotating problem cut out as a
    domain of their own (same mesh size, potential and initial data), the
    sequential Schwarz oracle (form B) set up on them (one sparse LU per
    strip) and one Schwarz map evaluated (every strip's fixed point to
    1e-13).  Scaled by (strips / nsample) and by the GPU's Schwarz iterations
    per step; the oracle's L_h build and GMRES are not counted, so this
    overstates the oracle's rate."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.schwarz import SchwarzOracle
    nsample = min(nsample, pb.nsub)
    cells = list(pb.strip_cells[:nsample])
    ncx = sum(cells)
    sub = pb.replace(ncx=ncx, nsub=nsample, strip_cells=cells, xr=pb.xl + pb.hx * ncx)
    Wsub = np.ascontiguousarray(W1[:ncx + 1])
    usub = np.ascontiguousarray(u0[:ncx + 1])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        orc = SchwarzOracle(sub, Wsub, form="B", tol_q=1e-13)
        t_fac = time.perf_counter() - t0
        g0 = np.zeros((2 * (nsample - 1), pb.ncy + 1), complex)
        t1 = time.perf_counter()
        orc.R(g0, usub)
        t_map = time.perf_counter() - t1
    scale = pb.nsub / nsample
    per_step = scale * (t_fac + k_per_step * t_map)
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    return {"value": dof / per_step, "unit": "dof-steps/s", "cores": 1, "kind": "oracle",
            "host_nproc": os.cpu_count(),
            "sample": (f"FP64 sequential Schwarz oracle (form B) on {nsample} of the {pb.nsub} "
                       f"strips of this workload ({(ncx + 1) * (pb.ncy + 1)} nodes): strip LUs "
                       f"{t_fac:.1f}s + one Schwarz map {t_map:.1f}s, scaled by "
                       f"{pb.nsub}/{nsample} strips and {k_per_step:.1f} Schwarz iterations per "
                       f"step (the GPU's); L_h build and GMRES not counted"),
            "seconds": t_fac + t_map}


def profile_factor(pb, args, dev):
    """Profiler mode of the rotating workload: setup with the classical
    algorithm (the factor and the strip solve do not depend on the
    algorithm; it skips the L_h build), the first factorisation, then
    --profile-factor refactorisations of the rotating problem
    (osm_factor_rotating), then --profile-solves strip solves of a seeded
    right-hand side, then one 1 GiB device-to-device copy (the calibration
    kernel of the HBM byte counters).  --team and --solve-shape fix the
    solve's team and tile shape; with both given no solve runs before the
    timed ones (no autotuning)."""
    import torch
    from paper_1603_05110_amd import osm
    opts = dict(solver_opts(args.prec), algo="classical", team=args.team,
                solve_shape=args.solve_shape, strip_order=args.strip_order)
    s = osm.OsmSolver(pb, dev, **opts)
    s.factor_rotating(1)
    torch.cuda.synchronize()
    s.kernel_timing(True)
    for n in range(2, 2 + args.profile_factor):
        s.factor_rotating(n)
    torch.cuda.synchronize()
    s.kernel_timing(False)
    ms, n, fl = s.factor_timing()
    order = s.strip_order()
    solve = None
    if args.profile_solves > 0:
        gen = torch.Generator(device="cpu").manual_seed(1603)
        b = torch.randn((s.lt, s.ny), dtype=torch.complex128, generator=gen).to(dev)
        torch.cuda.synchronize()
        s.kernel_timing(True)
        for _ in range(args.profile_solves):
            s.strip_solve(b)
        torch.cuda.synchronize()
        sms, sn = s.kernel_timing(False)
        nbytes = s.kernel_work() / max(sn, 1)
        savg = sms / max(sn, 1)
        solve = {"launches": sn, "avg_launch_ms": savg, "bytes_per_launch": nbytes,
                 "achieved_GBs": nbytes / (savg * 1e-3) / 1e9 if savg > 0 else 0.0,
                 "workgroups_per_strip": s.solve_team(), "tile_shape": s.solve_shape(),
                 "source_sha256": kernel_source_sha256("ysolve" if order == "y"
                                                       else "strip_solve")}
    s.close()
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "profile-factor", "prec": args.prec, "factors": args.profile_factor,
                      "strip_order": order,
                      "update_launches": n, "update_avg_ms": ms / max(n, 1),
                      "update_tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0,
                      "update_flops": fl,
                      "update_source_sha256": kernel_source_sha256("yfactor" if order == "y"
                                                                   else "sweep_update"),
                      "solve": solve, "copy_bytes": 2 * src.numel() * 8}), flush=True)


def rot_leg(pb, u0, opts, steps, warmup, dev, ncmp=0, keep_first=False, label="main"):
    """One timed run of the rotating workload: setup, first factorisation
    (with the autotuners), --warmup untimed steps, then `steps` timed steps
    of factor(W_n) + step, with HIP-event timing of the factor and solve
    kernels.  Returns the rates, the kernel statistics and the states after
    step 1 and step ncmp (when asked)."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import osm
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    t = time.perf_counter()
    s = osm.OsmSolver(pb, dev, **opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    u = torch.from_numpy(u0).to(dev)
    t = time.perf_counter()
    s.factor_rotating(1)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t
    order = s.strip_order()
    print(f"bench[{label}]: setup {t_setup:.1f}s, first factor + autotune {t_first:.1f}s, "
          f"strip order {order}", file=sys.stderr, flush=True)
    if warmup > 0:
        uw = u.clone()
        for n in range(1, warmup + 1):
            s.factor_rotating(n)
            s.step(uw)
        del uw
    torch.cuda.synchronize()
    s.kernel_timing(True)
    stats, t_fac = [], 0.0
    u_first = u_cmp = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, steps + 1):
        ta = time.perf_counter()
        s.factor_rotating(n)
        torch.cuda.synchronize()
        t_fac += time.perf_counter() - ta
        stats.append(s.step(u))
        if n == 1 and keep_first:
            u_first = u.clone()
        if n == ncmp:
            u_cmp = u.clone()
        print(f"bench[{label}]: step {n}: k {stats[-1]['k']} gmres {stats[-1]['gmres_total']} "
              f"q {stats[-1]['q_total']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    kern = s.kernel_timing(False)
    solve_work = s.kernel_work()
    fac_ms, fac_n, fac_fl = s.factor_timing()
    team, shape = s.solve_team(), s.solve_shape()
    s.close()
    del u
    torch.cuda.empty_cache()
    avg_ms = kern[0] / max(kern[1], 1)
    nbytes = solve_work / max(kern[1], 1)
    out = {"order": order, "value": dof * steps / T, "T": T, "ms_per_step": 1e3 * T / steps,
           "factor_s_per_step": t_fac / steps, "setup_s": t_setup, "first_s": t_first,
           "stats": stats,
           "solve": {"launches": kern[1], "avg_launch_ms": avg_ms, "bytes_per_launch": nbytes,
                     "ms_per_step": kern[0] / steps,
                     "achieved_GBs": nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0,
                     "workgroups_per_strip": team, "tile_shape": shape},
           "factor": {"launches": fac_n, "avg_launch_ms": fac_ms / max(fac_n, 1),
                      "ms_per_step": fac_ms / steps, "flops_timed": fac_fl,
                      "tflops": fac_fl / (fac_ms * 1e-3) / 1e12 if fac_ms > 0 else 0.0},
           "u_first": u_first, "u_cmp": u_cmp}
    print(f"bench[{label}]: {T:.2f}s for {steps} steps ({t_fac:.2f}s factor), "
          f"{out['value']:.4g} dof-steps/s", file=sys.stderr, flush=True)
    return out


def iters_of(stats):
    import numpy as np
    return {"k_mean": float(np.mean([x["k"] for x in stats])),
            "k_max": int(np.max([x["k"] for x in stats])),
            "q_total": int(sum(x["q_total"] for x in stats)),
            "gmres_total": int(sum(x["gmres_total"] for x in stats))}


def run_rotating(args, dev):
    """Rotating GPE at full size (2048^2 cells, 64 uneven strips), solved in
    the rotating frame: the step potential changes every step, so every step
    refactors every strip (osm_factor_rotating) before its Schwarz
    iterations.  A truncated horizon of --steps steps is timed (the full
    1000-step horizon is the same work repeated).  The strip order is the
    autotuner's choice (--strip-order tuned): the y-line order's factor and
    solve are FP64.  Beside it: the node-line order (ny x ny blocks, complex
    FP32 + refinement) over --node-steps steps, the plain FP64 node-line
    path over the first --fp64-steps steps (with the relative L2 difference
    of the two), the first step checked against the discrete equation the
    FP64 oracle solves, and the oracle's rate on a bounded sample of the same
    workload."""
    import numpy as np
    import torch

    from workloads import c5

    wl = c5(steps=args.steps)
    pb, u0 = wl.problems[0], wl.u0[0]
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    if args.profile_factor > 0:
        profile_factor(pb, args, dev)
        return
    print(f"bench: {pb.name} dof={dof} prec={args.prec} steps={args.steps} "
          f"strip order {args.strip_order}", file=sys.stderr, flush=True)
    ncmp = min(args.fp64_steps, args.steps) if args.fp64_steps > 0 else 0
    opts = dict(solver_opts(args.prec), strip_order=args.strip_order,
                lh_form=args.lh_form)
    main = rot_leg(pb, u0, opts, args.steps, args.warmup, dev, ncmp=ncmp,
                   keep_first=not args.no_cpu_baseline)
    order = main["order"]

    # the node-line order (ny x ny blocks on the matrix cores), the other
    # choice of the strip order
    node = None
    if order != "node" and args.node_steps > 0:
        nl = rot_leg(pb, u0, dict(solver_opts(args.prec), strip_order="node",
                                  lh_form=args.lh_form), args.node_steps, 1, dev, label="node")
        upd_t = nl["factor"]["tflops"]
        node = {"value": nl["value"], "steps": args.node_steps, "ms_per_step": nl["ms_per_step"],
                "factor_s_per_step": nl["factor_s_per_step"], "iters": iters_of(nl["stats"]),
                "prec": args.prec,
                "sweep_update": {"bound": "mfma", "achieved": upd_t, "unit": "TFLOP/s",
                                 "peak": MFMA_FP32_PEAK_TFLOPS if args.prec == "c32"
                                 else MFMA_FP64_PEAK_TFLOPS,
                                 "avg_launch_ms": nl["factor"]["avg_launch_ms"],
                                 "launches": nl["factor"]["launches"],
                                 "traffic": measured_traffic("rot2048", args.prec,
                                                             "sweep_update")},
                "solve": dict(nl["solve"], bound="hbm", peak=HBM_PEAK_GBS,
                              traffic=measured_traffic("rot2048", args.prec, "strip_solve",
                                                       nl["solve"]["tile_shape"]))}

    # the plain FP64 node-line path over the first ncmp steps, from the same u0
    fp64 = None
    if ncmp > 0 and (args.prec != "fp64" or order != "node"):
        lg = rot_leg(pb, u0, dict(solver_opts("fp64"), strip_order="node",
                                  lh_form=args.lh_form), ncmp, 0, dev, ncmp=ncmp, label="fp64")
        diff = float(torch.linalg.vector_norm(main["u_cmp"] - lg["u_cmp"]) /
                     torch.linalg.vector_norm(lg["u_cmp"]))
        fp64 = {"value": lg["value"], "steps": ncmp, "ms_per_step": lg["ms_per_step"],
                "setup_s": lg["setup_s"], "k": [x["k"] for x in lg["stats"]],
                "rel_l2_vs_main": diff,
                "note": "node-line order, FP64 factor and solve; same steps from the same u0; "
                        "factor(W_n) inside the timed steps"}
        print(f"bench: fp64 node-line {fp64['value']:.4g} dof-steps/s; main vs fp64 after "
              f"{ncmp} steps {diff:.3e}", file=sys.stderr, flush=True)
        del lg
    main["u_cmp"] = None
    torch.cuda.empty_cache()

    check, cpu = None, None
    if not args.no_cpu_baseline:
        from oracle.fem import StripMatrices, weighted_mass_2d
        from oracle.rotating import step_potential
        u1 = main["u_first"].cpu().numpy()
        main["u_first"] = None
        W1 = step_potential(pb, 1)
        mats = StripMatrices(pb.ncx, pb.ncy, pb.hx, pb.hy)
        K = mats.operator(W1, pb.dt, pb.lap_coef, pb.p_bc, pb.p_bc)
        v = 0.5 * (u0 + u1).ravel()
        F = (2j / pb.dt) * (mats.M @ u0.ravel())
        r = K @ v + weighted_mass_2d((pb.beta * np.abs(v) ** 2).reshape(u0.shape), pb.hx,
                                     pb.hy) @ v - F
        check = {"step": 1, "rel_residual_discrete_equation": float(np.linalg.norm(r) / np.linalg.norm(F)),
                 "bound": 2.5e-11}
        del K, r, v, F, mats
        print(f"bench: step-1 residual {check['rel_residual_discrete_equation']:.3e}",
              file=sys.stderr, flush=True)
        kps = float(np.mean([x["k"] for x in main["stats"]]))
        cpu = cpu_sample_rotating(pb, W1, u0, kps)
        print(f"bench: oracle {cpu['value']:.4g} dof-steps/s ({cpu['seconds']:.1f}s sampled)",
              file=sys.stderr, flush=True)

    sv, fc = main["solve"], main["factor"]
    if order == "y":
        # the y-line order: FP64 factor (ALU, latency-bound chains), inverses
        # stored as prec says, solve in FP64
        solve_obj = {"kernel": "ysolve (forward, middle, backward)", "bound": "hbm",
                     "achieved": sv["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sv["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic("rot2048", args.prec, "ysolve"),
                     "bytes_per_launch": sv["bytes_per_launch"],
                     "avg_launch_ms": sv["avg_launch_ms"], "launches": sv["launches"],
                     "ms_per_step": sv["ms_per_step"]}
        factor_obj = {"kernel": "yfactor (halves, middle)", "bound": "alu",
                      "achieved": fc["tflops"], "peak": FP64_VALU_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": fc["tflops"] / FP64_VALU_PEAK_TFLOPS,
                      "traffic": measured_traffic("rot2048", args.prec, "yfactor"),
                      "flops_timed": fc["flops_timed"], "avg_launch_ms": fc["avg_launch_ms"],
                      "launches": fc["launches"], "ms_per_step": fc["ms_per_step"],
                      "note": "algorithmic flops: per y-line 8 (n^3 + 6 n^2) for the "
                              "inversion and the two coupling products"}
        dominant = solve_obj if sv["ms_per_step"] >= fc["ms_per_step"] else factor_obj
        other = factor_obj if dominant is solve_obj else solve_obj
        roofline = dominant
    else:
        roofline = {"kernel": "sweep_update", "bound": "mfma", "achieved": fc["tflops"],
                    "peak": MFMA_FP32_PEAK_TFLOPS if args.prec == "c32" else MFMA_FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s",
                    "frac": fc["tflops"] / (MFMA_FP32_PEAK_TFLOPS if args.prec == "c32"
                                            else MFMA_FP64_PEAK_TFLOPS),
                    "traffic": measured_traffic("rot2048", args.prec, "sweep_update"),
                    "flops_timed": fc["flops_timed"], "avg_launch_ms": fc["avg_launch_ms"],
                    "launches": fc["launches"],
                    "note": ("algorithmic flops: 8 real flops per complex multiply-add over "
                             "the upper 64x64 tiles each pass updates; the kernel issues 6 "
                             "(three real products)")}
        other = {"kernel": "strip_solve", "bound": "hbm", "achieved": sv["achieved_GBs"],
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sv["achieved_GBs"] / HBM_PEAK_GBS,
                 "traffic": measured_traffic("rot2048", args.prec, "strip_solve",
                                             sv["tile_shape"]),
                 "bytes_per_launch": sv["bytes_per_launch"], "avg_launch_ms": sv["avg_launch_ms"],
                 "launches": sv["launches"], "workgroups_per_strip": sv["workgroups_per_strip"],
                 "tile_shape": sv["tile_shape"]}
    dtype = "c64+f64-refine" if args.prec == "c32" else "c128"
    out = {
        "metric": METRIC,
        "value": main["value"],
        "unit": "dof-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "rotating GPE in the rotating frame, Omega_r=0.7, "
                               "V=-(x^2+1.2y^2)/2, f=-500|u|^2, (-16,16)^2, 2048^2 cells, "
                               "64 uneven strips, p=5, dt=5e-4, vortex Gaussian, preconditioned, "
                               "refactor every step",
                   "dof": dof, "strips": pb.nsub, "algo": "precond", "prec": args.prec,
                   "strip_order": order, "strip_order_option": args.strip_order,
                   "lh_form": args.lh_form,
                   "timed": "per step: factor(W_n) + Schwarz/GMRES",
                   "horizon": f"{args.steps} of 1000 steps"},
        "iters": iters_of(main["stats"]),
        "roofline": roofline,
        "other_kernel": other,
        "factor": {"s_per_step": main["factor_s_per_step"]},
        "setup_s": main["setup_s"],
        "first_factor_and_autotune_s": main["first_s"],
        "node_line_order": node,
        "fp64_gpu": fp64,
        "check": check,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# Section 5.1.3, Table Influence_p_NL_2_32: first-step iterations on the
# first mesh, {p: (N=2 zero cls, pd, random cls, pd, N=32 zero cls, pd,
# random cls, pd)}
PAPER_E5 = {5: (57, 6, 548, 6, 57, 6, 582, 6), 10: (35, 6, 297, 6, 35, 6, 316, 6),
            15: (32, 6, 227, 6, 33, 6, 241, 6), 20: (36, 6, 200, 6, 36, 6, 212, 6),
            25: (41, 6, 189, 6, 41, 6, 200, 6), 30: (46, 6, 186, 6, 47, 6, 200, 6),
            35: (53, 6, 188, 6, 53, 6, 204, 6), 40: (59, 6, 194, 6, 60, 6, 211, 6),
            45: (66, 6, 208, 6, 66, 6, 223, 6), 50: (73, 6, 216, 6, 73, 6, 234, 6)}

# Section 5.2.2, Table time_dx32, Robin p = 180: hours for T = 0.1 (1000
# steps) on 92 x 16 Sandy Bridge cores, one MPI rank per strip
PAPER_E6_HOURS = {"classical": {2: 5.68, 4: 2.66, 8: 1.28, 16: 0.68, 32: 0.33},
                  "precond": {2: 3.49, 4: 1.60, 8: 0.77, 16: 0.44, 32: 0.24}}


def run_paper_e5(args, dev):
    """The paper's Robin p-sweep (Section 5.1.3): the first time step of the
    cubic NLS on the first mesh (4097 x 129 nodes), N = 2 and 32 strips,
    zero and seeded random first interface vectors (SplitMix64, uniform
    real and imaginary parts), classical and preconditioned, with the
    paper's stopping rule (1e-10, absolute).  Prints every iteration count
    beside the printed one."""
    import torch

    from paper_1603_05110_amd import osm
    from workloads import nls_mesh1

    plist = [float(x) for x in args.p_list.split(",")] if args.p_list else sorted(PAPER_E5)
    rows = []
    t_all = time.perf_counter()
    for N in (2, 32):
        for p in plist:
            wl = nls_mesh1(N, p, steps=1)
            pb, u0, W = wl.problems[0], wl.u0[0], wl.V[0]
            paper = PAPER_E5.get(int(p))
            for si, start in enumerate(("zero", "random")):
                for ai, algo in enumerate(("classical", "precond")):
                    s = osm.OsmSolver(pb, dev, algo=algo, prec=args.prec, tol_k=1e-10,
                                      tol_k_relative=False, max_k=5000, tol_q=1e-13,
                                      max_q=200, warm_start=True, tol_gmres=1e-12,
                                      g1_init=1 if start == "random" else 0, seed=1)
                    s.factor(torch.from_numpy(W).to(dev))
                    u = torch.from_numpy(u0).to(dev)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = s.step(u)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    s.close()
                    col = (0 if N == 2 else 4) + 2 * si + ai
                    ref = paper[col] if paper else None
                    rows.append({"N": N, "p": p, "start": start, "algo": algo, "k": st["k"],
                                 "paper_k": ref, "q": st["q_total"],
                                 "gmres": st["gmres_total"], "step_s": dt})
                    print(f"bench: N={N} p={p:g} {start} {algo}: k {st['k']} (paper {ref}), "
                          f"{dt:.2f}s", file=sys.stderr, flush=True)
    ratio = [r["k"] / r["paper_k"] for r in rows if r["paper_k"]]
    dof = 4097 * 129
    out = {"metric": "first-step Schwarz iterations vs the paper's Table Influence_p_NL_2_32",
           "value": float(max(abs(x - 1.0) for x in ratio)) if ratio else None,
           "unit": "max relative deviation of k from the paper", "n_gpus": 1,
           "higher_is_better": False, "dtype": "c64+f64-refine" if args.prec == "c32" else "c128",
           "data": "synthetic",
           "config": {"workload": "paper Section 5.1 mesh 1: cubic NLS, (-16,16)x(-8,8), "
                                  "dx=1/128, dy=1/8, dt=0.01, u0=exp(-x^2-y^2-0.5ix), first step",
                      "dof": dof, "p": plist, "strips": [2, 32]},
           "rows": rows, "seconds": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)


def run_paper_e6(args, dev):
    """The paper's BEC runs with Robin p = 180 (Section 5.2.2, Table
    time_dx32): the rotating GPE on (-16,16)^2 with 1025^2 nodes, N = 2..32
    equal strips, classical and preconditioned, dt = 1e-4, refactored every
    step (rotating frame).  --steps of the 1000-step horizon are timed; the
    paper's hours are converted to dof-steps/s for context (its machine: 92
    nodes of 16 Sandy Bridge cores, one MPI rank per strip)."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import osm
    from workloads import bec_1025

    runs = []
    for algo in ("classical", "precond"):
        for N in (2, 4, 8, 16, 32):
            wl = bec_1025(N, steps=args.steps)
            pb, u0 = wl.problems[0], wl.u0[0]
            dof = (pb.ncx + 1) * (pb.ncy + 1)
            opts = dict(algo=algo, prec=args.prec, tol_k=1e-10, tol_k_relative=False,
                        max_k=5000, tol_q=1e-13, max_q=200, warm_start=True,
                        tol_gmres=3e-2, gmres_restart=50, max_gmres=4000,
                        strip_order=args.strip_order, lh_form=args.lh_form)
            s = osm.OsmSolver(pb, dev, **opts)
            s.factor_rotating(1)
            order = s.strip_order()
            u = torch.from_numpy(u0).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ks = []
            for n in range(1, args.steps + 1):
                s.factor_rotating(n)
                ks.append(s.step(u)["k"])
            torch.cuda.synchronize()
            T = time.perf_counter() - t0
            s.close()
            hours = PAPER_E6_HOURS[algo][N]
            runs.append({"algo": algo, "N": N, "strip_order": order,
                         "value": dof * args.steps / T,
                         "ms_per_step": 1e3 * T / args.steps, "k_mean": float(np.mean(ks)),
                         "k_max": int(np.max(ks)),
                         "paper_hours_T0.1": hours,
                         "paper_dof_steps_per_s": dof * 1000 / (hours * 3600.0)})
            print(f"bench: {algo} N={N} ({order}): {runs[-1]['value']:.4g} dof-steps/s, k mean "
                  f"{runs[-1]['k_mean']:.1f} (paper {runs[-1]['paper_dof_steps_per_s']:.3g})",
                  file=sys.stderr, flush=True)
    best = max(runs, key=lambda r: r["value"])
    out = {"metric": METRIC, "value": best["value"], "unit": "dof-steps/s", "n_gpus": 1,
           "steps": args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": "c64+f64-refine" if args.prec == "c32" else "c128",
           "data": "synthetic",
           "config": {"workload": "paper Section 5.2.2: rotating GPE, (-16,16)^2, 1024^2 cells, "
                                  "omega=0.4, beta=10.15, dt=1e-4, Robin p=180, refactor every "
                                  "step", "dof": 1025 * 1025,
                      "strip_order_option": args.strip_order,
                      "horizon": f"{args.steps} of 1000 steps",
                      "best": {"algo": best["algo"], "N": best["N"],
                               "strip_order": best["strip_order"]}},
           "runs": runs}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for rot2048, 200 for gpe512)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="c32", choices=["fp64", "c32"])
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="steps of the plain FP64 GPU path timed for comparison (0 = skip; "
                         "default 3 for rot2048, 50 for gpe512)")
    ap.add_argument("--parity-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="rot2048",
                    choices=["rot2048", "gpe512", "batch64", "learned1024", "paper-e5",
                             "paper-e6"],
                    help="rot2048: the rotating GPE on 2048^2 cells and 64 strips, refactored "
                         "every step (default, the largest single-GPU configuration); gpe512: "
                         "the 512^2 GPE instance; batch64: the batch of 64 independent NLS "
                         "instances; learned1024: the learned interface guess, trained and "
                         "then run on a 1024^2 GPE; paper-e5: the paper's Robin p-sweep on "
                         "its first NLS mesh (first-step iteration counts); paper-e6: the "
                         "paper's BEC runs on 1025^2 nodes with Robin p=180")
    ap.add_argument("--train-runs", type=int, default=34)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--profile-solve", type=int, default=0, metavar="LAUNCHES",
                    help="profiler mode (gpe512): only factor + LAUNCHES strip solves + a 1 GiB copy")
    ap.add_argument("--batch-algo", default="classical", choices=["classical", "precond"],
                    help="batch64: the Schwarz algorithm of every instance")
    ap.add_argument("--sequential", action=argparse.BooleanOptionalAction, default=True,
                    help="batch64: also run the 64 instances one by one (FP64 and c32)")
    ap.add_argument("--p-list", default="",
                    help="paper-e5: comma-separated Robin parameters (default: 5,10,...,50)")
    ap.add_argument("--profile-factor", type=int, default=0, metavar="FACTORS",
                    help="profiler mode (rot2048): setup + FACTORS refactorisations + "
                         "--profile-solves strip solves + a 1 GiB copy")
    ap.add_argument("--profile-solves", type=int, default=5)
    ap.add_argument("--team", type=int, default=0,
                    help="profiler modes: workgroups per strip in the solve (0 = autotune)")
    ap.add_argument("--strip-order", default="tuned", choices=["node", "y", "tuned"],
                    help="rot2048, gpe512, learned1024, paper-e6: unknown order of the strip "
                         "factor (tuned: the autotuner times both after the first "
                         "factorisation)")
    ap.add_argument("--node-steps", type=int, default=5,
                    help="rot2048: steps of the node-line order timed beside a y-line main run "
                         "(0 = skip)")
    ap.add_argument("--lh-form", default="auto", choices=["auto", "dense", "modal"],
                    help="L_h as dense blocks per strip class or in the modal form (auto: "
                         "modal where ny > 1088, or ny >= 1025 with ny - 1 a power of two: by FFT)")
    ap.add_argument("--solve-shape", type=int, default=0,
                    help="profiler modes: strip-solve tile shape + 1 (0 = autotune)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"rot2048": 20, "gpe512": 200, "paper-e6": 20}.get(args.workload, 2)
    if args.fp64_steps is None:
        args.fp64_steps = 3 if args.workload == "rot2048" else 50
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the strips of one instance are spread over the workgroups of one MI355X.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from workloads import c2

    dev = "cuda:0"
    if args.workload == "batch64":
        run_batch(args, dev)
        return
    if args.workload == "learned1024":
        run_learned(args, dev)
        return
    if args.workload == "rot2048":
        run_rotating(args, dev)
        return
    if args.workload == "paper-e5":
        run_paper_e5(args, dev)
        return
    if args.workload == "paper-e6":
        run_paper_e6(args, dev)
        return
    wl = c2()
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    print(f"bench: {pb.name} dof={dof} prec={args.prec} steps={args.steps}", file=sys.stderr,
          flush=True)
    if args.profile_solve > 0:
        profile_solve(pb, V, args.prec, args.profile_solve, dev, args.team, args.solve_shape)
        return

    main_run = run_gpu(pb, u0, V, args.prec, args.steps, args.warmup, dev,
                       lh_form=args.lh_form, strip_order=args.strip_order)
    T = main_run["seconds"]
    st = main_run["stats"]
    value = dof * args.steps / T
    ks = [x["k"] for x in st]
    qs = [x["q_total"] for x in st]
    gm = [x["gmres_total"] for x in st]
    print(f"bench: {args.prec} {T:.3f}s for factor+{args.steps} steps, {value:.4g} dof-steps/s",
          file=sys.stderr, flush=True)

    avg_ms = main_run["solve_ms"] / max(main_run["solve_launches"], 1)
    nbytes = main_run["solve_work"] / max(main_run["solve_launches"], 1)
    order = main_run["order"]
    if order == "y":
        solve_kernel = "ysolve (forward, middle, backward)"
        traffic = measured_traffic("gpe512", args.prec, "ysolve")
    else:
        # tile shapes 0-3: full-row kernel, 4-7: upper-triangle kernel
        solve_kernel = ("strip_solve_pf_kernel" if main_run["shape"] < 4
                        else "strip_solve_sym_kernel")
        traffic = measured_traffic("gpe512", args.prec, "strip_solve", main_run["shape"])
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0

    fp64 = None
    if args.prec != "fp64" and args.fp64_steps > 0:
        r = run_gpu(pb, u0, V, "fp64", args.fp64_steps, args.warmup, dev)
        fp64 = {"value": dof * args.fp64_steps / r["seconds"], "steps": args.fp64_steps,
                "ms_per_step": 1e3 * r["seconds"] / args.fp64_steps,
                "solve_kernel_ms": r["solve_ms"] / max(r["solve_launches"], 1)}
        print(f"bench: fp64 {fp64['value']:.4g} dof-steps/s", file=sys.stderr, flush=True)

    # parity of the first steps against the FP64 CPU oracle, and its throughput
    parity = None
    cpu = None
    if args.parity_steps > 0 and not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle.step import MonolithicStepper
        r = run_gpu(pb, u0, V, args.prec, args.parity_steps, 0, dev, measure=False)
        ugpu = r["u"].cpu().numpy()
        with threadpool_limits(1):
            t0 = time.perf_counter()
            ost = MonolithicStepper(pb, V, form="B", tol_q=1e-14)
            t_fac = time.perf_counter() - t0
            u = np.array(u0, dtype=complex)
            t1 = time.perf_counter()
            for _ in range(args.parity_steps):
                u, _, _ = ost.step(u)
            t_step = (time.perf_counter() - t1) / args.parity_steps
        err = float(np.linalg.norm(ugpu - u) / np.linalg.norm(u))
        parity = {"steps": args.parity_steps, "rel_l2_vs_oracle": err}
        cpu = {"value": dof * args.steps / (t_fac + args.steps * t_step),
               "unit": "dof-steps/s", "cores": 1, "kind": "oracle",
               "sample": (f"FP64 monolithic oracle (SciPy splu, fixed point form B) on the same "
                          f"workload: factor {t_fac:.2f}s + {args.parity_steps} steps at "
                          f"{t_step:.2f}s/step, extrapolated to the {args.steps}-step job")}
        print(f"bench: parity rel L2 {err:.3e}; oracle {cpu['value']:.4g} dof-steps/s",
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "dof-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64-refine" if args.prec == "c32" else "c128",
        "data": "synthetic",
        "config": {"workload": "GPE trap V=-(x^2+y^2)/2, f=-50|u|^2, (-8,8)^2, 512x512 cells, "
                               "16 equal strips, Robin p=5, dt=1e-3, preconditioned GMRES",
                   "dof": dof, "strips": pb.nsub, "algo": "precond", "prec": args.prec,
                   "strip_order": order, "strip_order_option": args.strip_order,
                   "lh_form": args.lh_form, "timed": "factor(W) + steps"},
        "iters": {"k_mean": float(np.mean(ks)), "k_max": int(np.max(ks)),
                  "q_total": int(np.sum(qs)), "gmres_total": int(np.sum(gm)),
                  "gmres_per_step": float(np.mean(gm))},
        "roofline": {"kernel": solve_kernel, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": nbytes,
                     "avg_launch_ms": avg_ms,
                     "launches": main_run["solve_launches"],
                     "workgroups_per_strip": main_run["team"],
                     "tile_shape": main_run["shape"]},
        "setup_s": main_run["setup_s"],
        "factor_s": main_run["factor_s"],
        "fp64_gpu": fp64,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
