#!/usr/bin/env python3
"""Throughput of the optimized Schwarz time loop on one MI355X.

Workload: the GPE with harmonic trap V = -(x^2+y^2)/2, f(u) = -50|u|^2,
c = 1/2 on (-8,8)^2 with 512 x 512 cells (263,169 nodes), 16 equal x-strips,
Robin p = 5 (transmission and physical), dt = 1e-3, preconditioned algorithm
with GMRES on P = I - L_h; u0 = normalised Gaussian + 1e-3 seeded complex
noise.  Synthetic, seeded inputs.

A "step" is one time step: the stationary nonlinear problem of the step is
solved by preconditioned Schwarz iterations, each of which runs the strip
fixed point (residual stencil + block-tridiagonal substitution per
iteration) and GMRES on the interface.  The timed region covers the
factorisation of the strip operators for W_n plus K steps with the inputs
resident in HBM; L_h is built once at setup (outside the timed region, its
time is reported).

Printed: one JSON line with dof-steps/s, iterations, a roofline entry for
the strip-solve kernel (live HIP-event timing of every launch in the timed
region), the plain FP64 GPU path for comparison, the parity of the first
steps against the FP64 CPU oracle, and the oracle's own throughput.
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

# HBM bytes per strip-solve launch from rocprofv3 FETCH_SIZE + WRITE_SIZE on
# this workload, each scaled by the counter's reading for a 1 GiB copy
# (fetch x2.0, write x1.0); valid only for the full-row kernel whose source
# text (the strip_solve_pf_kernel template) hashes to source_sha256.
SOLVE_TRAFFIC = {"c32": {"bytes": 2.2672e+09,
                         "source_sha256": "f9cd27c1f2eef86c94452add056158ca7fb70bf24c4a5a5bf5c6fdc5c1de7edc",
                         "summary": "profiles/strip_solve_c32_gpe512_hbm_counters.md"}}


def pf_kernel_source():
    """Source text the counters describe: the full-row strip-solve kernel
    template (its definition up to the closing brace) and the wave-sum
    helpers it calls."""
    csrc = os.path.join(ROOT, "paper_1603_05110_amd", "csrc")
    try:
        src = open(os.path.join(csrc, "kernels_solve.hip")).read()
        hdr = open(os.path.join(csrc, "osm_internal.h")).read()
    except OSError:
        return None
    key = "void strip_solve_pf_kernel(SolveArgs a) {"
    i = src.find(key)
    if i < 0:
        return None
    i = src.rfind("template <", 0, i)
    j = src.find("\n}\n", i)
    a = hdr.find("template <int CTRL>")
    b = hdr.find("\n}\n", hdr.find("double wave_sum_f64(double v)"))
    if j < 0 or a < 0 or b < 0:
        return None
    return src[i:j + 3] + hdr[a:b + 3]


def measured_traffic(prec, kernel_name):
    import hashlib
    rec = SOLVE_TRAFFIC.get(prec)
    if rec is None or not kernel_name.startswith("strip_solve_pf_kernel"):
        return None
    src = pf_kernel_source()
    if src is None:
        return None
    sha = hashlib.sha256(src.encode()).hexdigest()
    return rec["bytes"] if sha == rec["source_sha256"] else None


def solver_opts(prec):
    return dict(algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True, max_k=500,
                tol_q=1e-13, max_q=200, warm_start=True, tol_gmres=3e-2,
                gmres_restart=50, max_gmres=2000, eta_q=3e-2, q_estimate=1)


def run_gpu(pb, u0, V, prec, steps, warmup, dev, measure=True):
    import torch
    from paper_1603_05110_amd import osm
    t = time.perf_counter()
    s = osm.OsmSolver(pb, dev, **solver_opts(prec))
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
    s.close()
    return dict(seconds=t1 - t0, factor_s=t_fac, setup_s=t_setup, stats=stats, u=u,
                solve_ms=kern[0], solve_launches=kern[1], solve_work=work, team=team, shape=shape)


def profile_solve(pb, V, prec, launches, dev):
    """Kernel-level measurement mode for profilers: factor once, then run
    `launches` strip solves on a seeded right-hand side, then one
    device-to-device copy of 1 GiB (the calibration kernel for the HBM byte
    counters: its algorithmic traffic is 1 GiB read + 1 GiB written)."""
    import torch
    from paper_1603_05110_amd import osm
    s = osm.OsmSolver(pb, dev, **solver_opts(prec))
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
    team = s.solve_team()
    s.close()
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    avg = ms / max(n, 1)
    print(json.dumps({"mode": "profile-solve", "prec": prec, "launches": n, "avg_launch_ms": avg,
                      "bytes_per_launch": nbytes, "achieved_GBs": nbytes / (avg * 1e-3) / 1e9,
                      "workgroups_per_strip": team, "copy_bytes": 2 * src.numel() * 8}),
          flush=True)


def run_batch(args, dev):
    """Batch of 64 independent cubic-NLS instances (grids 256..768 squared,
    8-32 uneven strips, seeded p and potentials), classical algorithm.  The
    timed region is the refactorisation of every instance plus K steps, each
    step replaying the captured graph of a chunk of Schwarz iterations; the
    solve roofline comes from one more step run launch by launch with HIP
    events around every batched solve."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import osm
    from workloads import c3

    wl = c3()
    pbs = wl.problems
    dofs = [(pb.ncx + 1) * (pb.ncy + 1) for pb in pbs]
    dof = sum(dofs)
    opts = dict(prec=args.prec, tol_k=1e-12, tol_k_relative=True, tol_q=1e-13, max_k=5000,
                max_q=200)
    print(f"bench: C3 batch {len(pbs)} instances, {dof} dofs, prec={args.prec}", file=sys.stderr,
          flush=True)
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
                               "V = 8 seeded Gaussians (max|V|=5), dt=0.01, classical, "
                               "graph-replayed chunks, autotuned solve tiles",
                   "dof": dof, "instances": len(pbs), "strips": sum(pb.nsub for pb in pbs),
                   "algo": "classical", "prec": args.prec, "timed": "factor(W) + steps"},
        "iters": {"k_mean": float(ks.mean()), "k_max": int(ks.max()),
                  "q_total": int(qs.sum())},
        "roofline": {"kernel": "batch_solve", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_timed": nbytes, "launches": launches,
                     "avg_launch_ms": ms / max(launches, 1),
                     "measured_on": "one extra step, launch by launch"},
        "tuning": tuning,
        "setup_s": t_setup,
        "first_factor_and_autotune_s": t_tune,
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

    opts = dict(solver_opts("c32"))
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
                      "fallbacks": int(sum(x["fallback_used"] for x in st)),
                      "u": u.cpu().numpy()}
        print(f"bench: {name}: {runs[name]['value']:.4g} dof-steps/s, k {runs[name]['k_total']}, "
              f"gmres {runs[name]['gmres_total']}", file=sys.stderr, flush=True)
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


def run_rotating(args, dev):
    """Rotating GPE at full size (2048^2 cells, 64 uneven strips), solved in
    the rotating frame: the step potential changes every step, so every step
    refactors all 2112 strip lines (osm_factor_rotating) before its Schwarz
    iterations.  A truncated horizon of --steps steps is timed (the full
    1000-step horizon is the same work repeated)."""
    import numpy as np
    import torch

    from paper_1603_05110_amd import osm
    from workloads import c5

    wl = c5(steps=args.steps)
    pb, u0 = wl.problems[0], wl.u0[0]
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    print(f"bench: {pb.name} dof={dof} prec={args.prec} steps={args.steps}", file=sys.stderr,
          flush=True)
    opts = solver_opts(args.prec)
    t = time.perf_counter()
    s = osm.OsmSolver(pb, dev, **opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    print(f"bench: setup (L_h built) {t_setup:.1f}s", file=sys.stderr, flush=True)
    u = torch.from_numpy(u0).to(dev)
    t = time.perf_counter()
    s.factor_rotating(1)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t
    print(f"bench: first factor + solve autotune {t_first:.1f}s", file=sys.stderr, flush=True)
    if args.warmup > 0:
        uw = u.clone()
        for n in range(1, args.warmup + 1):
            s.factor_rotating(n)
            s.step(uw)
        del uw
    torch.cuda.synchronize()
    s.kernel_timing(True)
    stats, t_fac = [], 0.0
    u_first = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, args.steps + 1):
        ta = time.perf_counter()
        s.factor_rotating(n)
        torch.cuda.synchronize()
        t_fac += time.perf_counter() - ta
        stats.append(s.step(u))
        if n == 1:
            u_first = u.clone()
        print(f"bench: step {n}: k {stats[-1]['k']} gmres {stats[-1]['gmres_total']} "
              f"q {stats[-1]['q_total']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    kern = s.kernel_timing(False)
    solve_work = s.kernel_work()
    fac_ms, fac_n, fac_fl = s.factor_timing()
    team, shape = s.solve_team(), s.solve_shape()
    s.close()
    value = dof * args.steps / T
    avg_ms = kern[0] / max(kern[1], 1)
    nbytes = solve_work / max(kern[1], 1)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    upd_avg_ms = fac_ms / max(fac_n, 1)
    upd_tflops = fac_fl / (fac_ms * 1e-3) / 1e12 if fac_ms > 0 else 0.0
    print(f"bench: {T:.2f}s for {args.steps} steps ({t_fac:.2f}s factor), {value:.4g} dof-steps/s",
          file=sys.stderr, flush=True)
    # the FP64 oracle: the first step checked against the discrete equation
    # with the oracle's assembled operators (a monolithic direct solve at
    # 4.2 M nodes is out of reach), and the oracle's throughput on the same
    # problem at 512^2 cells
    check, cpu = None, None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle.fem import StripMatrices, weighted_mass_2d
        from oracle.rotating import step_potential
        from oracle.step import run_monolithic
        u1 = u_first.cpu().numpy()
        del u_first
        mats = StripMatrices(pb.ncx, pb.ncy, pb.hx, pb.hy)
        K = mats.operator(step_potential(pb, 1), pb.dt, pb.lap_coef, pb.p_bc, pb.p_bc)
        v = 0.5 * (u0 + u1).ravel()
        F = (2j / pb.dt) * (mats.M @ u0.ravel())
        r = K @ v + weighted_mass_2d((pb.beta * np.abs(v) ** 2).reshape(u0.shape), pb.hx,
                                     pb.hy) @ v - F
        check = {"step": 1, "rel_residual_discrete_equation": float(np.linalg.norm(r) / np.linalg.norm(F)),
                 "bound": 2.5e-11}
        del K, r, v, F, mats
        print(f"bench: step-1 residual {check['rel_residual_discrete_equation']:.3e}",
              file=sys.stderr, flush=True)
        sw = c5(ncells=512, nsub=16, steps=1)
        spb, su0 = sw.problems[0], sw.u0[0]
        with threadpool_limits(1):
            t1 = time.perf_counter()
            run_monolithic(spb, su0, lambda k: step_potential(spb, k), 1, tol_q=1e-14)
            tc = time.perf_counter() - t1
        sdof = (spb.ncx + 1) * (spb.ncy + 1)
        cpu = {"value": sdof / tc, "unit": "dof-steps/s", "cores": 1, "kind": "oracle",
               "sample": (f"FP64 monolithic oracle (SciPy splu, form B) on the same rotating "
                          f"problem at 512^2 cells ({sdof} dofs), one step including its "
                          f"factorisation ({tc:.1f}s); the 2048^2 system is 16x larger")}
        print(f"bench: oracle {cpu['value']:.4g} dof-steps/s", file=sys.stderr, flush=True)
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
        "config": {"workload": "rotating GPE in the rotating frame, Omega_r=0.7, "
                               "V=-(x^2+1.2y^2)/2, f=-500|u|^2, (-16,16)^2, 2048^2 cells, "
                               "64 uneven strips, p=5, dt=5e-4, vortex Gaussian, preconditioned, "
                               "refactor every step",
                   "dof": dof, "strips": pb.nsub, "algo": "precond", "prec": args.prec,
                   "timed": "per step: factor(W_n) + Schwarz/GMRES",
                   "horizon": f"{args.steps} of 1000 steps"},
        "iters": {"k_mean": float(np.mean([x["k"] for x in stats])),
                  "q_total": int(sum(x["q_total"] for x in stats)),
                  "gmres_total": int(sum(x["gmres_total"] for x in stats))},
        "roofline": {"kernel": "sweep_update", "bound": "mfma", "achieved": upd_tflops,
                     "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": upd_tflops / MFMA_FP32_PEAK_TFLOPS if args.prec == "c32"
                     else upd_tflops / MFMA_FP64_PEAK_TFLOPS,
                     "traffic": None, "flops_timed": fac_fl, "avg_launch_ms": upd_avg_ms,
                     "launches": fac_n,
                     "note": ("8 real flops per complex multiply-add; the kernel issues 6 "
                              "(three real products)")},
        "solve": {"kernel": "strip_solve", "bound": "hbm", "achieved": achieved,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "bytes_per_launch": nbytes, "avg_launch_ms": avg_ms, "launches": kern[1],
                  "workgroups_per_strip": team, "tile_shape": shape},
        "factor": {"s_per_step": t_fac / args.steps,
                   "update_ms_per_step": fac_ms / args.steps},
        "setup_s": t_setup,
        "first_factor_and_autotune_s": t_first,
        "check": check,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="c32", choices=["fp64", "c32"])
    ap.add_argument("--fp64-steps", type=int, default=50,
                    help="steps of the plain FP64 GPU path timed for comparison (0 = skip)")
    ap.add_argument("--parity-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="gpe512", choices=["gpe512", "batch64", "learned1024", "rot2048"],
                    help="gpe512: the single GPE instance (default); batch64: the batch of "
                         "64 independent NLS instances; learned1024: the learned interface "
                         "guess, trained and then run on a 1024^2 GPE; rot2048: the rotating "
                         "GPE on 2048^2 cells and 64 strips, refactored every step")
    ap.add_argument("--train-runs", type=int, default=34)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--profile-solve", type=int, default=0, metavar="LAUNCHES",
                    help="profiler mode: only factor + LAUNCHES strip solves + a 1 GiB copy")
    args = ap.parse_args()
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
    wl = c2()
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    dof = (pb.ncx + 1) * (pb.ncy + 1)
    print(f"bench: {pb.name} dof={dof} prec={args.prec} steps={args.steps}", file=sys.stderr,
          flush=True)
    if args.profile_solve > 0:
        profile_solve(pb, V, args.prec, args.profile_solve, dev)
        return

    main_run = run_gpu(pb, u0, V, args.prec, args.steps, args.warmup, dev)
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
    # tile shapes 0-3: full-row kernel, 4-7: upper-triangle kernel
    solve_kernel = "strip_solve_pf_kernel" if main_run["shape"] < 4 else "strip_solve_sym_kernel"
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
                   "timed": "factor(W) + steps"},
        "iters": {"k_mean": float(np.mean(ks)), "k_max": int(np.max(ks)),
                  "q_total": int(np.sum(qs)), "gmres_total": int(np.sum(gm)),
                  "gmres_per_step": float(np.mean(gm))},
        "roofline": {"kernel": solve_kernel, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.prec, solve_kernel), "bytes_per_launch": nbytes,
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
