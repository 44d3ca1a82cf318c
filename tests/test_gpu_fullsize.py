"""Full-size parity of the configurations against the FP64 oracle.

* GPE 512^2 cells, 16 strips (the preconditioned, complex-FP32 workload):
  three steps against the monolithic oracle, globally, per strip and by the
  largest entry error; and the full 200-step horizon of the complex-FP32
  path against the FP64 GPU path, every step compared.
* GPE 1024^2 cells, 32 strips (the learned-start workload's problem): two
  steps against the monolithic oracle.
* Rotating GPE 2048^2 cells, 64 uneven strips: three steps of the
  complex-FP32 path and of the y-line-order path against the FP64 GPU path
  (the monolithic oracle does not fit a test at 4.2 M nodes; its discrete
  equation and sampled strip solves are checked in test_gpu_c5.py).

Solver settings are the benchmark's: relative Schwarz tolerance 1e-12,
inexact inner solves with the error-estimate test, GMRES tolerance 3e-2.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.step import run_monolithic  # noqa: E402
from workloads import c2, c4, c5  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def opts(prec, **kw):
    return dict(algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True, max_k=500,
                tol_q=1e-13, max_q=200, warm_start=True, tol_gmres=3e-2, gmres_restart=50,
                max_gmres=2000, eta_q=3e-2, q_estimate=1, **kw)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_against(got, ref, pb, tol, what):
    """Global relative L2, per x-strip relative L2 (node-lines of each
    strip) and the largest entry error relative to the largest entry."""
    g = rel(got, ref)
    mx = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    s0 = 0
    worst = 0.0
    for c in pb.strip_cells:
        sl = slice(s0, s0 + c + 1)
        worst = max(worst, rel(got[sl], ref[sl]))
        s0 += c
    log(f"  {what}: rel L2 {g:.3e}, worst strip {worst:.3e}, max-abs {mx:.3e}")
    assert g < tol and worst < tol and mx < tol, what


def run_gpu(pb, u0, V, prec, steps):
    from paper_1603_05110_amd import osm
    s = osm.OsmSolver(pb, DEV, **opts(prec))
    s.factor(torch.from_numpy(V).to(DEV))
    u = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV)
    for _ in range(steps):
        s.step(u)
    s.close()
    return u.cpu().numpy()


@pytest.mark.parametrize("prec", ["c32", "fp64"])
def test_gpe512_three_steps_match_monolithic(prec):
    wl = c2()
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    log(f"GPE 512^2 / 16 strips, {prec}, 3 steps vs monolithic")
    got = run_gpu(pb, u0, V, prec, 3)
    ref = run_monolithic(pb, u0, V, 3, tol_q=1e-14)
    check_against(got, ref, pb, 1e-10, f"{prec} vs oracle")


def test_gpe512_full_horizon_c32_against_fp64():
    """200 steps: the complex-FP32 path and the FP64 path advanced side by
    side, compared after every step (final value and maximum over steps)."""
    from paper_1603_05110_amd import osm
    wl = c2()
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    log(f"GPE 512^2 / 16 strips, {pb.steps} steps, c32 against FP64")
    Wd = torch.from_numpy(V).to(DEV)
    s32 = osm.OsmSolver(pb, DEV, **opts("c32"))
    s64 = osm.OsmSolver(pb, DEV, **opts("fp64"))
    s32.factor(Wd)
    s64.factor(Wd)
    u32 = torch.from_numpy(u0).to(DEV)
    u64 = u32.clone()
    worst = 0.0
    for n in range(pb.steps):
        s32.step(u32)
        s64.step(u64)
        e = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
        worst = max(worst, e)
    s32.close()
    s64.close()
    final = e
    log(f"  final rel L2 {final:.3e}, max over steps {worst:.3e}")
    assert worst < 1e-10
    a, b = u32.cpu().numpy(), u64.cpu().numpy()
    check_against(a, b, pb, 1e-10, "c32 vs FP64 at the last step")


def test_gpe1024_two_steps_match_monolithic():
    wl = c4(steps=2)
    pb, u0, V = wl.problems[0], wl.u0[0], wl.V[0]
    log(f"GPE 1024^2 / 32 strips, c32, 2 steps vs monolithic")
    got = run_gpu(pb, u0, V, "c32", 2)
    ref = run_monolithic(pb, u0, V, 2, tol_q=1e-14)
    check_against(got, ref, pb, 1e-10, "c32 vs oracle")


def test_rotating_2048_c32_against_fp64():
    from paper_1603_05110_amd import osm
    wl = c5(steps=3)
    pb, u0 = wl.problems[0], wl.u0[0]
    out = {}
    for prec in ("c32", "fp64", "y"):
        log(f"rotating 2048^2 / 64 strips, {prec}, 3 steps")
        o = opts("fp64", strip_order="y") if prec == "y" else opts(prec)
        s = osm.OsmSolver(pb, DEV, **o)
        u = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV)
        for n in range(1, 4):
            s.factor_rotating(n)
            st = s.step(u)
            log(f"  step {n}: k={st['k']} gmres={st['gmres_total']}")
        s.close()
        out[prec] = u.cpu().numpy()
        del u
        torch.cuda.empty_cache()
    check_against(out["c32"], out["fp64"], pb, 1e-10, "c32 vs FP64")
    check_against(out["y"], out["fp64"], pb, 1e-10, "y-line order vs node-line FP64")
