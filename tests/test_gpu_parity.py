"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes span several 64-wide tiles and 32-wide pivot blocks with ragged tails
(ny = 100, 129), uneven strips and both transmission/physical Robin values.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.schwarz import SchwarzOracle, run_schwarz  # noqa: E402
from oracle.step import run_monolithic  # noqa: E402
from workloads import Problem, c1, equal_strips  # noqa: E402


def _osm():
    from paper_1603_05110_amd import osm
    return osm


DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_problem(ncx=30, ncy=99, cells=(9, 12, 9), beta=4.0, p=3.0, pbc=2.0, c=1.0,
                  dt=0.02):
    return Problem(-4.0, 4.0, -3.0, 3.0, ncx, ncy, len(cells), list(cells),
                   lap_coef=c, beta=beta, p=p, p_bc=pbc, dt=dt)


def rand_state(pb, seed, amp=0.5):
    rng = np.random.default_rng(seed)
    s = (pb.ncx + 1, pb.ncy + 1)
    u = amp * (rng.standard_normal(s) + 1j * rng.standard_normal(s))
    W = rng.standard_normal(s)
    return u, W


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def packed(orc, arrays):
    return np.concatenate([np.asarray(a).reshape(-1, orc.ny) for a in arrays], axis=0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("c32", 2e-4)])
@pytest.mark.parametrize("shape", [(30, 99, (9, 12, 9)), (20, 128, (10, 10)),
                                   (24, 64, (5, 7, 6, 6))])
def test_strip_solve_matches_oracle(prec, tol, shape):
    ncx, ncy, cells = shape
    log(f"strip_solve {prec} {shape}")
    osm = _osm()
    pb = small_problem(ncx=ncx, ncy=ncy, cells=cells)
    _, W = rand_state(pb, 1)
    orc = SchwarzOracle(pb, W)
    rng = np.random.default_rng(2)
    bs = [rng.standard_normal((c + 1, pb.ncy + 1)) + 1j * rng.standard_normal((c + 1, pb.ncy + 1))
          for c in cells]
    ref = [orc._lu[j].solve(bs[j].ravel()).reshape(bs[j].shape) for j in range(len(cells))]
    s = osm.OsmSolver(pb, DEV, prec=prec)
    s.factor(to_dev(W))
    x = s.strip_solve(to_dev(packed(orc, bs))).cpu().numpy()
    s.close()
    assert rel(x, packed(orc, ref)) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("c32", 2e-6)])
@pytest.mark.parametrize("ncy", [99, 512])
@pytest.mark.parametrize("solve_shape", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_solve_tile_shape_matches_oracle(prec, tol, ncy, solve_shape):
    """Every kernel and tile shape of the strip solve (full rows or upper
    triangles of the stored inverses, waves per workgroup x rows held in
    registers), forced instead of autotuned, at 2 and 9 column chunks."""
    log(f"strip_solve shape {solve_shape} {prec} ny={ncy + 1}")
    osm = _osm()
    cells = (4, 5, 3)
    pb = Problem(-3.0, 3.0, -16.0, 16.0, sum(cells), ncy, 3, list(cells), lap_coef=0.5, beta=-20.0,
                 p=4.0, p_bc=4.0, dt=5e-3)
    _, W = rand_state(pb, 7)
    orc = SchwarzOracle(pb, W)
    rng = np.random.default_rng(8)
    bs = [rng.standard_normal((c + 1, pb.ncy + 1)) + 1j * rng.standard_normal((c + 1, pb.ncy + 1))
          for c in cells]
    ref = [orc._lu[j].solve(bs[j].ravel()).reshape(bs[j].shape) for j in range(len(cells))]
    want = packed(orc, ref)
    for team in (0, 4):
        s = osm.OsmSolver(pb, DEV, prec=prec, solve_shape=solve_shape, team=team)
        s.factor(to_dev(W))
        x = s.strip_solve(to_dev(packed(orc, bs))).cpu().numpy()
        assert s.solve_shape() == solve_shape - 1
        s.close()
        assert np.all(np.isfinite(x)), team
        assert rel(x, want) < tol, team
        # every strip on its own, and the largest entry error
        for j in range(len(cells)):
            o = orc.starts[j] + j
            sl = slice(o, o + cells[j] + 1)
            assert rel(x[sl], want[sl]) < tol, (team, j)
        assert np.max(np.abs(x - want)) < tol * np.max(np.abs(want)), team


@pytest.mark.parametrize("prec,tol,ncy", [("c32", 2e-6, 1000), ("c32", 2e-6, 2048),
                                          ("fp64", 1e-12, 1000)])
@pytest.mark.parametrize("solve_shape", [5, 6, 7, 8])
def test_upper_triangle_tiles_on_long_lines(prec, tol, ncy, solve_shape):
    """The upper-triangle kernel's tiles for 17 and 33 column chunks (lines of
    1001 and 2049 nodes, the rotating workload's), forced, with the
    autotuned team and a team of 3: rows read through range-checked buffer
    loads, the diagonal taken out once, rows past the end of a wave's list."""
    log(f"upper-triangle shape {solve_shape} {prec} ny={ncy + 1}")
    osm = _osm()
    cells = (4, 6, 3)
    pb = Problem(-3.0, 3.0, -16.0, 16.0, sum(cells), ncy, 3, list(cells), lap_coef=0.5, beta=-20.0,
                 p=4.0, p_bc=4.0, dt=5e-3)
    _, W = rand_state(pb, 9)
    orc = SchwarzOracle(pb, W)
    rng = np.random.default_rng(10)
    bs = [rng.standard_normal((c + 1, pb.ncy + 1)) + 1j * rng.standard_normal((c + 1, pb.ncy + 1))
          for c in cells]
    ref = [orc._lu[j].solve(bs[j].ravel()).reshape(bs[j].shape) for j in range(len(cells))]
    want = packed(orc, ref)
    for team in (0, 3):
        s = osm.OsmSolver(pb, DEV, prec=prec, solve_shape=solve_shape, team=team)
        s.factor(to_dev(W))
        x = s.strip_solve(to_dev(packed(orc, bs))).cpu().numpy()
        assert s.solve_shape() == solve_shape - 1
        s.close()
        assert np.all(np.isfinite(x)), team
        assert rel(x, want) < tol, team
        for j in range(len(cells)):
            o = orc.starts[j] + j
            sl = slice(o, o + cells[j] + 1)
            assert rel(x[sl], want[sl]) < tol, (team, j)
        assert np.max(np.abs(x - want)) < tol * np.max(np.abs(want)), team


@pytest.mark.parametrize("fixed_k,fixed_q", [(1, 1), (3, 2)])
def test_fixed_iteration_classical_matches_oracle(fixed_k, fixed_q):
    """Same (k, q) counts, cold fixed-point start: rounding-level agreement of
    the iteration itself (g and the strip solutions)."""
    log(f"fixed iteration k={fixed_k} q={fixed_q}")
    osm = _osm()
    pb = small_problem()
    u, W = rand_state(pb, 3)
    orc = SchwarzOracle(pb, W)
    g0 = np.zeros((2 * (pb.nsub - 1), pb.ncy + 1), complex)
    res = orc.classical(u, g0, fixed_k=fixed_k, fixed_q=fixed_q)
    s = osm.OsmSolver(pb, DEV, fixed_k=fixed_k, fixed_q=fixed_q, warm_start=False)
    s.factor(to_dev(W))
    ud = to_dev(u)
    st = s.step(ud)
    g = s.get_interface().cpu().numpy()
    v = s.get_strip_solution().cpu().numpy()
    s.close()
    assert st["k"] == fixed_k and st["q_total"] == fixed_k * fixed_q
    assert rel(g, res["g"]) < 1e-11
    assert rel(v, packed(orc, res["vs"])) < 1e-11
    unew = orc.assemble_global(res["vs"], u)
    assert rel(ud.cpu().numpy(), unew) < 1e-11


def test_schwarz_map_matches_oracle():
    log("interface R")
    osm = _osm()
    pb = small_problem()
    u, W = rand_state(pb, 4)
    orc = SchwarzOracle(pb, W, tol_q=1e-14)
    rng = np.random.default_rng(5)
    g = rng.standard_normal((4, pb.ncy + 1)) + 1j * rng.standard_normal((4, pb.ncy + 1))
    ref, _, _ = orc.R(g, u)
    s = osm.OsmSolver(pb, DEV, tol_q=1e-14, warm_start=False)
    s.factor(to_dev(W))
    got = s.interface_apply(osm.OSM_IFACE_R, to_dev(u), to_dev(g)).cpu().numpy()
    s.close()
    assert rel(got, ref) < 1e-11


@pytest.mark.parametrize("cells,pbc", [((9, 12, 9), 2.0), ((10, 10, 10), 3.0)])
def test_lh_blocks_match_oracle(cells, pbc):
    log(f"L_h blocks {cells}")
    osm = _osm()
    pb = small_problem(cells=cells, pbc=pbc, ncx=sum(cells))
    orc = SchwarzOracle(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    B = orc.build_Lh()
    s = osm.OsmSolver(pb, DEV, algo="precond")
    blk = s.get_lh_blocks().cpu().numpy()
    s.close()
    N = pb.nsub
    for j in range(N):
        if j >= 1:
            assert rel(blk[j, 0], B[(2 * (j - 1), 2 * (j - 1) + 1)]) < 1e-11
        if 1 <= j <= N - 2:
            assert rel(blk[j, 1], B[(2 * (j - 1), 2 * j)]) < 1e-11
            assert rel(blk[j, 2], B[(2 * j + 1, 2 * (j - 1) + 1)]) < 1e-11
        if j <= N - 2:
            assert rel(blk[j, 3], B[(2 * j + 1, 2 * j)]) < 1e-11


def test_pinv_gmres_matches_direct_solve():
    log("P^-1 by GMRES")
    osm = _osm()
    pb = small_problem(ncy=40)
    orc = SchwarzOracle(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    orc.build_Lh()
    n = 4 * (pb.ncy + 1)
    rng = np.random.default_rng(6)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.linalg.solve(np.eye(n) - orc.Lh_dense(), y)
    s = osm.OsmSolver(pb, DEV, algo="precond", tol_gmres=1e-13)
    x = s.interface_apply(osm.OSM_IFACE_PINV, None, to_dev(y.reshape(4, -1))).cpu().numpy()
    s.close()
    assert rel(x.ravel(), ref) < 1e-11


def smooth_problem(pbc=2.0):
    """48 x 63 cells on (-8,8)^2, uneven strips, GPE scaling: the classical
    iteration converges here in about 300 iterations per step."""
    from workloads import gaussian_boost
    pb = Problem(-8.0, 8.0, -8.0, 8.0, 48, 63, 3, [15, 18, 15], lap_coef=0.5, beta=-5.0,
                 p=2.0, p_bc=pbc, dt=0.01)
    u = gaussian_boost(pb, k=1.0)
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return pb, u, 0.5 * np.sin(X) * np.cos(Y)


@pytest.mark.parametrize("algo,prec", [("classical", "fp64"), ("precond", "fp64"),
                                       ("classical", "c32"), ("precond", "c32")])
def test_converged_steps_match_monolithic(algo, prec):
    log(f"converged steps {algo} {prec}")
    osm = _osm()
    pb, u, W = smooth_problem()
    ref = run_monolithic(pb, u, W, 3, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo=algo, prec=prec, tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14, max_k=4000)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(3):
        st = s.step(ud)
        log(f"  k={st['k']} q={st['q_total']} gmres={st['gmres_total']}")
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("algo,prec", [("classical", "fp64"), ("precond", "c32")])
def test_error_estimate_fixed_point_matches_monolithic(algo, prec):
    """The error-estimate stopping test of the inner fixed point
    (q_estimate = 1, with inexact inner solves) converges to the same step as
    the monolithic oracle, with no more fixed-point iterations than the
    paper's test."""
    log(f"q_estimate {algo} {prec}")
    osm = _osm()
    pb, u, W = smooth_problem()
    ref = run_monolithic(pb, u, W, 3, tol_q=1e-14)
    q = {}
    for est in (0, 1):
        s = osm.OsmSolver(pb, DEV, algo=algo, prec=prec, tol_k=1e-12, tol_k_relative=True,
                          tol_q=1e-14, max_k=4000, eta_q=1e-2, tol_gmres=1e-2,
                          q_estimate=est)
        s.factor(to_dev(W))
        ud = to_dev(u)
        q[est] = 0
        for _ in range(3):
            st = s.step(ud)
            q[est] += st["q_total"]
            log(f"  est={est} k={st['k']} q={st['q_total']} gmres={st['gmres_total']}")
        s.close()
        assert rel(ud.cpu().numpy(), ref) < 1e-10
    assert q[1] <= q[0]


def test_c1_matches_oracle():
    """Configuration C1 (cubic NLS, 128^2 cells, 2 strips, p = 1, 20 steps,
    classical FP64) against the monolithic oracle: 1e-10 relative L2."""
    log("C1 full")
    osm = _osm()
    wl = c1()
    pb, u0, W = wl.problems[0], wl.u0[0], wl.V[0]
    ref = run_monolithic(pb, u0, W, pb.steps, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo="classical", tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14, max_k=5000)
    s.factor(to_dev(W))
    ud = to_dev(u0)
    for n in range(pb.steps):
        st = s.step(ud)
        if n % 5 == 0:
            log(f"  step {n}: k={st['k']} q={st['q_total']}")
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "c32"])
def test_rotating_frame_refactor_every_step_matches_oracle(prec):
    """Rotating-frame GPE (Section 5.2.1): W_n computed on the device from
    the rotated anisotropic trap and refactored every step, uneven strips."""
    log(f"rotating frame {prec}")
    from oracle.rotating import step_potential
    from workloads import gaussian_boost
    osm = _osm()
    pb = Problem(-6.0, 6.0, -6.0, 6.0, 40, 71, 3, [12, 16, 12], lap_coef=0.5, beta=-20.0,
                 p=3.0, p_bc=3.0, dt=0.02, omega=-0.7, vxx=-0.5, vyy=-0.6)
    u0 = gaussian_boost(pb, k=0.5, a=0.5)
    steps = 4
    ref = run_monolithic(pb, u0, lambda n: step_potential(pb, n), steps, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14)
    ud = to_dev(u0)
    for n in range(1, steps + 1):
        s.factor_rotating(n)
        s.step(ud)
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


def test_neumann_mass_invariance():
    """p_bc = 0: the discrete mass is invariant (exact identity of the
    scheme, any size); transmission p > 0 between strips."""
    log("mass invariance")
    osm = _osm()
    pb, u, W = smooth_problem(pbc=0.0)
    s = osm.OsmSolver(pb, DEV, algo="precond", tol_k=1e-13, tol_k_relative=True, tol_q=1e-14)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(3):
        st = s.step(ud)
        assert abs(st["mass_after"] - st["mass_before"]) < 1e-11 * st["mass_before"]
    s.close()


@pytest.mark.parametrize("algo", ["classical", "precond"])
def test_c32_with_values_below_fp32_range_matches_monolithic(algo):
    """u0 = exp(-(x^2+y^2)) exp(ix) on (-10,10)^2: the edge strips hold values
    near 1e-44 and below, outside FP32's normal range.  The per-strip
    power-of-two scaling of the complex-FP32 solve keeps the refined
    iteration converging to the FP64 answer in every strip."""
    log(f"c32 tiny tails {algo}")
    osm = _osm()
    from workloads import gaussian_boost
    pb = Problem(-10.0, 10.0, -10.0, 10.0, 48, 63, 4, [10, 14, 12, 12], lap_coef=1.0, beta=1.0,
                 p=3.0, p_bc=3.0, dt=0.01)
    u = gaussian_boost(pb, k=1.0)
    W = np.zeros((pb.ncx + 1, pb.ncy + 1))
    assert np.abs(u[0]).max() < 1e-40
    ref = run_monolithic(pb, u, W, 2, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo=algo, prec="c32", tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14, max_k=4000)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(2):
        s.step(ud)
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("ncy", [1024, 2048])
@pytest.mark.parametrize("prec", ["fp64", "c32"])
def test_wide_lines_match_monolithic(ncy, prec):
    """Lines of 1025 and 2049 nodes (the widths of the 1024^2 and 2048^2
    workloads: 17 and 33 column chunks) on a few x-cells: the wide-line
    kernels of the factor, the solve and the L_h matvec against the oracle."""
    log(f"wide lines ny={ncy + 1} {prec}")
    osm = _osm()
    from workloads import gaussian_boost
    pb = Problem(-3.0, 3.0, -16.0, 16.0, 12, ncy, 3, [4, 5, 3], lap_coef=0.5, beta=-20.0,
                 p=4.0, p_bc=4.0, dt=5e-3)
    u = gaussian_boost(pb, k=0.5, a=0.7)
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    W = -0.5 * (X ** 2 + 1.2 * Y ** 2) / 16.0
    ref = run_monolithic(pb, u, W, 2, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(2):
        st = s.step(ud)
        log(f"  k={st['k']} q={st['q_total']} gmres={st['gmres_total']}")
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10
