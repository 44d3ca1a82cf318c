"""GPU parity of the strip factor and solve in y-line order (the strip's
unknowns taken y-line by y-line: K_j block tridiagonal with nx x nx blocks
along the ny y-lines) against the FP64 oracle.

* The stored factor: each y-line's block is the inverse of a Schur
  complement, which by its definition is one diagonal block of the inverse
  of a principal submatrix of K_j (leading y-lines below the middle line,
  trailing ones above it, all of K_j for the middle line), formed here from
  the oracle's assembled strip matrix with a dense inverse.
* The strip solve against the oracle's sparse LU of every strip, globally,
  per strip and by the largest entry, on shapes with odd and even ny, ny = 3,
  strips of 3 and of 64 node-lines (the limit) and uneven strips.
* Converged steps (classical and preconditioned) against the monolithic
  oracle, the rotating-frame refactor, and the autotuned order.
* Complex FP32 storage of the inverses (prec c32): the half-chain y-lines'
  stored blocks are exactly the FP64 blocks rounded (the complements are
  formed in FP64 either way), the middle line's within FP32 rounding; the
  strip solve within FP32 accuracy; converged steps to the FP64 bar, the
  fixed point's FP64 residual refining.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.schwarz import SchwarzOracle  # noqa: E402
from oracle.step import run_monolithic  # noqa: E402
from workloads import Problem  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _osm():
    from paper_1603_05110_amd import osm
    return osm


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(ncx, ncy, cells, beta=4.0, p=3.0, pbc=2.0, c=1.0, dt=0.02):
    return Problem(-4.0, 4.0, -3.0, 3.0, ncx, ncy, len(cells), list(cells), lap_coef=c,
                   beta=beta, p=p, p_bc=pbc, dt=dt)


def potential(pb, seed):
    return np.random.default_rng(seed).standard_normal((pb.ncx + 1, pb.ncy + 1))


def strip_matrix_y(orc, j):
    """K_j dense, unknowns renumbered y-line by y-line: (l, a) -> a nx + l."""
    K = orc.mats[j].operator(orc.Wj[j], orc.pb.dt, orc.pb.lap_coef, orc.pl[j],
                             orc.pr[j]).toarray()
    nx, ny = orc.cells[j] + 1, orc.ny
    perm = (np.arange(nx)[None, :] * ny + np.arange(ny)[:, None]).ravel()
    return K[np.ix_(perm, perm)], nx


def _yfactor(pb, W, prec):
    osm = _osm()
    s = osm.OsmSolver(pb, DEV, strip_order="y", prec=prec)
    s.factor(to_dev(W))
    assert s.strip_order() == "y"
    got = [f.cpu().numpy() for f in s.get_yfactor()]
    s.close()
    return got


@pytest.mark.parametrize("prec", ["fp64", "c32"])
@pytest.mark.parametrize("ncy,cells", [(9, (3, 5, 4)), (10, (4, 2, 6)), (2, (3, 3))])
def test_factor_blocks_are_inverses_of_schur_complements(ncy, cells, prec):
    log(f"y-order factor blocks ny={ncy + 1} cells={cells} {prec}")
    pb = problem(sum(cells), ncy, cells)
    W = potential(pb, 3)
    orc = SchwarzOracle(pb, W)
    got = _yfactor(pb, W, prec)
    if prec == "c32":
        assert got[0].dtype == np.complex64
        g64 = _yfactor(pb, W, "fp64")
        m = pb.ncy // 2
        for j in range(pb.nsub):
            for a in range(pb.ncy + 1):
                if a != m:   # the chains never read their stored blocks back
                    assert np.array_equal(got[j][a], g64[j][a].astype(np.complex64)), (j, a)
    tol = 1e-12 if prec == "fp64" else 1e-6
    ny, m = pb.ncy + 1, pb.ncy // 2
    for j in range(pb.nsub):
        Ky, nx = strip_matrix_y(orc, j)
        for a in range(ny):
            if a < m:       # leading y-lines 0 .. a: last diagonal block
                sub = np.linalg.inv(Ky[:(a + 1) * nx, :(a + 1) * nx])
                want = sub[a * nx:, a * nx:]
            elif a > m:     # trailing y-lines a .. ny-1: first diagonal block
                sub = np.linalg.inv(Ky[a * nx:, a * nx:])
                want = sub[:nx, :nx]
            else:
                want = np.linalg.inv(Ky)[a * nx:(a + 1) * nx, a * nx:(a + 1) * nx]
            assert rel(got[j][a], want) < tol, (j, a)


@pytest.mark.parametrize("prec", ["fp64", "c32"])
@pytest.mark.parametrize("ncx,ncy,cells", [(30, 99, (9, 12, 9)), (20, 128, (10, 10)),
                                           (24, 64, (5, 7, 6, 6)), (6, 2, (2, 2, 2)),
                                           (70, 40, (63, 7))])
def test_strip_solve_matches_oracle(ncx, ncy, cells, prec):
    log(f"y-order strip solve {ncx}x{ncy} {cells} {prec}")
    tol = 1e-12 if prec == "fp64" else 1e-5
    osm = _osm()
    pb = problem(ncx, ncy, cells)
    W = potential(pb, 1)
    orc = SchwarzOracle(pb, W)
    rng = np.random.default_rng(2)
    bs = [rng.standard_normal((c + 1, pb.ncy + 1)) + 1j * rng.standard_normal((c + 1, pb.ncy + 1))
          for c in cells]
    ref = [orc._lu[j].solve(bs[j].ravel()).reshape(bs[j].shape) for j in range(len(cells))]
    want = np.concatenate(ref)
    s = osm.OsmSolver(pb, DEV, strip_order="y", prec=prec)
    s.factor(to_dev(W))
    x = s.strip_solve(to_dev(np.concatenate(bs))).cpu().numpy()
    s.close()
    assert np.all(np.isfinite(x))
    log(f"  rel {rel(x, want):.2e}")
    assert rel(x, want) < tol
    o = 0
    for j, c in enumerate(cells):
        assert rel(x[o:o + c + 1], ref[j]) < tol, j
        o += c + 1
    assert np.max(np.abs(x - want)) < tol * np.max(np.abs(want))


def smooth_problem():
    from workloads import gaussian_boost
    pb = Problem(-8.0, 8.0, -8.0, 8.0, 48, 63, 3, [15, 18, 15], lap_coef=0.5, beta=-5.0,
                 p=2.0, p_bc=2.0, dt=0.01)
    u = gaussian_boost(pb, k=1.0)
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return pb, u, 0.5 * np.sin(X) * np.cos(Y)


@pytest.mark.parametrize("algo,order,prec", [("classical", "y", "c32"), ("precond", "y", "c32"),
                                             ("precond", "tuned", "c32"),
                                             ("precond", "y", "fp64")])
def test_converged_steps_match_monolithic(algo, order, prec):
    log(f"y-order converged steps {algo} {order} {prec}")
    osm = _osm()
    pb, u, W = smooth_problem()
    ref = run_monolithic(pb, u, W, 3, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo=algo, prec=prec, tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14, max_k=4000, strip_order=order)
    s.factor(to_dev(W))
    log(f"  order in use: {s.strip_order()}")
    ud = to_dev(u)
    for _ in range(3):
        st = s.step(ud)
        log(f"  k={st['k']} q={st['q_total']} gmres={st['gmres_total']}")
        # the fixed point refines the FP32-stored factors; nothing with FP64
        assert st["refine_total"] == (st["q_total"] if prec == "c32" else 0)
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "c32"])
def test_rotating_frame_refactor_every_step_matches_oracle(prec):
    log(f"y-order rotating frame {prec}")
    from oracle.rotating import step_potential
    from workloads import gaussian_boost
    osm = _osm()
    pb = Problem(-6.0, 6.0, -6.0, 6.0, 40, 71, 3, [12, 16, 12], lap_coef=0.5, beta=-20.0,
                 p=3.0, p_bc=3.0, dt=0.02, omega=-0.7, vxx=-0.5, vyy=-0.6)
    u0 = gaussian_boost(pb, k=0.5, a=0.5)
    steps = 4
    ref = run_monolithic(pb, u0, lambda n: step_potential(pb, n), steps, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo="precond", tol_k=1e-12, tol_k_relative=True, tol_q=1e-14,
                      strip_order="y", prec=prec)
    ud = to_dev(u0)
    for n in range(1, steps + 1):
        s.factor_rotating(n)
        s.step(ud)
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


def test_node_line_factor_is_not_served_in_y_order():
    osm = _osm()
    pb = problem(20, 16, (10, 10))
    W = potential(pb, 4)
    s = osm.OsmSolver(pb, DEV, strip_order="y")
    s.factor(to_dev(W))
    with pytest.raises(osm.OsmError) as e:
        s.get_factor()
    assert e.value.status == osm.OSM_ESTATE
    s.close()
    s = osm.OsmSolver(pb, DEV)
    s.factor(to_dev(W))
    with pytest.raises(osm.OsmError) as e:
        s.get_yfactor()
    assert e.value.status == osm.OSM_ESTATE
    s.close()
