"""GPU parity of the interface operators and of the random first interface
vector (Section 5, initial vectors) through the C ABI, against the FP64
oracle: g - R(g) (the right-hand side of eq. algo_pd), L_h g (eq. Lmpi,
free linear part of the Schwarz map), the seeded random g_1^0 bit for bit,
and Schwarz iterations started from it."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.schwarz import SchwarzOracle, random_interface  # noqa: E402
from oracle.step import run_monolithic  # noqa: E402
from workloads import Problem  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def problem(cells=(9, 12, 9), ncy=99, p=3.0, pbc=2.0, c=1.0, beta=4.0, dt=0.02):
    return Problem(-4.0, 4.0, -3.0, 3.0, sum(cells), ncy, len(cells), list(cells),
                   lap_coef=c, beta=beta, p=p, p_bc=pbc, dt=dt)


def state(pb, seed, amp=0.5):
    rng = np.random.default_rng(seed)
    s = (pb.ncx + 1, pb.ncy + 1)
    return amp * (rng.standard_normal(s) + 1j * rng.standard_normal(s)), rng.standard_normal(s)


def test_i_minus_r_matches_oracle():
    log("interface I - R")
    from paper_1603_05110_amd import osm
    pb = problem()
    u, W = state(pb, 14)
    orc = SchwarzOracle(pb, W, tol_q=1e-14)
    rng = np.random.default_rng(15)
    g = rng.standard_normal((4, pb.ncy + 1)) + 1j * rng.standard_normal((4, pb.ncy + 1))
    Rg, _, _ = orc.R(g, u)
    s = osm.OsmSolver(pb, DEV, tol_q=1e-14, warm_start=False)
    s.factor(to_dev(W))
    got = s.interface_apply(osm.OSM_IFACE_I_MINUS_R, to_dev(u), to_dev(g)).cpu().numpy()
    s.close()
    ref = g - Rg
    assert rel(got, ref) < 1e-11
    for t in range(g.shape[0]):     # every trace on its own
        assert rel(got[t], ref[t]) < 1e-10, t


@pytest.mark.parametrize("cells,prec", [((9, 12, 9), "fp64"), ((10, 10, 10, 10), "fp64"),
                                        ((7, 11, 8), "c32")])
def test_lh_apply_matches_oracle(cells, prec):
    """L_h is built in FP64 in both precisions (its inexactness would only
    slow the outer iteration), so both match the oracle's blocks applied to
    a random vector."""
    log(f"interface L_h {cells} {prec}")
    from paper_1603_05110_amd import osm
    pb = problem(cells=cells, ncy=70)
    orc = SchwarzOracle(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    orc.build_Lh()
    nt = 2 * (pb.nsub - 1)
    rng = np.random.default_rng(16)
    g = rng.standard_normal((nt, pb.ncy + 1)) + 1j * rng.standard_normal((nt, pb.ncy + 1))
    ref = orc.Lh_matvec(g.ravel()).reshape(g.shape)
    s = osm.OsmSolver(pb, DEV, algo="precond", prec=prec)
    got = s.interface_apply(osm.OSM_IFACE_LH, None, to_dev(g)).cpu().numpy()
    s.close()
    assert rel(got, ref) < 1e-12
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", [0, 1603])
def test_random_first_interface_vector_is_the_oracles(seed):
    """g1_init = 1: before the first step the interface holds the seeded
    SplitMix64 vector; the device generator and the oracle's give the same
    bits."""
    log(f"random g_1^0 seed {seed}")
    from paper_1603_05110_amd import osm
    pb = problem()
    s = osm.OsmSolver(pb, DEV, g1_init=1, seed=seed)
    g0 = s.get_interface().cpu().numpy()
    s.close()
    ref = random_interface(seed, (2 * (pb.nsub - 1), pb.ncy + 1))
    assert np.array_equal(g0, ref)


def test_fixed_iterations_from_the_random_start_match_oracle():
    log("fixed iterations from random g_1^0")
    from paper_1603_05110_amd import osm
    pb = problem()
    u, W = state(pb, 17)
    orc = SchwarzOracle(pb, W)
    g0 = random_interface(99, (2 * (pb.nsub - 1), pb.ncy + 1))
    res = orc.classical(u, g0, fixed_k=3, fixed_q=2)
    s = osm.OsmSolver(pb, DEV, fixed_k=3, fixed_q=2, warm_start=False, g1_init=1, seed=99)
    s.factor(to_dev(W))
    ud = to_dev(u)
    s.step(ud)
    g = s.get_interface().cpu().numpy()
    s.close()
    assert rel(g, res["g"]) < 1e-11
    assert rel(ud.cpu().numpy(), orc.assemble_global(res["vs"], u)) < 1e-11


@pytest.mark.parametrize("algo", ["classical", "precond"])
def test_random_start_converges_to_the_monolithic_step(algo):
    """Started from the random vector the iterations reach the same step as
    from zero (the converged answer does not depend on the start)."""
    log(f"converged from random g_1^0 {algo}")
    from paper_1603_05110_amd import osm
    from workloads import gaussian_boost
    # smooth data on which the classical iteration takes a few hundred
    # iterations per step (rough random data takes thousands)
    pb = Problem(-8.0, 8.0, -8.0, 8.0, 48, 63, 3, [15, 18, 15], lap_coef=0.5, beta=-5.0,
                 p=2.0, p_bc=2.0, dt=0.01)
    u = gaussian_boost(pb, k=1.0)
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    W = 0.5 * np.sin(X) * np.cos(Y)
    ref = run_monolithic(pb, u, W, 2, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo=algo, tol_k=1e-12, tol_k_relative=True, tol_q=1e-14,
                      max_k=5000, g1_init=1, seed=7)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(2):
        st = s.step(ud)
        log(f"  k={st['k']}")
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10
