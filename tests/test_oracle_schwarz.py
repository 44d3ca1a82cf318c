"""Pins of the oracle's Schwarz iteration: converged Schwarz equals the
monolithic solve, the free map is affine with linear part L_h, the block
structure of Proposition 3.1, and the preconditioned iteration converges in
one outer step when P = I - L_h is exact."""
import numpy as np
import pytest

from oracle.schwarz import SchwarzOracle, gmres, run_schwarz
from oracle.step import run_monolithic
from workloads import Problem, equal_strips


def prob(ncx=24, ncy=10, nsub=3, cells=None, beta=5.0, p=3.0, pbc=3.0, c=1.0,
         dt=0.02):
    return Problem(-4, 4, -2, 2, ncx, ncy, nsub,
                   cells if cells is not None else equal_strips(ncx, nsub),
                   lap_coef=c, beta=beta, p=p, p_bc=pbc, dt=dt)


def data(pb, seed):
    rng = np.random.default_rng(seed)
    s = (pb.ncx + 1, pb.ncy + 1)
    u = 0.5 * (rng.standard_normal(s) + 1j * rng.standard_normal(s))
    W = rng.standard_normal(s)
    return u, W


@pytest.mark.parametrize("cells,c,pbc", [(None, 1.0, 3.0), ([5, 11, 8], 0.5, 0.0),
                                          ([4, 4, 9, 7], 1.0, 1.0)])
@pytest.mark.parametrize("algo", ["classical", "precond"])
def test_converged_schwarz_equals_monolithic(cells, c, pbc, algo):
    nsub = 3 if cells is None else len(cells)
    pb = prob(nsub=nsub, cells=cells, c=c, pbc=pbc)
    u, W = data(pb, 1)
    ref = run_monolithic(pb, u, W, 2, tol_q=1e-14)
    got, _, stats, _ = run_schwarz(pb, u, W, 2, algo=algo, tol=1e-13,
                                   relative=True, tol_q=1e-14)
    assert np.linalg.norm(got - ref) < 1e-11 * np.linalg.norm(ref)


def test_free_map_is_affine_with_linear_part_Lh():
    pb = prob(beta=0.0, cells=[6, 10, 8])
    u, _ = data(pb, 2)
    W0 = np.zeros_like(u, dtype=float)
    orc = SchwarzOracle(pb, W0)
    orc.build_Lh()
    rng = np.random.default_rng(3)
    g = rng.standard_normal((4, pb.ncy + 1)) + 1j * rng.standard_normal((4, pb.ncy + 1))
    R0, _, _ = orc.R(np.zeros_like(g), u)
    Rg, _, _ = orc.R(g, u)
    lin = orc.Lh_matvec(g.ravel()).reshape(g.shape)
    assert np.max(np.abs((Rg - R0) - lin)) < 1e-12 * np.max(np.abs(lin))


def test_prop31_equal_strips_give_four_distinct_blocks():
    pb = prob(ncx=30, nsub=5, beta=0.0)
    orc = SchwarzOracle(pb, np.zeros((31, 11)))
    B = orc.build_Lh()
    ny = pb.ncy + 1
    # rows: 2i = new r_i (from strip i+1), 2i+1 = new l_{i+1} (from strip i)
    X1 = [B[(2 * (j - 1), 2 * (j - 1) + 1)] for j in range(1, 5)]
    X2 = [B[(2 * (j - 1), 2 * j)] for j in range(1, 4)]
    X3 = [B[(2 * j + 1, 2 * (j - 1) + 1)] for j in range(1, 4)]
    X4 = [B[(2 * j + 1, 2 * j)] for j in range(0, 4)]
    for fam in (X1, X2, X3, X4):
        for X in fam[1:]:
            assert np.max(np.abs(X - fam[0])) < 1e-12
    # mirror symmetry of a strip with equal Robin parameters on both edges
    assert np.max(np.abs(X1[0] - X4[0])) < 1e-12
    assert np.max(np.abs(X2[0] - X3[0])) < 1e-12
    assert X1[0].shape == (ny, ny)


def test_free_linear_preconditioned_converges_in_one_step():
    pb = prob(beta=0.0, cells=[7, 9, 8])
    u, _ = data(pb, 4)
    orc = SchwarzOracle(pb, np.zeros(u.shape))
    res = orc.precond(u, np.zeros((4, pb.ncy + 1), complex), tol=1e-11,
                      relative=True, pinv="direct")
    assert res["k"] <= 2
    # after the first outer step the increment is at rounding level
    res1 = orc.precond(u, np.zeros((4, pb.ncy + 1), complex), fixed_k=1,
                       pinv="direct")
    Rg, _, _ = orc.R(res1["g"], u)
    assert np.linalg.norm(Rg - res1["g"]) < 1e-11 * np.linalg.norm(res1["g"])


def test_gmres_matches_direct_solve():
    pb = prob(beta=0.0, cells=[7, 9, 8])
    orc = SchwarzOracle(pb, np.zeros((25, 11)))
    orc.build_Lh()
    rng = np.random.default_rng(5)
    y = rng.standard_normal(44) + 1j * rng.standard_normal(44)
    P = np.eye(44) - orc.Lh_dense()
    x, it = gmres(lambda z: z - orc.Lh_matvec(z), y, rtol=1e-13)
    assert np.linalg.norm(x - np.linalg.solve(P, y)) < 1e-11 * np.linalg.norm(x)
    assert it > 0
    # one restart cycle that reaches the tolerance returns without a second
    # cycle: the residual estimate of the rotated Hessenberg system is exact
    x1, it1 = gmres(lambda z: z - orc.Lh_matvec(z), y, rtol=1e-10, restart=44)
    assert it1 <= 44
    assert np.linalg.norm(y - (x1 - orc.Lh_matvec(x1))) < 1e-9 * np.linalg.norm(y)


def test_gmres_on_a_complex_nonnormal_matrix():
    """Dense complex test matrix with known solution: the least-squares
    residual tracked by the rotations equals the true residual."""
    rng = np.random.default_rng(11)
    n = 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    xs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = gmres(lambda z: A @ z, A @ xs, rtol=1e-12, restart=n)
    assert it < n
    assert np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)


def test_warm_start_and_forms_do_not_change_the_answer():
    pb = prob(cells=[7, 9, 8])
    u, W = data(pb, 6)
    a, _, _, _ = run_schwarz(pb, u, W, 1, tol=1e-13, relative=True, tol_q=1e-14)
    b, _, _, _ = run_schwarz(pb, u, W, 1, tol=1e-13, relative=True, tol_q=1e-14,
                             warm=True)
    c, _, _, _ = run_schwarz(pb, u, W, 1, tol=1e-13, relative=True, tol_q=1e-14,
                             form="A")
    assert np.linalg.norm(a - b) < 1e-11 * np.linalg.norm(a)
    assert np.linalg.norm(a - c) < 1e-11 * np.linalg.norm(a)


def test_preconditioner_cuts_iterations():
    """Qualitative claim of Section 5.1 (Tables 1 and 3): the preconditioned
    algorithm needs far fewer outer iterations than the classical one."""
    pb = prob(ncx=32, nsub=4, beta=1.0, p=2.0, pbc=2.0, dt=0.01)
    u, _ = data(pb, 7)
    W = np.zeros(u.shape)
    _, _, sc, _ = run_schwarz(pb, u, W, 1, algo="classical", tol=1e-10)
    _, _, sp_, _ = run_schwarz(pb, u, W, 1, algo="precond", tol=1e-10)
    assert sp_[0]["k"] * 3 < sc[0]["k"]


def test_random_interface_generator_matches_published_splitmix64():
    """The random first interface vector (Section 5, initial vectors) is
    drawn from SplitMix64; its outputs must be the generator's published
    test values (seed 0, and seed 1234567), and the derived uniforms must
    have the mean and variance of U[0, 1)."""
    from oracle.schwarz import random_interface, splitmix64
    got0 = [int(v) for v in splitmix64(0, np.arange(4))]
    assert got0 == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                    0xF88BB8A8724C81EC]
    got1 = [int(v) for v in splitmix64(1234567, np.arange(5))]
    assert got1 == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                    4593380528125082431, 16408922859458223821]
    g = random_interface(42, (6, 20001))
    for part in (g.real, g.imag):
        assert part.min() >= 0.0 and part.max() < 1.0
        n = part.size
        assert abs(part.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
        assert abs(part.var() - 1 / 12) < 0.002
    # entry k takes outputs 2k (real part) and 2k + 1 (imaginary part)
    first = splitmix64(42, np.arange(2)) >> np.uint64(11)
    assert g[0, 0] == complex(float(first[0]) * 2.0 ** -53, float(first[1]) * 2.0 ** -53)


def test_bicgstab_matches_dense_solve():
    """BiCGStab (the other Krylov method Section 4.2 names for P x = y)
    against a dense solve: a complex non-normal system and P = I - L_h of a
    small strip problem."""
    from oracle.schwarz import bicgstab
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = bicgstab(lambda v: A @ v, b, rtol=1e-13)
    assert it < n
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-11 * np.linalg.norm(x)
    pb = Problem(-2.0, 2.0, -1.0, 1.0, 12, 9, 3, [4, 5, 3], lap_coef=1.0, beta=0.0, p=2.0,
                 p_bc=2.0, dt=0.05)
    orc = SchwarzOracle(pb, np.zeros((13, 10)))
    orc.build_Lh()
    P = np.eye(4 * 10) - orc.Lh_dense()
    y = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    x, _ = bicgstab(lambda v: v - orc.Lh_matvec(v), y, rtol=1e-13)
    assert np.linalg.norm(x - np.linalg.solve(P, y)) < 1e-11 * np.linalg.norm(x)


def test_interface_krylov_solves_the_linear_step():
    """f = 0: R is affine, so GMRES on (I - L) g = d with Schwarz-map products
    reaches the monolithic step (and the classical iteration's limit), with
    a non-zero potential and uneven strips."""
    from oracle.schwarz import interface_krylov
    from oracle.step import run_monolithic
    pb = Problem(-3.0, 3.0, -2.0, 2.0, 18, 15, 3, [5, 7, 6], lap_coef=0.5, beta=0.0, p=2.0,
                 p_bc=1.5, dt=0.02)
    rng = np.random.default_rng(11)
    s = (19, 16)
    u = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    W = rng.standard_normal(s)
    ref = run_monolithic(pb, u, W, 1, tol_q=1e-14)
    orc = SchwarzOracle(pb, W, tol_q=1e-14)
    g0 = np.zeros((4, 16), complex)
    res = interface_krylov(orc, u, g0, tol=1e-13, relative=True)
    got = orc.assemble_global(res["vs"], u)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11
    cls = orc.classical(u, g0, tol=1e-14, relative=True)
    assert np.linalg.norm(res["g"] - cls["g"]) < 1e-10 * np.linalg.norm(cls["g"])
    assert res["gmres_total"] < cls["k"]
