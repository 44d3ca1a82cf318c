"""The oracle's iteration counts against the paper's printed ones.

Section 5.1.3, Table Influence_p_NL_2_32: the first time step of the cubic
NLS on the first mesh (4097 x 129 nodes on (-16,16) x (-8,8), dt = 0.01,
u0 = exp(-x^2 - y^2 - 0.5 i x), f = |u|^2), zero first interface vector,
Robin transmission, stopping rule ||g^{k+1} - g^k||_2 < 1e-10 (Section 5).
The printed counts at p = 15 are 32 (classical) and 6 (preconditioned) for
N = 2, and 33 and 6 for N = 32.  The counts are pinned within +-20%: the
paper ran PETSc and Pardiso, whose rounding and GMRES settings are not
stated.  These are the only values the paper prints for the method's
convergence, so they pin the discretisation, the transmission update, the
Schwarz map and the preconditioner together.

The other table entries (p = 5 and 50, and the random first vector) take
several minutes each on one core; they run with OSM_FULL_PINS=1.
"""
import os

import numpy as np
import pytest

from oracle.schwarz import SchwarzOracle, random_interface
from workloads import nls_mesh1


def first_step_count(N, p, algo, start="zero"):
    wl = nls_mesh1(N, p)
    pb, u0, W = wl.problems[0], wl.u0[0], wl.V[0]
    orc = SchwarzOracle(pb, W, tol_q=1e-13)
    shape = (2 * (N - 1), pb.ncy + 1)
    g0 = np.zeros(shape, complex) if start == "zero" else random_interface(start, shape)
    # warm fixed-point starts change only the inner iterations, not the
    # Schwarz iterates (each inner fixed point is converged to 1e-13)
    if algo == "classical":
        r = orc.classical(u0, g0, tol=1e-10, relative=False, warm=True)
    else:
        r = orc.precond(u0, g0, tol=1e-10, relative=False, warm=True, gmres_rtol=1e-12)
    return r["k"]


def within(k, paper, frac=0.2):
    return abs(k - paper) <= frac * paper


def test_classical_count_mesh1_p15_32_strips():
    k = first_step_count(32, 15.0, "classical")
    assert within(k, 33), k


def test_preconditioned_count_mesh1_p15_2_strips():
    k = first_step_count(2, 15.0, "precond")
    assert within(k, 6), k


FULL = pytest.mark.skipif(os.environ.get("OSM_FULL_PINS") != "1",
                          reason="several minutes per entry; set OSM_FULL_PINS=1")


@FULL
@pytest.mark.slow
@pytest.mark.parametrize("N,p,algo,paper", [
    (2, 15.0, "classical", 32), (32, 15.0, "precond", 6),
    (2, 5.0, "classical", 57), (2, 5.0, "precond", 6),
    (2, 50.0, "classical", 73), (2, 50.0, "precond", 6),
])
def test_table_entries_zero_start(N, p, algo, paper):
    k = first_step_count(N, p, algo)
    assert within(k, paper), k


@FULL
@pytest.mark.slow
@pytest.mark.parametrize("algo,paper", [("classical", 227), ("precond", 6)])
def test_counts_from_a_random_start(algo, paper):
    """The random column of the table at p = 15, N = 2.  The paper does not
    state the random vector's distribution; with real and imaginary parts
    uniform on [0, 1) (PETSc's default for complex vectors) the oracle takes
    226 classical iterations against the printed 227."""
    k = first_step_count(2, 15.0, algo, start=1)
    assert within(k, paper), k
