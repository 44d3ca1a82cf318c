"""GPU parity of the S_pade^m transmission condition (Section 2.1, eqs. TCS,
TCS_phi; Section 2.2, eq. NproblemSPNL; Proposition 3.2) through the C ABI
against the FP64 oracle (oracle/pade.py): the strip solve of the eliminated
arrow system, fixed iterations of the classical algorithm, converged steps
of both algorithms against the monolithic solve, and the L_h blocks."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.pade import PadeSchwarz, PadeStrip, pade_monolithic  # noqa: E402
from workloads import Problem  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def problem(cells=(5, 7, 6), ncy=70, m=6, beta=2.0, c=0.5, dt=0.02):
    return Problem(-3.0, 3.0, -2.0, 2.0, sum(cells), ncy, len(cells), list(cells),
                   lap_coef=c, beta=beta, p=0.0, p_bc=0.0, dt=dt, tc="pade", pade_m=m)


def state(pb, seed, amp=0.4):
    rng = np.random.default_rng(seed)
    s = (pb.ncx + 1, pb.ncy + 1)
    return amp * (rng.standard_normal(s) + 1j * rng.standard_normal(s)), rng.standard_normal(s)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("c32", 2e-5)])
@pytest.mark.parametrize("ncy,m", [(70, 6), (129, 20)])
def test_strip_solve_with_pade_edges_matches_oracle(prec, tol, ncy, m):
    """K_eff^{-1} b per strip, K_eff the strip operator with the edge
    functions eliminated: the zeta part of the oracle's arrow solve with
    right-hand side (b, 0)."""
    log(f"pade strip solve {prec} ny={ncy + 1} m={m}")
    from paper_1603_05110_amd import osm
    pb = problem(ncy=ncy, m=m)
    _, W = state(pb, 3)
    orc = PadeSchwarz(pb, W)
    rng = np.random.default_rng(4)
    bs, ref = [], []
    for j, c in enumerate(pb.strip_cells):
        st = orc.strips[j]
        b = rng.standard_normal((c + 1, ncy + 1)) + 1j * rng.standard_normal((c + 1, ncy + 1))
        x = st.lu.solve(np.concatenate([b.ravel(), np.zeros(2 * st.m * st.ny)]))[:st.nz]
        bs.append(b)
        ref.append(x.reshape(b.shape))
    s = osm.OsmSolver(pb, DEV, prec=prec)
    s.factor(to_dev(W))
    x = s.strip_solve(to_dev(np.concatenate(bs))).cpu().numpy()
    s.close()
    want = np.concatenate(ref)
    assert rel(x, want) < tol
    o = 0
    for j, c in enumerate(pb.strip_cells):
        assert rel(x[o:o + c + 1], want[o:o + c + 1]) < tol, j
        o += c + 1


@pytest.mark.parametrize("fixed_k,fixed_q", [(1, 1), (3, 2)])
def test_fixed_iterations_with_pade_match_oracle(fixed_k, fixed_q):
    """Same (k, q) counts from zeta^0 = u_{n-1}, phi^0 = 0: the residual form
    with the edge functions as extra unknowns reproduces the oracle's
    iterates (the nonlinearity on the right, eq. NproblemSPNL)."""
    log(f"pade fixed iterations k={fixed_k} q={fixed_q}")
    from paper_1603_05110_amd import osm
    pb = problem()
    u, W = state(pb, 5)
    orc = PadeSchwarz(pb, W)
    g0 = np.zeros((2 * (pb.nsub - 1), pb.ncy + 1), complex)
    res = orc.classical(u, g0, fixed_k=fixed_k, fixed_q=fixed_q)
    s = osm.OsmSolver(pb, DEV, fixed_k=fixed_k, fixed_q=fixed_q, warm_start=False)
    s.factor(to_dev(W))
    ud = to_dev(u)
    s.step(ud)
    g = s.get_interface().cpu().numpy()
    s.close()
    assert rel(g, res["g"]) < 1e-11
    assert rel(ud.cpu().numpy(), orc.assemble_global(res["vs"], u)) < 1e-11


@pytest.mark.parametrize("algo,prec", [("classical", "fp64"), ("precond", "fp64"),
                                       ("precond", "c32")])
def test_converged_pade_steps_match_monolithic(algo, prec):
    log(f"pade converged steps {algo} {prec}")
    from paper_1603_05110_amd import osm
    pb = problem(cells=(6, 8, 7, 6), ncy=63, m=8, beta=-4.0)
    u, W = state(pb, 7, amp=0.3)
    W = 0.3 * W
    ref = pade_monolithic(pb, u, W, 2, tol_q=1e-14)
    s = osm.OsmSolver(pb, DEV, algo=algo, prec=prec, tol_k=1e-12, tol_k_relative=True,
                      tol_q=1e-14, max_k=3000)
    s.factor(to_dev(W))
    ud = to_dev(u)
    for _ in range(2):
        st = s.step(ud)
        log(f"  k={st['k']} q={st['q_total']} gmres={st['gmres_total']}")
    s.close()
    assert rel(ud.cpu().numpy(), ref) < 1e-10


def test_pade_lh_blocks_match_oracle():
    """Proposition 3.2: the four blocks of every strip, against the oracle's
    L_h assembled column by column from the free problem."""
    log("pade L_h blocks")
    from paper_1603_05110_amd import osm
    pb = problem(cells=(5, 6, 5), ncy=40, m=5)
    orc = PadeSchwarz(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    L = orc.build_Lh()
    s = osm.OsmSolver(pb, DEV, algo="precond")
    blk = s.get_lh_blocks().cpu().numpy()
    s.close()
    ny = pb.ncy + 1
    B = lambda r, c: L[r * ny:(r + 1) * ny, c * ny:(c + 1) * ny]
    N = pb.nsub
    for j in range(N):
        if j >= 1:
            assert rel(blk[j, 0], B(2 * (j - 1), 2 * (j - 1) + 1)) < 1e-11
        if 1 <= j <= N - 2:
            assert rel(blk[j, 1], B(2 * (j - 1), 2 * j)) < 1e-11
            assert rel(blk[j, 2], B(2 * j + 1, 2 * (j - 1) + 1)) < 1e-11
        if j <= N - 2:
            assert rel(blk[j, 3], B(2 * j + 1, 2 * j)) < 1e-11
