"""GPU parity of batched instances (independent problems of different mesh
sizes, strip layouts, Robin parameters and potentials solved together)
against the FP64 oracle, instance by instance."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.schwarz import SchwarzOracle  # noqa: E402
from oracle.step import run_monolithic  # noqa: E402
from workloads import (Problem, c3, dirichlet_strips, gaussian_boost,  # noqa: E402
                       gaussian_bumps_potential, rng_for)

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def mixed_batch(sizes=((24, 48, (6, 8, 10)), (30, 99, (9, 12, 9)), (16, 128, (8, 8)),
                       (40, 70, (4, 9, 7, 11, 9)))):
    """Instances of different ny (49 .. 129, ragged against 64-wide tiles),
    strip counts and uneven widths, p in [1, 10], smooth random potentials."""
    rng = rng_for(3, salt=11)
    pbs, us, Ws = [], [], []
    for i, (ncx, ncy, cells) in enumerate(sizes):
        p = float(rng.uniform(1.0, 10.0))
        pb = Problem(-10, 10, -10, 10, ncx, ncy, len(cells), list(cells), lap_coef=1.0,
                     beta=1.0, p=p, p_bc=p, dt=0.01, name=f"mixed-{i}")
        Ws.append(gaussian_bumps_potential(pb, rng))
        us.append(gaussian_boost(pb, k=1.0))
        pbs.append(pb)
    return pbs, us, Ws


def test_batch_fixed_iteration_matches_oracle():
    """Same (k, q) counts and cold fixed-point starts in every instance:
    rounding-level agreement of the iteration with the sequential oracle."""
    from paper_1603_05110_amd import osm
    log("batch fixed iteration")
    pbs, us, Ws = mixed_batch()
    b = osm.OsmBatch(pbs, DEV, fixed_k=3, fixed_q=2, warm_start=False)
    b.factor([to_dev(W) for W in Ws])
    ud = [to_dev(u) for u in us]
    st = b.step(ud)
    log(f"  tuning {b.tuning()}")
    b.close()
    for i, pb in enumerate(pbs):
        orc = SchwarzOracle(pb, Ws[i])
        g0 = np.zeros((2 * (pb.nsub - 1), pb.ncy + 1), complex)
        res = orc.classical(us[i], g0, fixed_k=3, fixed_q=2)
        unew = orc.assemble_global(res["vs"], us[i])
        assert st[i]["k"] == 3 and st[i]["q_total"] == 6
        assert rel(ud[i].cpu().numpy(), unew) < 1e-11, i


@pytest.mark.parametrize("prec", ["fp64", "c32"])
def test_batch_converged_steps_match_monolithic(prec):
    from paper_1603_05110_amd import osm
    log(f"batch converged {prec}")
    pbs, us, Ws = mixed_batch()
    steps = 2
    refs = [run_monolithic(pb, u, W, steps, tol_q=1e-14) for pb, u, W in zip(pbs, us, Ws)]
    b = osm.OsmBatch(pbs, DEV, prec=prec, tol_k=1e-12, tol_k_relative=True, tol_q=1e-14,
                     max_k=4000)
    b.factor([to_dev(W) for W in Ws])
    ud = [to_dev(u) for u in us]
    for _ in range(steps):
        st = b.step(ud)
        log("  k " + " ".join(str(s["k"]) for s in st))
    b.close()
    for i in range(len(pbs)):
        assert rel(ud[i].cpu().numpy(), refs[i]) < 1e-10, i


def test_batch_equals_instances_run_alone():
    """The batch replays a fixed graph until every instance has met its own
    test; an instance that converges early is frozen, so each result equals
    the single-instance path's to the iteration tolerance."""
    from paper_1603_05110_amd import osm
    log("batch vs single")
    pbs, us, Ws = mixed_batch()
    opts = dict(tol_k=1e-12, tol_k_relative=True, tol_q=1e-14, max_k=4000)
    b = osm.OsmBatch(pbs, DEV, **opts)
    b.factor([to_dev(W) for W in Ws])
    ud = [to_dev(u) for u in us]
    st = b.step(ud)
    b.close()
    for i, pb in enumerate(pbs):
        s = osm.OsmSolver(pb, DEV, **opts)
        s.factor(to_dev(Ws[i]))
        u1 = to_dev(us[i])
        s1 = s.step(u1)
        s.close()
        assert abs(s1["k"] - st[i]["k"]) <= 1
        assert rel(ud[i].cpu().numpy(), u1.cpu().numpy()) < 1e-11, i


@pytest.mark.parametrize("prec", ["fp64", "c32"])
def test_preconditioned_batch_matches_monolithic(prec):
    """The preconditioned algorithm (eq. algo_pd) per instance of a batch:
    every instance's L_h of its own strip classes, its GMRES on P x = y
    inside the replayed chunk and, when a chunk is not enough, continued by
    the host; two converged steps against the monolithic oracle."""
    from paper_1603_05110_amd import osm
    log(f"preconditioned batch {prec}")
    pbs, us, Ws = mixed_batch()
    steps = 2
    refs = [run_monolithic(pb, u, W, steps, tol_q=1e-14) for pb, u, W in zip(pbs, us, Ws)]
    b = osm.OsmBatch(pbs, DEV, algo="precond", prec=prec, tol_k=1e-12, tol_k_relative=True,
                     tol_q=1e-14, max_k=200, tol_gmres=1e-2)
    b.factor([to_dev(W) for W in Ws])
    ud = [to_dev(u) for u in us]
    for _ in range(steps):
        st = b.step(ud)
        log("  k " + " ".join(str(s["k"]) for s in st) + ", GMRES " +
            " ".join(str(s["gmres_total"]) for s in st))
    b.close()
    for i in range(len(pbs)):
        assert rel(ud[i].cpu().numpy(), refs[i]) < 1e-10, i
        assert st[i]["gmres_total"] > 0


def test_preconditioned_batch_equals_instances_run_alone():
    """Each preconditioned instance of the batch takes the single-instance
    path's iterations (within one) and reaches its answer; both take far
    fewer Schwarz iterations than the classical batch."""
    from paper_1603_05110_amd import osm
    log("preconditioned batch vs single")
    pbs, us, Ws = mixed_batch()
    opts = dict(tol_k=1e-12, tol_k_relative=True, tol_q=1e-14, max_k=4000, tol_gmres=1e-2)
    b = osm.OsmBatch(pbs, DEV, algo="precond", **opts)
    b.factor([to_dev(W) for W in Ws])
    ud = [to_dev(u) for u in us]
    st = b.step(ud)
    b.close()
    bc = osm.OsmBatch(pbs, DEV, **opts)
    bc.factor([to_dev(W) for W in Ws])
    stc = bc.step([to_dev(u) for u in us])
    bc.close()
    for i, pb in enumerate(pbs):
        s = osm.OsmSolver(pb, DEV, algo="precond", **opts)
        s.factor(to_dev(Ws[i]))
        u1 = to_dev(us[i])
        s1 = s.step(u1)
        s.close()
        log(f"  instance {i}: batch k {st[i]['k']}, alone {s1['k']}, classical {stc[i]['k']}")
        assert abs(s1["k"] - st[i]["k"]) <= 1
        assert st[i]["k"] < stc[i]["k"]
        assert rel(ud[i].cpu().numpy(), u1.cpu().numpy()) < 1e-10, i


def _edge_term(pb, u_old, u_new):
    """v* M^Gamma_d v over the two physical x-edges, v = (u_n + u_{n-1})/2."""
    hy = pb.hy
    n = pb.ncy + 1
    M1 = np.diag(np.full(n, 4 * hy / 6)) + np.diag(np.full(n - 1, hy / 6), 1) \
        + np.diag(np.full(n - 1, hy / 6), -1)
    M1[0, 0] = M1[-1, -1] = 2 * hy / 6
    v = 0.5 * (u_old + u_new)
    return float(np.real(np.conj(v[0]) @ M1 @ v[0] + np.conj(v[-1]) @ M1 @ v[-1]))


def test_c3_batch_full_size():
    """The 64-instance batch at full size (grids 256..768, 8-32 uneven
    strips), one complex-FP32 step: one instance of every grid size and the
    slowest instance against the monolithic FP64 oracle (relative L2 and
    largest entry error of each), and the discrete mass identity of the
    scheme in every instance (mass change = -2 c p dt v* M^Gamma v, exact at
    convergence).  The slowest instance runs the step's last launches alone,
    with the largest re-planned teams."""
    from paper_1603_05110_amd import osm
    log("C3 full batch, 1 step c32")
    wl = c3()
    pbs = wl.problems
    b = osm.OsmBatch(pbs, DEV, prec="c32", tol_k=1e-12, tol_k_relative=True, tol_q=1e-14,
                     max_k=4000)
    b.factor([to_dev(W) for W in wl.V])
    log(f"  tuning {b.tuning()}")
    ud = [to_dev(u) for u in wl.u0]
    st = b.step(ud)
    b.close()
    ks = [s["k"] for s in st]
    log(f"  k min {min(ks)} max {max(ks)} mean {np.mean(ks):.1f}")
    got = [u.cpu().numpy() for u in ud]
    del ud
    for i, pb in enumerate(pbs):
        d_mass = st[i]["mass_after"] - st[i]["mass_before"]
        rhs = -2.0 * pb.lap_coef * pb.p_bc * pb.dt * _edge_term(pb, wl.u0[i], got[i])
        assert abs(d_mass - rhs) < 1e-11 * st[i]["mass_before"], i
    picks = {}
    for i, pb in enumerate(pbs):
        picks.setdefault(pb.ncx, i)
    slowest = int(np.argmax(ks))
    check = sorted(set(picks.values()) | {slowest})
    for i in check:
        pb = pbs[i]
        ref = run_monolithic(pb, wl.u0[i], wl.V[i], 1, tol_q=1e-14)
        e = rel(got[i], ref)
        mx = float(np.max(np.abs(got[i] - ref)) / np.max(np.abs(ref)))
        log(f"  instance {i}: {pb.ncx}^2, {pb.nsub} strips, k {ks[i]}: rel L2 {e:.3e}, "
            f"max-abs {mx:.3e}")
        assert e < 1e-10 and mx < 1e-10, i
