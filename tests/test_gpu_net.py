"""GPU parity of the learned interface guess: the network's HIP forward,
gradient and Adam step against the FP64 oracle (oracle/nn.py) on the same
bf16-rounded parameters; the in-step feature extraction against the oracle's
features; and what the trained network gains over the paper's start
(the previous converged interface vector) on a held-out problem."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import nn  # noqa: E402
from oracle.step import run_monolithic  # noqa: E402
from workloads import c4_family, net_init, rng_for  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _net(theta, max_traces=64):
    from paper_1603_05110_amd import osm
    net = osm.OsmNet(max_traces, DEV)
    net.set_params(torch.from_numpy(theta))
    return net


def _data(T, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((T, nn.CIN, L)).astype(np.float32)
    t = (0.3 * rng.standard_normal((T, nn.COUT, L))).astype(np.float32)
    return x, t


@pytest.mark.parametrize("T,L", [(3, 150), (2, 5), (5, 1025)])
def test_forward_matches_oracle(T, L):
    """Tiles of 64 positions with a ragged tail (150), a trace shorter than
    the halo (5) and the C4 interface length (1025)."""
    log(f"net forward T={T} L={L}")
    theta = net_init(1) * 3.0
    net = _net(theta)
    x, _ = _data(T, L, 2)
    y = net.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    rounded = net.get_params(rounded=True).cpu().numpy().astype(np.float64)
    net.close()
    assert np.array_equal(rounded, nn.bf16_round(theta))
    ref, _ = nn.forward(rounded, x.astype(np.float64))
    assert rel(y, ref) < 1e-5


@pytest.mark.parametrize("T,L", [(4, 150), (3, 513)])
def test_loss_gradient_matches_oracle(T, L):
    log(f"net gradient T={T} L={L}")
    theta = net_init(2) * 3.0
    net = _net(theta)
    x, t = _data(T, L, 3)
    loss, g = net.loss_grad(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV))
    g = g.cpu().numpy()
    net.close()
    rl, rg = nn.loss_and_grad(nn.bf16_round(theta), x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - rl) < 1e-6 * rl
    assert rel(g, rg) < 1e-5
    # every parameter block individually
    o = 0
    for shp in nn.SHAPES:
        k = int(np.prod(shp))
        assert rel(g[o:o + k], rg[o:o + k]) < 1e-4
        o += k


def test_adam_step_matches_oracle():
    log("net adam")
    theta = net_init(3) * 2.0
    net = _net(theta)
    x, t = _data(4, 100, 4)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    lr = 1e-2
    loss0 = net.train_step(xd, td, lr)
    master = net.get_params().cpu().numpy().astype(np.float64)
    rounded = net.get_params(rounded=True).cpu().numpy().astype(np.float64)
    net.close()
    rl, rg = nn.loss_and_grad(nn.bf16_round(theta), x.astype(np.float64), t.astype(np.float64))
    assert abs(loss0 - rl) < 1e-6 * rl
    opt = nn.Adam(theta.astype(np.float64), lr=lr)
    want = opt.step(rg)
    # first Adam step moves each parameter by about lr: compare the move
    assert rel(master - theta, want - theta) < 1e-4
    # the bf16 copy is the rounding of the FP32 master
    assert np.array_equal(rounded, nn.bf16_round(master))


def _family(seed, ncells=64, nsub=4, steps=40):
    return c4_family(rng_for(4, salt=seed), ncells=ncells, nsub=nsub, steps=steps)


def _opts(guess=0):
    return dict(algo="precond", prec="fp64", tol_k=1e-12, tol_k_relative=True, tol_q=1e-14,
                tol_gmres=1e-4, eta_q=1e-2, guess=guess)


def test_features_match_oracle():
    from paper_1603_05110_amd import osm
    log("guess features")
    pb, u0, V = _family(7, steps=3)
    s = osm.OsmSolver(pb, DEV, **_opts())
    s.factor(torch.from_numpy(V).to(DEV))
    rng = np.random.default_rng(5)
    gs = [rng.standard_normal((2 * (pb.nsub - 1), pb.ncy + 1))
          + 1j * rng.standard_normal((2 * (pb.nsub - 1), pb.ncy + 1)) for _ in range(3)]
    gd = [torch.from_numpy(g).to(DEV) for g in gs]
    x, t = s.guess_features(gd[1], gd[2], gd[0])
    s.close()
    rx, sc = nn.features(pb, gs[1], gs[2], V)
    rt = nn.targets(gs[0], gs[1], gs[2], sc)
    assert rel(x.cpu().numpy(), rx) < 1e-7
    assert rel(t.cpu().numpy(), rt) < 1e-7


def _run(pb, u0, V, steps, guess, net=None, algo="precond"):
    from paper_1603_05110_amd import osm
    o = _opts(guess)
    if algo == "classical":
        o.update(algo="classical", eta_q=0.0, max_k=5000)
    s = osm.OsmSolver(pb, DEV, **o)
    if net is not None:
        s.set_guess_net(net)
    s.factor(torch.from_numpy(V).to(DEV))
    u = torch.from_numpy(u0).to(DEV)
    st = [s.step(u) for _ in range(steps)]
    s.close()
    return u.cpu().numpy(), st


def test_learned_guess_gains_over_previous_vector():
    """Train on traces of three family members (trap width w, beta seeded),
    then run a held-out member.  The network's prediction is closer to g_n
    than g_{n-1} is; with the classical algorithm, whose iteration count
    follows the distance of the start from the fixed point, it needs fewer
    Schwarz iterations than the paper's start; every answer is the oracle's.
    (The preconditioned iteration removes the linear part of the error in
    its first step whatever the start, so its count hardly moves.)"""
    from paper_1603_05110_amd import learned, osm
    log("learned guess gain")
    Xs, Ts = [], []
    for seed in (11, 12, 13):
        pb, u0, V = _family(seed)
        s = osm.OsmSolver(pb, DEV, **_opts())
        s.factor(torch.from_numpy(V).to(DEV))
        X, T, _ = learned.collect_traces(s, torch.from_numpy(u0).to(DEV), pb.steps)
        s.close()
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    log(f"  {X.shape[0]} traces of length {X.shape[2]}")
    net = osm.OsmNet(256, DEV)
    net.set_params(torch.from_numpy(net_init(0)))
    losses = learned.train(net, X, T, epochs=150, batch=64, lr=3e-3, seed=0)
    log(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.5 * losses[0]
    pb, u0, V = _family(99, steps=8)
    # prediction error against the converged vectors of the paper's run
    s = osm.OsmSolver(pb, DEV, **_opts())
    s.factor(torch.from_numpy(V).to(DEV))
    u = torch.from_numpy(u0).to(DEV)
    gs, r_nn, r_ex = [], [], []
    for n in range(pb.steps):
        s.step(u)
        gs.append(s.get_interface().clone())
        if len(gs) >= 3:
            g0, g1, g2 = (g.cpu().numpy() for g in (gs[-1], gs[-2], gs[-3]))
            x, _ = s.guess_features(gs[-2], gs[-3])
            y = net.forward(x).cpu().numpy().astype(np.float64)
            _, sc = nn.features(pb, g1, g2, V)
            gp = nn.guess(g1, g2, y, sc)
            r_nn.append(np.linalg.norm(g0 - gp) / np.linalg.norm(g0 - g1))
            r_ex.append(np.linalg.norm(g0 - (2 * g1 - g2)) / np.linalg.norm(g0 - g1))
    s.close()
    log(f"  |g_n - guess| / |g_n - g_n-1|: learned {np.mean(r_nn):.4f}, "
        f"extrapolated {np.mean(r_ex):.4f}")
    assert np.mean(r_nn) < 0.5
    ref = run_monolithic(pb, u0, V, pb.steps, tol_q=1e-14)
    k = {}
    for name, guess in [("previous", 0), ("learned", 2), ("extrapolated", 3)]:
        u_c, st = _run(pb, u0, V, pb.steps, guess, net if guess == 2 else None, "classical")
        assert rel(u_c, ref) < 1e-10, name
        k[name] = sum(x["k"] for x in st[2:])
        if guess == 2:
            assert sum(x["fallback_used"] for x in st) == 0
            # the library's own judge ratio agrees with the host's measure
            gr = [x["guess_ratio"] for x in st if x["guess_ratio"] > 0]
            log(f"  device guess ratio, learned: mean {np.mean(gr):.4f} over {len(gr)} steps")
            assert len(gr) == pb.steps - 2 and np.mean(gr) < 0.5
    log(f"  classical Schwarz iterations, steps 3..{pb.steps}: {k}")
    assert k["learned"] < k["previous"]
    assert np.mean(r_nn) < np.mean(r_ex)
    u_p, st_p = _run(pb, u0, V, pb.steps, 2, net)
    net.close()
    assert rel(u_p, ref) < 1e-10
    log(f"  preconditioned with the learned start: k = {[x['k'] for x in st_p]}")


def test_bad_network_falls_back_and_keeps_the_answer():
    from paper_1603_05110_amd import osm
    log("fallback")
    pb, u0, V = _family(21, steps=8)
    net = osm.OsmNet(16, DEV)
    net.set_params(torch.from_numpy(net_init(5) * 200.0))
    ref = run_monolithic(pb, u0, V, pb.steps, tol_q=1e-14)
    u, st = _run(pb, u0, V, pb.steps, 2, net)
    net.close()
    assert rel(u, ref) < 1e-10
    codes = [x["fallback_used"] for x in st]
    ratios = [x["guess_ratio"] for x in st]
    log(f"  fallback codes per step {codes}, guess ratios {[round(r, 3) for r in ratios]}")
    assert sum(c > 0 for c in codes) >= 1
    # a step restarted after its predicted start failed is followed by a
    # step that does not use the prediction
    for a, b in zip(codes, codes[1:]):
        if a == 2:
            assert b >= 1, codes
    # the judge: a prediction that ended farther from g_n than g_{n-1}
    # (ratio > 1) is not used on the next step, a closer one is
    for n in range(len(st) - 1):
        if ratios[n] > 0 and codes[n] != 2:
            assert (codes[n + 1] == 1) == (ratios[n] > 1.0), (n, ratios, codes)
