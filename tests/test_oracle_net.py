"""Pins of the learned-guess oracle (oracle/nn.py) against things other than
itself: a library cross-correlation, central finite differences, the closed
form of Adam's first step, exact bfloat16 values and the exact inverse
relation between targets and guesses."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import nn
from workloads import Problem


def _theta(rng, scale=0.3):
    return rng.standard_normal(nn.NPARAM) * scale


def test_bf16_round_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even -> 1
    # 1 + 3 * 2^-9 lies above the midpoint -> 1 + 2^-7
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0,
                     3.0e38])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5, 0.0, 2.99e38])
    got = nn.bf16_round(vals)
    assert np.all(got[:6] == want[:6])
    assert abs(got[6] / 3.0e38 - 1) < 2.0 ** -8
    # every result has at most 8 significant bits
    rng = np.random.default_rng(0)
    r = nn.bf16_round(rng.standard_normal(1000))
    m, _ = np.frexp(r)
    assert np.all(np.abs(m * 256 - np.round(m * 256)) == 0)


def test_conv1d_matches_library_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, nn.CIN, 37))
    w = rng.standard_normal((5, nn.CIN, nn.KW))
    b = rng.standard_normal(5)
    y = nn.conv1d(x, w, b)
    for t in range(3):
        for o in range(5):
            ref = b[o] + sum(correlate(x[t, c], w[o, c], mode="same") for c in range(nn.CIN))
            assert np.allclose(y[t, o], ref, rtol=1e-13, atol=1e-13)


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(nn.gelu(x) - nn.gelu(-x), x, atol=1e-15)
    assert nn.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (nn.gelu(x + h) - nn.gelu(x - h)) / (2 * h)
    assert np.allclose(nn.gelu_grad(x), fd, atol=1e-9)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    theta = _theta(rng)
    x = rng.standard_normal((2, nn.CIN, 23))
    tgt = rng.standard_normal((2, nn.COUT, 23))
    loss, g = nn.loss_and_grad(theta, x, tgt)
    idx = rng.choice(nn.NPARAM, 60, replace=False)
    # every parameter block is probed
    bounds = np.cumsum([0] + [int(np.prod(s)) for s in nn.SHAPES])
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        idx = np.concatenate([idx, [lo, hi - 1]])
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn.loss_and_grad(tp, x, tgt)[0] - nn.loss_and_grad(tm, x, tgt)[0]) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-3), i


def test_adam_first_steps_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    opt = nn.Adam(np.zeros(3), lr=0.01)
    th = opt.step(g)
    # bias correction makes mhat = g and vhat = g^2 on the first step
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=0)
    g2 = np.array([1.0, 1.0, 1.0])
    th2 = opt.step(g2)
    m = 0.9 * 0.1 * g + 0.1 * g2
    v = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    step = 0.01 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(th2, th - step, rtol=1e-14, atol=1e-16)


def _pb(cells=(6, 7, 5)):
    return Problem(-2, 2, -1, 1, sum(cells), 20, len(cells), list(cells), lap_coef=1.0,
                   beta=1.0, p=2.0, p_bc=2.0, dt=0.01)


def test_features_targets_guess_are_consistent():
    pb = _pb()
    rng = np.random.default_rng(3)
    ntr, ny = 2 * (pb.nsub - 1), pb.ncy + 1
    g0, g1, g2 = (rng.standard_normal((ntr, ny)) + 1j * rng.standard_normal((ntr, ny))
                  for _ in range(3))
    W = 30.0 * rng.standard_normal((pb.ncx + 1, ny))
    x, s = nn.features(pb, g1, g2, W)
    # scaled inputs of g_{n-1} have unit mean square per trace
    assert np.allclose(np.mean(x[:, :4] ** 2, axis=(1, 2)) * 2, 1.0)
    assert np.max(np.abs(x[:, 8])) == pytest.approx(1.0)
    # potential channel taken on the interface line (first line of strip i+1)
    lines = nn.interface_lines(pb)
    assert lines == [6, 13]
    assert np.allclose(x[1, 8] * max(1.0, np.max(np.abs(W[13]))), W[13])
    # the guess built from the exact targets is the next interface vector
    y = nn.targets(g0, g1, g2, s)
    assert np.allclose(nn.guess(g1, g2, y, s), g0, rtol=1e-13, atol=1e-13)
    # zero output is linear extrapolation; on a sequence linear in n the
    # targets vanish
    assert np.allclose(nn.guess(g1, g2, np.zeros_like(y), s), 2 * g1 - g2)
    assert np.allclose(nn.targets(3 * g1 - 2 * g2, 2 * g1 - g2, g1, s), 0, atol=1e-14)
    # a zero trace gets scale 1
    g1z = g1.copy()
    g1z[0] = 0
    g1z[1] = 0
    _, sz = nn.features(pb, g1z, g2, W)
    assert sz[0] == 1.0
