"""Learned interface guess: FP64 reference of the network, its features,
its loss gradient and its optimiser.

Oracle code (test infrastructure).  The paper starts each time step's
Schwarz iteration from the converged interface vector of the previous step
(Section 5, initial vectors).  The learned guess replaces that start by a
prediction from the last two converged vectors, corrected by a small 1-D
convolutional network; the converged solve is unchanged (the Schwarz fixed
point does not depend on its start), only the iteration count can change.

Per interface i (between strips i and i+1), along the ny nodes of the
interface line:

* scale s_i = sqrt( (sum |r_i^{n-1}|^2 + sum |l_{i+1}^{n-1}|^2) / (2 ny) ),
  or 1 when that is zero;
* input channels (9): Re r, Im r, Re l, Im l of g_{n-1}, the same of g_{n-2}
  (all divided by s_i), and W_n on the interface line divided by
  max(1, max |W_n| on that line);
* output channels (4): Re, Im of the part of the change that linear
  extrapolation misses, (r_i^n - 2 r_i^{n-1} + r_i^{n-2}) / s_i, and the same
  for l_{i+1}; the guess is g^{NN} = 2 g_{n-1} - g_{n-2} + s_i * output, so an
  untrained network (output near zero) starts from linear extrapolation;
* network: conv1d(9 -> 64, kernel 5, zero padding 2) -> GELU (exact, with
  erf) -> conv1d(64 -> 4, kernel 5, zero padding 2); cross-correlation
  convention y[o, a] = b[o] + sum_{c, k} w[o, c, k] x[c, a + k - 2];
* weights and biases are held in bfloat16 (round to nearest even from the
  float32 master copy); the arithmetic here is FP64 on those values;
* loss: mean squared error over every output value of a batch;
* optimiser: Adam (Kingma & Ba) with bias correction.

Parameters are one flat vector in the order W1 (64, 9, 5), b1 (64),
W2 (4, 64, 5), b2 (4): 4228 values.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

CIN, HID, COUT, KW = 9, 64, 4, 5
PAD = KW // 2
SHAPES = [(HID, CIN, KW), (HID,), (COUT, HID, KW), (COUT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unflatten(theta: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def flatten(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def bf16_round(a) -> np.ndarray:
    """Values of float32(a) rounded to bfloat16 (8-bit significand), round to
    nearest, ties to even, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def conv1d(x, w, b):
    """x (T, C, L), w (O, C, K), b (O,) -> (T, O, L), zero padding K//2."""
    T, C, L = x.shape
    O, _, K = w.shape
    xp = np.zeros((T, C, L + 2 * PAD))
    xp[:, :, PAD:PAD + L] = x
    y = np.zeros((T, O, L)) + b[None, :, None]
    for k in range(K):
        y += np.einsum("oc,tcl->tol", w[:, :, k], xp[:, :, k:k + L])
    return y


def forward(theta, x):
    """Returns the output (T, 4, L) and the cache of the hidden layer."""
    W1, b1, W2, b2 = unflatten(theta)
    h = conv1d(x, W1, b1)
    z = gelu(h)
    y = conv1d(z, W2, b2)
    return y, (x, h, z)


def loss_and_grad(theta, x, target):
    """MSE over all outputs and its gradient with respect to theta."""
    W1, b1, W2, b2 = unflatten(theta)
    y, (x, h, z) = forward(theta, x)
    n = y.size
    loss = float(np.sum((y - target) ** 2) / n)
    dy = 2.0 * (y - target) / n
    T, _, L = y.shape
    # second layer
    zp = np.zeros((T, HID, L + 2 * PAD))
    zp[:, :, PAD:PAD + L] = z
    dW2 = np.zeros_like(W2)
    for k in range(KW):
        dW2[:, :, k] = np.einsum("tol,tcl->oc", dy, zp[:, :, k:k + L])
    db2 = dy.sum(axis=(0, 2))
    # back through the second convolution: dz[c, a] = sum_{o,k} W2[o,c,k] dy[o, a-k+PAD]
    dyp = np.zeros((T, COUT, L + 2 * PAD))
    dyp[:, :, PAD:PAD + L] = dy
    dz = np.zeros((T, HID, L))
    for k in range(KW):
        dz += np.einsum("oc,tol->tcl", W2[:, :, k], dyp[:, :, 2 * PAD - k:2 * PAD - k + L])
    dh = dz * gelu_grad(h)
    xp = np.zeros((T, CIN, L + 2 * PAD))
    xp[:, :, PAD:PAD + L] = x
    dW1 = np.zeros_like(W1)
    for k in range(KW):
        dW1[:, :, k] = np.einsum("tcl,til->ci", dh, xp[:, :, k:k + L])
    db1 = dh.sum(axis=(0, 2))
    return loss, flatten([dW1, db1, dW2, db2])


class Adam:
    """theta <- theta - lr * mhat / (sqrt(vhat) + eps) on the float master
    parameters; the network uses bf16_round(theta)."""

    def __init__(self, theta, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.theta = np.array(theta, dtype=np.float64)
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.theta


def interface_lines(pb):
    """Global x node-line of every interface (the first line of strip i+1)."""
    starts = np.concatenate([[0], np.cumsum(pb.strip_cells)])
    return [int(starts[i + 1]) for i in range(pb.nsub - 1)]


def features(pb, g1, g2, W):
    """Inputs (N-1, 9, ny) and scales (N-1,) from g_{n-1} = g1, g_{n-2} = g2
    (interface layout (2(N-1), ny)) and the nodal potential W_n."""
    N = pb.nsub
    ny = pb.ncy + 1
    x = np.zeros((N - 1, CIN, ny))
    s = np.ones(N - 1)
    lines = interface_lines(pb)
    for i in range(N - 1):
        r1, l1 = g1[2 * i], g1[2 * i + 1]
        r2, l2 = g2[2 * i], g2[2 * i + 1]
        e = (np.sum(np.abs(r1) ** 2) + np.sum(np.abs(l1) ** 2)) / (2 * ny)
        si = np.sqrt(e) if e > 0 else 1.0
        s[i] = si
        for c, v in enumerate([r1.real, r1.imag, l1.real, l1.imag,
                               r2.real, r2.imag, l2.real, l2.imag]):
            x[i, c] = v / si
        wl = np.asarray(W[lines[i]], dtype=np.float64)
        x[i, 8] = wl / max(1.0, float(np.max(np.abs(wl))))
    return x, s


def targets(g0, g1, g2, s):
    """Outputs (N-1, 4, ny) the network is trained to produce: what linear
    extrapolation from g_{n-2} = g2 and g_{n-1} = g1 misses of g_n = g0,
    per-trace scaled."""
    T = len(s)
    y = np.zeros((T, COUT, g0.shape[1]))
    for i in range(T):
        dr = (g0[2 * i] - 2 * g1[2 * i] + g2[2 * i]) / s[i]
        dl = (g0[2 * i + 1] - 2 * g1[2 * i + 1] + g2[2 * i + 1]) / s[i]
        y[i] = [dr.real, dr.imag, dl.real, dl.imag]
    return y


def guess(g1, g2, y, s):
    """g^{NN} = 2 g_{n-1} - g_{n-2} + s * (network output), interface layout."""
    g = 2 * np.array(g1, dtype=complex) - np.array(g2, dtype=complex)
    for i in range(len(s)):
        g[2 * i] += s[i] * (y[i, 0] + 1j * y[i, 1])
        g[2 * i + 1] += s[i] * (y[i, 2] + 1j * y[i, 3])
    return g
