"""Training data and training loop of the learned interface guess.

Plumbing only: the time steps, the feature extraction, the network's
forward and backward passes and the optimiser all run in libosm's HIP
kernels (include/osm.h, learned guess); this module keeps the last
converged interface vectors of a run, stacks the resulting (input, target)
tensors on the device and feeds shuffled minibatches to the training step.
"""
from __future__ import annotations

import torch

from . import osm


def collect_traces(solver: "osm.OsmSolver", u: torch.Tensor, steps: int):
    """Runs `steps` time steps of an already factored solver (its guess
    option must be the paper's, 0) and returns the inputs (M, 9, ny) and
    targets (M, 4, ny) of every interface of every step n >= 3 (three
    converged vectors g_n, g_{n-1}, g_{n-2} are needed per sample)."""
    hist = []
    xs, ts = [], []
    stats = []
    for _ in range(steps):
        stats.append(solver.step(u))
        hist.append(solver.get_interface().clone())
        if len(hist) > 3:
            hist.pop(0)
        if len(hist) == 3:
            x, t = solver.guess_features(hist[1], hist[0], hist[2])
            xs.append(x)
            ts.append(t)
    if not xs:
        return None, None, stats
    return torch.cat(xs), torch.cat(ts), stats


def train(net: "osm.OsmNet", X: torch.Tensor, T: torch.Tensor, epochs: int, batch: int,
          lr: float, seed: int = 0, log=None):
    """Adam over shuffled minibatches of traces; returns the mean loss of
    every epoch (the loss of each minibatch before its update)."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    M = X.shape[0]
    batch = min(batch, net.max_traces)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(M, generator=gen).to(X.device)
        tot, nb = 0.0, 0
        for b0 in range(0, M, batch):
            idx = perm[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            tot += net.train_step(xb, tb, lr)
            nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses
