"""Rotating-frame potential of the GPE (Section 5.2.1, eqs. x1Ax, GPE_Trans,
u1u).  Oracle code (test infrastructure).

In the rotating Lagrangian coordinates x~ = A(t)^T x, with
A(t) = [[cos wt, sin wt], [-sin wt, cos wt]], the GPE loses its rotation term
and carries the time-dependent potential V_t(t, x~) = V(A(t) x~).  The time
scheme uses W_n = (V_t(t_n) + V_t(t_{n-1}))/2 (Section 2.1), so the potential
changes at every step.
"""
from __future__ import annotations

import numpy as np


def lab_coords(xt, yt, omega, t):
    """(x, y) = A(t) (x~, y~)."""
    c, s = np.cos(omega * t), np.sin(omega * t)
    return c * xt + s * yt, -s * xt + c * yt


def rotating_potential(pb, t):
    """V_t(t, .) at the nodes for V(x, y) = vxx x^2 + vyy y^2."""
    xt = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    yt = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    XT, YT = np.meshgrid(xt, yt, indexing="ij")
    X, Y = lab_coords(XT, YT, pb.omega, t)
    return pb.vxx * X ** 2 + pb.vyy * Y ** 2


def step_potential(pb, n):
    """W_n = (V_t(t_n) + V_t(t_{n-1})) / 2 with t_n = n dt."""
    return 0.5 * (rotating_potential(pb, n * pb.dt) + rotating_potential(pb, (n - 1) * pb.dt))
