"""Independent closed forms used to pin the oracle.

None of these reuse the oracle's finite-element assembly: they come from the
mathematics of the continuous or semi-discrete problem (separation of
variables, exact solutions of the free Schroedinger equation, scalar
reductions) and only take the mesh sizes as input.
"""
from __future__ import annotations

import numpy as np


def cos_basis(ncells: int) -> np.ndarray:
    """C[i, k] = cos(k pi i / n): the Neumann (DCT-I) vectors that
    diagonalise the 1-D Q1 pencil (stiffness, mass) with natural ends."""
    i = np.arange(ncells + 1)[:, None]
    k = np.arange(ncells + 1)[None, :]
    return np.cos(np.pi * i * k / ncells)


def pencil_eigs(ncells: int, h: float) -> np.ndarray:
    """Generalised eigenvalues of S1 v = lam M1 v for DCT-I modes:
    lam_k = 6 (1 - cos t_k) / (h^2 (2 + cos t_k)), t_k = k pi / n.  Derived
    from the three-term recurrences (h/6)(1,4,1) and (1/h)(-1,2,-1), whose
    end rows (2,1) and (1,-1) keep the same ratio for cosine vectors."""
    t = np.pi * np.arange(ncells + 1) / ncells
    return 6.0 * (1.0 - np.cos(t)) / (h * h * (2.0 + np.cos(t)))


def free_neumann_step(u, ncx, ncy, hx, hy, dt, c, w):
    """One step of the free linear scheme with Neumann boundaries on all
    sides and constant potential w, by separation of variables: each 2-D
    cosine mode is multiplied by (2i/dt + c L - w) / (2i/dt - c L + w)."""
    Cx, Cy = cos_basis(ncx), cos_basis(ncy)
    a = np.linalg.solve(Cx, np.linalg.solve(Cy, u.T).T)
    L = pencil_eigs(ncx, hx)[:, None] + pencil_eigs(ncy, hy)[None, :]
    rho = (2j / dt + c * L - w) / (2j / dt - c * L + w)
    return Cx @ (a * rho) @ Cy.T


def hat_mass_stiff(ncells, h):
    """1-D mass and stiffness built from point values of hat functions with
    3-point Gauss-Legendre quadrature on each cell (no element formulas)."""
    gx, gw = np.polynomial.legendre.leggauss(3)
    n = ncells + 1
    M = np.zeros((n, n))
    S = np.zeros((n, n))
    for e in range(ncells):
        xs = e * h + 0.5 * h * (gx + 1.0)
        ws = 0.5 * h * gw
        for a in range(n):
            for b in range(n):
                fa = np.clip(1 - np.abs(xs / h - a), 0, None)
                fb = np.clip(1 - np.abs(xs / h - b), 0, None)
                da = np.where(np.abs(xs / h - a) < 1, -np.sign(xs / h - a) / h, 0.0)
                db = np.where(np.abs(xs / h - b) < 1, -np.sign(xs / h - b) / h, 0.0)
                M[a, b] += np.sum(ws * fa * fb)
                S[a, b] += np.sum(ws * da * db)
    return M, S


def free_robin_x_step(u, ncx, ncy, hx, hy, dt, c, w, pbc):
    """One free linear step with Robin parameter pbc on the x-edges and
    Neumann in y: cosine modes in y, then for each mode m a 1-D complex
    system  [(2i/dt + w - c lam_m) M1 - c S1 + i c pbc E] V = 2i/dt M1 U
    in x, with M1, S1 from hat-function quadrature and E = e_0 e_0^T +
    e_n e_n^T."""
    M1, S1 = hat_mass_stiff(ncx, hx)
    E = np.zeros((ncx + 1, ncx + 1))
    E[0, 0] = E[-1, -1] = 1.0
    Cy = cos_basis(ncy)
    lam = pencil_eigs(ncy, hy)
    U = np.linalg.solve(Cy, u.T).T            # u[i,:] = sum_m U[i,m] Cy[:,m]
    V = np.zeros_like(U)
    for m in range(ncy + 1):
        A = (2j / dt + w - c * lam[m]) * M1 - c * S1 + 1j * c * pbc * E
        V[:, m] = np.linalg.solve(A, (2j / dt) * (M1 @ U[:, m]))
    v = V @ Cy.T
    return 2 * v - u


def spreading_gaussian(x, y, t, c=1.0, k=1.0):
    """Exact solution of i u_t + c Lap u = 0 on R^2 with
    u(0) = exp(-(x^2+y^2)) exp(i k x): a Gaussian that spreads and moves
    with group velocity 2ck."""
    a = 1.0 + 4j * c * t
    X, Y = np.meshgrid(x, y, indexing="ij")
    return (1.0 / a) * np.exp(-((X - 2 * c * k * t) ** 2 + Y ** 2) / a
                              + 1j * k * X - 1j * c * k * k * t)


def constant_state_step(u, dt, beta, w=0.0):
    """Spatially constant data with Neumann boundaries: the step reduces to
    the scalar equation (2i/dt + w + beta|v|^2) v = 2i/dt u.  With
    alpha = dt (w + beta rho)/2, rho = |v|^2 solves rho (1 + alpha^2) = |u|^2
    (monotone in rho, one positive root) and u_n = u (1 + i alpha)/(1 - i alpha)."""
    m2 = abs(u) ** 2
    lo, hi = 0.0, m2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        al = dt * (w + beta * mid) / 2
        if mid * (1 + al * al) < m2:
            lo = mid
        else:
            hi = mid
    rho = 0.5 * (lo + hi)
    al = dt * (w + beta * rho) / 2
    return u * (1 + 1j * al) / (1 - 1j * al)
