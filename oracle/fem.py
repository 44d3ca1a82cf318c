"""Q1 finite elements on a uniform rectangular mesh (Section 2.2, the matrix
formulation eq. NproblemRobinNL and the matrix list before it).

Oracle code (test infrastructure).  Nodes are numbered x-major, y-fast:
global index I = i*ny + k for node (x_i, y_k), ny = ncy + 1.

Matrices (names follow the paper):
  M      mass matrix, int v w
  S      stiffness matrix, int grad v . grad w
  M_W    generalized mass matrix, int W v w.  The paper does not say which
         quadrature it uses; here W is replaced by its Q1 interpolant and the
         product of three Q1 functions is integrated exactly.
  MG_l, MG_r  boundary mass on the left (x = a) and right (x = b) edges,
         int_Gamma v w.  On an edge line it equals the 1-D y-mass matrix.

The strip operator with Laplacian coefficient c and Robin parameters pl, pr
on its two x-edges is
  K(phi) = 2i/dt M - c S + M_phi + i c (pl MG_l + pr MG_r),
the left-hand side of eq. NproblemRobinNL with the nonlinearity folded into
the potential phi = W + beta|zeta|^2 (c multiplies the boundary term because
it comes from integrating c*Lap by parts).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mass_1d(n: int, h: float) -> sp.csr_matrix:
    """1-D Q1 mass on n cells: element matrix (h/6)[[2,1],[1,2]] assembled."""
    rows, cols, vals = [], [], []
    for e in range(n):
        for a in range(2):
            for b in range(2):
                rows.append(e + a)
                cols.append(e + b)
                vals.append(h / 3.0 if a == b else h / 6.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n + 1))


def stiff_1d(n: int, h: float) -> sp.csr_matrix:
    """1-D Q1 stiffness on n cells: element matrix (1/h)[[1,-1],[-1,1]]."""
    rows, cols, vals = [], [], []
    for e in range(n):
        for a in range(2):
            for b in range(2):
                rows.append(e + a)
                cols.append(e + b)
                vals.append(1.0 / h if a == b else -1.0 / h)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n + 1))


def triple_1d(a: int, b: int, c: int) -> float:
    """int over the reference element [0,1] of psi_a psi_b psi_c for the two
    linear shape functions psi_0 = 1-s, psi_1 = s (exact)."""
    return 0.25 if a == b == c else 1.0 / 12.0


def mass_2d(ncx, ncy, hx, hy):
    return sp.kron(mass_1d(ncx, hx), mass_1d(ncy, hy), format="csr")


def stiff_2d(ncx, ncy, hx, hy):
    return (sp.kron(stiff_1d(ncx, hx), mass_1d(ncy, hy))
            + sp.kron(mass_1d(ncx, hx), stiff_1d(ncy, hy))).tocsr()


def edge_mass_2d(ncx, ncy, hy, side: str):
    """Boundary mass on the x-edge line i=0 ('l') or i=ncx ('r')."""
    e = np.zeros(ncx + 1)
    e[0 if side == "l" else ncx] = 1.0
    return sp.kron(sp.diags(e), mass_1d(ncy, hy), format="csr")


def weighted_mass_2d(W: np.ndarray, hx: float, hy: float) -> sp.csr_matrix:
    """M_W[I,J] = sum over elements of sum_L W_L int psi_L psi_I psi_J, the
    triple products integrated exactly.  W has nodal shape (ncx+1, ncy+1)."""
    W = np.asarray(W, dtype=float)
    ncx, ncy = W.shape[0] - 1, W.shape[1] - 1
    ny = ncy + 1
    ex, ey = np.meshgrid(np.arange(ncx), np.arange(ncy), indexing="ij")
    ex = ex.ravel()
    ey = ey.ravel()
    local = [(0, 0), (0, 1), (1, 0), (1, 1)]
    rows, cols, vals = [], [], []
    for (ai, ak) in local:          # test function psi_A
        gi = (ex + ai) * ny + (ey + ak)
        for (bi, bk) in local:      # trial function psi_B
            gj = (ex + bi) * ny + (ey + bk)
            v = np.zeros(ex.shape)
            for (ci, ck) in local:  # interpolant of W
                coef = hx * triple_1d(ci, ai, bi) * hy * triple_1d(ck, ak, bk)
                v = v + coef * W[ex + ci, ey + ck]
            rows.append(gi)
            cols.append(gj)
            vals.append(v)
    n = (ncx + 1) * ny
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                 np.concatenate(cols))), shape=(n, n))


def weighted_mass_apply(W: np.ndarray, v: np.ndarray, hx: float, hy: float) -> np.ndarray:
    """M_W v without assembling M_W: (M_W v)_I = sum over elements e, local
    potential node L and local trial node J of W_L v_J int_e psi_L psi_I psi_J,
    the same exact triple products as weighted_mass_2d.  W and v are nodal
    arrays (ncx+1, ncy+1); the element sums run over whole shifted slices of
    the node grid (element (ex, ey) has local node (a, b) at (ex+a, ey+b))."""
    W = np.asarray(W, dtype=float)
    v = np.asarray(v)
    ncx, ncy = W.shape[0] - 1, W.shape[1] - 1
    out = np.zeros(v.shape, dtype=np.result_type(v, W))
    local = [(0, 0), (0, 1), (1, 0), (1, 1)]

    def sl(a, b):
        return (slice(a, a + ncx), slice(b, b + ncy))

    for (ai, ak) in local:          # test function psi_I
        acc = np.zeros((ncx, ncy), dtype=out.dtype)
        for (bi, bk) in local:      # trial function psi_J
            for (ci, ck) in local:  # interpolant of W
                coef = hx * triple_1d(ci, ai, bi) * hy * triple_1d(ck, ak, bk)
                acc += coef * W[sl(ci, ck)] * v[sl(bi, bk)]
        out[sl(ai, ak)] += acc
    return out


class StripMatrices:
    """The constant matrices of one (sub)domain made of `ncx` cells in x and
    `ncy` cells in y with mesh sizes hx, hy."""

    def __init__(self, ncx: int, ncy: int, hx: float, hy: float):
        self.ncx, self.ncy, self.hx, self.hy = ncx, ncy, hx, hy
        self.nx, self.ny = ncx + 1, ncy + 1
        self.M = mass_2d(ncx, ncy, hx, hy)
        self.S = stiff_2d(ncx, ncy, hx, hy)
        self.MGl = edge_mass_2d(ncx, ncy, hy, "l")
        self.MGr = edge_mass_2d(ncx, ncy, hy, "r")
        self.My = mass_1d(ncy, hy)

    def operator(self, phi: np.ndarray, dt: float, c: float, pl: float,
                 pr: float) -> sp.csc_matrix:
        """K(phi) = 2i/dt M - c S + M_phi + i c (pl MG_l + pr MG_r)."""
        K = ((2j / dt) * self.M - c * self.S + weighted_mass_2d(phi, self.hx, self.hy)
             + 1j * c * (pl * self.MGl + pr * self.MGr))
        return K.tocsc()

    def mass_norm2(self, u: np.ndarray) -> float:
        """u* M u for a nodal array of this domain."""
        v = u.ravel()
        return float(np.real(np.vdot(v, self.M @ v)))
