"""The absorbing transmission condition S_pade^m (Sections 2.1 and 2.2).

Oracle code (test infrastructure).  The operator of eq. TCS,
    S v = -i sum_s a_s v + i sum_s a_s d_s phi_s,
with phi_s solving the edge equation of eq. TCS_phi,
    (2i/dt + c d_yy + W + f(v) + d_s) phi_s = v   on the edge line,
is the Pade approximation of -i sqrt(2i/dt + c d_yy + W + f(v)) with the
branch cut rotated by theta:
    a_s = e^{i theta/2} / (m cos^2((2s-1) pi / (4m))),
    d_s = e^{i theta} tan^2((2s-1) pi / (4m)),        s = 1 .. m
(the sums start at s = 1: a_0 = 0, which makes sqrt(z) ~ sum_s a_s z/(z + d_s)).

The strip problem is the arrow system of eq. NproblemSPNL: the strip
unknowns zeta and, on each of the strip's two edges, m edge vectors phi_s,
    [ K_S   B_1 .. B_m ] [zeta ]   [ 2i/dt M h - M_f zeta^{q-1} - c M^G Q^T (l; r) ]
    [ C     D_1        ] [phi_1] = [ - M^G_f phi_1^{q-1}                          ]
    [ ..          ..   ] [ ..  ]   [ ..                                            ]
with K_S = 2i/dt M - c S + M_W + i c (sum a_s) M^G (both edges),
B_s = -i c a_s d_s M^G Q^T, C = -Q M^G and
D_s = 2i/dt M^G - c S^G + M^G_W + d_s M^G (1-D edge matrices: mass, stiffness,
weighted mass along y), the nonlinearity f(zeta) = beta |zeta|^2 taken from
the previous iterate on the right (the paper's form for this condition).  c
multiplies every boundary term (the weak form of c Lap) and the edge
Laplacian (Section 5.2.1: 1/2 for the GPE).  The flux update of eq. fluxlr
with this S is
    new l_{j+1} = -r_j + 2 S v_j (right edge of strip j, its phi),
    new r_j     = -l_{j+1} + 2 S v_{j+1} (left edge of strip j+1, its phi).
The physical x-edges carry the same condition with zero data (eq. BC with
eq. BCS2p).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import (StripMatrices, mass_1d, stiff_1d, triple_1d, weighted_mass_2d,
                  weighted_mass_apply)
from .schwarz import gmres
from .step import NoConvergence


def pade_coefficients(m: int, theta: float = np.pi / 4):
    """(a_s, d_s), s = 1 .. m, of eq. TCS."""
    s = np.arange(1, m + 1)
    ang = (2 * s - 1) * np.pi / (4 * m)
    a = np.exp(1j * theta / 2) / (m * np.cos(ang) ** 2)
    d = np.exp(1j * theta) * np.tan(ang) ** 2
    return a, d


def pade_sqrt(z, m: int, theta: float = np.pi / 4):
    """sum_s a_s z / (z + d_s): the rotated Pade approximation of sqrt(z)."""
    a, d = pade_coefficients(m, theta)
    z = np.asarray(z, dtype=complex)
    return sum(a[k] * z / (z + d[k]) for k in range(m))


def weighted_mass_1d(w: np.ndarray, h: float) -> sp.csr_matrix:
    """int w psi_i psi_j along one line, w replaced by its linear
    interpolant, triple products exact (the 1-D factor of M_W)."""
    n = len(w) - 1
    rows, cols, vals = [], [], []
    for e in range(n):
        for a in range(2):
            for b in range(2):
                v = sum(h * triple_1d(c, a, b) * w[e + c] for c in range(2))
                rows.append(e + a)
                cols.append(e + b)
                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n + 1))


def edge_operator(pb, w_edge: np.ndarray, ds: complex) -> sp.csr_matrix:
    """D_s = 2i/dt M^G - c S^G + M^G_W + d_s M^G on one edge line."""
    My = mass_1d(pb.ncy, pb.hy)
    Sy = stiff_1d(pb.ncy, pb.hy)
    return ((2j / pb.dt + ds) * My - pb.lap_coef * Sy
            + weighted_mass_1d(w_edge, pb.hy)).tocsr()


class PadeStrip:
    """The arrow system of one strip (or of the whole domain) with S_pade^m
    on both x-edges, factored once per potential (the nonlinearity sits on
    the right-hand side)."""

    def __init__(self, pb, ncx: int, W: np.ndarray):
        self.pb = pb
        self.m = pb.pade_m
        self.a, self.d = pade_coefficients(pb.pade_m, pb.pade_theta)
        self.mats = StripMatrices(ncx, pb.ncy, pb.hx, pb.hy)
        self.nx, self.ny = ncx + 1, pb.ncy + 1
        self.W = np.asarray(W, dtype=float)
        c = pb.lap_coef
        mt = self.mats
        nz = self.nx * self.ny
        My = mass_1d(pb.ncy, pb.hy)
        K = ((2j / pb.dt) * mt.M - c * mt.S + weighted_mass_2d(self.W, pb.hx, pb.hy)
             + 1j * c * np.sum(self.a) * (mt.MGl + mt.MGr))
        blocks = [[None] * (1 + 2 * self.m) for _ in range(1 + 2 * self.m)]
        blocks[0][0] = K
        for e, line in enumerate((0, self.nx - 1)):
            Q = sp.csr_matrix((np.ones(self.ny), (line * self.ny + np.arange(self.ny),
                                                  np.arange(self.ny))), shape=(nz, self.ny))
            for s in range(self.m):
                k = 1 + e * self.m + s
                blocks[0][k] = (-1j * c * self.a[s] * self.d[s]) * (Q @ My)
                blocks[k][0] = -(My @ Q.T)
                blocks[k][k] = edge_operator(pb, self.W[line], self.d[s])
        self.A = sp.bmat(blocks, format="csc")
        self.lu = spla.splu(self.A)
        self.nz = nz

    def edge_values(self, zeta, e):
        z = zeta.reshape(self.nx, self.ny)
        return z[0] if e == 0 else z[-1]

    def solve(self, F, zeta0, tol_q, max_q, fixed_q=None):
        """Fixed point of eq. localpbS2p from zeta^0 = zeta0, phi^0 = 0, on
        the whole unknown vector (zeta, phi).  F is the zeta right-hand side
        without the nonlinear term.  Returns (zeta, phi[e][s], q)."""
        pb = self.pb
        ny, m = self.ny, self.m
        X = np.zeros(self.nz + 2 * m * ny, complex)
        X[:self.nz] = zeta0.ravel()
        nq = fixed_q if fixed_q is not None else max_q
        for q in range(1, nq + 1):
            zeta = X[:self.nz]
            rho = pb.beta * np.abs(zeta) ** 2
            rhs = np.zeros_like(X)
            rhs[:self.nz] = F - weighted_mass_apply(
                rho.reshape(self.nx, ny), zeta.reshape(self.nx, ny), pb.hx, pb.hy).ravel()
            for e in range(2):
                fe = rho.reshape(self.nx, ny)[0 if e == 0 else -1]
                Mf = weighted_mass_1d(fe, pb.hy)
                for s in range(m):
                    k = self.nz + (e * m + s) * ny
                    rhs[k:k + ny] = -(Mf @ X[k:k + ny])
            Xn = self.lu.solve(rhs)
            inc = np.linalg.norm(Xn - X)
            X = Xn
            if not np.isfinite(inc):
                raise NoConvergence("fixed point diverged")
            if fixed_q is None and inc <= tol_q * np.linalg.norm(X):
                break
        else:
            if fixed_q is None:
                raise NoConvergence("S_pade fixed point did not converge")
        zeta = X[:self.nz].reshape(self.nx, ny)
        phi = [[X[self.nz + (e * m + s) * ny:self.nz + (e * m + s + 1) * ny] for s in range(m)]
               for e in range(2)]
        return zeta, phi, q

    def S_apply(self, v_edge, phi_edge):
        """S v = -i sum a_s v + i sum a_s d_s phi_s on one edge (eq. TCSdist)."""
        out = -1j * np.sum(self.a) * v_edge
        for s in range(self.m):
            out = out + 1j * self.a[s] * self.d[s] * phi_edge[s]
        return out


def pade_monolithic(pb, u0, W, steps, tol_q=1e-13, max_q=200):
    """Whole-domain steps with S_pade^m on the physical x-edges."""
    st = PadeStrip(pb, pb.ncx, W)
    u = np.array(u0, dtype=complex)
    for _ in range(steps):
        F = (2j / pb.dt) * (st.mats.M @ u.ravel())
        v, _, _ = st.solve(F, u, tol_q, max_q)
        u = 2.0 * v - u
    return u


class PadeSchwarz:
    """The classical and preconditioned Schwarz iterations with S_pade^m
    transmission (and physical) conditions; layout of g as in schwarz.py."""

    def __init__(self, pb, W, tol_q=1e-13, max_q=200):
        self.pb = pb
        self.N = pb.nsub
        self.ny = pb.ncy + 1
        self.cells = list(pb.strip_cells)
        self.starts = np.concatenate([[0], np.cumsum(self.cells)[:-1]]).astype(int)
        self.tol_q, self.max_q = tol_q, max_q
        self.W = np.asarray(W, dtype=float)
        self.strips = [PadeStrip(pb, c, self.restrict(self.W, j)) for j, c in enumerate(self.cells)]
        self.Lh_blocks = None

    def restrict(self, u, j):
        s, c = self.starts[j], self.cells[j]
        return np.array(u[s:s + c + 1])

    def assemble_global(self, vs, u_old):
        acc = np.zeros(u_old.shape, dtype=complex)
        cnt = np.zeros(u_old.shape[0])
        for j, v in enumerate(vs):
            s, c = self.starts[j], self.cells[j]
            acc[s:s + c + 1] += v
            cnt[s:s + c + 1] += 1
        return 2.0 * (acc / cnt[:, None]) - u_old

    def traces(self, g, j):
        ny = self.ny
        l = g[2 * (j - 1) + 1] if j >= 1 else np.zeros(ny, complex)
        r = g[2 * j] if j <= self.N - 2 else np.zeros(ny, complex)
        return l, r

    def strip_rhs(self, j, u_old_j, l, r):
        pb = self.pb
        st = self.strips[j]
        F = ((2j / pb.dt) * (st.mats.M @ u_old_j.ravel())).reshape(st.nx, st.ny)
        My = mass_1d(pb.ncy, pb.hy)
        F[0] -= pb.lap_coef * (My @ l)
        F[-1] -= pb.lap_coef * (My @ r)
        return F.ravel()

    def R(self, g, u_old, fixed_q=None):
        out = []
        for j in range(self.N):
            l, r = self.traces(g, j)
            uj = self.restrict(u_old, j)
            zeta, phi, q = self.strips[j].solve(self.strip_rhs(j, uj, l, r), uj, self.tol_q,
                                                self.max_q, fixed_q)
            out.append((zeta, phi))
        gn = np.empty_like(g)
        for i in range(self.N - 1):
            left, right = self.strips[i], self.strips[i + 1]
            zl, pl = out[i]
            zr, pr = out[i + 1]
            gn[2 * i] = -g[2 * i + 1] + 2 * right.S_apply(zr[0], pr[0])        # new r_i
            gn[2 * i + 1] = -g[2 * i] + 2 * left.S_apply(zl[-1], pl[1])        # new l_{i+1}
        return gn, [o[0] for o in out], [o[1] for o in out]

    def classical(self, u_old, g0, tol=1e-10, relative=False, max_k=10000, fixed_k=None,
                  fixed_q=None):
        g = np.array(g0, dtype=complex)
        nk = fixed_k if fixed_k is not None else max_k
        for k in range(1, nk + 1):
            gn, vs, phis = self.R(g, u_old, fixed_q)
            inc = np.linalg.norm(gn - g)
            g = gn
            ref = max(np.linalg.norm(g), 1e-300)
            if fixed_k is None and inc < (tol * ref if relative else tol):
                return dict(g=g, vs=vs, phis=phis, k=k, inc=inc)
        if fixed_k is None:
            raise NoConvergence("classical S_pade Schwarz did not converge")
        return dict(g=g, vs=vs, phis=phis, k=nk, inc=inc)

    def build_Lh(self):
        """L_h of the free problem (V = 0, f = 0, u_{n-1} = 0), whose Schwarz
        map is linear (Proposition 3.2 states its blocks; built numerically
        here, as for Robin): for every strip and each of its input traces,
        the strip's arrow system is solved for all ny unit traces at once
        and the new traces 2 S v (minus the opposite input on the same edge)
        are read off both edges."""
        pb0 = self.pb.replace(beta=0.0)
        ny, N = self.ny, self.N
        nt = 2 * (N - 1)
        L = np.zeros((nt * ny, nt * ny), complex)
        My = mass_1d(pb0.ncy, pb0.hy).toarray()
        eye = np.eye(ny)
        for j in range(N):
            st = PadeStrip(pb0, self.cells[j], np.zeros((self.cells[j] + 1, ny)))
            inputs = []
            if j >= 1:
                inputs.append(("l", 2 * (j - 1) + 1))
            if j <= N - 2:
                inputs.append(("r", 2 * j))
            for side, col in inputs:
                B = np.zeros((st.A.shape[0], ny), complex)
                line = 0 if side == "l" else st.nx - 1
                B[line * ny:(line + 1) * ny] = -pb0.lap_coef * My
                X = st.lu.solve(B)
                Z = X[:st.nz].reshape(st.nx, ny, ny)
                phis = [[X[st.nz + (e * st.m + s) * ny:st.nz + (e * st.m + s + 1) * ny]
                         for s in range(st.m)] for e in range(2)]
                if j >= 1:      # left edge of strip j -> new r_{j-1}
                    blk = 2 * st.S_apply(Z[0], phis[0])
                    if side == "l":
                        blk = blk - eye
                    L[2 * (j - 1) * ny:(2 * (j - 1) + 1) * ny, col * ny:(col + 1) * ny] = blk
                if j <= N - 2:  # right edge of strip j -> new l_{j+1}
                    blk = 2 * st.S_apply(Z[-1], phis[1])
                    if side == "r":
                        blk = blk - eye
                    L[(2 * j + 1) * ny:(2 * j + 2) * ny, col * ny:(col + 1) * ny] = blk
        self.Lh = L
        return L

    def precond(self, u_old, g0, tol=1e-10, relative=False, max_k=1000, gmres_rtol=1e-12):
        if self.Lh_blocks is None:
            self.Lh_blocks = self.build_Lh()
        P = np.eye(self.Lh.shape[0]) - self.Lh
        g = np.array(g0, dtype=complex)
        gm_total = 0
        for k in range(1, max_k + 1):
            Rg, vs, phis = self.R(g, u_old)
            y = (g - Rg).ravel()
            x, it = gmres(lambda z: P @ z, y, rtol=gmres_rtol)
            gm_total += it
            inc = np.linalg.norm(x)
            g = g - x.reshape(g.shape)
            ref = max(np.linalg.norm(g), 1e-300)
            if inc < (tol * ref if relative else tol):
                return dict(g=g, vs=vs, phis=phis, k=k, gmres_total=gm_total, inc=inc)
        raise NoConvergence("preconditioned S_pade Schwarz did not converge")
