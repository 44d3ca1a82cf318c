"""Sequential optimized Schwarz iteration on x-strips (Sections 2-4).

Oracle code (test infrastructure).  Follows the paper's discrete algorithm:

* Decomposition (Section 2.1, Fig. figsub3): strip j owns cells
  [s_j, s_j + cells_j) in x; its node-lines s_j .. s_j + cells_j include both
  edge lines, so an interface line is duplicated (non-overlapping FEM).
* Local problem (eqs. algolocal, NproblemRobinNL): with the transmission data
  (l_j, r_j) on its two edges the strip solves
      K_j(W + beta|v|^2) v = 2i/dt M_j u_{j,n-1} - c M^Gamma Q^T (l_j; r_j)
  by the fixed point of step.py (forms A/B), started from zeta^0 = u_{j,n-1}.
  K_j carries the Robin term i c p on interface edges and i c p_bc on the
  physical edges of the two extreme strips, where l_1 = r_N = 0.
* Flux update (eqs. fluxlr, AlgoGraph with S = -ip):
      new l_{j+1} = -r_j     - 2ip Q_r v_j,
      new r_j     = -l_{j+1} - 2ip Q_l v_{j+1}.
* Interface vector (eq. algo_d) g = (r_1, l_2, r_2, ..., r_{N-1}, l_N); here
  stored as an array of shape (2(N-1), ny) with g[2i] = r_i and
  g[2i+1] = l_{i+1} for the interface i between strips i and i+1 (0-based).
* Classical algorithm: g^{k+1} = R(g^k), stop when ||g^{k+1} - g^k|| < tol
  (Section 5, stopping rule).
* Preconditioned algorithm (eq. algo_pd, read as
  g^{k+1} = g^k - P^{-1}(g^k - R(g^k))) with P = I - L_h, where L_h is the
  linear part of the Schwarz map of the free problem V = 0, f = 0
  (Section 3, eq. Lmpi).  L_h is built numerically, column by column, as the
  free map applied to unit vectors (Section 4.2 does the same with the
  formulas of Proposition 3.1); P x = y is solved by GMRES or directly.
* Krylov solvers: P x = y by GMRES or by BiCGStab (Section 4.2 names both);
  for f = 0, where R is affine, the interface problem (I - L) g = d
  (eq. interfacepb_d) solved directly by GMRES with one Schwarz map per
  product (interface_krylov).
* The output v_{j,n} comes from the last evaluation of R; the global u_n
  takes 2 v - u_{n-1} on every line, the mean of the two copies on interface
  lines.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import StripMatrices, weighted_mass_apply
from .step import NoConvergence


def splitmix64(seed: int, j: np.ndarray) -> np.ndarray:
    """Output j (0-based) of SplitMix64 seeded with `seed` (Steele, Lea and
    Flood, "Fast splittable pseudorandom number generators", 2014): the state
    after j + 1 increments by the golden-ratio constant, mixed by two
    xor-shift-multiply rounds and a final xor-shift.  uint64 arithmetic
    wraps modulo 2^64."""
    j = np.asarray(j, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (j + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def random_interface(seed: int, shape) -> np.ndarray:
    """The random first interface vector g_1^0 (Section 5, initial vectors):
    entry k (row-major) is u(2k) + i u(2k+1), u(j) = (output j >> 11) 2^-53,
    uniform on [0, 1) (the paper does not state the distribution; this is a
    PETSc-style uniform real and imaginary part)."""
    n = int(np.prod(shape))
    k = np.arange(n, dtype=np.uint64)
    scale = 2.0 ** -53
    re = (splitmix64(seed, 2 * k) >> np.uint64(11)).astype(np.float64) * scale
    im = (splitmix64(seed, 2 * k + np.uint64(1)) >> np.uint64(11)).astype(np.float64) * scale
    return (re + 1j * im).reshape(shape)


def gmres(matvec, b, rtol=1e-12, restart=50, maxiter=2000):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations
    (textbook form), x0 = 0.  Returns (x, total inner iterations)."""
    n = b.shape[0]
    x = np.zeros(n, dtype=complex)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0
    total = 0
    while total < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return x, total
        V = np.zeros((restart + 1, n), dtype=complex)
        H = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        e = np.zeros(restart + 1, dtype=complex)
        e[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            w = matvec(V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            # complex Givens rotation [[conj(c), conj(s)], [-s, c]] with
            # c = a/rho, s = b/rho maps (a, b) to (rho, 0)
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den else 1.0
            sn[j] = bb / den if den else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            e[j + 1] = -sn[j] * e[j]
            e[j] = np.conj(cs[j]) * e[j]
            total += 1
            j_done = j + 1
            if abs(e[j + 1]) <= rtol * bnorm or total >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), e[:j_done])
        x = x + V[:j_done].T @ y
        if abs(e[j_done]) <= rtol * bnorm:
            r = b - matvec(x)
            if np.linalg.norm(r) <= 10 * rtol * bnorm:
                return x, total
    return x, total


def bicgstab(matvec, b, rtol=1e-12, maxiter=2000):
    """BiCGStab without preconditioning (van der Vorst, 1992), x0 = 0 and
    the shadow residual equal to the first residual; the complex inner
    product is conjugate-linear in its first argument.  Stops when
    ||r|| <= rtol ||b||.  Returns (x, iterations)."""
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0
    r = b.copy()
    rh = b.copy()
    rho_old = alpha = omega = 1.0 + 0.0j
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    for it in range(1, maxiter + 1):
        rho = np.vdot(rh, r)
        beta = (rho / rho_old) * (alpha / omega)
        rho_old = rho
        p = r + beta * (p - omega * v)
        v = matvec(p)
        alpha = rho / np.vdot(rh, v)
        s = r - alpha * v
        t = matvec(s)
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        if np.linalg.norm(r) <= rtol * bnorm:
            return x, it
    return x, maxiter


class SchwarzOracle:
    def __init__(self, pb, W: np.ndarray, form: str = "B", tol_q: float = 1e-13,
                 max_q: int = 200):
        self.pb = pb
        self.form = form
        self.tol_q = tol_q
        self.max_q = max_q
        self.N = pb.nsub
        self.ny = pb.ncy + 1
        cells = list(pb.strip_cells)
        assert len(cells) == self.N and sum(cells) == pb.ncx
        self.cells = cells
        self.starts = np.concatenate([[0], np.cumsum(cells)[:-1]]).astype(int)
        self.mats = [StripMatrices(c, pb.ncy, pb.hx, pb.hy) for c in cells]
        self.pl = [pb.p_bc if j == 0 else pb.p for j in range(self.N)]
        self.pr = [pb.p_bc if j == self.N - 1 else pb.p for j in range(self.N)]
        self._free_lu = None
        self.Lh_blocks = None
        self.set_potential(W)

    # ---- data movement between the global mesh and strips -------------
    def restrict(self, u: np.ndarray, j: int) -> np.ndarray:
        s, c = self.starts[j], self.cells[j]
        return np.array(u[s:s + c + 1, :])

    def assemble_global(self, vs, u_old: np.ndarray) -> np.ndarray:
        acc = np.zeros(u_old.shape, dtype=complex)
        cnt = np.zeros(u_old.shape[0])
        for j, v in enumerate(vs):
            s, c = self.starts[j], self.cells[j]
            acc[s:s + c + 1] += v
            cnt[s:s + c + 1] += 1
        vbar = acc / cnt[:, None]
        return 2.0 * vbar - u_old

    # ---- local problems ------------------------------------------------
    def set_potential(self, W: np.ndarray):
        pb = self.pb
        self.W = np.asarray(W, dtype=float)
        self.Wj = [self.restrict(self.W, j) for j in range(self.N)]
        self._lu = [None] * self.N
        if self.form == "B":
            for j in range(self.N):
                K = self.mats[j].operator(self.Wj[j], pb.dt, pb.lap_coef,
                                          self.pl[j], self.pr[j])
                self._lu[j] = spla.splu(K)

    def traces(self, g: np.ndarray, j: int):
        """(l_j, r_j) read from the interface vector; zero on physical edges."""
        ny = self.ny
        l = g[2 * (j - 1) + 1] if j >= 1 else np.zeros(ny, complex)
        r = g[2 * j] if j <= self.N - 2 else np.zeros(ny, complex)
        return l, r

    def strip_rhs(self, j: int, u_old_j: np.ndarray, l, r) -> np.ndarray:
        """2i/dt M_j u_{j,n-1} - c M^Gamma Q^T (l; r)."""
        pb = self.pb
        m = self.mats[j]
        F = (2j / pb.dt) * (m.M @ u_old_j.ravel())
        F = F.reshape(m.nx, m.ny)
        F[0] -= pb.lap_coef * (m.My @ l)
        F[-1] -= pb.lap_coef * (m.My @ r)
        return F.ravel()

    def solve_strip(self, j, u_old_j, l, r, zeta0=None, fixed_q=None):
        pb = self.pb
        m = self.mats[j]
        shape = (m.nx, m.ny)
        F = self.strip_rhs(j, u_old_j, l, r)
        zeta = (u_old_j if zeta0 is None else zeta0).ravel().astype(complex)
        nq = fixed_q if fixed_q is not None else self.max_q
        for q in range(1, nq + 1):
            rho = pb.beta * np.abs(zeta) ** 2
            if self.form == "A":
                K = m.operator(self.Wj[j] + rho.reshape(shape), pb.dt, pb.lap_coef,
                               self.pl[j], self.pr[j])
                znew = spla.spsolve(K, F)
            else:
                Mz = weighted_mass_apply(rho.reshape(shape), zeta.reshape(shape), pb.hx, pb.hy)
                znew = self._lu[j].solve(F - Mz.ravel())
            inc = np.linalg.norm(znew - zeta)
            zeta = znew
            if not np.isfinite(inc):
                raise NoConvergence("fixed point diverged")
            if fixed_q is None and inc <= self.tol_q * np.linalg.norm(zeta):
                return zeta.reshape(shape), q
        if fixed_q is None:
            raise NoConvergence("strip fixed point did not converge")
        return zeta.reshape(shape), nq

    # ---- the Schwarz map R ---------------------------------------------
    def flux(self, g: np.ndarray, vs) -> np.ndarray:
        """Eq. fluxlr with S = -ip: every trace is updated from the k-th
        iterate of the neighbouring strip (Jacobi)."""
        p = self.pb.p
        gn = np.empty_like(g)
        for i in range(self.N - 1):
            l_next = g[2 * i + 1]
            r_i = g[2 * i]
            gn[2 * i] = -l_next - 2j * p * vs[i + 1][0]       # new r_i
            gn[2 * i + 1] = -r_i - 2j * p * vs[i][-1]          # new l_{i+1}
        return gn

    def R(self, g, u_old, zetas=None, fixed_q=None):
        vs, qs = [], []
        for j in range(self.N):
            l, r = self.traces(g, j)
            z0 = None if zetas is None else zetas[j]
            v, q = self.solve_strip(j, self.restrict(u_old, j), l, r, z0, fixed_q)
            vs.append(v)
            qs.append(q)
        return self.flux(g, vs), vs, qs

    # ---- classical and preconditioned iterations -----------------------
    @staticmethod
    def _converged(inc, ref, tol, relative):
        return inc < (tol * max(ref, 1e-300) if relative else tol)

    def classical(self, u_old, g0, tol=1e-10, relative=False, max_k=10000,
                  fixed_k=None, fixed_q=None, warm=False):
        g = np.array(g0, dtype=complex)
        q_total = 0
        zetas = None
        nk = fixed_k if fixed_k is not None else max_k
        for k in range(1, nk + 1):
            gn, vs, qs = self.R(g, u_old, zetas, fixed_q)
            q_total += sum(qs)
            if warm:
                zetas = vs
            inc = np.linalg.norm(gn - g)
            g = gn
            if fixed_k is None and self._converged(inc, np.linalg.norm(g), tol, relative):
                return dict(g=g, vs=vs, k=k, q_total=q_total, inc=inc)
        if fixed_k is None:
            raise NoConvergence(f"classical Schwarz did not converge in {max_k}")
        return dict(g=g, vs=vs, k=nk, q_total=q_total, inc=inc)

    # ---- free interface operator L_h (Section 3, eq. Lmpi) -------------
    def free_solver(self, j):
        """LU of the free strip operator K_j(0) (V = 0, f = 0)."""
        if self._free_lu is None:
            self._free_lu = [None] * self.N
        if self._free_lu[j] is None:
            pb = self.pb
            m = self.mats[j]
            K = m.operator(np.zeros((m.nx, m.ny)), pb.dt, pb.lap_coef,
                           self.pl[j], self.pr[j])
            self._free_lu[j] = spla.splu(K)
        return self._free_lu[j]

    def build_Lh(self):
        """Blocks of L_h as a dict {(row, col): (ny, ny) array} over the
        trace index t of g (t = 0 .. 2(N-1)-1).  Column t is the free Schwarz
        map (u_{n-1} = 0, V = 0, beta = 0) applied to unit vectors in trace
        t; only the strip that reads trace t responds."""
        pb = self.pb
        ny, N, p, c = self.ny, self.N, pb.p, pb.lap_coef
        blocks = {}
        for j in range(N):
            m = self.mats[j]
            lu = self.free_solver(j)
            inputs = []
            if j >= 1:
                inputs.append(("l", 2 * (j - 1) + 1))
            if j <= N - 2:
                inputs.append(("r", 2 * j))
            for side, col in inputs:
                # right-hand sides -c M^Gamma Q^T e_s for s = 0..ny-1
                B = np.zeros((m.nx, ny, ny), dtype=complex)
                line = 0 if side == "l" else m.nx - 1
                B[line] = -c * m.My.toarray()
                Vsol = lu.solve(B.reshape(m.nx * ny, ny)).reshape(m.nx, ny, ny)
                eye = np.eye(ny)
                if j >= 1:      # out_left of strip j -> new r_{j-1}
                    blk = -2j * p * Vsol[0]
                    if side == "l":
                        blk = blk - eye
                    blocks[(2 * (j - 1), col)] = blk
                if j <= N - 2:  # out_right of strip j -> new l_{j+1}
                    blk = -2j * p * Vsol[-1]
                    if side == "r":
                        blk = blk - eye
                    blocks[(2 * j + 1, col)] = blk
        self.Lh_blocks = blocks
        return blocks

    def Lh_matvec(self, x: np.ndarray) -> np.ndarray:
        ny = self.ny
        X = x.reshape(-1, ny)
        Y = np.zeros_like(X)
        for (r, c), blk in self.Lh_blocks.items():
            Y[r] += blk @ X[c]
        return Y.ravel()

    def Lh_dense(self) -> np.ndarray:
        ny = self.ny
        nt = 2 * (self.N - 1)
        L = np.zeros((nt * ny, nt * ny), dtype=complex)
        for (r, c), blk in self.Lh_blocks.items():
            L[r * ny:(r + 1) * ny, c * ny:(c + 1) * ny] = blk
        return L

    def Lh_sparse(self) -> sp.csc_matrix:
        ny = self.ny
        nt = 2 * (self.N - 1)
        rows, cols, vals = [], [], []
        for (r, c), blk in self.Lh_blocks.items():
            rr, cc = np.meshgrid(np.arange(ny), np.arange(ny), indexing="ij")
            rows.append((r * ny + rr).ravel())
            cols.append((c * ny + cc).ravel())
            vals.append(blk.ravel())
        n = nt * ny
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                     np.concatenate(cols))), shape=(n, n))

    def precond(self, u_old, g0, tol=1e-10, relative=False, max_k=1000,
                pinv="gmres", gmres_rtol=1e-12, gmres_restart=50, fixed_k=None,
                fixed_q=None, warm=False):
        if self.Lh_blocks is None:
            self.build_Lh()
        shape = g0.shape
        if pinv == "direct":
            P = sp.identity(self.Lh_sparse().shape[0], dtype=complex, format="csc") - self.Lh_sparse()
            Plu = spla.splu(P.tocsc())
        g = np.array(g0, dtype=complex)
        q_total = 0
        gm_total = 0
        zetas = None
        nk = fixed_k if fixed_k is not None else max_k
        for k in range(1, nk + 1):
            Rg, vs, qs = self.R(g, u_old, zetas, fixed_q)
            q_total += sum(qs)
            if warm:
                zetas = vs
            y = (g - Rg).ravel()
            if pinv == "direct":
                x = Plu.solve(y)
            elif pinv == "bicgstab":
                x, it = bicgstab(lambda z: z - self.Lh_matvec(z), y, rtol=gmres_rtol)
                gm_total += it
            else:
                x, it = gmres(lambda z: z - self.Lh_matvec(z), y, rtol=gmres_rtol,
                              restart=gmres_restart)
                gm_total += it
            inc = np.linalg.norm(x)
            g = g - x.reshape(shape)
            if fixed_k is None and self._converged(inc, np.linalg.norm(g), tol, relative):
                return dict(g=g, vs=vs, k=k, q_total=q_total, gmres_total=gm_total, inc=inc)
        if fixed_k is None:
            raise NoConvergence(f"preconditioned Schwarz did not converge in {max_k}")
        return dict(g=g, vs=vs, k=nk, q_total=q_total, gmres_total=gm_total, inc=inc)


def interface_krylov(orc, u_old, g0, tol=1e-10, relative=False, restart=50, maxiter=5000):
    """For f = 0 the Schwarz map is affine in g, R(g) = L g + d with
    d = R(0), so the fixed point of eq. algo_d solves the interface problem
    (I - L) g = d (eq. interfacepb_d), here by GMRES on the correction
    delta = g - g0: (I - L) delta = R(g0) - g0, every product
    x -> x - (R(x) - d) being one Schwarz map (all strip solves).  Stops
    when the residual is below tol (or tol ||R(g0) - g0|| when relative).
    Returns the converged g, the strip solutions of R(g), the Schwarz maps
    applied (products plus the three maps at d, g0 and g) and the GMRES
    iterations."""
    assert orc.pb.beta == 0.0, "the interface problem is linear only for f = 0"
    d, _, _ = orc.R(np.zeros_like(g0), u_old)
    Rg0, _, _ = orc.R(g0, u_old)
    b = (Rg0 - g0).ravel()
    maps = [0]

    def matvec(x):
        maps[0] += 1
        Rx, _, _ = orc.R(x.reshape(g0.shape), u_old)
        return x - (Rx - d).ravel()

    bn = np.linalg.norm(b)
    rtol = (tol if relative else tol / bn) if bn > 0 else 1.0
    delta, its = gmres(matvec, b, rtol=rtol, restart=restart, maxiter=maxiter)
    g = g0 + delta.reshape(g0.shape)
    _, vs, _ = orc.R(g, u_old)
    return dict(g=g, vs=vs, k=maps[0] + 3, gmres_total=its)


def run_schwarz(pb, u0, W, steps, algo="classical", g0=None, tol=1e-10,
                relative=False, form="B", tol_q=1e-13, warm=False, **kw):
    """Time loop: g_1^0 = g0 (zero by default), g_n^0 = g_{n-1}^infinity
    (Section 5, initial vectors).  W: nodal array or callable n -> W_n."""
    static = not callable(W)
    orc = SchwarzOracle(pb, W if static else W(1), form=form, tol_q=tol_q)
    ny = pb.ncy + 1
    g = np.zeros((2 * (pb.nsub - 1), ny), complex) if g0 is None else np.array(g0, complex)
    u = np.array(u0, dtype=complex)
    stats = []
    for n in range(1, steps + 1):
        if not static and n > 1:
            orc.set_potential(W(n))
        if algo == "classical":
            res = orc.classical(u, g, tol=tol, relative=relative, warm=warm, **kw)
        elif algo == "interface":
            res = interface_krylov(orc, u, g, tol=tol, relative=relative, **kw)
        else:
            res = orc.precond(u, g, tol=tol, relative=relative, warm=warm, **kw)
        u = orc.assemble_global(res["vs"], u)
        g = res["g"]
        stats.append({k: v for k, v in res.items() if k not in ("g", "vs")})
    return u, g, stats, orc
