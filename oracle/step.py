"""Monolithic (whole-domain) time step of the Duran-Sanz-Serna scheme.

Oracle code (test infrastructure).  Section 2.1, eq. CNS: with
v_n = (u_n + u_{n-1})/2 and W_n = (V_n + V_{n-1})/2 every step solves the
stationary nonlinear problem
    2i/dt v + c Lap v + W_n v + beta|v|^2 v = 2i/dt u_{n-1}
and sets u_n = 2 v_n - u_{n-1}.  After Q1 discretisation (Section 2.2) this
is  K(W_n + beta|v|^2) v = 2i/dt M u_{n-1}  on the whole domain, with the
physical Robin parameter p_bc on both x-edges (Neumann in y).

The nonlinearity is resolved by the fixed point of Section 2.2
(eq. localpbrobin) started from zeta^0 = u_{n-1}, in one of two forms that
share the same fixed point:
  form 'A'  K(W + beta|zeta^{q-1}|^2) zeta^q = F          (nonlinearity frozen
            in the matrix, as in eq. NproblemRobinNL);
  form 'B'  K(W) zeta^q = F - M_{beta|zeta^{q-1}|^2} zeta^{q-1}   (nonlinearity
            moved to the right-hand side, as the paper does for the absorbing
            condition in eq. NproblemSPNL; the matrix is factored once per W).
The iteration stops when ||zeta^q - zeta^{q-1}||_2 <= tol_q ||zeta^q||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import StripMatrices, weighted_mass_apply


class NoConvergence(RuntimeError):
    pass


class MonolithicStepper:
    def __init__(self, pb, W: np.ndarray, form: str = "B", tol_q: float = 1e-13,
                 max_q: int = 200):
        self.pb = pb
        self.mats = StripMatrices(pb.ncx, pb.ncy, pb.hx, pb.hy)
        self.form = form
        self.tol_q = tol_q
        self.max_q = max_q
        self.set_potential(W)

    def set_potential(self, W: np.ndarray):
        pb = self.pb
        self.W = np.asarray(W, dtype=float)
        self._lu = None
        if self.form == "B":
            K = self.mats.operator(self.W, pb.dt, pb.lap_coef, pb.p_bc, pb.p_bc)
            self._lu = spla.splu(K)

    def solve_stationary(self, u_old: np.ndarray):
        """Return (v, q_iterations) for one step's stationary problem."""
        pb = self.pb
        shape = (pb.ncx + 1, pb.ncy + 1)
        F = (2j / pb.dt) * (self.mats.M @ u_old.ravel())
        zeta = u_old.ravel().astype(complex)
        for q in range(1, self.max_q + 1):
            rho = pb.beta * np.abs(zeta) ** 2
            if self.form == "A":
                K = self.mats.operator(self.W + rho.reshape(shape), pb.dt,
                                       pb.lap_coef, pb.p_bc, pb.p_bc)
                znew = spla.spsolve(K, F)
            else:
                Mz = weighted_mass_apply(rho.reshape(shape), zeta.reshape(shape), pb.hx, pb.hy)
                znew = self._lu.solve(F - Mz.ravel())
            inc = np.linalg.norm(znew - zeta)
            zeta = znew
            if not np.isfinite(inc):
                raise NoConvergence("fixed point diverged")
            if inc <= self.tol_q * np.linalg.norm(zeta):
                return zeta.reshape(shape), q
        raise NoConvergence(f"fixed point did not converge in {self.max_q} iterations")

    def step(self, u_old: np.ndarray):
        v, q = self.solve_stationary(u_old)
        return 2.0 * v - u_old, v, q


def run_monolithic(pb, u0: np.ndarray, W, steps: int, form: str = "B",
                   tol_q: float = 1e-13, record_mass: bool = False):
    """Advance `steps` steps.  W is a nodal array (static potential) or a
    callable n -> W_n (time-dependent potential, refactored every step)."""
    static = not callable(W)
    st = MonolithicStepper(pb, W if static else W(1), form=form, tol_q=tol_q)
    u = np.array(u0, dtype=complex)
    masses = [st.mats.mass_norm2(u)]
    vs = []
    for n in range(1, steps + 1):
        if not static and n > 1:
            st.set_potential(W(n))
        u, v, _ = st.step(u)
        vs.append(v)
        masses.append(st.mats.mass_norm2(u))
    if record_mass:
        return u, np.array(masses), vs, st
    return u
