"""Pins of the oracle's monolithic time step: closed forms, a dense Newton
solve, the two fixed-point forms, the discrete mass identity and the order of
accuracy against the exact spreading Gaussian."""
import numpy as np
import pytest
import scipy.optimize

from oracle import fem
from oracle.step import MonolithicStepper, run_monolithic
from tests.closed_forms import (constant_state_step, free_neumann_step,
                                free_robin_x_step, spreading_gaussian)
from workloads import Problem, equal_strips


def small_problem(ncx=12, ncy=10, beta=0.0, p=0.0, c=1.0, dt=0.05, L=3.0):
    return Problem(-L, L, -L * 0.8, L * 0.8, ncx, ncy, 2, equal_strips(ncx, 2),
                   lap_coef=c, beta=beta, p=max(p, 1.0), p_bc=p, dt=dt)


def rand_u(pb, seed):
    rng = np.random.default_rng(seed)
    s = (pb.ncx + 1, pb.ncy + 1)
    return rng.standard_normal(s) + 1j * rng.standard_normal(s)


@pytest.mark.parametrize("c,w", [(1.0, 0.0), (0.5, -1.3)])
def test_free_neumann_step_matches_cosine_modes(c, w):
    pb = small_problem(c=c)
    u = rand_u(pb, 3)
    W = np.full((pb.ncx + 1, pb.ncy + 1), w)
    un, _, _ = MonolithicStepper(pb, W).step(u)
    ref = free_neumann_step(u, pb.ncx, pb.ncy, pb.hx, pb.hy, pb.dt, c, w)
    assert np.max(np.abs(un - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("c,pbc", [(1.0, 2.0), (0.5, 7.5)])
def test_free_robin_step_matches_mode_solves(c, pbc):
    pb = small_problem(c=c, p=pbc)
    u = rand_u(pb, 4)
    W = np.full((pb.ncx + 1, pb.ncy + 1), 0.7)
    un, _, _ = MonolithicStepper(pb, W).step(u)
    ref = free_robin_x_step(u, pb.ncx, pb.ncy, pb.hx, pb.hy, pb.dt, c, 0.7, pbc)
    assert np.max(np.abs(un - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("form", ["A", "B"])
def test_constant_state_nonlinear_closed_form(form):
    pb = small_problem(ncx=4, ncy=3, beta=-40.0, dt=0.02)
    u0 = 0.8 * np.exp(0.3j)
    u = np.full((pb.ncx + 1, pb.ncy + 1), u0, dtype=complex)
    un, _, _ = MonolithicStepper(pb, np.zeros(u.shape), form=form).step(u)
    ref = constant_state_step(u0, pb.dt, pb.beta)
    assert np.max(np.abs(un - ref)) < 1e-13


def test_nonlinear_step_matches_dense_newton():
    """G(v) = K(W + beta|v|^2) v - 2i/dt M u = 0 solved by a generic root
    finder on the real/imaginary split with dense matrices."""
    pb = small_problem(ncx=4, ncy=3, beta=10.0, p=1.5, dt=0.02)
    rng = np.random.default_rng(5)
    u = 0.6 * rand_u(pb, 6)
    W = rng.standard_normal((pb.ncx + 1, pb.ncy + 1))
    st = MonolithicStepper(pb, W, form="B", tol_q=1e-14)
    _, v, _ = st.step(u)
    m = st.mats
    F = (2j / pb.dt) * (m.M @ u.ravel())
    shape = u.shape

    def G(xr):
        z = xr[:xr.size // 2] + 1j * xr[xr.size // 2:]
        K = m.operator(W + pb.beta * np.abs(z.reshape(shape)) ** 2, pb.dt,
                       pb.lap_coef, pb.p_bc, pb.p_bc)
        r = K @ z - F
        return np.concatenate([r.real, r.imag])

    x0 = np.concatenate([u.ravel().real, u.ravel().imag])
    sol = scipy.optimize.root(G, x0, method="hybr", tol=1e-15)
    vn = sol.x[:sol.x.size // 2] + 1j * sol.x[sol.x.size // 2:]
    assert np.max(np.abs(vn - v.ravel())) < 1e-11 * np.max(np.abs(vn))


def test_forms_A_and_B_agree():
    pb = small_problem(ncx=10, ncy=8, beta=-30.0, p=2.0, dt=0.02)
    u = 0.7 * rand_u(pb, 7)
    W = np.random.default_rng(8).standard_normal(u.shape)
    ua = run_monolithic(pb, u, W, 3, form="A", tol_q=1e-14)
    ub = run_monolithic(pb, u, W, 3, form="B", tol_q=1e-14)
    assert np.linalg.norm(ua - ub) < 1e-12 * np.linalg.norm(ua)


@pytest.mark.parametrize("pbc", [0.0, 3.0])
def test_discrete_mass_identity(pbc):
    """||u_n||_M^2 - ||u_{n-1}||_M^2 = -2 c p_bc dt v* M^Gamma v (imaginary
    part of v* times the step equation); invariant when p_bc = 0."""
    pb = small_problem(ncx=10, ncy=9, beta=10.0, p=pbc, c=0.5, dt=0.02)
    u = 0.5 * rand_u(pb, 9)
    W = np.random.default_rng(10).standard_normal(u.shape)
    st = MonolithicStepper(pb, W, form="B", tol_q=1e-14)
    for _ in range(3):
        m0 = st.mats.mass_norm2(u)
        un, v, _ = st.step(u)
        m1 = st.mats.mass_norm2(un)
        vv = v.ravel()
        bnd = np.real(np.vdot(vv, (st.mats.MGl + st.mats.MGr) @ vv))
        assert abs((m1 - m0) - (-2 * pb.lap_coef * pbc * pb.dt * bnd)) < 1e-12 * m0
        u = un


def test_spreading_gaussian_second_order():
    """Linear free run on (-10,10)^2 against the exact solution: error
    decreases like h^2 + dt^2 (refining both by 2 divides it by ~4)."""
    errs = []
    T = 0.2
    for n, dt in [(64, 0.02), (128, 0.01), (256, 0.005)]:
        pb = Problem(-10, 10, -10, 10, n, n, 2, [n // 2] * 2, lap_coef=1.0,
                     beta=0.0, p=1.0, p_bc=1.0, dt=dt)
        x = pb.xl + pb.hx * np.arange(n + 1)
        y = pb.yb + pb.hy * np.arange(n + 1)
        u0 = spreading_gaussian(x, y, 0.0)
        steps = int(round(T / dt))
        u = run_monolithic(pb, u0, np.zeros(u0.shape), steps)
        ex = spreading_gaussian(x, y, T)
        errs.append(np.max(np.abs(u - ex)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), (errs, rates)
