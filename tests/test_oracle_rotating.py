"""Pins of the rotating-frame potential (Section 5.2.1, eqs. x1Ax, u1u)."""
import numpy as np

from oracle.rotating import lab_coords, rotating_potential, step_potential
from workloads import Problem


def prob(omega=0.7, vxx=-0.5, vyy=-0.6):
    return Problem(-4, 4, -3, 3, 16, 12, 2, [8, 8], lap_coef=0.5, beta=-10.0, p=3.0,
                   p_bc=3.0, dt=0.01, omega=omega, vxx=vxx, vyy=vyy)


def grid(pb):
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    return np.meshgrid(x, y, indexing="ij")


def test_time_zero_is_the_lab_potential():
    pb = prob()
    X, Y = grid(pb)
    assert np.max(np.abs(rotating_potential(pb, 0.0) - (pb.vxx * X ** 2 + pb.vyy * Y ** 2))) < 1e-14


def test_quarter_turn_swaps_the_axes():
    """omega t = pi/2: A(t) x~ = (y~, -x~), so V_t = vxx y~^2 + vyy x~^2."""
    pb = prob()
    X, Y = grid(pb)
    t = np.pi / (2 * pb.omega)
    assert np.max(np.abs(rotating_potential(pb, t) - (pb.vxx * Y ** 2 + pb.vyy * X ** 2))) < 1e-12


def test_isotropic_trap_does_not_rotate():
    pb = prob(vxx=-0.5, vyy=-0.5)
    for t in (0.3, 1.7, 4.0):
        assert np.max(np.abs(rotating_potential(pb, t) - rotating_potential(pb, 0.0))) < 1e-12


def test_rotation_is_orthogonal_and_step_average():
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(5), rng.standard_normal(5)
    X, Y = lab_coords(x, y, 0.9, 1.3)
    assert np.allclose(X ** 2 + Y ** 2, x ** 2 + y ** 2, rtol=0, atol=1e-14)
    pb = prob()
    W3 = step_potential(pb, 3)
    ref = 0.5 * (rotating_potential(pb, 3 * pb.dt) + rotating_potential(pb, 2 * pb.dt))
    assert np.max(np.abs(W3 - ref)) < 1e-15
