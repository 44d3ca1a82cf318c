"""Pins of the oracle's Q1 assembly against quadrature and invariants."""
import numpy as np
import pytest

from oracle import fem
from tests.closed_forms import hat_mass_stiff


@pytest.mark.parametrize("n,h", [(1, 0.5), (4, 0.25), (7, 0.13)])
def test_1d_matrices_match_hat_quadrature(n, h):
    M, S = hat_mass_stiff(n, h)
    assert np.allclose(fem.mass_1d(n, h).toarray(), M, rtol=0, atol=1e-15)
    assert np.allclose(fem.stiff_1d(n, h).toarray(), S, rtol=0, atol=1e-13)


def _bilinear_gauss_weighted_mass(W, hx, hy):
    """int W_h psi_I psi_J by 3x3 Gauss-Legendre on every element, with the
    bilinear interpolant W_h and shape functions evaluated pointwise."""
    ncx, ncy = W.shape[0] - 1, W.shape[1] - 1
    ny = ncy + 1
    n = (ncx + 1) * ny
    out = np.zeros((n, n))
    g, gw = np.polynomial.legendre.leggauss(3)
    for ex in range(ncx):
        for ey in range(ncy):
            for sa, wa in zip(g, gw):
                for sb, wb in zip(g, gw):
                    s = 0.5 * (sa + 1)
                    t = 0.5 * (sb + 1)
                    wq = 0.25 * hx * hy * wa * wb
                    shp = {(0, 0): (1 - s) * (1 - t), (1, 0): s * (1 - t),
                           (0, 1): (1 - s) * t, (1, 1): s * t}
                    Wq = sum(W[ex + a, ey + b] * f for (a, b), f in shp.items())
                    for (a, b), fa in shp.items():
                        I = (ex + a) * ny + ey + b
                        for (c, d), fb in shp.items():
                            J = (ex + c) * ny + ey + d
                            out[I, J] += wq * Wq * fa * fb
    return out


def test_weighted_mass_matches_gauss_quadrature():
    rng = np.random.default_rng(0)
    W = rng.standard_normal((4, 3))
    got = fem.weighted_mass_2d(W, 0.3, 0.7).toarray()
    ref = _bilinear_gauss_weighted_mass(W, 0.3, 0.7)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_invariants():
    ncx, ncy, hx, hy = 6, 5, 0.4, 0.3
    m = fem.StripMatrices(ncx, ncy, hx, hy)
    one = np.ones((ncx + 1) * (ncy + 1))
    area = ncx * hx * ncy * hy
    assert abs(one @ (m.M @ one) - area) < 1e-13
    assert np.max(np.abs(m.S @ one)) < 1e-13
    # boundary mass: each x-edge has length ncy*hy
    assert abs(one @ ((m.MGl + m.MGr) @ one) - 2 * ncy * hy) < 1e-13
    # constant potential: M_W = w M
    Wc = np.full((ncx + 1, ncy + 1), 2.5)
    assert np.max(np.abs((fem.weighted_mass_2d(Wc, hx, hy) - 2.5 * m.M).toarray())) < 1e-13
    # symmetry of every matrix
    W = np.random.default_rng(1).standard_normal((ncx + 1, ncy + 1))
    for A in (m.M, m.S, fem.weighted_mass_2d(W, hx, hy)):
        assert abs(A - A.T).max() < 1e-15
    # total integral of the interpolant: 1^T M_W 1 = int W_h
    MW = fem.weighted_mass_2d(W, hx, hy)
    trap = sum(hx * hy / 4 * (W[i, k] + W[i + 1, k] + W[i, k + 1] + W[i + 1, k + 1])
               for i in range(ncx) for k in range(ncy))
    assert abs(one @ (MW @ one) - trap) < 1e-13


def test_operator_is_complex_symmetric_with_definite_imaginary_part():
    m = fem.StripMatrices(5, 4, 0.2, 0.25)
    W = np.random.default_rng(2).standard_normal((6, 5))
    K = m.operator(W, 0.01, 0.5, 3.0, 1.0).toarray()
    assert np.max(np.abs(K - K.T)) < 1e-12
    assert np.linalg.eigvalsh(K.imag).min() > 0


@pytest.mark.parametrize("shape", [(2, 2), (5, 8), (17, 3)])
def test_matrix_free_weighted_mass_equals_the_assembled_matrix(shape):
    """The fixed point applies M_phi without assembling it; element by
    element it must give the assembled matrix's product (same exact triple
    products), for a complex vector and an arbitrary potential."""
    from oracle.fem import weighted_mass_2d, weighted_mass_apply
    rng = np.random.default_rng(sum(shape))
    W = rng.standard_normal(shape)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    a = (weighted_mass_2d(W, 0.37, 0.61) @ v.ravel()).reshape(shape)
    b = weighted_mass_apply(W, v, 0.37, 0.61)
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(a)) * 10
