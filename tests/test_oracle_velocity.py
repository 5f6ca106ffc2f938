"""Pins of the Q2 velocity space and the conservative projection (App. B).

* the Gauss-Legendre nodes and weights integrate polynomials of degree 5
  exactly on every cell (the quadrature assumption of Sec. 3.2);
* the 1D projection equals brute-force adaptive quadrature of its defining
  integrals (Gaussian times each Lagrange polynomial, the first and last
  cells extended to infinity);
* the projected Maxwellian's discrete moments equal the Maxwellian's
  moments over R^d (eq. cons_projection_exactness) in 2D and 3D, also for
  Maxwellians reaching out of the velocity box;
* a centred Maxwellian projects to a symmetric set of values.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import problems as P
from oracle import kinetic, velocity


def test_grid_matches_problem_grid_and_is_exact_to_degree_5():
    x, w = velocity.grid_1d(7, 5.0)
    g = P.gl_velocity_grid(7, 5.0, 2)
    np.testing.assert_allclose(g.nodes_1d, x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(g.weights_1d, w, rtol=1e-15)
    h = 10.0 / 7
    for c in range(7):
        a = -5.0 + c * h
        sl = slice(3 * c, 3 * c + 3)
        for k in range(6):
            exact = ((a + h) ** (k + 1) - a ** (k + 1)) / (k + 1)
            assert abs(np.sum(w[sl] * x[sl] ** k) - exact) <= 1e-13 * max(1.0, abs(exact))


@pytest.mark.parametrize("u,theta", [(0.3, 0.8), (-2.7, 0.4), (4.6, 1.3), (0.0, 3.0)])
def test_projection_1d_matches_brute_force_quadrature(u, theta):
    n_cells, L = 5, 5.0
    p = velocity.project_gaussian_1d(u, theta, n_cells, L)
    x, w = velocity.grid_1d(n_cells, L)
    h = 2 * L / n_cells
    xi, _ = velocity.gl_reference()
    g = lambda t: math.exp(-(t - u) ** 2 / (2 * theta))
    for c in range(n_cells):
        lo = -math.inf if c == 0 else -L + c * h
        hi = math.inf if c == n_cells - 1 else -L + (c + 1) * h
        centre = -L + (c + 0.5) * h
        for i in range(3):
            others = [m for m in range(3) if m != i]

            def ell(t, i=i, others=others):
                y = (t - centre) / (0.5 * h)
                r = 1.0
                for m in others:
                    r *= (y - xi[m]) / (xi[i] - xi[m])
                return r
            if math.isinf(lo) or math.isinf(hi):
                # split at the cell so the finite part is resolved
                edge = -L + h if math.isinf(lo) else -L + (n_cells - 1) * h
                parts = [(lo, edge), (edge, -L + h)] if math.isinf(lo) else \
                    [(-L + c * h, L), (L, hi)]
            else:
                parts = [(lo, hi)]
            val = sum(integrate.quad(lambda t: g(t) * ell(t), a_, b_, epsabs=1e-15,
                                     epsrel=1e-13, limit=200)[0] for a_, b_ in parts
                      if a_ < b_)
            assert abs(p[3 * c + i] - val / w[3 * c + i]) <= 1e-12 * max(1.0, abs(p).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_projected_maxwellian_moments_are_exact(dim):
    rng = np.random.default_rng(80 + dim)
    n_cells, L = 6, 6.0
    g = P.gl_velocity_grid(n_cells, L, dim)
    npts = 40
    n = rng.uniform(0.1, 2.0, npts)
    u = rng.uniform(-3.0, 3.0, (npts, dim))
    u[0] = [5.5] + [0.0] * (dim - 1)       # centred near the box edge
    th = rng.uniform(0.3, 2.5, npts)
    th[1] = 4.0                            # wide: much mass outside the box
    Mv = velocity.projected_maxwellian(n, u, th, n_cells, L)
    U = kinetic.moments(Mv, g.v, g.w)
    Uref = np.concatenate([n[:, None], n[:, None] * u,
                           (0.5 * n * (dim * th + np.sum(u * u, axis=1)))[:, None]], axis=1)
    assert np.abs(U - Uref).max() <= 1e-12 * np.abs(Uref).max()
    # the point values alone do not have this property
    Mi = kinetic.maxwellian_values(n, u, th, g.v)
    assert np.abs(kinetic.moments(Mi, g.v, g.w) - Uref).max() > 1e-4


def test_centred_projection_is_symmetric():
    p = velocity.project_gaussian_1d(0.0, 1.1, 8, 6.0)
    np.testing.assert_allclose(p, p[::-1], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("u,theta", [(0.3, 0.7), (-1.1, 1.4)])
def test_projection_1d_relative_accuracy_on_a_fine_grid(u, theta):
    """64 cells on [-7, 7] (the Sod strip's reference grid): every value, also
    many half-cells from u where the closed form's expansion cancels, equals
    adaptive quadrature of its defining integral to 1e-13 of itself."""
    n_cells, L = 64, 7.0
    p = velocity.project_gaussian_1d(u, theta, n_cells, L)
    x, w = velocity.grid_1d(n_cells, L)
    h = 2 * L / n_cells
    xi, _ = velocity.gl_reference()
    g = lambda t: math.exp(-(t - u) ** 2 / (2 * theta))  # noqa: E731
    checked = 0
    for c in range(1, n_cells - 1):
        lo, hi, centre = -L + c * h, -L + (c + 1) * h, -L + (c + 0.5) * h
        if abs(centre - u) > 5.0 * math.sqrt(theta):
            continue
        for i in range(3):
            others = [m for m in range(3) if m != i]

            def ell(t, i=i, others=others):
                y = (t - centre) / (0.5 * h)
                r = 1.0
                for m in others:
                    r *= (y - xi[m]) / (xi[i] - xi[m])
                return r
            val = integrate.quad(lambda t: g(t) * ell(t), lo, hi, epsabs=0.0, epsrel=1.2e-14,
                                 limit=200)[0] / w[3 * c + i]
            assert abs(p[3 * c + i] - val) <= 1e-13 * abs(val), (c, i, p[3 * c + i], val)
            checked += 1
    assert checked > 100
