"""Oracle pins: velocity moments, primitive variables and discrete Maxwellians.

* A nodal Maxwellian on a resolved trapezoid grid has the closed-form
  moments of eq. moments: (n, n u, n|u|^2/2 + (d/2) n theta) -- trapezoid
  quadrature is spectrally accurate for Gaussians.
* MATCHED: the discrete moments of the returned Gaussian equal U; applied to
  the moments of a nodal Gaussian it returns that Gaussian's coefficients;
  Newton converges quadratically.
* Coefficient form: exp(a + b.v + c|v|^2) reproduces the Maxwellian formula
  of Sec. 2 and inverts back to (n, u, theta).
"""
import math

import numpy as np
import pytest

import problems as P
from oracle import kinetic
from tests.conftest import read_golden


def test_trapezoid_weights_integrate_polynomials_on_tensor_grid():
    vg = P.tensor_velocity_grid(16, 6.0, 2)
    # trapezoid rule is exact for affine functions on each axis
    assert abs(vg.w.sum() - 144.0) < 1e-12
    assert abs((vg.w * vg.v[:, 0]).sum()) < 1e-12
    assert abs((vg.w * vg.v[:, 0] * vg.v[:, 1]).sum()) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_moments_of_nodal_maxwellian_closed_form(dim):
    vg = P.tensor_velocity_grid(48 if dim == 2 else 40, 10.0, dim)
    rng = np.random.default_rng(dim)
    n = rng.uniform(0.1, 2.0, 5)
    u = rng.uniform(-0.5, 0.5, (5, dim))
    th = rng.uniform(0.6, 1.3, 5)
    f = kinetic.maxwellian_values(n, u, th, vg.v)
    U = kinetic.moments(f, vg.v, vg.w)
    exact = np.concatenate([n[:, None], n[:, None] * u,
                            (0.5 * n * np.sum(u * u, 1) + 0.5 * dim * n * th)[:, None]], 1)
    assert np.abs(U - exact).max() <= 1e-13 * np.abs(exact).max()
    n2, u2, th2 = kinetic.primitive(U, dim)
    assert np.allclose(n2, n, rtol=1e-13) and np.allclose(u2, u, atol=1e-13)
    assert np.allclose(th2, th, rtol=1e-12)


def test_coefficient_form_matches_formula():
    vg = P.tensor_velocity_grid(12, 6.0, 2)
    n, u, th = np.array([0.7]), np.array([[0.3, -0.2]]), np.array([0.9])
    coef = kinetic.direct_coefficients(n, u, th)
    a = kinetic.coef_values(coef, vg.v)
    b = n[0] / (2 * math.pi * th[0]) * np.exp(-np.sum((vg.v - u[0]) ** 2, 1) / (2 * th[0]))
    assert np.abs(a[0] - b).max() <= 1e-14 * b.max()
    n2, u2, th2 = kinetic.coefficients_to_primitive(coef, 2)
    assert np.allclose([n2[0], th2[0]], [n[0], th[0]], rtol=1e-14)
    assert np.allclose(u2, u, atol=1e-15)


@pytest.mark.parametrize("dim,n1,L", [(2, 16, 6.0), (2, 8, 6.0), (3, 10, 6.0)])
def test_matched_maxwellian_moments_exact(dim, n1, L):
    vg = P.tensor_velocity_grid(n1, L, dim)
    rng = np.random.default_rng(n1)
    # moments of Sod-like states, some hot and shifted enough that the nodal
    # Gaussian misses the discrete moments by far more than 1e-14
    n = rng.uniform(0.1, 1.5, 6)
    u = rng.uniform(-1.0, 1.0, (6, dim))
    th = rng.uniform(0.5, 2.0, 6)
    f = kinetic.maxwellian_values(n, u, th, vg.v) * (1 + 0.1 * np.cos(vg.v[:, 0]))[None]
    U = kinetic.moments(f, vg.v, vg.w)
    coef, nfb = kinetic.matched_coefficients(U, vg.v, vg.w)
    assert nfb == 0
    U2 = kinetic.moments(kinetic.coef_values(coef, vg.v), vg.v, vg.w)
    assert np.abs(U2 - U).max() <= 2e-14 * np.abs(U).max()
    # direct Gaussian does *not* match (so the test above is not vacuous)
    n0, u0, th0 = kinetic.primitive(U, dim)
    Ud = kinetic.moments(kinetic.maxwellian_values(n0, u0, th0, vg.v), vg.v, vg.w)
    assert np.abs(Ud - U).max() > 1e-10 * np.abs(U).max()


def test_matched_idempotent_on_nodal_gaussian():
    vg = P.tensor_velocity_grid(10, 5.0, 2)
    coef_true = np.array([[-1.3, 0.4, -0.2, -0.6], [0.2, -0.1, 0.3, -0.45]])
    U = kinetic.moments(kinetic.coef_values(coef_true, vg.v), vg.v, vg.w)
    coef, nfb = kinetic.matched_coefficients(U, vg.v, vg.w)
    assert nfb == 0
    assert np.abs(coef - coef_true).max() < 1e-12


def test_matched_newton_quadratic_convergence():
    vg = P.tensor_velocity_grid(8, 6.0, 2)
    U = kinetic.moments(kinetic.maxwellian_values(np.array([1.0]), np.array([[0.8, 0.0]]),
                                                  np.array([1.6]), vg.v), vg.v, vg.w)[0]
    P_ = np.concatenate([np.ones((64, 1)), vg.v, np.sum(vg.v ** 2, 1)[:, None]], 1)
    E = kinetic.collision_invariants(vg.v)
    n, u, th = kinetic.primitive(U, 2)
    x = kinetic.direct_coefficients(np.array([n]), u[None], np.array([th]))[0]
    res = []
    for _ in range(6):
        M = np.exp(P_ @ x)
        r = (vg.w * M) @ E - U
        res.append(np.linalg.norm(r))
        x = x - np.linalg.solve(E.T @ ((vg.w * M)[:, None] * P_), r)
    # quadratic: log residual roughly doubles while above round-off
    big = [r for r in res if r > 1e-13]
    assert len(big) >= 3
    for a, b in zip(big[1:], big[2:]):
        assert b < 10 * a * a / res[0] + 1e-13


def test_sod_states_from_paper(golden):
    g = golden("sod_states.txt")
    st = P.sod_state(2)
    n, u, th = st.params(np.array([[0.25, 0.5], [0.75, 0.5]]))
    assert [n[0], u[0, 0], th[0]] == [float(x) for x in g["H"]]
    assert [n[1], u[1, 0], th[1]] == [float(x) for x in g["XminusH"]]


def test_linear_maxwellian_and_collision_frequency():
    U = np.array([[2.0, 0.0, 0.0, 3.0]])
    c = kinetic.linear_coefficients(U, 6.0, 2)
    assert np.isclose(np.exp(c[0, 0]), 2.0 / 144.0)
    nu = kinetic.collision_frequency(U, 2, "kn", kn=0.01)
    # n = 2, theta = (2*3/2 - 0)/2 = 1.5 -> nu = 2/sqrt(1.5)/0.01
    assert np.isclose(nu[0], 2.0 / math.sqrt(1.5) / 0.01)


def test_matched_fallback_is_sticky_within_a_stage():
    """On an 8-point grid without v = 0 no non-negative discrete
    distribution has mean 0 and variance below 0.857^2 per axis, so the
    moments (1, 0, theta = 0.3) have no matched Maxwellian: Newton fails and
    the node takes DIRECT.  With the stage's sticky flags the node then
    stays on DIRECT even for realisable moments (A5 reading)."""
    from oracle import solver
    vg = P.tensor_velocity_grid(8, 6.0, 2)
    assert np.min(np.abs(vg.v[:, 0])) > 0.8
    U_bad = np.array([[1.0, 0.0, 0.0, 0.3], [1.0, 0.0, 0.0, 1.0]])     # theta 0.3 and 1.0
    sticky = np.zeros(2, dtype=bool)
    coef, nfb = solver.maxwellian_coefficients(U_bad, vg.v, vg.w, "MATCHED", 0.0, sticky)
    assert nfb == 1 and sticky.tolist() == [True, False]
    n, u, th = kinetic.primitive(U_bad, 2)
    np.testing.assert_array_equal(coef[0], kinetic.direct_coefficients(n, u, th)[0])
    # realisable moments at both nodes: node 0 stays on DIRECT, node 1 matches
    U_ok = np.array([[1.0, 0.0, 0.0, 1.2], [1.0, 0.0, 0.0, 1.2]])
    coef, nfb = solver.maxwellian_coefficients(U_ok, vg.v, vg.w, "MATCHED", 0.0, sticky)
    assert nfb == 1 and sticky.tolist() == [True, False]
    n, u, th = kinetic.primitive(U_ok, 2)
    direct = kinetic.direct_coefficients(n, u, th)
    np.testing.assert_array_equal(coef[0], direct[0])
    assert np.abs(coef[1] - direct[1]).max() > 1e-8
    U2 = kinetic.moments(kinetic.coef_values(coef[1:], vg.v), vg.v, vg.w)
    assert np.abs(U2 - U_ok[1:]).max() <= 1e-14 * np.abs(U_ok).max() * 10
    # without sticky flags the same call matches both nodes
    coef, nfb = solver.maxwellian_coefficients(U_ok, vg.v, vg.w, "MATCHED", 0.0)
    assert nfb == 0
