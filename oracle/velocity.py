"""Q2 discontinuous-Galerkin velocity space and its conservative projection.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use the oracle; the library never does.

* Velocity space (Sec. 3.2, eq. discrete_space_v): [-L, L]^d cut into n
  uniform cells per axis, Q^{k_v} on each with k_v = 2 and the tensor
  Lagrange basis at the 3 Gauss-Legendre points of every cell; those points
  and the Gauss-Legendre weights (times h/2) are the velocity nodes and the
  quadrature weights (the rule is exact to degree 5 = 2 k_v + 1, the
  assumption of Sec. 3.2).
* Projection (App. B, eq. cons_projection_equation): P zeta in W_v with
      int_V (P zeta) xi dv = int_{R^d} zeta (E xi) dv   for every xi in W_v,
  where E extends the first and last cells' polynomials to -inf and +inf.
  For the Maxwellian, P factors over the axes into 1D projections of
  Gaussians.  With the Lagrange basis at Gauss-Legendre points the cell
  mass matrix is the diagonal of the quadrature weights, so the value at
  node i of cell c is
      p_i = (1/w_i) int_{I~_c} g(x) l_i(x) dx,
  I~_c the cell, extended to -inf for the first cell and to +inf for the
  last; the integrals of the Gaussian times 1, x, x^2 over an interval are
  written with erf/erfc and exp (or, where that closed form cancels, by
  Gauss-Legendre quadrature; project_gaussian_1d).  The moments (1, v, |v|^2/2) of the
  projected Maxwellian equal the Maxwellian's own moments over R^d
  (eq. cons_projection_exactness).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

N_LOCAL = 3  # Gauss-Legendre points per cell (k_v = 2)


def gl_reference():
    """Reference nodes xi_i in [-1, 1] and weights of 3-point Gauss-Legendre."""
    xi, wr = np.polynomial.legendre.leggauss(N_LOCAL)
    return xi, wr


def lagrange_monomials():
    """C[k][i]: l_i(xi) = sum_k C[k][i] xi^k for the Lagrange basis at the
    reference Gauss-Legendre points."""
    xi, _ = gl_reference()
    vand = np.vander(xi, N_LOCAL, increasing=True)   # vand[m][k] = xi_m^k
    return np.linalg.inv(vand)


def grid_1d(n_cells: int, L: float):
    """1D nodes and weights of the velocity space, cell by cell."""
    xi, wr = gl_reference()
    h = 2.0 * L / n_cells
    centres = -L + h * (np.arange(n_cells) + 0.5)
    x = (centres[:, None] + 0.5 * h * xi[None, :]).ravel()
    w = np.tile(0.5 * h * wr, n_cells)
    return x, w


def gaussian_moments(ta, tb):
    """G_m = int_ta^tb t^m exp(-t^2/2) dt for m = 0, 1, 2 (ta may be -inf,
    tb +inf).  G_0 uses erfc when both limits lie on one side of 0."""
    ta = np.asarray(ta, dtype=np.float64)
    tb = np.asarray(tb, dtype=np.float64)
    c = math.sqrt(0.5 * math.pi)
    r = 1.0 / math.sqrt(2.0)
    g0 = np.where(ta >= 0.0, c * (special.erfc(ta * r) - special.erfc(tb * r)),
                  np.where(tb <= 0.0, c * (special.erfc(-tb * r) - special.erfc(-ta * r)),
                           c * (special.erf(tb * r) - special.erf(ta * r))))
    with np.errstate(invalid="ignore"):
        ea = np.where(np.isfinite(ta), np.exp(-0.5 * ta * ta), 0.0)
        eb = np.where(np.isfinite(tb), np.exp(-0.5 * tb * tb), 0.0)
        tea = np.where(np.isfinite(ta), ta * ea, 0.0)
        teb = np.where(np.isfinite(tb), tb * eb, 0.0)
    return g0, ea - eb, g0 + tea - teb


N_QUAD = 20  # Gauss-Legendre points for the cell integrals in the quadrature regime


def project_gaussian_1d(u, theta, n_cells: int, L: float) -> np.ndarray:
    """Nodal values of the projection of g(x) = exp(-(x-u)^2/(2 theta)) onto
    the 1D velocity space: [..., 3 n_cells] for arrays u, theta.

    The cell integrals m_k = int g(x) y^k dx (y the cell's reference
    coordinate) are evaluated two ways, both exact up to rounding:
    * closed form: with x = u + sigma t, y = al + be t, from the Gaussian
      moments G_m (erf/erfc);
    * quadrature: with t = t_c + s (t_c the cell centre, s in [-d, d],
      d = (h/2)/sigma), m_k = sigma be^k exp(-t_c^2/2) K_k where
      K_k = int_{-d}^{d} s^k exp(-t_c s - s^2/2) ds, by 20-point
      Gauss-Legendre; for d <= 1 and |t_c| d <= 3 the integrand is an entire
      function whose 2N-th derivative bounds the rule's error below 1e-20
      relative.
    The closed form expands y^2 = (al + be t)^2 and loses about
    log10(12 al^2) digits where al is large (a cell many half-widths from
    u, on a fine grid); the quadrature has no such cancellation, so it is
    used in its regime (interior cells with d <= 1 and |t_c| d <= 3), the
    closed form elsewhere (the extended end cells, coarse cells)."""
    u = np.asarray(u, dtype=np.float64)[..., None]
    theta = np.asarray(theta, dtype=np.float64)[..., None]
    sig = np.sqrt(theta)
    h = 2.0 * L / n_cells
    lo = -L + h * np.arange(n_cells)
    hi = lo + h
    lo = np.where(np.arange(n_cells) == 0, -np.inf, lo)
    hi = np.where(np.arange(n_cells) == n_cells - 1, np.inf, hi)
    g0, g1, g2 = gaussian_moments((lo - u) / sig, (hi - u) / sig)     # [..., n_cells]
    centres = -L + h * (np.arange(n_cells) + 0.5)
    al = (u - centres) / (0.5 * h)       # x = centre + (h/2) y,  y = al + be t
    be = sig / (0.5 * h)
    m0 = sig * g0                        # int g(x) y^k dx, k = 0, 1, 2
    m1 = sig * (al * g0 + be * g1)
    m2 = sig * (al * al * g0 + 2.0 * al * be * g1 + be * be * g2)
    # quadrature regime
    tc = (centres - u) / sig
    d = 1.0 / be
    interior = (np.arange(n_cells) > 0) & (np.arange(n_cells) < n_cells - 1)
    quad = interior & (d <= 1.0) & (np.abs(tc) * d <= 3.0)
    if np.any(quad):
        xq, wq = np.polynomial.legendre.leggauss(N_QUAD)
        s = d[..., None] * xq                                       # [..., 1|n, N]
        e = np.exp(-tc[..., None] * s - 0.5 * s * s) * (d[..., None] * wq)
        K0 = e.sum(-1)
        K1 = (e * s).sum(-1)
        K2 = (e * s * s).sum(-1)
        scale = sig * np.exp(-0.5 * tc * tc)
        m0 = np.where(quad, scale * K0, m0)
        m1 = np.where(quad, scale * be * K1, m1)
        m2 = np.where(quad, scale * be * be * K2, m2)
    C = lagrange_monomials()
    _, wr = gl_reference()
    w = 0.5 * h * wr
    p = (C[0][None, :] * m0[..., None] + C[1][None, :] * m1[..., None]
         + C[2][None, :] * m2[..., None]) / w                           # [..., n_cells, 3]
    return p.reshape(p.shape[:-2] + (n_cells * N_LOCAL,))


def projected_maxwellian(n, u, theta, n_cells: int, L: float) -> np.ndarray:
    """P M_{n,u,theta} at the velocity nodes, [..., N_v] with the tensor
    index's first axis slowest: n (2 pi theta)^{-d/2} prod_a P g_a."""
    n = np.asarray(n, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    dim = u.shape[-1]
    out = (n * (2.0 * math.pi * theta) ** (-0.5 * dim))[..., None]
    for a in range(dim):
        pa = project_gaussian_1d(u[..., a], theta, n_cells, L)
        out = (out[..., :, None] * pa[..., None, :]).reshape(out.shape[:-1] + (-1,))
    return out
