"""Picard (source) iteration, DIRK stages and the explicit time-step bound.

* DIRK (Sec. 3.5, eq. dirk, eq. dirk-stages, eq. q-stages,
  eq. dirk-recursive-def): each stage s solves the steady problem
  eq. bgk-ss with sigma = nu + 1/(dt A_ss) and
  q^(s) = (f^k + dt sum_{r<s} A_sr F^(r)) / (dt A_ss);
  F^(s) = (f^(s) - f^k - dt sum_{r<s} A_sr F^(r)) / (dt A_ss);
  f^{k+1} = f^k + dt sum_s b_s F^(s).
* Picard (Sec. 4, eq. bgk-ss-picard): the Maxwellian and nu are lagged at
  iterate l, the sweep gives f^{l+1}, the moments of f^{l+1} give the next
  Maxwellian.  Stage 1 starts from f^k and stage s > 1 from the converged
  f^(s-1) (design note A3; the printed "s = 0" case is read as s = 1).
  On the Q2 velocity space of Sec. 3.2 the Maxwellian can instead be the
  conservative projection of App. B (mode PROJECTED, velocity.py).  Wall
  facets (bounce-back, reflection) take their data from the iterate before
  each sweep (walls.py).
* Stopping rule (eq. convergence-criteria, design note A13):
  max_m |U^{l+1,m} - U^{l,m}| / max(|U^{l,m}|, |U^{l,0}| s_m)
      < tau / max(1, max_i nu_i dt),
  with s_0 = s_2 = 0 and s_1 = 1 (guards the zero momentum of a gas at
  rest), unweighted l2 norms over DG nodes, momentum measured with the
  Euclidean norm of each node's vector.  After l_max iterations the stage
  fails (the GPU library reports BGK_E_NOT_CONVERGED).
* Time step (eq. explicit-dt): dt_e = (1/d) (1/(2k+1)) h_min / max_j |v_j|
  with h_min = (min cell measure)^{1/d}; dt = C dt_e.
* Tableaus (App. A): backward Euler; the L-stable two-stage DIRK with
  gamma = 1 - sqrt(2)/2; the L-stable three-stage DIRK with gamma the root
  of x^3 - 3x^2 + 3x/2 - 1/6 near 0.4359 (its printed 6-digit constants are
  derived exactly from gamma); the two-stage B-stable DIRK with
  gamma = (3 + sqrt(3))/6.
"""
from __future__ import annotations

import math

import numpy as np

from . import kinetic, transport, velocity, walls as wallbc
from .geometry import Geometry


class NonPhysicalError(RuntimeError):
    """Moments with n <= 0 or theta <= 0 at some node: no Maxwellian exists."""


def tableau(name: str):
    if name == "BE":
        return np.array([[1.0]]), np.array([1.0]), np.array([1.0])
    if name == "DIRK2":
        g = 1.0 - math.sqrt(2.0) / 2.0
        A = np.array([[g, 0.0], [math.sqrt(2.0) / 2.0, g]])
        return A, A[-1].copy(), A.sum(axis=1)
    if name == "DIRK3":
        # root of x^3 - 3x^2 + 3x/2 - 1/6 in (0.4, 0.5) by bisection
        lo, hi = 0.4, 0.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (mid ** 3 - 3 * mid ** 2 + 1.5 * mid - 1.0 / 6.0) > 0:
                lo = mid
            else:
                hi = mid
        g = 0.5 * (lo + hi)
        b1 = -(6 * g * g - 16 * g + 1) / 4.0
        b2 = (6 * g * g - 20 * g + 5) / 4.0
        A = np.array([[g, 0, 0], [(1 - g) / 2.0, g, 0], [b1, b2, g]])
        return A, A[-1].copy(), A.sum(axis=1)
    if name == "BDIRK2":
        g = (3.0 + math.sqrt(3.0)) / 6.0
        A = np.array([[g, 0.0], [1.0 - 2.0 * g, g]])
        return A, np.array([0.5, 0.5]), A.sum(axis=1)
    raise ValueError(name)


def explicit_dt(geo: Geometry, V: np.ndarray, cfl: float) -> float:
    h_min = float(np.min(geo.vol)) ** (1.0 / geo.dim)
    vmax = float(np.max(np.linalg.norm(V, axis=1)))
    return cfl * (1.0 / geo.dim) * (1.0 / (2 * geo.order + 1)) * h_min / vmax


def relative_changes(U_new: np.ndarray, U_old: np.ndarray, dim: int) -> np.ndarray:
    """The three ratios of eq. convergence-criteria with the A13 guard."""
    blocks = [slice(0, 1), slice(1, 1 + dim), slice(1 + dim, 2 + dim)]
    n0 = np.linalg.norm(U_old[..., 0])
    out = np.zeros(3)
    for m, sl in enumerate(blocks):
        num = np.linalg.norm(U_new[..., sl] - U_old[..., sl])
        den = np.linalg.norm(U_old[..., sl])
        if m == 1:
            den = max(den, n0)
        out[m] = num / den
    return out


def maxwellian_coefficients(U, V, w, mode: str, L: float, sticky=None):
    """Maxwellian coefficients per node.  MATCHED with ``sticky`` (bool per
    node, updated in place): a node whose Newton solve has failed once keeps
    the DIRECT coefficients for the rest of the stage (design reading A5:
    an iterate alternating between the two would never converge)."""
    dim = V.shape[1]
    if mode == "DIRECT":
        n, u, th = kinetic.primitive(U, dim)
        return kinetic.direct_coefficients(n, u, th), 0
    if mode == "MATCHED":
        if sticky is None:
            return kinetic.matched_coefficients(U, V, w)
        failed = np.zeros(sticky.shape, dtype=bool)
        coef, nfb = kinetic.matched_coefficients(U, V, w, force_direct=sticky, failed=failed)
        sticky |= failed
        return coef, nfb
    if mode == "LINEAR":
        return kinetic.linear_coefficients(U, L, dim), 0
    raise ValueError(mode)


def picard_stage(geo: Geometry, V, w, q, gbc, sigma_shift, f_init, gens, lagged, *, dt,
                 mode="MATCHED", nu_model="const", nu_const=1.0, kn=1.0, tau=1e-10,
                 lmax=2000, fixed_iters=None, U_init=None, L=0.0, vcells=0, walls=None):
    """Picard iteration for one DIRK stage.  Returns (f, U, iterations, history).

    mode PROJECTED (the Q2 velocity space of Sec. 3.2 with ``vcells`` cells
    per axis on [-L, L]): the Maxwellian is the conservative projection of
    App. B of M_{n,u,theta} with (n, u, theta) from U.
    ``walls`` (optional, [n_bfaces] of walls.INFLOW / BOUNCE_BACK / REFLECT):
    before each sweep the wall facets' data are taken from the current
    iterate (walls.py)."""
    dim = geo.dim
    f = f_init
    U = kinetic.moments(f, V, w) if U_init is None else U_init
    hist = []
    nfb = 0
    sticky = np.zeros(U.shape[:-1], dtype=bool)
    for ell in range(lmax):
        collisional = not (nu_model == "const" and nu_const == 0.0)
        needs_theta = not (mode == "LINEAR" and nu_model == "const")
        n_, _, th_ = kinetic.primitive(U, dim)
        ok = np.all(n_ > 0) and np.all(np.isfinite(n_))
        if needs_theta:
            ok = ok and np.all(th_ > 0) and np.all(np.isfinite(th_))
        if collisional and not ok:
            raise NonPhysicalError("non-physical moments (n <= 0 or theta <= 0)")
        nu = kinetic.collision_frequency(U, dim, nu_model, nu_const, kn)
        if np.any(nu != 0.0) and mode == "PROJECTED":
            Mv = velocity.projected_maxwellian(n_, kinetic.primitive(U, dim)[1], th_, vcells, L)
        elif np.any(nu != 0.0):
            coef, fb = maxwellian_coefficients(U, V, w, mode, L, sticky)
            nfb += fb
            Mv = kinetic.coef_values(coef, V)
        else:                      # collision term vanishes: no Maxwellian needed
            Mv = np.zeros_like(q)
        g_it = gbc if walls is None else wallbc.wall_values(geo, V, f, walls, gbc)
        f_new = transport.sweep(geo, V, nu + sigma_shift, nu, Mv, q, g_it, gens, lagged, f)
        U_new = kinetic.moments(f_new, V, w)
        ratio = relative_changes(U_new, U, dim)
        hist.append(float(ratio.max()))
        f, U = f_new, U_new
        if fixed_iters is not None:
            if ell + 1 >= fixed_iters:
                return f, U, ell + 1, hist, nfb
            continue
        if ratio.max() < tau / max(1.0, float(np.max(nu)) * dt):
            return f, U, ell + 1, hist, nfb
    raise RuntimeError("Picard iteration did not converge")


def bgk_step(geo: Geometry, V, w, f, gbc, dt, gens, lagged=None, *, scheme="BE",
             mode="MATCHED", nu_model="const", nu_const=1.0, kn=1.0, tau=1e-10, lmax=2000,
             fixed_iters=None, U_guess=None, L=0.0, vcells=0, walls=None):
    """One DIRK time step of the discretised BGK equation.

    ``gbc`` is either the boundary data [n_bf][n_fp][N_v] or a callable
    gbc(stage_index) returning it.  ``U_guess`` (optional) replaces the
    moments of f^k as the first stage's initial Picard iterate.  ``walls``
    marks bounce-back and reflecting boundary facets (picard_stage).
    Returns (f^{k+1}, stats dict).
    """
    A, b, _ = tableau(scheme)
    S = A.shape[0]
    Fs = []
    stage_f = f
    iters, hists, nfb_tot = [], [], 0
    for s in range(S):
        acc = f.copy()
        for r in range(s):
            acc = acc + dt * A[s, r] * Fs[r]
        q = acc / (dt * A[s, s])
        g = gbc(s) if callable(gbc) else gbc
        f_s, U_s, it, hist, nfb = picard_stage(
            geo, V, w, q, g, 1.0 / (dt * A[s, s]), stage_f, gens, lagged, dt=dt, mode=mode,
            nu_model=nu_model, nu_const=nu_const, kn=kn, tau=tau, lmax=lmax,
            fixed_iters=fixed_iters, U_init=U_guess if s == 0 else None, L=L, vcells=vcells,
            walls=walls)
        Fs.append((f_s - acc) / (dt * A[s, s]))
        stage_f = f_s
        iters.append(it)
        hists.append(hist)
        nfb_tot += nfb
    f_new = f.copy()
    for s in range(S):
        f_new = f_new + dt * b[s] * Fs[s]
    return f_new, {"iters": iters, "hist": hists, "fallbacks": nfb_tot, "U": U_s}


def initial_condition(geo: Geometry, V, state) -> np.ndarray:
    """Nodal interpolation of the initial Maxwellians (design note A7)."""
    n, u, th = state.params(geo.node_x.reshape(-1, geo.dim))
    return kinetic.maxwellian_values(n, u, th, V).reshape(geo.n_cells, geo.n_p, -1)


def boundary_values(geo: Geometry, V, state) -> np.ndarray:
    """Inflow data: the state's Maxwellian at each boundary facet node (A8)."""
    n, u, th = state.params(geo.bnode_x.reshape(-1, geo.dim))
    return kinetic.maxwellian_values(n, u, th, V).reshape(geo.bnode_x.shape[0], geo.n_fp, -1)
