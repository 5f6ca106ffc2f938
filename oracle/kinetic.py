"""Velocity moments, primitive variables, discrete Maxwellians, collision frequency.

* Moments (eq. moments, Sec. 4 before eq. convergence-criteria): at every DG
  node U = sum_j w_j e(v_j) f_j with e = (1, v, |v|^2/2).
* Primitive variables (eq. primitive_g, with the 1/n_d typo read as 1/n_g):
  n = U_0, u = U_1/n, theta = (2 U_2/n - |u|^2)/d.
* Maxwellian (Sec. 2): M_{n,u,theta}(v) = n (2 pi theta)^{-d/2} exp(-|v-u|^2/(2 theta)).
* Discrete Maxwellian (eq. Maxwellian-projection restated for the velocity
  quadrature in use; design note A5):
    DIRECT   - the Maxwellian of (n, u, theta) sampled at the nodes;
    MATCHED  - the nodal Gaussian exp(a + b.v + c|v|^2) whose discrete moments
               equal U exactly, found by Newton's method from DIRECT;
    LINEAR   - the simplified linear Maxwellian N_h = n/|V| (eq. linear-Maxwellian).
* Collision frequency (design note A12): constant, or nu = n theta^{-1/2}/Kn.

Maxwellians are carried as exponential-family coefficients (a, b, c) with
M(v) = exp(a + b.v + c|v|^2); ``direct_coefficients`` converts (n, u, theta).
"""
from __future__ import annotations

import math

import numpy as np


def collision_invariants(V: np.ndarray) -> np.ndarray:
    """e(v_j) = (1, v_j, |v_j|^2/2), shape [N_v][d+2]."""
    V = np.asarray(V, dtype=np.float64)
    return np.concatenate([np.ones((V.shape[0], 1)), V, 0.5 * np.sum(V * V, axis=1)[:, None]],
                          axis=1)


def moments(f: np.ndarray, V: np.ndarray, w: np.ndarray) -> np.ndarray:
    """U[..., m] = sum_j w_j e_m(v_j) f[..., j]."""
    E = collision_invariants(V) * np.asarray(w)[:, None]
    return np.einsum("...j,jm->...m", f, E)


def primitive(U: np.ndarray, dim: int):
    n = U[..., 0]
    u = U[..., 1:1 + dim] / n[..., None]
    theta = (2.0 * U[..., 1 + dim] / n - np.sum(u * u, axis=-1)) / dim
    return n, u, theta


def maxwellian_values(n, u, theta, V) -> np.ndarray:
    """M_{n,u,theta}(v_j) for arrays of parameters (leading shape) -> [..., N_v]."""
    V = np.asarray(V, dtype=np.float64)
    dim = V.shape[1]
    d2 = np.sum((V[None, :, :] - u.reshape(-1, dim)[:, None, :]) ** 2, axis=2)
    th = theta.reshape(-1)[:, None]
    out = n.reshape(-1)[:, None] * (2.0 * math.pi * th) ** (-0.5 * dim) * np.exp(-d2 / (2.0 * th))
    return out.reshape(tuple(n.shape) + (V.shape[0],))


def coef_values(coef: np.ndarray, V: np.ndarray) -> np.ndarray:
    """exp(a + b.v_j + c|v_j|^2) for coef[..., d+2] = (a, b, c) -> [..., N_v]."""
    V = np.asarray(V, dtype=np.float64)
    dim = V.shape[1]
    c2 = coef.reshape(-1, dim + 2)
    expo = c2[:, :1] + c2[:, 1:1 + dim] @ V.T + c2[:, 1 + dim:] * np.sum(V * V, axis=1)[None, :]
    return np.exp(expo).reshape(tuple(coef.shape[:-1]) + (V.shape[0],))


def direct_coefficients(n, u, theta) -> np.ndarray:
    """(a, b, c) with exp(a + b.v + c|v|^2) = M_{n,u,theta}(v)."""
    dim = u.shape[-1]
    c = -0.5 / theta
    b = u / theta[..., None]
    a = np.log(n) - 0.5 * dim * np.log(2.0 * math.pi * theta) - 0.5 * np.sum(u * u, axis=-1) / theta
    return np.concatenate([a[..., None], b, c[..., None]], axis=-1)


def coefficients_to_primitive(coef: np.ndarray, dim: int):
    """Inverse of direct_coefficients: theta = -1/(2c), u = b theta,
    n = exp(a + |u|^2/(2 theta)) (2 pi theta)^{d/2}."""
    a, b, c = coef[..., 0], coef[..., 1:1 + dim], coef[..., 1 + dim]
    theta = -0.5 / c
    u = b * theta[..., None]
    n = np.exp(a + 0.5 * np.sum(u * u, axis=-1) / theta) * (2.0 * math.pi * theta) ** (0.5 * dim)
    return n, u, theta


def matched_coefficients(U: np.ndarray, V: np.ndarray, w: np.ndarray, tol=1e-14, maxit=30,
                         force_direct=None, failed=None):
    """Newton solve of sum_j w_j e(v_j) exp(a + b.v_j + c|v_j|^2) = U per node.

    Starts from the DIRECT coefficients; stops when the residual is below
    tol*|U| (Euclidean) or after maxit iterations, in which case that node
    falls back to DIRECT.  Nodes flagged in ``force_direct`` (bool per node)
    skip Newton and take DIRECT; ``failed`` (bool per node, written) marks
    the nodes that took DIRECT.  Returns (coef[N][d+2], n_fallback), the
    count including forced nodes.
    """
    V = np.asarray(V, dtype=np.float64)
    dim = V.shape[1]
    Uf = U.reshape(-1, dim + 2)
    n, u, th = primitive(Uf, dim)
    coef0 = direct_coefficients(n, u, th)
    E = collision_invariants(V)                                 # rows e_j
    P = np.concatenate([np.ones((V.shape[0], 1)), V, np.sum(V * V, axis=1)[:, None]], axis=1)
    out = coef0.copy()
    nfb = 0
    fd = None if force_direct is None else np.asarray(force_direct).reshape(-1)
    fl = None if failed is None else failed.reshape(-1)
    for i in range(Uf.shape[0]):
        if fd is not None and fd[i]:
            nfb += 1
            if fl is not None:
                fl[i] = True
            continue
        x = coef0[i].copy()
        ok = False
        with np.errstate(all="ignore"):
            for _ in range(maxit + 1):
                M = np.exp(P @ x)
                r = (w * M) @ E - Uf[i]
                if np.linalg.norm(r) <= tol * np.linalg.norm(Uf[i]):
                    ok = True
                    break
                Jac = E.T @ ((w * M)[:, None] * P)
                try:
                    x = x - np.linalg.solve(Jac, r)
                except np.linalg.LinAlgError:
                    break
                if not np.all(np.isfinite(x)):
                    break
        if ok and np.all(np.isfinite(x)) and x[-1] < 0.0:
            out[i] = x
        else:
            nfb += 1
            if fl is not None:
                fl[i] = True
    return out.reshape(U.shape[:-1] + (dim + 2,)), nfb


def linear_coefficients(U: np.ndarray, L: float, dim: int) -> np.ndarray:
    """N_h = n/|V| with |V| = (2L)^d, as (a, 0, 0) coefficients."""
    n = U[..., 0]
    out = np.zeros(U.shape[:-1] + (dim + 2,))
    out[..., 0] = np.log(n / (2.0 * L) ** dim)
    return out


def collision_frequency(U: np.ndarray, dim: int, model: str, nu_const=1.0, kn=1.0):
    if model == "const":
        return np.full(U.shape[:-1], float(nu_const))
    n, _, th = primitive(U, dim)
    return n / np.sqrt(th) / kn
