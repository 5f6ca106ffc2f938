"""Reference for the learned Picard initial guess (not part of the paper).

The network maps per-DG-node features to a correction of the primitive
state: inputs (n, u_1, u_2, u_3, theta) at step t-1, its change from t-2
to t-1, and dt*nu at t-1 (11 features; 2D states have u_3 = 0), three hidden layers of 64 with
the exact GELU g(z) = z Phi(z) = z (1 + erf(z/sqrt 2))/2, and 5 linear
outputs (the normalised difference between (n, u, theta) at t and its
linear extrapolation from t-2 and t-1).  Loss: mean
squared error over rows and outputs.

Two paths:
  * FP64: plain forward and back-propagation (the mathematical reference,
    pinned by finite differences).
  * BF16: emulates the GPU kernels' rounding -- inputs, weights and hidden
    activations rounded to bfloat16 (round to nearest even), products summed
    in float32, biases, GELU and its derivative in float32; in the backward
    pass the upstream gradients are rounded to bfloat16 before each product.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

ARCH = (11, 64, 64, 64, 5)


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _mm(a, b, mode):
    if mode == "fp64":
        return a @ b
    # bf16 operands, exact products, float32 sums
    return (bf16(a).astype(np.float64) @ bf16(b).astype(np.float64)).astype(np.float32)


def forward(params, X, mode="fp64"):
    """Returns (Y, cache).  X [N][11] already normalised."""
    L = len(ARCH) - 1
    h = np.asarray(X, dtype=np.float64 if mode == "fp64" else np.float32)
    cache = {"h": [h], "z": []}
    for l in range(1, L + 1):
        W, b = params[f"W{l}"], params[f"b{l}"]
        if mode == "fp64":
            z = h @ W + b
        else:
            z = _mm(h, W, mode) + np.asarray(b, dtype=np.float32)
        cache["z"].append(z)
        if l < L:
            h = gelu(z) if mode == "fp64" else gelu(z.astype(np.float64)).astype(np.float32)
            cache["h"].append(h)
        else:
            h = z
    return h, cache


def backward(params, cache, dY, mode="fp64"):
    """Gradients of sum(dY * Y) with respect to every parameter."""
    L = len(ARCH) - 1
    grads = {}
    dz = np.asarray(dY, dtype=np.float64 if mode == "fp64" else np.float32)
    for l in range(L, 0, -1):
        h = cache["h"][l - 1]
        W = params[f"W{l}"]
        if mode == "fp64":
            grads[f"W{l}"] = h.T @ dz
            grads[f"b{l}"] = dz.sum(axis=0)
            dh = dz @ W.T
        else:
            grads[f"W{l}"] = _mm(h.T, dz, mode)
            grads[f"b{l}"] = dz.astype(np.float32).sum(axis=0, dtype=np.float32)
            dh = _mm(dz, np.asarray(W).T, mode)
        if l > 1:
            z = cache["z"][l - 2]
            if mode == "fp64":
                dz = dh * gelu_grad(z)
            else:
                dz = (dh * gelu_grad(z.astype(np.float64)).astype(np.float32)).astype(np.float32)
    return grads


def loss_and_grads(params, X, T, mode="fp64"):
    """MSE loss = mean over rows and outputs of (Y - T)^2, and its gradients."""
    Y, cache = forward(params, X, mode)
    n = Y.shape[0] * Y.shape[1]
    diff = Y - T
    loss = float(np.sum(np.asarray(diff, dtype=np.float64) ** 2) / n)
    dY = 2.0 * diff / n
    if mode != "fp64":
        dY = dY.astype(np.float32)
    return loss, backward(params, cache, dY, mode)


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def features(U_tm1, U_tm2, nu_dt, dim):
    """Raw features per node: the primitive state (n, u1, u2, u3, theta) at
    t-1, its change from t-2 to t-1 (the two steps' states given as state
    and difference, so that the small change survives rounding of the
    inputs to bfloat16), and dt*nu at t-1."""
    out = np.zeros((U_tm1.shape[0], 11))
    p1 = primitive_state(U_tm1, dim)
    p2 = primitive_state(U_tm2, dim)
    out[:, 0:5] = p1
    out[:, 5:10] = p1 - p2
    out[:, 10] = nu_dt
    return out


def targets(U_t, U_tm1, U_tm2, dim):
    """Raw targets per node: the primitive state at t minus its linear
    extrapolation 2 p(t-1) - p(t-2), so that a zero output reproduces the
    extrapolated guess."""
    p0 = primitive_state(U_t, dim)
    p1 = primitive_state(U_tm1, dim)
    p2 = primitive_state(U_tm2, dim)
    return p0 - (p1 + (p1 - p2))


def guess(delta, U_tm1, U_tm2, dim):
    """Initial moments from a predicted correction: p = p(t-1) + (p(t-1) -
    p(t-2)) + delta, back to conserved moments."""
    p1 = primitive_state(U_tm1, dim)
    p2 = primitive_state(U_tm2, dim)
    return moments_from_primitive(p1 + (p1 - p2) + delta, dim)


def primitive_state(U, dim):
    """(n, u1, u2, u3, theta) per node (u3 = 0 in 2D)."""
    out = np.zeros((U.shape[0], 5))
    n = U[:, 0]
    u = U[:, 1:1 + dim] / n[:, None]
    out[:, 0] = n
    out[:, 1:1 + dim] = u
    out[:, 4] = (2.0 * U[:, 1 + dim] / n - np.sum(u * u, axis=1)) / dim
    return out


def moments_from_primitive(p, dim):
    """U = (n, n u, n|u|^2/2 + (d/2) n theta) (eq. moments)."""
    n = p[:, 0]
    u = p[:, 1:1 + dim]
    U = np.zeros((p.shape[0], dim + 2))
    U[:, 0] = n
    U[:, 1:1 + dim] = n[:, None] * u
    U[:, 1 + dim] = 0.5 * n * np.sum(u * u, axis=1) + 0.5 * dim * n * p[:, 4]
    return U
