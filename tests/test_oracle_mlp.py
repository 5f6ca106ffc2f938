"""Oracle pins for the learned-guess network (no paper reference: the
network is an addition; pins are mathematical).

* FP64 back-propagation equals central finite differences of the loss.
* GELU: g(0) = 0, g(z) - g(-z) = z (erf is odd), derivative equals finite
  differences, and the known value g(1) = Phi(1) = 0.8413447460685429.
* bfloat16 rounding: exact values pass through, halfway cases round to even.
* A network with zero weights outputs its last bias.
"""
import math

import numpy as np

import problems as P
from oracle import mlp


def test_bf16_rounding_rules():
    one = np.float32(1.0)
    assert mlp.bf16(one) == one
    # 1 + 2^-8 is exactly halfway between 1 and 1 + 2^-7 -> ties to even (1.0)
    assert mlp.bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6 -> even is 1 + 2^-6
    assert mlp.bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    assert np.max(np.abs(mlp.bf16(x) - x) / np.abs(x)) <= 2.0 ** -8


def test_gelu_values_and_derivative():
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    z = np.linspace(-4, 4, 17)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-9)


def test_zero_weights_output_last_bias():
    p = P.mlp_init_params(1)
    for k in p:
        p[k] = np.zeros_like(p[k])
    p["b4"] = np.arange(5.0)
    Y, _ = mlp.forward(p, np.random.default_rng(0).normal(size=(7, 11)))
    assert np.array_equal(Y, np.tile(np.arange(5.0), (7, 1)))


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = P.mlp_init_params(5)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    X = rng.normal(size=(9, 11))
    T = rng.normal(size=(9, 5))
    loss, g = mlp.loss_and_grads(p, X, T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(p, X, T)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(p, X, T)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (k, i, an, fd)


def test_bf16_path_close_to_fp64():
    rng = np.random.default_rng(4)
    p = P.mlp_init_params(6)
    X = rng.normal(size=(64, 11))
    T = rng.normal(size=(64, 5))
    Y64, _ = mlp.forward(p, X)
    Y16, _ = mlp.forward(p, X, "bf16")
    assert np.max(np.abs(Y16 - Y64)) <= 0.05 * np.max(np.abs(Y64))


def test_primitive_roundtrip():
    rng = np.random.default_rng(5)
    for dim in (2, 3):
        p = np.zeros((10, 5))
        p[:, 0] = rng.uniform(0.1, 2, 10)
        p[:, 1:1 + dim] = rng.normal(size=(10, dim))
        p[:, 4] = rng.uniform(0.5, 2, 10)
        U = mlp.moments_from_primitive(p, dim)
        assert np.allclose(mlp.primitive_state(U, dim), p)


def test_targets_measure_the_departure_from_linear_extrapolation():
    """A primitive state moving linearly in time has zero targets, and
    guess(targets) returns the state at t (inverse pair)."""
    rng = np.random.default_rng(6)
    for dim in (2, 3):
        p2 = np.zeros((12, 5))
        p2[:, 0] = rng.uniform(0.5, 1.5, 12)
        p2[:, 1:1 + dim] = rng.normal(scale=0.3, size=(12, dim))
        p2[:, 4] = rng.uniform(0.7, 1.3, 12)
        step = np.zeros_like(p2)
        step[:, 0] = rng.uniform(-0.01, 0.01, 12)
        step[:, 1:1 + dim] = rng.uniform(-0.01, 0.01, (12, dim))
        step[:, 4] = rng.uniform(-0.01, 0.01, 12)
        U2 = mlp.moments_from_primitive(p2, dim)
        U1 = mlp.moments_from_primitive(p2 + step, dim)
        Ut = mlp.moments_from_primitive(p2 + 2 * step, dim)
        assert np.abs(mlp.targets(Ut, U1, U2, dim)).max() < 1e-13
        Uo = mlp.moments_from_primitive(p2 + 2 * step + 0.01 * rng.normal(size=p2.shape) *
                                        np.r_[1, np.ones(dim), np.zeros(3 - dim), 1], dim)
        np.testing.assert_allclose(mlp.guess(mlp.targets(Uo, U1, U2, dim), U1, U2, dim), Uo,
                                   rtol=1e-13, atol=1e-13)


def _adam_run(p0, grads_seq, **kw):
    params = {"w": np.array(p0, dtype=np.float64)}
    state = {}
    for g in grads_seq:
        mlp.adam(params, {"w": np.array(g, dtype=np.float64)}, state, **kw)
    return params["w"]


def test_adam_first_step_is_normalised_gradient():
    """After one step the bias-corrected moments are exactly g and g^2, so
    the update is -lr g / (|g| + eps) per parameter, whatever b1 and b2 are
    (Kingma & Ba, Alg. 1).  Small gradients check where eps enters."""
    rng = np.random.default_rng(3)
    g = rng.normal(size=50) * np.logspace(-9, 1, 50)
    p0 = rng.normal(size=50)
    for b1, b2 in [(0.9, 0.999), (0.5, 0.9)]:
        p1 = _adam_run(p0, [g], lr=1e-3, b1=b1, b2=b2, eps=1e-8)
        np.testing.assert_allclose(p1 - p0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a zero gradient leaves the parameter unchanged
    assert _adam_run([2.5], [[0.0]])[0] == 2.5


def test_adam_constant_gradient_moves_equal_steps():
    """With a constant gradient the bias correction is exact at every step
    (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so every step is the first
    step's size; a wrong correction exponent breaks this."""
    g = np.array([0.3, -2.0, 1e-7])
    p0 = np.zeros(3)
    step = -1e-2 * g / (np.abs(g) + 1e-8)
    for t in (1, 2, 5, 20):
        pt = _adam_run(p0, [g] * t, lr=1e-2)
        np.testing.assert_allclose(pt, t * step, rtol=1e-12, atol=0)


def test_adam_two_steps_hand_computed():
    """p0 = 1, g1 = 0.5, g2 = -0.25, lr 1e-3, b1 0.9, b2 0.999, eps 1e-8:
    step 1 gives m = 0.05, v = 2.5e-4, m^ = 0.5, v^ = 0.25, p1 = 1 - 1e-3 *
    0.5 / (0.5 + 1e-8) = 0.99900000002; step 2 gives m = 0.045 - 0.025 =
    0.02, v = 2.4975e-4 + 6.25e-5 = 3.1225e-4, m^ = 0.02 / 0.19 = 2/19,
    v^ = 3.1225e-4 / 0.001999, p2 = p1 - 1e-3 (2/19) / (sqrt(v^) + 1e-8)
    = 0.9987336629870784."""
    p = _adam_run([1.0], [[0.5]])
    assert abs(p[0] - 0.99900000002) < 1e-15
    p = _adam_run([1.0], [[0.5], [-0.25]])
    assert abs(p[0] - 0.9987336629870784) < 1e-15
