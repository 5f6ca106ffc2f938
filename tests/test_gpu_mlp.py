"""Learned initial guess on the GPU: BF16 MFMA forward/backward and Adam
against the BF16-emulating oracle, the feature/target/guess kernels, and the
gain of the trained network in Picard iterations."""
import numpy as np
import pytest

import problems as P
from oracle import kinetic
from oracle import mlp as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B
    from paper_2608_19150_amd import learned


def _params(seed, bias_scale=0.1):
    p = P.mlp_init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for l in range(1, 5):
        p[f"b{l}"] = rng.uniform(-bias_scale, bias_scale, size=p[f"b{l}"].shape)
    return {k: np.asarray(v, dtype=np.float32) for k, v in p.items()}


def _stats(seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=11).astype(np.float32), rng.uniform(0.5, 2.0, 11).astype(np.float32),
            rng.normal(size=5).astype(np.float32), rng.uniform(0.5, 2.0, 5).astype(np.float32))


def _normalise(A, mu, sd):
    return ((np.asarray(A, np.float32) - mu) / sd).astype(np.float32)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 11)).astype(np.float32)
    T = rng.normal(size=(n, 5)).astype(np.float32)
    return X, T


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [1, 37, 1237])
def test_forward_matches_bf16_oracle(n):
    params, st = _params(11), _stats(12)
    X, _ = _data(n, 13)
    m = B.Mlp(params)
    m.set_normalization(*st)
    Y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    Yn, _ = om.forward(params, _normalise(X, st[0], st[1]), mode="bf16")
    Yref = (Yn * st[3] + st[2]).astype(np.float32)
    Y64n, _ = om.forward({k: v.astype(np.float64) for k, v in params.items()},
                         _normalise(X, st[0], st[1]).astype(np.float64), mode="fp64")
    Y64 = Y64n * st[3] + st[2]
    err = np.abs(Y - Yref).max() / np.abs(Yref).max()
    assert err <= 1e-3, err
    if n > 100:
        # the emulation models the kernel's rounding far better than FP64 does
        assert _rel(Y, Yref) < 0.25 * _rel(Y, Y64), (_rel(Y, Yref), _rel(Y, Y64))


@pytest.mark.parametrize("n", [1237, 20000])
def test_gradients_match_bf16_oracle(n):
    params, st = _params(21), _stats(22)
    X, T = _data(n, 23)
    m = B.Mlp(params)
    m.set_normalization(*st)
    loss, g = m.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    g = B.mlp_unflatten(g.cpu().numpy())
    lref, gref = om.loss_and_grads(params, _normalise(X, st[0], st[1]),
                                   _normalise(T, st[2], st[3]), mode="bf16")
    assert abs(float(loss.item()) - lref) <= 1e-4 * lref
    for k in gref:
        assert _rel(g[k], gref[k]) <= 1e-2, (k, _rel(g[k], gref[k]))
        # every element: within 2% of itself plus 1e-3 of the tensor's largest
        # entry (the two sides accumulate FP32 partial sums in different orders,
        # which only matters where an element is a cancellation of large terms)
        dev = np.abs(g[k] - gref[k])
        bound = 2e-2 * np.abs(gref[k]) + 1e-3 * np.abs(gref[k]).max()
        print(k, "worst element deviation / bound", float((dev / bound).max()), flush=True)
        assert np.all(dev <= bound), (k, float((dev / bound).max()))
    # and close to the exact FP64 gradient (BF16 operand rounding only)
    _, g64 = om.loss_and_grads({k: v.astype(np.float64) for k, v in params.items()},
                               _normalise(X, st[0], st[1]).astype(np.float64),
                               _normalise(T, st[2], st[3]).astype(np.float64), mode="fp64")
    for k in g64:
        assert _rel(g[k], g64[k]) <= 5e-2, (k, _rel(g[k], g64[k]))


def test_gradients_are_reproducible():
    params, st = _params(31), _stats(32)
    X, T = _data(30000, 33)
    m = B.Mlp(params)
    m.set_normalization(*st)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    l1, g1 = m.loss_grad(Xd, Td)
    l2, g2 = m.loss_grad(Xd, Td)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_steps_match_oracle_update():
    params, st = _params(41), _stats(42)
    X, T = _data(3000, 43)
    m = B.Mlp(params)
    m.set_normalization(*st)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    ref = {k: v.astype(np.float64) for k, v in params.items()}
    state = {}
    lr = 1e-3
    for _ in range(3):
        _, g = m.loss_grad(Xd, Td)
        gd = {k: v.astype(np.float64) for k, v in B.mlp_unflatten(g.cpu().numpy()).items()}
        om.adam(ref, gd, state, lr=lr)
        m.adam_step(Xd, Td, lr)
        got = m.get_params()
        for k in ref:
            assert np.abs(got[k] - ref[k]).max() <= 1e-3 * lr + 1e-6 * np.abs(ref[k]).max(), k


def test_training_reduces_loss():
    rng = np.random.default_rng(51)
    X = rng.normal(size=(8192, 11)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 5] * X[:, 10], np.tanh(X[:, 1] - X[:, 6]),
                  X[:, 2] ** 2 - 1.0, 0.3 * X[:, 3], np.cos(X[:, 4] + X[:, 9])],
                 axis=1).astype(np.float32)
    m = B.Mlp(_params(52, bias_scale=0.0))
    m.set_normalization(np.zeros(11), np.ones(11), T.mean(0), T.std(0))
    hist = learned.train(m, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), epochs=60,
                         batch=1024, lr=3e-3, seed=0)
    assert hist[-1] < 0.1 * hist[0], hist[::10]


def _states(n, dim, seed):
    rng = np.random.default_rng(seed)
    prim = np.zeros((n, 5))
    prim[:, 0] = rng.uniform(0.2, 2.0, n)
    prim[:, 1:1 + dim] = rng.uniform(-0.5, 0.5, (n, dim))
    prim[:, 4] = rng.uniform(0.5, 1.5, n)
    return om.moments_from_primitive(prim, dim)


def _dag(dim):
    pr = P.small_problem(dim=dim, order=1, n_side=3, n_1d=4, state="sod", nu_model="kn", kn=0.1)
    return B.Dag.from_problem(pr)


@pytest.mark.parametrize("dim", [2, 3])
def test_features_and_targets_match_oracle(dim):
    d = _dag(dim)
    n = d.n_nodes
    U1, U2, Ut = _states(n, dim, 61), _states(n, dim, 62), _states(n, dim, 63)
    dt, kn = 0.01, 0.05
    X = B.mlp_features(d, torch.from_numpy(U1).cuda(), torch.from_numpy(U2).cuda(), dt,
                       nu_model="kn", kn=kn).cpu().numpy()
    nu = kinetic.collision_frequency(U1, dim, "kn", kn=kn)
    Xref = om.features(U1, U2, dt * nu, dim)
    np.testing.assert_allclose(X, Xref.astype(np.float32), rtol=2e-7, atol=1e-7)
    T = B.mlp_targets(d, torch.from_numpy(Ut).cuda(), torch.from_numpy(U1).cuda(),
                      torch.from_numpy(U2).cuda()).cpu().numpy()
    Tref = om.targets(Ut, U1, U2, dim)
    np.testing.assert_allclose(T, Tref.astype(np.float32), rtol=2e-7, atol=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_guess_matches_oracle_and_falls_back(dim):
    d = _dag(dim)
    n = d.n_nodes
    # two nearby steps: the extrapolated state stays physical
    U1 = _states(n, dim, 71)
    p1 = om.primitive_state(U1, dim)
    rng = np.random.default_rng(72)
    mask = np.r_[1.0, np.ones(dim), np.zeros(3 - dim), 1.0]
    U2 = om.moments_from_primitive(p1 * (1.0 + 0.02 * rng.uniform(-1, 1, p1.shape) * mask), dim)
    dt, kn = 0.02, 0.1
    params = _params(73)
    st = (np.zeros(11, np.float32), np.ones(11, np.float32), np.zeros(5, np.float32),
          np.full(5, 0.01, np.float32))
    m = B.Mlp(params)
    m.set_normalization(*st)
    U1d, U2d = torch.from_numpy(U1).cuda(), torch.from_numpy(U2).cuda()
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    Ug = m.guess(d, U1d, U2d, dt, nu_model="kn", kn=kn, n_fallback=nf).cpu().numpy()
    assert int(nf.item()) == 0
    nu = kinetic.collision_frequency(U1, dim, "kn", kn=kn)
    Xn = _normalise(om.features(U1, U2, dt * nu, dim), st[0], st[1])
    Yn, _ = om.forward(params, Xn, mode="bf16")
    delta = (Yn * st[3] + st[2]).astype(np.float32).astype(np.float64)
    Uref = om.guess(delta, U1, U2, dim)
    # the prediction is a small correction and BF16 effects scale with it:
    # compare against 1% of the correction's size
    corr = np.abs(Uref - om.guess(np.zeros_like(delta), U1, U2, dim)).max()
    err = np.abs(Ug - Uref).max()
    print(f"guess error {err:.3e}, correction {corr:.3e}")
    assert corr > 1e-4 * np.abs(U1).max()
    assert err <= 1e-2 * corr
    # an impossible prediction (density change -100) falls back to U^{t-1}
    bad = dict(params)
    bad["b4"] = np.array([-100.0, 0, 0, 0, 0], np.float32)
    m.set_params(bad)
    m.set_normalization(st[0], st[1], st[2], np.ones(5, np.float32))
    nf.zero_()
    Ug = m.guess(d, U1d, U2d, dt, nu_model="kn", kn=kn, n_fallback=nf).cpu().numpy()
    assert int(nf.item()) == n
    assert np.array_equal(Ug, U1)


KN = (1e-3, 1e-1)   # collision-dominated: Picard contracts slowly (rho ~ nu dt / (1 + nu dt))


def test_learned_guess_beats_extrapolation_and_plain_guess():
    """Trained on 400 solver trajectories of seeded 3D Riemann problems, the
    network's initial iterate needs fewer Picard iterations on 12 held-out
    problems (seeds 7000-7011) than both the plain previous-step guess and
    linear extrapolation 2 U^k - U^(k-1) (the network predicts a correction
    to it), and the converged moments agree with the plain run to the
    stopping tolerance.  Training is seeded and the gradients are
    reproducible, so the counts are too."""
    train = [P.learned_guess_problem(3, 5000 + i, 4 + i % 3, 12, kn_range=KN) for i in range(400)]
    mlp, info = learned.fit(train, n_steps=8, tau=1e-9, epochs=24, batch=4096, lr=2e-3, seed=0)
    print({k: v for k, v in info.items() if k != "loss"}, info["loss"][::6], flush=True)
    # sharp Riemann data can drive a node's DG moments non-physical (no
    # limiter in the method); such runs are reported and left out
    assert len(info["skipped"]) <= 10
    assert all("[-5]" in msg for _, msg in info["skipped"])
    assert info["loss"][-1] < 0.8 * info["loss"][0]
    tot = {"plain": 0, "linear": 0, "learned": 0}
    evaluated = 0
    for i in range(12):
        pr = P.learned_guess_problem(3, 7000 + i, 4 + i % 3, 12, kn_range=KN)
        try:
            res = learned.compare(pr, mlp, n_steps=8, tau=1e-9)
        except B.BGKError as e:
            assert e.code == B.BGK_E_NONPHYSICAL
            continue
        evaluated += 1
        for k in tot:
            tot[k] += sum(res[k]["iters"][1:])
        print(pr.name, {k: v["iters"] for k, v in res.items()},
              {k: v["fallbacks"] for k, v in res.items()}, flush=True)
        # each step stops at a relative change below tau / max(1, nu dt); with
        # the contraction rho ~ nu dt / (1 + nu dt) a run is within about tau
        # of the fixed point per step; allow 18 tau per step over 8 steps
        err = learned.moment_difference(res["learned"]["U"][-1], res["plain"]["U"][-1], 3)
        assert max(err) <= 8 * 18 * 1e-9, err
    print("Picard iterations after step 1:", tot, flush=True)
    assert evaluated >= 10
    assert tot["learned"] < tot["linear"] < tot["plain"], tot
