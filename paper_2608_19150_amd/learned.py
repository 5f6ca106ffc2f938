"""Learned Picard initial guess: trajectory generation, training and use.

The solver produces its own training data: backward-Euler runs of seeded
problems record the converged nodal moments U^k after every step.  A sample
pairs the features of (U^k, U^{k-1}, dt nu(U^k)) with the difference between
the primitive state (n, u, theta) at k+1 and its linear extrapolation from
k-1 and k; the network (BF16 MFMA kernels of the library) is fitted to it
with minibatch Adam on the GPU, so an uninformed network falls back to the
extrapolated guess.  At
run time the prediction replaces the plain initial iterate U^k of the first
Picard iteration of step k -> k+1 (Sec. 4 starts Picard from the previous
stage); the converged iteration, with its tolerance unchanged, remains the
judge of the result, and nodes with an invalid prediction fall back to U^k.

The first step of a run has no U^{k-1} and uses the plain guess.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import Mlp, Solver, mlp_features, mlp_targets, moments, problem_setup

GUESS_MODES = ("plain", "linear", "learned")


class Trajectory:
    """One problem's backward-Euler run on the GPU, recording U^k (user order)."""

    def __init__(self, pr, *, tau=1e-9, precision=0, l_max=2000, dag_kw=None):
        self.pr = pr
        self.dag, self.f0, self.bc, self.dt = problem_setup(pr, **(dag_kw or {}))
        self.tau = tau
        self.solver = Solver(self.dag, dt=self.dt, bc_coef=self.bc, tableau=pr.tableau, tau=tau,
                             l_max=l_max, precision=precision, mode="MATCHED",
                             nu_model=pr.nu_model, nu_const=pr.nu_const, kn=pr.kn)

    def nu_kw(self):
        return {"nu_model": self.pr.nu_model, "nu_const": self.pr.nu_const, "kn": self.pr.kn}

    def run(self, n_steps, guess="plain", mlp=None, n_fallback=None):
        """Runs n_steps from the initial state.  guess: 'plain' (U^k),
        'linear' (2 U^k - U^{k-1}) or 'learned' (mlp).  Returns a dict with
        the moment history U[0..n_steps] (device), Picard iterations and
        wall seconds per step."""
        if guess not in GUESS_MODES:
            raise ValueError(guess)
        if guess == "learned" and mlp is None:
            raise ValueError("learned guess needs an Mlp")
        f = self.f0.clone()
        U = [moments(self.dag, f)]
        iters, secs = [], []
        for k in range(n_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Ug = None
            if k >= 1 and guess == "linear":
                Ug = 2.0 * U[k] - U[k - 1]
            elif k >= 1 and guess == "learned":
                Ug = mlp.guess(self.dag, U[k], U[k - 1], self.dt, n_fallback=n_fallback,
                               **self.nu_kw())
            Unext = torch.empty_like(U[0])
            st = self.solver.step(f, U_guess=Ug, U_out=Unext)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            iters.append(st["total_iters"])
            U.append(Unext)
        return {"U": U, "iters": iters, "seconds": secs}


def samples(traj, U):
    """(X, T) device float32 samples of one recorded moment history."""
    Xs, Ts = [], []
    for k in range(1, len(U) - 1):
        Xs.append(mlp_features(traj.dag, U[k], U[k - 1], traj.dt, **traj.nu_kw()))
        Ts.append(mlp_targets(traj.dag, U[k + 1], U[k], U[k - 1]))
    return torch.cat(Xs), torch.cat(Ts)


def normalization(X, T):
    """Inputs: per-column mean and standard deviation (a column with no
    spread gets std 1, so it is only centred).  Outputs: scaled by their
    root mean square but not centred, so that a zero network output is the
    extrapolated guess exactly (most nodes of a run barely change, and a
    centred output would shift all of them by the targets' mean)."""
    X64 = X.double()
    mu = X64.mean(0)
    sd = X64.std(0, unbiased=False)
    sd = torch.where(sd > 1e-6 * torch.clamp(mu.abs(), min=1.0), sd, torch.ones_like(sd))
    rms = T.double().pow(2).mean(0).sqrt()
    rms = torch.where(rms > 0, rms, torch.ones_like(rms))
    return (mu.float().cpu().numpy(), sd.float().cpu().numpy(),
            np.zeros(T.shape[1], dtype=np.float32), rms.float().cpu().numpy())


def train(mlp, X, T, *, epochs=20, batch=4096, lr=1e-3, seed=0, log_every=0):
    """Minibatch Adam over shuffled rows; returns the per-epoch mean loss."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = X.shape[0]
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        nb = 0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            mlp.adam_step(xb, tb, lr, loss=loss)
            acc += loss.double()[0]
            nb += 1
        hist.append(float(acc) / nb)
        if log_every and (ep + 1) % log_every == 0:
            print(f"[learned] epoch {ep + 1} loss {hist[-1]:.4e}", flush=True)
    return hist


def glorot_params(seed, arch=None):
    """Glorot-uniform weights, zero biases (W_l [fan_in][fan_out])."""
    from . import MLP_ARCH
    arch = MLP_ARCH if arch is None else arch
    rng = np.random.default_rng(seed)
    out = {}
    for l in range(len(arch) - 1):
        fi, fo = arch[l], arch[l + 1]
        lim = np.sqrt(6.0 / (fi + fo))
        out[f"W{l + 1}"] = rng.uniform(-lim, lim, size=(fi, fo))
        out[f"b{l + 1}"] = np.zeros(fo)
    return out


def generate(problems, *, n_steps=8, tau=1e-9, max_rows=0, seed=0, log_every=0):
    """Runs one trajectory per problem and returns (per-problem samples,
    skipped, seconds).  Each entry is (problem name, dim, X, T); with
    max_rows > 0 a trajectory keeps a seeded random subset of that many
    rows.  Problems whose run fails (non-physical or not converged) are
    skipped and listed with their error."""
    from . import BGKError
    out, skipped = [], []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    t0 = time.perf_counter()
    for i, pr in enumerate(problems):
        if log_every and i and i % log_every == 0:
            print(f"[learned] {i} trajectories, {time.perf_counter() - t0:.1f} s", flush=True)
        try:
            tr = Trajectory(pr, tau=tau)
            res = tr.run(n_steps)
        except BGKError as e:
            skipped.append((pr.name, str(e)))
            continue
        X, T = samples(tr, res["U"])
        if max_rows and X.shape[0] > max_rows:
            keep = torch.randperm(X.shape[0], device="cuda", generator=gen)[:max_rows]
            X, T = X.index_select(0, keep).contiguous(), T.index_select(0, keep).contiguous()
        out.append((pr.name, pr.mesh.dim, X, T))
        del tr
    torch.cuda.synchronize()
    return out, skipped, time.perf_counter() - t0


def fit_samples(data, *, epochs=20, batch=4096, lr=1e-3, seed=0, init_params=None, log_every=0):
    """Fits a network (Glorot start from `seed` unless init_params is given)
    to the rows of the given trajectories; returns (mlp, info)."""
    X = torch.cat([d[2] for d in data])
    T = torch.cat([d[3] for d in data])
    mlp = Mlp(glorot_params(seed) if init_params is None else init_params)
    mlp.set_normalization(*normalization(X, T))
    t0 = time.perf_counter()
    hist = train(mlp, X, T, epochs=epochs, batch=batch, lr=lr, seed=seed, log_every=log_every)
    torch.cuda.synchronize()
    return mlp, {"samples": int(X.shape[0]), "trajectories": len(data), "loss": hist,
                 "train_s": time.perf_counter() - t0}


def fit(problems, *, n_steps=8, tau=1e-9, epochs=20, batch=4096, lr=1e-3, seed=0,
        init_params=None, log_every=0, max_rows=0):
    """Generates one trajectory per problem, fits a network to all of them
    and returns (mlp, info) (generate, then fit_samples)."""
    data, skipped, gen_s = generate(problems, n_steps=n_steps, tau=tau, max_rows=max_rows,
                                    seed=seed)
    mlp, info = fit_samples(data, epochs=epochs, batch=batch, lr=lr, seed=seed,
                            init_params=init_params, log_every=log_every)
    info.update({"skipped": skipped, "generate_s": gen_s})
    return mlp, info


def compare(pr, mlp, *, n_steps=8, tau=1e-9, modes=GUESS_MODES):
    """Runs the same problem with each guess; returns per-mode iterations,
    seconds and final moments (device)."""
    out = {}
    tr = Trajectory(pr, tau=tau)
    for mode in modes:
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        r = tr.run(n_steps, guess=mode, mlp=mlp, n_fallback=nf)
        out[mode] = {"iters": r["iters"], "seconds": r["seconds"], "U": r["U"],
                     "fallbacks": int(nf.item())}
    return out


def moment_difference(U, Uref, dim):
    """Per moment block: ||U - Uref|| / max(||Uref||, s ||Uref_0||), with
    s = 1 for the momentum (whose reference may vanish) and 0 otherwise."""
    Ua, Ub = U.double().cpu().numpy(), Uref.double().cpu().numpy()
    n0 = np.linalg.norm(Ub[:, 0])
    errs = []
    for m, sl in enumerate([slice(0, 1), slice(1, 1 + dim), slice(1 + dim, 2 + dim)]):
        den = np.linalg.norm(Ub[:, sl])
        if m == 1:
            den = max(den, n0)
        errs.append(float(np.linalg.norm(Ua[:, sl] - Ub[:, sl]) / den))
    return errs
