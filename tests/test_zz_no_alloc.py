"""The allocation-free moments entry point (moments_noalloc) against the
allocating one (moments), through the C ABI: the same kernels, so U and the
three convergence ratios must be equal bit for bit.  Calls in a row, each on
a mesh needing less scratch than the one before (the fixed scratch keeps the
previous call's contents and must not leak into the next), the first with
the velocity-split reduction, plus a call without U_prev."""
import numpy as np
import pytest

import problems as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2608_19150_amd as B  # noqa: E402


def _case(pr, seed):
    d = B.Dag.from_problem(pr)
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 1, d.f_shape)
    f_old = f * (1 + 1e-3 * rng.normal(size=f.shape))
    fs = d.pack(B._dev(f))
    U_old = B.moments(d, d.pack(B._dev(f_old)))
    return d, fs, U_old


def test_moments_noalloc_equals_moments_on_consecutive_calls():
    # 8281 velocities on 4232 triangles: the velocity-split reduction, whose
    # chunk sums also live in the fixed scratch
    split = P.small_problem(dim=2, order=1, n_side=46, n_1d=91, seed=10)
    # 22,999 tetrahedra: 256-cell moment blocks
    wide = P.small_problem(dim=3, order=1, n_side=15, n_1d=4, seed=13)
    big = P.small_problem(dim=3, order=1, n_side=4, n_1d=8, seed=11)      # more moment blocks
    small = P.small_problem(dim=2, order=2, n_side=3, n_1d=6, seed=12)    # fewer
    for pr, seed in ((split, 3), (wide, 4), (big, 1), (small, 2)):
        d, fs, U_old = _case(pr, seed)
        U_ref, r_ref = B.moments(d, fs, U_prev=U_old)
        U = torch.full_like(U_ref, float("nan"))
        r = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        B.moments_noalloc(d, fs, U, U_prev=U_old, rel3=r)
        torch.cuda.synchronize()
        print(pr.mesh.n_cells, "cells:", r.cpu().numpy(), r_ref.cpu().numpy(), flush=True)
        assert torch.equal(U, U_ref)
        assert torch.equal(r, r_ref)
        U2 = torch.full_like(U_ref, float("nan"))
        B.moments_noalloc(d, fs, U2)
        assert torch.equal(U2, U_ref)


def test_moments_noalloc_rejects_missing_pairs():
    d, fs, U_old = _case(P.small_problem(dim=2, order=1, n_side=3, n_1d=4), 3)
    U = torch.empty((d.n_nodes, d.dim + 2), dtype=torch.float64, device="cuda")
    with pytest.raises(B.BGKError):
        B.moments_noalloc(d, fs, U, U_prev=U_old, rel3=None)
