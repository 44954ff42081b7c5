"""cn_solve_direct: Crank-Nicolson steps solved with the factor alone, u <- F^-1 g (the remark on
eps = 1e-6 in Sec. 3).

eps = 0 makes the factor exact, so the steps must match the oracle's direct steps with the
sparse direct solve.  For eps > 0 the factor is one of several valid ones; a step is compared
with the GPU's own apply of the oracle's right-hand side (which the other tests pin to the
oracle), and its residual against the oracle's A.  Both ways of forming g run: in the first
apply stage, and as its own launch (HIFCN_NO_RHS_FUSE, and every factor whose level 0 has no
first-stage test).
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cn, fd
from workloads import gen

pytestmark = pytest.mark.gpu


def _factor(a, dt, n, dim, leaf, eps, store="f64", fused=True):
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    if not fused:
        os.environ["HIFCN_NO_RHS_FUSE"] = "1"
    try:
        return hifcn.factor(a_dev, dt, n, dim, eps, store=store, leaf=leaf)
    finally:
        os.environ.pop("HIFCN_NO_RHS_FUSE", None)


def _exact_steps(A, B, u0, dt, steps, react):
    lu = spla.splu(A.tocsc())
    return cn.cn_solve_direct(B, u0, dt, steps, lu.solve, react)


EXACT = [("2d-n32-m8", 32, 2, 8), ("2d-n40-m4", 40, 2, 4), ("3d-n12-m4", 12, 3, 4)]


@pytest.mark.parametrize("fused", [True, False], ids=["rhs-in-apply", "rhs-launch"])
@pytest.mark.parametrize("case", EXACT, ids=[c[0] for c in EXACT])
def test_exact_factor_direct_steps_match_oracle(case, fused, gpu_lib):
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name} fused={fused}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 41)
    u0 = gen.bumps(n, dim, 3, 42)
    dt = 0.05
    react = (1, 1.0, 2.0)
    A, B = fd.cn_matrices(a, dt)
    us = _exact_steps(A, B, u0, dt, 3, react)
    h = _factor(a, dt, n, dim, leaf, 0.0, fused=fused)
    for steps in (1, 2, 3):  # odd counts end with a copy back into u
        u = torch.tensor(u0.ravel(), device="cuda")
        h.cn_solve_direct(u, steps, reaction=react)
        got = u.cpu().numpy()
        assert np.linalg.norm(got - us[steps]) <= 1e-10 * np.linalg.norm(us[steps]), steps
    u = torch.tensor(u0.ravel(), device="cuda")
    h.cn_solve_direct(u, 0, reaction=react)
    assert np.array_equal(u.cpu().numpy(), u0.ravel())
    h.close()


APPROX = [("2d-n64-m8", 64, 2, 8, "f64", 1e-12), ("2d-n64-m8", 64, 2, 8, "f32", 2e-6),
          ("2d-n127-m8", 127, 2, 8, "bf16", 2e-6), ("3d-n16-m4", 16, 3, 4, "f32", 2e-6)]


@pytest.mark.parametrize("fused", [True, False], ids=["rhs-in-apply", "rhs-launch"])
@pytest.mark.parametrize("case", APPROX, ids=[f"{c[0]}-{c[4]}" for c in APPROX])
def test_direct_step_is_apply_of_oracle_rhs(case, fused, gpu_lib):
    """u^1 = F^-1 g^0 element by element, g^0 from the oracle; and then the second step."""
    import torch
    name, n, dim, leaf, store, tol = case
    print(f"[case] {name} {store} fused={fused}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 43)
    u0 = gen.bumps(n, dim, 4, 44)
    dt = 1.0 / (n + 1)
    react = (1, 1.0, 10.0)
    A, B = fd.cn_matrices(a, dt)
    h = _factor(a, dt, n, dim, leaf, 1e-6, store=store, fused=fused)
    u = torch.tensor(u0.ravel(), device="cuda")
    h.cn_solve_direct(u, 1, reaction=react)
    u1 = u.cpu().numpy()
    g0 = cn.cn_rhs(B, u0.ravel(), dt, react)
    want = h.apply(torch.tensor(g0, device="cuda")).cpu().numpy()
    # the same apply of g^0 formed in another order: equal to the rounding of g (the reduced
    # storage forms round their FP32 inputs, which may flip in the last place)
    assert np.max(np.abs(u1 - want)) <= tol * np.max(np.abs(want))
    h.cn_solve_direct(u, 1, reaction=react)
    g1 = cn.cn_rhs(B, u1, dt, react)
    want2 = h.apply(torch.tensor(g1, device="cuda")).cpu().numpy()
    assert np.max(np.abs(u.cpu().numpy() - want2)) <= 10 * tol * np.max(np.abs(want2))
    h.close()


def test_direct_steps_fisher256_residual_and_cg_agreement(gpu_lib):
    """The 256^2 Fisher workload at eps = 1e-6: ten direct steps stay within the inverse-error
    bound of the CG steps (relative residual ||A u - g|| / ||g|| per step small), and agree with
    CG to the size of that bound."""
    import torch
    w = gen.workload("fisher2d-256")
    A, B = fd.cn_matrices(w.a_cells, w.dt)
    h = _factor(w.a_cells, w.dt, w.n, 2, w.leaf, 1e-6, store="f64")
    u = torch.tensor(w.u0.ravel(), device="cuda")
    prev = w.u0.ravel().copy()
    for k in range(10):
        h.cn_solve_direct(u, 1, reaction=w.reaction)
        cur = u.cpu().numpy()
        g = cn.cn_rhs(B, prev, w.dt, w.reaction)
        rel = np.linalg.norm(A @ cur - g) / np.linalg.norm(g)
        assert rel <= 1e-4, (k, rel)
        prev = cur
    uc = torch.tensor(w.u0.ravel(), device="cuda")
    h.cn_solve(uc, 10, rtol=1e-12, reaction=w.reaction)
    d = np.linalg.norm(u.cpu().numpy() - uc.cpu().numpy()) / np.linalg.norm(uc.cpu().numpy())
    assert d <= 1e-4, d
    h.close()


def test_direct_rejects_bad_arguments(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    n = 16
    a = gen.grf_coefficient(n, 2, 0.1, 45)
    h = _factor(a, 0.05, n, 2, 4, 1e-6)
    u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    with pytest.raises(hifcn.HifError):
        h.cn_solve_direct(u, -1)
    with pytest.raises(hifcn.HifError):
        h.cn_solve_direct(u, 1, reaction=(7, 1.0, 1.0))
    h.close()
