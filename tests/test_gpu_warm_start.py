"""Warm-started PCG (hif_cg_opts_t.warm_start = 1: x0 = u^k) against the oracle's warm start
(Algorithm 1's pcg from the initial guess u^k, r0 = g - A u^k, the same test against
rtol ||g||).  Cases: a 2D grid whose cold steps take the plain right-hand-side launch, one whose
cold steps make g in the first apply stage (the warm start always takes the launch), and 3D.
Also: g = 0 gives u = 0 with no iteration, and the batched step refuses the option."""
import ctypes

import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, dim, leaf, eps, dt
    ("2d-n63", 63, 2, 8, 1e-3, 0.05),
    ("2d-n64-fused-rhs", 64, 2, 8, 1e-3, 0.05),
    ("3d-n16", 16, 3, 4, 1e-3, 0.05),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_warm_start_cn_matches_oracle(case, gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    name, n, dim, leaf, eps, dt = case
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 21)
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 22)
    react = (1, 1.0, 1.0)
    steps, rtol = 3, 1e-10
    us, its, _ = cn.cn_solve(A, B, u0, dt, steps, lambda r: phif.phif_apply(F, r), rtol, react,
                             warm_start=True)
    h = hifcn.factor(torch.tensor(a, device="cuda"), dt, n, dim, eps, store="f64", leaf=leaf)
    # cold steps first (on a handle whose cold steps make g in the first apply stage, that
    # stage's partials are then live), warm steps, and cold steps again on the same handle
    uc1 = torch.tensor(u0.ravel(), device="cuda")
    cits, _ = h.cn_solve(uc1, steps, rtol=rtol, reaction=react)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, rel = h.cn_solve(u, steps, rtol=rtol, reaction=react, warm_start=True)
    ug = u.cpu().numpy()
    ref = us[-1]
    assert np.linalg.norm(ug - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.abs(ug - ref).max() <= 1e-9 * np.abs(ref).max()
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    assert (rel <= rtol).all()
    # x0 = 0 and x0 = u^k reach the same steps within the tolerance
    uc = uc1.cpu().numpy()
    assert np.linalg.norm(ug - uc) <= 1e-8 * np.linalg.norm(uc)
    # a warm-started solve leaves nothing behind for the next cold one
    uc2 = torch.tensor(u0.ravel(), device="cuda")
    cits2, _ = h.cn_solve(uc2, steps, rtol=rtol, reaction=react)
    assert list(cits2) == list(cits)
    assert np.abs(uc2.cpu().numpy() - uc).max() <= 1e-13 * np.abs(uc).max()
    print(f"  warm n_i {[int(v) for v in gits]} (oracle {its}), cold n_i {[int(v) for v in cits]}",
          flush=True)
    h.close()


def test_warm_start_zero_rhs_gives_zero(gpu_lib):
    """u^k = 0 and no reaction: g = 0, so the step leaves u = 0 with no iteration."""
    import torch
    from paper_2004_05566_amd import hifcn
    n = 32
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.15, 3), device="cuda")
    h = hifcn.factor(a, 0.05, n, 2, 1e-3, store="f64", leaf=8)
    u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    its, rel = h.cn_solve(u, 2, rtol=1e-8, warm_start=True)
    assert list(its) == [0, 0] and not u.any()
    h.close()


def test_batched_step_refuses_warm_start(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    n = 32
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.15, 4), device="cuda")
    h = hifcn.factor(a, 0.05, n, 2, 1e-3, store="f64", leaf=8)
    u = torch.tensor(gen.bumps(n, 2, 2, 5).ravel(), device="cuda")
    u_before = u.clone()
    lib = hifcn.raw_library()
    hs = (ctypes.c_void_p * 1)(h._p())
    us = (ctypes.c_void_p * 1)(u.data_ptr())
    o = (hifcn._CgOpts * 1)(hifcn._CgOpts(1e-8, 100, 1))
    its = np.zeros(1, np.int32)
    rel = np.zeros(1)
    sts = np.zeros(1, np.int32)
    st = lib.cn_batch_step(hs, None, o, us, 1, its.ctypes.data_as(ctypes.c_void_p),
                           rel.ctypes.data_as(ctypes.c_void_p),
                           sts.ctypes.data_as(ctypes.c_void_p), None)
    assert st == hifcn.HIF_ERR_ARG
    torch.cuda.synchronize()
    assert torch.equal(u, u_before)
    h.close()


def test_warm_steps_one_call_each_equal_warm_solve(gpu_lib):
    """cn_step called step by step and cn_solve (which queues each step behind the previous one)
    run the same warm-started arithmetic: bitwise equal states and iteration counts."""
    import torch
    from paper_2004_05566_amd import hifcn
    n = 64
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.15, 41), device="cuda")
    h = hifcn.factor(a, 0.05, n, 2, 1e-3, store="f32", leaf=8)
    u0 = gen.bumps(n, 2, 3, 42).ravel()
    react = (1, 1.0, 1.0)
    u1 = torch.tensor(u0, device="cuda")
    its_solve, _ = h.cn_solve(u1, 4, rtol=1e-10, reaction=react, warm_start=True)
    u2 = torch.tensor(u0, device="cuda")
    its_step = []
    for _ in range(4):
        it, _ = h.cn_step(u2, rtol=1e-10, reaction=react, warm_start=True)
        its_step.append(int(it))
    assert torch.equal(u1, u2)
    assert [int(v) for v in its_solve] == its_step
    h.close()


def test_warm_start_nan_state_reports_no_convergence_and_keeps_u(gpu_lib):
    """A NaN in u^k makes ||g||^2 and ||r0||^2 NaN: HIF_ERR_NO_CONV after no iteration, u left
    as it was (as for x0 = 0)."""
    import torch
    from paper_2004_05566_amd import hifcn
    n = 32
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.15, 43), device="cuda")
    h = hifcn.factor(a, 0.05, n, 2, 1e-3, store="f64", leaf=8)
    u0 = gen.bumps(n, 2, 3, 44).ravel()
    u0[77] = np.nan
    for call in ("step", "solve"):
        u = torch.tensor(u0, device="cuda")
        with pytest.raises(hifcn.HifError) as ei:
            if call == "step":
                h.cn_step(u, rtol=1e-10, warm_start=True)
            else:
                h.cn_solve(u, 3, rtol=1e-10, warm_start=True)
        assert ei.value.status == hifcn.HIF_ERR_NO_CONV, call
        got = u.cpu().numpy()
        assert np.isnan(got[77]) and np.array_equal(np.delete(got, 77), np.delete(u0, 77)), call
    h.close()
