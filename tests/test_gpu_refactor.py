"""Time-dependent coefficients (Sec. 4): hif_set_coefficient (new operator, factor kept) and
hif_refactor (factor rebuilt in the same handle), against the oracle's cn_solve_varying.

A refactored handle applies the same operator as a handle factored from scratch with that
coefficient; a CN run whose coefficient drifts, with the factor rebuilt every K steps, gives the
oracle's u (1e-10 relative at rtol 1e-12) and its iteration counts (+-1) for K = 1 and K = 3.
"""
import numpy as np
import pytest

from oracle import cn, fd
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _factor(a, dt, n, dim, leaf, eps, store="f64"):
    from paper_2004_05566_amd import hifcn
    return hifcn.factor(_dev(a), dt, n, dim, eps, store=store, leaf=leaf)


def test_set_coefficient_changes_the_operator_not_the_factor(gpu_lib):
    import torch
    n, dt = 48, 0.05
    a_at = gen.drifting_coefficient(n, 2, 0.2, 61, amp=1.0, period=1.0)
    a0, a1 = a_at(0.0), a_at(0.25)
    h = _factor(a0, dt, n, 2, 8, 1e-6)
    x = torch.tensor(np.random.default_rng(62).normal(size=n * n), device="cuda")
    z0 = h.apply(x)
    h.set_coefficient(_dev(a1))
    A1, B1 = fd.cn_matrices(a1, dt)
    y = h.spmv(x).cpu().numpy()
    want = A1 @ x.cpu().numpy()
    assert np.max(np.abs(y - want)) <= 1e-13 * np.max(np.abs(want))
    assert torch.equal(h.apply(x), z0)
    u0 = gen.bumps(n, 2, 3, 63)
    react = (1, 1.0, 2.0)
    u = torch.tensor(u0.ravel(), device="cuda")
    h.cn_solve(u, 2, rtol=1e-12, reaction=react)
    ref = u0.ravel().copy()
    import scipy.sparse.linalg as spla
    for _ in range(2):
        ref = spla.spsolve(A1.tocsc(), cn.cn_rhs(B1, ref, dt, react))
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    h.close()


CASES = [("2d-n64-m8", 64, 2, 8, "f64"), ("2d-n64-m8", 64, 2, 8, "f32"),
         ("2d-n127-m8", 127, 2, 8, "bf16"), ("3d-n12-m4", 12, 3, 4, "f64")]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[4]}" for c in CASES])
def test_refactor_matches_a_fresh_factor(case, gpu_lib):
    import torch
    name, n, dim, leaf, store = case
    print(f"[case] {name} {store}", flush=True)
    dt = 0.05
    a_at = gen.drifting_coefficient(n, dim, 0.2, 64, amp=1.0, period=1.0)
    a0, a1 = a_at(0.0), a_at(0.3)
    h = _factor(a0, dt, n, dim, leaf, 1e-6, store)
    h.refactor(_dev(a1))
    h1 = _factor(a1, dt, n, dim, leaf, 1e-6, store)
    i, i1 = h.info(), h1.info()
    i.pop("build_mfma_ms")
    i1.pop("build_mfma_ms")
    assert i == i1
    rng = np.random.default_rng(65)
    for _ in range(2):
        x = torch.tensor(rng.normal(size=n ** dim), device="cuda")
        y, y1 = h.apply(x), h1.apply(x)
        assert torch.linalg.norm(y - y1) <= 1e-13 * torch.linalg.norm(y1)
        assert torch.equal(h.spmv(x), h1.spmv(x))
    u = torch.tensor(gen.bumps(n, dim, 3, 66).ravel(), device="cuda")
    u1 = u.clone()
    its, _ = h.cn_solve(u, 2, rtol=1e-12)
    its1, _ = h1.cn_solve(u1, 2, rtol=1e-12)
    assert list(its) == list(its1)
    assert torch.linalg.norm(u - u1) <= 1e-12 * torch.linalg.norm(u1)
    h.close()
    h1.close()


@pytest.mark.parametrize("every", [1, 3])
def test_drifting_coefficient_cn_matches_oracle(every, gpu_lib):
    import torch
    n, leaf, eps = 64, 8, 1e-6
    dt = 1.0 / (n + 1)
    steps = 6
    react = (1, 1.0, 10.0)
    a_at = gen.drifting_coefficient(n, 2, 0.2, 67, amp=1.0, period=8 * dt)
    u0 = gen.bumps(n, 2, 4, 68)
    us, its = cn.cn_solve_varying(a_at, n, 2, leaf, eps, dt, u0, steps, every, 1e-12, react)
    u = torch.tensor(u0.ravel(), device="cuda")
    h = None
    gits = []
    for k in range(steps):
        a_k = _dev(a_at((k + 0.5) * dt))
        if h is None:
            h = _factor(a_at(0.5 * dt), dt, n, 2, leaf, eps)
        elif k % every == 0:
            h.refactor(a_k)
        else:
            h.set_coefficient(a_k)
        it, _ = h.cn_solve(u, 1, rtol=1e-12, reaction=react)
        gits.append(int(it[0]))
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(x - y) for x, y in zip(gits, its)) <= 1, (gits, its)
    h.close()


def test_refactor_errors_keep_the_old_factor(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    from oracle import phif
    from tests.hifb import factor_to_hifb
    n, dt = 32, 0.05
    a = gen.grf_coefficient(n, 2, 0.2, 69)
    h = _factor(a, dt, n, 2, 8, 1e-6)
    x = torch.tensor(np.random.default_rng(70).normal(size=n * n), device="cuda")
    y0 = h.apply(x)
    with pytest.raises(hifcn.HifError) as ei:  # a < 0: A indefinite at this dt
        h.refactor(_dev(-a))
    assert ei.value.status == hifcn.HIF_ERR_NOT_SPD
    with pytest.raises(ValueError):
        h.refactor(_dev(a[:-1]))
    assert torch.equal(h.apply(x), y0)
    A, _ = fd.cn_matrices(a, dt)
    hi = hifcn.import_factor(_dev(a), dt, n, 2, factor_to_hifb(phif.phif_build(A, n, 2, 8, 1e-6)),
                             store="f64", leaf=8)
    with pytest.raises(hifcn.HifError):
        hi.refactor(_dev(a))
    hi.close()
    h.close()


def test_refactored_handle_serves_every_step_entry_point(gpu_lib):
    """After hif_refactor: the direct steps, the PCG steps and the batched step all see the new
    factor and operator (a handle factored from scratch is the reference for each)."""
    import torch
    from paper_2004_05566_amd import hifcn
    n, dt = 64, 1.0 / 65
    a_at = gen.drifting_coefficient(n, 2, 0.2, 71, amp=1.0, period=1.0)
    a1 = a_at(0.4)
    h = _factor(a_at(0.0), dt, n, 2, 8, 1e-6)
    h.refactor(_dev(a1))
    h1 = _factor(a1, dt, n, 2, 8, 1e-6)
    u0 = torch.tensor(gen.bumps(n, 2, 3, 72).ravel(), device="cuda")
    react = (1, 1.0, 10.0)
    ua, ub = u0.clone(), u0.clone()
    h.cn_solve_direct(ua, 3, reaction=react)
    h1.cn_solve_direct(ub, 3, reaction=react)
    assert torch.linalg.norm(ua - ub) <= 1e-12 * torch.linalg.norm(ub)
    ua, ub = u0.clone(), u0.clone()
    s = torch.cuda.Stream()
    its, _, sts = hifcn.cn_batch_step([h], [ua], [react], [1e-12], [100], [s])
    torch.cuda.synchronize()
    it1, _ = h1.cn_step(ub, rtol=1e-12, maxit=100, reaction=react)
    assert int(sts[0]) == hifcn.HIF_OK and int(its[0]) == it1
    assert torch.linalg.norm(ua - ub) <= 1e-12 * torch.linalg.norm(ub)
    h.close()
    h1.close()
