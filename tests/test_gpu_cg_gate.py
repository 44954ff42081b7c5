"""PCG convergence test run by the first stage of the preconditioner apply.

Inside a batch of queued iterations the test after each update (and the one on the right-hand
side) runs in the level-0 cell stage, which then reads r and hands z = r over for every DOF it
does not overwrite.  The same factor built with HIFCN_NO_CG_GATE=1 runs the test as its own
launch; both sum the partials in one order, so the solves agree bit for bit, iteration counts
and residual reports included.
"""
import os

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [("2d-n64-f32", 64, 2, 8, "f32"), ("2d-n100-f64", 100, 2, 8, "f64"),
         ("2d-n48-bf16", 48, 2, 8, "bf16"), ("3d-n16-f32", 16, 3, 4, "f32"),
         ("2d-n33-f64", 33, 2, 4, "f64")]


def _factor(a, n, dim, leaf, store, gate, rhs=False):
    """gate: the convergence test in the first apply stage; rhs: the right-hand side made there
    too (both read at factor time)."""
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    if not gate:
        os.environ["HIFCN_NO_CG_GATE"] = "1"
    if not rhs:
        os.environ["HIFCN_NO_RHS_FUSE"] = "1"
    try:
        return hifcn.factor(a_dev, 0.05, n, dim, 1e-6, store=store, leaf=leaf)
    finally:
        os.environ.pop("HIFCN_NO_CG_GATE", None)
        os.environ.pop("HIFCN_NO_RHS_FUSE", None)


@pytest.mark.parametrize("rtol", [1e-10, 1e-2])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gated_solve_is_bitwise_equal(case, rtol, gpu_lib):
    import torch
    name, n, dim, leaf, store = case
    print(f"[case] {name} rtol {rtol}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.12, 91)
    u0 = gen.bumps(n, dim, 3, 92).ravel()
    out = []
    for gate in (True, False):
        h = _factor(a, n, dim, leaf, store, gate)
        u = torch.tensor(u0, device="cuda")
        its, rel = h.cn_solve(u, 4, rtol=rtol, reaction=(1, 1.0, 1.0))
        out.append((u, list(its), rel.tolist()))
        h.close()
    (u1, i1, r1), (u0_, i0, r0) = out
    assert i1 == i0 and r1 == r0
    assert torch.equal(u1, u0_)
    if rtol == 1e-2 and store != "bf16":  # the test after the first update ends the step
        assert min(i1) <= 1, i1


def test_gated_apply_zero_rhs_stops_at_once(gpu_lib):
    """g = 0: the test in the first stage ends the solve before any work."""
    import torch
    n = 64
    h = _factor(gen.grf_coefficient(n, 2, 0.12, 93), n, 2, 8, "f32", True)
    u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    its, rel = h.cn_solve(u, 2)
    assert list(its) == [0, 0] and not u.any()
    h.close()


def _solve(h, u0, steps, **kw):
    import torch
    u = torch.tensor(u0, device="cuda")
    its, rel = h.cn_solve(u, steps, **kw)
    return u, list(its), list(rel)


@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_steps_queued_ahead_match_one_at_a_time(case, gpu_lib):
    """Each CN step is queued before the previous one's outcome is read; when that step needs
    more iterations than predicted, the step queued ahead does nothing and is queued again.
    Same arithmetic either way: bitwise equal to queuing one step at a time (HIFCN_NO_AHEAD)."""
    name, n, dim, leaf, store = case
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.12, 98)
    # a large first step then small ones: the predicted iteration count misses in places
    u0 = (5.0 * gen.bumps(n, dim, 4, 99)).ravel()
    h = _factor(a, n, dim, leaf, store, True, rhs=True)
    out = []
    for ahead in (True, False):
        if not ahead:
            os.environ["HIFCN_NO_AHEAD"] = "1"
        try:
            out.append(_solve(h, u0, 6, rtol=1e-11, reaction=(1, 1.0, 1.0)))
        finally:
            os.environ.pop("HIFCN_NO_AHEAD", None)
    h.close()
    (u1, i1, r1), (u0_, i0, r0) = out
    assert i1 == i0 and r1 == r0
    assert torch_equal(u1, u0_)


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def test_failed_step_stops_the_steps_queued_ahead(gpu_lib):
    """A step that hits maxit ends the solve there: the step queued behind it changes nothing,
    so u holds the failed step's last iterate (as when steps are queued one at a time)."""
    from paper_2004_05566_amd import hifcn
    n = 48
    a = gen.grf_coefficient(n, 2, 0.12, 100)
    u0 = gen.bumps(n, 2, 3, 101).ravel()
    h = _factor(a, n, 2, 8, "f64", True, rhs=True)
    res = []
    for ahead in (True, False):
        if not ahead:
            os.environ["HIFCN_NO_AHEAD"] = "1"
        import torch
        u = torch.tensor(u0, device="cuda")
        try:
            with pytest.raises(hifcn.HifError) as ei:
                h.cn_solve(u, 4, rtol=1e-30, maxit=1)
            assert ei.value.status == hifcn.HIF_ERR_NO_CONV
        finally:
            os.environ.pop("HIFCN_NO_AHEAD", None)
        res.append(u)
    h.close()
    assert torch_equal(res[0], res[1])
    assert not torch_equal(res[0], torch.tensor(u0, device="cuda"))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rhs_made_by_first_stage_matches_own_launch(case, gpu_lib):
    """The first apply stage of a step makes the right-hand side (g, r = g, x = 0 and ||g||^2
    per cell); HIFCN_NO_RHS_FUSE=1 makes it in a launch of its own.  g and the iterates are the
    same arithmetic; only ||g||^2 is summed in another order, so u agrees bit for bit when the
    iteration counts do, and ||r||/||g|| to rounding."""
    import torch
    name, n, dim, leaf, store = case
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.12, 102)
    u0 = gen.bumps(n, dim, 3, 103).ravel()
    out = []
    for fused in (True, False):
        h = _factor(a, n, dim, leaf, store, True, rhs=fused)
        out.append(_solve(h, u0, 4, rtol=1e-10, reaction=(1, 1.0, 1.0)))
        h.close()
    (u1, i1, r1), (u0_, i0, r0) = out
    assert i1 == i0
    assert torch.equal(u1, u0_)
    assert np.allclose(r1, r0, rtol=1e-9, atol=0)


def test_rhs_made_by_first_stage_zero_rhs(gpu_lib):
    """g = 0 with the right-hand side made in the first stage: the first update stops the step,
    u = 0 after no iteration."""
    import torch
    n = 64
    h = _factor(gen.grf_coefficient(n, 2, 0.12, 104), n, 2, 8, "f32", True, rhs=True)
    u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    its, rel = h.cn_solve(u, 3)
    assert list(its) == [0, 0, 0] and list(rel) == [0.0, 0.0, 0.0] and not u.any()
    h.close()


SWEEP = [(24, 2, 4, "f64", 1e-11, 0.3), (40, 2, 8, "f32", 1e-9, 2.0), (57, 2, 8, "bf16", 1e-8, 1.0),
         (72, 2, 8, "f32", 1e-12, 4.0), (100, 2, 8, "f64", 1e-10, 0.5), (12, 3, 4, "f32", 1e-10, 1.0),
         (20, 3, 4, "f64", 1e-12, 3.0)]


@pytest.mark.parametrize("cfg", SWEEP, ids=[f"n{c[0]}-d{c[1]}-{c[3]}" for c in SWEEP])
def test_pipeline_matches_plain_path(cfg, gpu_lib):
    """Every PCG step folded into the apply and steps queued ahead, against the plain sequence of
    launches (test, right-hand side and each step on their own): the same iteration counts and u
    to rounding, over grids, stores, tolerances and amplitudes that make the predicted iteration
    count miss now and then."""
    import torch
    n, dim, leaf, store, rtol, amp = cfg
    print(f"[case] {cfg}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 200 + n)
    u0 = (amp * gen.bumps(n, dim, 3, 300 + n)).ravel()
    out = []
    for plain in (False, True):
        h = _factor(a, n, dim, leaf, store, not plain, rhs=not plain)
        if plain:
            os.environ["HIFCN_NO_AHEAD"] = "1"
        try:
            out.append(_solve(h, u0, 5, rtol=rtol, reaction=(1, 1.0, 1.0)))
        finally:
            os.environ.pop("HIFCN_NO_AHEAD", None)
        h.close()
    (u1, i1, r1), (u0_, i0, r0) = out
    assert i1 == i0, (i1, i0)
    assert torch.linalg.norm(u1 - u0_) <= 1e-12 * torch.linalg.norm(u0_)
    assert np.allclose(r1, r0, rtol=1e-8, atol=0)
