"""Argument checks of the binding and the library's handling of a non-finite state.

The C ABI takes raw device pointers, so the binding checks every tensor's length against the
handle (ValueError before any launch).  A NaN in u makes ||g||^2 non-finite: the step must end
with HIF_ERR_NO_CONV after no iteration and leave u as it was, whether the right-hand side is
formed by the first apply stage or by a launch of its own.
"""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _handle(n=32, store="f64"):
    import torch
    from paper_2004_05566_amd import hifcn
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.1, 5), device="cuda")
    return hifcn.factor(a, 1e-2, n, 2, 1e-4, store=store)


def test_wrong_lengths_raise_before_launch(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    n = 32
    short = torch.ones(n * n - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        hifcn.factor(torch.ones((n + 1) ** 2 - 1, dtype=torch.float64, device="cuda"), 1e-2, n, 2,
                     1e-4)
    with pytest.raises(ValueError):
        hifcn.import_factor(torch.ones(n * n, dtype=torch.float64, device="cuda"), 1e-2, n, 2,
                            b"")
    h = _handle(n)
    good = torch.ones(n * n, dtype=torch.float64, device="cuda")
    for call in (lambda: h.apply(short), lambda: h.apply(good, out=short),
                 lambda: h.spmv(short), lambda: h.spmv(good, out=short),
                 lambda: h.cn_solve(short, 1), lambda: h.cn_step(short),
                 lambda: h.cn_solve_direct(short, 1),
                 lambda: h.set_coefficient(torch.ones(n * n, dtype=torch.float64, device="cuda")),
                 lambda: h.refactor(torch.ones(7, dtype=torch.float64, device="cuda")),
                 lambda: hifcn.cn_batch_step([h], [short], [(0, 0.0, 1.0)], [1e-8], [10],
                                             [torch.cuda.current_stream()]),
                 lambda: hifcn.cn_batch_step([h], [good, good], [(0, 0.0, 1.0)], [1e-8], [10],
                                             [torch.cuda.current_stream()])):
        with pytest.raises(ValueError):
            call()
    # nothing ran: the handle still works
    its, _ = h.cn_solve(good, 1, rtol=1e-10)
    assert its[0] >= 1
    h.close()


@pytest.mark.parametrize("fused", [True, False], ids=["rhs-in-apply", "rhs-launch"])
def test_nan_state_reports_no_convergence_and_keeps_u(fused, gpu_lib, monkeypatch):
    import torch
    from paper_2004_05566_amd import hifcn
    if not fused:
        monkeypatch.setenv("HIFCN_NO_RHS_FUSE", "1")
    h = _handle()
    u0 = gen.bumps(32, 2, 3, 9).ravel()
    u0[100] = np.nan
    for call in ("step", "solve", "batch"):
        u = torch.tensor(u0, device="cuda")
        with pytest.raises(hifcn.HifError) as ei:
            if call == "step":
                h.cn_step(u, rtol=1e-10)
            elif call == "solve":
                h.cn_solve(u, 3, rtol=1e-10)
            else:
                its, rel, sts = hifcn.cn_batch_step([h], [u], [(0, 0.0, 1.0)], [1e-10], [50],
                                                    [torch.cuda.current_stream()])
                assert sts[0] == hifcn.HIF_ERR_NO_CONV and its[0] == 0
                raise hifcn.HifError(int(sts[0]), "batch")
        assert ei.value.status == hifcn.HIF_ERR_NO_CONV, call
        got = u.cpu().numpy()
        assert np.isnan(got[100]) and np.array_equal(np.delete(got, 100), np.delete(u0, 100)), call
    # an Inf as well, and the handle recovers with a finite state
    u1 = gen.bumps(32, 2, 3, 9).ravel()
    u1[5] = np.inf
    u = torch.tensor(u1, device="cuda")
    with pytest.raises(hifcn.HifError) as ei:
        h.cn_step(u, rtol=1e-10)
    assert ei.value.status == hifcn.HIF_ERR_NO_CONV
    assert np.array_equal(u.cpu().numpy(), u1)
    u = torch.tensor(gen.bumps(32, 2, 3, 9).ravel(), device="cuda")
    its, _ = h.cn_solve(u, 2, rtol=1e-10)
    assert all(1 <= i <= 20 for i in its)
    h.close()
