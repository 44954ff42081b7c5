"""The multi-workgroup pivoted QR of large IDs against the one-workgroup QR and the oracle.

HIFCN_QR_MULTI_MIN=1 sends every ID through the per-step launches; both paths take the same
pivots with the same lane split of every reduction, so the ranks and skeletons are identical;
the products after the QR run on the matrix cores in the multi-workgroup path, so the factors
agree to rounding.
"""
import os

import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [("2d-n40-m4", 40, 2, 4), ("2d-n64-m8", 64, 2, 8), ("3d-n12-m4", 12, 3, 4),
         ("3d-n16-m4", 16, 3, 4)]


def _factor(a, dt, n, dim, leaf, eps, qr_min, store="f64"):
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    old = os.environ.get("HIFCN_QR_MULTI_MIN")
    os.environ["HIFCN_QR_MULTI_MIN"] = str(qr_min)
    try:
        return hifcn.factor(a_dev, dt, n, dim, eps, store=store, leaf=leaf)
    finally:
        if old is None:
            del os.environ["HIFCN_QR_MULTI_MIN"]
        else:
            os.environ["HIFCN_QR_MULTI_MIN"] = old


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_multi_workgroup_qr_matches_one_workgroup_qr(case, eps, gpu_lib):
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name} eps={eps}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 71)
    h1 = _factor(a, 0.05, n, dim, leaf, eps, 1)
    h0 = _factor(a, 0.05, n, dim, leaf, eps, 1 << 30)
    assert h1.info()["entries"] == h0.info()["entries"]
    x = torch.tensor(np.random.default_rng(5).normal(size=n ** dim), device="cuda")
    y1, y0 = h1.apply(x), h0.apply(x)
    assert torch.linalg.norm(y1 - y0) <= 1e-12 * torch.linalg.norm(y0)
    h1.close()
    h0.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_multi_workgroup_qr_cn_matches_oracle(case, gpu_lib):
    import torch
    name, n, dim, leaf = case
    eps = 1e-6
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 72)
    dt = 0.05
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 73)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 2, lambda r: phif.phif_apply(F, r), 1e-12)
    h = _factor(a, dt, n, dim, leaf, eps, 1)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 2, rtol=1e-12)
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()
