"""Blocked front elimination on the matrix cores (large cells and the root of the GPU build).

HIFCN_FRONT_MIN=1 routes every dense-H cell and the root through the front path, so small grids
exercise it against the oracle: eps = 0 must give the exact inverse, eps > 0 the oracle's u to
1e-10 with iteration counts within 1, and the two GPU paths must agree with each other.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [("2d-n15-m4", 15, 2, 4), ("2d-n40-m4", 40, 2, 4), ("2d-n70-m4", 70, 2, 4),
         ("3d-n8-m4", 8, 3, 4), ("3d-n12-m4", 12, 3, 4), ("2d-n10-root", 10, 2, 8)]


def _factor(a, dt, n, dim, leaf, eps, front_min, store="f64"):
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    old = os.environ.get("HIFCN_FRONT_MIN")
    os.environ["HIFCN_FRONT_MIN"] = str(front_min)
    try:
        return hifcn.factor(a_dev, dt, n, dim, eps, store=store, leaf=leaf)
    finally:
        if old is None:
            del os.environ["HIFCN_FRONT_MIN"]
        else:
            os.environ["HIFCN_FRONT_MIN"] = old


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_front_path_eps_zero_is_exact_inverse(case, gpu_lib):
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name}", flush=True)
    a = gen.iid_loguniform_cells(n, dim, 3)
    dt = 0.05
    A, _ = fd.cn_matrices(a, dt)
    h = _factor(a, dt, n, dim, leaf, 0.0, 1)
    rng = np.random.default_rng(4)
    r = rng.normal(size=A.shape[0])
    z = h.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    exact = spla.spsolve(A.tocsc(), r)
    assert np.linalg.norm(z - exact) <= 1e-10 * np.linalg.norm(exact)
    h.close()


@pytest.mark.parametrize("case", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_front_path_cn_matches_oracle(case, gpu_lib):
    import torch
    name, n, dim, leaf = case
    eps = 1e-6
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 11)
    dt = 0.05
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 12)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 3, lambda r: phif.phif_apply(F, r), 1e-12, react)
    h = _factor(a, dt, n, dim, leaf, eps, 1)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 3, rtol=1e-12, reaction=react)
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_front_and_workgroup_paths_agree(case, gpu_lib):
    """Same factor from both elimination paths (eps = 0: no rank decision can differ)."""
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 21)
    dt = 0.1
    h1 = _factor(a, dt, n, dim, leaf, 0.0, 1)
    h2 = _factor(a, dt, n, dim, leaf, 0.0, 1 << 30)
    x = torch.tensor(np.random.default_rng(7).normal(size=n ** dim), device="cuda")
    y1, y2 = h1.apply(x), h2.apply(x)
    assert torch.linalg.norm(y1 - y2) <= 1e-12 * torch.linalg.norm(y2)
    assert h1.info()["entries"] == h2.info()["entries"]
    h1.close()
    h2.close()


def test_front_path_detects_non_spd(gpu_lib):
    from paper_2004_05566_amd import hifcn
    n = 12
    a = -np.ones((n + 1, n + 1))
    with pytest.raises(hifcn.HifError) as e:
        _factor(a, 1.0, n, 2, 4, 1e-6, 1)
    assert e.value.status == hifcn.HIF_ERR_NOT_SPD


def test_front_path_large_3d_cells(gpu_lib):
    """3D n = 32, m = 4: level-1 and level-2 cells and the root exceed 128 interior DOFs and
    take the front path by default; CN against the oracle at eps = 1e-6."""
    import torch
    n, dim, leaf, eps = 32, 3, 4, 1e-6
    a = gen.grf_coefficient(n, dim, 0.15, 31)
    dt = 0.05
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 32)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 2, lambda r: phif.phif_apply(F, r), 1e-12)
    h = _factor(a, dt, n, dim, leaf, eps, 128)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 2, rtol=1e-12)
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()
