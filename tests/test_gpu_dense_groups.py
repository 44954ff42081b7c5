"""Group stages as one dense product per group against the stored blocks applied step by step
(HIFCN_NO_DENSE_GROUPS=1).

In levels that qualify, each group's forward step (block Jacobi, then the skeletonization of
eq_T / eq2_9) is multiplied out into G at factor time and the backward step is G^T: the same
operator, so F^-1 agrees to rounding, stays symmetric, and CN steps give the oracle's u.
"""
import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, dim, leaf, eps, store, tolerance of the F^-1 comparison
    ("2d-n64-f64", 64, 2, 8, 1e-3, "f64", 1e-12),
    ("2d-n127-f64-eps1e-6", 127, 2, 8, 1e-6, "f64", 1e-12),
    ("2d-n128-f32", 128, 2, 8, 1e-3, "f32", 1e-5),
    ("3d-n16-f64", 16, 3, 4, 1e-3, "f64", 1e-12),
    ("3d-n16-f32", 16, 3, 4, 1e-3, "f32", 1e-5),
]


def _pair(n, dim, leaf, eps, store, monkeypatch, dt=0.1):
    import torch
    from paper_2004_05566_amd import hifcn
    a = torch.tensor(gen.grf_coefficient(n, dim, 0.15, 81), device="cuda")
    monkeypatch.delenv("HIFCN_NO_DENSE_GROUPS", raising=False)
    hd = hifcn.factor(a, dt, n, dim, eps, store=store, leaf=leaf, dense_top=0)
    monkeypatch.setenv("HIFCN_NO_DENSE_GROUPS", "1")
    hp = hifcn.factor(a, dt, n, dim, eps, store=store, leaf=leaf, dense_top=0)
    monkeypatch.delenv("HIFCN_NO_DENSE_GROUPS")
    return hd, hp


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_dense_groups_apply_equals_stepwise(case, gpu_lib, monkeypatch):
    import torch
    name, n, dim, leaf, eps, store, tol = case
    print(f"[case] {name}", flush=True)
    hd, hp = _pair(n, dim, leaf, eps, store, monkeypatch)
    N = n ** dim
    for seed in (1, 2):
        x = torch.tensor(gen.normal_vector(N, seed), device="cuda")
        zd, zp = hd.apply(x), hp.apply(x)
        d = (torch.abs(zd - zp).max() / torch.abs(zp).max()).item()
        print(f"  max|dz| / max|z| = {d:.2e}", flush=True)
        assert d <= tol, d
        assert not torch.equal(zd, zp)  # the dense path ran
    # symmetric: x.F^-1 y = y.F^-1 x
    x = torch.tensor(gen.normal_vector(N, 3), device="cuda")
    y = torch.tensor(gen.normal_vector(N, 4), device="cuda")
    fx, fy = hd.apply(x), hd.apply(y)
    srel = abs(torch.dot(y, fx) - torch.dot(x, fy)) / (torch.linalg.norm(x) * torch.linalg.norm(fy))
    assert srel.item() <= (1e-12 if store == "f64" else 1e-5)
    hd.close()
    hp.close()


def test_dense_groups_cn_matches_oracle(gpu_lib):
    """CN steps with dense group stages (and no dense top, so every level's groups run): the
    oracle's u to 1e-10 with iteration counts within one."""
    import torch
    from paper_2004_05566_amd import hifcn
    n, leaf, eps, dt = 63, 8, 1e-3, 0.05
    a = gen.grf_coefficient(n, 2, 0.15, 11)
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, 2, leaf, eps)
    u0 = gen.bumps(n, 2, 3, 12)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 3, lambda r: phif.phif_apply(F, r), 1e-12, react)
    h = hifcn.factor(torch.tensor(a, device="cuda"), dt, n, 2, eps, store="f64", leaf=leaf,
                     dense_top=0)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 3, rtol=1e-12, reaction=react)
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert np.abs(ug - us[-1]).max() <= 1e-10 * np.abs(us[-1]).max()
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()
