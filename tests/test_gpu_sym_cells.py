"""Level-0 cells held as A_II^-1 (one symmetric product per sweep) against the same factor with
L^-1 (two triangular products per sweep, HIFCN_NO_SYM_CELLS=1), and against the oracle.

Both forms apply the same E_0 (eq2_3): the forward sweep gives c_B = A_BI A_II^-1 y_I either way
and the backward sweep x_I = A_II^-1 (y_I - A_IB x_B).  They differ only in rounding, so F^-1
must agree to a bound set by the conditioning of the level-0 interior blocks, and CN steps must
give the oracle's u.  Cases: 2D cells of 7^2 / 8^2 interiors, 3D cells of 3^3 interiors (whose
boundary of up to 98 DOFs spans two passes of the wavefront), reaction on and off, and the
first apply stage in its three forms (plain, with the PCG test, forming the right-hand side).
"""
import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, dim, leaf, eps, dt, coefficient, tolerance of the F^-1 comparison (FP64)
    ("2d-n32-m8", 32, 2, 8, 1e-6, 1e-2, "grf", 1e-12),
    ("2d-n64-m8-iid", 64, 2, 8, 1e-4, 1e-1, "iid", 1e-9),
    ("2d-n40-m4", 40, 2, 4, 1e-3, 5e-2, "grf", 1e-12),
    ("3d-n12-m4", 12, 3, 4, 1e-4, 2e-2, "grf", 1e-12),
]


def _coef(kind, n, dim, seed):
    return gen.iid_loguniform_cells(n, dim, seed) if kind == "iid" else \
        gen.grf_coefficient(n, dim, 0.15, seed)


def _pair(case, store, monkeypatch):
    import torch
    from paper_2004_05566_amd import hifcn
    name, n, dim, leaf, eps, dt, kind, _ = case
    a = torch.tensor(_coef(kind, n, dim, 71), device="cuda")
    monkeypatch.delenv("HIFCN_NO_SYM_CELLS", raising=False)
    hs = hifcn.factor(a, dt, n, dim, eps, store=store, leaf=leaf)
    monkeypatch.setenv("HIFCN_NO_SYM_CELLS", "1")
    ht = hifcn.factor(a, dt, n, dim, eps, store=store, leaf=leaf)
    monkeypatch.delenv("HIFCN_NO_SYM_CELLS")
    return hs, ht


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_symmetric_cells_apply_equals_triangular(case, gpu_lib, monkeypatch):
    import torch
    print(f"[case] {case[0]}", flush=True)
    hs, ht = _pair(case, "f64", monkeypatch)
    assert hs.factor_bytes() == ht.factor_bytes()
    N = hs.N
    for seed in (1, 2):
        x = torch.tensor(gen.normal_vector(N, seed), device="cuda")
        zs, zt = hs.apply(x), ht.apply(x)
        d = (torch.abs(zs - zt).max() / torch.abs(zt).max()).item()
        print(f"  max|dz| / max|z| = {d:.2e}", flush=True)
        assert d <= case[7], d
    # in place, and symmetric
    y = torch.tensor(gen.normal_vector(N, 3), device="cuda")
    fy = hs.apply(y)
    x = torch.tensor(gen.normal_vector(N, 4), device="cuda")
    fx = x.clone()
    hs.apply(fx, out=fx)
    s = abs(torch.dot(x, fy) - torch.dot(y, fx)) / (torch.linalg.norm(x) * torch.linalg.norm(fy))
    assert s.item() <= 1e-12
    hs.close()
    ht.close()


@pytest.mark.parametrize("store,tol", [("f32", 2e-5), ("bf16", 3e-2)])
def test_symmetric_cells_reduced_storage(store, tol, gpu_lib, monkeypatch):
    import torch
    case = CASES[0]
    hs, ht = _pair(case, store, monkeypatch)
    x = torch.tensor(gen.normal_vector(hs.N, 5), device="cuda")
    zs, zt = hs.apply(x), ht.apply(x)
    assert (torch.linalg.norm(zs - zt) / torch.linalg.norm(zt)).item() <= tol
    hs.close()
    ht.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("path", ["default", "no-rhs-fuse", "no-gate"])
def test_symmetric_cells_cn_matches_oracle(case, path, gpu_lib, monkeypatch):
    """CN steps with the PCG test and the right-hand side made inside the first apply stage
    (the default where level 0 allows it), or as launches of their own: the oracle's u to
    1e-10 (rtol 1e-12 on both sides) with iteration counts within one."""
    import torch
    from paper_2004_05566_amd import hifcn
    name, n, dim, leaf, eps, dt, kind, _ = case
    print(f"[case] {name} {path}", flush=True)
    if path == "no-rhs-fuse":
        monkeypatch.setenv("HIFCN_NO_RHS_FUSE", "1")
    elif path == "no-gate":
        monkeypatch.setenv("HIFCN_NO_CG_GATE", "1")
    a = _coef(kind, n, dim, 71)
    u0 = gen.bumps(n, dim, 3, 72)
    react = (1, 1.0, 1.0) if dim == 2 else (0, 0.0, 1.0)
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 3, lambda r: phif.phif_apply(F, r), 1e-12, react)
    h = hifcn.factor(torch.tensor(a, device="cuda"), dt, n, dim, eps, store="f64", leaf=leaf)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, grel = h.cn_solve(u, 3, rtol=1e-12, reaction=react)
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert np.abs(ug - us[-1]).max() <= 1e-10 * np.abs(us[-1]).max()
    assert all(abs(int(x) - int(y)) <= 1 for x, y in zip(gits, its)), (list(gits), its)
    # the factor as the solver (its steps queue the first stage with the right-hand side)
    ud = torch.tensor(u0.ravel(), device="cuda")
    h.cn_solve_direct(ud, 2, reaction=react)
    ref = cn.cn_solve_direct(B, u0, dt, 2, lambda r: phif.phif_apply(F, r), react)[-1]
    # the oracle's factor and the GPU's differ in their skeletons, so the two direct solves agree
    # only to the factors' accuracy (O(eps)); a broken first stage would be off by O(1)
    assert np.linalg.norm(ud.cpu().numpy() - ref) <= 100 * eps * np.linalg.norm(ref)
    h.close()
