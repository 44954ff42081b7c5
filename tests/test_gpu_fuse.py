"""Fused apply launches (group stage of level l with the cell stage of level l+1; the last level's
groups with the root) against the unfused launch sequence and the oracle.

HIFCN_NO_FUSE=1 at factor time keeps one launch per stage.  Both sequences do the same
arithmetic with different lane splits of the dot products, so they agree to rounding.  The dense
top (HIFCN_DENSE_TOP) is off here so that every level's stages run.
"""
import os

import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [("2d-n32-m8", 32, 2, 8), ("2d-n64-m8", 64, 2, 8), ("2d-n40-m4", 40, 2, 4),
         ("2d-n127-m8", 127, 2, 8), ("3d-n12-m4", 12, 3, 4), ("3d-n16-m4", 16, 3, 4)]


def _factor(a, dt, n, dim, leaf, eps, store, fuse):
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    old = {k: os.environ.pop(k, None) for k in ("HIFCN_NO_FUSE", "HIFCN_DENSE_TOP")}
    if not fuse:
        os.environ["HIFCN_NO_FUSE"] = "1"
    os.environ["HIFCN_DENSE_TOP"] = "0"  # every level's stages run (the fusions are tested)
    try:
        return hifcn.factor(a_dev, dt, n, dim, eps, store=store, leaf=leaf)
    finally:
        for k, v in old.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_apply_matches_unfused(case, store, gpu_lib):
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name} {store}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 61)
    h1 = _factor(a, 0.05, n, dim, leaf, 1e-4, store, True)
    h0 = _factor(a, 0.05, n, dim, leaf, 1e-4, store, False)
    x = torch.tensor(np.random.default_rng(3).normal(size=n ** dim), device="cuda")
    y1, y0 = h1.apply(x), h0.apply(x)
    tol = {"f64": 1e-13, "f32": 1e-5, "bf16": 1e-2}[store]
    assert torch.linalg.norm(y1 - y0) <= tol * torch.linalg.norm(y0)
    levels = h1.info()["levels"]
    # the fused factor runs no separate cell stage above level 0 and no separate backward
    # group stage on the last level; the unfused one runs every stage
    fused_cells = 0
    for lev in range(1, levels):
        h1.profile_stage(lev, "cell_fwd", True)
        h1.apply(x)
        fused_cells += h1.profile_read()["launches"] == 0
        h1.profile_stage(lev, "cell_fwd", False)
        h0.profile_stage(lev, "cell_fwd", True)
        h0.apply(x)
        assert h0.profile_read()["launches"] == 1
        h0.profile_stage(lev, "cell_fwd", False)
    if dim == 2:
        assert fused_cells == levels - 1
    h1.close()
    h0.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_cn_matches_oracle(case, gpu_lib):
    import torch
    name, n, dim, leaf = case
    eps = 1e-6
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 62)
    dt = 0.05
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 63)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 2, lambda r: phif.phif_apply(F, r), 1e-12, react)
    h = _factor(a, dt, n, dim, leaf, eps, "f64", True)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 2, rtol=1e-12, reaction=react)
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()


def test_fused_root_profile_bytes(gpu_lib):
    """The fused root launch reports the bytes of the root and both group stages it runs."""
    import torch
    n = 64
    a = gen.grf_coefficient(n, 2, 0.1, 64)
    h1 = _factor(a, 0.05, n, 2, 8, 1e-4, "f32", True)
    h0 = _factor(a, 0.05, n, 2, 8, 1e-4, "f32", False)
    x = torch.tensor(np.random.default_rng(4).normal(size=n * n), device="cuda")
    levels = h1.info()["levels"]
    got = {}
    for h, key in ((h1, "fused"), (h0, "plain")):
        tot = 0
        for stage, lev in (("root", levels), ("group_fwd", levels - 1), ("group_bwd", levels - 1)):
            h.profile_stage(lev, stage, True)
            h.apply(x)
            p = h.profile_read()
            h.profile_stage(lev, stage, False)
            tot += p["bytes"] if p["launches"] else 0
        got[key] = tot
    assert got["fused"] == got["plain"] > 0
    h1.close()
    h0.close()
