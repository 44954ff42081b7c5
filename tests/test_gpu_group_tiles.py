"""Dense group stages: the whole step of each group as one dense matrix G (forward) and G^T
(backward), formed at factor time from the group's blocks and applied over row and column tiles
of all the level's groups (used for groups too large for one workgroup's LDS).

HIFCN_GROUP_TILES=1 at factor time puts the groups of every level in dense form, so small
problems exercise the path against the staged kernels and the oracle.  Both apply the same
operator, multiplied out in a different order, so they agree to rounding.
"""
import os

import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [("2d-n32-m8", 32, 2, 8), ("2d-n127-m8", 127, 2, 8), ("2d-n40-m4", 40, 2, 4),
         ("3d-n12-m4", 12, 3, 4), ("3d-n16-m4", 16, 3, 4)]


def _factor(a, dt, n, dim, leaf, eps, store, tiles, top="0"):
    """top: HIFCN_DENSE_TOP (off by default here, so that every level's group stages run;
    None keeps the library's default)."""
    import torch
    from paper_2004_05566_amd import hifcn
    a_dev = torch.tensor(a, dtype=torch.float64, device="cuda")
    old = {k: os.environ.pop(k, None) for k in ("HIFCN_GROUP_TILES", "HIFCN_DENSE_TOP")}
    if tiles:
        os.environ["HIFCN_GROUP_TILES"] = "1"
    if top is not None:
        os.environ["HIFCN_DENSE_TOP"] = top
    try:
        return hifcn.factor(a_dev, dt, n, dim, eps, store=store, leaf=leaf)
    finally:
        for k, v in old.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_group_tiles_match_staged(case, store, gpu_lib):
    import torch
    name, n, dim, leaf = case
    print(f"[case] {name} {store}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.1, 71)
    h1 = _factor(a, 0.05, n, dim, leaf, 1e-4, store, True)
    h0 = _factor(a, 0.05, n, dim, leaf, 1e-4, store, False)
    rng = np.random.default_rng(5)
    for _ in range(2):  # the scratch vectors are reused from one apply to the next
        x = torch.tensor(rng.normal(size=n ** dim), device="cuda")
        y1, y0 = h1.apply(x), h0.apply(x)
        tol = {"f64": 1e-13, "f32": 1e-5, "bf16": 1e-2}[store]
        assert torch.linalg.norm(y1 - y0) <= tol * torch.linalg.norm(y0)
    h1.close()
    h0.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_group_tiles_cn_matches_oracle(case, gpu_lib):
    import torch
    name, n, dim, leaf = case
    eps, dt = 1e-6, 0.05
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 72)
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, dim, leaf, eps)
    u0 = gen.bumps(n, dim, 3, 73)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 2, lambda r: phif.phif_apply(F, r), 1e-12, react)
    h = _factor(a, dt, n, dim, leaf, eps, "f64", True)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 2, rtol=1e-12, reaction=react)
    assert np.linalg.norm(u.cpu().numpy() - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    h.close()


def test_multi_launch_stage_timing(gpu_lib):
    """A stage of several launches is timed from the start of its first launch to the end of
    its last: the dense group stages and the dense root of a 32^3 grid (product, then the
    write-back of the results)."""
    import torch
    n, dim, leaf = 32, 3, 8
    a = gen.grf_coefficient(n, dim, 0.15, 74)
    h = _factor(a, 0.02, n, dim, leaf, 1e-4, "f32", False)
    levels = h.info()["levels"]
    x = torch.tensor(np.random.default_rng(6).normal(size=n ** dim), device="cuda")
    h.apply(x)
    total = {}
    for lev, stage in ((levels - 1, "group_fwd"), (levels - 1, "group_bwd"), (levels, "root")):
        h.profile_stage(lev, stage, True)
        for _ in range(3):
            h.apply(x)
        p = h.profile_read()
        h.profile_stage(lev, stage, False)
        assert p["launches"] == 3 and p["ms"] > 0 and p["bytes"] > 0, (lev, stage, p)
        total[stage] = p["ms"] / 3
    # the three stages run in sequence inside one apply, so together they take less than it
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(10):
        h.apply(x)
    t1.record()
    torch.cuda.synchronize()
    assert sum(total.values()) < t0.elapsed_time(t1) / 10, total
    h.close()


@pytest.mark.parametrize("top", [None, "0"], ids=["top", "notop"])
@pytest.mark.parametrize("n,dim,leaf", [(64, 2, 8), (32, 3, 8)])
def test_apply_bytes_sum_of_stages(n, dim, leaf, top, gpu_lib):
    """hif_get_info's apply_bytes is the sum of the bytes every stage reports (fused launches
    count the stages they run; dense forms count the dense matrices)."""
    import torch
    a = gen.grf_coefficient(n, dim, 0.15, 75)
    h = _factor(a, 0.02, n, dim, leaf, 1e-4, "f32", False, top)
    levels = h.info()["levels"]
    x = torch.tensor(np.random.default_rng(7).normal(size=n ** dim), device="cuda")
    tot = 0
    for lev in range(levels + 1):
        for st in ("cell_fwd", "group_fwd", "root", "group_bwd", "cell_bwd"):
            if (st == "root") != (lev == levels):
                continue
            h.profile_stage(lev, st, True)
            h.apply(x)
            p = h.profile_read()
            h.profile_stage(lev, st, False)
            tot += p["bytes"] if p["launches"] else 0
    assert tot == h.info()["apply_bytes"] > 0
    h.close()
