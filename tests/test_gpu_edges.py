"""The 3D factor with the edges skeletonized as well as the faces (Sec. 2.2, 3D paragraph;
HIF_FACTOR_SKEL_EDGES) against the oracle built with skel_edges=True.

With the stencil, every DOF of an edge neighbours DOFs of the four faces around it, which stay
active through the level, so an edge's coupling block keeps full rank at practical eps.  At
eps = 0.5 the edges of these grids (coefficient i.i.d. per cell) do lose DOFs, so those cases
run the build's edge IDs and the apply's edge stages with real compression (the factor is a
poor preconditioner there, which CG absorbs in more iterations); at eps = 1e-3 the edges keep
every DOF and the factor must equal the faces-only one.
"""
import numpy as np
import pytest

from oracle import cn, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, leaf, eps
    ("n8-m4-eps0.5", 8, 4, 0.5),
    ("n12-m3-eps0.5", 12, 3, 0.5),
    ("n16-m4-eps0.5", 16, 4, 0.5),
    ("n16-m4-eps1e-3", 16, 4, 1e-3),
]


def _edge_redundant(F):
    """Redundant DOFs of the oracle's skeletonized 3D edges (two coordinates on a separator)."""
    from oracle import geometry
    coords = fd.node_grid_coords(F.n, 3)
    tot = 0
    for lev, lv in enumerate(F.levels):
        S = geometry.separators(F.n, F.leaf, lev)
        for s in lv.skels:
            dof = (s.redund if len(s.redund) else s.skel)[0]
            if int(np.isin(coords[dof], S).sum()) == 2:
                tot += len(s.redund)
    return tot


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_edge_skeletonization_cn_matches_oracle(case, gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    name, n, leaf, eps = case
    print(f"[case] {name}", flush=True)
    a = gen.iid_loguniform_cells(n, 3, 7)
    dt = 0.05
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, 3, leaf, eps, skel_edges=True)
    F0 = phif.phif_build(A, n, 3, leaf, eps)
    red = _edge_redundant(F)
    assert (red > 0) == (eps > 0.1), red
    u0 = gen.bumps(n, 3, 3, 12)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, 3, lambda r: phif.phif_apply(F, r), 1e-12, react)
    ad = torch.tensor(a, device="cuda")
    h = hifcn.factor(ad, dt, n, 3, eps, store="f64", leaf=leaf, skel_edges=True)
    h0 = hifcn.factor(ad, dt, n, 3, eps, store="f64", leaf=leaf)
    u = torch.tensor(u0.ravel(), device="cuda")
    gits, _ = h.cn_solve(u, 3, rtol=1e-12, maxit=2000, reaction=react)
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - us[-1]) <= 1e-10 * np.linalg.norm(us[-1])
    assert np.abs(ug - us[-1]).max() <= 1e-10 * np.abs(us[-1]).max()
    assert max(abs(int(x) - int(y)) for x, y in zip(gits, its)) <= 1, (list(gits), its)
    # the root (the skeleton DOFs every level left) of the oracle's factor's size, up to the
    # one or two rank decisions that rounding may tip where a pivot ratio meets eps
    info, info0 = h.info(), h0.info()
    assert info["levels"] == len(F.levels)
    slack = 2
    assert abs(info["root"] - len(F.root_idx)) <= slack, (info["root"], len(F.root_idx))
    assert abs(info0["root"] - len(F0.root_idx)) <= slack
    # F^-1 symmetric, and a preconditioner of the oracle's quality
    x = gen.normal_vector(n ** 3, 5)
    y = gen.normal_vector(n ** 3, 6)
    Fx = h.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    Fy = h.apply(torch.tensor(y, device="cuda")).cpu().numpy()
    assert abs(y @ Fx - x @ Fy) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(Fy)
    g_err = np.linalg.norm(x - A @ Fx) / np.linalg.norm(x)
    o_err = np.linalg.norm(x - A @ phif.phif_apply(F, x)) / np.linalg.norm(x)
    assert g_err <= 10 * o_err + 1e-12, (g_err, o_err)
    F0x = h0.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    if red > 0:  # fewer DOFs reach the root than with the faces alone
        assert info["root"] < info0["root"]
    else:        # every edge kept all its DOFs: the faces-only factor, but for the order in
        # which the edges' DOFs reach the next level (pivot order), which changes rounding
        assert abs(info["root"] - info0["root"]) <= slack
        assert np.linalg.norm(Fx - F0x) <= 10 * eps * np.linalg.norm(F0x)
    h.close()
    h0.close()


def test_edge_skeletonization_imported_apply_matches_oracle(gpu_lib):
    """The oracle's factor with compressed edges loaded as data (hif_import): the GPU apply
    against the oracle's apply, element by element."""
    import torch
    from paper_2004_05566_amd import hifcn
    from tests.hifb import factor_to_hifb
    n, leaf, eps = 12, 3, 0.5
    a = gen.iid_loguniform_cells(n, 3, 7)
    A, _ = fd.cn_matrices(a, 0.05)
    F = phif.phif_build(A, n, 3, leaf, eps, skel_edges=True)
    assert _edge_redundant(F) > 0
    ad = torch.tensor(a, device="cuda")
    h = hifcn.import_factor(ad, 0.05, n, 3, factor_to_hifb(F), store="f64", leaf=leaf)
    for seed in (1, 2):
        r = gen.normal_vector(n ** 3, seed)
        z = h.apply(torch.tensor(r, device="cuda")).cpu().numpy()
        ref = phif.phif_apply(F, r)
        assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()
    h.close()


def test_edge_flag_rejects_unknown_bits(gpu_lib):
    import ctypes
    import torch
    from paper_2004_05566_amd import hifcn
    n = 8
    a = torch.ones((n + 1) ** 3, dtype=torch.float64, device="cuda")
    o = hifcn._FactorOpts()
    o.dense_top = -1
    o.flags = 2
    h = ctypes.c_void_p()
    g = hifcn._grid(n, 3, 4)
    st = hifcn._lib.hif_factor_ex(ctypes.c_void_p(a.data_ptr()), 0.05, ctypes.byref(g), 1e-3,
                                  hifcn.STORE["f64"], ctypes.byref(o), hifcn._stream(None),
                                  ctypes.byref(h))
    assert st == 1 and not h.value
