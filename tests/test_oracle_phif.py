"""Pins of the oracle's PHIF (Sec. 2.2) and ID (eq2_5).

The block oracle is checked against (a) the dense-literal transcription of the paper's N x N
factor matrices, (b) the exact inverse when eps = 0 (the method then degenerates to a nested
dissection block Cholesky and F = A), (c) the structural identities the paper states after each
step, (d) symmetry and positive definiteness of F^-1, and (e) geometric counts of active DOFs.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import cn, fd, geometry, interp, phif, phif_dense
from workloads import gen


def _problem(n, dim, seed=7, dt=0.05):
    a = gen.iid_loguniform_cells(n, dim, seed)
    A, B = fd.cn_matrices(a, dt)
    return A, B


CASES = [(15, 2, 4), (7, 3, 4), (8, 3, 4)]


@pytest.mark.parametrize("n,dim,m", CASES)
@pytest.mark.parametrize("eps", [0.0, 1e-6, 1e-3])
def test_block_oracle_equals_dense_literal(n, dim, m, eps):
    A, _ = _problem(n, dim)
    F = phif.phif_build(A, n, dim, m, eps)
    D = phif_dense.phif_dense(A.toarray(), n, dim, m, eps)
    Fi = phif.phif_dense_inverse(F)
    assert np.linalg.norm(Fi - D.Finv) <= 1e-12 * np.linalg.norm(D.Finv)
    # same skeleton sizes on every edge
    ranks_block = [sorted(len(s.skel) for s in lv.skels) for lv in F.levels]
    ranks_dense = [sorted(k for _, k in r) for r in D.ranks]
    assert ranks_block == ranks_dense


@pytest.mark.parametrize("n,dim,m", [(15, 2, 4), (32, 2, 8), (8, 3, 4)])
def test_eps_zero_reproduces_exact_inverse(n, dim, m):
    A, _ = _problem(n, dim, seed=3)
    Ad = A.toarray()
    F = phif.phif_build(A, n, dim, m, 0.0)
    Fi = phif.phif_dense_inverse(F)
    assert np.linalg.norm(Fi - np.linalg.inv(Ad)) <= 1e-11 * np.linalg.norm(np.linalg.inv(Ad))
    D = phif_dense.phif_dense(Ad, n, dim, m, 0.0)
    assert np.linalg.norm(D.F - Ad) <= 1e-11 * np.linalg.norm(Ad)   # eqA with nothing dropped


def test_structural_identities_after_each_step():
    n, dim, m, eps = 15, 2, 4, 1e-4
    A, _ = _problem(n, dim, seed=9)
    D = phif_dense.phif_dense(A.toarray(), n, dim, m, eps)
    N = n * n
    for lev, step, Amat, info in D.snapshots:
        scale = np.abs(Amat).max()
        if step == 1:
            # eq2_3: interiors become identity blocks decoupled from everything else
            for I in info["cells"]:
                rest = np.setdiff1d(np.arange(N), I)
                assert np.allclose(Amat[np.ix_(I, I)], np.eye(len(I)), atol=1e-12)
                assert np.abs(Amat[np.ix_(I, rest)]).max() <= 1e-12 * scale
        if step == 2:
            # jacobi-precond / eq3_2: every edge and corner diagonal block is the identity
            for g in info["groups"]:
                assert np.allclose(Amat[np.ix_(g, g)], np.eye(len(g)), atol=1e-12)
        if step == 3:
            # eq2_9: redundant DOFs end up as identity rows decoupled from the rest
            for (g, skel, red, T) in info["edges"]:
                rest = np.setdiff1d(np.arange(N), red)
                assert np.allclose(Amat[np.ix_(red, red)], np.eye(len(red)), atol=1e-12)
                if len(red):
                    assert np.abs(Amat[np.ix_(red, rest)]).max() <= 1e-12 * scale
                # X = I - T (I + T^T T)^-1 T^T on the skeleton block
                X = np.eye(len(skel)) - T @ np.linalg.solve(np.eye(len(red)) + T.T @ T, T.T)
                assert np.allclose(Amat[np.ix_(skel, skel)], X, atol=1e-12)
    # eq3_4: A_L is the identity outside the root block
    out = np.setdiff1d(np.arange(N), D.root_idx)
    assert np.allclose(D.AL[np.ix_(out, out)], np.eye(len(out)), atol=1e-12)


def test_id_residual_bound_eq2_5():
    """||A_{R,I~} - A_{R,I^} T|| <= 10 eps ||A_{R,I}|| for every edge (the dropped block)."""
    n, dim, m = 15, 2, 4
    A, _ = _problem(n, dim, seed=13)
    for eps in [1e-2, 1e-4, 1e-6]:
        D = phif_dense.phif_dense(A.toarray(), n, dim, m, eps)
        for lev, step, Amat, info in D.snapshots:
            if step != 3:
                continue
        # recompute from the step-2 snapshot of each level
        snaps = {(l, s): (Am, inf) for l, s, Am, inf in D.snapshots}
        for lev in range(len(D.Rs)):
            A2, _ = snaps[(lev, 2)]
            _, inf3 = snaps[(lev, 3)]
            for (g, skel, red, T) in inf3["edges"]:
                rest = np.setdiff1d(np.arange(A2.shape[0]), g)
                active_rows = rest[np.abs(A2[np.ix_(rest, g)]).sum(axis=1) > 0]
                Mblk = A2[np.ix_(active_rows, g)]
                if len(red) == 0:
                    continue
                res = A2[np.ix_(active_rows, red)] - A2[np.ix_(active_rows, skel)] @ T
                assert np.linalg.norm(res, 2) <= 10 * eps * np.linalg.norm(Mblk, 2)


def test_id_on_exactly_low_rank_matrix():
    rng = np.random.default_rng(1)
    U = rng.normal(size=(40, 3))
    V = rng.normal(size=(3, 9))
    Mlow = U @ V
    sk, rd, T = interp.interp_decomp(Mlow, 1e-10)
    assert len(sk) == 3 and len(rd) == 6
    assert np.allclose(Mlow[:, rd], Mlow[:, sk] @ T, atol=1e-10)
    sk0, rd0, T0 = interp.interp_decomp(np.zeros((5, 4)), 1e-6)
    assert len(sk0) == 0 and len(rd0) == 4
    skf, rdf, _ = interp.interp_decomp(rng.normal(size=(20, 5)), 0.0)
    assert len(skf) == 5 and len(rdf) == 0


@pytest.mark.parametrize("n,dim,m,eps", [(15, 2, 4, 1e-3), (32, 2, 8, 1e-6), (8, 3, 4, 1e-3)])
def test_inverse_symmetric_positive_definite(n, dim, m, eps):
    A, _ = _problem(n, dim, seed=21)
    F = phif.phif_build(A, n, dim, m, eps)
    Fi = phif.phif_dense_inverse(F)
    assert np.linalg.norm(Fi - Fi.T) <= 1e-13 * np.linalg.norm(Fi)
    sla.cholesky(0.5 * (Fi + Fi.T), lower=True)   # raises if not SPD


def test_inverse_error_decreases_with_eps():
    n, dim, m = 31, 2, 4
    A, _ = _problem(n, dim, seed=2, dt=0.1)
    Ad = A.toarray()
    errs = []
    for eps in [1e-2, 1e-4, 1e-6, 0.0]:
        F = phif.phif_build(A, n, dim, m, eps)
        E = np.eye(A.shape[0]) - Ad @ phif.phif_dense_inverse(F)
        errs.append(np.linalg.norm(E, 2))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-10 and errs[2] < 1e-3


@pytest.mark.parametrize("n,dim,m", [(32, 2, 8), (31, 2, 4), (16, 3, 4)])
def test_active_counts_match_geometry_at_eps_zero(n, dim, m):
    """With no compression, level l eliminates exactly the DOFs with no coordinate in S_l that
    survived level l-1 (those with a coordinate in S_{l-1}); brute-force count over the grid."""
    A, _ = _problem(n, dim, seed=5)
    F = phif.phif_build(A, n, dim, m, 0.0)
    L = geometry.num_levels(n, m)
    pts = np.array(np.meshgrid(*([np.arange(1, n + 1)] * dim), indexing="ij")).reshape(dim, -1).T
    alive = np.ones(len(pts), bool)
    for lev in range(L):
        S = set(geometry.separators(n, m, lev).tolist())
        on = np.array([any(int(c) in S for c in p) for p in pts])
        before = alive.sum()
        alive = alive & on
        assert F.active_counts[lev] == (before, alive.sum(), alive.sum())
    assert len(F.root_idx) == alive.sum()
    if (n, dim, m) == (32, 2, 8):
        assert F.active_counts[0][0] - F.active_counts[0][1] == 841   # 29^2 interiors


def test_iterations_do_not_grow_with_n():
    """Sec. 3: PHIF-PCG iteration counts are essentially independent of N."""
    its = []
    for n in [31, 63, 127]:
        a = gen.grf_coefficient(n, 2, 0.1, 17)
        A, B = fd.cn_matrices(a, 1.0 / (n + 1))
        F = phif.phif_build(A, n, 2, 8, 1e-3)
        u0 = gen.bumps(n, 2, 3, 18)
        _, it, _ = cn.cn_solve(A, B, u0, 1.0 / (n + 1), 2, lambda r: phif.phif_apply(F, r), 1e-12)
        its.append(np.mean(it))
    assert max(its) - min(its) <= 1.5
    assert max(its) <= 8


def test_inverse_error_estimate_against_dense_norm():
    """The power-iteration estimate of ||I - A F^-1||_2 (Sec. 3, Example 1) against the exact
    2-norm from an SVD of the dense I - A F^-1: never above it (every Rayleigh-type ratio of
    E^T E is at most ||E||^2), within 2% of it after enough steps, and 0 at eps = 0 (F = A)."""
    from oracle import estimate
    n, m = 31, 8
    a = gen.iid_loguniform_cells(n, 2, 41)
    A, _ = fd.cn_matrices(a, 0.05)
    x0 = gen.normal_vector(n * n, 42)
    for eps in (1e-2, 1e-4):
        F = phif.phif_build(A, n, 2, m, eps)
        E = np.eye(n * n) - A @ phif.phif_dense_inverse(F)
        exact = np.linalg.norm(E, 2)
        est = estimate.inverse_error_power(A, lambda r: phif.phif_apply(F, r), x0, 200)
        assert est <= exact * (1 + 1e-10), (est, exact)
        assert est >= 0.98 * exact, (est, exact)
        assert exact > 0
    F0 = phif.phif_build(A, n, 2, m, 0.0)
    assert estimate.inverse_error_power(A, lambda r: phif.phif_apply(F0, r), x0, 20) < 1e-12


def test_sequential_id_order_exact_at_eps0_and_close_otherwise():
    """The sequential order of the edge IDs within a level (each from the matrix the earlier
    edges left) against the level-synchronous reading: both exact at eps = 0 (no compression,
    F = A), the same structure of levels, and inverse errors of the same order at eps > 0."""
    import scipy.sparse.linalg as spla
    n, m = 63, 8
    a = gen.iid_loguniform_cells(n, 2, 43)
    A, _ = fd.cn_matrices(a, 0.05)
    r = gen.normal_vector(n * n, 44)
    ref = spla.spsolve(A.tocsc(), r)
    for order in ("level", "sequential"):
        F = phif.phif_build(A, n, 2, m, 0.0, id_order=order)
        assert np.linalg.norm(phif.phif_apply(F, r) - ref) <= 1e-11 * np.linalg.norm(ref)
    Fl = phif.phif_build(A, n, 2, m, 1e-3, id_order="level")
    Fs = phif.phif_build(A, n, 2, m, 1e-3, id_order="sequential")
    assert len(Fl.levels) == len(Fs.levels)
    el = np.linalg.norm(r - A @ phif.phif_apply(Fl, r)) / np.linalg.norm(r)
    es = np.linalg.norm(r - A @ phif.phif_apply(Fs, r)) / np.linalg.norm(r)
    assert 0.1 < es / el < 10, (el, es)


def _skel_kind(F, lev, s):
    """Axes on a separator of level lev for the DOFs of skeletonized group s (3D: 1 face,
    2 edge)."""
    coords = fd.node_grid_coords(F.n, F.dim)
    S = geometry.separators(F.n, F.leaf, lev)
    dof = (s.redund if len(s.redund) else s.skel)[0]
    return int(np.isin(coords[dof], S).sum())


EDGE_CASES = [(7, 4, 0.0), (7, 4, 1e-6), (7, 4, 1e-3), (7, 4, 0.4),
              (8, 4, 0.0), (8, 4, 1e-6), (8, 4, 1e-3), (8, 4, 0.4),
              (12, 3, 1e-3), (12, 3, 0.4)]


@pytest.mark.parametrize("n,m,eps", EDGE_CASES)
def test_edge_skeletonization_block_equals_dense_literal(n, m, eps):
    """3D with the edges skeletonized as well as the faces (Sec. 2.2, 3D paragraph): the block
    oracle against the paper's N x N factor matrices multiplied out, with the same skeleton size
    on every face and edge; eps = 0 gives A^-1.  Only at eps = 0.4 do the edges of these grids
    lose DOFs (see the test below), so that case runs the edge path with compression."""
    A, _ = _problem(n, 3)
    F = phif.phif_build(A, n, 3, m, eps, skel_edges=True)
    D = phif_dense.phif_dense(A.toarray(), n, 3, m, eps, skel_edges=True)
    Fi = phif.phif_dense_inverse(F)
    assert np.linalg.norm(Fi - D.Finv) <= 1e-12 * np.linalg.norm(D.Finv)
    ranks_block = [sorted(len(s.skel) for s in lv.skels) for lv in F.levels]
    ranks_dense = [sorted(k for _, k in r) for r in D.ranks]
    assert ranks_block == ranks_dense
    kinds = [_skel_kind(F, l, s) for l, lv in enumerate(F.levels) for s in lv.skels]
    assert kinds.count(2) > 0 and set(kinds) == {1, 2}
    if eps == 0.0:
        Ainv = np.linalg.inv(A.toarray())
        assert np.linalg.norm(Fi - Ainv) <= 1e-11 * np.linalg.norm(Ainv)
    if eps == 0.4:
        red = sum(len(s.redund) for l, lv in enumerate(F.levels) for s in lv.skels
                  if _skel_kind(F, l, s) == 2)
        assert red > 0
        F0 = phif.phif_build(A, n, 3, m, eps)
        assert F.active_counts[-1][2] < F0.active_counts[-1][2]


@pytest.mark.parametrize("order", ["level", "sequential"])
def test_edges_keep_full_rank_under_stencil_coupling(order):
    """Under the stencil, each DOF of a 3D edge is a direct neighbour of DOFs on the four faces
    around it, which stay active through the level (cell elimination removes only interiors), so
    the coupling block of an edge holds a full-rank part and its ID keeps every column at any
    practical eps: the factor with skeletonized edges is the faces-only factor."""
    n, m = 16, 4
    a = gen.grf_coefficient(n, 3, 0.15, 7)
    A, _ = fd.cn_matrices(a, 0.05)
    r = gen.normal_vector(n ** 3, 8)
    for eps in (1e-3, 1e-2):
        F = phif.phif_build(A, n, 3, m, eps, skel_edges=True, id_order=order)
        F0 = phif.phif_build(A, n, 3, m, eps, id_order=order)
        edges = [s for l, lv in enumerate(F.levels) for s in lv.skels if _skel_kind(F, l, s) == 2]
        assert len(edges) > 0 and all(len(s.redund) == 0 for s in edges)
        assert F.active_counts == F0.active_counts
        assert np.array_equal(phif.phif_apply(F, r), phif.phif_apply(F0, r))
