"""Block PHIF: recursively preconditioned hierarchical interpolative factorization (Sec. 2.2).

Build, for levels l = 0..L-1, the three steps of Sec. 2.2 on the active matrix A_l, then the
root:

  (1) cell elimination (eq2_3, eq3_1): for every cell interior I with boundary B,
      A_II = L L^T, G = L^-1 A_IB, and the Schur complement X_BB = A_BB - G^T G.  Cell
      interiors are disjoint and only couple to their own boundary, so all cells of a level use
      the same A_l and their updates are summed.
  (2) block Jacobi (jacobi-precond, eq3_2): for every edge and corner (3D: face, edge, corner)
      g, A_gg = L_g L_g^T and every coupling becomes L_g^-1 A_gh L_h^-T; the diagonal blocks
      are then the identity (set exactly).
  (3) skeletonization (eq2_4, eq2_5, eq_T, eq2_9, eq3_3) of every edge (3D: face, and with
      skel_edges also every edge, the variant the 3D paragraph of Sec. 2.2 allows): an ID of the
      coupling of the edge to the rest of the active DOFs splits it into redundant I~ and
      skeleton I^ with A_{R,I~} ~= A_{R,I^} T; the residual block is dropped, the redundant DOFs
      are eliminated with L_s = chol(I + T^T T) and the skeleton diagonal block becomes
      X = I - T (I + T^T T)^-1 T^T.  All edges of a level take their ID from the matrix after
      step (2) (level-synchronous); the paper does not fix an order.
  root: the remaining active DOFs, A_root = L_r L_r^T (eq3_4).

Apply z = F^-1 r (eqAinv): F^-1 = R_0 ... R_{L-1} A_L^-1 R_{L-1}^T ... R_0^T with
R_l = E_l C_l K_l, i.e. a forward sweep of E_l^T, C_l^T, K_l^T for l = 0..L-1, the root solve,
and a backward sweep of K_l, C_l, E_l for l = L-1..0.  Per block:

  E^T (cell):  w = L^-1 y_I;  y_B -= G^T w;  y_I = w
  C^T (group): y_g = L_g^-1 y_g
  K^T (edge):  y_I~ -= T^T y_I^;  y_I~ = L_s^-1 y_I~;  y_I^ += T L_s^-T y_I~
  root:        y_r = L_r^-T L_r^-1 y_r
  K (edge):    x_I~ = L_s^-T (x_I~ + L_s^-1 T^T x_I^);  x_I^ -= T x_I~
  C (group):   x_g = L_g^-T x_g
  E (cell):    x_I = L^-T (x_I - G x_B)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fd import node_grid_coords
from .geometry import (cell_closure_keys, group_active, key_kind, num_levels, separators)
from .interp import interp_decomp


class NotSPD(ValueError):
    pass


@dataclass
class CellBlock:
    I: np.ndarray        # interior DOFs (global ids)
    B: np.ndarray        # boundary DOFs (global ids)
    L: np.ndarray        # chol(A_II), lower
    G: np.ndarray        # L^-1 A_IB


@dataclass
class GroupBlock:
    idx: np.ndarray      # DOFs of the edge / corner (3D: face / edge / corner)
    L: np.ndarray        # chol(A_gg), lower


@dataclass
class SkelBlock:
    redund: np.ndarray   # I~ (global ids)
    skel: np.ndarray     # I^ (global ids)
    T: np.ndarray        # |I^| x |I~|
    Ls: np.ndarray       # chol(I + T^T T), lower


@dataclass
class Level:
    cells: list = field(default_factory=list)
    groups: list = field(default_factory=list)
    skels: list = field(default_factory=list)


@dataclass
class Factor:
    N: int
    dim: int
    n: int
    leaf: int
    eps: float
    levels: list
    root_idx: np.ndarray
    root_L: np.ndarray
    active_counts: list  # per level: (active before step 1, after step 1, after step 3)


def _chol(Amat: np.ndarray) -> np.ndarray:
    try:
        return sla.cholesky(Amat, lower=True)
    except np.linalg.LinAlgError as exc:  # pragma: no cover - exercised through NotSPD
        raise NotSPD(str(exc)) from exc


def _dense(Acur: sp.csr_matrix, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """The dense block Acur[rows, cols].  The nonzeros of the selected rows are matched to the
    requested columns by binary search over the sorted column list, so the cost follows the
    nonzeros of those rows rather than the order of the matrix."""
    out = np.zeros((len(rows), len(cols)))
    if len(rows) == 0 or len(cols) == 0:
        return out
    rows = np.asarray(rows)
    start, stop = Acur.indptr[rows], Acur.indptr[rows + 1]
    cnt = stop - start
    row = np.repeat(np.arange(len(rows)), cnt)               # output row of each nonzero
    k = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt) + np.repeat(start, cnt)
    col, val = Acur.indices[k], Acur.data[k]
    order = np.argsort(cols, kind="stable")
    scol = np.asarray(cols)[order]
    pos = np.minimum(np.searchsorted(scol, col), len(scol) - 1)
    hit = scol[pos] == col
    out[row[hit], order[pos[hit]]] = val[hit]
    return out


def _keep(Acur: sp.csr_matrix, keep: np.ndarray) -> sp.csr_matrix:
    D = sp.diags(keep.astype(np.float64))
    return (D @ Acur @ D).tocsr()


def skel_kinds(dim: int, skel_edges: bool) -> tuple:
    """Group kinds (axes on a separator) skeletonized in step (3): 2D edges; 3D faces, and 3D
    edges too when skel_edges is set (Sec. 2.2, 3D paragraph).  2D edges are always
    skeletonized, so the flag changes nothing there."""
    return (1, 2) if dim == 3 and skel_edges else (1,)


def phif_build(A: sp.spmatrix, n: int, dim: int, leaf: int, eps: float,
               id_order: str = "level", skel_edges: bool = False) -> Factor:
    """Build the PHIF factor of the SPD matrix A on the n^dim grid (Sec. 2.2).

    skel_edges: in 3D, skeletonize the edges of every level as well as its faces (kinds from
    skel_kinds); faces come first in the sequential order.

    id_order: how the edges of a level meet each other's eliminations in step (3) (eq3_3 takes
    the product over the edges but not their order).  "level": every ID sees the matrix after
    step (2) of the level (the reading used throughout).  "sequential": the edges are
    skeletonized one after another in key order, each ID from the matrix the earlier ones left.
    An earlier edge's skeletonization drops its (R, I~) residual and eliminates I~; the
    couplings of its skeleton are unchanged, so the only difference a later edge sees is that
    the rows of the earlier edges' redundant DOFs are gone from its block."""
    if id_order not in ("level", "sequential"):
        raise ValueError(f"unknown id_order {id_order!r}")
    A = sp.csr_matrix(A, dtype=np.float64)
    N = A.shape[0]
    assert N == n ** dim
    coords = node_grid_coords(n, dim)
    L = num_levels(n, leaf)
    active = np.ones(N, dtype=bool)
    Acur = A.copy()
    levels = []
    counts = []
    for lev in range(L):
        S = separators(n, leaf, lev)
        groups = group_active(np.flatnonzero(active), coords, S)
        n_before = int(active.sum())
        level = Level()

        # (1) cell elimination
        cell_keys = [k for k in groups if key_kind(k) == 0]
        rows, cols, vals = [], [], []
        elim = np.zeros(N, dtype=bool)
        for ck in cell_keys:
            I = groups[ck]
            bkeys = [k for k in cell_closure_keys(ck, S) if k in groups]
            B = np.concatenate([groups[k] for k in bkeys]) if bkeys else np.zeros(0, np.int64)
            Lc = _chol(_dense(Acur, I, I))
            G = sla.solve_triangular(Lc, _dense(Acur, I, B), lower=True)
            X = G.T @ G
            rr, cc = np.meshgrid(B, B, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(-X.ravel())
            level.cells.append(CellBlock(I, B, Lc, G))
            elim[I] = True
        active &= ~elim
        Acur = _keep(Acur, active)
        if rows:
            Acur = (Acur + sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                                  np.concatenate(cols))),
                                         shape=(N, N))).tocsr()
        n_after_elim = int(active.sum())

        # (2) block Jacobi on every remaining group (edges and corners; 3D faces too)
        sep_keys = [k for k in groups if key_kind(k) > 0]
        prow, pcol, pval = [], [], []
        drow, dcol = [], []
        for sk in sep_keys:
            g = groups[sk]
            Lg = _chol(_dense(Acur, g, g))
            Linv = sla.solve_triangular(Lg, np.eye(len(g)), lower=True)
            rr, cc = np.meshgrid(g, g, indexing="ij")
            prow.append(rr.ravel())
            pcol.append(cc.ravel())
            pval.append(Linv.ravel())
            drow.append(rr.ravel())
            dcol.append(cc.ravel())
            level.groups.append(GroupBlock(g, Lg))
        if sep_keys:
            P = sp.coo_matrix((np.concatenate(pval), (np.concatenate(prow),
                                                      np.concatenate(pcol))), shape=(N, N)).tocsr()
            Acur = (P @ Acur @ P.T).tocsr()
            # the diagonal blocks are the identity by construction: store them exactly
            dr, dc = np.concatenate(drow), np.concatenate(dcol)
            old = np.asarray(Acur[dr, dc]).ravel()
            Acur = (Acur + sp.coo_matrix(((dr == dc).astype(float) - old, (dr, dc)),
                                         shape=(N, N))).tocsr()

        # (3) skeletonization of every edge (3D: face, and edge with skel_edges), IDs from the
        # matrix after step (2)
        skel_keys = [k for kd in skel_kinds(dim, skel_edges) for k in sep_keys
                     if key_kind(k) == kd]
        red_all = np.zeros(N, dtype=bool)
        xr, xc, xv = [], [], []
        Acsc = Acur.tocsc()
        for sk in skel_keys:
            g = groups[sk]
            col = Acsc[:, g]
            nz = np.unique(col.nonzero()[0])
            R = np.setdiff1d(nz, g)
            if id_order == "sequential":
                R = R[~red_all[R]]
            Mblk = _dense(Acur, R, g)
            sk_pos, rd_pos, T = interp_decomp(Mblk, eps)
            nr = len(rd_pos)
            Smat = np.eye(nr) + T.T @ T
            Ls = _chol(Smat)
            X = np.eye(len(sk_pos)) - T @ sla.cho_solve((Ls, True), T.T) if nr else \
                np.eye(len(sk_pos))
            skel = g[sk_pos]
            red = g[rd_pos]
            level.skels.append(SkelBlock(red, skel, T, Ls))
            red_all[red] = True
            rr, cc = np.meshgrid(skel, skel, indexing="ij")
            xr.append(rr.ravel())
            xc.append(cc.ravel())
            xv.append((X - np.eye(len(skel))).ravel())
        active &= ~red_all
        Acur = _keep(Acur, active)
        if xr:
            Acur = (Acur + sp.coo_matrix((np.concatenate(xv), (np.concatenate(xr),
                                                                np.concatenate(xc))),
                                         shape=(N, N))).tocsr()
        counts.append((n_before, n_after_elim, int(active.sum())))
        levels.append(level)

    ridx = np.flatnonzero(active)
    Lr = _chol(_dense(Acur, ridx, ridx)) if len(ridx) else np.zeros((0, 0))
    return Factor(N, dim, n, leaf, eps, levels, ridx, Lr, counts)


def phif_apply(F: Factor, r: np.ndarray) -> np.ndarray:
    """z = F^-1 r by eqAinv: forward sweep, root solve, backward sweep.

    ``r`` is a vector of length N or an (N, k) block of k right-hand sides."""
    y = np.array(r, dtype=np.float64)
    y = y.reshape(F.N, -1).copy() if y.ndim > 1 else y.ravel().copy()
    for level in F.levels:
        for c in level.cells:                       # E_l^T
            w = sla.solve_triangular(c.L, y[c.I], lower=True)
            y[c.B] -= c.G.T @ w
            y[c.I] = w
        for g in level.groups:                      # C_l^T
            y[g.idx] = sla.solve_triangular(g.L, y[g.idx], lower=True)
        for s in level.skels:                       # K_l^T
            t = y[s.redund] - s.T.T @ y[s.skel]
            t = sla.solve_triangular(s.Ls, t, lower=True)
            y[s.skel] += s.T @ sla.solve_triangular(s.Ls.T, t, lower=False)
            y[s.redund] = t
    if len(F.root_idx):                              # A_L^-1
        y[F.root_idx] = sla.cho_solve((F.root_L, True), y[F.root_idx])
    for level in reversed(F.levels):
        for s in level.skels:                       # K_l
            t = y[s.redund] + sla.solve_triangular(s.Ls, s.T.T @ y[s.skel], lower=True)
            t = sla.solve_triangular(s.Ls.T, t, lower=False)
            y[s.skel] -= s.T @ t
            y[s.redund] = t
        for g in level.groups:                      # C_l
            y[g.idx] = sla.solve_triangular(g.L.T, y[g.idx], lower=False)
        for c in level.cells:                       # E_l
            y[c.I] = sla.solve_triangular(c.L.T, y[c.I] - c.G @ y[c.B], lower=False)
    return y


def phif_dense_inverse(F: Factor) -> np.ndarray:
    """F^-1 as a dense matrix, applied to the identity (tiny grids only)."""
    return phif_apply(F, np.eye(F.N))
