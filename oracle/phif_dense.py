"""Dense-literal PHIF for tiny grids: the N x N factor matrices of Sec. 2.2, as written.

Every factor is formed as a full N x N matrix exactly in the block layout the paper prints
(stored sparse only to keep the products cheap) and multiplied into the dense active matrix:

  step (1)  E_{I} of eq2_3: identity except rows I, with L_I^-T on (I, I) and
            -A_II^-1 A_BI^T on (I, B); E_l = prod_i E_{I_i} (eq3_1); A <- E_l^T A E_l.
  step (2)  C_{I} of jacobi-precond: identity except L_I^-T on (I, I); C_l = prod_i C_{I_i}
            (eq3_2); A <- C_l^T A C_l.
  step (3)  for each edge (3D: face; with skel_edges faces, then edges) with the ID taken from
            A after step (2): Z_I of eq_T
            (-T in the (I^, I~) position), A <- Z^T A Z, the O(eps) coupling between I~ and the
            rest is dropped (the approximation sign of eq_T), then E_{I~} of eq2_9 (L_s^-T on
            (I~, I~), (I + T^T T)^-1 T^T on (I~, I^)), A <- E^T A E; K_l = prod_i Z_i E_i (eq3_3).

R_l = E_l C_l K_l; A_L is the identity except on the root block (eq3_4);
F^-1 = R_0 ... R_{L-1} A_L^-1 R_{L-1}^T ... R_0^T (eqAinv) and F = R_0^-T ... A_L ... R_0^-1
(eqA) are returned as dense matrices, together with the active matrices after every step so that
the structural claims of Sec. 2.2 can be checked.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fd import node_grid_coords
from .geometry import cell_closure_keys, group_active, key_kind, num_levels, separators
from .interp import interp_decomp


@dataclass
class DenseResult:
    Finv: np.ndarray
    F: np.ndarray
    AL: np.ndarray
    root_idx: np.ndarray
    Rs: list
    snapshots: list = field(default_factory=list)  # (level, step, A, info)
    ranks: list = field(default_factory=list)      # per level: list of (edge dofs, k)


def _put(Mat: sp.lil_matrix, rows, cols, block):
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            Mat[i, j] = block[a, b]


def phif_dense(A: np.ndarray, n: int, dim: int, leaf: int, eps: float,
               skel_edges: bool = False) -> DenseResult:
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[0]
    coords = node_grid_coords(n, dim)
    L = num_levels(n, leaf)
    active = np.ones(N, dtype=bool)
    Acur = A.copy()
    Rs = []
    snaps = []
    ranks = []
    for lev in range(L):
        S = separators(n, leaf, lev)
        groups = group_active(np.flatnonzero(active), coords, S)

        # step (1): cell elimination, E_l = prod_i E_{I_i}
        El = sp.identity(N, format="csr")
        cells = [k for k in groups if key_kind(k) == 0]
        for ck in cells:
            I = groups[ck]
            bkeys = [k for k in cell_closure_keys(ck, S) if k in groups]
            B = np.concatenate([groups[k] for k in bkeys])
            AII = Acur[np.ix_(I, I)]
            ABI = Acur[np.ix_(B, I)]
            LI = sla.cholesky(AII, lower=True)
            EI = sp.lil_matrix(sp.identity(N))
            _put(EI, I, I, sla.inv(LI).T)
            _put(EI, I, B, -np.linalg.solve(AII, ABI.T))
            El = El @ EI.tocsr()
        Acur = np.asarray(El.T @ Acur @ El)
        for ck in cells:
            active[groups[ck]] = False
        snaps.append((lev, 1, Acur.copy(), {"cells": [groups[k] for k in cells]}))

        # step (2): block Jacobi on edges and corners (3D: faces, edges, corners)
        seps = [k for k in groups if key_kind(k) > 0]
        Cl = sp.lil_matrix(sp.identity(N))
        for sk in seps:
            g = groups[sk]
            Lg = sla.cholesky(Acur[np.ix_(g, g)], lower=True)
            _put(Cl, g, g, sla.inv(Lg).T)
        Cl = Cl.tocsr()
        Acur = np.asarray(Cl.T @ Acur @ Cl)
        snaps.append((lev, 2, Acur.copy(), {"groups": [groups[k] for k in seps]}))

        # step (3): skeletonize edges (3D: faces, then edges with skel_edges); every ID from the
        # matrix after step (2)
        kinds = (1, 2) if dim == 3 and skel_edges else (1,)
        edges = [k for kd in kinds for k in seps if key_kind(k) == kd]
        act_ids = np.flatnonzero(active)
        ids = []
        for ek in edges:
            g = groups[ek]
            R = np.setdiff1d(act_ids, g)
            sk_pos, rd_pos, T = interp_decomp(Acur[np.ix_(R, g)], eps)
            ids.append((g, g[sk_pos], g[rd_pos], T))
        ranks.append([(g, len(sk)) for g, sk, _, _ in ids])
        Kl = sp.identity(N, format="csr")
        residuals = []
        for g, skel, red, T in ids:
            Z = sp.lil_matrix(sp.identity(N))
            _put(Z, skel, red, -T)
            Z = Z.tocsr()
            Acur = np.asarray(Z.T @ Acur @ Z)
            rest = np.setdiff1d(np.arange(N), g)
            residuals.append(np.linalg.norm(Acur[np.ix_(rest, red)], 2) if len(red) else 0.0)
            Acur[np.ix_(rest, red)] = 0.0
            Acur[np.ix_(red, rest)] = 0.0
            Smat = np.eye(len(red)) + T.T @ T
            Ls = sla.cholesky(Smat, lower=True)
            Es = sp.lil_matrix(sp.identity(N))
            _put(Es, red, red, sla.inv(Ls).T)
            _put(Es, red, skel, np.linalg.solve(Smat, T.T))
            Es = Es.tocsr()
            Acur = np.asarray(Es.T @ Acur @ Es)
            Kl = Kl @ Z @ Es
            active[red] = False
        snaps.append((lev, 3, Acur.copy(), {"edges": ids, "residuals": residuals}))
        Rs.append((El @ Cl @ Kl).toarray())

    ridx = np.flatnonzero(active)
    AL = np.eye(N)
    AL[np.ix_(ridx, ridx)] = Acur[np.ix_(ridx, ridx)]
    ALinv = np.eye(N)
    if len(ridx):
        ALinv[np.ix_(ridx, ridx)] = np.linalg.inv(Acur[np.ix_(ridx, ridx)])
    Rprod = np.eye(N)
    for R in Rs:
        Rprod = Rprod @ R
    Finv = Rprod @ ALinv @ Rprod.T
    Rinv = np.linalg.inv(Rprod)
    F = Rinv.T @ AL @ Rinv
    return DenseResult(Finv, F, Acur, ridx, Rs, snaps, ranks)
