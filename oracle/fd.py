"""Finite-difference discretisation of the diffusion term (Sec. 2; eq1, eq2).

The paper discretises div(a grad u) with the standard five-point stencil on a uniform grid
(seven-point in 3D) with zero Dirichlet data, giving a sparse symmetric negative definite M.
It does not say how a(x) enters the stencil; this oracle takes each link coefficient as the
arithmetic mean of the cells sharing the link (2 cells in 2D, 4 in 3D), with a given on the
(n+1)^d cells between nodes:

    (M u)_j = h^-2 sum_d [ a_{j+e_d/2} (u_{j+e_d} - u_j) - a_{j-e_d/2} (u_j - u_{j-e_d}) ],

u = 0 on boundary nodes, h = 1/(n+1), nodes j = 1..n per axis, C order with x fastest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def link_coefficients(a_cells: np.ndarray) -> list[np.ndarray]:
    """Per-axis link coefficients from cell values.

    Returns ``[ax, ay(, az)]``; the array for axis d holds the coefficient of the link between
    node j and j + e_d for every interior-or-boundary pair along that axis, i.e. it has n+1
    entries along axis d and n along the others (links touching the Dirichlet boundary
    included).  Array axes follow the node arrays: (y, x) in 2D, (z, y, x) in 3D.
    """
    dim = a_cells.ndim
    n = a_cells.shape[0] - 1
    out = []
    for d in range(dim):           # d = 0 -> x (last array axis), 1 -> y, 2 -> z
        ax_arr = dim - 1 - d       # array axis of this spatial direction
        # The link along direction d between node j and j+e_d lies at fixed node indices in
        # the other directions; the cells sharing it are the 2^(dim-1) cells with cell index
        # j_d along d and {j_o - 1, j_o} (0-based cells) along every other direction o.
        acc = np.zeros([n + 1 if a == ax_arr else n for a in range(dim)])
        others = [a for a in range(dim) if a != ax_arr]
        count = 0
        for mask in range(1 << len(others)):
            sl = [slice(None)] * dim
            sl[ax_arr] = slice(0, n + 1)
            for bit, o in enumerate(others):
                sl[o] = slice(1, n + 1) if (mask >> bit) & 1 else slice(0, n)
            acc = acc + a_cells[tuple(sl)]
            count += 1
        out.append(acc / count)
    return out


def stiffness(a_cells: np.ndarray) -> sp.csr_matrix:
    """The stiffness matrix M of eq2 (symmetric negative definite), assembled link by link."""
    dim = a_cells.ndim
    n = a_cells.shape[0] - 1
    N = n ** dim
    h = 1.0 / (n + 1)
    links = link_coefficients(a_cells)
    idx = np.arange(N).reshape((n,) * dim)
    rows, cols, vals = [], [], []
    diag = np.zeros((n,) * dim)
    for d in range(dim):
        ax_arr = dim - 1 - d
        w = links[d] / h ** 2
        # link k along axis connects node k-1 and k (0-based nodes 0..n-1, boundary at -1, n)
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax_arr] = slice(0, n)        # link to the node below: links 0..n-1
        hi[ax_arr] = slice(1, n + 1)    # link to the node above: links 1..n
        diag -= w[tuple(lo)] + w[tuple(hi)]
        # off-diagonal couplings between node k and k+1 (both interior): links 1..n-1
        mid = [slice(None)] * dim
        mid[ax_arr] = slice(1, n)
        a_sl = [slice(None)] * dim
        b_sl = [slice(None)] * dim
        a_sl[ax_arr] = slice(0, n - 1)
        b_sl[ax_arr] = slice(1, n)
        i0 = idx[tuple(a_sl)].ravel()
        i1 = idx[tuple(b_sl)].ravel()
        wv = w[tuple(mid)].ravel()
        rows += [i0, i1]
        cols += [i1, i0]
        vals += [wv, wv]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return M.tocsr()


def cn_matrices(a_cells: np.ndarray, dt: float) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """A = I - dt/2 M and B = I + dt/2 M of the Crank-Nicolson scheme (eq_CN)."""
    M = stiffness(a_cells)
    I = sp.identity(M.shape[0], format="csr")
    return (I - 0.5 * dt * M).tocsr(), (I + 0.5 * dt * M).tocsr()


def node_grid_coords(n: int, dim: int) -> np.ndarray:
    """(N, dim) array of 1-based node indices (j_x, j_y[, j_z]) in global DOF order."""
    idx = np.indices((n,) * dim).reshape(dim, -1)  # array axes (.., y, x)
    return (idx[::-1].T + 1).astype(np.int64)       # -> columns (x, y, z)
