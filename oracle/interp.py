"""Interpolative decomposition by column-pivoted QR (Sec. 2.2 step 3, eq2_5).

The paper approximates the redundant columns of the edge coupling block by its skeleton
columns, A_{R,I~} ~= A_{R,I^} T, to relative precision eps.  It names the ID but not the
algorithm; this oracle uses the standard construction: Householder QR with column pivoting,
A P = Q R (LAPACK dgeqp3 through SciPy), numerical rank

    k = min{ j : |R_jj| <= eps |R_11| }   (0-based; |R_jj| is non-increasing under pivoting,
                                           so this equals the count of |R_jj| > eps |R_11|
                                           in exact arithmetic),

skeletons = the first k pivots, redundant = the rest, T = R11^-1 R12 (k x (n - k)).
A zero block gives k = 0; eps = 0 keeps every column with a non-zero pivot.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def interp_decomp(Amat: np.ndarray, eps: float):
    """Return (skel, redund, T) as positions into the columns of ``Amat``."""
    nrow, ncol = Amat.shape
    if ncol == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 0))
    if nrow == 0 or not np.any(Amat):
        return np.zeros(0, np.int64), np.arange(ncol), np.zeros((0, ncol))
    R, P = sla.qr(Amat, mode="r", pivoting=True)
    d = np.abs(np.diag(R))
    k = len(d)
    for j in range(len(d)):
        if d[j] <= eps * d[0]:
            k = j
            break
    R11 = R[:k, :k]
    R12 = R[:k, k:]
    T = sla.solve_triangular(R11, R12, lower=False) if k > 0 else np.zeros((0, ncol))
    return P[:k].astype(np.int64), P[k:].astype(np.int64), T
