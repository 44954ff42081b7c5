"""Estimate of the inverse error ||I - A F^-1||_2 (Sec. 3, Example 1).

The paper judges how close the factor is to A^-1 by estimating ||I - A F^-1||_2 with a
randomized power iteration (about 7.9e-6 at eps = 1e-6 on the 4095^2 grid).  With
E = I - A F^-1 and A, F^-1 symmetric, E^T = I - F^-1 A; the power iteration on E^T E from a
start vector x0 gives lambda_k = ||E^T E x_k|| with x_{k+1} = E^T E x_k / lambda_k, and
sqrt(lambda_k) increases towards the largest singular value of E.  For any unit x,
||E^T E x|| <= ||E||^2, so every estimate is a lower bound (up to rounding).
"""
from __future__ import annotations

import numpy as np


def inverse_error_power(A, apply_inv, x0: np.ndarray, iters: int) -> float:
    """sqrt(lambda) after `iters` steps of the power iteration on E^T E (E = I - A F^-1),
    started from x0 / ||x0||; apply_inv(r) returns F^-1 r."""
    x = np.asarray(x0, dtype=np.float64).ravel()
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = x - A @ apply_inv(x)          # E x
        z = y - apply_inv(A @ y)          # E^T E x
        lam = float(np.linalg.norm(z))
        if lam == 0.0:
            return 0.0
        x = z / lam
    return float(np.sqrt(lam))
