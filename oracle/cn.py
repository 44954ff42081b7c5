"""Crank-Nicolson time stepping with explicit reaction and PCG (Sec. 2.1, Sec. 2.3).

Each step forms g = (I + dt/2 M) u^k + dt r(u^k) (eq_CN with the reaction treated explicitly)
and solves (I - dt/2 M) u^{k+1} = g by preconditioned conjugate gradient (Algorithm 1).

PCG details the paper leaves open, as read here: standard PCG with x0 = 0, beta = rho_new/rho;
stop as soon as the recurrence residual satisfies ||r_i||_2 <= rtol ||g||_2; the iteration
count n_i is the number of products of A with a search direction; g = 0 gives u = 0 and n_i = 0.
Optionally (warm start, off by default) x0 = u^k, the state before the step: r_0 = g - A x0,
the same test against rtol ||g||_2 (already met at r_0: n_i = 0, u^{k+1} = u^k).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def reaction(u: np.ndarray, kind: int, k1: float, k2: float) -> np.ndarray:
    """Pointwise reaction r(u): kind 0 -> 0, kind 1 -> k1 u (1 - u/k2) (logistic, eq_nr)."""
    if kind == 0:
        return np.zeros_like(u)
    if kind == 1:
        return k1 * u * (1.0 - u / k2)
    raise ValueError(f"unknown reaction kind {kind}")


def cn_rhs(B, u: np.ndarray, dt: float, react=(0, 0.0, 0.0)) -> np.ndarray:
    """g = (I + dt/2 M) u + dt r(u)  (eq_CN, explicit reaction as in Sec. 2.1)."""
    return B @ u + dt * reaction(u, *react)


class NoConvergence(RuntimeError):
    pass


@dataclass
class PcgResult:
    x: np.ndarray
    iters: int
    relres: float      # recurrence residual ||r|| / ||g|| at exit
    converged: bool


def pcg(A, b: np.ndarray, precond, rtol: float, maxit: int = 500, x0=None) -> PcgResult:
    """Preconditioned CG for SPD A (the pcg(A, b, P) of Algorithm 1).

    ``A`` is anything supporting ``A @ x``; ``precond(r)`` returns P r.  ``x0``: the initial
    guess (None: 0); with one, r_0 = b - A x0 and PCG stops at once if ||r_0|| <= rtol ||b||.
    """
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if nb == 0.0:
        return PcgResult(x, 0, 0.0, True)
    if x0 is None:
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64).copy()
        r = b - A @ x
        nr0 = float(np.linalg.norm(r))
        if not np.isfinite(nr0):
            return PcgResult(x, 0, nr0 / nb, False)
        if nr0 <= rtol * nb:
            return PcgResult(x, 0, nr0 / nb, True)
    z = precond(r)
    p = z.copy()
    rho = float(r @ z)
    nr = nb
    for i in range(1, maxit + 1):
        q = A @ p
        alpha = rho / float(p @ q)
        x += alpha * p
        r -= alpha * q
        nr = float(np.linalg.norm(r))
        if not np.isfinite(nr):
            return PcgResult(x, i, nr / nb, False)
        if nr <= rtol * nb:
            return PcgResult(x, i, nr / nb, True)
        z = precond(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return PcgResult(x, maxit, nr / nb, False)


def cn_solve(A, B, u0: np.ndarray, dt: float, steps: int, precond, rtol: float,
             react=(0, 0.0, 0.0), maxit: int = 500, warm_start: bool = False):
    """Algorithm 1: for k = 1..steps, g = B u^{k-1} + dt r^{k-1}; u^k = pcg(A, g, F^-1)
    (with warm_start, from the initial guess u^{k-1}).

    Returns (u_steps, iters, relres) with u_steps[k] = u^k (u_steps[0] = u0).
    """
    u = u0.astype(np.float64).ravel().copy()
    us = [u.copy()]
    iters, rel = [], []
    for _ in range(steps):
        g = cn_rhs(B, u, dt, react)
        res = pcg(A, g, precond, rtol, maxit, x0=u if warm_start else None)
        if not res.converged:
            raise NoConvergence(f"PCG did not converge in {maxit} iterations")
        u = res.x
        us.append(u.copy())
        iters.append(res.iters)
        rel.append(res.relres)
    return us, iters, rel


def cn_solve_direct(B, u0: np.ndarray, dt: float, steps: int, solve, react=(0, 0.0, 0.0)):
    """The factor used as the solver, without CG (Sec. 3, the remark on eps = 1e-6): for
    k = 1..steps, g = B u^{k-1} + dt r(u^{k-1}) and u^k = solve(g) with solve = F^-1.

    Returns u_steps with u_steps[k] = u^k (u_steps[0] = u0).
    """
    u = u0.astype(np.float64).ravel().copy()
    us = [u.copy()]
    for _ in range(steps):
        u = solve(cn_rhs(B, u, dt, react))
        us.append(u.copy())
    return us


def cn_solve_varying(a_at, n: int, dim: int, leaf: int, eps: float, dt: float, u0: np.ndarray,
                     steps: int, refactor_every: int, rtol: float, react=(0, 0.0, 0.0),
                     maxit: int = 500):
    """A time-dependent coefficient a(x, t) (Sec. 4): the factor is rebuilt once every
    `refactor_every` steps and reused in between.

    Read here: step k (from t_k = k dt to t_k + dt) takes the coefficient at the midpoint,
    a(., t_k + dt/2), on both sides of eq_CN, which keeps the scheme second order in time; the
    factor is built from that step's coefficient at k = 0, K, 2K, ... (K = refactor_every) and
    preconditions PCG (Algorithm 1) for the K steps that follow.

    Returns (u_steps, iters): u_steps[k] = u^k (u_steps[0] = u0), iters[k-1] = n_i of step k.
    """
    from oracle import fd, phif
    u = u0.astype(np.float64).ravel().copy()
    us = [u.copy()]
    iters = []
    F = None
    for k in range(steps):
        A, B = fd.cn_matrices(a_at((k + 0.5) * dt), dt)
        if k % refactor_every == 0:
            F = phif.phif_build(A, n, dim, leaf, eps)
        res = pcg(A, cn_rhs(B, u, dt, react), lambda r: phif.phif_apply(F, r), rtol, maxit)
        if not res.converged:
            raise NoConvergence(f"PCG did not converge in {maxit} iterations")
        u = res.x
        us.append(u.copy())
        iters.append(res.iters)
    return us, iters
