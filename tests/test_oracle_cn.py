"""Pins of the oracle's Crank-Nicolson + PCG (eq_CN, Algorithm 1)."""
import json
import os

import numpy as np
import scipy.sparse.linalg as spla

from oracle import cn, fd, phif
from workloads import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _direct(A, B, u0, dt, steps, react):
    lu = spla.splu(A.tocsc())
    u = u0.ravel().copy()
    for _ in range(steps):
        u = lu.solve(cn.cn_rhs(B, u, dt, react))
    return u


def test_cn_sine_mode_closed_form():
    """Constant a, u0 = v11: u^k = G^k v11 (closed form in tests/golden)."""
    g = json.load(open(os.path.join(GOLD, "cn_sine_mode_32.json")))
    w = gen.workload("heat2d-32")
    A, B = fd.cn_matrices(w.a_cells, w.dt)
    F = phif.phif_build(A, w.n, 2, 8, w.eps)
    us, iters, rel = cn.cn_solve(A, B, w.u0, w.dt, g["steps"], lambda r: phif.phif_apply(F, r),
                                 1e-12)
    v = w.u0.ravel()
    for k in range(g["steps"] + 1):
        assert np.allclose(us[k], g["G"] ** k * v, rtol=0, atol=1e-11)
    assert np.isclose(us[-1].max(), g["max_u10"], rtol=1e-10)
    assert max(iters) <= 3


def test_cn_matches_sparse_direct_solve_with_reaction():
    n = 24
    a = gen.grf_coefficient(n, 2, 0.1, 11)
    u0 = gen.bumps(n, 2, 4, 12)
    dt = 1e-2
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, 2, 4, 1e-4)
    react = (1, 1.0, 1.0)
    us, iters, _ = cn.cn_solve(A, B, u0, dt, 5, lambda r: phif.phif_apply(F, r), 1e-12, react)
    ud = _direct(A, B, u0, dt, 5, react)
    assert np.linalg.norm(us[-1] - ud) <= 1e-10 * np.linalg.norm(ud)


def test_reaction_logistic_fixed_points_slope_and_peak():
    """r(u) = k1 u (1 - u/k2) (Sec. 3, Example 2) is fixed by facts of the logistic law rather
    than by its formula: it vanishes at the two equilibria u = 0 and u = k2, grows at rate k1
    near 0, is a quadratic (its second difference is the constant -2 k1 / k2 h^2), peaks at
    u = k2/2 with value k1 k2 / 4, and is negative beyond k2 and below 0.  k1, k2 are chosen
    distinct from each other and from 1 so that a swapped or dropped parameter fails."""
    k1, k2 = 3.0, 5.0
    r = lambda u: cn.reaction(np.asarray(u, dtype=float), 1, k1, k2)  # noqa: E731
    assert np.array_equal(r([0.0, k2]), [0.0, 0.0])
    h = 1e-3   # the central difference of a quadratic is exact up to rounding
    assert abs((r([h])[0] - r([-h])[0]) / (2 * h) - k1) < 1e-9
    u = np.linspace(-2.0, 8.0, 41)
    d2 = (r(u + h) - 2 * r(u) + r(u - h)) / h ** 2
    assert np.allclose(d2, -2 * k1 / k2, rtol=0, atol=1e-4)
    assert r([k2 / 2])[0] == k1 * k2 / 4
    grid = np.linspace(-1.0, 6.0, 7001)
    assert np.isclose(grid[np.argmax(r(grid))], k2 / 2)
    assert np.all(r([-0.5, k2 + 0.5]) < 0) and np.all(r([0.5, k2 - 0.5]) > 0)
    # the logistic workloads take k1 = k2 = 1: r(u) = u (1 - u), zero at 0 and 1, peak 1/4
    r1 = cn.reaction(np.array([0.0, 0.5, 1.0]), 1, 1.0, 1.0)
    assert np.array_equal(r1, [0.0, 0.25, 0.0])
    assert not cn.reaction(u, 0, k1, k2).any()


def test_reaction_enters_the_step_explicitly():
    """With the reaction explicit (Sec. 2.1), one CN step from a spatially constant state on
    a grid with a = 0 (no diffusion) is the forward-Euler step of the logistic ODE: the right
    side is u + dt r(u) and A = I.  Checked against the ODE's Euler step written out."""
    n, dt = 6, 0.05
    A, B = fd.cn_matrices(np.zeros((n + 1, n + 1)), dt)
    assert abs(A - _eye(n * n)).max() == 0
    u0 = np.full(n * n, 0.3)
    g = cn.cn_rhs(B, u0, dt, (1, 2.0, 4.0))
    assert np.allclose(g, 0.3 + dt * 2.0 * 0.3 * (1 - 0.3 / 4.0), rtol=0, atol=1e-15)


def _eye(N):
    import scipy.sparse as sp
    return sp.identity(N, format="csr")


def test_pcg_exact_preconditioner_one_iteration_and_zero_rhs():
    n = 15
    a = gen.iid_loguniform_cells(n, 2, 4)
    A, _ = fd.cn_matrices(a, 0.1)
    F = phif.phif_build(A, n, 2, 4, 0.0)     # eps = 0: no compression, F = A
    b = np.random.default_rng(0).normal(size=n * n)
    res = cn.pcg(A, b, lambda r: phif.phif_apply(F, r), 1e-12)
    assert res.converged and res.iters == 1
    res0 = cn.pcg(A, np.zeros(n * n), lambda r: phif.phif_apply(F, r), 1e-12)
    assert res0.iters == 0 and not res0.x.any()


def test_pcg_initial_guess_exact_preconditioner_and_exact_guess():
    """Warm start (x0 given): with F = A (eps = 0) one iteration lands on A^-1 b from any x0,
    which fixes r0 = b - A x0 (a wrong sign or a missing product misses A^-1 b); the exact
    solution as x0 takes no iteration; b = 0 gives x = 0 whatever x0."""
    n = 15
    a = gen.iid_loguniform_cells(n, 2, 4)
    A, _ = fd.cn_matrices(a, 0.1)
    F = phif.phif_build(A, n, 2, 4, 0.0)
    rng = np.random.default_rng(1)
    b = rng.normal(size=n * n)
    xs = spla.spsolve(A.tocsc(), b)
    x0 = rng.normal(size=n * n)
    res = cn.pcg(A, b, lambda r: phif.phif_apply(F, r), 1e-12, x0=x0)
    assert res.converged and res.iters == 1
    assert np.abs(res.x - xs).max() <= 1e-10 * np.abs(xs).max()
    res = cn.pcg(A, b, lambda r: phif.phif_apply(F, r), 1e-12, x0=xs)
    assert res.converged and res.iters == 0 and np.array_equal(res.x, xs)
    res = cn.pcg(A, np.zeros(n * n), lambda r: phif.phif_apply(F, r), 1e-12, x0=x0)
    assert res.converged and res.iters == 0 and not res.x.any()


def test_warm_started_steps_within_the_tolerance_of_direct_steps():
    """x0 = u^k: every step's solution is within rtol ||g|| of the exact step solution
    (A = I - dt/2 M >= I, so ||A^-1|| <= 1), as it is from x0 = 0."""
    n, dt, steps, rtol = 31, 0.05, 3, 1e-8
    a = gen.grf_coefficient(n, 2, 0.15, 12)
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, 2, 8, 1e-3)
    u0 = gen.bumps(n, 2, 3, 13)
    react = (1, 1.0, 1.0)
    us, its, _ = cn.cn_solve(A, B, u0, dt, steps, lambda r: phif.phif_apply(F, r), rtol, react,
                             warm_start=True)
    lu = spla.splu(A.tocsc())
    for k in range(steps):
        g = cn.cn_rhs(B, us[k], dt, react)
        exact = lu.solve(g)
        assert np.linalg.norm(us[k + 1] - exact) <= 1.01 * rtol * np.linalg.norm(g)
    assert min(its) >= 1


def test_pcg_unpreconditioned_matches_textbook_cg_solution():
    n = 10
    A, _ = fd.cn_matrices(np.ones((n + 1, n + 1)), 0.01)
    b = np.arange(n * n, dtype=float)
    res = cn.pcg(A, b, lambda r: r, 1e-13, maxit=1000)
    assert np.allclose(res.x, spla.spsolve(A.tocsc(), b), rtol=1e-11)
    # CG in exact arithmetic terminates in at most as many steps as distinct eigenvalues
    assert res.iters <= n * n


def test_second_order_in_space_and_time():
    """Halving h and dt together divides the error of u(T) by about 4 (a = 1, exact PDE
    solution e^{-2 pi^2 t} sin(pi x) sin(pi y)); second order as stated in Sec. 2.1."""
    def err(n):
        h = 1.0 / (n + 1)
        dt = h
        T = 0.05
        steps = int(round(T / dt))
        dt = T / steps
        A, B = fd.cn_matrices(np.ones((n + 1, n + 1)), dt)
        u0 = gen.sine_mode(n, 2)
        ud = _direct(A, B, u0, dt, steps, (0, 0, 0))
        exact = np.exp(-2 * np.pi ** 2 * T) * u0.ravel()
        return np.abs(ud - exact).max()
    e1, e2 = err(15), err(31)
    assert 3.0 < e1 / e2 < 5.0


def test_direct_steps_with_exact_factor_are_exact_cn_steps():
    """eps = 0 makes the factor exact (no skeleton is dropped), so F^-1 g is the sparse direct
    solve of each CN step."""
    n = 20
    a = gen.grf_coefficient(n, 2, 0.1, 31)
    u0 = gen.bumps(n, 2, 3, 32)
    dt = 2e-2
    A, B = fd.cn_matrices(a, dt)
    F = phif.phif_build(A, n, 2, 4, 0.0)
    react = (1, 1.0, 2.0)
    us = cn.cn_solve_direct(B, u0, dt, 3, lambda g: phif.phif_apply(F, g), react)
    assert len(us) == 4 and np.array_equal(us[0], u0.ravel())
    for k in (1, 3):
        ud = _direct(A, B, u0, dt, k, react)
        assert np.linalg.norm(us[k] - ud) <= 1e-11 * np.linalg.norm(ud)


def test_direct_step_error_within_the_inverse_error_bound():
    """Every eigenvalue of A = I - dt/2 M is >= 1, so the direct step's error against the exact
    step is at most ||I - A F^-1||_2 ||g||_2; the error shrinks with eps (Sec. 3)."""
    n = 32
    a = gen.grf_coefficient(n, 2, 0.1, 33)
    u0 = gen.bumps(n, 2, 3, 34)
    dt = 1.0 / (n + 1)
    A, B = fd.cn_matrices(a, dt)
    g = cn.cn_rhs(B, u0.ravel(), dt)
    exact = spla.spsolve(A.tocsc(), g)
    assert np.linalg.eigvalsh(A.toarray()).min() >= 1.0 - 1e-12
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        F = phif.phif_build(A, n, 2, 8, eps)
        Fi = np.column_stack([phif.phif_apply(F, e) for e in np.eye(n * n)])
        bound = np.linalg.norm(np.eye(n * n) - A @ Fi, 2) * np.linalg.norm(g)
        u1 = cn.cn_solve_direct(B, u0, dt, 1, lambda v: phif.phif_apply(F, v))[1]
        err = np.linalg.norm(u1 - exact)
        assert err <= bound * (1 + 1e-9), (eps, err, bound)
        errs.append(err / np.linalg.norm(exact))
    assert errs[0] > errs[2] and errs[2] < 1e-5, errs


def _midpoint_direct(a_at, u0, dt, steps, react=(0, 0.0, 0.0)):
    u = u0.ravel().copy()
    for k in range(steps):
        A, B = fd.cn_matrices(a_at((k + 0.5) * dt), dt)
        u = spla.spsolve(A.tocsc(), B @ u + dt * cn.reaction(u, *react))
    return u


def test_varying_coefficient_exact_factor_is_the_midpoint_cn_solve():
    n = 16
    a_at = gen.drifting_coefficient(n, 2, 0.2, 51, amp=0.8, period=0.2)
    u0 = gen.bumps(n, 2, 3, 52)
    dt = 0.02
    react = (1, 1.0, 2.0)
    us, its = cn.cn_solve_varying(a_at, n, 2, 4, 0.0, dt, u0, 4, 1, 1e-13, react)
    ref = _midpoint_direct(a_at, u0, dt, 4, react)
    assert np.linalg.norm(us[-1] - ref) <= 1e-10 * np.linalg.norm(ref)
    assert its == [1, 1, 1, 1]


def test_varying_coefficient_second_order_in_time():
    """With the midpoint coefficient the time error falls 4x per halving of dt (left-point
    coefficients would give 2x)."""
    n = 15
    a_at = gen.drifting_coefficient(n, 2, 0.3, 53, amp=1.0, period=0.2)
    u0 = gen.sine_mode(n, 2)
    T = 0.05
    ref = _midpoint_direct(a_at, u0, T / 512, 512)
    errs = []
    for m in (16, 32, 64):
        us, _ = cn.cn_solve_varying(a_at, n, 2, 4, 1e-10, T / m, u0, m, 1, 1e-14)
        errs.append(np.linalg.norm(us[-1] - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.6 and 3.6 < r2 < 4.6, errs


def test_stale_factor_still_converges_to_the_step_solution():
    """Reusing the first factor for every step changes the iteration counts, not u."""
    n = 32
    a_at = gen.drifting_coefficient(n, 2, 0.2, 55, amp=1.0, period=0.4)
    u0 = gen.bumps(n, 2, 3, 56)
    dt = 1.0 / 33
    fresh, it1 = cn.cn_solve_varying(a_at, n, 2, 8, 1e-6, dt, u0, 6, 1, 1e-12)
    stale, it6 = cn.cn_solve_varying(a_at, n, 2, 8, 1e-6, dt, u0, 6, 6, 1e-12)
    ref = _midpoint_direct(a_at, u0, dt, 6)
    for us in (fresh, stale):
        assert np.linalg.norm(us[-1] - ref) <= 1e-10 * np.linalg.norm(ref)
    assert it6[0] == it1[0] and sum(it6) > sum(it1), (it1, it6)
