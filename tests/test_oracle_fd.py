"""Pins of the oracle's finite-difference operator (Sec. 2: five/seven-point stencil)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fd


def _lap1d(n):
    h = 1.0 / (n + 1)
    return sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / h ** 2


@pytest.mark.parametrize("dim,n", [(2, 9), (2, 16), (3, 6)])
def test_constant_coefficient_is_kronecker_sum(dim, n):
    """a = 1: M is the Kronecker sum of 1D second differences (textbook identity)."""
    M = fd.stiffness(np.ones((n + 1,) * dim))
    D = _lap1d(n)
    I = sp.identity(n)
    if dim == 2:
        K = sp.kron(I, D) + sp.kron(D, I)
    else:
        K = sp.kron(sp.kron(I, I), D) + sp.kron(sp.kron(I, D), I) + sp.kron(sp.kron(D, I), I)
    assert abs(M - K).max() < 1e-9 * abs(K).max()


@pytest.mark.parametrize("p,q", [(1, 1), (2, 3), (5, 1)])
def test_sine_eigenpairs(p, q):
    """M v_pq = lam_pq v_pq with lam_pq = -(4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2))."""
    n = 20
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    v = np.outer(np.sin(q * np.pi * x), np.sin(p * np.pi * x)).ravel()   # rows y, cols x
    lam = -(4 / h ** 2) * (np.sin(p * np.pi * h / 2) ** 2 + np.sin(q * np.pi * h / 2) ** 2)
    M = fd.stiffness(np.ones((n + 1, n + 1)))
    assert np.allclose(M @ v, lam * v, rtol=0, atol=1e-9 * abs(lam))


def test_symmetric_negative_definite_and_row_sums():
    rng = np.random.default_rng(3)
    n = 12
    a = 10 ** rng.uniform(-2, 2, size=(n + 1, n + 1))
    M = fd.stiffness(a).toarray()
    assert np.array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).max() < 0
    # constant a: rows of nodes away from the boundary sum to zero (stencil annihilates constants)
    Mc = fd.stiffness(np.full((n + 1, n + 1), 2.5)).toarray().reshape(n, n, n * n)
    assert np.allclose(Mc[1:-1, 1:-1].sum(axis=-1), 0.0, atol=1e-8)


def test_link_coefficient_is_mean_of_adjacent_cells():
    """Each link's coefficient is the mean of the cells touching it, read off one coupling at a
    time from explicit cell coordinates (2 cells in 2D, 4 in 3D)."""
    rng = np.random.default_rng(5)
    n = 5
    h = 1.0 / (n + 1)
    a = rng.uniform(0.5, 2.0, size=(n + 1, n + 1))
    M = fd.stiffness(a)
    # x-link between nodes (jx, jy) and (jx+1, jy), 1-based; cells touching it: x-cell jx,
    # y-cells jy-1 and jy (0-based cell c spans [c h, (c+1) h]).
    jx, jy = 2, 3
    i0 = (jy - 1) * n + (jx - 1)
    expect = 0.5 * (a[jy - 1, jx] + a[jy, jx]) / h ** 2
    assert np.isclose(M[i0, i0 + 1], expect)
    # y-link between (jx, jy) and (jx, jy+1)
    expect_y = 0.5 * (a[jy, jx - 1] + a[jy, jx]) / h ** 2
    assert np.isclose(M[i0, i0 + n], expect_y)
    a3 = rng.uniform(0.5, 2.0, size=(n + 1,) * 3)
    M3 = fd.stiffness(a3)
    jx, jy, jz = 2, 4, 3
    i0 = ((jz - 1) * n + (jy - 1)) * n + (jx - 1)
    exp3 = 0.25 * (a3[jz - 1, jy - 1, jx] + a3[jz - 1, jy, jx] + a3[jz, jy - 1, jx]
                   + a3[jz, jy, jx]) / h ** 2
    assert np.isclose(M3[i0, i0 + 1], exp3)


def test_second_order_consistency_variable_coefficient():
    """(M u)(x_j) -> div(a grad u)(x_j) with O(h^2) error for smooth a and u (manufactured)."""
    def run(n):
        h = 1.0 / (n + 1)
        c = h * (np.arange(n + 1) + 0.5)
        cy, cx = np.meshgrid(c, c, indexing="ij")
        a = 1.0 + cx + cy ** 2
        x = h * np.arange(1, n + 1)
        y, xx = np.meshgrid(x, x, indexing="ij")
        u = np.sin(np.pi * xx) * np.sin(np.pi * y)
        # div(a grad u) = a lap u + a_x u_x + a_y u_y with a_x = 1, a_y = 2y
        A = 1.0 + xx + y ** 2
        lap = -2 * np.pi ** 2 * u
        ux = np.pi * np.cos(np.pi * xx) * np.sin(np.pi * y)
        uy = np.pi * np.sin(np.pi * xx) * np.cos(np.pi * y)
        exact = A * lap + 1.0 * ux + 2 * y * uy
        return np.abs(fd.stiffness(a) @ u.ravel() - exact.ravel()).max()
    e1, e2 = run(31), run(63)
    assert 3.3 < e1 / e2 < 4.7
