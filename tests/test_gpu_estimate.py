"""hif_inverse_error: the power-iteration estimate of ||I - A F^-1||_2 (Sec. 3, Example 1)
against the oracle's (oracle/estimate.py) on the paper's 2D heat workload at 255^2 and 511^2.

With the oracle's own factor loaded by hif_import, the GPU runs the same iteration on the same
F from the same start vector, so the estimates agree to rounding.  With the GPU-built factor
(skeletons chosen by the GPU's own pivoting) they agree in order of magnitude.  On a small
grid the estimate is checked against the exact norm from the dense I - A F^-1.
"""
import numpy as np
import pytest

from oracle import estimate, fd, phif
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,iters", [(255, 20), (511, 8)])
def test_estimate_matches_oracle(n, iters, gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    from tests.hifb import factor_to_hifb
    w = gen.paper_heat(n, 2, 1e-6, steps=1)
    print(f"[case] paper heat 2d n={n}", flush=True)
    A, _ = fd.cn_matrices(w.a_cells, w.dt)
    F = phif.phif_build(A, n, 2, w.leaf, w.eps)
    x0 = gen.normal_vector(w.N, 9500 + n)
    ref = estimate.inverse_error_power(A, lambda r: phif.phif_apply(F, r), x0, iters)
    a = torch.tensor(w.a_cells, device="cuda")
    x0d = torch.tensor(x0, device="cuda")
    hi = hifcn.import_factor(a, w.dt, n, 2, factor_to_hifb(F), store="f64", leaf=w.leaf)
    est = hi.inverse_error(x0d, iters)
    print(f"  oracle {ref:.6e}, GPU on the oracle's factor {est:.6e}", flush=True)
    assert abs(est - ref) <= 1e-6 * ref, (est, ref)
    assert hi.inverse_error(x0d, iters) == est          # deterministic
    assert hi.inverse_error(x0d, 0) == 0.0
    hi.close()
    hb = hifcn.factor(a, w.dt, n, 2, w.eps, store="f64", leaf=w.leaf)
    eb = hb.inverse_error(x0d, iters)
    print(f"  GPU-built factor {eb:.6e}", flush=True)
    assert 0.2 * ref <= eb <= 5 * ref, (eb, ref)
    hb.close()


def test_estimate_is_a_lower_bound_of_the_dense_norm(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    from tests.hifb import factor_to_hifb
    n, leaf = 31, 8
    a = gen.iid_loguniform_cells(n, 2, 41)
    A, _ = fd.cn_matrices(a, 0.05)
    F = phif.phif_build(A, n, 2, leaf, 1e-2)
    exact = np.linalg.norm(np.eye(n * n) - A @ phif.phif_dense_inverse(F), 2)
    ad = torch.tensor(a, device="cuda")
    h = hifcn.import_factor(ad, 0.05, n, 2, factor_to_hifb(F), store="f64", leaf=leaf)
    x0 = torch.tensor(gen.normal_vector(n * n, 42), device="cuda")
    est = h.inverse_error(x0, 200)
    assert est <= exact * (1 + 1e-10) and est >= 0.98 * exact, (est, exact)
    h.close()
    # eps = 0: no compression, F = A up to rounding
    h0 = hifcn.factor(ad, 0.05, n, 2, 0.0, store="f64", leaf=leaf)
    assert h0.inverse_error(x0, 10) < 1e-10
    h0.close()
