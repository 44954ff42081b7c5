"""Host-side logic of the serving layer and its input generators (no GPU)."""
import numpy as np

from workloads import gen


def test_percentiles_nearest_rank():
    from paper_2004_05566_amd.serve import percentiles
    x = np.arange(1, 101) / 100.0
    p = percentiles(np.random.default_rng(0).permutation(x))
    assert p["p50"] == 0.50 and p["p99"] == 0.99
    assert percentiles([3.0]) == {"p50": 3.0, "p99": 3.0}


def test_estimate_grows_with_size_and_precision():
    from paper_2004_05566_amd.serve import estimate_bytes
    e = [estimate_bytes(n, 2, "f32") for n in (64, 128, 256, 512)]
    assert all(a < b for a, b in zip(e, e[1:]))
    assert estimate_bytes(256, 2, "bf16") < estimate_bytes(256, 2, "f32") < \
        estimate_bytes(256, 2, "f64")
    # the stored FP32 factor of the 512^2 requests measures about 40 entries per DOF: the
    # estimate must cover it plus its FP64 build copy
    assert estimate_bytes(512, 2, "f32") > 512 ** 2 * 40 * (4 + 8)


def test_spectral_field_range_and_correlation():
    a = gen.spectral_grf_coefficient(255, 2, 0.1, 1)
    assert a.shape == (256, 256)
    assert np.isclose(a.min(), 0.1) and np.isclose(a.max(), 10.0)
    g = np.log(a)
    g = (g - g.mean()) / g.std()
    # squared-exponential covariance exp(-r^2 / (2 l^2)) at short lags (r in cell widths / 256)
    for lag in (5, 13):
        emp = (g[:, :-lag] * g[:, lag:]).mean()
        assert abs(emp - np.exp(-(lag / 256) ** 2 / 0.02)) < 0.05, lag
    assert np.array_equal(a, gen.spectral_grf_coefficient(255, 2, 0.1, 1))


def test_serving_requests_mix():
    reqs = gen.serving_requests(24, sizes=(16, 32))
    assert {w.n for w in reqs} <= {16, 32}
    assert {w.dt for w in reqs} <= {1e-3, 1e-2, 1e-1}
    assert all(w.steps == 50 and w.reaction == (1, 1.0, 1.0) for w in reqs)
    assert len({w.a_cells.tobytes() for w in reqs}) == 24


def test_poisson_arrivals():
    t = gen.poisson_arrivals(20000, 40.0, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 40.0) < 1.0


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus above 1 ends with a message and a non-zero status before
    anything touches a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]
