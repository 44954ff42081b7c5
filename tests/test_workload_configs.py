"""The JSON workload configs (workloads/configs/*.json): every field present and valid, and each
named workload equal, array for array, to the generator calls its recipe names (the committed
full-size expected values were written from exactly these inputs)."""
import json
import os

import numpy as np
import pytest

from workloads import gen

EXPECT = {
    # name: (a, u0) from the generators directly
    "heat2d-32": lambda: (np.ones((33, 33)), gen.sine_mode(32, 2)),
    "fisher2d-256": lambda: (gen.grf_coefficient(256, 2, 0.1, 2001), gen.bumps(256, 2, 10, 2002)),
    "heat2d-1024": lambda: (gen.iid_loguniform_cells(1024, 2, 3001),
                            gen.iid_uniform_nodes(1024, 2, 3002)),
    "heat3d-64": lambda: (gen.grf_coefficient(64, 3, 0.15, 4001),
                          gen.sine_mode(64, 3)
                          + 0.1 * np.random.Generator(np.random.PCG64(4002)).normal(size=(64,) * 3)),
}
SETTINGS = {
    # name: (dt, steps, eps, rtol, reaction, store)
    "heat2d-32": (1e-2, 10, 1e-6, 1e-10, (0, 0.0, 0.0), "f64"),
    "fisher2d-256": (1e-3, 100, 1e-4, 1e-8, (1, 1.0, 1.0), "f32"),
    "heat2d-1024": (1e-1, 20, 1e-3, 1e-8, (0, 0.0, 0.0), "f32"),
    "heat3d-64": (1e-2, 20, 1e-4, 1e-8, (0, 0.0, 0.0), "f32"),
}


def test_every_named_workload_has_a_config():
    assert set(gen.config_names()) == set(EXPECT)


@pytest.mark.parametrize("name", sorted(EXPECT))
def test_config_reproduces_the_generators(name):
    w = gen.workload(name)
    a, u0 = EXPECT[name]()
    assert w.name == name and w.a_cells.shape == a.shape and w.u0.shape == u0.shape
    assert np.array_equal(w.a_cells, a) and np.array_equal(w.u0, u0)
    assert (w.dt, w.steps, w.eps, w.rtol, tuple(w.reaction), w.store) == SETTINGS[name]
    assert w.leaf == 8 and w.maxit == 500 and w.x0 == "zero"


def test_config_file_path_and_overrides(tmp_path):
    src = os.path.join(gen.CONFIG_DIR, "fisher2d-256.json")
    cfg = json.load(open(src))
    cfg.update(name="fisher2d-64-warm", n=64, x0="previous", maxit=50)
    p = tmp_path / "w.json"
    p.write_text(json.dumps(cfg))
    w = gen.workload(str(p), eps=1e-6)
    assert (w.n, w.N, w.x0, w.maxit, w.eps) == (64, 64 * 64, "previous", 50, 1e-6)
    assert np.array_equal(w.a_cells, gen.grf_coefficient(64, 2, 0.1, 2001))


def test_config_rejects_missing_or_bad_fields():
    cfg = json.load(open(os.path.join(gen.CONFIG_DIR, "heat2d-32.json")))
    for bad in ({"x0": "random"}, {"store": "f16"}, {"a": {"kind": "unknown"}}):
        with pytest.raises(ValueError):
            gen.load_config({**cfg, **bad})
    del cfg["maxit"]
    with pytest.raises(ValueError):
        gen.load_config(cfg)
