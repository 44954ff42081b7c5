"""Checkpoint and resume of a Crank-Nicolson run (eq_CN): the state of the run is (u^k, k), and
the factor is a deterministic function of (a, dt, grid, eps, leaf, storage), so a resumed run
rebuilds it instead of saving it.  Run k steps, write u^k and k to a file, drop the handle, build
a new one from the same inputs, read the file back and run the remaining steps: u and every
step's iteration count are bitwise those of the run that was never interrupted."""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, dim, leaf, eps, store, dt, reaction (kind, k1, k2)
    ("fisher2d-128-f64", 128, 2, 8, 1e-3, "f64", 0.05, (1, 1.0, 1.0)),
    ("heat2d-127-f32", 127, 2, 8, 1e-3, "f32", 1.0 / 128, (0, 0.0, 1.0)),
    ("heat3d-16-f64", 16, 3, 4, 1e-3, "f64", 0.05, (0, 0.0, 1.0)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_resume_from_checkpoint_is_bitwise(case, tmp_path, gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    name, n, dim, leaf, eps, store, dt, react = case
    print(f"[case] {name}", flush=True)
    a = gen.grf_coefficient(n, dim, 0.15, 31)
    u0 = gen.bumps(n, dim, 3, 32).ravel()
    total, k = 6, 3

    def handle():
        return hifcn.factor(torch.tensor(a, device="cuda"), dt, n, dim, eps, store=store,
                            leaf=leaf)

    h = handle()
    u = torch.tensor(u0, device="cuda")
    its_full, _ = h.cn_solve(u, total, rtol=1e-10, reaction=react)
    u_full = u.cpu().numpy()
    h.close()

    h = handle()
    u = torch.tensor(u0, device="cuda")
    its_a, _ = h.cn_solve(u, k, rtol=1e-10, reaction=react)
    path = tmp_path / "cn_state.npz"
    np.savez(path, u=u.cpu().numpy(), k=k, its=np.asarray(its_a))
    h.close()
    del u

    state = np.load(path)
    h = handle()
    u = torch.tensor(state["u"], device="cuda")
    its_b, _ = h.cn_solve(u, total - int(state["k"]), rtol=1e-10, reaction=react)
    h.close()
    assert np.array_equal(u.cpu().numpy(), u_full)
    assert list(state["its"]) + list(its_b) == list(its_full)
    print(f"  n_i {[int(v) for v in its_full]}", flush=True)
