"""Write the full-size expected values of the oracle (tests/golden/fullsize_*.npz).

    python tests/golden/make_fullsize.py [heat2d-1024] [heat3d-64] [fisher2d-256]

Calls only the oracle (``oracle/``) and the seeded input generators (``workloads/``).  For each
workload it runs Algorithm 1 for two Crank-Nicolson steps at rtol 1e-12 with the block PHIF
factor of every tolerance eps listed below (Sec. 2.2, eqAinv), and, as the plain definition of
the same steps, a sparse LU solve of eq_CN.  Stored per workload:

  idx            sampled node indices (seeded, sorted, int64)
  u{k}           u^k at those nodes from the PHIF-PCG run of the first eps (k = 1, 2)
  norm{k}, amax{k}, sum{k}    ||u^k||_2, max|u^k| and sum(u^k) over every node
  iters_eps{e}   the oracle's CG iteration counts per step for eps = e
  ulu{k}         u^k at the sampled nodes from the sparse LU solve (the plain definition)
  direct_rel{k}  ||u^k_pcg - u^k_lu|| / ||u^k_lu||  (how far the oracle's PCG is from the LU
                 solve at rtol 1e-12; at kappa(A) ~ 4e7 this is ~1e-9, which bounds how closely
                 any FP64 PCG result can be compared with another)
  spread{k}      ||u^k(eps_2) - u^k(eps_1)|| / ||u^k(eps_1)|| between the oracle's PCG runs
                 with the two factors (workloads with two eps only)
  quality_eps{e} ||r - A F^-1 r|| / ||r|| of the oracle's factor for eps = e at the seeded
                 r ~ N(0, 1) of seed 9200 + n (how good a preconditioner the method gives there)
  symm_eps{e}    |x.F^-1 y - y.F^-1 x| / (||x|| ||F^-1 y||) at the seeded x, y of seeds
                 9300 + n, 9400 + n (F^-1 is symmetric; a record of the oracle's rounding)

The 1024^2 build takes about a minute per eps and the 64^3 build about five on one core.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cn, fd, phif  # noqa: E402
from workloads import gen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
STEPS = 2
RTOL = 1e-12
SAMPLES = 32768
CASES = {"heat2d-1024": (1e-3, 1e-6), "heat3d-64": (1e-4,), "fisher2d-256": (1e-4,)}


def make(name: str) -> str:
    w = gen.workload(name)
    A, B = fd.cn_matrices(w.a_cells, w.dt)
    out = {"idx": gen.sample_indices(w.N, SAMPLES, 9100 + w.n), "steps": np.int64(STEPS),
           "rtol": np.float64(RTOL)}
    lu = spla.splu(A.tocsc())
    ud = [w.u0.ravel().copy()]
    for _ in range(STEPS):
        ud.append(lu.solve(cn.cn_rhs(B, ud[-1], w.dt, w.reaction)))
    first = None
    for eps in CASES[name]:
        t0 = time.time()
        F = phif.phif_build(A, w.n, w.dim, w.leaf, eps)
        t1 = time.time()
        us, its, _ = cn.cn_solve(A, B, w.u0, w.dt, STEPS, lambda r: phif.phif_apply(F, r),
                                 RTOL, w.reaction)
        print(f"{name} eps {eps:g}: build {t1 - t0:.0f} s, steps {time.time() - t1:.0f} s, "
              f"iters {its}", flush=True)
        out[f"iters_eps{eps:g}"] = np.asarray(its, dtype=np.int64)
        r = gen.normal_vector(w.N, 9200 + w.n)
        out[f"quality_eps{eps:g}"] = np.float64(np.linalg.norm(r - A @ phif.phif_apply(F, r))
                                                / np.linalg.norm(r))
        x, y = gen.normal_vector(w.N, 9300 + w.n), gen.normal_vector(w.N, 9400 + w.n)
        fy = phif.phif_apply(F, y)
        out[f"symm_eps{eps:g}"] = np.float64(abs(x @ fy - y @ phif.phif_apply(F, x))
                                             / (np.linalg.norm(x) * np.linalg.norm(fy)))
        if first is None:
            first = us
            for k in range(1, STEPS + 1):
                out[f"u{k}"] = us[k][out["idx"]]
                out[f"norm{k}"] = np.float64(np.linalg.norm(us[k]))
                out[f"amax{k}"] = np.float64(np.abs(us[k]).max())
                out[f"sum{k}"] = np.float64(us[k].sum())
                out[f"direct_rel{k}"] = np.float64(np.linalg.norm(us[k] - ud[k])
                                                   / np.linalg.norm(ud[k]))
                out[f"ulu{k}"] = ud[k][out["idx"]]
        else:
            for k in range(1, STEPS + 1):
                d = np.linalg.norm(us[k] - first[k]) / np.linalg.norm(first[k])
                out[f"spread{k}"] = np.float64(d)
                print(f"  step {k}: ||u(eps {eps:g}) - u(first eps)|| / ||u|| = {d:.2e}")
    path = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(path, **out)
    return path


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        print("wrote", make(nm), flush=True)
