"""Seeded generators for the synthetic parabolic workloads.

Grid convention (shared by every consumer as plain data):
  * ``n`` interior nodes per dimension, spacing h = 1/(n+1), node j (1-based) at x = j*h;
    zero Dirichlet values on the boundary nodes j = 0 and j = n+1.
  * Node arrays have shape (n,)*d in C order with the x index fastest (last axis = x).
  * Coefficient arrays live on the (n+1)^d cells between nodes; cell c (0-based) spans
    [c*h, (c+1)*h] per axis and is sampled at its centre (c+1/2)*h.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def node_coords(n: int, dim: int) -> list[np.ndarray]:
    """Coordinates of interior nodes, as an ``np.meshgrid`` list ordered (x, y[, z])."""
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    # C order with x fastest: axes are (z, y, x) in 3D and (y, x) in 2D.
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    return grids[::-1]  # -> [x, y(, z)] each of shape (n,)*dim


def cell_centres(n: int, dim: int) -> list[np.ndarray]:
    """Centres of the (n+1)^dim cells, same ordering convention as ``node_coords``."""
    h = 1.0 / (n + 1)
    c = h * (np.arange(n + 1) + 0.5)
    grids = np.meshgrid(*([c] * dim), indexing="ij")
    return grids[::-1]


def grf_coefficient(n: int, dim: int, length: float, seed: int, lo: float = 0.1,
                    hi: float = 10.0, features: int = 1024) -> np.ndarray:
    """Lognormal-type smooth field a = exp(g) on the cells, mapped to [lo, hi].

    g is a random-Fourier-feature draw of a Gaussian field with squared-exponential covariance
    of length ``length``: g(x) = sqrt(2/K) sum_k cos(w_k . x + b_k), w_k ~ N(0, length^-2 I),
    b_k ~ U(0, 2 pi).  g is min-max normalised and mapped so that log a spans
    [log lo, log hi] exactly (contrast hi/lo).
    """
    rng = _rng(seed)
    w = rng.normal(0.0, 1.0 / length, size=(features, dim))
    b = rng.uniform(0.0, 2.0 * np.pi, size=features)
    pts = np.stack([c.ravel() for c in cell_centres(n, dim)], axis=1)  # (P, dim) as (x, y, z)
    g = np.zeros(pts.shape[0])
    chunk = 1 << 15
    for s in range(0, pts.shape[0], chunk):
        g[s:s + chunk] = np.cos(pts[s:s + chunk] @ w.T + b).sum(axis=1)
    g *= np.sqrt(2.0 / features)
    t = (g - g.min()) / (g.max() - g.min())
    a = np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * t)
    return a.reshape((n + 1,) * dim)


def drifting_coefficient(n: int, dim: int, length: float, seed: int, amp: float = 0.5,
                         period: float = 1.0, lo: float = 0.1, hi: float = 10.0):
    """A coefficient that changes smoothly in time: a(x, t) = a0(x) exp(amp sin(2 pi t / period)
    b(x)), with a0 a smooth field on [lo, hi] and b a second one on [-1, 1] (both drawn as in
    grf_coefficient).  Returns the function t -> a(., t) on the cells."""
    a0 = grf_coefficient(n, dim, length, seed, lo, hi)
    b = np.log(grf_coefficient(n, dim, length, seed + 1, np.exp(-1.0), np.exp(1.0)))

    def at(t: float) -> np.ndarray:
        return a0 * np.exp(amp * np.sin(2.0 * np.pi * t / period) * b)
    return at


def spectral_grf_coefficient(n: int, dim: int, length: float, seed: int, lo: float = 0.1,
                             hi: float = 10.0) -> np.ndarray:
    """Lognormal field a = exp(g) on the cells, mapped to [lo, hi], drawn by FFT filtering.

    g is white noise on a grid twice the cell grid per axis (so the periodic wrap-around of the
    FFT does not correlate opposite sides of the unit domain), filtered by the square root of
    the spectral density exp(-(2 pi f length)^2 / 2) of the squared-exponential covariance of
    length ``length``, and cropped to the (n+1)^dim cells.  Same distribution family as
    grf_coefficient at O(P log P) cost, for the many mid-size requests of the serving workload.
    """
    rng = _rng(seed)
    m = 2 * (n + 1)
    noise = rng.normal(size=(m,) * dim)
    f = np.fft.fftfreq(m, d=1.0 / (n + 1))  # cycles per unit length
    f2 = sum(np.meshgrid(*([f ** 2] * dim), indexing="ij"))
    g = np.fft.ifftn(np.fft.fftn(noise) * np.exp(-((2 * np.pi * length) ** 2) * f2 / 4)).real
    g = g[(slice(0, n + 1),) * dim]
    t = (g - g.min()) / (g.max() - g.min())
    return np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * t)


def normal_vector(N: int, seed: int) -> np.ndarray:
    """N iid standard normal values (probe vectors of the parity tests)."""
    return _rng(seed).normal(size=N)


def sample_indices(N: int, count: int, seed: int) -> np.ndarray:
    """min(N, count) distinct indices in [0, N), sorted (where a full-size comparison samples)."""
    return np.sort(_rng(seed).choice(N, size=min(N, count), replace=False)).astype(np.int64)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s, from 0) of a Poisson process of `rate` requests per second."""
    return np.cumsum(_rng(seed).exponential(1.0 / rate, size=count))


def iid_loguniform_cells(n: int, dim: int, seed: int, lo_exp: float = -2.0,
                         hi_exp: float = 2.0) -> np.ndarray:
    """Per-cell iid 10^U(lo_exp, hi_exp) on the (n+1)^dim cells."""
    rng = _rng(seed)
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size=(n + 1,) * dim)


def iid_uniform_nodes(n: int, dim: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    return rng.uniform(0.0, 1.0, size=(n,) * dim)


def sine_mode(n: int, dim: int, p: int = 1) -> np.ndarray:
    """prod_d sin(p pi x_d) at the interior nodes."""
    u = np.ones((n,) * dim)
    for c in node_coords(n, dim):
        u = u * np.sin(p * np.pi * c)
    return u


def bumps(n: int, dim: int, count: int, seed: int, width2: float = 0.005) -> np.ndarray:
    """clip(sum_i exp(-|x - c_i|^2 / width2), 0, 1), c_i ~ U(0.1, 0.9)^dim."""
    rng = _rng(seed)
    centres = rng.uniform(0.1, 0.9, size=(count, dim))
    xs = node_coords(n, dim)
    u = np.zeros((n,) * dim)
    for c in centres:
        r2 = np.zeros((n,) * dim)
        for d in range(dim):
            r2 = r2 + (xs[d] - c[d]) ** 2
        u += np.exp(-r2 / width2)
    return np.clip(u, 0.0, 1.0)


def gaussian_sum_coefficient(n: int, dim: int, m: int, sigma2: float, lo: float, hi: float,
                             seed: int) -> np.ndarray:
    """Sec. 3 coefficient (eq 2d_coeff / 3d_coeff): the sum over m centres x_i ~ U(0,1)^d of
    exp(-|x - x_i|^2 / sigma2), on the cells, rescaled and shifted affinely onto [lo, hi]."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(m, dim))  # (x, y[, z]) per centre
    pts = [c for c in cell_centres(n, dim)]          # [x, y(, z)] grids
    s = np.zeros(pts[0].shape)
    for c in centres:
        r2 = sum((pts[k] - c[k]) ** 2 for k in range(dim))
        s += np.exp(-r2 / sigma2)
    t = (s - s.min()) / (s.max() - s.min())
    return lo + (hi - lo) * t


def gaussian_initial(n: int, dim: int, centres, sigma2: float) -> np.ndarray:
    """Sec. 3 initial data (eq 2d_h_u0 / 3d_u0): a sum of Gaussians exp(-|x - c|^2 / sigma2)
    at the nodes, one per centre c (each centre a coordinate repeated on every axis)."""
    x = node_coords(n, dim)
    u = np.zeros(x[0].shape)
    for c in centres:
        u += np.exp(-sum((x[k] - c) ** 2 for k in range(dim)) / sigma2)
    return u


@dataclass
class Workload:
    """One synthetic parabolic solve: grid, coefficient, initial state and solver settings."""

    name: str
    dim: int
    n: int
    a_cells: np.ndarray
    u0: np.ndarray
    dt: float
    steps: int
    eps: float
    rtol: float
    reaction: tuple = (0, 0.0, 0.0)  # (kind, k1, k2): 0 none, 1 k1*u*(1-u/k2)
    leaf: int = 8
    store: str = "f32"
    maxit: int = 500
    x0: str = "zero"  # PCG initial guess: "zero" (x0 = 0) or "previous" (x0 = u^k)
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.dim


def paper_heat(n: int, dim: int, eps: float, seed: int = 6000, steps: int = 100,
               logistic: bool = False) -> Workload:
    """The paper's Sec. 3 experiments.  Example 1 (heat): 2D with a(x) from m = 100 Gaussians
    (sigma_2^2 = 0.005) rescaled onto [0.1, 10], u0 two Gaussians at c = 0.35, 0.65
    (sigma^2 = 0.05), dt = h; 3D with m = 1000 Gaussians onto [0.05, 20], u0 one Gaussian at
    c = 0.5, dt = 0.1 h.  Example 2 (logistic, r(u) = k1 u (1 - u/k2), k1 = 1, k2 = 10): the same
    coefficients (3D: m = 200), u0 one Gaussian at c = 0.5 scaled by 2 / (3 sqrt(2 pi sigma^2))
    in 2D and (2 pi sigma)^(-3/2) (sigma = sqrt(0.05)) in 3D.  The centres are random (no seeds
    printed), so iteration counts compare with the paper's tables as ranges only.  rtol 1e-12."""
    h = 1.0 / (n + 1)
    s2 = 0.05
    if dim == 2:
        a = gaussian_sum_coefficient(n, 2, 100, 0.005, 0.1, 10.0, seed)
        dt = h
        if logistic:
            u0 = 2.0 / (3.0 * np.sqrt(2.0 * np.pi * s2)) * gaussian_initial(n, 2, (0.5,), s2)
        else:
            u0 = gaussian_initial(n, 2, (0.35, 0.65), s2)
    else:
        a = gaussian_sum_coefficient(n, 3, 200 if logistic else 1000, 0.005, 0.05, 20.0, seed)
        dt = 0.1 * h
        u0 = gaussian_initial(n, 3, (0.5,), s2)
        if logistic:
            u0 = u0 * (2.0 * np.pi * np.sqrt(s2)) ** -1.5
    kind = "logistic" if logistic else "heat"
    return Workload(f"paper-{kind}{dim}d-{n}-eps{eps:g}", dim, n, a, u0, dt, steps, eps, 1e-12,
                    reaction=(1, 1.0, 10.0) if logistic else (0, 0.0, 0.0))


def serving_request(i: int, seed_base: int = 5000, sizes=(64, 128, 256, 512)) -> Workload:
    """Request i of the serving workload: an independent 2D Fisher-KPP solve (r = u(1-u)) with
    its own lognormal coefficient, n drawn from `sizes`, dt from {1e-3, 1e-2, 1e-1}, 50 steps."""
    rng = _rng(seed_base + 10 * i)
    n = int(rng.choice(list(sizes)))
    dt = float(rng.choice([1e-3, 1e-2, 1e-1]))
    a = spectral_grf_coefficient(n, 2, 0.1, seed_base + 10 * i + 1)
    u0 = bumps(n, 2, 10, seed_base + 10 * i + 2)
    return Workload(f"req{i}", 2, n, a, u0, dt, 50, 1e-4, 1e-8, reaction=(1, 1.0, 1.0))


def serving_requests(count: int = 256, seed_base: int = 5000, sizes=(64, 128, 256, 512)
                     ) -> list[Workload]:
    """The serving workload: `count` independent requests (see serving_request)."""
    return [serving_request(i, seed_base, sizes) for i in range(count)]


CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def _coefficient(n: int, dim: int, spec: dict) -> np.ndarray:
    """Cell coefficients a on the (n+1)^dim cells from a config's "a" object."""
    k = spec["kind"]
    if k == "constant":
        return np.full((n + 1,) * dim, float(spec["value"]))
    if k == "grf":
        return grf_coefficient(n, dim, float(spec["length"]), int(spec["seed"]),
                               float(spec.get("lo", 0.1)), float(spec.get("hi", 10.0)))
    if k == "spectral_grf":
        return spectral_grf_coefficient(n, dim, float(spec["length"]), int(spec["seed"]),
                                        float(spec.get("lo", 0.1)), float(spec.get("hi", 10.0)))
    if k == "iid_loguniform":
        return iid_loguniform_cells(n, dim, int(spec["seed"]), float(spec.get("lo_exp", -2.0)),
                                    float(spec.get("hi_exp", 2.0)))
    if k == "gaussian_sum":
        return gaussian_sum_coefficient(n, dim, int(spec["m"]), float(spec["sigma2"]),
                                        float(spec["lo"]), float(spec["hi"]), int(spec["seed"]))
    raise ValueError(f"unknown coefficient kind {k!r}")


def _initial(n: int, dim: int, spec: dict) -> np.ndarray:
    """Initial state u0 on the n^dim nodes from a config's "u0" object."""
    k = spec["kind"]
    if k == "sine_mode":
        return sine_mode(n, dim, int(spec.get("p", 1)))
    if k == "sine_plus_noise":  # the sine mode plus `noise` times standard normal values
        rng = _rng(int(spec["seed"]))
        return sine_mode(n, dim, int(spec.get("p", 1))) + float(spec["noise"]) * rng.normal(
            size=(n,) * dim)
    if k == "bumps":
        return bumps(n, dim, int(spec["count"]), int(spec["seed"]),
                     float(spec.get("width2", 0.005)))
    if k == "iid_uniform":
        return iid_uniform_nodes(n, dim, int(spec["seed"]))
    if k == "gaussian":
        return float(spec.get("scale", 1.0)) * gaussian_initial(n, dim, tuple(spec["centres"]),
                                                                float(spec["sigma2"]))
    raise ValueError(f"unknown initial-state kind {k!r}")


CONFIG_FIELDS = ("name", "dim", "n", "leaf", "a", "u0", "dt", "steps", "eps", "store", "rtol",
                 "maxit", "x0", "reaction")


def load_config(cfg, **override) -> Workload:
    """A workload from a JSON config (a path or an already parsed dict): grid (dim, n), leaf box
    size m, the recipes of a and u0 with their seeds, dt, steps, eps, storage, rtol, maxit, the
    PCG initial guess ("zero": x0 = 0, "previous": x0 = u^k) and the reaction (kind, k1, k2).
    Keyword arguments replace top-level fields."""
    if not isinstance(cfg, dict):
        with open(cfg) as f:
            cfg = json.load(f)
    cfg = {**cfg, **override}
    missing = [k for k in CONFIG_FIELDS if k not in cfg]
    if missing:
        raise ValueError(f"config {cfg.get('name')!r} lacks {missing}")
    if cfg["x0"] not in ("zero", "previous"):
        raise ValueError("x0 must be 'zero' or 'previous'")
    if cfg["store"] not in ("f32", "f64", "bf16"):
        raise ValueError("store must be f32, f64 or bf16")
    n, dim = int(cfg["n"]), int(cfg["dim"])
    return Workload(cfg["name"], dim, n, _coefficient(n, dim, cfg["a"]), _initial(n, dim, cfg["u0"]),
                    float(cfg["dt"]), int(cfg["steps"]), float(cfg["eps"]), float(cfg["rtol"]),
                    reaction=tuple(cfg["reaction"]), leaf=int(cfg["leaf"]),
                    store=cfg["store"], maxit=int(cfg["maxit"]), x0=cfg["x0"],
                    extra={"config": cfg})


def config_names() -> list[str]:
    """Names of the committed workload configs (configs/<name>.json)."""
    return sorted(f[:-5] for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))


WORKLOADS = {name: (lambda name=name, **kw: load_config(os.path.join(CONFIG_DIR, name + ".json"),
                                                        **kw))
             for name in config_names()}


def workload(name: str, **kw) -> Workload:
    """A committed workload by name (configs/<name>.json), or any config file by its path."""
    if name.endswith(".json"):
        return load_config(name, **kw)
    return WORKLOADS[name](**kw)
