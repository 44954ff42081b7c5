"""Quad-tree / oct-tree levels and grouping of active DOFs (Sec. 2.2).

The paper assumes n = 1/h = 2^L m, so that every cell has m-1 interior nodes per axis and the
cells are separated by single lines (planes) of nodes.  For grids whose interior node count n
is not of the form 2^L m - 1 this oracle reads the partition as follows:

  * L = max{ l : m 2^l <= n + 1 };
  * the separator coordinates at level l are S_l = { k m 2^l : 1 <= k <= 2^(L-l) - 1 } per
    axis (1-based node indices), so S_0 contains S_1 contains ... and S_L is empty;
  * at level l an active DOF with c of its coordinates in S_l is a cell interior (c = 0), an
    edge (c = 1 in 2D; a face in 3D), a corner (c = 2 in 2D) or, in 3D, an edge (c = 2) or a
    corner (c = 3); the group key is, per axis, either ("s", coordinate) or ("c", index of the
    separator interval containing the coordinate).

For n = 2^L m - 1 this is exactly the paper's layout; for n = 2^L m the last cell per axis has
m interior nodes instead of m - 1.
"""
from __future__ import annotations

import numpy as np


def num_levels(n: int, m: int) -> int:
    L = 0
    while m * (2 ** (L + 1)) <= n + 1:
        L += 1
    return L


def separators(n: int, m: int, level: int) -> np.ndarray:
    L = num_levels(n, m)
    if level >= L:
        return np.zeros(0, dtype=np.int64)
    step = m * 2 ** level
    return step * np.arange(1, 2 ** (L - level), dtype=np.int64)


def group_keys(coords: np.ndarray, S: np.ndarray) -> list[tuple]:
    """Group key of each DOF (rows of ``coords``, 1-based (x, y[, z])) at a level with
    separator set ``S``.  Key entries per axis: (0, cell_interval) or (1, separator_coord)."""
    keys = []
    onsep = np.isin(coords, S)
    interval = np.searchsorted(S, coords, side="left")  # number of separators < coord
    for row in range(coords.shape[0]):
        keys.append(tuple((1, int(coords[row, a])) if onsep[row, a] else (0, int(interval[row, a]))
                          for a in range(coords.shape[1])))
    return keys


def key_kind(key: tuple) -> int:
    """Number of axes on which the group sits on a separator (0 = cell interior)."""
    return sum(k[0] for k in key)


def cell_closure_keys(cell_key: tuple, S: np.ndarray) -> list[tuple]:
    """Keys of all groups on the boundary of a cell: per axis either the cell's own interval or
    one of the (existing) separators bounding it; at least one axis on a separator."""
    options = []
    for kind, val in cell_key:
        assert kind == 0
        opts = [(0, val)]
        if val - 1 >= 0:
            opts.append((1, int(S[val - 1])))   # separator below the interval
        if val < len(S):
            opts.append((1, int(S[val])))       # separator above the interval
        options.append(opts)
    out = [()]
    for opts in options:
        out = [o + (x,) for o in out for x in opts]
    return [k for k in out if key_kind(k) > 0]


def group_active(active_ids: np.ndarray, coords: np.ndarray, S: np.ndarray) -> dict:
    """Map group key -> sorted array of global DOF ids, for the active DOFs ``active_ids``."""
    keys = group_keys(coords[active_ids], S)
    groups: dict = {}
    for dof, key in zip(active_ids.tolist(), keys):
        groups.setdefault(key, []).append(dof)
    return {k: np.array(sorted(v), dtype=np.int64) for k, v in sorted(groups.items())}
