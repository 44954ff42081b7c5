"""Serialise an oracle PHIF factor into the HIFB blob read by hif_import (test fixture).

The format is the data layout documented in include/hifcn.h; nothing here computes anything
of the method: it only writes the oracle's blocks (L, G, L_g, T, L_s, L_r) as they are.
"""
import struct

import numpy as np


def _i32(v):
    return np.asarray(v, dtype="<i4").tobytes()


def _f64(m):
    return np.ascontiguousarray(m, dtype="<f8").tobytes()


def factor_to_hifb(F) -> bytes:
    out = [struct.pack("<6i", 0x42464948, 1, F.dim, F.n, F.leaf, len(F.levels))]
    for lv in F.levels:
        out.append(struct.pack("<i", len(lv.cells)))
        for c in lv.cells:
            out += [struct.pack("<2i", len(c.I), len(c.B)), _i32(c.I), _i32(c.B), _f64(c.L),
                    _f64(c.G)]
        out.append(struct.pack("<i", len(lv.groups)))
        for g in lv.groups:
            out += [struct.pack("<i", len(g.idx)), _i32(g.idx), _f64(g.L)]
        out.append(struct.pack("<i", len(lv.skels)))
        for s in lv.skels:
            out += [struct.pack("<2i", len(s.redund), len(s.skel)), _i32(s.redund), _i32(s.skel),
                    _f64(s.T), _f64(s.Ls)]
    out += [struct.pack("<i", len(F.root_idx)), _i32(F.root_idx), _f64(F.root_L)]
    return b"".join(out)
