"""Level-wise linear quantization, symbols and stream order (oracle).

Reading of the paper's quantization stage (Sec. 2: each multilevel
coefficient is replaced by an integer multiple of its level's bin width):

* y = float64(c) * (1 / b_l), the reciprocal taken in float64;
* q = sign(y) * floor(|y| + 0.5)  (round half away from zero);
* dequantized value c^ = T(float64(q) * b_l), so |c - c^| <= b_l/2 up to the
  final rounding to T.

Symbols for the entropy coder: with R = dict_size/2, s = q + R when |q| < R,
else the escape symbol 0; escaped q values are kept, in stream order, in a
separate outlier list.

Stream order: the coarsest grid in C order, then levels 1..L; within a
level the sub-grids by odd-dimension mask m = 1 .. 2^D-1 ascending (bit d of
m set <=> the dimension-d index is a new node), each sub-grid dense in C order
over (new indices if the bit is set else coarse indices).
"""
from __future__ import annotations

import numpy as np

from .grid import Hierarchy


def level_subgrids(hier: Hierarchy, l: int):
    """Index sets (per dimension) of each sub-grid of level l, in stream order."""
    D = hier.D
    out = []
    for m in range(1, 1 << D):
        sets = []
        for d in range(D):
            sets.append(hier.fidx(l, d) if (m >> d) & 1 else hier.cidx(l, d))
        out.append(sets)
    return out


def to_stream(coarsest, cbars, hier: Hierarchy):
    """Flatten (coarsest, cbar_1..cbar_L) into the coefficient stream."""
    parts = [np.ravel(coarsest)]
    for l in range(1, hier.L + 1):
        for sets in level_subgrids(hier, l):
            parts.append(np.ravel(cbars[l][np.ix_(*sets)]))
    return np.concatenate(parts)


def from_stream(stream, hier: Hierarchy, T):
    """Inverse of to_stream: returns (coarsest, [cbar_1..cbar_L]) with zeros at coarse nodes."""
    counts = hier.level_counts()
    pos = 0
    n0 = counts[0]
    coarsest = np.asarray(stream[:n0], dtype=T).reshape(hier.sizes[0])
    pos = n0
    cbars = [None] * (hier.L + 1)
    for l in range(1, hier.L + 1):
        cb = np.zeros(hier.sizes[l], dtype=T)
        for sets in level_subgrids(hier, l):
            shp = tuple(len(s) for s in sets)
            k = int(np.prod(shp))
            cb[np.ix_(*sets)] = np.asarray(stream[pos:pos + k], dtype=T).reshape(shp)
            pos += k
        cbars[l] = cb
    assert pos == len(stream)
    return coarsest, cbars


def level_offsets(hier: Hierarchy):
    c = hier.level_counts()
    return np.concatenate([[0], np.cumsum(c)]).astype(np.int64)


def quantize(c, b: float):
    """Integer multiples of b (round half away from zero), decided in float64."""
    inv_b = np.float64(1.0) / np.float64(b)
    y = np.asarray(c).astype(np.float64) * inv_b
    return (np.sign(y) * np.floor(np.abs(y) + 0.5)).astype(np.int64)


def dequantize(q, b: float, T):
    return (np.asarray(q, dtype=np.int64).astype(np.float64) * np.float64(b)).astype(T)


def quantize_stream(stream, hier: Hierarchy, bins):
    off = level_offsets(hier)
    q = np.empty(len(stream), dtype=np.int64)
    for l in range(hier.L + 1):
        q[off[l]:off[l + 1]] = quantize(stream[off[l]:off[l + 1]], bins[l])
    return q


def dequantize_stream(q, hier: Hierarchy, bins, T):
    off = level_offsets(hier)
    c = np.empty(len(q), dtype=T)
    for l in range(hier.L + 1):
        c[off[l]:off[l + 1]] = dequantize(q[off[l]:off[l + 1]], bins[l], T)
    return c


def to_symbols(q, dict_size: int):
    """Symbols (uint16-range ints) and outlier values in stream order."""
    R = dict_size // 2
    q = np.asarray(q, dtype=np.int64)
    inside = np.abs(q) < R
    sym = np.where(inside, q + R, 0).astype(np.int64)
    return sym, q[~inside].copy()


def from_symbols(sym, outliers, dict_size: int):
    R = dict_size // 2
    sym = np.asarray(sym, dtype=np.int64)
    q = sym - R
    esc = sym == 0
    if int(esc.sum()) != len(outliers):
        raise ValueError("outlier count does not match escape symbols")
    q[esc] = np.asarray(outliers, dtype=np.int64)
    return q
