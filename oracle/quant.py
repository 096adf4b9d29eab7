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

Escaped values (a reading: the paper leaves the lossless layout open).  An
escaped q has |q| >= R; it is stored as the unsigned code v = 2 (|q| - R) +
[q < 0].  Per level, in stream order, the codes take w_l bits each, w_l the
bit length of the level's largest code (0 when that code is 0 or the level
has no escapes), concatenated most-significant-bit first into 32-bit words;
every level starts on a word boundary.  A level that escapes often at a tight
tolerance then costs about log2(max|q|) bits per escape instead of 64, and
the coarse levels, whose values are large, do not widen the fine ones.

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


def escape_code(q, R: int) -> np.ndarray:
    """v = 2 (|q| - R) + [q < 0] for escaped values (|q| >= R)."""
    q = np.asarray(q, dtype=np.int64)
    return (2 * (np.abs(q) - R) + (q < 0)).astype(np.uint64)


def escape_value(v, R: int) -> np.ndarray:
    """Inverse of escape_code."""
    v = np.asarray(v, dtype=np.uint64)
    mag = (v >> np.uint64(1)).astype(np.int64) + R
    return np.where((v & np.uint64(1)) == 1, -mag, mag)


def escape_table(q, hier: Hierarchy, dict_size: int):
    """Per level: the number of escaped values and their width w_l."""
    R = dict_size // 2
    off = level_offsets(hier)
    q = np.asarray(q, dtype=np.int64)
    counts, widths = [], []
    for l in range(hier.L + 1):
        ql = q[off[l]:off[l + 1]]
        v = escape_code(ql[np.abs(ql) >= R], R)
        counts.append(len(v))
        widths.append(int(v.max()).bit_length() if len(v) else 0)
    return counts, widths


def pack_escapes(q, hier: Hierarchy, dict_size: int):
    """Per level: escape count and width w_l; the packed 32-bit words of all levels."""
    R = dict_size // 2
    off = level_offsets(hier)
    q = np.asarray(q, dtype=np.int64)
    counts, widths = escape_table(q, hier, dict_size)
    words = []
    for l in range(hier.L + 1):
        ql = q[off[l]:off[l + 1]]
        v = escape_code(ql[np.abs(ql) >= R], R)
        w = widths[l]
        if len(v) == 0 or w == 0:
            continue
        shifts = np.arange(w - 1, -1, -1, dtype=np.uint64)
        bits = ((v[:, None] >> shifts[None, :]) & np.uint64(1)).astype(np.uint8).ravel()
        bits = np.concatenate([bits, np.zeros((-len(bits)) % 32, dtype=np.uint8)])
        words.append(np.frombuffer(np.packbits(bits).tobytes(), dtype=">u4").astype(np.uint32))
    allw = np.concatenate(words) if words else np.zeros(0, dtype=np.uint32)
    return counts, widths, allw


def escape_words(counts, widths):
    """32-bit words of each level's packed escapes."""
    return [(int(c) * int(w) + 31) // 32 for c, w in zip(counts, widths)]


def unpack_escapes(words, counts, widths, dict_size: int, block: int = 1 << 20):
    """Escaped q values of all levels in stream order from the packed words."""
    R = dict_size // 2
    words = np.asarray(words, dtype=np.uint32)
    out = []
    pos = 0
    for c, w, nw in zip(counts, widths, escape_words(counts, widths)):
        c, w = int(c), int(w)
        seg = words[pos:pos + nw]
        pos += nw
        if c == 0:
            continue
        if w == 0:
            out.append(escape_value(np.zeros(c, dtype=np.uint64), R))
            continue
        for k0 in range(0, c, block):
            k1 = min(c, k0 + block)
            b0, b1 = k0 * w, k1 * w
            sub = seg[b0 // 32:(b1 + 31) // 32].astype(">u4")
            bits = np.unpackbits(sub.view(np.uint8))[b0 % 32:b0 % 32 + (b1 - b0)].reshape(k1 - k0, w)
            v = np.zeros(k1 - k0, dtype=np.uint64)
            for t in range(w):
                v = (v << np.uint64(1)) | bits[:, t].astype(np.uint64)
            out.append(escape_value(v, R))
    if pos != len(words):
        raise ValueError("escape words do not match the level counts and widths")
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)

