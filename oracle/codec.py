"""End-to-end compression and decompression to the self-describing format (oracle).

The paper's high-level calls compress an array under a tolerance and error
bound type, and decompress from the buffer alone, whose self-describing
header carries the version, error bound, topology and coder (Sec. 2.1 and
Sec. 3, first listing); compression ratio is input bytes over output bytes.

Wire format (little-endian; offsets in bytes):

    0  'MGHP'             magic
    4  u16 version = 2
    6  u8  dtype           0 = float32, 1 = float64
    7  u8  ndim            1..4
    8  u8  eb              0 = absolute, 1 = relative
    9  u8  alloc           0 = plain, 1 = learned, 2 = count-weighted
   10  u8  coord_flags     bit d set: dimension d stores its coordinates
   11  u8  fallback        1 when a learned allocation fell back to plain
   12  u32 L               number of levels
   16  u32 dict_size
   20  u32 chunk_symbols
   24  f64 tol
   32  f64 tau_abs
   40  f64 maxabs          max |u|
   48  u64 n_symbols
   56  u64 n_chunks
   64  u64 n_outliers
   72  u64 payload_words
   80  u8  norm            0 = L-infinity, 1 = s-norm with smoothness s
   81  u8[7] zero
   88  f64 s
   96  u64 shape[ndim]
       f64 coords          for each flagged dimension, its n_d coordinates
       f64 bins[L+1]
       u64 level_escapes[L+1]      escaped values per level
       u32 level_escape_bits[L+1]  their width per level
       u8  code_len[dict_size]
       u32 chunk_bits[n_chunks]
       u32 chunk_esc[n_chunks]     escape symbols per chunk
       u32 payload[payload_words]
       u32 escapes[]               per level, ceil(count * width / 32) words
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass

import numpy as np

from . import alloc as A
from . import huffman as H
from . import quant as Q
from . import snorm as SN
from . import transform as X
from .grid import Hierarchy

MAGIC = b"MGHP"
VERSION = 2
FIXED = 96
NORM_LINF, NORM_S = 0, 1
ALLOC_PLAIN, ALLOC_LEARNED, ALLOC_COUNT = 0, 1, 2


@dataclass
class Parts:
    """Everything the compressor computes, for stage-by-stage comparisons."""

    hier: Hierarchy
    T: type
    maxabs: float
    tau_abs: float
    tau_eff: float
    bins: list
    stream: np.ndarray
    q: np.ndarray
    symbols: np.ndarray
    outliers: np.ndarray
    hist: np.ndarray
    lengths: np.ndarray
    codes: np.ndarray
    chunk_bits: list
    chunk_esc: list
    words: list
    esc_counts: list
    esc_widths: list
    esc_words: np.ndarray


def compress_parts(u, tol, rel=True, coords=None, dict_size=8192, chunk=1024, bins=None,
                   alloc="plain", norm="linf", s=0.0, tau=None):
    """norm "linf" bounds the maximum error (alloc.py); norm "s" bounds the
    s-norm of the error (snorm.py; relative only for s = 0, plain widths only).
    tau, when given, replaces the bound computed from tol (a float64 norm that
    another implementation summed in another order)."""
    u = np.asarray(u)
    T = u.dtype.type
    if T not in (np.float32, np.float64):
        raise TypeError("float32 or float64 input")
    if not np.all(np.isfinite(u)):
        raise ValueError("non-finite input")
    if not tol > 0:
        raise ValueError("tolerance must be positive")
    hier = Hierarchy(u.shape, coords)
    maxabs = float(np.max(np.abs(u))) if u.size else 0.0
    if norm == "s":
        if alloc != "plain":
            raise ValueError("the s-norm bound takes the plain allocation")
        if rel and s != 0.0:
            raise ValueError("a relative s-norm bound needs s = 0")
        if tau is None:
            tau = tol * math.sqrt(SN.l2_norm_sq(u, hier)) if rel else tol
        tau_eff = SN.tau_effective(tau, maxabs, hier, s, T)
        if bins is None:
            bins = SN.bins_for(hier, tau_eff, s)
            if SN.out_of_range(tau, maxabs, hier, s, T, bins):
                raise ValueError("tolerance outside the supported range")
    else:
        if tau is None:
            tau = A.tau_abs(tol, maxabs, rel)
        tau_eff = A.tau_effective(tau, maxabs, hier.L, T)
        if bins is None:
            bins = A.plain_bins(hier, tau_eff) if alloc == "plain" else A.count_weighted_bins(hier, tau_eff)
            if A.out_of_range(tau, maxabs, hier.L, T, bins):
                raise ValueError("tolerance outside the supported range")
    coarsest, cbars = X.decompose(u, hier, T)
    stream = Q.to_stream(coarsest, cbars, hier)
    q = Q.quantize_stream(stream, hier, bins)
    sym, outl = Q.to_symbols(q, dict_size)
    hist = H.histogram(sym, dict_size)
    lengths = H.code_lengths(hist)
    codes = H.canonical_codes(lengths)
    cbits, words = H.encode(sym, lengths, codes, chunk)
    esc = [int(np.count_nonzero(sym[k:k + chunk] == 0)) for k in range(0, len(sym), chunk)]
    ecount, ewidth, ewords = Q.pack_escapes(q, hier, dict_size)
    return Parts(hier, T, maxabs, tau, tau_eff, list(map(float, bins)), stream, q, sym, outl, hist,
                 lengths, codes, cbits, esc, words, ecount, ewidth, ewords)


def serialize(p: Parts, tol, rel, coords, dict_size, chunk, alloc_code=ALLOC_PLAIN, fallback=0, norm=NORM_LINF,
              s=0.0) -> bytes:
    hier = p.hier
    D = hier.D
    flags = 0
    coord_blob = b""
    if coords is not None:
        for d in range(D):
            if coords[d] is not None:
                flags |= 1 << d
                coord_blob += np.asarray(coords[d], dtype="<f8").tobytes()
    n = len(p.symbols)
    nch = len(p.chunk_bits)
    head = struct.pack("<4sHBBBBBBIIIdddQQQQB7xd", MAGIC, VERSION, 0 if p.T is np.float32 else 1, D,
                       1 if rel else 0, alloc_code, flags, fallback, hier.L, dict_size, chunk,
                       float(tol), float(p.tau_abs), float(p.maxabs), n, nch, len(p.outliers),
                       len(p.words), norm, float(s))
    assert len(head) == FIXED
    out = [head, np.asarray(hier.shape, dtype="<u8").tobytes(), coord_blob,
           np.asarray(p.bins, dtype="<f8").tobytes(),
           np.asarray(p.esc_counts, dtype="<u8").tobytes(),
           np.asarray(p.esc_widths, dtype="<u4").tobytes(),
           np.asarray(p.lengths, dtype=np.uint8).tobytes(),
           np.asarray(p.chunk_bits, dtype="<u4").tobytes(),
           np.asarray(p.chunk_esc, dtype="<u4").tobytes(),
           np.asarray(p.words, dtype="<u4").tobytes(),
           np.asarray(p.esc_words, dtype="<u4").tobytes()]
    return b"".join(out)


def compress(u, tol, rel=True, coords=None, dict_size=8192, chunk=1024, bins=None, alloc="plain", norm="linf",
             s=0.0, tau=None):
    p = compress_parts(u, tol, rel, coords, dict_size, chunk, bins, alloc, norm, s, tau)
    code = ALLOC_PLAIN if (alloc == "plain" and bins is None) else (ALLOC_COUNT if alloc == "count" else ALLOC_LEARNED)
    if norm == "s":
        code = ALLOC_PLAIN
    return serialize(p, tol, rel, coords, dict_size, chunk, code, norm=NORM_S if norm == "s" else NORM_LINF,
                     s=s if norm == "s" else 0.0)


@dataclass
class Header:
    dtype: type
    ndim: int
    rel: bool
    alloc: int
    fallback: int
    L: int
    dict_size: int
    chunk: int
    tol: float
    tau_abs: float
    maxabs: float
    n: int
    n_chunks: int
    n_outliers: int
    payload_words: int
    norm: int
    s: float
    shape: tuple
    coords: list
    bins: list
    esc_counts: list
    esc_widths: list
    offsets: dict


def parse(buf: bytes) -> Header:
    if len(buf) < FIXED or buf[:4] != MAGIC:
        raise ValueError("not a compressed buffer")
    (_, ver, dt, D, rel, al, flags, fb, L, dsz, ch, tol, tau, mx, n, nch, nout,
     nw, norm, s) = struct.unpack_from("<4sHBBBBBBIIIdddQQQQB7xd", buf, 0)
    if ver != VERSION or dt > 1 or not 1 <= D <= 4:
        raise ValueError("unsupported header")
    pos = FIXED
    shape = tuple(int(v) for v in np.frombuffer(buf, "<u8", D, pos))
    pos += 8 * D
    coords = [None] * D
    for d in range(D):
        if (flags >> d) & 1:
            coords[d] = np.frombuffer(buf, "<f8", shape[d], pos).copy()
            pos += 8 * shape[d]
    bins = [float(v) for v in np.frombuffer(buf, "<f8", L + 1, pos)]
    pos += 8 * (L + 1)
    ecount = [int(v) for v in np.frombuffer(buf, "<u8", L + 1, pos)]
    pos += 8 * (L + 1)
    ewidth = [int(v) for v in np.frombuffer(buf, "<u4", L + 1, pos)]
    pos += 4 * (L + 1)
    if sum(ecount) != nout or any(w > 64 for w in ewidth):
        raise ValueError("escape table")
    off = {"code_len": pos}
    pos += dsz
    off["chunk_bits"] = pos
    pos += 4 * nch
    off["chunk_esc"] = pos
    pos += 4 * nch
    off["payload"] = pos
    pos += 4 * nw
    off["escapes"] = pos
    pos += 4 * sum(Q.escape_words(ecount, ewidth))
    off["end"] = pos
    if pos > len(buf):
        raise ValueError("truncated buffer")
    return Header(np.float32 if dt == 0 else np.float64, D, bool(rel), al, fb, L, dsz, ch, tol, tau,
                  mx, n, nch, nout, nw, norm, s, shape, coords, bins, ecount, ewidth, off)


def decompress(buf: bytes):
    h = parse(buf)
    hier = Hierarchy(h.shape, h.coords)
    lengths = np.frombuffer(buf, np.uint8, h.dict_size, h.offsets["code_len"]).astype(np.int64)
    codes = H.canonical_codes(lengths)
    cbits = [int(v) for v in np.frombuffer(buf, "<u4", h.n_chunks, h.offsets["chunk_bits"])]
    words = [int(v) for v in np.frombuffer(buf, "<u4", h.payload_words, h.offsets["payload"])]
    nesc = sum(Q.escape_words(h.esc_counts, h.esc_widths))
    outl = Q.unpack_escapes(np.frombuffer(buf, "<u4", nesc, h.offsets["escapes"]), h.esc_counts, h.esc_widths,
                            h.dict_size)
    sym = H.decode(words, cbits, lengths, codes, h.n, h.chunk)
    q = Q.from_symbols(sym, outl, h.dict_size)
    stream = Q.dequantize_stream(q, hier, h.bins, h.dtype)
    coarsest, cbars = Q.from_stream(stream, hier, h.dtype)
    return X.recompose(coarsest, cbars, hier, h.dtype)
