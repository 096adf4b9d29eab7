"""Refactoring into precision segments, greedy retrieval and recomposition (oracle).

Test infrastructure only, like the rest of this package.

The paper's second module (Sec. 2, software design) refactors the multilevel
coefficients into precision segments of different significance per level by
bitplane encoding, accumulates the error that each segment removes, and on
retrieval fetches, greedily, the segment that lowers the error estimate the
most, then recomposes; the second listing of Sec. 3 requests a tolerance,
asks which components are needed, and reconstructs, tolerance after
tolerance.  The paper gives no formulas; the readings used here:

* coefficients: the stream of the decomposition in the working type T
  (transform.py, quant.py stream order); level l is its range
  [off_l, off_{l+1});
* level exponent: with M_l = max |c| over the level, e_l is the integer with
  M_l = f 2^e_l, 1/2 <= f < 1, so every |c| < 2^e_l (none for an all-zero
  level);
* B bitplanes (1 <= B <= 32): the magnitude integer m = floor(|c| 2^(B - e_l))
  < 2^B, exact in float64 (a scaling by a power of two, then a floor); the
  sign bit is c < 0;
* precision segments of a level, in this order: the sign plane, then
  magnitude planes k = 0 .. B-1, plane k holding bit B-1-k of every m.  A
  plane packs the level's coefficients in stream order, most significant
  bit first, into 32-bit words (coefficient i of the level at bit 31 - i%32
  of word i/32), W_l = ceil(N_l / 32) words per plane;
* error accumulation: R_l[k] = max over the level of (m mod 2^(B-k)),
  k = 0 .. B, the largest magnitude residual, in units of 2^(e_l - B), that
  is left when the first k planes are known;
* reconstruction from k planes: m_k = m with its low B-k bits cleared,
  c^ = T(+-m_k 2^(e_l - B)).  Then |c - c^| <= E_l[k] with
  E_l[k] = (R_l[k] + 1) 2^(e_l - B) + [k > 0] eps_T 2^e_l, the last term
  covering the rounding of c^ to T;
* estimator, L-infinity (the bound of the compression allocation, alloc.py,
  with per-level errors E_l[k_l] in place of b_l/2):
  est = rho + E_0[k_0] + sum_{l>=1} (1 + K_l) E_l[k_l],
  rho = 4 (L+1) eps_T ||u||_inf the transform's rounding reserve;
  s-norm (snorm.py): est = rho max(1, 2^(s L)) sqrt(W_0)
  + sqrt(sum_l 4^(s l) W_l E_l[k_l]^2);
* greedy retrieval: starting from the planes already held (none at first),
  while est > tau, fetch the next plane of the level with the largest
  decrease of the estimator's level term per byte fetched (the sign plane
  is fetched with a level's first magnitude plane); ties go to the lowest
  level.  The level term is w_l E_l (w_0 = 1, w_l = 1 + K_l) for the
  L-infinity estimator and 4^(s l) W_l E_l^2 for the s-norm.  A request
  starts from the planes held, so a tighter tolerance only adds segments;
* relative tolerances: tau = tol ||u||_inf (L-infinity), tau = tol ||u||
  (s-norm with s = 0), both norms recorded at refactoring.

Metadata (little-endian; the segment area follows at offset meta_bytes):

    0  'MGRF'          magic
    4  u16 version = 1
    6  u8  dtype        0 = float32, 1 = float64
    7  u8  ndim
    8  u8  planes B
    9  u8  coord_flags  bit d: dimension d stores its coordinates
   10  u16 zero
   12  u32 L
   16  f64 maxabs       ||u||_inf
   24  f64 l2norm       ||u|| (P1 mass matrix)
   32  u64 shape[ndim]
       f64 coords       for each flagged dimension, its coordinates
       i32 exponent[L+1]       e_l, or -2^31 for an all-zero level
       u32 R[(L+1) (B+1)]      level-major
       u64 level_offset[L+2]   byte offset of each level's sign plane in the
                               segment area (the last: the area's size)
       zero padding to a multiple of 8 bytes

Segment area: per level, the sign plane then planes 0 .. B-1.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass

import numpy as np

from . import alloc as A
from . import quant as Q
from . import snorm as SN
from . import transform as X
from .grid import Hierarchy

MAGIC = b"MGRF"
VERSION = 1
FIXED = 32
NO_EXP = -(2 ** 31)


def level_exponent(maxabs_level: float):
    """e with maxabs = f 2^e, 1/2 <= f < 1 (None for 0)."""
    if maxabs_level == 0.0:
        return None
    return math.frexp(float(maxabs_level))[1]


def magnitudes(c, e, B):
    """m = floor(|c| 2^(B - e)) as uint64, and the sign bits."""
    a = np.abs(np.asarray(c).astype(np.float64))
    m = np.floor(np.ldexp(a, B - e)).astype(np.uint64)
    s = (np.asarray(c) < 0).astype(np.uint64)
    return m, s


def pack_bits(bits):
    """0/1 values -> 32-bit words, element i at bit 31 - i % 32 of word i // 32."""
    bits = np.asarray(bits, dtype=np.uint8)
    pad = (-len(bits)) % 32
    b = np.concatenate([bits, np.zeros(pad, dtype=np.uint8)])
    return np.frombuffer(np.packbits(b).tobytes(), dtype=">u4").astype(np.uint32)


def unpack_bits(words, n):
    w = np.asarray(words, dtype=np.uint32).astype(">u4")
    return np.unpackbits(w.view(np.uint8))[:n].astype(np.uint64)


def residual_table(m, B):
    """R[k] = max(m mod 2^(B-k)), k = 0..B (zeros for an empty level)."""
    out = []
    for k in range(B + 1):
        mask = np.uint64((1 << (B - k)) - 1)
        out.append(int((m & mask).max()) if len(m) else 0)
    return out


@dataclass
class Refactored:
    hier: Hierarchy
    T: type
    B: int
    maxabs: float
    l2norm: float
    exps: list
    R: list  # per level, B+1 integers
    planes: list  # per level: list of B+1 word arrays (sign plane first)
    coords: list


def words_per_plane(n: int) -> int:
    return (n + 31) // 32


def refactor(u, B=32, coords=None, l2norm=None) -> Refactored:
    """l2norm, when given, replaces ||u|| computed here (a float64 sum that
    another implementation took in another order)."""
    u = np.asarray(u)
    T = u.dtype.type
    if T not in (np.float32, np.float64):
        raise TypeError("float32 or float64 input")
    if not 1 <= B <= 32:
        raise ValueError("1 <= B <= 32 bitplanes")
    if not np.all(np.isfinite(u)):
        raise ValueError("non-finite input")
    hier = Hierarchy(u.shape, coords)
    maxabs = float(np.max(np.abs(u))) if u.size else 0.0
    l2 = math.sqrt(SN.l2_norm_sq(u, hier)) if l2norm is None else float(l2norm)
    coarsest, cbars = X.decompose(u, hier, T)
    stream = Q.to_stream(coarsest, cbars, hier)
    off = Q.level_offsets(hier)
    exps, R, planes = [], [], []
    for l in range(hier.L + 1):
        c = stream[off[l]:off[l + 1]]
        e = level_exponent(float(np.max(np.abs(c.astype(np.float64))))) if len(c) else None
        exps.append(e)
        if e is None:
            m = np.zeros(len(c), dtype=np.uint64)
            s = np.zeros(len(c), dtype=np.uint64)
        else:
            m, s = magnitudes(c, e, B)
        R.append(residual_table(m, B))
        segs = [pack_bits(s)]
        for k in range(B):
            segs.append(pack_bits((m >> np.uint64(B - 1 - k)) & np.uint64(1)))
        planes.append(segs)
    return Refactored(hier, T, B, maxabs, l2, exps, R, planes, coords)


def level_offsets_bytes(hier: Hierarchy, B: int):
    counts = hier.level_counts()
    out = [0]
    for n in counts:
        out.append(out[-1] + 4 * (B + 1) * words_per_plane(n))
    return out


def serialize(r: Refactored) -> bytes:
    hier = r.hier
    D = hier.D
    flags = 0
    blob = b""
    if r.coords is not None:
        for d in range(D):
            if r.coords[d] is not None:
                flags |= 1 << d
                blob += np.asarray(r.coords[d], dtype="<f8").tobytes()
    head = struct.pack("<4sHBBBBHIdd", MAGIC, VERSION, 0 if r.T is np.float32 else 1, D, r.B, flags, 0, hier.L,
                       float(r.maxabs), float(r.l2norm))
    assert len(head) == FIXED
    parts = [head, np.asarray(hier.shape, dtype="<u8").tobytes(), blob,
             np.asarray([NO_EXP if e is None else e for e in r.exps], dtype="<i4").tobytes(),
             np.asarray([v for row in r.R for v in row], dtype="<u4").tobytes(),
             np.asarray(level_offsets_bytes(hier, r.B), dtype="<u8").tobytes()]
    meta = b"".join(parts)
    meta += b"\0" * ((-len(meta)) % 8)
    segs = b"".join(np.asarray(p, dtype="<u4").tobytes() for lv in r.planes for p in lv)
    return meta + segs


@dataclass
class Meta:
    T: type
    B: int
    L: int
    maxabs: float
    l2norm: float
    shape: tuple
    coords: list
    exps: list
    R: list
    level_off: list
    meta_bytes: int


def parse(buf: bytes) -> Meta:
    if len(buf) < FIXED or buf[:4] != MAGIC:
        raise ValueError("not a refactored buffer")
    _, ver, dt, D, B, flags, _, L, mx, l2 = struct.unpack_from("<4sHBBBBHIdd", buf, 0)
    if ver != VERSION or dt > 1 or not 1 <= D <= 4 or not 1 <= B <= 32:
        raise ValueError("unsupported metadata")
    pos = FIXED
    shape = tuple(int(v) for v in np.frombuffer(buf, "<u8", D, pos))
    pos += 8 * D
    coords = [None] * D
    for d in range(D):
        if (flags >> d) & 1:
            coords[d] = np.frombuffer(buf, "<f8", shape[d], pos).copy()
            pos += 8 * shape[d]
    exps = [None if v == NO_EXP else int(v) for v in np.frombuffer(buf, "<i4", L + 1, pos)]
    pos += 4 * (L + 1)
    flat = [int(v) for v in np.frombuffer(buf, "<u4", (L + 1) * (B + 1), pos)]
    pos += 4 * (L + 1) * (B + 1)
    R = [flat[l * (B + 1):(l + 1) * (B + 1)] for l in range(L + 1)]
    loff = [int(v) for v in np.frombuffer(buf, "<u8", L + 2, pos)]
    pos += 8 * (L + 2)
    pos += (-pos) % 8
    return Meta(np.float32 if dt == 0 else np.float64, B, L, mx, l2, shape, coords, exps, R, loff, pos)


def level_errors(meta: Meta, l: int):
    """E_l[k], k = 0..B (zeros for an all-zero level)."""
    e = meta.exps[l]
    B = meta.B
    if e is None:
        return [0.0] * (B + 1)
    eps = float(np.finfo(meta.T).eps)
    out = []
    for k in range(B + 1):
        v = math.ldexp(float(meta.R[l][k] + 1), e - B)
        if k > 0:
            v += math.ldexp(eps, e)
        out.append(v)
    return out


class Estimator:
    """Level weights and the estimate of a plane allocation (see the module docstring)."""

    def __init__(self, meta: Meta, norm: str = "linf", s: float = 0.0):
        self.meta = meta
        self.norm = norm
        self.s = s
        hier = Hierarchy(meta.shape, meta.coords)
        self.hier = hier
        L = meta.L
        rho = 4.0 * (L + 1) * float(np.finfo(meta.T).eps) * meta.maxabs
        self.E = [level_errors(meta, l) for l in range(L + 1)]
        if norm == "linf":
            K = A.level_K(hier)
            self.w = [1.0] + [1.0 + K[l] for l in range(1, L + 1)]
            self.reserve = rho
        elif norm == "s":
            W = SN.level_weights(hier)
            self.w = [float(np.power(2.0, 2.0 * s * l)) * W[l] for l in range(L + 1)]
            self.reserve = rho * SN.reserve_factor(hier, s)
        else:
            raise ValueError("norm is 'linf' or 's'")
        counts = hier.level_counts()
        self.plane_bytes = [4 * words_per_plane(n) for n in counts]

    def term(self, l: int, k: int) -> float:
        e = self.E[l][k]
        return self.w[l] * e if self.norm == "linf" else self.w[l] * e * e

    def estimate(self, ks) -> float:
        tot = 0.0
        for l in range(self.meta.L + 1):
            tot += self.term(l, ks[l])
        return self.reserve + (tot if self.norm == "linf" else math.sqrt(tot))

    def cost(self, l: int, k: int) -> float:
        return float(self.plane_bytes[l] * (2 if k == 0 else 1))


def tau_of(meta: Meta, tol: float, rel: bool, norm: str, s: float) -> float:
    if not rel:
        return tol
    if norm == "linf":
        return tol * meta.maxabs
    if s != 0.0:
        raise ValueError("a relative s-norm bound needs s = 0")
    return tol * meta.l2norm


def request(meta: Meta, tol: float, rel: bool = True, norm: str = "linf", s: float = 0.0, have=None):
    """Planes per level to hold so that the estimate meets tau, starting from `have`
    (planes already held); returns (planes, estimate)."""
    if not tol > 0.0:
        raise ValueError("tolerance must be positive")
    est = Estimator(meta, norm, s)
    tau = tau_of(meta, tol, rel, norm, s)
    L, B = meta.L, meta.B
    k = [0] * (L + 1) if have is None else [int(v) for v in have]
    if len(k) != L + 1 or any(not 0 <= v <= B for v in k):
        raise ValueError("held planes")
    active = [e is not None for e in meta.exps]
    k = greedy(est, tau, k, B, active)
    return k, est.estimate(k)


def greedy(est, tau: float, k, B: int, active):
    """Adds one plane at a time, to the active level with the largest term decrease
    per byte (lowest level on ties), until est.estimate(k) <= tau or every plane is held."""
    k = list(k)
    while est.estimate(k) > tau:
        best, best_ratio = -1, 0.0
        for l in range(len(k)):
            if k[l] >= B or not active[l]:
                continue
            gain = est.term(l, k[l]) - est.term(l, k[l] + 1)
            ratio = gain / est.cost(l, k[l])
            if best < 0 or ratio > best_ratio:
                best, best_ratio = l, ratio
        if best < 0:
            break
        k[best] += 1
    return k


def segment_ranges(meta: Meta, have, want):
    """Byte ranges (offset from the start of the buffer, length) to fetch to go from
    `have` to `want` planes per level: one contiguous range per level at most."""
    out = []
    for l in range(meta.L + 1):
        h, w = int(have[l]), int(want[l])
        if w <= h:
            continue
        pb = (meta.level_off[l + 1] - meta.level_off[l]) // (meta.B + 1)
        first = 0 if h == 0 else h + 1  # plane slots: 0 = sign, 1 + k = magnitude plane k
        last = w + 1
        out.append((meta.meta_bytes + meta.level_off[l] + first * pb, (last - first) * pb))
    return out


def reconstruct_stream(buf: bytes, meta: Meta, planes):
    """Coefficient stream (type T) from the first planes[l] planes of every level."""
    hier = Hierarchy(meta.shape, meta.coords)
    counts = hier.level_counts()
    T = meta.T
    B = meta.B
    out = []
    for l in range(meta.L + 1):
        n = counts[l]
        k = int(planes[l])
        e = meta.exps[l]
        if k == 0 or e is None:
            out.append(np.zeros(n, dtype=T))
            continue
        W = words_per_plane(n)
        base = meta.meta_bytes + meta.level_off[l]
        sign = unpack_bits(np.frombuffer(buf, "<u4", W, base), n)
        m = np.zeros(n, dtype=np.uint64)
        for j in range(k):
            bits = unpack_bits(np.frombuffer(buf, "<u4", W, base + 4 * W * (1 + j)), n)
            m |= bits << np.uint64(B - 1 - j)
        mag = np.ldexp(m.astype(np.float64), e - B)
        out.append(np.where(sign == 1, -mag, mag).astype(T))
    return np.concatenate(out)


def reconstruct(buf: bytes, planes):
    meta = parse(buf)
    hier = Hierarchy(meta.shape, meta.coords)
    stream = reconstruct_stream(buf, meta, planes)
    coarsest, cbars = Q.from_stream(stream, hier, meta.T)
    return X.recompose(coarsest, cbars, hier, meta.T)
