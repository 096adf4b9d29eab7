"""Out-of-core (chunked) compression of a host-resident array (oracle).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

The paper's high-level API takes arrays larger than device memory: its
out-of-core layer partitions the array into chunks that fit on the device and
streams them through the compressor (Sec. 2.1, high-level APIs; Sec. 2.2,
software architecture).  The paper fixes neither the chunk shape nor the
container, so this reading is taken:

* chunks are slabs of `slab` planes along the slowest dimension (dimension 0),
  the last one ending at n0; a last slab of fewer than 3 planes joins the one
  before it (a slab is a grid of its own and needs 3 nodes per side to form
  a level);
* every slab is compressed as an independent field with the absolute
  tolerance the whole array implies (relative: tol * max |u| over the whole
  array), so the L-infinity bound holds on every slab and therefore on the
  array; a nonuniform dimension 0 passes each slab its own coordinates;
* the slabs' self-describing streams (codec module) follow a fixed header.

Container (little-endian; offsets in bytes):

    0  'MGCK'            magic
    4  u32 version = 1
    8  u32 ndim
   12  u32 dtype          0 = float32, 1 = float64
   16  u64 shape[4]       unused dimensions 0
   48  u64 slab           planes per slab as requested
   56  u64 n_slabs
   64  f64 tol
   72  u32 eb             0 = absolute, 1 = relative to max |u|
   76  u32 0
   80  f64 tau_abs        the absolute tolerance every slab was compressed with
   88  u64 offsets[n_slabs + 1]   byte offset of each slab's stream; the last
                                  is the container's length
       slab streams
"""
from __future__ import annotations

import struct

import numpy as np

from . import alloc as A
from . import codec

MAGIC = b"MGCK"
VERSION = 1
FIXED = 88


def slab_bounds(n0: int, slab: int):
    """[(p0, p1)] of the slabs along dimension 0 (the reading above)."""
    if slab < 3:
        raise ValueError("slab must hold at least 3 planes")
    b = [(p, min(p + slab, n0)) for p in range(0, n0, slab)]
    if len(b) > 1 and b[-1][1] - b[-1][0] < 3:
        b[-2] = (b[-2][0], n0)
        b.pop()
    return b


def compress_chunked(u, tol, slab, rel=True, coords=None, dict_size=8192, chunk=1024):
    u = np.ascontiguousarray(u)
    T = u.dtype.type
    bounds = slab_bounds(u.shape[0], slab)
    maxabs = float(np.abs(u).max())
    tau = A.tau_abs(tol, maxabs, rel)
    streams = []
    for p0, p1 in bounds:
        cc = None
        if coords is not None:
            cc = [None if c is None else np.asarray(c, dtype=np.float64) for c in coords]
            if cc[0] is not None:
                cc[0] = cc[0][p0:p1]
        streams.append(codec.compress(u[p0:p1], tau, rel=False, coords=cc, dict_size=dict_size, chunk=chunk))
    head = FIXED + 8 * (len(bounds) + 1)
    offs = [head]
    for s in streams:
        offs.append(offs[-1] + len(s))
    shape4 = list(u.shape) + [0] * (4 - u.ndim)
    hdr = MAGIC + struct.pack("<III4QQQdIId", VERSION, u.ndim, 0 if T == np.float32 else 1, *shape4, slab,
                              len(bounds), float(tol), 1 if rel else 0, 0, tau)
    assert len(hdr) == FIXED
    return hdr + struct.pack(f"<{len(offs)}Q", *offs) + b"".join(streams)


def parse_chunked(buf: bytes):
    if buf[:4] != MAGIC:
        raise ValueError("not a chunked container")
    ver, ndim, dt, s0, s1, s2, s3, slab, ns, tol, eb, _, tau = struct.unpack("<III4QQQdIId", buf[4:FIXED])
    if ver != VERSION:
        raise ValueError("container version")
    shape = (s0, s1, s2, s3)[:ndim]
    offs = struct.unpack(f"<{ns + 1}Q", buf[FIXED:FIXED + 8 * (ns + 1)])
    return {"ndim": ndim, "dtype": dt, "shape": shape, "slab": slab, "n_slabs": ns, "tol": tol, "eb": eb,
            "tau_abs": tau, "offsets": offs}


def decompress_chunked(buf: bytes):
    c = parse_chunked(buf)
    T = np.float32 if c["dtype"] == 0 else np.float64
    out = np.empty(c["shape"], dtype=T)
    bounds = slab_bounds(c["shape"][0], c["slab"])
    assert len(bounds) == c["n_slabs"]
    offs = c["offsets"]
    for k, (p0, p1) in enumerate(bounds):
        out[p0:p1] = codec.decompress(buf[offs[k]:offs[k + 1]])
    return out
