"""Second-stage lossless coder: zero suppression by two-level bitmaps (oracle).

Test infrastructure only, like the rest of this package.

The paper ends its pipeline with a lossless stage after the entropy coder
(Sec. 2: quantization or precision segments "are compressed through lossless
encoding"; the code table lists a general-purpose lossless library for it).
The reading used here keeps what that stage removes from this pipeline's
output -- runs of zero bits: the all-zero shortest code of a dominant
Huffman symbol, and the high bitplanes of the refactoring, whose words are
mostly zero -- and codes every chunk independently so that a GPU encodes and
decodes all of them at once:

* the input is a byte string, padded with zero bytes to whole little-endian
  32-bit words;
* words are grouped into chunks of C = 4096 (the last may be shorter, m
  words);
* level-1 bitmap: ceil(m/32) words, bit 31 - i%32 of word i/32 set when data
  word i is nonzero; level-2 bitmap: ceil(ceil(m/32)/32) words, the same for
  the level-1 words;
* a coded chunk is the level-2 bitmap, then the nonzero level-1 words, then
  the nonzero data words, each in order; when that is not shorter than m
  words the chunk is stored raw.  A chunk's stored length tells which: m
  words means raw, fewer means coded.

Container (little-endian):

    0  'MGZS'        magic
    4  u16 version = 1
    6  u16 zero
    8  u64 raw_bytes
   16  u64 n_chunks
   24  u64 offset[n_chunks + 1]   word offsets of the chunks in the data area
       u32 data[offset[n_chunks]]
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"MGZS"
VERSION = 1
CHUNK = 4096
FIXED = 24


def _bitmap(nonzero):
    bits = np.asarray(nonzero, dtype=np.uint8)
    pad = (-len(bits)) % 32
    b = np.concatenate([bits, np.zeros(pad, dtype=np.uint8)])
    return np.frombuffer(np.packbits(b).tobytes(), dtype=">u4").astype(np.uint32)


def _unbitmap(words, n):
    w = np.asarray(words, dtype=np.uint32).astype(">u4")
    return np.unpackbits(w.view(np.uint8))[:n].astype(bool)


def code_chunk(w):
    """Stored words of one chunk (coded, or the chunk itself when that is not shorter)."""
    w = np.asarray(w, dtype=np.uint32)
    m = len(w)
    b1 = _bitmap(w != 0)
    b2 = _bitmap(b1 != 0)
    coded = np.concatenate([b2, b1[b1 != 0], w[w != 0]]).astype(np.uint32)
    return coded if len(coded) < m else w.copy()


def decode_chunk(stored, m):
    stored = np.asarray(stored, dtype=np.uint32)
    if len(stored) == m:
        return stored.copy()
    if len(stored) > m:
        raise ValueError("chunk longer than raw")
    n1 = (m + 31) // 32
    n2 = (n1 + 31) // 32
    if len(stored) < n2:
        raise ValueError("truncated chunk")
    b2 = stored[:n2]
    nz1 = _unbitmap(b2, n1)
    k1 = int(nz1.sum())
    if len(stored) < n2 + k1:
        raise ValueError("truncated chunk")
    b1 = np.zeros(n1, dtype=np.uint32)
    b1[nz1] = stored[n2:n2 + k1]
    if np.any(b1[nz1] == 0):
        raise ValueError("zero level-1 word marked nonzero")
    nz = _unbitmap(b1, m)
    if len(stored) != n2 + k1 + int(nz.sum()):
        raise ValueError("chunk length does not match its bitmaps")
    out = np.zeros(m, dtype=np.uint32)
    out[nz] = stored[n2 + k1:]
    return out


def words_of(data: bytes) -> np.ndarray:
    pad = (-len(data)) % 4
    return np.frombuffer(bytes(data) + b"\0" * pad, dtype="<u4").astype(np.uint32)


def encode(data: bytes) -> bytes:
    w = words_of(data)
    nch = (len(w) + CHUNK - 1) // CHUNK
    parts, offs = [], [0]
    for k in range(nch):
        c = code_chunk(w[k * CHUNK:(k + 1) * CHUNK])
        parts.append(c)
        offs.append(offs[-1] + len(c))
    head = struct.pack("<4sHHQQ", MAGIC, VERSION, 0, len(data), nch)
    body = np.concatenate(parts).astype("<u4").tobytes() if parts else b""
    return head + np.asarray(offs, dtype="<u8").tobytes() + body


def decode(buf: bytes) -> bytes:
    if len(buf) < FIXED or buf[:4] != MAGIC:
        raise ValueError("not a zero-suppressed buffer")
    _, ver, _, raw, nch = struct.unpack_from("<4sHHQQ", buf, 0)
    if ver != VERSION:
        raise ValueError("unsupported version")
    nwords = (raw + 3) // 4
    if nch != (nwords + CHUNK - 1) // CHUNK:
        raise ValueError("chunk count")
    offs = np.frombuffer(buf, "<u8", nch + 1, FIXED)
    data = np.frombuffer(buf, "<u4", int(offs[-1]), FIXED + 8 * (nch + 1))
    out = []
    for k in range(nch):
        m = min(CHUNK, nwords - k * CHUNK)
        out.append(decode_chunk(data[offs[k]:offs[k + 1]], m))
    w = np.concatenate(out) if out else np.zeros(0, dtype=np.uint32)
    return w.astype("<u4").tobytes()[:raw]
