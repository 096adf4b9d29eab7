"""Histogram, Huffman codebook and chunked bit packing (oracle).

The paper compresses the quantized integers losslessly before writing them
(Sec. 2, final stage).  The coder used here is a canonical Huffman code over a
fixed-size symbol dictionary; the paper does not fix its details, so the
following rules are chosen to make the output reproducible bit for bit:

* code lengths: leaves are the symbols with nonzero count sorted by
  (count, symbol); two FIFO queues (leaves, merged nodes); each merge takes
  the smaller head, the leaf queue winning ties, and the merged weight is the
  sum; a symbol's length is its leaf depth.  One distinct symbol gets length
  1; an empty stream gets no codes;
* canonical codes: symbols ordered by (length, symbol), first code 0, then
  code_k = (code_{k-1} + 1) << (len_k - len_{k-1});
* packing: the stream is cut into chunks of ``chunk`` symbols; each chunk's
  codes are concatenated most-significant-bit first into 32-bit words (first
  bit at bit 31), the chunk starts word-aligned and ends zero-padded, and its
  bit count is recorded.  The payload is the chunks in order.

Written with plain Python loops: meant for the small inputs of the tests.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def histogram(symbols, dict_size: int) -> np.ndarray:
    return np.bincount(np.asarray(symbols, dtype=np.int64), minlength=dict_size).astype(np.int64)


def code_lengths(counts) -> np.ndarray:
    counts = [int(c) for c in counts]
    n = len(counts)
    lengths = np.zeros(n, dtype=np.int64)
    leaves = sorted((c, s) for s, c in enumerate(counts) if c > 0)
    if not leaves:
        return lengths
    if len(leaves) == 1:
        lengths[leaves[0][1]] = 1
        return lengths
    weight = [c for c, _ in leaves]
    parent = [-1] * len(leaves)
    leafq = deque(range(len(leaves)))
    nodeq = deque()

    def pop():
        if leafq and (not nodeq or weight[leafq[0]] <= weight[nodeq[0]]):
            return leafq.popleft()
        return nodeq.popleft()

    while len(leafq) + len(nodeq) > 1:
        a = pop()
        b = pop()
        k = len(weight)
        weight.append(weight[a] + weight[b])
        parent.append(-1)
        parent[a] = k
        parent[b] = k
        nodeq.append(k)
    depth = [0] * len(weight)
    for k in range(len(weight) - 2, -1, -1):  # parents are created after their children
        depth[k] = depth[parent[k]] + 1
    for i, (_, s) in enumerate(leaves):
        lengths[s] = depth[i]
    return lengths


def canonical_codes(lengths) -> np.ndarray:
    lengths = [int(v) for v in lengths]
    codes = np.zeros(len(lengths), dtype=np.uint64)
    order = sorted((L, s) for s, L in enumerate(lengths) if L > 0)
    code = 0
    prev = None
    for L, s in order:
        if prev is not None:
            code = (code + 1) << (L - prev)
        codes[s] = code
        prev = L
    return codes


def encode(symbols, lengths, codes, chunk: int):
    """Returns (chunk_bits list, payload words list of ints)."""
    lengths = [int(v) for v in lengths]
    codes = [int(v) for v in codes]
    symbols = [int(v) for v in symbols]
    chunk_bits = []
    words = []
    for start in range(0, len(symbols), chunk):
        buf = 0
        nb = 0
        total = 0
        for s in symbols[start:start + chunk]:
            L = lengths[s]
            if L == 0:
                raise ValueError("symbol without a code")
            buf = (buf << L) | codes[s]
            nb += L
            total += L
            while nb >= 32:
                nb -= 32
                words.append((buf >> nb) & 0xFFFFFFFF)
                buf &= (1 << nb) - 1
        if nb:
            words.append((buf << (32 - nb)) & 0xFFFFFFFF)
        chunk_bits.append(total)
    return chunk_bits, words


def decode(words, chunk_bits, lengths, codes, n: int, chunk: int):
    lengths = [int(v) for v in lengths]
    table = {(int(lengths[s]), int(codes[s])): s for s in range(len(lengths)) if lengths[s] > 0}
    out = []
    w0 = 0
    for k, nbits in enumerate(chunk_bits):
        count = min(chunk, n - k * chunk)
        nwords = (int(nbits) + 31) // 32
        bits = 0
        for w in words[w0:w0 + nwords]:
            bits = (bits << 32) | int(w)
        total = 32 * nwords
        pos = 0
        for _ in range(count):
            code = 0
            L = 0
            while True:
                if pos >= nbits:
                    raise ValueError("chunk payload ends inside a code")
                bit = (bits >> (total - 1 - pos)) & 1
                pos += 1
                code = (code << 1) | bit
                L += 1
                s = table.get((L, code))
                if s is not None:
                    out.append(s)
                    break
        if pos != nbits:
            raise ValueError("chunk bit count does not match its codes")
        w0 += nwords
    return np.asarray(out, dtype=np.int64)
