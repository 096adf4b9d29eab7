"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle cannot decompose a 513^3 or 500^3 field in seconds, so these tests
check what it can compute one node at a time, plus properties that hold at any
size:

* finest-level coefficients (the residual of the multilinear interpolation,
  Sec. 2.2) at sampled nodes, bit-exact, found through the stream layout the
  oracle defines (level by level, sub-grids in mask order);
* whole compressed chunks of the finest level: the oracle quantizes its own
  coefficients with its own bins (Sec. 2.3, plain allocation), maps them to
  symbols and decodes the chunk from the library's payload with its own
  bit-serial decoder: symbols, outliers and chunk bit counts must agree
  exactly, including the ragged last chunk of the stream;
* the header's max |u|, tau and bins against the oracle's;
* the code lengths form a complete prefix code (Kraft sum 1);
* decompose then recompose returns the input within the rounding reserve the
  error budget sets aside, 4 (L + 1) eps max |u|;
* the decompressed field is within tau of the input.

Workloads: 513^3 float32 spectral k^-5/3 (seed 2) at rel tol 1e-2, 1e-3, 1e-4;
500^3 float64 with geometric coordinates (ratio 1.01 per dimension), spectral
k^-3 plus a tanh front (seed 3), at rel tol 1e-4.
"""
import math

import numpy as np
import pytest

import fieldgen
from oracle import alloc as A
from oracle import codec
from oracle import huffman as H
from oracle import quant as Q
from oracle import transform as X
from oracle.grid import Hierarchy

pytestmark = pytest.mark.gpu


def say(*a):
    print("[fullsize]", *a, flush=True)


class Layout:
    """Node <-> stream position for the finest level, from the oracle's sub-grid sets."""

    def __init__(self, hier):
        self.h = hier
        self.L = hier.L
        self.off = Q.level_offsets(hier)
        self.sets = Q.level_subgrids(hier, self.L)
        self.shapes = [tuple(len(s) for s in sets) for sets in self.sets]
        sizes = [int(np.prod(s)) for s in self.shapes]
        self.sub_start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    def node_of(self, pos):
        """Grid node of stream position pos (which must lie in the finest level)."""
        j = int(pos - self.off[self.L])
        m = int(np.searchsorted(self.sub_start, j, side="right")) - 1
        idx = np.unravel_index(j - int(self.sub_start[m]), self.shapes[m])
        return tuple(int(self.sets[m][d][idx[d]]) for d in range(self.h.D))

    def pos_of(self, p):
        D = self.h.D
        m = 0
        local = []
        for d in range(D):
            f = self.h.fidx(self.L, d)
            k = int(np.searchsorted(f, p[d]))
            if k < len(f) and f[k] == p[d]:
                m |= 1 << d
                local.append(k)
            else:
                local.append(int(np.searchsorted(self.h.cidx(self.L, d), p[d])))
        assert m != 0, "coarse node"
        sub = m - 1
        return int(self.off[self.L] + self.sub_start[sub] + np.ravel_multi_index(local, self.shapes[sub]))


def _field_513(torch):
    say("generate 513^3 f32 spectral k^-5/3 seed 2")
    u = fieldgen.spectral((513, 513, 513), -5.0 / 3.0, 2, device="cuda").to(torch.float32).contiguous()
    return u, None


def _field_500(torch):
    say("generate 500^3 f64 geometric front seed 3")
    u, coords = fieldgen.front3d(500, 3, 1.01, device="cuda")
    return u.to(torch.float64).contiguous(), coords


WORKLOADS = {"513f32": (_field_513, np.float32, [1e-2, 1e-3, 1e-4]),
             "500f64": (_field_500, np.float64, [1e-4])}


@pytest.fixture(scope="module")
def cache():
    d = {}
    yield d
    d.clear()


def _setup(lib, cache, name):
    import torch

    if cache.get("name") != name:
        cache.clear()
        torch.cuda.empty_cache()
        make, T, tols = WORKLOADS[name]
        u, coords = make(torch)
        say("autotune", tuple(u.shape))
        lib.mgard_autotune(u, coords)
        uh = u.cpu().numpy()
        hier = Hierarchy(u.shape, coords)
        cache.update(name=name, u=u, coords=coords, uh=uh, hier=hier, lay=Layout(hier), T=T, tols=tols)
    return cache


def _sample_fine_nodes(hier, rng, k):
    shape = hier.shape
    pts = []
    fine = [np.zeros(n, dtype=bool) for n in shape]
    for d in range(hier.D):
        fine[d][hier.fidx(hier.L, d)] = True
    # the faces and corners of the grid's far end, where the last (possibly
    # uneven) interval sits, then uniform samples
    n = shape
    for p in [(1, 1, 1), (n[0] - 2, n[1] - 2, n[2] - 2), (n[0] - 2, 0, n[2] - 1), (0, n[1] - 2, 1),
              (n[0] - 1, n[1] - 1, n[2] - 2), (1, n[1] - 1, 0)]:
        if any(fine[d][p[d]] for d in range(3)):
            pts.append(p)
    while len(pts) < k:
        p = tuple(int(rng.integers(0, s)) for s in shape)
        if any(fine[d][p[d]] for d in range(3)):
            pts.append(p)
    return pts


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_decompose(lib, cache, name):
    import torch

    c = _setup(lib, cache, name)
    u, uh, hier, lay, T = c["u"], c["uh"], c["hier"], c["lay"], c["T"]
    L, offs = lib.mgard_stream_layout(u.shape)
    assert L == hier.L and offs == [int(v) for v in lay.off]
    say("decompose", name)
    coeff = lib.mgard_decompose(u, c["coords"])
    pts = _sample_fine_nodes(hier, np.random.default_rng(5), 3000)
    pos = [lay.pos_of(p) for p in pts]
    for p, q in zip(pts[:50], pos[:50]):
        assert lay.node_of(q) == p
    got = coeff[torch.tensor(pos, device=u.device)].cpu().numpy()
    want = np.array([X.coefficient_at(uh, hier, p, T) for p in pts], dtype=T)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(pts[i], float(got[i]), float(want[i])) for i in bad[:5]]
    say("recompose", name)
    rec = lib.mgard_recompose(coeff, u.shape, c["coords"])
    del coeff
    maxabs = float(np.abs(uh).max())
    err = float((rec - u).abs().max())
    reserve = 4.0 * (hier.L + 1) * float(np.finfo(T).eps) * maxabs
    say("decompose-recompose L_inf", err, "reserve", reserve)
    assert err <= reserve


def _expected_chunk(uh, hier, lay, T, bins, start, count, dict_size, memo):
    vals = []
    for j in range(start, start + count):
        if j not in memo:
            memo[j] = X.coefficient_at(uh, hier, lay.node_of(j), T)
        vals.append(memo[j])
    q = Q.quantize(np.array(vals, dtype=T), bins[hier.L])
    return Q.to_symbols(q, dict_size)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_compressed_chunks_and_roundtrip(lib, cache, name):
    c = _setup(lib, cache, name)
    u, uh, hier, lay, T = c["u"], c["uh"], c["hier"], c["lay"], c["T"]
    memo = c.setdefault("memo", {})
    maxabs = float(np.abs(uh).max())
    for tol in c["tols"]:
        say("compress", name, "tol", tol)
        buf, nb, info = lib.mgard_compress(u, tol, c["coords"])
        blob = buf[:nb].cpu().numpy().tobytes()
        hd = codec.parse(blob)
        tau = A.tau_abs(tol, maxabs, True)
        assert hd.maxabs == maxabs and hd.tau_abs == tau and hd.L == hier.L
        assert hd.shape == hier.shape and hd.n == int(lay.off[-1])
        assert hd.bins == A.plain_bins(hier, A.tau_effective(tau, maxabs, hier.L, T))
        lengths = np.frombuffer(blob, np.uint8, hd.dict_size, hd.offsets["code_len"]).astype(np.int64)
        used = lengths[lengths > 0]
        assert sum(math.ldexp(1.0, -int(v)) for v in used) == 1.0
        codes = H.canonical_codes(lengths)
        cbits = np.frombuffer(blob, "<u4", hd.n_chunks, hd.offsets["chunk_bits"]).astype(np.int64)
        cesc = np.frombuffer(blob, "<u4", hd.n_chunks, hd.offsets["chunk_esc"]).astype(np.int64)
        words = np.frombuffer(blob, "<u4", hd.payload_words, hd.offsets["payload"])
        outl = np.frombuffer(blob, "<i8", hd.n_outliers, hd.offsets["outliers"])
        wstart = np.concatenate([[0], np.cumsum((cbits + 31) // 32)])
        ostart = np.concatenate([[0], np.cumsum(cesc)])
        assert wstart[-1] == hd.payload_words and ostart[-1] == hd.n_outliers
        ch = hd.chunk
        first = -(-int(lay.off[hier.L]) // ch)
        last = hd.n_chunks - 1  # ragged: the stream's tail lies in the finest level
        rng = np.random.default_rng(int(tol * 1e6) + 3)
        picks = sorted({first, last, *[int(k) for k in rng.integers(first, last, 10)]})
        say("check chunks", picks)
        for k in picks:
            start = k * ch
            count = min(ch, hd.n - start)
            sym, out = _expected_chunk(uh, hier, lay, T, hd.bins, start, count, hd.dict_size, memo)
            assert int(cbits[k]) == int(lengths[sym].sum()), k
            dec = H.decode([int(w) for w in words[wstart[k]:wstart[k + 1]]], [int(cbits[k])], lengths, codes,
                           count, ch)
            assert np.array_equal(np.asarray(dec, dtype=np.int64), sym), k
            assert np.array_equal(outl[ostart[k]:ostart[k + 1]], out), k
        say("decompress", name, "ratio", u.numel() * u.element_size() / nb)
        rec = lib.mgard_decompress(buf, nb)
        err = float((rec - u).abs().max())
        say("L_inf / tau", err / tau)
        assert err <= tau
        del rec, buf
