"""Parity at the full workload sizes, in the launch configuration the benchmark times.

Element by element against the oracle:

* the whole coefficient stream of mgard_decompose (every level, the coarse
  grids included) equals the oracle's decomposition in the same working
  precision (normwise bound 1e-6 max|u| for float32, 1e-13 for float64 first,
  then bit equality);
* for every tolerance, the whole symbol stream of mgard_compress (decoded by
  the library's decoder from the buffer's payload), the chunk bit counts and
  escape counts, the escaped values (unpacked by the oracle), the histogram's
  code lengths and the header's max |u|, tau and bins equal the oracle's
  quantization of its own stream with its own bins;
* a few whole chunks are also decoded by the oracle's bit-serial decoder from
  the library's payload (the first of the finest level and the ragged last);
* decompose then recompose returns the input within the rounding reserve the
  error budget sets aside, 4 (L + 1) eps max |u|, and the decompressed field
  is within tau of the input.

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


@pytest.fixture(scope="module", params=list(WORKLOADS))
def cache(request, lib):
    """One workload at a time (tests are grouped by it): the field on the device,
    its host copy, the hierarchy and, once computed, the oracle's stream."""
    import torch

    name = request.param
    torch.cuda.empty_cache()
    make, T, tols = WORKLOADS[name]
    u, coords = make(torch)
    say("autotune", tuple(u.shape))
    lib.mgard_autotune(u, coords)
    uh = u.cpu().numpy()
    hier = Hierarchy(u.shape, coords)
    d = dict(name=name, u=u, coords=coords, uh=uh, hier=hier, lay=Layout(hier), T=T, tols=tols)
    yield d
    d.clear()
    torch.cuda.empty_cache()


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


def _oracle_stream(c):
    if "stream" not in c:
        say("oracle decompose", c["name"])
        hier, T = c["hier"], c["T"]
        c["stream"] = Q.to_stream(*X.decompose(c["uh"], hier, T), hier)
    return c["stream"]


def test_fullsize_decompose_every_level(lib, cache):
    c = cache
    name = c["name"]
    u, uh, hier, lay, T = c["u"], c["uh"], c["hier"], c["lay"], c["T"]
    L, offs = lib.mgard_stream_layout(u.shape)
    assert L == hier.L and offs == [int(v) for v in lay.off]
    say("decompose", name)
    coeff = lib.mgard_decompose(u, c["coords"])
    got = coeff.cpu().numpy()
    want = _oracle_stream(c)
    maxabs = float(np.abs(uh).max())
    bound = (1e-6 if T == np.float32 else 1e-13) * maxabs
    for l in range(hier.L + 1):
        a, b = got[lay.off[l]:lay.off[l + 1]], want[lay.off[l]:lay.off[l + 1]]
        d = float(np.abs(a.astype(np.float64) - b.astype(np.float64)).max()) if len(a) else 0.0
        assert d <= bound, (name, l, d)
        bad = np.flatnonzero(a != b)
        assert bad.size == 0, (name, l, bad.size, [(int(i), float(a[i]), float(b[i])) for i in bad[:3]])
    # the stream layout: sampled positions map to the nodes the oracle's per-node value names
    pts = _sample_fine_nodes(hier, np.random.default_rng(5), 200)
    for p in pts:
        q = lay.pos_of(p)
        assert lay.node_of(q) == p
        assert got[q] == X.coefficient_at(uh, hier, p, T)
    del got
    say("recompose", name)
    rec = lib.mgard_recompose(coeff, u.shape, c["coords"])
    del coeff
    err = float((rec - u).abs().max())
    reserve = 4.0 * (hier.L + 1) * float(np.finfo(T).eps) * maxabs
    say("decompose-recompose L_inf", err, "reserve", reserve)
    assert err <= reserve


def test_fullsize_symbols_escapes_and_roundtrip(lib, cache):
    import torch

    c = cache
    name = c["name"]
    u, uh, hier, lay, T = c["u"], c["uh"], c["hier"], c["lay"], c["T"]
    stream = _oracle_stream(c)
    maxabs = float(np.abs(uh).max())
    for tol in c["tols"]:
        say("compress", name, "tol", tol)
        buf, nb, info = lib.mgard_compress(u, tol, c["coords"])
        blob = buf[:nb].cpu().numpy().tobytes()
        hd = codec.parse(blob)
        tau = A.tau_abs(tol, maxabs, True)
        assert hd.maxabs == maxabs and hd.tau_abs == tau and hd.L == hier.L
        assert hd.shape == hier.shape and hd.n == int(lay.off[-1])
        bins = A.plain_bins(hier, A.tau_effective(tau, maxabs, hier.L, T))
        assert hd.bins == bins
        say("  oracle quantize")
        q = Q.quantize_stream(stream, hier, bins)
        sym, outl = Q.to_symbols(q, hd.dict_size)
        counts, widths = Q.escape_table(q, hier, hd.dict_size)
        del q
        lengths_ref = H.code_lengths(H.histogram(sym, hd.dict_size))
        lengths = np.frombuffer(blob, np.uint8, hd.dict_size, hd.offsets["code_len"]).astype(np.int64)
        assert np.array_equal(lengths, lengths_ref)
        used = lengths[lengths > 0]
        assert sum(math.ldexp(1.0, -int(v)) for v in used) == 1.0
        ch = hd.chunk
        cbits = np.frombuffer(blob, "<u4", hd.n_chunks, hd.offsets["chunk_bits"]).astype(np.int64)
        cesc = np.frombuffer(blob, "<u4", hd.n_chunks, hd.offsets["chunk_esc"]).astype(np.int64)
        starts = np.arange(0, hd.n, ch)
        assert np.array_equal(cbits, np.add.reduceat(lengths[sym], starts))
        assert np.array_equal(cesc, np.add.reduceat((sym == 0).astype(np.int64), starts))
        say("  whole symbol stream (library decoder)")
        po, pw = hd.offsets["payload"], hd.payload_words
        payload = buf[po:po + 4 * pw].view(torch.int32)
        bits_d = buf[hd.offsets["chunk_bits"]:hd.offsets["chunk_bits"] + 4 * hd.n_chunks].view(torch.int32)
        lens_d = buf[hd.offsets["code_len"]:hd.offsets["code_len"] + hd.dict_size]
        dec = lib.mgard_huffman_decode(payload, bits_d, hd.n, lens_d, hd.dict_size, ch)
        assert np.array_equal(lib.u16(dec), sym.astype(np.uint16))
        del dec, payload
        say("  escapes", hd.n_outliers, "widths", hd.esc_widths)
        assert hd.esc_counts == counts and hd.esc_widths == widths
        nesc = sum(Q.escape_words(hd.esc_counts, hd.esc_widths))
        esc_words = np.frombuffer(blob, "<u4", nesc, hd.offsets["escapes"])
        assert np.array_equal(Q.unpack_escapes(esc_words, hd.esc_counts, hd.esc_widths, hd.dict_size), outl)
        # a few chunks through the oracle's bit-serial decoder as well
        codes = H.canonical_codes(lengths)
        words = np.frombuffer(blob, "<u4", pw, po)
        wstart = np.concatenate([[0], np.cumsum((cbits + 31) // 32)])
        first = -(-int(lay.off[hier.L]) // ch)
        for k in sorted({0, first, hd.n_chunks - 1}):
            count = min(ch, hd.n - k * ch)
            got = H.decode([int(w) for w in words[wstart[k]:wstart[k + 1]]], [int(cbits[k])], lengths, codes,
                           count, ch)
            assert np.array_equal(np.asarray(got, dtype=np.int64), sym[k * ch:k * ch + count]), k
        del sym, outl
        say("decompress", name, "ratio", u.numel() * u.element_size() / nb)
        rec = lib.mgard_decompress(buf, nb)
        err = float((rec - u).abs().max())
        say("L_inf / tau", err / tau)
        assert err <= tau
        del rec, buf


def test_fullsize_l2_bound(lib, cache):
    """The relative L2 bound at 1e-3 (the paper's cosmology setting, Sec. 4) on the
    full-size workload: tau from ||u|| within 1e-10 of the oracle's; the header's
    widths equal the oracle's s-norm widths for that tau; the whole symbol
    stream equals the oracle's quantization of its own stream with them; the
    decompressed field's L2 error, measured by the oracle in float64 and by the
    library, stays within tau."""
    import torch

    from oracle import snorm as SN

    c = cache
    u, uh, hier, lay, T = c["u"], c["uh"], c["hier"], c["lay"], c["T"]
    stream = _oracle_stream(c)
    tol = 1e-3
    say("l2 compress", c["name"])
    buf, nb, info = lib.mgard_compress(u, tol, c["coords"], norm="s", s=0.0)
    blob = buf[:nb].cpu().numpy().tobytes()
    hd = codec.parse(blob)
    nrm = math.sqrt(SN.l2_norm_sq(uh, hier))
    assert abs(hd.tau_abs - tol * nrm) <= 1e-10 * tol * nrm
    assert abs(lib.mgard_l2_norm(u, c["coords"]) - nrm) <= 1e-10 * nrm
    maxabs = float(np.abs(uh).max())
    bins = SN.bins_for(hier, SN.tau_effective(hd.tau_abs, maxabs, hier, 0.0, T), 0.0)
    assert hd.bins == bins
    q = Q.quantize_stream(stream, hier, bins)
    sym, outl = Q.to_symbols(q, hd.dict_size)
    counts, widths = Q.escape_table(q, hier, hd.dict_size)
    del q
    assert hd.esc_counts == counts and hd.esc_widths == widths
    po, pw = hd.offsets["payload"], hd.payload_words
    dec = lib.mgard_huffman_decode(buf[po:po + 4 * pw].view(torch.int32),
                                   buf[hd.offsets["chunk_bits"]:hd.offsets["chunk_bits"] + 4 * hd.n_chunks].view(
                                       torch.int32), hd.n,
                                   buf[hd.offsets["code_len"]:hd.offsets["code_len"] + hd.dict_size], hd.dict_size,
                                   hd.chunk)
    assert np.array_equal(lib.u16(dec), sym.astype(np.uint16))
    del dec, sym
    nesc = sum(Q.escape_words(hd.esc_counts, hd.esc_widths))
    esc_words = np.frombuffer(blob, "<u4", nesc, hd.offsets["escapes"])
    assert np.array_equal(Q.unpack_escapes(esc_words, hd.esc_counts, hd.esc_widths, hd.dict_size), outl)
    rec = lib.mgard_decompress(buf, nb)
    e_dev = (rec.double() - u.double()).contiguous()
    err_lib = lib.mgard_l2_norm(e_dev, c["coords"])
    e = rec.cpu().numpy().astype(np.float64) - uh.astype(np.float64)
    err = math.sqrt(SN.l2_norm_sq(e, hier))
    say("L2 error / tau", err / hd.tau_abs, "ratio", u.numel() * u.element_size() / nb)
    assert abs(err_lib - err) <= 1e-9 * err
    assert err <= hd.tau_abs
