"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bars: floating-point stages agree with the oracle in the same working
precision (same rounding order, so the expected result is bit-identical; the
normwise tolerance 1e-6 max|u| for float32 and 1e-13 max|u| for float64 is
asserted first), and float32 results stay within 1e-6 max|u| of the float64
oracle.  Integer stages (quantized symbols, histogram, code lengths, codes,
payload words) must be bit-exact.  Inputs are seeded and synthetic.
"""
import sys
import zlib

import numpy as np
import pytest
import torch

import fieldgen
from oracle import alloc as A
from oracle import codec, grid, huffman as H, quant as Q
from oracle import transform as X

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.array(x, order="C")).to(DEV)  # a writable copy, also of read-only buffers


def host(t):
    return t.detach().cpu().numpy()


def tol_for(T):
    return 1e-6 if T == np.float32 else 1e-13


CASES = {
    "c1-129x129-f64": ((129, 129), np.float64, None),
    "3d-33x20x17-f32-nonuniform": ((33, 20, 17), np.float32, "rand"),
    "3d-17x18x19-f64-nonuniform": ((17, 18, 19), np.float64, "rand"),
    "1d-1000-f32": ((1000,), np.float32, None),
    "4d-9x10x7x6-f64": ((9, 10, 7, 6), np.float64, "rand"),
    "batchdims-2x65x1x33-f32": ((2, 65, 1, 33), np.float32, None),
    "even-64x50-f32": ((64, 50), np.float32, None),
    "3d-65x65x65-f32": ((65, 65, 65), np.float32, None),
    "3d-129x130x131-f32-nonuniform": ((129, 130, 131), np.float32, "rand"),
    "3d-64x50x37-f64": ((64, 50, 37), np.float64, None),
}


def make_case(name):
    shape, T, cmode = CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name.startswith("c1"):
        u = fieldgen.bumps2d(129, seed=1)
    elif name.startswith("3d-65"):
        u = fieldgen.spectral(shape, -5.0 / 3.0, 2)
    else:
        u = fieldgen.random_field(shape, rng)
    u = u.astype(T)
    coords = [fieldgen.random_coords(n, rng) for n in shape] if cmode == "rand" else None
    return u, coords


@pytest.mark.parametrize("name", list(CASES))
def test_decompose_matches_oracle(lib, name):
    u, coords = make_case(name)
    T = u.dtype.type
    say("decompose", name)
    h = grid.Hierarchy(u.shape, coords)
    ref = Q.to_stream(*X.decompose(u, h, T), h)
    got = host(lib.mgard_decompose(dev(u), coords))
    scale = float(np.abs(u).max())
    assert np.abs(got.astype(np.float64) - ref).max() <= tol_for(T) * scale
    mism = int(np.count_nonzero(got != ref))
    assert mism == 0, f"{mism} of {ref.size} coefficients differ in the last bits"


@pytest.mark.parametrize("name", ["3d-33x20x17-f32-nonuniform", "3d-65x65x65-f32", "batchdims-2x65x1x33-f32"])
def test_f32_decompose_close_to_f64_oracle(lib, name):
    u, coords = make_case(name)
    say("f32 vs f64 oracle", name)
    h = grid.Hierarchy(u.shape, coords)
    ref = Q.to_stream(*X.decompose(u.astype(np.float64), h, np.float64), h)
    got = host(lib.mgard_decompose(dev(u), coords)).astype(np.float64)
    off = Q.level_offsets(h)
    scale = float(np.abs(u).max())
    for l in range(h.L + 1):
        d = np.abs(got[off[l]:off[l + 1]] - ref[off[l]:off[l + 1]]).max()
        assert d <= 1e-6 * scale, (l, d / scale)


@pytest.mark.parametrize("name", list(CASES))
def test_recompose_matches_oracle(lib, name):
    u, coords = make_case(name)
    T = u.dtype.type
    say("recompose", name)
    h = grid.Hierarchy(u.shape, coords)
    c0, cb = X.decompose(u, h, T)
    stream = Q.to_stream(c0, cb, h)
    ref = X.recompose(*Q.from_stream(stream, h, T), h, T)
    got = host(lib.mgard_recompose(dev(stream), u.shape, coords))
    assert got.dtype == T
    assert np.abs(got.astype(np.float64) - ref).max() <= tol_for(T) * float(np.abs(u).max())
    assert int(np.count_nonzero(got != ref)) == 0
    if T == np.float64:
        assert np.abs(got - u).max() <= 1e-12 * np.abs(u).max()


def test_gpu_roundtrip_f64_nonuniform(lib):
    rng = np.random.default_rng(7)
    shape = (40, 33, 27)
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    u = fieldgen.random_field(shape, rng)
    say("roundtrip f64", shape)
    c = lib.mgard_decompose(dev(u), xs)
    r = host(lib.mgard_recompose(c, shape, xs))
    assert np.abs(r - u).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("name", ["c1-129x129-f64", "3d-33x20x17-f32-nonuniform"])
@pytest.mark.parametrize("dict_size", [256, 8192])
def test_quantize_dequantize_stage(lib, name, dict_size):
    u, coords = make_case(name)
    T = u.dtype.type
    say("quantize stage", name, dict_size)
    h = grid.Hierarchy(u.shape, coords)
    stream = Q.to_stream(*X.decompose(u, h, T), h)
    bins = [1e-3 * (1.0 + 0.1 * l) for l in range(h.L + 1)]
    q = Q.quantize_stream(stream, h, bins)
    sym_ref, out_ref = Q.to_symbols(q, dict_size)
    sym, qside = lib.mgard_quantize(dev(stream), u.shape, bins, dict_size)
    s = lib.u16(sym).astype(np.int64)
    assert np.array_equal(s, sym_ref)
    esc = sym_ref == 0
    assert np.array_equal(host(qside)[esc], out_ref)
    deq = host(lib.mgard_dequantize(sym, qside, u.shape, bins, torch.float32 if T == np.float32 else torch.float64,
                                    dict_size))
    assert np.array_equal(deq, Q.dequantize_stream(q, h, bins, T))


def _symbol_streams():
    rng = np.random.default_rng(12)
    u = fieldgen.bumps2d()
    p = codec.compress_parts(u, 1e-4, dict_size=8192)
    yield "c1-1e-4", p.symbols, 8192, 4096
    lap = np.clip(np.round(rng.laplace(512, 30, size=200_003)), 0, 1023).astype(np.int64)
    yield "laplace-1024", lap, 1024, 512
    yield "single-symbol", np.full(5000, 77, dtype=np.int64), 256, 256
    wide = rng.integers(0, 8192, size=100_000)
    yield "uniform-8192", wide, 8192, 8192
    geo = np.minimum(rng.geometric(0.02, size=300_000), 4095).astype(np.int64)
    yield "geometric-4096", geo, 4096, 1024


@pytest.mark.parametrize("case", list(range(5)))
def test_huffman_stages_bitexact(lib, case):
    name, sym, dict_size, chunk = list(_symbol_streams())[case]
    say("huffman", name)
    dsym = dev(sym.astype(np.int16) if sym.max() < 32768 else sym.astype(np.uint16).view(np.int16))
    hist, esc = lib.mgard_histogram(dsym, dict_size, chunk)
    href = H.histogram(sym, dict_size)
    assert np.array_equal(host(hist), href)
    eref = [int(np.count_nonzero(sym[k:k + chunk] == 0)) for k in range(0, len(sym), chunk)]
    assert list(host(esc)[:len(eref)]) == eref
    lens, codes = lib.mgard_huffman_codebook(hist, dict_size)
    lref = H.code_lengths(href)
    cref = H.canonical_codes(lref)
    assert np.array_equal(host(lens).astype(np.int64), lref)
    assert np.array_equal(host(codes).view(np.uint64)[lref > 0], cref[lref > 0])
    bits, payload = lib.mgard_huffman_encode(dsym, lens, codes, dict_size, chunk)
    bref, wref = H.encode(sym, lref, cref, chunk)
    assert list(host(bits).astype(np.int64)) == bref
    got_w = host(payload).view(np.uint32).astype(np.int64)
    ref_w = np.asarray(wref, dtype=np.int64)
    bad = np.nonzero(got_w != ref_w)[0]
    if len(bad):
        woff = np.concatenate([[0], np.cumsum((np.asarray(bref) + 31) // 32)])
        ks = np.searchsorted(woff, bad[:8], side="right") - 1
        say("payload mismatches", len(bad), "first", list(bad[:8]), "chunks", list(ks),
            "gpu", [hex(int(v)) for v in got_w[bad[:8]]], "ref", [hex(int(v)) for v in ref_w[bad[:8]]])
        _, payload2 = lib.mgard_huffman_encode(dsym, lens, codes, dict_size, chunk)
        say("repeat run identical:", bool(np.array_equal(host(payload2), host(payload))))
    assert len(bad) == 0
    # decode the oracle's payload on the GPU
    dec = lib.mgard_huffman_decode(dev(np.asarray(wref, dtype=np.uint32).view(np.int32)),
                                   dev(np.asarray(bref, dtype=np.uint32).view(np.int32)), len(sym), lens,
                                   dict_size, chunk)
    assert np.array_equal(lib.u16(dec).astype(np.int64), sym)


def test_huffman_long_codes_bitexact(lib):
    """A complete prefix code with lengths 1..40 (codes longer than 32 bits) through encode and decode."""
    say("huffman long codes")
    dict_size, chunk = 256, 256
    lens = np.zeros(dict_size, dtype=np.int64)
    lens[:41] = list(range(1, 41)) + [40]
    codes = H.canonical_codes(lens)
    rng = np.random.default_rng(3)
    sym = rng.integers(0, 41, size=5001)
    bref, wref = H.encode(sym, lens, codes, chunk)
    dlens = dev(lens.astype(np.uint8))
    dcodes = dev(codes.view(np.int64))
    bits, payload = lib.mgard_huffman_encode(dev(sym.astype(np.int16)), dlens, dcodes, dict_size, chunk)
    assert list(host(bits).astype(np.int64)) == bref
    assert np.array_equal(host(payload).view(np.uint32).astype(np.int64), np.asarray(wref, dtype=np.int64))
    dec = lib.mgard_huffman_decode(dev(np.asarray(wref, dtype=np.uint32).view(np.int32)),
                                   dev(np.asarray(bref, dtype=np.uint32).view(np.int32)), len(sym), dlens,
                                   dict_size, chunk)
    assert np.array_equal(lib.u16(dec).astype(np.int64), sym)


def _adversarial_histograms():
    rng = np.random.default_rng(21)
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(8192, dtype=np.int64)
    h[rng.choice(8192, 40, replace=False)] = fib
    yield "fibonacci-40", h  # one leaf per depth: the merge's sequential stretches
    yield "equal-8192", np.full(8192, 3, dtype=np.int64)
    h = np.zeros(256, dtype=np.int64)
    h[[5, 200]] = [7, 1]
    yield "two-symbols", h
    h = np.zeros(1024, dtype=np.int64)
    h[rng.choice(1024, 300, replace=False)] = rng.integers(1, 4, 300)
    yield "ties-1024", h
    h = rng.integers(0, 2, 8192) * rng.integers(1, 1 << 34, 8192)
    yield "large-counts", h.astype(np.int64)  # weights beyond 32 bits
    x = np.clip(np.round(rng.normal(4096, 900, 2_000_000)), 0, 8191).astype(np.int64)
    yield "normal-8192", np.bincount(x, minlength=8192)


@pytest.mark.parametrize("case", list(range(6)))
def test_codebook_adversarial(lib, case):
    """Code lengths and canonical codes from histograms that stress the batched merge."""
    name, h = list(_adversarial_histograms())[case]
    say("codebook", name)
    lens, codes = lib.mgard_huffman_codebook(dev(h), len(h))
    lref = H.code_lengths(h)
    cref = H.canonical_codes(lref)
    assert np.array_equal(host(lens).astype(np.int64), lref)
    assert np.array_equal(host(codes).view(np.uint64)[lref > 0], cref[lref > 0])


@pytest.mark.parametrize("top,draw,chunk", [(25, "geometric", 512), (32, "uniform", 1024), (32, "geometric", 256)])
def test_huffman_many_lengths_bitexact(lib, top, draw, chunk):
    """A complete prefix code with `top` distinct lengths 1..top, all <= 32 (the
    decoder's prefix table with windows that meet two and more lengths; with
    top = 32, codes longer than the encoder's packed 26 bits)."""
    say("huffman many lengths", top, draw, chunk)
    dict_size = 256
    lens = np.zeros(dict_size, dtype=np.int64)
    lens[:top + 1] = list(range(1, top + 1)) + [top]
    codes = H.canonical_codes(lens)
    rng = np.random.default_rng(4 + top)
    if draw == "geometric":
        sym = np.minimum(rng.geometric(0.3, size=20_001) - 1, top)
    else:  # every length equally often: most windows lie among the long codes
        sym = rng.integers(0, top + 1, size=20_001)
    bref, wref = H.encode(sym, lens, codes, chunk)
    dlens = dev(lens.astype(np.uint8))
    bits, payload = lib.mgard_huffman_encode(dev(sym.astype(np.int16)), dlens, dev(codes.view(np.int64)),
                                             dict_size, chunk)
    assert list(host(bits).astype(np.int64)) == bref
    assert np.array_equal(host(payload).view(np.uint32).astype(np.int64), np.asarray(wref, dtype=np.int64))
    dec = lib.mgard_huffman_decode(dev(np.asarray(wref, dtype=np.uint32).view(np.int32)),
                                   dev(np.asarray(bref, dtype=np.uint32).view(np.int32)), len(sym), dlens,
                                   dict_size, chunk)
    assert np.array_equal(lib.u16(dec).astype(np.int64), sym)


def _prefix_case(name):
    """Complete prefix codes at the edges of the decoder's 12-bit prefix table."""
    if name == "one-symbol":  # a single code, one bit long
        lens = np.zeros(256, dtype=np.int64)
        lens[7] = 1
        return 256, lens, np.full(9_001, 7)
    if name == "lengths-1-to-13":  # 1..12 once, 13 twice: the two 13-bit codes share a prefix
        lens = np.zeros(256, dtype=np.int64)
        lens[:14] = list(range(1, 13)) + [13, 13]
        return 256, lens, None
    if name == "all-12":  # every prefix is one whole code
        return 4096, np.full(4096, 12, dtype=np.int64), None
    if name == "all-13":  # every prefix holds two codes
        return 8192, np.full(8192, 13, dtype=np.int64), None
    if name == "short-and-14":  # lengths 1, 3 and 14: prefixes of one code, or of four
        lens = np.zeros(8192, dtype=np.int64)
        lens[0] = 1
        lens[1:3] = 3
        lens[3:3 + 4096] = 14  # 2^-1 + 2 * 2^-3 + 4096 * 2^-14 = 1
        return 8192, lens, None
    raise KeyError(name)


@pytest.mark.parametrize("name,chunk", [("one-symbol", 256), ("lengths-1-to-13", 1024), ("all-12", 768),
                                        ("all-13", 8192), ("short-and-14", 512)])
def test_huffman_prefix_table_edges_bitexact(lib, name, chunk):
    """Decoding of codes whose lengths sit at the prefix table's width (12 bits): a code per
    prefix, two or four codes per prefix, a one-bit single code; oracle encode, GPU encode
    equal to it and GPU decode back to the symbols."""
    dict_size, lens, sym = _prefix_case(name)
    say("huffman prefix edges", name, chunk)
    codes = H.canonical_codes(lens)
    used = np.flatnonzero(lens)
    rng = np.random.default_rng(len(used) + chunk)
    if sym is None:
        sym = used[rng.integers(0, len(used), size=30_001)]
    bref, wref = H.encode(sym, lens, codes, chunk)
    dlens = dev(lens.astype(np.uint8))
    bits, payload = lib.mgard_huffman_encode(dev(sym.astype(np.int16)), dlens, dev(codes.view(np.int64)),
                                             dict_size, chunk)
    assert list(host(bits).astype(np.int64)) == bref
    assert np.array_equal(host(payload).view(np.uint32).astype(np.int64), np.asarray(wref, dtype=np.int64))
    dec = lib.mgard_huffman_decode(dev(np.asarray(wref, dtype=np.uint32).view(np.int32)),
                                   dev(np.asarray(bref, dtype=np.uint32).view(np.int32)), len(sym), dlens,
                                   dict_size, chunk)
    assert np.array_equal(lib.u16(dec).astype(np.int64), sym)


@pytest.mark.parametrize("name,tol", [("c1-129x129-f64", 1e-3), ("c1-129x129-f64", 1e-5),
                                      ("3d-33x20x17-f32-nonuniform", 1e-2), ("3d-65x65x65-f32", 1e-3),
                                      ("even-64x50-f32", 1e-4), ("4d-9x10x7x6-f64", 1e-3)])
def test_compressed_bytes_equal_oracle(lib, name, tol):
    u, coords = make_case(name)
    say("compress bytes", name, tol)
    ref = codec.compress(u, tol, coords=coords)
    buf, nbytes, info = lib.mgard_compress(dev(u), tol, coords)
    got = host(buf[:nbytes]).tobytes()
    assert nbytes == len(ref)
    assert got == ref
    # GPU decompression of the oracle's buffer equals the oracle's decompression
    r = host(lib.mgard_decompress(dev(np.frombuffer(ref, dtype=np.uint8)), len(ref)))
    rref = codec.decompress(ref)
    assert np.array_equal(r, rref)
    assert np.abs(r.astype(np.float64) - u.astype(np.float64)).max() <= tol * np.abs(u).max()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_maxabs_every_alignment_and_tail(lib, dt):
    """max|u| equals numpy's whatever the array's start within 16 bytes and
    whatever its length (ragged ends, several trips of the grid-stride loop),
    with the largest magnitude first, in the middle or last; a NaN or
    infinity in the last element is still reported."""
    rng = np.random.default_rng(71)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    E = 16 // np.dtype(dt).itemsize
    big = (1 << 25) + 3  # several trips of the grid-stride loop
    base = torch.zeros(big + E, dtype=tdt, device=DEV)
    say("maxabs", np.dtype(dt).name)
    for n in [1, 2, 3, 5, 7, 4099, 1000003, big]:
        x = rng.standard_normal(n).astype(dt)
        for off in range(E) if n < big else (0, 1):
            for k in (0, n // 2, n - 1):
                keep = x[k]
                x[k] = -1e3
                v = base[off:off + n]
                v.copy_(torch.from_numpy(x))
                x[k] = keep
                assert lib.mgard_maxabs(v) == 1e3, (n, off, k)
    for bad in (np.nan, np.inf):
        x = np.ones(4099, dtype=dt)
        x[-1] = bad
        with pytest.raises(lib.MgardError) as e:
            lib.mgard_maxabs(dev(x))
        assert e.value.code == -5


def test_error_paths(lib):
    say("error paths")
    u = np.ones((33, 33), dtype=np.float32)
    u[3, 4] = np.nan
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(u), 1e-3)
    assert e.value.code == -5
    u[3, 4] = np.inf
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(u), 1e-3)
    assert e.value.code == -5
    v = fieldgen.bumps2d(65).astype(np.float32)
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(v), 0.0)
    assert e.value.code == -4
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(v), 1e-3, out=torch.empty(100, dtype=torch.uint8, device=DEV))
    assert e.value.code == -6
    buf, nbytes, _ = lib.mgard_compress(dev(v), 1e-3)
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_decompress(buf, nbytes - 8)
    assert e.value.code == -7
    # corrupt one chunk bit count: the payload no longer decodes
    hd = codec.parse(host(buf[:nbytes]).tobytes())
    bad = buf[:nbytes].clone()
    o = hd.offsets["chunk_bits"]
    bad[o] = (int(bad[o]) + 1) % 256
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_decompress(bad, nbytes)
    assert e.value.code == -7
    # zero field: all coefficients quantize to zero
    z = torch.zeros((17, 17), dtype=torch.float64, device=DEV)
    b2, n2, _ = lib.mgard_compress(z, 1e-3)
    assert torch.equal(lib.mgard_decompress(b2, n2), z)


def test_tolerance_outside_range_rejected(lib):
    """Tolerances whose rounding reserve exceeds tau/2 (float32, 1e-7) or whose
    max|u| / b reaches 2^49 (float64, 1D n = 5, rel 4.5e-15) are refused with
    MGARD_ERR_TOL, as the oracle refuses them; the neighbours are accepted."""
    say("tolerance range")
    u = fieldgen.bumps2d(65).astype(np.float32)
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(u), 1e-7)
    assert e.value.code == -4
    with pytest.raises(ValueError):
        codec.compress(u, 1e-7)
    lib.mgard_compress(dev(u), 1e-4)
    w = np.array([1.0, -0.5, 0.25, 0.75, -1.0])
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(dev(w), 4.5e-15)
    assert e.value.code == -4
    with pytest.raises(ValueError):
        codec.compress(w, 4.5e-15)
    buf, nb, _ = lib.mgard_compress(dev(w), 1e-13)
    assert host(buf[:nb]).tobytes() == codec.compress(w, 1e-13)


def _escape_buffer(lib):
    """A valid buffer with many escapes (dictionary of 256 at a tight bound)."""
    u = fieldgen.bumps2d(129, seed=1)
    buf, nbytes, info = lib.mgard_compress(dev(u), 1e-6, dict_size=256)
    assert info["n_outliers"] > 100
    return u, buf[:nbytes].clone(), nbytes, codec.parse(host(buf[:nbytes]).tobytes())


def test_malformed_escape_counts_rejected(lib):
    """A buffer whose header outlier count or per-chunk escape counts disagree
    with its symbols is refused with MGARD_ERR_FORMAT before any escape
    position is stored (the positions buffer holds n_outliers entries)."""
    say("malformed escape counts")
    u, buf, nbytes, hd = _escape_buffer(lib)
    rec = lib.mgard_decompress(buf, nbytes)
    assert float((rec - dev(u)).abs().max()) <= 1e-6 * float(np.abs(u).max())
    nout = hd.n_outliers
    esc = np.frombuffer(host(buf).tobytes(), "<u4", hd.n_chunks, hd.offsets["chunk_esc"])
    k = int(np.argmax(esc))
    cases = {}
    for name, v in [("n_outliers-1", nout - 1), ("n_outliers=0", 0)]:
        b = buf.clone()
        b[64:72] = torch.from_numpy(np.frombuffer(np.uint64(v).tobytes(), np.uint8).copy()).to(DEV)
        cases[name] = b
    for name, delta in [("chunk_esc+1", 1), ("chunk_esc+2^20", 1 << 20), ("chunk_esc-1", -1)]:
        b = buf.clone()
        o = hd.offsets["chunk_esc"] + 4 * k
        v = np.uint32(int(esc[k]) + delta)
        b[o:o + 4] = torch.from_numpy(np.frombuffer(v.tobytes(), np.uint8).copy()).to(DEV)
        cases[name] = b
    # the per-level escape table: a width beyond 64 bits, and one escape moved
    # to another level (the counts still add up to n_outliers)
    lesc = codec.FIXED + 8 * len(hd.shape) + 8 * (hd.L + 1)
    lbits = lesc + 8 * (hd.L + 1)
    b = buf.clone()
    b[lbits:lbits + 4] = torch.from_numpy(np.frombuffer(np.uint32(65).tobytes(), np.uint8).copy()).to(DEV)
    cases["width 65"] = b
    l1 = max(l for l in range(hd.L + 1) if hd.esc_counts[l] > 0)
    l0 = l1 - 1 if l1 > 0 else l1 + 1
    cnt = list(hd.esc_counts)
    cnt[l1] -= 1
    cnt[l0] += 1
    b = buf.clone()
    b[lesc:lesc + 8 * (hd.L + 1)] = torch.from_numpy(np.asarray(cnt, dtype="<u8").view(np.uint8).copy()).to(DEV)
    cases["escape moved to level %d" % l0] = b
    for name, b in cases.items():
        say("  case", name)
        with pytest.raises(lib.MgardError) as e:
            lib.mgard_decompress(b, nbytes)
        assert e.value.code == -7, name
    # the library still decodes the intact buffer afterwards
    assert torch.equal(lib.mgard_decompress(buf, nbytes), rec)

