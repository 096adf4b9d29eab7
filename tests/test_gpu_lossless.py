"""The second-stage lossless coder on the GPU against the oracle, through the C-ABI.

* containers byte-equal to oracle/lossless.py's for inputs of many lengths
  (whole and partial words, one chunk and more, a ragged last chunk) and
  zero densities, and decoding returns the input;
* compression with the lossless stage writes the oracle's container of the
  oracle's stream when that is smaller, else the plain stream, and
  decompresses to the same field as the plain stream;
* malformed containers (offsets, bitmaps, truncation) give MGARD_ERR_FORMAT;
* at full size: the 513^3 compressed streams and the refactored buffer,
  coded and decoded back.
"""
import numpy as np
import pytest

import fieldgen
from oracle import codec
from oracle import lossless as Z

pytestmark = pytest.mark.gpu


def say(*a):
    print("[lossless]", *a, flush=True)


def _dev(b: bytes):
    import torch

    pad = (-len(b)) % 8
    t = torch.from_numpy(np.frombuffer(b + b"\0" * pad, dtype=np.uint8).copy()).cuda()
    return t


@pytest.mark.parametrize("nbytes", [1, 3, 4, 5, 100, 4 * 4096, 4 * 4096 + 1, 4 * 4096 * 3 + 102, 1_000_003])
@pytest.mark.parametrize("density", [0.0, 0.002, 0.1, 0.6, 1.0])
def test_container_equals_the_oracle(lib, nbytes, density):
    rng = np.random.default_rng(nbytes * 7 + int(density * 1000))
    nw = (nbytes + 3) // 4
    w = rng.integers(1, 2 ** 32, nw, dtype=np.uint64).astype(np.uint32)
    w[rng.random(nw) >= density] = 0
    data = w.tobytes()[:nbytes]
    ref = Z.encode(data)
    d = _dev(data)
    enc, nb = lib.mgard_lossless_encode(d, nbytes)
    assert nb == len(ref)
    assert enc[:nb].cpu().numpy().tobytes() == ref
    dec, raw = lib.mgard_lossless_decode(enc, nb)
    assert raw == nbytes
    assert dec[:raw].cpu().numpy().tobytes() == data


def test_empty_input(lib):
    import torch

    d = torch.zeros(8, dtype=torch.uint8, device="cuda")
    enc, nb = lib.mgard_lossless_encode(d, 0)
    assert enc[:nb].cpu().numpy().tobytes() == Z.encode(b"")
    _, raw = lib.mgard_lossless_decode(enc, nb, out=torch.zeros(8, dtype=torch.uint8, device="cuda"))
    assert raw == 0


@pytest.mark.parametrize("tol", [3e-1, 1e-1, 1e-3])
def test_compression_with_the_lossless_stage(lib, tol):
    import torch

    u = fieldgen.bumps2d(129, seed=1)
    plain = codec.compress(u, tol)
    coded = Z.encode(plain)
    want = coded if len(coded) < len(plain) else plain
    du = torch.from_numpy(u).cuda()
    buf, nb, _ = lib.mgard_compress(du, tol, lossless=True)
    say(f"tol {tol}: plain {len(plain)} B, coded {len(coded)} B")
    assert buf[:nb].cpu().numpy().tobytes() == want
    rec = lib.mgard_decompress(buf, nb).cpu().numpy()
    assert np.array_equal(rec, codec.decompress(plain))


def test_malformed_containers(lib):
    rng = np.random.default_rng(9)
    w = np.zeros(3 * 4096 + 50, np.uint32)
    w[rng.integers(0, len(w), 40)] = rng.integers(1, 1000, 40)
    ref = bytearray(Z.encode(w.tobytes()))
    nch = 4
    base = Z.FIXED + 8 * (nch + 1)

    def refuse(b, n=None):
        with pytest.raises(lib.MgardError) as e:
            lib.mgard_lossless_decode(_dev(bytes(b)), len(b) if n is None else n,
                                      raw_bytes=len(w) * 4)
        assert e.value.code == -7

    bad = bytearray(ref)
    bad[Z.FIXED + 8:Z.FIXED + 16] = (10 ** 9).to_bytes(8, "little")  # offset past the data
    refuse(bad)
    bad = bytearray(ref)
    bad[base:base + 4] = (0xFFFFFFFF).to_bytes(4, "little")  # level-2 bitmap of chunk 0
    refuse(bad)
    refuse(ref, len(ref) - 4)  # truncated data area
    bad = bytearray(ref)
    bad[16:24] = (7).to_bytes(8, "little")  # chunk count
    refuse(bad)


def test_fullsize_streams(lib):
    import torch

    n = 513
    u = fieldgen.spectral((n, n, n), -5.0 / 3.0, 2, device="cuda").to(torch.float32).contiguous()
    for tol in [1e-1, 1e-2, 1e-3]:
        buf, nb, _ = lib.mgard_compress(u, tol)
        enc, cb = lib.mgard_lossless_encode(buf, nb)
        dec, raw = lib.mgard_lossless_decode(enc, cb)
        assert raw == nb and torch.equal(dec[:nb], buf[:nb])
        say(f"513^3 tol {tol}: stream {nb / 1e6:.2f} MB -> {cb / 1e6:.2f} MB")
        lb, lnb, _ = lib.mgard_compress(u, tol, lossless=True)
        assert lnb == min(nb, cb)
        rec = lib.mgard_decompress(lb, lnb)
        assert float((rec.double() - u.double()).abs().max()) <= tol * float(u.abs().max())
    rb, rnb = lib.mgard_refactor(u, 32)
    enc, cb = lib.mgard_lossless_encode(rb, rnb)
    dec, raw = lib.mgard_lossless_decode(enc, cb)
    assert raw == rnb and torch.equal(dec[:rnb], rb[:rnb])
    say(f"513^3 refactored: {rnb / 1e6:.1f} MB -> {cb / 1e6:.1f} MB")
