"""The encoder entry point that allocates nothing (mgard_huffman_encode_noalloc).

It must give exactly what mgard_huffman_encode gives (chunk bit counts,
payload words and length; those are tied to the oracle's bit packing by the
parity tests, and here once more for the smaller input), on two calls in a
row, the second with a smaller input, through the C-ABI with caller buffers
allocated before the calls.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import huffman as H

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[noalloc]", *a, flush=True)


def _symbols(n, seed, dict_size):
    """Seeded symbols with a two-sided geometric spread around the dictionary's middle."""
    rng = np.random.default_rng(seed)
    q = rng.geometric(0.02, size=n) * rng.choice([-1, 1], size=n)
    R = dict_size // 2
    s = np.where(np.abs(q) < R, q + R, 0)
    return s.astype(np.uint16)


def _codebook(lib, sym_d, dict_size, chunk):
    hist, _ = lib.mgard_histogram(sym_d, dict_size, chunk)
    return lib.mgard_huffman_codebook(hist, dict_size)


@pytest.mark.parametrize("dict_size,chunk", [(8192, 1024), (1024, 256), (8192, 4096)])
def test_noalloc_encode_equals_encode_on_two_calls(lib, dict_size, chunk):
    cases = [(3_000_000 + 517, 1), (100_003, 2)]  # the second call is smaller
    # every buffer is allocated before the first no-allocation call
    prepared = []
    for n, seed in cases:
        s = _symbols(n, seed + dict_size + chunk, dict_size)
        sym_d = torch.from_numpy(s.view(np.int16).copy()).to(DEV)
        lens, codes = _codebook(lib, sym_d, dict_size, chunk)
        bits_ref, pay_ref = lib.mgard_huffman_encode(sym_d, lens, codes, dict_size, chunk)
        nch = (n + chunk - 1) // chunk
        bits = torch.full((nch,), -1, dtype=torch.int32, device=DEV)
        payload = torch.full((pay_ref.numel() + 64,), -1, dtype=torch.int32, device=DEV)
        prepared.append((s, sym_d, lens, codes, bits_ref, pay_ref, bits, payload))
    torch.cuda.synchronize()
    for (n, _), (s, sym_d, lens, codes, bits_ref, pay_ref, bits, payload) in zip(cases, prepared):
        say("call", n, dict_size, chunk)
        words = lib.mgard_huffman_encode_noalloc(sym_d, lens, codes, bits, payload, dict_size, chunk)
        torch.cuda.synchronize()
        assert words == pay_ref.numel()
        assert torch.equal(bits, bits_ref)
        assert torch.equal(payload[:words], pay_ref)
    # the smaller input, against the oracle's bit packing of the same codebook
    s, sym_d, lens, codes, bits_ref, pay_ref, bits, payload = prepared[1]
    hl = lens.cpu().numpy().astype(np.int64)
    cb, words = H.encode(s.astype(np.int64), hl, H.canonical_codes(hl), chunk)
    assert np.array_equal(bits.cpu().numpy().astype(np.int64), np.asarray(cb, dtype=np.int64))
    assert np.array_equal(payload[: len(words)].cpu().numpy().view(np.uint32), np.asarray(words, dtype=np.uint32))


def test_noalloc_encode_limits(lib):
    """Beyond MGARD_NOALLOC_MAX_CHUNKS chunks, or into a payload buffer that is too
    small, the call fails with MGARD_ERR_CAPACITY (-6)."""
    dict_size, chunk = 8192, 256
    s = _symbols(50_000, 3, dict_size)
    sym_d = torch.from_numpy(s.view(np.int16).copy()).to(DEV)
    lens, codes = _codebook(lib, sym_d, dict_size, chunk)
    bits = torch.empty(((50_000 + chunk - 1) // chunk,), dtype=torch.int32, device=DEV)
    small = torch.empty((16,), dtype=torch.int32, device=DEV)
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_huffman_encode_noalloc(sym_d, lens, codes, bits, small, dict_size, chunk)
    assert e.value.code == -6
    # a symbol count needing one chunk more than the limit is refused on the host,
    # before any device work (the buffers are never read)
    L = lib.load_library()
    words = C.c_uint64(0)
    o = lib.make_opts()
    too_many = (2097152 + 1) * chunk
    rc = L.mgard_huffman_encode_noalloc(lib._ptr(sym_d), too_many, dict_size, chunk, lib._ptr(lens),
                                        lib._ptr(codes), lib._ptr(bits), lib._ptr(small), small.numel(),
                                        C.byref(words), C.byref(o))
    assert rc == -6
    # and the entry point still works afterwards
    big = torch.empty((50_000,), dtype=torch.int32, device=DEV)
    bits_ref, pay_ref = lib.mgard_huffman_encode(sym_d, lens, codes, dict_size, chunk)
    w = lib.mgard_huffman_encode_noalloc(sym_d, lens, codes, bits, big, dict_size, chunk)
    assert w == pay_ref.numel() and torch.equal(big[:w], pay_ref) and torch.equal(bits, bits_ref)
