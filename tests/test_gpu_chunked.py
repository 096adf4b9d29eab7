"""Out-of-core (chunked) compression of host-resident arrays against the oracle.

The container and every slab stream must equal, byte for byte, what the
oracle's chunked compressor writes from the same array; decompression must
equal the oracle's, value for value, and stay within the array's tolerance.
Cases cover a ragged last slab, a remainder below 3 planes joining the slab
before it, a single slab, 2D and 3D, float32 and float64, a nonuniform
dimension 0 (each slab gets its own coordinates), absolute and relative
tolerances, and pageable as well as pinned host memory.
"""
import numpy as np
import pytest

import fieldgen
from oracle import chunked as K

pytestmark = pytest.mark.gpu


def say(*a):
    print("[chunked]", *a, flush=True)


CASES = {
    # name: (shape, dtype, slab, tol, rel, nonuniform, seed)
    "3d-60x33x41-f32-slab16": ((60, 33, 41), np.float32, 16, 1e-3, True, False, 51),
    "3d-50x21x19-f32-slab16-merge": ((50, 21, 19), np.float32, 16, 1e-3, True, False, 52),
    "3d-30x17x25-f64-slab8-nonuniform": ((30, 17, 25), np.float64, 8, 1e-4, True, True, 53),
    "2d-70x45-f64-slab9-abs": ((70, 45), np.float64, 9, 2e-3, False, False, 54),
    "3d-20x33x33-f32-one-slab": ((20, 33, 33), np.float32, 64, 1e-2, True, False, 55),
}


def _case(name):
    shape, T, slab, tol, rel, nonuni, seed = CASES[name]
    u = fieldgen.spectral(shape, -5.0 / 3.0, seed).astype(T)
    rng = np.random.default_rng(seed)
    coords = [fieldgen.random_coords(n, rng) for n in shape] if nonuni else None
    return u, coords, slab, tol, rel


@pytest.mark.parametrize("name", list(CASES))
def test_chunked_container_and_decompression_equal_oracle(lib, name):
    import torch

    u, coords, slab, tol, rel = _case(name)
    say("compress", name)
    ref = K.compress_chunked(u, tol, slab, rel=rel, coords=coords)
    uh = torch.from_numpy(u).pin_memory()
    buf, nb = lib.mgard_compress_chunked(uh, tol, slab, coords=coords, eb="rel" if rel else "abs")
    got = buf[:nb].numpy().tobytes()
    assert nb == len(ref)
    assert got == ref
    say("decompress", name)
    rec = lib.mgard_decompress_chunked(buf, nb).numpy()
    want = K.decompress_chunked(ref)
    assert rec.dtype == u.dtype and rec.shape == u.shape
    assert np.array_equal(rec, want)
    tau = K.parse_chunked(ref)["tau_abs"]
    assert float(np.abs(rec.astype(np.float64) - u.astype(np.float64)).max()) <= tau


def test_chunked_pageable_host_memory_gives_the_same_bytes(lib):
    import torch

    u, coords, slab, tol, rel = _case("3d-60x33x41-f32-slab16")
    say("pageable")
    a, na = lib.mgard_compress_chunked(torch.from_numpy(u), tol, slab)
    b, nb = lib.mgard_compress_chunked(torch.from_numpy(u).pin_memory(), tol, slab)
    assert na == nb and torch.equal(a[:na], b[:nb])
    out = torch.empty(u.shape, dtype=torch.float32)
    rec = lib.mgard_decompress_chunked(a, na, out=out)
    assert np.array_equal(rec.numpy(), K.decompress_chunked(b[:nb].numpy().tobytes()))


def test_chunked_rejects_bad_arguments(lib):
    import torch

    u = torch.from_numpy(fieldgen.spectral((20, 17, 17), -2.0, 56).astype(np.float32))
    say("errors")
    with pytest.raises(lib.MgardError):
        lib.mgard_compress_chunked(u, 1e-3, 2)  # slabs need 3 planes
    with pytest.raises(lib.MgardError):
        lib.mgard_compress_chunked(u, 1e-3, 8, out=torch.empty(64, dtype=torch.uint8))  # capacity
    buf, nb = lib.mgard_compress_chunked(u, 1e-3, 8)
    bad = buf[:nb].clone()
    bad[100:108] = 255  # the slab offset table
    with pytest.raises(lib.MgardError):
        lib.mgard_decompress_chunked(bad, nb)


@pytest.mark.parametrize("keep", ["0", "1", "3"])
def test_chunked_slabs_kept_between_passes_or_not_give_the_same_bytes(lib, monkeypatch, keep):
    """With a relative tolerance the first slabs stay on the device between the
    max pass and the compression pass as memory allows; capping that count
    (none, one, some of the 5 slabs) must not change the bytes."""
    import torch

    u, coords, slab, tol, rel = _case("3d-60x33x41-f32-slab16")
    ref = K.compress_chunked(u, tol, 12)
    monkeypatch.setenv("MGARD_CHUNKED_KEEP", keep)
    say("keep", keep)
    buf, nb = lib.mgard_compress_chunked(torch.from_numpy(u).pin_memory(), tol, 12)
    assert buf[:nb].numpy().tobytes() == ref
