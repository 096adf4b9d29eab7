"""The side-stream overlaps stay ordered with the caller's stream.

Compression counts the finest level's chunks on a per-device side stream, and
decompression runs the finest level's correction there; both fork from and
join back to the stream the call is enqueued on.  Calls issued on a
non-default stream must give the bytes and fields the same calls give on the
default stream (which the parity tests tie to the oracle): a missing join
would let a call's end-of-call synchronisation, or the next call's kernels,
run ahead of the side-stream work.  The shapes are 3D with levels above the
small-level kernels, so both overlaps are taken.
"""
import pytest

import fieldgen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[streams]", *a, flush=True)


def _fields(torch):
    specs = [((65, 70, 60), 31, torch.float32), ((40, 97, 33), 32, torch.float32), ((50, 45, 66), 33, torch.float64)]
    return [fieldgen.spectral(shape, -5.0 / 3.0, seed, device="cuda").to(dt).contiguous() for shape, seed, dt in specs]


def test_side_stream_work_is_ordered_on_a_user_stream(lib):
    import torch

    fields = _fields(torch)
    tol = 1e-3
    say("reference on the default stream")
    ref = []
    for u in fields:
        buf, nb, _ = lib.mgard_compress(u, tol)
        ref.append((buf[:nb].clone(), lib.mgard_decompress(buf, nb).clone()))
    torch.cuda.synchronize()

    s = torch.cuda.Stream()
    outs = []
    say("on a user stream")
    with torch.cuda.stream(s):
        for rep in range(3):
            for u in fields:
                buf, nb, _ = lib.mgard_compress(u, tol)
                outs.append((buf, nb, lib.mgard_decompress(buf, nb)))
    s.synchronize()
    for k, (buf, nb, rec) in enumerate(outs):
        i = k % len(fields)
        want_bytes, want_rec = ref[i]
        assert nb == want_bytes.numel(), k
        assert torch.equal(buf[:nb], want_bytes), k
        assert torch.equal(rec, want_rec), k
