"""Batched compression (one graph launch for many uneven fields) and the autotuner.

A batch must produce, for every field, exactly the bytes a single
mgard_compress call produces (whose bytes the parity tests tie to the oracle),
on every replay of the captured graph, with unrelated eager work between
replays.  Tuning changes launch shapes only, never the bytes.
"""
import json

import numpy as np
import pytest

import fieldgen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[batch]", *a, flush=True)


def _fields(torch):
    specs = [((65, 90), "f32", 11), ((100, 70), "f64", 12), ((33, 40, 35), "f32", 13), ((50, 33, 45), "f32", 14),
             ((20, 24, 17), "f64", 15), ((129, 65), "f32", 16), ((17, 17, 17), "f32", 17), ((3, 40, 9), "f32", 18)]
    out, coords = [], []
    for shape, dt, seed in specs:
        u = fieldgen.spectral(shape, -3.0, seed, device="cuda")
        out.append(u.to(torch.float32 if dt == "f32" else torch.float64).contiguous())
        coords.append(None)
    # one nonuniform 3D field
    coords[4] = [fieldgen.geometric_coords(n) for n in specs[4][0]]
    return out, coords


def test_batch_matches_single_calls(lib):
    import torch

    fields, coords = _fields(torch)
    tol = 1e-3
    say("plan", len(fields), "fields")
    b = lib.Batch(fields, tol, coords=coords)
    refs = []
    for f, c in zip(fields, coords):
        buf, nb, _ = lib.mgard_compress(f, tol, c)
        refs.append(buf[:nb].clone())
    other = fieldgen.spectral((64, 64), -2.0, 99, device="cuda").to(torch.float32)
    for rep in range(3):
        say("replay", rep)
        b.launch()
        lib.mgard_compress(other, 1e-2)  # eager work between replays
        res = b.results()
        for i, (got, size) in enumerate(res):
            assert size == refs[i].numel(), (rep, i)
            assert torch.equal(got, refs[i]), (rep, i)
    for i, (got, size) in enumerate(b.results()):
        rec = lib.mgard_decompress(got, size)
        f = fields[i]
        tau = tol * float(f.abs().max())
        assert float((rec - f).abs().max()) <= tau
    b.close()


def test_batch_rejects_learned_and_small_output(lib):
    import torch

    f = fieldgen.spectral((33, 33), -2.0, 3, device="cuda").to(torch.float32)
    with pytest.raises(lib.MgardError):
        lib.Batch([f], 1e-3, alloc="learned")
    with pytest.raises(lib.MgardError):
        lib.Batch([f], -1.0)


def test_autotune_records_every_level_and_keeps_bytes(lib, tmp_path, monkeypatch):
    import torch

    path = tmp_path / "tune.json"
    monkeypatch.setenv("MGARD_TUNE_FILE", str(path))
    u = fieldgen.spectral((41, 37, 45), -5.0 / 3.0, 21, device="cuda").to(torch.float32)
    buf, nb, info = lib.mgard_compress(u, 1e-3)
    before = buf[:nb].clone()
    say("autotune", tuple(u.shape))
    lib.mgard_autotune(u)
    buf, nb2, _ = lib.mgard_compress(u, 1e-3)
    assert nb2 == nb and torch.equal(buf[:nb2], before)
    table = json.loads(path.read_text())
    L, offs = lib.mgard_stream_layout(u.shape)
    sizes = [tuple(u.shape)]
    for _ in range(L - 1):
        sizes.append(tuple(s // 2 + 1 for s in sizes[-1]))
    for s in sizes:
        key = "%dx%dx%d" % s
        assert table["coeff_seg:f32:" + key] >= 1
        assert table["scatter_planes:f32:" + key] >= 1
    rec = lib.mgard_decompress(buf, nb2)
    assert float((rec - u).abs().max()) <= info["tau_abs"]


def test_batch_reports_nonfinite_fields(lib):
    """A field holding a NaN or an infinity gets size 0 in the batch's size
    array; the other fields still match their single compressions."""
    import torch

    good = fieldgen.spectral((40, 33), -3.0, 31, device="cuda").to(torch.float32).contiguous()
    nanf = good.clone()
    nanf[5, 7] = float("nan")
    inff = fieldgen.spectral((17, 20, 19), -3.0, 32, device="cuda").to(torch.float64).contiguous()
    inff[3, 4, 5] = float("inf")
    say("nonfinite fields")
    b = lib.Batch([good, nanf, inff], 1e-3)
    b.launch()
    res = b.results()
    assert res[1][1] == 0 and res[2][1] == 0
    buf, nb, _ = lib.mgard_compress(good, 1e-3)
    assert res[0][1] == nb and torch.equal(res[0][0], buf[:nb])
    b.close()



def test_batch_256_uneven_fields_match_single_calls(lib):
    """The 256-field uneven-shape batch the benchmark times (2D 65..2049 per side,
    3D 33..257, slopes U[-4, -5/3], rel tol 1e-3): every batched field equals its
    single compression byte for byte, and the smallest 2D and 3D fields equal the
    oracle's bytes."""
    import torch

    from oracle import codec

    specs = fieldgen.batch_specs()
    host, fields = [], []
    for i, sp in enumerate(specs):
        h = fieldgen.spectral(sp.shape, sp.beta, sp.seed).astype(np.float32)
        host.append(h)
        fields.append(torch.from_numpy(h).cuda())
        if (i + 1) % 64 == 0:
            say("generated", i + 1, "fields")
    tol = 1e-3
    say("plan 256 fields")
    b = lib.Batch(fields, tol)
    b.launch()
    res = b.results()
    for i, f in enumerate(fields):
        buf, nb, _ = lib.mgard_compress(f, tol)
        assert res[i][1] == nb, (i, specs[i].shape)
        assert torch.equal(res[i][0], buf[:nb]), (i, specs[i].shape)
        if (i + 1) % 64 == 0:
            say("compared", i + 1, "fields")
    for D in (2, 3):
        k = min((i for i in range(len(specs)) if len(specs[i].shape) == D), key=lambda i: host[i].size)
        say("oracle bytes", specs[k].shape)
        assert res[k][0].cpu().numpy().tobytes() == codec.compress(host[k], tol), specs[k].shape
    b.close()
