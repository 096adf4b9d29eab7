"""GPU parity of the L2 / s-norm bound (MGARD_NORM_S) against the oracle.

The relative bound needs ||u||, a float64 sum over the field that the device
and the oracle add up in different orders: the tolerance taken from it is
compared within 1e-12 relative, then the oracle is given the device's tau, and
everything after it (widths, symbols, escapes, the whole buffer) must agree
byte for byte.  Absolute bounds agree byte for byte from the start.  The
decompressed fields meet the bound in the oracle's float64 s-norm.
"""
import math
import zlib

import numpy as np
import pytest
import torch

import fieldgen
from oracle import codec, grid
from oracle import snorm as SN

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[snorm]", *a, flush=True)


def dev(x):
    return torch.from_numpy(np.array(x, order="C")).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    "2d-65x65-f64-unit": ((65, 65), np.float64, "unit"),
    "2d-64x50-f32": ((64, 50), np.float32, None),
    "3d-33x20x17-f32-nonuniform": ((33, 20, 17), np.float32, "rand"),
    "3d-17x18x19-f64-nonuniform": ((17, 18, 19), np.float64, "rand"),
    "4d-9x10x7x6-f64": ((9, 10, 7, 6), np.float64, "rand"),
    "batchdims-2x65x1x33-f32": ((2, 65, 1, 33), np.float32, "unit"),
    "1d-1000-f64": ((1000,), np.float64, "unit"),
}


def make_case(name):
    shape, T, cmode = CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    u = fieldgen.random_field(shape, rng).astype(T)
    if cmode == "rand":
        coords = [fieldgen.random_coords(n, rng) for n in shape]
    elif cmode == "unit":
        coords = [np.linspace(0.0, 1.0, n) if n > 1 else None for n in shape]
    else:
        coords = None
    return u, coords


@pytest.mark.parametrize("name", list(CASES))
def test_l2_norm_matches_oracle(lib, name):
    u, coords = make_case(name)
    say("l2 norm", name)
    h = grid.Hierarchy(u.shape, coords)
    ref = math.sqrt(SN.l2_norm_sq(u, h))
    got = lib.mgard_l2_norm(dev(u), coords)
    assert abs(got - ref) <= 1e-12 * ref, (got, ref)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("s,eb,tol", [(0.0, "rel", 1e-3), (0.0, "rel", 1e-4), (0.0, "abs", 1e-3), (1.0, "abs", 1e-3),
                                      (-1.0, "abs", 1e-3), (0.5, "abs", 1e-2)])
def test_snorm_bytes_and_bound(lib, name, s, eb, tol):
    u, coords = make_case(name)
    T = u.dtype.type
    h = grid.Hierarchy(u.shape, coords)
    if eb == "abs":
        tol = tol * math.sqrt(SN.l2_norm_sq(u, h))  # an absolute bound of the field's own scale
    say("s-norm", name, s, eb, tol)
    rel = eb == "rel"
    try:
        ref_parts = codec.compress_parts(u, tol, rel=rel, coords=coords, norm="s", s=s)
    except ValueError:
        with pytest.raises(lib.MgardError) as e:
            lib.mgard_compress(dev(u), tol, coords, eb=eb, norm="s", s=s)
        assert e.value.code == -4
        return
    buf, nb, info = lib.mgard_compress(dev(u), tol, coords, eb=eb, norm="s", s=s)
    got = host(buf[:nb]).tobytes()
    hd = codec.parse(got)
    assert hd.norm == codec.NORM_S and hd.s == s
    if rel:
        assert abs(hd.tau_abs - ref_parts.tau_abs) <= 1e-12 * ref_parts.tau_abs
    else:
        assert hd.tau_abs == ref_parts.tau_abs
    # with the device's tau the oracle writes the same bytes
    ref = codec.compress(u, tol, rel=rel, coords=coords, norm="s", s=s, tau=hd.tau_abs)
    assert len(got) == len(ref) and got == ref
    bins, tau = lib.mgard_bin_widths(dev(u), tol, coords, eb=eb, norm="s", s=s)
    assert bins == hd.bins and tau == hd.tau_abs
    r = host(lib.mgard_decompress(buf, nb))
    assert np.array_equal(r, codec.decompress(ref))
    e = r.astype(np.float64) - u.astype(np.float64)
    err2 = SN.s_norm_sq(e, h, s)
    assert err2 <= hd.tau_abs ** 2, (math.sqrt(err2), hd.tau_abs)


def test_snorm_refusals(lib):
    u = dev(fieldgen.bumps2d(33).astype(np.float32))
    for kw in (dict(eb="rel", norm="s", s=1.0), dict(alloc="count", norm="s"), dict(alloc="learned", norm="s")):
        with pytest.raises(lib.MgardError) as e:
            lib.mgard_compress(u, 1e-3, **kw)
        assert e.value.code == -1, kw
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_compress(u, 1e-8, norm="s")
    assert e.value.code == -4
