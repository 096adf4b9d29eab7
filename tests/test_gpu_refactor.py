"""Refactoring on the GPU against the oracle, through the C-ABI.

* the whole refactored buffer (metadata with exponents, residual table,
  max|u| and ||u||, then every bitplane segment) equals the oracle's byte
  for byte, on 1D-4D, float32/float64, uniform and nonuniform grids and
  several plane counts;
* reconstructions from the plane counts the retrieval plan asks for, at a
  sequence of tolerances (progressive: each request starts from the planes
  already held and the buffer holds only the fetched ranges), equal the
  oracle's reconstructions value for value and meet the requested bound;
* at full size (513^3 float32), the metadata equals the oracle's computed
  from the library's own coefficient stream (whose equality with the
  oracle's decomposition the full-size decomposition test establishes),
  sampled segment words equal the oracle's packing, and reconstructions meet
  the requested L-infinity bound.
"""
import numpy as np
import pytest

import fieldgen
from oracle import quant as Q
from oracle import refactor as RF
from oracle.grid import Hierarchy

pytestmark = pytest.mark.gpu


def say(*a):
    print("[refactor]", *a, flush=True)


def _field(shape, seed, T, nonuniform):
    u = fieldgen.spectral(shape, -5.0 / 3.0, seed).astype(T)
    coords = None
    if nonuniform:
        rng = np.random.default_rng(seed + 11)
        coords = [np.cumsum(rng.uniform(0.5, 1.5, n)) for n in shape]
    return u, coords


CASES = [((65, 65), 1, np.float64, 32, False), ((33, 34, 35), 2, np.float32, 32, True),
         ((1000,), 3, np.float32, 20, False), ((17, 18, 19), 4, np.float64, 32, True),
         ((9, 8, 7, 6), 5, np.float32, 12, False), ((129, 130, 131), 6, np.float32, 32, False),
         ((3, 5), 7, np.float64, 32, False)]


@pytest.mark.parametrize("shape,seed,T,B,nonuni", CASES)
def test_refactored_buffer_equals_the_oracle(lib, shape, seed, T, B, nonuni):
    import torch

    u, coords = _field(shape, seed, T, nonuni)
    say("refactor", shape, T.__name__, B)
    ud = torch.from_numpy(u.copy()).cuda()
    # ||u|| is a float64 sum taken in another order on the device: equal to
    # the oracle's to rounding, and then the oracle takes the device's value
    l2 = lib.mgard_l2_norm(ud, coords)
    r = RF.refactor(u, B, coords)
    assert abs(l2 - r.l2norm) <= 1e-13 * r.l2norm
    ref = RF.serialize(RF.refactor(u, B, coords, l2norm=l2))
    buf, nb = lib.mgard_refactor(ud, B, coords)
    assert nb == len(ref) == lib.mgard_refactor_bound(shape, lib.F64 if T is np.float64 else lib.F32, B, coords)
    got = buf[:nb].cpu().numpy().tobytes()
    assert got == ref


@pytest.mark.parametrize("shape,seed,T,B,nonuni", CASES)
def test_progressive_reconstruction_equals_the_oracle(lib, shape, seed, T, B, nonuni):
    import torch

    u, coords = _field(shape, seed, T, nonuni)
    buf, nb = lib.mgard_refactor(torch.from_numpy(u.copy()).cuda(), B, coords)
    host = buf[:nb].cpu().numpy().tobytes()
    meta = RF.parse(host)
    head = host[:meta.meta_bytes]
    # the buffer a reader fills in: metadata, then only the fetched ranges
    part = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    part[:meta.meta_bytes] = buf[:meta.meta_bytes]
    have = None
    for tol in [1e-1, 1e-2, 1e-3, 1e-4, 1e-6]:
        want, est = lib.mgard_refactor_request(head, tol, have=have)
        for off, n in lib.mgard_refactor_ranges(head, have, want):
            part[off:off + n] = buf[off:off + n]
        rec = lib.mgard_reconstruct(part, nb, want).cpu().numpy()
        ora = RF.reconstruct(host, want)
        assert rec.dtype == ora.dtype and np.array_equal(rec, ora), tol
        err = float(np.max(np.abs(rec.astype(np.float64) - u.astype(np.float64))))
        assert err <= est
        if est > tol * meta.maxabs:  # only when every plane is held already
            assert want == [B if e is not None else 0 for e in meta.exps]
        have = want


def test_snorm_request_and_reconstruction(lib):
    import torch

    u, coords = _field((65, 66), 8, np.float64, True)
    buf, nb = lib.mgard_refactor(torch.from_numpy(u.copy()).cuda(), 32, coords)
    host = buf[:nb].cpu().numpy().tobytes()
    meta = RF.parse(host)
    for tol in [1e-2, 1e-4]:
        want, est = lib.mgard_refactor_request(host[:meta.meta_bytes], tol, norm="s", s=0.0)
        assert (want, est) == RF.request(meta, tol, norm="s", s=0.0)
        rec = lib.mgard_reconstruct(buf, nb, want).cpu().numpy()
        assert np.array_equal(rec, RF.reconstruct(host, want))


def test_refactor_errors(lib):
    import torch

    u = torch.ones((9, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_refactor(u, 33)
    assert e.value.code == -1
    u[3, 4] = float("nan")
    with pytest.raises(lib.MgardError) as e:
        lib.mgard_refactor(u, 16)
    assert e.value.code == -5
    good = torch.ones((9, 9), dtype=torch.float32, device="cuda")
    buf, nb = lib.mgard_refactor(good, 16)
    L = RF.parse(buf[:nb].cpu().numpy().tobytes()).L
    with pytest.raises(lib.MgardError) as e:  # more planes than stored
        lib.mgard_reconstruct(buf, nb, [17] * (L + 1))
    assert e.value.code == -1
    with pytest.raises(lib.MgardError) as e:  # truncated
        lib.mgard_reconstruct(buf, nb - 4, [16] * (L + 1))
    assert e.value.code == -7


def test_fullsize_refactor_513_f32(lib):
    import torch

    n = 513
    say("generate", n)
    u = fieldgen.spectral((n, n, n), -5.0 / 3.0, 2, device="cuda").to(torch.float32).contiguous()
    shape = tuple(u.shape)
    B = 32
    say("refactor")
    buf, nb = lib.mgard_refactor(u, B)
    meta = RF.parse(buf[:65536].cpu().numpy().tobytes())
    hier = Hierarchy(shape)
    say("decompose (library) for the oracle's metadata")
    stream = lib.mgard_decompose(u).cpu().numpy()
    off = Q.level_offsets(hier)
    assert abs(meta.maxabs - float(u.abs().max())) == 0.0
    rng = np.random.default_rng(3)
    for l in range(hier.L + 1):
        c = stream[off[l]:off[l + 1]]
        e = RF.level_exponent(float(np.max(np.abs(c.astype(np.float64)))))
        assert meta.exps[l] == e
        m_, s_ = RF.magnitudes(c, e, B)
        assert meta.R[l] == RF.residual_table(m_, B), l
        W = RF.words_per_plane(len(c))
        # sampled words of every plane: the first, the last and 64 random ones
        idx = np.unique(np.concatenate([[0, W - 1], rng.integers(0, W, 64)]))
        seg0 = meta.meta_bytes + meta.level_off[l]
        words = buf[seg0:seg0 + 4 * W * (B + 1)].cpu().numpy().view(np.uint32).reshape(B + 1, W)
        for wi in idx:
            lo, hi = 32 * int(wi), min(32 * int(wi) + 32, len(c))
            assert int(words[0, wi]) == int(RF.pack_bits(s_[lo:hi])[0])
            for k in range(B):
                ref = int(RF.pack_bits((m_[lo:hi] >> np.uint64(B - 1 - k)) & np.uint64(1))[0])
                assert int(words[1 + k, wi]) == ref, (l, k, wi)
    head = buf[:meta.meta_bytes].cpu().numpy().tobytes()
    have = None
    for tol in [1e-2, 1e-3, 1e-4]:
        want, est = lib.mgard_refactor_request(head, tol, have=have)
        rec = lib.mgard_reconstruct(buf, nb, want)
        err = float((rec.double() - u.double()).abs().max())
        tau = tol * meta.maxabs
        fetched = sum(length for _, length in lib.mgard_refactor_ranges(head, None, want))
        say(f"tol {tol}: planes {want}, fetched {fetched / 1e6:.1f} MB of {nb / 1e6:.1f} MB, "
            f"error/tau {err / tau:.3f}, estimate/tau {est / tau:.3f}")
        assert err <= est <= tau
        have = want
