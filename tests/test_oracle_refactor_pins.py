"""Pins of the refactoring oracle (bitplane segments, error table, greedy retrieval).

Each pin ties oracle/refactor.py to something other than itself: a worked
example derived by hand (tests/golden/hand_values.json), brute-force maxima
over every plane count, the end-to-end error of reconstructions against the
requested tolerance (L-infinity and s-norm), the layout of the segment area
(a buffer holding only the fetched byte ranges reconstructs the same field),
and the retrieval order's independence of the tolerance.
"""
import json
import math
import os

import numpy as np
import pytest

import fieldgen
from oracle import quant as Q
from oracle import refactor as RF
from oracle import snorm as SN
from oracle import transform as X
from oracle.grid import Hierarchy

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_values.json")))


def test_bitplanes_hand_example():
    g = GOLD["bitplanes_small"]
    c = np.asarray(g["c"], dtype=np.float64)
    B = g["planes"]
    e = RF.level_exponent(float(np.abs(c).max()))
    assert e == g["exponent"]
    m, s = RF.magnitudes(c, e, B)
    assert [int(v) for v in RF.pack_bits(s)] == [g["sign_word"]]
    words = [int(RF.pack_bits((m >> np.uint64(B - 1 - k)) & np.uint64(1))[0]) for k in range(B)]
    assert words == g["plane_words"]
    assert RF.residual_table(m, B) == g["R"]
    m2 = m & ~np.uint64((1 << (B - 2)) - 1)
    rec = np.where(s == 1, -1.0, 1.0) * np.ldexp(m2.astype(np.float64), e - B)
    assert list(rec) == g["reconstruct_2_planes"]


class _FixedEstimator:
    """Greedy inputs given directly: terms w_l E_l[k], unit plane cost (double for the first plane)."""

    def __init__(self, w, E):
        self.w, self.E = w, E

    def term(self, l, k):
        return self.w[l] * self.E[l][k]

    def estimate(self, k):
        return sum(self.term(l, k[l]) for l in range(len(k)))

    def cost(self, l, k):
        return 2.0 if k == 0 else 1.0


def test_greedy_hand_example():
    g = GOLD["refactor_greedy_two_levels"]
    est = _FixedEstimator(g["w"], g["E"])
    k = [0, 0]
    order = []
    for _ in range(4):
        # a tolerance just below the current estimate: exactly one more plane
        before = list(k)
        k = RF.greedy(est, est.estimate(k) - 1e-12, k, 2, [True, True])
        assert sum(k) == sum(before) + 1
        order.append([l for l in range(2) if k[l] != before[l]][0])
    assert order == g["order"]
    assert RF.greedy(est, g["tau"], [0, 0], 2, [True, True]) == g["planes_at_tau"]


def _field(shape, seed, T, nonuniform=False):
    u = fieldgen.spectral(shape, -5.0 / 3.0, seed).astype(T)
    coords = None
    if nonuniform:
        rng = np.random.default_rng(seed + 100)
        coords = [np.cumsum(rng.uniform(0.5, 1.5, n)) for n in shape]
    return u, coords


CASES = [((33, 33), 1, np.float64, False), ((17, 19, 21), 2, np.float32, True), ((65,), 3, np.float32, False),
         ((9, 10, 11), 4, np.float64, True), ((5, 6, 7, 5), 5, np.float32, False)]


@pytest.mark.parametrize("shape,seed,T,nonuni", CASES)
def test_residual_table_is_the_brute_force_maximum(shape, seed, T, nonuni):
    """For every level and plane count k: max |c - c^_k| (float64, before the cast to T)
    lies in [R[k], R[k] + 1) units of 2^(e - B), and every |c - T(c^_k)| <= E[k]."""
    u, coords = _field(shape, seed, T, nonuni)
    B = 20
    r = RF.refactor(u, B, coords)
    buf = RF.serialize(r)
    meta = RF.parse(buf)
    hier = Hierarchy(u.shape, coords)
    coarsest, cbars = X.decompose(u, hier, T)
    stream = Q.to_stream(coarsest, cbars, hier).astype(np.float64)
    off = Q.level_offsets(hier)
    for l in range(hier.L + 1):
        c = stream[off[l]:off[l + 1]]
        e = meta.exps[l]
        E = RF.level_errors(meta, l)
        for k in range(B + 1):
            planes = [0] * (hier.L + 1)
            planes[l] = k
            ck = RF.reconstruct_stream(buf, meta, planes)[off[l]:off[l + 1]]
            if e is None:
                assert np.all(ck == 0)
                continue
            m, s = RF.magnitudes(c, e, B)
            mk = m & ~np.uint64((1 << (B - k)) - 1)
            exact = np.where(s == 1, -1.0, 1.0) * np.ldexp(mk.astype(np.float64), e - B)
            unit = math.ldexp(1.0, e - B)
            worst = float(np.max(np.abs(c - exact)))
            assert meta.R[l][k] * unit <= worst < (meta.R[l][k] + 1) * unit
            assert float(np.max(np.abs(c - ck.astype(np.float64)))) <= E[k]


@pytest.mark.parametrize("shape,seed,T,nonuni", CASES)
def test_reconstruction_meets_the_requested_linf_tolerance(shape, seed, T, nonuni):
    u, coords = _field(shape, seed, T, nonuni)
    buf = RF.serialize(RF.refactor(u, 32, coords))
    meta = RF.parse(buf)
    prev = [0] * (meta.L + 1)
    for tol in [1e-1, 1e-2, 1e-3, 1e-4]:
        k, est = RF.request(meta, tol, rel=True, have=prev)
        assert all(a >= b for a, b in zip(k, prev))  # only adds segments
        tau = tol * meta.maxabs
        rec = RF.reconstruct(buf, k)
        err = float(np.max(np.abs(rec.astype(np.float64) - u.astype(np.float64))))
        assert est <= tau and err <= est
        prev = k
    # the estimate with every plane is the smallest one can get
    kall, _ = RF.request(meta, 1e-30, rel=False)
    assert kall == [32 if e is not None else 0 for e in meta.exps]


def test_retrieval_order_does_not_depend_on_the_tolerance():
    """A request from the planes held at a looser tolerance equals the request
    made from nothing (the greedy picks one fixed sequence and stops by tau)."""
    u, coords = _field((33, 35, 31), 7, np.float32, True)
    meta = RF.parse(RF.serialize(RF.refactor(u, 24, coords)))
    for t1, t2 in [(1e-2, 1e-3), (1e-3, 1e-5), (3e-2, 2e-2)]:
        k1, _ = RF.request(meta, t1)
        assert RF.request(meta, t2, have=k1)[0] == RF.request(meta, t2)[0]


def test_segment_ranges_hold_everything_the_reconstruction_reads():
    """A buffer holding only the metadata and the fetched byte ranges reconstructs
    the same field as the whole buffer, request after request."""
    u, coords = _field((31, 29), 8, np.float64, True)
    buf = RF.serialize(RF.refactor(u, 32, coords))
    meta = RF.parse(buf)
    part = bytearray(len(buf))
    part[:meta.meta_bytes] = buf[:meta.meta_bytes]
    have = [0] * (meta.L + 1)
    for tol in [1e-1, 1e-3, 1e-6]:
        want, _ = RF.request(meta, tol, have=have)
        for off, n in RF.segment_ranges(meta, have, want):
            assert part[off:off + n] == bytes(n)  # never fetched before
            part[off:off + n] = buf[off:off + n]
        have = want
        assert np.array_equal(RF.reconstruct(bytes(part), have), RF.reconstruct(buf, have))


@pytest.mark.parametrize("s", [0.0, 1.0, -1.0])
def test_reconstruction_meets_the_snorm_request(s):
    u, coords = _field((33, 33), 9, np.float64, True)
    buf = RF.serialize(RF.refactor(u, 32, coords))
    meta = RF.parse(buf)
    hier = Hierarchy(u.shape, coords)
    for tol in [1e-1, 1e-3]:
        rel = s == 0.0
        tt = tol if rel else tol * math.sqrt(SN.s_norm_sq(u, hier, s))
        k, est = RF.request(meta, tt, rel=rel, norm="s", s=s)
        rec = RF.reconstruct(buf, k)
        err = math.sqrt(max(SN.s_norm_sq(rec - u, hier, s), 0.0))
        tau = tt * meta.l2norm if rel else tt
        assert est <= tau and err <= est


def test_all_zero_levels_and_refusals():
    u = np.zeros((9, 9), dtype=np.float32)
    buf = RF.serialize(RF.refactor(u, 8))
    meta = RF.parse(buf)
    assert all(e is None for e in meta.exps)
    k, est = RF.request(meta, 1e-3, rel=False)
    assert k == [0] * (meta.L + 1)
    assert np.all(RF.reconstruct(buf, k) == 0)
    with pytest.raises(ValueError):
        RF.refactor(np.ones((5, 5), np.float32), 33)
    with pytest.raises(ValueError):
        RF.request(meta, 0.0)
    with pytest.raises(ValueError):
        RF.parse(b"MGHP" + bytes(60))
