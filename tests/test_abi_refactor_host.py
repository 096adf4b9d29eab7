"""Host-only refactoring calls of the C-ABI against the oracle (no GPU work).

The metadata comes from the oracle's own refactoring of seeded fields, so the
library's retrieval plan (mgard_refactor_request), byte ranges
(mgard_refactor_ranges) and metadata parser (mgard_refactor_inspect) are
checked against oracle/refactor.py's greedy retrieval and layout: plane
counts equal, estimates equal to the last bit (same float64 expressions in
the same order on both sides).
"""
import numpy as np
import pytest

import fieldgen
import paper_2401_05994_amd as m
from oracle import refactor as RF


def _meta(shape, seed, T, B, nonuniform):
    u = fieldgen.spectral(shape, -5.0 / 3.0, seed).astype(T)
    coords = None
    if nonuniform:
        rng = np.random.default_rng(seed + 7)
        coords = [np.cumsum(rng.uniform(0.5, 1.5, n)) for n in shape]
    buf = RF.serialize(RF.refactor(u, B, coords))
    meta = RF.parse(buf)
    return buf, meta


CASES = [((33, 33), 1, np.float64, 32, False), ((17, 19, 21), 2, np.float32, 32, True),
         ((65,), 3, np.float32, 16, False), ((9, 10, 11), 4, np.float64, 24, True),
         ((5, 6, 7, 5), 5, np.float32, 32, False)]


@pytest.mark.parametrize("shape,seed,T,B,nonuni", CASES)
def test_request_and_ranges_equal_the_oracle(shape, seed, T, B, nonuni):
    buf, meta = _meta(shape, seed, T, B, nonuni)
    head = buf[:meta.meta_bytes]
    mb, L, Bl, tot = m.mgard_refactor_inspect(head)
    assert (mb, L, Bl, tot) == (meta.meta_bytes, meta.L, B, len(buf))
    for norm, s, rel in [("linf", 0.0, True), ("linf", 0.0, False), ("s", 0.0, True), ("s", 1.0, False),
                         ("s", -1.0, False)]:
        have = None
        for tol in [1e-1, 1e-2, 1e-3, 1e-5]:
            t = tol if rel else tol * meta.maxabs
            want, est = m.mgard_refactor_request(head, t, have=have, eb="rel" if rel else "abs", norm=norm, s=s)
            ow, oest = RF.request(meta, t, rel=rel, norm=norm, s=s, have=have)
            assert want == ow and est == oest, (norm, s, rel, tol)
            h0 = have if have is not None else [0] * (L + 1)
            assert m.mgard_refactor_ranges(head, have, want) == RF.segment_ranges(meta, h0, want)
            have = want


def test_refactor_metadata_refusals():
    buf, meta = _meta((17, 17), 6, np.float32, 8, False)
    head = buf[:meta.meta_bytes]
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_inspect(head[:40])
    assert e.value.code == -6  # more bytes needed
    bad = bytearray(head)
    bad[8] = 40  # 40 planes
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_inspect(bytes(bad))
    assert e.value.code == -7
    bad = bytearray(head)
    bad[0:4] = b"MGHP"
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_request(bytes(bad), 1e-3)
    assert e.value.code == -7
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_request(head, 0.0)
    assert e.value.code == -4
    # held planes above B are refused
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_request(head, 1e-3, have=[9] * (meta.L + 1))
    assert e.value.code == -1
    # a level offset table that does not match the shape is malformed: its last
    # entry (the segment area's size) sits after the fixed part, the shape,
    # the exponents and the residual table
    import struct

    bad = bytearray(head)
    pos = 32 + 8 * 2 + 4 * (meta.L + 1) + 4 * (meta.L + 1) * (8 + 1) + 8 * (meta.L + 1)
    assert struct.unpack_from("<Q", head, pos)[0] == meta.level_off[-1]
    struct.pack_into("<Q", bad, pos, meta.level_off[-1] + 4)
    with pytest.raises(m.MgardError) as e:
        m.mgard_refactor_request(bytes(bad), 1e-3)
    assert e.value.code == -7
