"""Pins of the second-stage lossless coder (oracle/lossless.py): a chunk coded
by hand, the size of a coded chunk from its definition (level-2 words plus
nonzero level-1 and data words), the raw fallback, round trips over lengths
and zero densities, and chunk independence."""
import json
import os

import numpy as np
import pytest

from oracle import lossless as Z

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_values.json")))


def test_chunk_coded_by_hand():
    g = GOLD["zero_suppression_chunk"]
    w = np.zeros(g["m"], dtype=np.uint32)
    for i, v in g["nonzero"].items():
        w[int(i)] = v
    stored = Z.code_chunk(w)
    assert [int(x) for x in stored] == g["stored"]
    assert np.array_equal(Z.decode_chunk(stored, g["m"]), w)


def test_all_zero_chunk_is_its_level2_bitmap():
    assert [int(x) for x in Z.code_chunk(np.zeros(4096, np.uint32))] == [0, 0, 0, 0]
    assert [int(x) for x in Z.code_chunk(np.zeros(5, np.uint32))] == [0]


@pytest.mark.parametrize("density", [0.0, 0.001, 0.05, 0.5, 0.97, 1.0])
def test_coded_length_from_the_definition(density):
    rng = np.random.default_rng(int(density * 1000) + 3)
    for m in [4096, 4000, 33, 1]:
        w = rng.integers(1, 2 ** 32, m, dtype=np.uint64).astype(np.uint32)
        w[rng.random(m) >= density] = 0
        n1 = (m + 31) // 32
        n2 = (n1 + 31) // 32
        nz1 = sum(1 for j in range(n1) if np.any(w[32 * j:32 * j + 32] != 0))
        coded = n2 + nz1 + int(np.count_nonzero(w))
        stored = Z.code_chunk(w)
        assert len(stored) == (coded if coded < m else m)
        assert np.array_equal(Z.decode_chunk(stored, m), w)


@pytest.mark.parametrize("nbytes", [0, 1, 3, 4, 4 * 4096, 4 * 4096 + 2, 4 * 4096 * 3 + 100, 200_003])
def test_round_trip(nbytes):
    rng = np.random.default_rng(nbytes)
    raw = rng.integers(0, 256, nbytes, dtype=np.uint8)
    raw[rng.random(nbytes) < 0.9] = 0  # mostly zero bytes
    data = raw.tobytes()
    enc = Z.encode(data)
    assert Z.decode(enc) == data


def test_chunks_are_independent():
    rng = np.random.default_rng(5)
    w = np.zeros(3 * 4096, np.uint32)
    w[rng.integers(0, len(w), 50)] = 1
    a = Z.encode(w.tobytes())
    w2 = w.copy()
    w2[4096 + 17] = 12345
    b = Z.encode(w2.tobytes())
    # chunk 0's stored words are unchanged, chunk 2's only moved
    oa = np.frombuffer(a, "<u8", 4, Z.FIXED)
    ob = np.frombuffer(b, "<u8", 4, Z.FIXED)
    da = np.frombuffer(a, "<u4", int(oa[-1]), Z.FIXED + 32)
    db = np.frombuffer(b, "<u4", int(ob[-1]), Z.FIXED + 32)
    assert np.array_equal(da[oa[0]:oa[1]], db[ob[0]:ob[1]])
    assert np.array_equal(da[oa[2]:oa[3]], db[ob[2]:ob[3]])
    assert Z.decode(b) == w2.tobytes()


def test_malformed_input():
    with pytest.raises(ValueError):
        Z.decode(b"MGHP" + bytes(40))
    enc = bytearray(Z.encode(np.zeros(100, np.uint32).tobytes()))
    enc[16] = 2  # chunk count
    with pytest.raises(ValueError):
        Z.decode(bytes(enc))
    with pytest.raises(ValueError):
        Z.decode_chunk(np.asarray([0x80000000], np.uint32), 40)  # level-1 word missing
