"""Pins of the oracle's key codec (App. "Lossless bit-level compression of
state information")."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import brute
import workloads as WL


def test_worked_example_packs_to_printed_words():
    # Worked example of the compression appendix: L=8 sites, d=16 (4 bits),
    # rows [6,0,0,1,0,2,0,15] and [14,0,0,0,0,0,0,1] in two 16-bit words.
    k1 = O.pack_fields([4] * 8, [6, 0, 0, 1, 0, 2, 0, 15], 1)[0]
    k2 = O.pack_fields([4] * 8, [14, 0, 0, 0, 0, 0, 0, 1], 1)[0]
    assert int(k1) == 0x6001020F
    assert int(k2) == 0xE0000001
    # the paper prints each row as two 16-bit words, most significant first
    assert (int(k1) >> 16, int(k1) & 0xFFFF) == (0b0110000000000001,
                                                 0b0000001000001111)
    assert (int(k2) >> 16, int(k2) & 0xFFFF) == (0b1110000000000000,
                                                 0b0000000000000001)


def test_fields_straddle_words():
    # 13 fields of 5 bits = 65 bits: field 0 sits at bits 60..64 and crosses
    # the boundary between word 1 (low) and word 0 (high).
    vals = [17, 3, 31, 0, 1, 2, 29, 8, 30, 4, 5, 6, 19]
    words = O.pack_fields([5] * 13, vals, 2)
    ref = 0
    for v in vals:
        ref = (ref << 5) | v
    assert [int(w) for w in words] == brute.int_to_words(ref, 2)


def test_memory_example_word_count():
    # 1e7 states of 100 sites with local dimension 8: the compressed table
    # needs ceil(100*3/32) = 10 four-byte words per row (382 MiB), the
    # uncompressed one 4 bytes per site (3.73 GiB).  The model codec adds
    # the 7-bit exciton field and still needs 40 bytes per row.
    omega = math.ceil(100 * math.log2(8) / 32)
    assert omega == 10
    assert abs(1e7 * omega * 4 / 2 ** 20 - 382) < 1   # 381.5 MiB
    assert round(1e7 * 100 * 4 / 2 ** 30, 2) == 3.73
    p = WL.model_params(dict(WL.CONFIGS["ring4"], extent=[100, 1, 1],
                             cutoff=[7]))
    m = O.Model(p)
    assert m.B == 100 * 3 + 7 and m.W == 5
    assert abs(1e7 * m.W * 8 / 2 ** 20 - 382) < 1


@pytest.mark.parametrize("name", ["ring4", "ring16", "sq6x6", "cube4", "ring12"])
def test_pack_matches_big_integer_and_round_trips(name):
    cfg = WL.CONFIGS[name]
    p = WL.model_params(cfg)
    m = O.Model(p)
    rng = np.random.default_rng(7)
    n = 200
    V = p["n_modes"]
    N = brute.sites(p)
    exc = rng.integers(0, N, n)
    occ = np.stack([rng.integers(0, p["cutoff"][f % V] + 1, n)
                    for f in range(N * V)], axis=1)
    keys = m.pack(exc, occ)
    for i in range(n):
        val, B = brute.key_int(p, int(exc[i]), occ[i])
        assert B == m.B
        assert [int(w) for w in keys[i]] == brute.int_to_words(val, m.W)
    e2, o2 = m.unpack(keys)
    assert np.array_equal(e2, exc) and np.array_equal(o2, occ)


def test_key_widths_of_workloads():
    expect = {"ring4": (14, 1), "ring16": (68, 2), "sq6x6": (150, 3),
              "cube4": (582, 10), "ring12": (52, 1)}
    for name, (B, W) in expect.items():
        m = O.Model(WL.model_params(WL.CONFIGS[name]))
        assert (m.B, m.W) == (B, W), name
