"""Seeded input generator: Philox4x32-10 known answers and R-MAT statistics."""
import numpy as np
import pytest

import rmatgen


# Known-answer vectors published with the Random123 reference implementation of
# Philox4x32-10 (Salmon et al., SC'11): (counter, key) -> output.
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    assert rmatgen.philox_block(ctr, key) == out


def test_philox_stream_layout():
    seed, stream = 0x1234_5678_9ABC, 7
    words = rmatgen.philox_words(seed, stream, 12, first=4)
    for w in range(12):
        b = (w + 4) // 4
        blk = rmatgen.philox_block([b & 0xFFFFFFFF, b >> 32, stream, 0],
                                   [seed & 0xFFFFFFFF, seed >> 32])
        assert words[w] == blk[(w + 4) % 4]


def test_rmat_quadrant_frequencies():
    # scale 1: one quadrant draw per edge; frequencies must match a/b/c/d.
    keys = rmatgen.rmat_keys(1, 400_000, seed=11)
    u = (keys >> np.uint64(32)).astype(np.int64)
    v = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    q = 2 * u + v
    freq = np.bincount(q, minlength=4) / len(q)
    expect = np.array([0.57, 0.19, 0.19, 0.05])
    sd = np.sqrt(expect * (1 - expect) / len(q))
    assert np.all(np.abs(freq - expect) < 5 * sd)


def test_rmat_keys_are_a_function_of_index():
    full = rmatgen.rmat_keys(12, 4, seed=3)
    part = rmatgen.rmat_keys(12, 4, seed=3, first=1000, count=500)
    assert np.array_equal(full[1000:1500], part)
    assert not np.array_equal(full, rmatgen.rmat_keys(12, 4, seed=4))


def test_rmat_edges_sorted_unique_in_range():
    src, dst = rmatgen.rmat_edges(10, 8, seed=1)
    keys = src.astype(np.int64) * 2**32 + dst
    assert np.all(np.diff(keys) > 0)
    assert src.min() >= 0 and src.max() < 1024 and dst.min() >= 0 and dst.max() < 1024
    assert len(src) < 8 * 1024


def test_derived_draws():
    w = rmatgen.uniform_f32(5, 10000, 0.1, 1.0)
    assert w.dtype == np.float32 and w.min() >= 0.1 and w.max() < 1.0
    z = rmatgen.normal_f32(5, 20000)
    assert abs(float(z.mean())) < 0.05 and abs(float(z.std()) - 1) < 0.05
    elig = np.zeros(100, dtype=bool)
    elig[::3] = True
    v = rmatgen.distinct_vertices(9, 20, 100, eligible=elig)
    assert len(set(v.tolist())) == 20 and all(elig[v])
    src = np.array([0, 0, 1, 2, 2, 2], dtype=np.int32)
    wn = rmatgen.row_normalized_weights(src, 4, seed=1)
    sums = np.bincount(src, weights=wn.astype(np.float64), minlength=4)
    assert np.allclose(sums[:3], 1.0, atol=1e-6) and sums[3] == 0
