"""Pins of the oracle's XXH64 and ODP-D64 against things other than itself.

XXH64: the independent python ``xxhash`` package (a separate implementation of
the public xxHash specification). ODP-D64: a composition of ``xxhash`` calls
written out below, sharing nothing with the oracle.
"""
import os

import numpy as np
import pytest

import oracle

xxhash = pytest.importorskip("xxhash")


def ref_xxh64(b, seed=0):
    return xxhash.xxh64_intdigest(bytes(b), seed)


def ref_d64(b):
    """ODP-D64 v1 composed from xxhash: 4096-byte leaves (seed 0), then groups of
    64 child digests, little-endian, hashed with seed = level, until one is left."""
    b = bytes(b)
    if len(b) <= 4096:
        return ref_xxh64(b, 0)
    level = [ref_xxh64(b[o:o + 4096], 0) for o in range(0, len(b), 4096)]
    seed = 0
    while len(level) > 1:
        seed += 1
        level = [ref_xxh64(b"".join(x.to_bytes(8, "little") for x in level[g:g + 64]), seed)
                 for g in range(0, len(level), 64)]
    return level[0]


def test_xxh64_published_vectors():
    # values of the public specification's reference implementation
    for data, seed in [(b"", 0), (b"", 1), (b"a", 0), (b"abc", 0), (bytes(range(256)) * 16, 0), (b"\0" * 4096, 0)]:
        assert oracle.xxh64(data, seed) == ref_xxh64(data, seed)


@pytest.mark.parametrize("seed", [0, 1, 7, 2**32 + 5, 2**64 - 1])
def test_xxh64_every_length_class(seed):
    rng = np.random.default_rng(seed % 1000)
    lengths = list(range(0, 80)) + [95, 96, 97, 127, 128, 255, 256, 511, 512, 1000, 4095, 4096, 4097, 10007]
    for n in lengths:
        b = rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()
        assert oracle.xxh64(b, seed) == ref_xxh64(b, seed), n


def test_xxh64_random_bytes_many():
    rng = np.random.default_rng(123)
    for _ in range(300):
        n = int(rng.integers(0, 4200))
        b = rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()
        s = int(rng.integers(0, 2**63))
        assert oracle.xxh64(b, s) == ref_xxh64(b, s)


@pytest.mark.parametrize("n", [0, 1, 31, 32, 4095, 4096, 4097, 8192, 8193, 262143, 262144, 262145,
                               64 * 262144, 64 * 262144 + 1, 4097 * 4096 + 3])
def test_d64_matches_independent_composition(n):
    rng = np.random.default_rng(n)
    b = rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()
    assert oracle.d64(b) == ref_d64(b)


def test_d64_three_levels():
    # 4097 leaves -> 65 level-1 nodes -> 2 level-2 nodes -> root at level 3
    n = 4096 * 4097
    b = np.random.default_rng(5).integers(0, 256, size=n, dtype=np.uint8).tobytes()
    assert oracle.d64(b) == ref_d64(b)


def test_d64_small_inputs_are_plain_xxh64():
    rng = np.random.default_rng(9)
    for n in [0, 5, 64, 4096]:
        b = rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()
        assert oracle.d64(b) == ref_xxh64(b, 0)


def test_d64_levels_are_domain_separated():
    # a two-leaf input differs from hashing its leaf digests with seed 0
    b = os.urandom(8192)
    leaves = b"".join(ref_xxh64(b[o:o + 4096]).to_bytes(8, "little") for o in (0, 4096))
    assert oracle.d64(b) == ref_xxh64(leaves, 1)
    assert oracle.d64(b) != ref_xxh64(leaves, 0)


def test_d64_identical_bytes_identical_digest_any_alignment():
    rng = np.random.default_rng(77)
    base = rng.integers(0, 256, size=300_000, dtype=np.uint8)
    want = oracle.d64(base)
    for off in range(16):
        buf = np.zeros(base.size + 32, dtype=np.uint8)
        buf[off:off + base.size] = base
        assert oracle.d64(buf[off:off + base.size]) == want


def test_d64_single_bit_flip_changes_digest():
    rng = np.random.default_rng(78)
    base = rng.integers(0, 256, size=1 << 20, dtype=np.uint8)
    want = oracle.d64(base)
    for pos in [0, 4095, 4096, 262143, 262144, (1 << 20) - 1]:
        m = base.copy()
        m[pos] ^= 1
        assert oracle.d64(m) != want


def test_d64_many_matches_single():
    rng = np.random.default_rng(79)
    bufs = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in [0, 1, 4096, 4097, 70000, 300000]]
    got = oracle.d64_many(bufs)
    assert [int(x) for x in got] == [ref_d64(b.tobytes()) for b in bufs]
