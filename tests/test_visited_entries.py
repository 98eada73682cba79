"""The visited cache's entries name ids exactly (no false positives) for the
bucket counts the search uses, checked exhaustively over every hash value.

With n_b buckets, 2^vb <= n_b < 2^(vb+1), and hashes h < 2^B, the bucket is
floor(h * n_b / 2^B) and the entry is h's place in its bucket scaled to
16 bits, 1 + floor((h * n_b mod 2^B) * 65535 / 2^B).  The device forms both
from 32-bit products of hs = h * 2^(32 - B): the high word of hs * n_b, and
1 + the high word of (hs * n_b mod 2^32) * 65535.  Distinct hashes must get
distinct (bucket, entry) pairs, with no entry 0 (an empty place).  The
device scales lo = (hs * n_b mod 2^32) without a multiply: with q = lo >> 16
and m = lo & 0xFFFF, 1 + floor(lo * 65535 / 2^32) = q + [m > q or lo = 0].
"""
import numpy as np
import pytest


def pairs(B, nb):
    h = np.arange(1 << B, dtype=np.uint64)
    hs = (h << np.uint64(32 - B)) & np.uint64(0xFFFFFFFF)
    p = hs * np.uint64(nb)
    bucket = p >> np.uint64(32)
    lo = p & np.uint64(0xFFFFFFFF)
    q, m = lo >> np.uint64(16), lo & np.uint64(0xFFFF)
    e = q + ((m > q) | (lo == 0)).astype(np.uint64)
    # the same values from the definition
    r = (h * np.uint64(nb)) & np.uint64((1 << B) - 1)
    assert np.array_equal(bucket, (h * np.uint64(nb)) >> np.uint64(B))
    assert np.array_equal(e, np.uint64(1) + ((r * np.uint64(65535)) >> np.uint64(B)))
    return bucket, e


@pytest.mark.parametrize("B,nb", [(20, 17), (20, 31), (20, 23), (19, 16), (19, 31),
                                  (17, 8192), (24, 257), (24, 374), (24, 511), (24, 654)])
def test_entries_name_hashes_exactly(B, nb):
    # B - vb = 16 with n_b > 2^vb (20/17 .. 24/511), and B - vb <= 15
    bucket, e = pairs(B, nb)
    assert int(bucket.max()) == nb - 1
    assert int(e.min()) >= 1 and int(e.max()) <= 0xFFFF
    key = (bucket << np.uint64(16)) | e
    assert np.unique(key).size == key.size


def test_sixteen_bits_need_more_than_2_pow_vb_buckets():
    # at n_b = 2^vb with B - vb = 16 a bucket spans 2^16 hashes, and two of
    # them share an entry; one more bucket is enough (the launch adds at
    # least one, else it takes 2^(vb+1) buckets)
    bucket, e = pairs(20, 16)
    key = (bucket << np.uint64(16)) | e
    assert np.unique(key).size < key.size


def test_scaling_without_a_multiply():
    # q + [m > q or lo = 0] equals 1 + floor(lo * 65535 / 2^32) on random
    # words and on every pair with m = q or m = q + 1 (where it turns)
    rng = np.random.default_rng(1)
    a = np.arange(65536, dtype=np.uint64)
    lo = np.concatenate([rng.integers(0, 1 << 32, 2_000_000, dtype=np.uint64),
                         (a << np.uint64(16)) + a,
                         (a << np.uint64(16)) + (a + np.uint64(1)) % np.uint64(65536),
                         np.array([0, 1, 0xFFFF, 0x10000, 0xFFFFFFFF], np.uint64)])
    q, m = lo >> np.uint64(16), lo & np.uint64(0xFFFF)
    alt = q + ((m > q) | (lo == 0)).astype(np.uint64)
    assert np.array_equal(alt, np.uint64(1) + ((lo * np.uint64(65535)) >> np.uint64(32)))
