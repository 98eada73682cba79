"""The index file (aqr_index_save / aqr_index_file_info / aqr_index_load):
round trip, and AQR_ERR_CORRUPT on truncation, bit flips, trailing bytes and
on files whose checksums are valid but whose contents break the index's
invariants.  The checksum is CRC-32C; a table-driven CRC-32C written here
from its definition (reflected polynomial 0x82F63B78) pins the library's
instruction-based one, and forges valid checksums for the structural cases.
"""
import struct

import numpy as np
import pytest

from paper_2602_21600_amd import aqr
from paper_2602_21600_amd import workloads as W

CORRUPT = 5
HEADER = 512
BLOCK = 64 << 20


def _crc32c_table():
    tab = []
    for i in range(256):
        c = i
        for _ in range(8):
            c = (c >> 1) ^ 0x82F63B78 if c & 1 else c >> 1
        tab.append(c)
    return tab


_TAB = _crc32c_table()


def crc32c(data: bytes) -> int:
    c = 0xFFFFFFFF
    for b in data:
        c = (c >> 8) ^ _TAB[(c ^ b) & 0xFF]
    return c ^ 0xFFFFFFFF


def test_crc32c_check_value():
    # the standard check value of CRC-32C over the ASCII digits 1..9
    assert crc32c(b"123456789") == 0xE3069283


@pytest.fixture(scope="module")
def built():
    X, _ = W.tiny(700, 40, seed=17, clusters=5, nq=1)
    qz, codes = aqr.aqr_quantize(X, aqr.default_qparams(M0=6, efc0=40))
    g = aqr.aqr_build(codes, X.shape[1], qz, threads=1, seed=5)
    return X, qz, codes, g


def _save(tmp_path, built, name="ix.aqr"):
    X, qz, codes, g = built
    p = tmp_path / name
    aqr.aqr_index_save(str(p), qz, g, codes, X)
    return p


def test_round_trip(tmp_path, built):
    X, qz, codes, g = built
    p = _save(tmp_path, built)
    info = aqr.aqr_index_file_info(str(p))
    assert info["n"] == 700 and info["d"] == 40 and info["d_pad"] == 48
    assert info["file_bytes"] == p.stat().st_size
    q2, g2, c2, X2 = aqr.aqr_index_load(str(p))
    np.testing.assert_array_equal(c2, codes)
    np.testing.assert_array_equal(X2, X)
    a, b = aqr.aqr_quantizer_info(qz), aqr.aqr_quantizer_info(q2)
    for f in ("d", "d_pad", "M", "efc", "delta", "p_lo", "p_hi", "s_dist", "eta", "w_mean"):
        assert a[f] == b[f], f
    for f in ("min", "max", "scale"):
        np.testing.assert_array_equal(a[f], b[f])
    ga, gb = aqr.aqr_graph_export(g), aqr.aqr_graph_export(g2)
    for f in ("level", "adj0", "upper_off", "upper_adj"):
        np.testing.assert_array_equal(ga[f], gb[f])
    assert ga["ep"] == gb["ep"] and ga["M"] == gb["M"]
    assert aqr.aqr_graph_info(g2)["efc"] == aqr.aqr_graph_info(g)["efc"]


def test_checksums_follow_crc32c(tmp_path, built):
    raw = _save(tmp_path, built).read_bytes()
    h = bytearray(raw[:HEADER])
    stored = struct.unpack_from("<I", h, 280)[0]
    h[280:284] = b"\0\0\0\0"
    assert crc32c(bytes(h)) == stored
    payload = struct.unpack_from("<Q", raw, 120)[0]
    nblocks = struct.unpack_from("<Q", raw, 128)[0]
    assert nblocks == (payload + BLOCK - 1) // BLOCK
    table = raw[HEADER + payload:HEADER + payload + 4 * nblocks]
    for b in range(nblocks):
        blk = raw[HEADER + b * BLOCK:HEADER + min(payload, (b + 1) * BLOCK)]
        assert struct.unpack_from("<I", table, 4 * b)[0] == crc32c(blk)
    assert struct.unpack_from("<I", raw, HEADER + payload + 4 * nblocks)[0] == crc32c(table)


def _expect_corrupt(path):
    with pytest.raises(aqr.AqrError) as e:
        aqr.aqr_index_load(str(path))
    assert e.value.status == CORRUPT, str(e.value)


def test_truncation_and_trailing_bytes(tmp_path, built):
    raw = _save(tmp_path, built).read_bytes()
    for cut in (1, 9, 100, len(raw) - HEADER, len(raw) - 10):
        p = tmp_path / f"cut{cut}.aqr"
        p.write_bytes(raw[:len(raw) - cut])
        _expect_corrupt(p)
    p = tmp_path / "long.aqr"
    p.write_bytes(raw + b"\0")
    _expect_corrupt(p)


def test_bit_flips(tmp_path, built):
    raw = _save(tmp_path, built).read_bytes()
    rng = np.random.default_rng(3)
    # header, every section of the payload, the checksum table, the end marker
    spots = [0, 20, 300, HEADER + 5, HEADER + 3000] + list(
        rng.integers(HEADER, len(raw), 6)) + [len(raw) - 14, len(raw) - 3]
    for i, pos in enumerate(spots):
        b = bytearray(raw)
        b[int(pos)] ^= 1 << (i % 8)
        p = tmp_path / f"flip{i}.aqr"
        p.write_bytes(bytes(b))
        _expect_corrupt(p)


def _forge(raw, edit):
    """Apply edit(payload bytearray, header fields) and recompute every CRC."""
    payload = struct.unpack_from("<Q", raw, 120)[0]
    nblocks = struct.unpack_from("<Q", raw, 128)[0]
    offs = struct.unpack_from("<9Q", raw, 136)
    body = bytearray(raw[HEADER:HEADER + payload])
    edit(body, offs)
    table = b"".join(struct.pack("<I", crc32c(bytes(body[b * BLOCK:(b + 1) * BLOCK])))
                     for b in range(nblocks))
    return raw[:HEADER] + bytes(body) + table + struct.pack("<I", crc32c(table)) + raw[-8:]


def test_valid_checksums_but_broken_contents(tmp_path, built):
    X, qz, codes, g = built
    raw = _save(tmp_path, built).read_bytes()
    p = tmp_path / "same.aqr"
    p.write_bytes(_forge(raw, lambda body, offs: None))
    aqr.aqr_index_load(str(p))  # forging without an edit keeps a valid file

    def pad_byte(body, offs):  # a non-zero padding byte in a code row
        body[offs[3] + 48 * 10 + 45] = 7

    def bad_neighbour(body, offs):  # a layer-0 neighbour id >= n
        struct.pack_into("<I", body, offs[6] + 4 * 5, 700)

    def bad_level(body, offs):  # a level that disagrees with the row offsets
        lv = struct.unpack_from("<i", body, offs[5] + 4 * 3)[0]
        struct.pack_into("<i", body, offs[5] + 4 * 3, lv + 1)

    def bad_scale(body, offs):  # a zero scale
        struct.pack_into("<f", body, offs[2] + 4 * 2, 0.0)

    for i, edit in enumerate((pad_byte, bad_neighbour, bad_level, bad_scale)):
        p = tmp_path / f"forged{i}.aqr"
        p.write_bytes(_forge(raw, edit))
        _expect_corrupt(p)


def test_not_an_index_and_missing_file(tmp_path):
    p = tmp_path / "junk.aqr"
    p.write_bytes(b"x" * 2000)
    _expect_corrupt(p)
    with pytest.raises(aqr.AqrError):
        aqr.aqr_index_load(str(tmp_path / "absent.aqr"))
