"""The library's files on the CPU: its CRC-32 equals zlib's (an independent
implementation of the same published checksum); a pruner checkpoint written
here by Python's struct/zlib is accepted by the library's host-side check
and every planted corruption (payload byte, header byte, truncation, wrong
magic, a size that does not match the dimensions) is rejected; a tuning
cache is counted and its damage detected.  No device is used."""

import os
import struct
import zlib

import numpy as np
import pytest


@pytest.fixture(scope="module")
def mhr():
    import paper_2406_07727_amd as m
    return m


def test_crc32_equals_zlib(mhr):
    rng = np.random.Generator(np.random.PCG64(1))
    for n in (0, 1, 7, 64, 1000, 65537):
        data = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        assert mhr.crc32(data) == zlib.crc32(data)
        # continuation from a running value
        assert mhr.crc32(data[n // 2:], mhr.crc32(data[:n // 2])) == zlib.crc32(data)
    assert mhr.crc32(b"123456789") == 0xCBF43926   # the published check value of CRC-32


def _checkpoint(dim, hidden, step, seed=3):
    """A pruner checkpoint in the documented layout, built with struct and
    zlib alone."""
    n = 4 * dim * hidden + hidden + hidden * hidden + hidden + hidden + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    payload = rng.standard_normal(3 * n).astype(np.float32).tobytes()
    head = b"MHRPRUN1" + struct.pack("<IIIIQI", 1, dim, hidden, step, n, zlib.crc32(payload))
    head += struct.pack("<I", zlib.crc32(head))
    return head + payload


def test_pruner_checkpoint_accepted_and_corruption_rejected(mhr, tmp_path):
    path = str(tmp_path / "p.ckpt")
    good = _checkpoint(16, 32, 123)
    with open(path, "wb") as f:
        f.write(good)
    assert mhr.pruner_file_info(path) == (16, 32, 123)
    cases = {
        "payload byte": good[:100] + bytes([good[100] ^ 1]) + good[101:],
        "header byte": good[:13] + bytes([good[13] ^ 4]) + good[14:],
        "truncated": good[:-4],
        "magic": b"MHRPRUNX" + good[8:],
        "too short": good[:20],
    }
    for name, data in cases.items():
        with open(path, "wb") as f:
            f.write(data)
        with pytest.raises(mhr.MhrError) as e:
            mhr.pruner_file_info(path)
        assert e.value.status == mhr.ERR_CORRUPT, name
    # sizes that disagree with the dimensions, with valid checksums
    bad = _checkpoint(16, 32, 1)
    n_wrong = struct.unpack("<Q", bad[24:32])[0] + 1
    head = bad[:24] + struct.pack("<Q", n_wrong) + bad[32:36]
    head += struct.pack("<I", zlib.crc32(head))
    with open(path, "wb") as f:
        f.write(head + bad[40:])
    with pytest.raises(mhr.MhrError) as e:
        mhr.pruner_file_info(path)
    assert e.value.status == mhr.ERR_CORRUPT
    # a later format version is refused as unsupported, not as damage
    head = bad[:8] + struct.pack("<I", 2) + bad[12:36]
    head += struct.pack("<I", zlib.crc32(head))
    with open(path, "wb") as f:
        f.write(head + bad[40:])
    with pytest.raises(mhr.MhrError) as e:
        mhr.pruner_file_info(path)
    assert e.value.status == 3
    with pytest.raises(mhr.MhrError) as e:
        mhr.pruner_file_info(str(tmp_path / "missing"))
    assert e.value.status == mhr.ERR_IO


def _record(arch, n, R, pairs, dim, dtype, scorer, nq, kmax, te, hl, gb, ms):
    body = arch.encode().ljust(32, b"\0") + struct.pack("<IIQIIIIIIIIfII", n, R, pairs, dim, dtype, scorer, nq, kmax,
                                                         te, hl, gb, ms, 0, 0)
    assert len(body) == 92
    return body + struct.pack("<I", zlib.crc32(body))


def test_tuning_cache_records(mhr, tmp_path):
    path = str(tmp_path / "tune.bin")
    recs = [_record("gfx950", 1000, 16, 5000, 128, 0, 0, 1024, 32, 32768, 12, 0, 1.25),
            _record("gfx950", 1000, 16, 5000, 128, 0, 1, 1024, 32, 65536, 11, 0, 3.5)]
    with open(path, "wb") as f:
        f.write(b"".join(recs))
    assert mhr.tuning_file_records(path) == 2
    data = bytearray(b"".join(recs))
    data[150] ^= 0x10
    with open(path, "wb") as f:
        f.write(bytes(data))
    with pytest.raises(mhr.MhrError) as e:
        mhr.tuning_file_records(path)
    assert e.value.status == mhr.ERR_CORRUPT
    with open(path, "wb") as f:
        f.write(b"".join(recs)[:-5])
    with pytest.raises(mhr.MhrError) as e:
        mhr.tuning_file_records(path)
    assert e.value.status == mhr.ERR_CORRUPT
