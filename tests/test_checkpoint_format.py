"""The particle checkpoint file format read by the library's host-only header
call (etpic_checkpoint_info), against files written here from the layout the
header documents (136-byte header, arrays in order, FNV-1a 64 checksums):
a valid file is accepted and reported as written; a foreign, truncated,
padded or corrupted one is EIO.  No GPU."""
import struct

import numpy as np
import pytest

from paper_2208_12795_amd import etpic as E

FNV_OFFSET, FNV_PRIME = 1469598103934665603, 1099511628211


def fnv1a(data, h=FNV_OFFSET):
    for b in bytes(data):
        h = ((h ^ b) * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def arrays(n, precision, has_id, seed=0):
    rng = np.random.default_rng(seed)
    tet = rng.integers(0, 1000, n).astype(np.int32)
    if precision == 2:
        lam = [rng.integers(0, 1 << 30, n).astype(np.uint32) for _ in range(3)]
    else:
        lam = [rng.random(n) for _ in range(3)]
    vdt = np.float64 if precision == 0 else np.float32
    vel = [rng.standard_normal(n).astype(vdt) for _ in range(3)]
    ids = np.arange(n, dtype=np.int64) if has_id else np.zeros(0, np.int64)
    return [tet, *lam, *vel, ids]


def header(n, precision, step, has_id, sums, n_tet=1000, n_vert=300, mesh_hash=12345, fix_sum=True):
    body = struct.pack("<8sIIqqqqQII8Q", b"ETPICCKP", 1, precision, n, step, n_tet, n_vert, mesh_hash,
                       1 if has_id else 0, 0, *sums)
    hs = fnv1a(body + b"\0" * 8) if fix_sum else 0
    return body + struct.pack("<Q", hs)


def write(path, n=37, precision=0, step=123, has_id=True, seed=0):
    arrs = arrays(n, precision, has_id, seed)
    sums = [fnv1a(a.tobytes()) for a in arrs]
    with open(path, "wb") as f:
        f.write(header(n, precision, step, has_id, sums))
        for a in arrs:
            f.write(a.tobytes())
    return arrs


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("has_id", [True, False])
def test_valid_file_is_read(tmp_path, precision, has_id):
    p = tmp_path / "ck.bin"
    write(p, n=53, precision=precision, step=-7 if has_id else 2 ** 40, has_id=has_id)
    info = E.checkpoint_info(str(p))
    assert info == {"n": 53, "precision": precision, "step": -7 if has_id else 2 ** 40, "has_id": has_id}
    assert len(header(0, 0, 0, False, [0] * 8)) == 136


def test_empty_particle_set(tmp_path):
    p = tmp_path / "empty.bin"
    write(p, n=0)
    assert E.checkpoint_info(str(p))["n"] == 0


def expect_eio(path):
    with pytest.raises(E.EtpicError) as ei:
        E.checkpoint_info(str(path))
    assert ei.value.code == E.EIO
    return str(ei.value)


def test_bad_files_are_rejected(tmp_path):
    good = tmp_path / "good.bin"
    write(good)
    raw = good.read_bytes()
    expect_eio(tmp_path / "missing.bin")
    cases = {
        "truncated_header": raw[:100],
        "truncated_arrays": raw[:-1],
        "padded": raw + b"\0",
        "foreign_magic": b"NOTACKPT" + raw[8:],
        "flipped_header_byte": raw[:20] + bytes([raw[20] ^ 1]) + raw[21:],
    }
    for name, data in cases.items():
        q = tmp_path / (name + ".bin")
        q.write_bytes(data)
        msg = expect_eio(q)
        assert msg, name
    # a header whose checksum is right but whose version is unknown
    body = bytearray(raw[:136])
    struct.pack_into("<I", body, 8, 2)
    struct.pack_into("<Q", body, 128, fnv1a(bytes(body[:128]) + b"\0" * 8))
    q = tmp_path / "version.bin"
    q.write_bytes(bytes(body) + raw[136:])
    assert "version" in expect_eio(q)
    # an implausible particle count with a consistent checksum
    body = bytearray(raw[:136])
    struct.pack_into("<q", body, 16, 1 << 62)
    struct.pack_into("<Q", body, 128, fnv1a(bytes(body[:128]) + b"\0" * 8))
    q = tmp_path / "count.bin"
    q.write_bytes(bytes(body) + raw[136:])
    assert "out of range" in expect_eio(q)
