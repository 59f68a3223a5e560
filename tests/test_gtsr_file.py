"""``.gtsr`` files (``gtsr_file_*``), on the CPU: meshes of both formats come
back byte for byte and decode (by the oracle's walk) to the same triples;
a reader rejects every kind of damage -- a flipped byte anywhere, a short or
long file, a wrong magic or version, a record whose array lies outside the
file, and a stream that breaks its format's invariants even when the file's
hash is recomputed to match -- with ECORRUPT, and a missing file with EIO."""
import os
import struct
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import meshgen  # noqa: E402
import oracle as O  # noqa: E402
import paper_2404_06359_amd as P  # noqa: E402

HEADER, RECORD = 64, 128


def _meshes():
    out = []
    for m, caps in ((meshgen.workload1(), (64, 126)), (meshgen.fan(300), (64, 126)),
                    (meshgen.delaunay(2000, meshgen.rng_for(4, 9)), (128, 256)), (meshgen.disjoint(20), (32, 64))):
        e = P.encode(m.tri, m.nverts, *caps)
        out.append(e)
    out.append(P.gts_from_reuse(out[0]))
    out.append(P.gts_from_reuse(out[2]))
    return out


def _fnv1a(b: bytes) -> int:
    h = 0xcbf29ce484222325
    for x in b:
        h = ((h ^ x) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def _rehash(data: bytearray):
    struct.pack_into("<Q", data, 40, _fnv1a(bytes(data[HEADER:])))


def _expect(path, code):
    with pytest.raises(P.GtsrError) as e:
        P.load(path)
    assert e.value.code == code, str(e.value)


def test_round_trip_both_formats(tmp_path):
    encs = _meshes()
    path = str(tmp_path / "pool.gtsr")
    P.save(path, encs)
    back = P.load(path)
    assert len(back) == len(encs)
    for a, b in zip(encs, back):
        assert a.format == b.format and a.strip_triangles == b.strip_triangles
        assert a.stats["input_triangles"] == b.stats["input_triangles"]
        assert a.stats["restarts"] == b.stats["restarts"]
        for f in ("meshlets", "bits", "reuse", "verts", "vert_off", "kept_off", "tri_ids"):
            np.testing.assert_array_equal(getattr(a, f), getattr(b, f), err_msg=f)
        if b.format == P.FORMAT_REUSE:
            want = O.decode_arrays(a.desc_bytes, a.bits, a.reuse, a.strip_triangles)
            got = O.decode_arrays(b.desc_bytes, b.bits, b.reuse, b.strip_triangles)
        else:
            want = O.decode_gts(O.GtsStream(a.desc_bytes, a.bits, a.reuse, a.strip_triangles))
            got = O.decode_gts(O.GtsStream(b.desc_bytes, b.bits, b.reuse, b.strip_triangles))
        np.testing.assert_array_equal(got, want)
    # no leftover temporary file; an empty pool is a valid file too
    assert sorted(os.listdir(tmp_path)) == ["pool.gtsr"]
    P.save(str(tmp_path / "empty.gtsr"), [])
    assert P.load(str(tmp_path / "empty.gtsr")) == []


def test_layout_of_the_header_and_records(tmp_path):
    encs = _meshes()[:2]
    path = str(tmp_path / "a.gtsr")
    P.save(path, encs)
    data = open(path, "rb").read()
    magic, version, count, table, dat, total, h = struct.unpack_from("<8sIIQQQQ", data, 0)
    assert magic == b"GTSRFILE" and version == 1 and count == 2 and table == HEADER and total == len(data)
    assert dat % 16 == 0 and dat >= HEADER + RECORD * count
    assert h == _fnv1a(data[HEADER:])
    for i, e in enumerate(encs):
        fmt, M = struct.unpack_from("<II", data, HEADER + RECORD * i)
        assert (fmt, M) == (e.format, e.meshlet_count)
        offs = struct.unpack_from("<7Q", data, HEADER + RECORD * i + 64)
        assert all(o % 16 == 0 and dat <= o <= total for o in offs)
        assert data[offs[0]:offs[0] + e.meshlets.nbytes] == e.meshlets.tobytes()
        assert data[offs[2]:offs[2] + e.reuse.nbytes] == e.reuse.tobytes()


def test_damage_is_rejected(tmp_path):
    encs = _meshes()
    path = str(tmp_path / "a.gtsr")
    P.save(path, encs)
    good = bytearray(open(path, "rb").read())
    bad = str(tmp_path / "bad.gtsr")

    def write(b):
        with open(bad, "wb") as f:
            f.write(bytes(b))

    rng = np.random.default_rng(7)
    for pos in list(rng.integers(HEADER, len(good), 12)) + [HEADER, len(good) - 1]:
        b = bytearray(good)
        b[int(pos)] ^= 0x10
        write(b)
        _expect(bad, P.ECORRUPT)
    write(good[:-16])
    _expect(bad, P.ECORRUPT)
    write(good + b"\0" * 16)
    _expect(bad, P.ECORRUPT)
    write(good[:40])
    _expect(bad, P.ECORRUPT)
    b = bytearray(good)
    b[0:8] = b"GTSRFILF"
    write(b)
    _expect(bad, P.ECORRUPT)
    b = bytearray(good)
    struct.pack_into("<I", b, 8, 2)
    write(b)
    _expect(bad, P.ECORRUPT)
    # an array offset past the end, with the hash made to match
    b = bytearray(good)
    struct.pack_into("<Q", b, HEADER + 64 + 8, len(good) + 16)
    _rehash(b)
    write(b)
    _expect(bad, P.ECORRUPT)
    # a meshlet count that no longer matches the arrays, hash made to match
    b = bytearray(good)
    struct.pack_into("<I", b, HEADER + 4, encs[0].meshlet_count + 1)
    _rehash(b)
    write(b)
    _expect(bad, P.ECORRUPT)
    write(b"")
    _expect(bad, P.ECORRUPT)
    _expect(str(tmp_path / "missing.gtsr"), P.EIO)


@pytest.mark.parametrize("which", ["reuse", "gts"])
def test_stream_invariants_are_checked_behind_a_valid_hash(tmp_path, which):
    """A file whose hash matches but whose stream breaks the format's rules:
    a reuse byte (GTS-Reuse) or an index byte (plain GTS) naming a vertex
    that has not appeared yet."""
    encs = _meshes()
    e = encs[0] if which == "reuse" else encs[4]
    path = str(tmp_path / "a.gtsr")
    P.save(path, [e])
    b = bytearray(open(path, "rb").read())
    reuse_off = struct.unpack_from("<7Q", b, HEADER + 64)[2]
    b[reuse_off] = 0xFF   # vertex 255: never introduced in the first meshlet
    _rehash(b)
    with open(path, "wb") as f:
        f.write(bytes(b))
    _expect(path, P.ECORRUPT)


def test_write_errors(tmp_path):
    e = _meshes()[0]
    with pytest.raises(P.GtsrError) as x:
        P.save(str(tmp_path / "no_such_dir" / "a.gtsr"), [e])
    assert x.value.code == P.EIO
    L = P.lib()
    m = P.FileMesh()
    m.format = 7
    assert L.gtsr_file_write(os.fsencode(str(tmp_path / "b.gtsr")), P.C.byref(m), 1) == P.EINVAL
    assert L.gtsr_file_write(None, None, 0) == P.EINVAL
    assert L.gtsr_file_open(None, None) == P.EINVAL


def test_save_refuses_incomplete_meshes(tmp_path):
    """An Encoded without its vertex lists (as the serving benchmark keeps
    them: streams and counts only) is refused before the writer reads its
    offsets."""
    e = _meshes()[0]
    slim = P.Encoded(e.meshlets, e.bits, e.reuse, np.zeros(0, np.uint32), np.zeros(1, np.uint64), e.stats)
    with pytest.raises(ValueError):
        P.save(str(tmp_path / "slim.gtsr"), [slim])
    short = P.Encoded(e.meshlets, e.bits, e.reuse, e.verts, e.vert_off, e.stats, e.kept_off, e.tri_ids[:-1])
    with pytest.raises(ValueError):
        P.save(str(tmp_path / "short.gtsr"), [short])
    assert not os.path.exists(tmp_path / "slim.gtsr") and not os.path.exists(tmp_path / "short.gtsr")
