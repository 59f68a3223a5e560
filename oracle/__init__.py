"""Oracle for the GTS-Reuse meshlet connectivity codec -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
``oracle.c``: sequential encoder, strip-walk decoders for GTS-Reuse and plain
GTS, stream checker, degenerate compaction) and
re-exports the pure-Python closed-form decoder from ``defn``.

Nothing here imports or loads the product package or its library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIBRARY names another build of oracle.c (the sanitized one, see
# build_sanitized); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
SANITIZED_PATH = os.path.join(os.path.dirname(HERE), "_build", "sanitize", "liboracle.so")

OK, EINVAL, ENOMEM, EDEGENERATE, ELIMIT, ECORRUPT = 0, -1, -2, -3, -4, -5

_lib = None


def build() -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, plain -O2)."""
    src = os.path.join(HERE, "oracle.c")
    tmp = f"{LIB_PATH}.{os.getpid()}.tmp"   # private per process: test workers may build at once
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                    "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_sanitized() -> str:
    """``oracle.c`` with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc), into ``_build/sanitize/liboracle.so``, for CPU test runs."""
    os.makedirs(os.path.dirname(SANITIZED_PATH), exist_ok=True)
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", f"{SANITIZED_PATH}.{os.getpid()}.tmp", os.path.join(HERE, "oracle.c"), "-lm"], check=True)
    os.replace(f"{SANITIZED_PATH}.{os.getpid()}.tmp", SANITIZED_PATH)
    return SANITIZED_PATH


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = C.CDLL(LIB_PATH)
    u8p, u32p, u64p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    vp = C.c_void_p
    L.oracle_encode.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(vp)]
    L.oracle_encode.restype = C.c_int
    L.oracle_enc_free.argtypes = [vp]
    L.oracle_enc_free.restype = None
    for name, rt in [("oracle_enc_meshlets", C.c_uint32), ("oracle_enc_desc", u8p),
                     ("oracle_enc_bits", u8p), ("oracle_enc_bits_bytes", C.c_uint64),
                     ("oracle_enc_reuse", u8p), ("oracle_enc_reuse_bytes", C.c_uint64),
                     ("oracle_enc_verts", u32p), ("oracle_enc_vert_off", u64p)]:
        f = getattr(L, name)
        f.argtypes = [vp]
        f.restype = rt
    L.oracle_enc_stat.argtypes = [vp, C.c_int]
    L.oracle_enc_stat.restype = C.c_uint64
    L.oracle_decode.argtypes = [vp, C.c_uint32, vp, C.c_uint64, vp, C.c_uint64, vp, C.c_uint64]
    L.oracle_decode.restype = C.c_int
    L.oracle_decode_range.argtypes = [vp, C.c_uint32, C.c_uint32, vp, C.c_uint64, vp, C.c_uint64,
                                      vp, C.c_uint64]
    L.oracle_decode_range.restype = C.c_int
    L.oracle_decode_meshlet.argtypes = [vp, vp, C.c_uint64, vp, C.c_uint64, vp, C.c_uint64]
    L.oracle_decode_meshlet.restype = C.c_int
    L.oracle_check_stream.argtypes = [vp, C.c_uint32, vp, C.c_uint64, vp, C.c_uint64, C.c_uint64]
    L.oracle_check_stream.restype = C.c_int
    L.oracle_gts_decode.argtypes = [vp, C.c_uint32, vp, C.c_uint64, vp, C.c_uint64, vp, C.c_uint64]
    L.oracle_gts_decode.restype = C.c_int
    L.oracle_gts_from_reuse.argtypes = [vp, C.c_uint32, vp, C.c_uint64, vp, C.c_uint64, vp, vp, C.c_uint64,
                                        vp, C.c_uint64]
    L.oracle_gts_from_reuse.restype = C.c_int
    L.oracle_compact.argtypes = [vp, C.c_uint64, vp, C.c_uint64, u64p, vp, C.c_uint32, vp]
    L.oracle_compact.restype = C.c_int
    L.oracle_min_strips.argtypes = [vp, C.c_uint32, u32p]
    L.oracle_min_strips.restype = C.c_int
    L.oracle_cones.argtypes = [vp, C.c_uint32, vp, vp, vp, vp, C.c_uint32, vp]
    L.oracle_cones.restype = C.c_int
    L.oracle_cull.argtypes = [vp, C.c_uint32, C.c_float, C.c_float, C.c_float, vp]
    L.oracle_cull.restype = C.c_int
    L.oracle_quantize.argtypes = [vp, C.c_uint32, C.c_uint32, vp, vp, C.c_uint32, C.c_uint32, vp, vp, vp, vp]
    L.oracle_quantize.restype = C.c_int
    L.oracle_dequantize.argtypes = [vp, vp, vp, C.c_uint32, C.c_uint32, vp, vp, vp]
    L.oracle_dequantize.restype = C.c_int
    _lib = L
    return L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


STAT_NAMES = ("input_triangles", "strip_triangles", "restarts", "reuse_count",
              "split_meshlets", "payload_bits", "stored_bytes")


@dataclass
class Stream:
    """One encoded mesh as numpy arrays (host memory)."""

    desc: np.ndarray     # uint8[16*M]
    bits: np.ndarray     # uint8[16*chunks]
    reuse: np.ndarray    # uint8[n]
    verts: np.ndarray    # uint32[sum V]   local -> global vertex ids
    vert_off: np.ndarray  # uint64[M+1]
    stats: dict

    @property
    def meshlets(self) -> int:
        return self.desc.size // 16

    @property
    def strip_triangles(self) -> int:
        return int(self.stats["strip_triangles"])

    def fields(self):
        """Descriptor fields as arrays: chunk_off, reuse_off, out_off, T_s, V."""
        d = self.desc.reshape(-1, 16)
        u32 = d[:, :12].copy().view("<u4").reshape(-1, 3)
        u16 = d[:, 12:16].copy().view("<u2").reshape(-1, 2)
        return (u32[:, 0].astype(np.int64), u32[:, 1].astype(np.int64), u32[:, 2].astype(np.int64),
                u16[:, 0].astype(np.int64), u16[:, 1].astype(np.int64))


def encode(tri: np.ndarray, nverts: int, max_vertices: int = 64, max_triangles: int = 126) -> Stream:
    """Encode a CCW triangle list with the oracle encoder."""
    L = lib()
    tri = np.ascontiguousarray(tri, dtype=np.uint32).reshape(-1, 3)
    h = C.c_void_p()
    rc = L.oracle_encode(_ptr(tri), tri.shape[0], nverts, max_vertices, max_triangles, C.byref(h))
    if rc != OK:
        raise OracleError(rc)
    try:
        M = L.oracle_enc_meshlets(h)

        def arr(p, n, dt):
            if n == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(p, shape=(n,)).copy().view(dt) if dt != np.uint8 \
                else np.ctypeslib.as_array(p, shape=(n,)).copy()

        desc = arr(L.oracle_enc_desc(h), 16 * M, np.uint8)
        bits = arr(L.oracle_enc_bits(h), L.oracle_enc_bits_bytes(h), np.uint8)
        reuse = arr(L.oracle_enc_reuse(h), L.oracle_enc_reuse_bytes(h), np.uint8)
        vert_off = np.ctypeslib.as_array(L.oracle_enc_vert_off(h), shape=(M + 1,)).copy()
        nv = int(vert_off[-1])
        verts = (np.ctypeslib.as_array(L.oracle_enc_verts(h), shape=(nv,)).copy()
                 if nv else np.zeros(0, np.uint32))
        stats = {k: int(L.oracle_enc_stat(h, i)) for i, k in enumerate(STAT_NAMES)}
    finally:
        L.oracle_enc_free(h)
    return Stream(desc, bits, reuse, verts, vert_off, stats)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned {code}")
        self.code = code


def decode(s: Stream, out: np.ndarray | None = None) -> np.ndarray:
    """Decode every meshlet by the sequential strip walk: uint8[T_s_total, 3]."""
    return decode_arrays(s.desc, s.bits, s.reuse, s.strip_triangles, out)


def decode_arrays(desc, bits, reuse, strip_triangles, out=None, m0=0, m1=None):
    L = lib()
    desc = np.ascontiguousarray(desc, np.uint8)
    bits = np.ascontiguousarray(bits, np.uint8)
    reuse = np.ascontiguousarray(reuse, np.uint8)
    M = desc.size // 16
    if m1 is None:
        m1 = M
    if out is None:
        out = np.zeros((strip_triangles, 3), np.uint8)
    rc = L.oracle_decode_range(_ptr(desc), m0, m1, _ptr(bits), bits.size, _ptr(reuse), reuse.size,
                               _ptr(out), out.size)
    if rc != OK:
        raise OracleError(rc)
    return out


@dataclass
class GtsStream:
    """A plain GTS stream (host memory): descriptors, 8-byte L/R words, one
    index byte per strip triangle after the first."""

    desc: np.ndarray     # uint8[16*M]: word_off, index_off, out_off, T_s, V
    words: np.ndarray    # uint8[8*chunks]
    index: np.ndarray    # uint8[sum(T_s - 1)]
    strip_triangles: int


def gts_from_reuse(desc, bits, reuse, strip_triangles) -> GtsStream:
    """Re-encode a GTS-Reuse stream as plain GTS (same strips and flags)."""
    L = lib()
    desc = np.ascontiguousarray(desc, np.uint8)
    bits = np.ascontiguousarray(bits, np.uint8)
    reuse = np.ascontiguousarray(reuse, np.uint8)
    M = desc.size // 16
    T = desc.reshape(-1, 16)[:, 12:14].copy().view("<u2").reshape(-1).astype(np.int64)
    gdesc = np.zeros(16 * M, np.uint8)
    words = np.zeros(bits.size // 2, np.uint8)
    index = np.zeros(int((T - 1).sum()) if M else 0, np.uint8)
    rc = L.oracle_gts_from_reuse(_ptr(desc), M, _ptr(bits), bits.size, _ptr(reuse), reuse.size,
                                 _ptr(gdesc), _ptr(words), words.size, _ptr(index), index.size)
    if rc != OK:
        raise OracleError(rc)
    return GtsStream(gdesc, words, index, int(strip_triangles))


def decode_gts(g: GtsStream, out=None) -> np.ndarray:
    """Decode a plain GTS stream by the strip walk: uint8[T_s_total, 3]."""
    L = lib()
    if out is None:
        out = np.zeros((g.strip_triangles, 3), np.uint8)
    rc = L.oracle_gts_decode(_ptr(g.desc), g.desc.size // 16, _ptr(g.words), g.words.size, _ptr(g.index),
                             g.index.size, _ptr(out), out.size)
    if rc != OK:
        raise OracleError(rc)
    return out


def compact(decoded: np.ndarray, desc=None):
    """Drop triples with a repeated index (restart degenerates), keeping order.
    Returns the kept triples and, with ``desc``, each meshlet's offset among
    them (M + 1 entries)."""
    L = lib()
    tris = np.ascontiguousarray(decoded, np.uint8).reshape(-1, 3)
    out = np.zeros_like(tris)
    kept = C.c_uint64()
    offs = None
    if desc is not None:
        desc = np.ascontiguousarray(desc, np.uint8)
        offs = np.zeros(desc.size // 16 + 1, np.uint64)
    rc = L.oracle_compact(_ptr(tris), tris.shape[0], _ptr(out), tris.shape[0], C.byref(kept),
                          _ptr(desc) if desc is not None else None, desc.size // 16 if desc is not None else 0,
                          _ptr(offs) if offs is not None else None)
    if rc != OK:
        raise OracleError(rc)
    return out[:kept.value], offs


def cones(s: Stream, decoded: np.ndarray, positions: np.ndarray) -> np.ndarray:
    """Per-meshlet normal cones ``float32[M, 4]`` from decoded triples."""
    L = lib()
    pos = np.ascontiguousarray(positions, np.float32)
    dec = np.ascontiguousarray(decoded, np.uint8)
    out = np.zeros((s.meshlets, 4), np.float32)
    rc = L.oracle_cones(_ptr(s.desc), s.meshlets, _ptr(dec), _ptr(s.verts), _ptr(s.vert_off), _ptr(pos),
                        pos.shape[0], _ptr(out))
    if rc != OK:
        raise OracleError(rc)
    return out


def cull(cone_arr: np.ndarray, view) -> np.ndarray:
    """``uint8[M]``: 1 where the meshlet is culled for view direction ``view``."""
    L = lib()
    c = np.ascontiguousarray(cone_arr, np.float32)
    out = np.zeros(c.shape[0], np.uint8)
    L.oracle_cull(_ptr(c), c.shape[0], float(view[0]), float(view[1]), float(view[2]), _ptr(out))
    return out


def min_strips(tri: np.ndarray) -> int:
    """Fewest strips covering a tiny CCW triangle set (brute force, T <= 16)."""
    L = lib()
    tri = np.ascontiguousarray(tri, np.uint32).reshape(-1, 3)
    out = C.c_uint32()
    rc = L.oracle_min_strips(_ptr(tri), tri.shape[0], C.byref(out))
    if rc != OK:
        raise OracleError(rc)
    return int(out.value)


@dataclass
class Quantized:
    """Crack-free fixed-point attributes: per channel origin and spacing,
    per meshlet the lowest grid value, per meshlet-local vertex b-bit offsets."""

    origin: np.ndarray   # float32[n]
    delta: np.ndarray    # float32[n]
    L: np.ndarray        # int32[M, n]
    q: np.ndarray        # uint16[sum V, n]


def quantize(attrs: np.ndarray, verts: np.ndarray, vert_off: np.ndarray, b: int = 16) -> Quantized:
    L_ = lib()
    attrs = np.ascontiguousarray(attrs, np.float32)
    nv, n = attrs.shape
    verts = np.ascontiguousarray(verts, np.uint32)
    vert_off = np.ascontiguousarray(vert_off, np.uint64)
    M = vert_off.size - 1
    origin = np.zeros(n, np.float32)
    delta = np.zeros(n, np.float32)
    Lm = np.zeros((M, n), np.int32)
    q = np.zeros((int(vert_off[-1]), n), np.uint16)
    rc = L_.oracle_quantize(_ptr(attrs), nv, n, _ptr(verts), _ptr(vert_off), M, b, _ptr(origin), _ptr(delta),
                            _ptr(Lm), _ptr(q))
    if rc != OK:
        raise OracleError(rc)
    return Quantized(origin, delta, Lm, q)


def dequantize(qz: Quantized, vert_off: np.ndarray) -> np.ndarray:
    L_ = lib()
    vert_off = np.ascontiguousarray(vert_off, np.uint64)
    M, n = qz.L.shape
    out = np.zeros(qz.q.shape, np.float32)
    rc = L_.oracle_dequantize(_ptr(qz.L), _ptr(qz.q), _ptr(vert_off), M, n, _ptr(qz.origin), _ptr(qz.delta),
                              _ptr(out))
    if rc != OK:
        raise OracleError(rc)
    return out


def check_stream(desc, bits, reuse, strip_triangles) -> int:
    """0 when the stream is structurally valid, else a negative code."""
    L = lib()
    desc = np.ascontiguousarray(desc, np.uint8)
    bits = np.ascontiguousarray(bits, np.uint8)
    reuse = np.ascontiguousarray(reuse, np.uint8)
    return L.oracle_check_stream(_ptr(desc), desc.size // 16, _ptr(bits), bits.size,
                                 _ptr(reuse), reuse.size, strip_triangles)


def round_trip_triangles(s: Stream, decoded: np.ndarray) -> np.ndarray:
    """Map decoded local triples to global ids, drop triples with a repeated
    id, rotate each so its smallest id leads (winding kept), and sort."""
    _, _, out_off, T, V = s.fields()
    M = s.meshlets
    tri_meshlet = np.repeat(np.arange(M), T)
    base = s.vert_off[:-1].astype(np.int64)[tri_meshlet]
    g = s.verts.astype(np.int64)[base[:, None] + decoded.astype(np.int64)]
    return canonical(g)


def canonical(tri: np.ndarray) -> np.ndarray:
    tri = np.asarray(tri, np.int64).reshape(-1, 3)
    keep = (tri[:, 0] != tri[:, 1]) & (tri[:, 1] != tri[:, 2]) & (tri[:, 0] != tri[:, 2])
    tri = tri[keep]
    r = np.argmin(tri, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    rot = np.take_along_axis(tri, idx, axis=1)
    order = np.lexsort((rot[:, 2], rot[:, 1], rot[:, 0]))
    return rot[order]


from .defn import decode_closed_form, decode_meshlet_closed_form  # noqa: E402
