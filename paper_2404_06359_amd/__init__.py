"""MI355X-native GTS-Reuse meshlet connectivity codec.

Thin Python binding over ``libgtsr.so`` (C ABI declared in ``include/gtsr.h``):
argument marshalling only.  Encoding runs in the library's C++ encoder on the
host; every decode step runs in the library's HIP kernels.  PyTorch supplies
device memory and streams.  There is no CPU decode path: if the library is
missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# GTSR_LIBRARY names another build of the same library (the host-sanitized
# one for CPU test runs); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("GTSR_LIBRARY") or os.path.join(PKG, "libgtsr.so")

OK, EINVAL, ENOMEM, EDEGENERATE, ELIMIT, ECORRUPT, EHIP, ECANCELED, EBUSY, EIO = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
FORMAT_REUSE, FORMAT_GTS = 0, 1

EXPORTED = (
    "encode_meshlets", "gtsr_encoded_view_get", "gtsr_encoded_free", "gtsr_validate",
    "gtsr_plan_batch", "decode_meshlets", "gtsr_decode_meshlets_cfg", "gtsr_decode_meshlets_many",
    "decode_meshlets_batched", "gtsr_batched_graph_create", "gtsr_graph_launch",
    "gtsr_graph_destroy", "gtsr_device_cu_count", "gtsr_last_error", "gtsr_autotune_batched",
    "gtsr_server_create", "gtsr_server_submit", "gtsr_server_poll", "gtsr_server_release", "gtsr_server_cancel",
    "gtsr_server_get_stats", "gtsr_server_replay", "gtsr_server_destroy",
    "gtsr_gts_from_reuse", "gtsr_decode_gts", "gtsr_decode_gts_batched", "gtsr_decode_compact",
    "gtsr_quantize_attributes", "gtsr_dequantize", "gtsr_min_strips", "gtsr_meshlet_cones",
    "gtsr_decode_culled", "gtsr_stream_calib", "gtsr_decode_batched_noalloc",
    "gtsr_file_write", "gtsr_file_open", "gtsr_file_mesh_count", "gtsr_file_mesh_get", "gtsr_file_close",
)


class GtsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Meshlet(C.Structure):
    _fields_ = [("chunk_off", C.c_uint32), ("reuse_off", C.c_uint32), ("out_off", C.c_uint32),
                ("tri_count", C.c_uint16), ("vert_count", C.c_uint16)]


ENCODE_EXACT_STRIPS = 1


class EncodeParams(C.Structure):
    _fields_ = [("max_vertices", C.c_uint32), ("max_triangles", C.c_uint32),
                ("threads", C.c_uint32), ("flags", C.c_uint32)]


class EncodedView(C.Structure):
    _fields_ = [("meshlet_count", C.c_uint32), ("reserved", C.c_uint32),
                ("input_triangles", C.c_uint64), ("strip_triangles", C.c_uint64),
                ("restarts", C.c_uint64), ("reuse_count", C.c_uint64), ("split_meshlets", C.c_uint64),
                ("meshlets", C.c_void_p), ("bits", C.c_void_p), ("bits_bytes", C.c_uint64),
                ("reuse", C.c_void_p), ("reuse_bytes", C.c_uint64),
                ("vertices", C.c_void_p), ("vert_off", C.c_void_p),
                ("payload_bits", C.c_uint64), ("stored_bytes", C.c_uint64), ("kept_off", C.c_void_p),
                ("tri_ids", C.c_void_p), ("exact_tried", C.c_uint64), ("exact_proven", C.c_uint64)]


class StreamDesc(C.Structure):
    _fields_ = [("meshlets", C.c_void_p), ("bits", C.c_void_p), ("reuse", C.c_void_p),
                ("meshlet_count", C.c_uint32), ("reserved", C.c_uint32),
                ("bits_bytes", C.c_uint64), ("reuse_bytes", C.c_uint64),
                ("strip_triangles", C.c_uint64)]


class FileMesh(C.Structure):
    _fields_ = [("format", C.c_uint32), ("meshlet_count", C.c_uint32), ("strip_triangles", C.c_uint64),
                ("input_triangles", C.c_uint64), ("restarts", C.c_uint64), ("meshlets", C.c_void_p),
                ("bits", C.c_void_p), ("bits_bytes", C.c_uint64), ("reuse", C.c_void_p),
                ("reuse_bytes", C.c_uint64), ("vertices", C.c_void_p), ("vertex_count", C.c_uint64),
                ("vert_off", C.c_void_p), ("kept_off", C.c_void_p), ("tri_ids", C.c_void_p)]


class LaunchCfg(C.Structure):
    _fields_ = [("waves_per_group", C.c_uint32), ("meshlets_per_wave", C.c_uint32),
                ("groups_per_cu", C.c_uint32), ("run_tris", C.c_uint32), ("items_per_claim", C.c_uint32)]


BATCHED_WORKSPACE_BYTES = 1024   # GTSR_BATCHED_WORKSPACE_BYTES


class TunePoint(C.Structure):
    _fields_ = [("target_tris", C.c_uint32), ("work_items", C.c_uint32), ("cfg", LaunchCfg),
                ("median_ms", C.c_float), ("min_ms", C.c_float), ("stage", C.c_uint32),
                ("reserved", C.c_uint32)]

    def as_dict(self) -> dict:
        return {"target_tris": self.target_tris, "work_items": self.work_items,
                "waves_per_group": self.cfg.waves_per_group, "groups_per_cu": self.cfg.groups_per_cu,
                "run_tris": self.cfg.run_tris, "items_per_claim": self.cfg.items_per_claim,
                "median_ms": self.median_ms, "min_ms": self.min_ms, "stage": self.stage}


class AttrStream(C.Structure):
    _fields_ = [("lowest", C.c_void_p), ("offsets", C.c_void_p), ("vert_off", C.c_void_p),
                ("origin", C.c_void_p), ("delta", C.c_void_p), ("meshlet_count", C.c_uint32),
                ("channels", C.c_uint32), ("offset_count", C.c_uint64)]


class ServerParams(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("max_inflight", C.c_uint32),
                ("max_batch", C.c_uint32), ("target_tris", C.c_uint32), ("max_items", C.c_uint32),
                ("cfg", LaunchCfg), ("reserved", C.c_uint32), ("reserved2", C.c_uint32)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "batches", "max_batch_seen",
                                           "strip_triangles", "max_arena_used", "arena_used", "pending",
                                           "cancelled", "failed")]


COMPLETION_DTYPE = np.dtype([("tag", "<u8"), ("mesh", "<u4"), ("status", "<i4"), ("out_offset", "<u8"),
                             ("out_bytes", "<u8"), ("t_submit_ns", "<u8"), ("t_admit_ns", "<u8"),
                             ("t_done_ns", "<u8")])
assert COMPLETION_DTYPE.itemsize == 56

MESH_ENTRY_DTYPE = np.dtype([("meshlets", "<u8"), ("bits", "<u8"), ("reuse", "<u8"), ("out", "<u8"),
                             ("meshlet_count", "<u4"), ("reserved0", "<u4"), ("bits_bytes", "<u8"),
                             ("reuse_bytes", "<u8"), ("strip_triangles", "<u8")])
assert MESH_ENTRY_DTYPE.itemsize == 64
WORK_ITEM_DTYPE = np.dtype([("mesh", "<u4"), ("first", "<u4"), ("end", "<u4"), ("reserved", "<u4")])
MESHLET_DTYPE = np.dtype([("chunk_off", "<u4"), ("reuse_off", "<u4"), ("out_off", "<u4"),
                          ("tri_count", "<u2"), ("vert_count", "<u2")])

_lib = None


def lib():
    """The loaded ``libgtsr.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2404_06359_amd.build.build() "
                           "(there is no fallback decode path)")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
    sig = {
        "encode_meshlets": (C.c_int, [vp, u64, u32, C.POINTER(EncodeParams), C.POINTER(vp)]),
        "gtsr_encoded_view_get": (C.c_int, [vp, C.POINTER(EncodedView)]),
        "gtsr_encoded_free": (None, [vp]),
        "gtsr_validate": (C.c_int, [C.POINTER(StreamDesc)]),
        "gtsr_plan_batch": (C.c_int, [vp, vp, u32, u32, vp, u32, C.POINTER(u32)]),
        "decode_meshlets": (C.c_int, [C.POINTER(StreamDesc), vp, u64, vp]),
        "gtsr_decode_meshlets_cfg": (C.c_int, [C.POINTER(StreamDesc), vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_decode_meshlets_many": (C.c_int, [vp, vp, vp, u32, C.POINTER(LaunchCfg), vp]),
        "decode_meshlets_batched": (C.c_int, [vp, u32, vp, u32, vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_batched_graph_create": (C.c_int, [vp, u32, vp, u32, vp, u64, u32, C.POINTER(LaunchCfg),
                                                C.POINTER(vp)]),
        "gtsr_graph_launch": (C.c_int, [vp, vp]),
        "gtsr_graph_destroy": (None, [vp]),
        "gtsr_device_cu_count": (u32, []),
        "gtsr_last_error": (C.c_char_p, []),
        "gtsr_autotune_batched": (C.c_int, [vp, u32, u32, vp, vp, u32, vp, u64, vp, u32, u32, vp, u32,
                                            C.POINTER(u32), C.POINTER(TunePoint), vp]),
        "gtsr_server_create": (C.c_int, [vp, vp, u32, C.POINTER(ServerParams), C.POINTER(vp)]),
        "gtsr_server_submit": (C.c_int, [vp, u32, u64]),
        "gtsr_server_poll": (C.c_int, [vp, vp, u32, C.POINTER(u32), u32]),
        "gtsr_server_release": (C.c_int, [vp, u64]),
        "gtsr_server_cancel": (C.c_int, [vp, u64]),
        "gtsr_server_get_stats": (C.c_int, [vp, C.POINTER(ServerStats)]),
        "gtsr_server_replay": (C.c_int, [vp, vp, vp, u32, u64, vp, C.POINTER(u64)]),
        "gtsr_server_destroy": (None, [vp]),
        "gtsr_gts_from_reuse": (C.c_int, [C.POINTER(StreamDesc), vp, vp, u64, vp, u64]),
        "gtsr_decode_gts": (C.c_int, [C.POINTER(StreamDesc), vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_decode_gts_batched": (C.c_int, [vp, u32, vp, u32, vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_decode_compact": (C.c_int, [C.POINTER(StreamDesc), u32, vp, vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_quantize_attributes": (C.c_int, [vp, u32, u32, vp, vp, u32, u32, vp, vp, vp, vp]),
        "gtsr_dequantize": (C.c_int, [C.POINTER(AttrStream), vp, u64, C.POINTER(LaunchCfg), vp]),
        "gtsr_min_strips": (C.c_int, [vp, u32, u64, C.POINTER(u32), C.POINTER(u32)]),
        "gtsr_meshlet_cones": (C.c_int, [vp, u64, vp, u32, vp, vp, u32, vp]),
        "gtsr_decode_culled": (C.c_int, [C.POINTER(StreamDesc), vp, C.c_float, C.c_float, C.c_float, vp, u64,
                                         C.POINTER(LaunchCfg), vp]),
        "gtsr_stream_calib": (C.c_int, [vp, u64, vp, u64, C.POINTER(LaunchCfg), C.POINTER(u64), vp]),
        "gtsr_decode_batched_noalloc": (C.c_int, [vp, u32, vp, u32, u32, C.POINTER(LaunchCfg), vp]),
        "gtsr_file_write": (C.c_int, [C.c_char_p, vp, u32]),
        "gtsr_file_open": (C.c_int, [C.c_char_p, C.POINTER(vp)]),
        "gtsr_file_mesh_count": (C.c_int, [vp, C.POINTER(u32)]),
        "gtsr_file_mesh_get": (C.c_int, [vp, u32, C.POINTER(FileMesh)]),
        "gtsr_file_close": (None, [vp]),
    }
    for name, (rt, args) in sig.items():
        f = getattr(L, name)
        f.restype = rt
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        msg = lib().gtsr_last_error().decode(errors="replace")
        raise GtsrError(rc, msg)


def _cfg(cfg) -> C.POINTER(LaunchCfg):
    if cfg is None:
        return None
    if isinstance(cfg, LaunchCfg):
        return C.byref(cfg)
    c = LaunchCfg(int(cfg.get("waves_per_group", 0)), int(cfg.get("meshlets_per_wave", 0)),
                  int(cfg.get("groups_per_cu", 0)), int(cfg.get("run_tris", 0)), int(cfg.get("items_per_claim", 0)))
    return C.byref(c)


# ---------------------------------------------------------------- host side

@dataclass
class Encoded:
    """Host-resident encoded mesh (numpy copies of the library's arrays)."""

    meshlets: np.ndarray      # MESHLET_DTYPE[M]
    bits: np.ndarray          # uint8
    reuse: np.ndarray         # uint8
    verts: np.ndarray         # uint32 local -> global
    vert_off: np.ndarray      # uint64[M+1]
    stats: dict = field(default_factory=dict)
    kept_off: np.ndarray = None   # uint32[M+1]: input triangles before each meshlet
    tri_ids: np.ndarray = None    # uint32[T]: meshlet m's input triangles at kept_off[m]..kept_off[m+1]
    format: int = FORMAT_REUSE    # FORMAT_GTS: bits = 8-byte L/R words, reuse = index bytes

    @property
    def meshlet_count(self) -> int:
        return int(self.meshlets.shape[0])

    @property
    def strip_triangles(self) -> int:
        return int(self.stats["strip_triangles"])

    @property
    def desc_bytes(self) -> np.ndarray:
        return self.meshlets.view(np.uint8).reshape(-1)

    def host_stream(self) -> StreamDesc:
        return StreamDesc(self.meshlets.ctypes.data if self.meshlets.size else None,
                          self.bits.ctypes.data if self.bits.size else None,
                          self.reuse.ctypes.data if self.reuse.size else None,
                          self.meshlet_count, 0, self.bits.size, self.reuse.size, self.strip_triangles)


def encode(tri: np.ndarray, nverts: int, max_vertices: int = 64, max_triangles: int = 126,
           threads: int = 0, exact_strips: bool = False) -> Encoded:
    """Encode a CCW triangle list (``uint32[T,3]``) with the library encoder;
    ``exact_strips`` searches each meshlet for fewer strips than the greedy
    rule finds (``GTSR_ENCODE_EXACT_STRIPS``)."""
    L = lib()
    tri = np.ascontiguousarray(tri, dtype=np.uint32).reshape(-1, 3)
    params = EncodeParams(max_vertices, max_triangles, threads, ENCODE_EXACT_STRIPS if exact_strips else 0)
    h = C.c_void_p()
    _check(L.encode_meshlets(tri.ctypes.data if tri.size else None, tri.shape[0], nverts,
                             C.byref(params), C.byref(h)))
    try:
        v = EncodedView()
        _check(L.gtsr_encoded_view_get(h, C.byref(v)))
        M = v.meshlet_count

        def take(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dt)
            buf = (C.c_uint8 * (n * np.dtype(dt).itemsize)).from_address(ptr)
            return np.frombuffer(buf, dtype=dt, count=n).copy()

        meshlets = take(v.meshlets, M, MESHLET_DTYPE)
        bits = take(v.bits, v.bits_bytes, np.uint8)
        reuse = take(v.reuse, v.reuse_bytes, np.uint8)
        vert_off = take(v.vert_off, M + 1, np.uint64)
        verts = take(v.vertices, int(vert_off[-1]) if M else 0, np.uint32)
        stats = {k: int(getattr(v, k)) for k in ("input_triangles", "strip_triangles", "restarts",
                                                 "reuse_count", "split_meshlets", "payload_bits",
                                                 "stored_bytes")}
        if exact_strips:
            stats["exact_tried"], stats["exact_proven"] = int(v.exact_tried), int(v.exact_proven)
        kept_off = take(v.kept_off, M + 1, np.uint32)
        tri_ids = take(v.tri_ids, int(v.input_triangles) if M else 0, np.uint32)
    finally:
        L.gtsr_encoded_free(h)
    return Encoded(meshlets, bits, reuse, verts, vert_off, stats, kept_off, tri_ids)


def tune_key(arch: str, cus: int, fmt: int, meshes: int, strip_tris: int, meshlets: int) -> str:
    """Autotune cache key: the device and the workload's size class (mesh
    count and strip-triangle total to the nearest power of two, strip
    triangles per meshlet to the nearest multiple of 8)."""
    import math

    lg = lambda x: int(round(math.log2(x))) if x > 0 else -1
    per = int(round(strip_tris / meshlets / 8.0)) * 8 if meshlets else 0
    return f"{arch}/cu{cus}/{'gts' if fmt == FORMAT_GTS else 'reuse'}/m2^{lg(meshes)}/t2^{lg(strip_tris)}/tpm{per}"


def tune_cache_get(path: str, key: str):
    """The recorded pick for key in a JSON autotune cache, or None (also when
    the file is missing or unreadable)."""
    import json

    try:
        with open(path) as f:
            data = json.load(f)
        rec = data.get("entries", {}).get(key)
    except (OSError, ValueError, AttributeError):
        return None
    if not isinstance(rec, dict) or not {"target_tris", "cfg", "best"} <= rec.keys():
        return None
    return rec


def tune_cache_put(path: str, key: str, rec: dict) -> None:
    """Record a pick under key (the file is rewritten whole, by rename)."""
    import json

    try:
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict) or not isinstance(data.get("entries"), dict):
            data = {}
    except (OSError, ValueError):
        data = {}
    data.setdefault("version", 1)
    data.setdefault("entries", {})[key] = rec
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _take(ptr, n, dt):
    """A numpy copy of n elements of dtype dt at a host address."""
    if n == 0 or not ptr:
        return np.zeros(0, dt)
    buf = (C.c_uint8 * (n * np.dtype(dt).itemsize)).from_address(ptr)
    return np.frombuffer(buf, dtype=dt, count=n).copy()


def save(path: str, encs) -> None:
    """Write encoded meshes (``Encoded``, either format) to a ``.gtsr`` file
    (``gtsr_file_write``)."""
    n = len(encs)
    arr = (FileMesh * max(n, 1))()
    keep = []
    ptr = lambda a: a.ctypes.data if a is not None and a.size else None
    for i, e in enumerate(encs):
        parts = [np.ascontiguousarray(x) for x in (e.meshlets, e.bits, e.reuse, e.verts, e.vert_off)]
        kept = None if e.kept_off is None or not e.kept_off.size else np.ascontiguousarray(e.kept_off, np.uint32)
        tids = None if e.tri_ids is None or not e.tri_ids.size else np.ascontiguousarray(e.tri_ids, np.uint32)
        # the writer takes M + 1 offsets and input_triangles ids on trust: check the arrays hold them
        M = e.meshlet_count
        if (parts[4].dtype != np.uint64 or parts[4].size != M + 1 or parts[3].dtype != np.uint32
                or (kept is not None and kept.size != M + 1)
                or (tids is not None and tids.size != int(e.stats.get("input_triangles", 0)))):
            raise ValueError(f"save: mesh {i} lacks its vertex lists, offsets or triangle ids "
                             "(a stream-only Encoded cannot be saved)")
        keep.append((parts, kept, tids))
        arr[i] = FileMesh(e.format, e.meshlet_count, e.strip_triangles, int(e.stats.get("input_triangles", 0)),
                          int(e.stats.get("restarts", 0)), ptr(parts[0]), ptr(parts[1]), parts[1].nbytes,
                          ptr(parts[2]), parts[2].nbytes, ptr(parts[3]), parts[3].size, ptr(parts[4]),
                          ptr(kept), ptr(tids))
    _check(lib().gtsr_file_write(os.fsencode(path), arr, n))


def load(path: str) -> list:
    """Read and check a ``.gtsr`` file (``gtsr_file_open``); returns its meshes
    as ``Encoded`` (numpy copies; the file's memory is released)."""
    L = lib()
    h = C.c_void_p()
    _check(L.gtsr_file_open(os.fsencode(path), C.byref(h)))
    try:
        cnt = C.c_uint32()
        _check(L.gtsr_file_mesh_count(h, C.byref(cnt)))
        out = []
        for i in range(cnt.value):
            g = FileMesh()
            _check(L.gtsr_file_mesh_get(h, i, C.byref(g)))
            M = g.meshlet_count
            stats = {"input_triangles": int(g.input_triangles), "strip_triangles": int(g.strip_triangles),
                     "restarts": int(g.restarts)}
            if g.format == FORMAT_REUSE:
                stats["reuse_count"] = int(g.reuse_bytes)
            out.append(Encoded(_take(g.meshlets, M, MESHLET_DTYPE), _take(g.bits, g.bits_bytes, np.uint8),
                               _take(g.reuse, g.reuse_bytes, np.uint8), _take(g.vertices, g.vertex_count, np.uint32),
                               _take(g.vert_off, M + 1, np.uint64), stats,
                               _take(g.kept_off, M + 1, np.uint32) if g.kept_off else None,
                               _take(g.tri_ids, g.input_triangles, np.uint32) if g.tri_ids else None,
                               int(g.format)))
        return out
    finally:
        L.gtsr_file_close(h)


def min_strips(tri: np.ndarray, node_limit: int = 1_000_000):
    """``gtsr_min_strips``: (fewest strips found, whether proven optimal)."""
    tri = np.ascontiguousarray(tri, dtype=np.uint32).reshape(-1, 3)
    s, p = C.c_uint32(), C.c_uint32()
    _check(lib().gtsr_min_strips(tri.ctypes.data if tri.size else None, tri.shape[0], node_limit, C.byref(s),
                                 C.byref(p)))
    return int(s.value), bool(p.value)


def meshlet_cones(tri: np.ndarray, positions: np.ndarray, enc: Encoded) -> np.ndarray:
    """``gtsr_meshlet_cones``: float32[M, 4] {axis, cutoff} per meshlet of ``enc``
    (the encoding of ``tri``), from vertex positions float32[V, 3]."""
    tri = np.ascontiguousarray(tri, np.uint32).reshape(-1, 3)
    pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
    M = enc.meshlet_count
    out = np.zeros((M, 4), np.float32)
    ptr = lambda a: a.ctypes.data if a is not None and a.size else None
    _check(lib().gtsr_meshlet_cones(ptr(tri), tri.shape[0], ptr(pos), pos.shape[0], ptr(enc.tri_ids),
                                    ptr(enc.kept_off), M, ptr(out)))
    return out


def decode_culled(ds: DeviceStream, cones_dev, view, out=None, stream=None, cfg=None):
    """``gtsr_decode_culled``: decode the meshlets whose cone does not face away
    from ``view``; culled meshlets' output is left as it was."""
    torch = _torch()
    # the decoder reads one float4 {axis, cutoff} per meshlet
    if cones_dev.numel() * cones_dev.element_size() < 16 * ds.meshlet_count or not cones_dev.is_contiguous():
        raise ValueError(f"decode_culled: cones must hold {ds.meshlet_count} contiguous float4 records")
    if out is None:
        out = torch.zeros((ds.strip_triangles, 3), dtype=torch.uint8, device=ds.meshlets.device)
    d = ds.desc()
    _check(lib().gtsr_decode_culled(C.byref(d), cones_dev.data_ptr(), float(view[0]), float(view[1]),
                                    float(view[2]), out.data_ptr(), out.numel(), _cfg(cfg), _stream_handle(stream)))
    return out


def gts_from_reuse(enc: Encoded) -> Encoded:
    """The same mesh re-encoded as plain GTS (``gtsr_gts_from_reuse``): the
    returned ``Encoded`` has ``format == FORMAT_GTS``, ``bits`` holding the
    8-byte L/R words and ``reuse`` the index bytes."""
    assert enc.format == FORMAT_REUSE
    L = lib()
    M = enc.meshlet_count
    gdesc = np.zeros(M, MESHLET_DTYPE)
    words = np.zeros(enc.bits.size // 2, np.uint8)
    index = np.zeros(max(0, enc.strip_triangles - M), np.uint8)
    s = enc.host_stream()
    _check(L.gtsr_gts_from_reuse(C.byref(s), gdesc.ctypes.data if M else None, words.ctypes.data if words.size else None,
                                 words.size, index.ctypes.data if index.size else None, index.size))
    stats = dict(enc.stats)
    stats["stored_bytes"] = 16 * M + words.size + index.size
    stats["payload_bits"] = enc.strip_triangles + 8 * index.size
    return Encoded(gdesc, words, index, enc.verts, enc.vert_off, stats, enc.kept_off, enc.tri_ids, FORMAT_GTS)


def validate(enc: Encoded) -> int:
    """0 if the host stream is structurally valid, else the library's code."""
    s = enc.host_stream()
    return lib().gtsr_validate(C.byref(s))


def validate_arrays(desc: np.ndarray, bits: np.ndarray, reuse: np.ndarray, strip_triangles: int) -> int:
    desc = np.ascontiguousarray(desc, np.uint8)
    bits = np.ascontiguousarray(bits, np.uint8)
    reuse = np.ascontiguousarray(reuse, np.uint8)
    s = StreamDesc(desc.ctypes.data if desc.size else None, bits.ctypes.data if bits.size else None,
                   reuse.ctypes.data if reuse.size else None, desc.size // 16, 0, bits.size, reuse.size,
                   strip_triangles)
    return lib().gtsr_validate(C.byref(s))


def plan_batch(meshlet_arrays, target_tris: int = 2048) -> np.ndarray:
    """Triangle-balanced work list (``WORK_ITEM_DTYPE``) over several meshes'
    host descriptor arrays."""
    L = lib()
    n = len(meshlet_arrays)
    arrs = [np.ascontiguousarray(a, MESHLET_DTYPE) for a in meshlet_arrays]
    ptrs = (C.c_void_p * max(n, 1))(*[a.ctypes.data if a.size else None for a in arrs])
    counts = np.array([a.shape[0] for a in arrs] or [0], np.uint32)
    cnt = C.c_uint32()
    _check(L.gtsr_plan_batch(ptrs, counts.ctypes.data, n, target_tris, None, 0, C.byref(cnt)))
    items = np.zeros(cnt.value, WORK_ITEM_DTYPE)
    _check(L.gtsr_plan_batch(ptrs, counts.ctypes.data, n, target_tris,
                             items.ctypes.data if items.size else None, cnt.value, C.byref(cnt)))
    return items


# -------------------------------------------------------------- device side

def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclass
class DeviceStream:
    """One encoded mesh resident in device memory (torch uint8 tensors)."""

    meshlets: object
    bits: object
    reuse: object
    meshlet_count: int
    strip_triangles: int
    input_triangles: int = 0
    format: int = FORMAT_REUSE

    def desc(self) -> StreamDesc:
        return StreamDesc(self.meshlets.data_ptr(), self.bits.data_ptr(), self.reuse.data_ptr(),
                          self.meshlet_count, 0, self.bits.numel(), self.reuse.numel(),
                          self.strip_triangles)

    @property
    def nbytes(self) -> int:
        return self.meshlets.numel() + self.bits.numel() + self.reuse.numel()


def upload_padded(a: np.ndarray, device="cuda"):
    """A uint8 device copy of ``a`` whose allocation is padded with zeros to a
    multiple of 16 bytes (the decoders read reuse bytes in 16-byte blocks);
    the returned tensor has ``a``'s length."""
    torch = _torch()
    flat = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
    n = flat.size
    buf = torch.zeros((n + 15) // 16 * 16 + 16, dtype=torch.uint8, device=device)
    if n:
        buf[:n].copy_(torch.from_numpy(flat))
    return buf[:n]


def to_device(enc: Encoded, device="cuda") -> DeviceStream:
    return DeviceStream(upload_padded(enc.meshlets, device), upload_padded(enc.bits, device),
                        upload_padded(enc.reuse, device), enc.meshlet_count, enc.strip_triangles,
                        int(enc.stats.get("input_triangles", 0)), enc.format)


def decode(ds: DeviceStream, out=None, stream=None, cfg=None):
    """Decode one mesh on the GPU (either format); returns ``uint8[strip_triangles, 3]``."""
    torch = _torch()
    L = lib()
    if out is None:
        out = torch.empty((ds.strip_triangles, 3), dtype=torch.uint8, device=ds.meshlets.device)
    d = ds.desc()
    f = L.gtsr_decode_gts if ds.format == FORMAT_GTS else L.gtsr_decode_meshlets_cfg
    _check(f(C.byref(d), out.data_ptr(), out.numel(), _cfg(cfg), _stream_handle(stream)))
    return out


def decode_compact(ds: DeviceStream, kept_off, out=None, stream=None, cfg=None):
    """Decode one mesh without its restart degenerates (``gtsr_decode_compact``).
    ``kept_off``: uint32[M+1] kept offsets (numpy or a device tensor); returns
    ``uint8[kept_off[M], 3]``."""
    torch = _torch()
    L = lib()
    if isinstance(kept_off, np.ndarray):
        kept_host = np.ascontiguousarray(kept_off, np.uint32)
        kept_dev = torch.from_numpy(kept_host.view(np.int32).copy()).to(ds.meshlets.device)
        total = int(kept_host[-1]) if kept_host.size else 0
    else:
        kept_dev = kept_off
        total = None
    # the decoder reads meshlet_count + 1 four-byte offsets
    if kept_dev.element_size() != 4 or kept_dev.numel() < ds.meshlet_count + 1 or not kept_dev.is_contiguous():
        raise ValueError(f"decode_compact: kept_off must hold {ds.meshlet_count + 1} contiguous 32-bit offsets")
    if out is None:
        if total is None:   # reads the last offset back from the device (synchronizes)
            total = int(kept_off[-1].item()) if kept_off.numel() else 0
        out = torch.empty((total, 3), dtype=torch.uint8, device=ds.meshlets.device)
    d = ds.desc()
    _check(L.gtsr_decode_compact(C.byref(d), ds.format, kept_dev.data_ptr(), out.data_ptr(), out.numel(),
                                 _cfg(cfg), _stream_handle(stream)))
    return out


class Batch:
    """Many device-resident meshes decoded by one batched launch.

    Holds the device mesh table, the work list and one output
    tensor per mesh (views into a single allocation)."""

    def __init__(self, streams, target_tris: int = 768, host_meshlets=None, device="cuda", outs=None):
        torch = _torch()
        self.streams = list(streams)
        n = len(self.streams)
        tris = [s.strip_triangles for s in self.streams]
        if outs is None:
            total = sum(tris)
            self.out_all = torch.empty(3 * total + 16, dtype=torch.uint8, device=device)
            outs, off = [], 0
            for t in tris:
                outs.append(self.out_all[3 * off: 3 * (off + t)].view(t, 3))
                off += t
        self.outs = outs
        table = np.zeros(n, MESH_ENTRY_DTYPE)
        for i, (s, o) in enumerate(zip(self.streams, self.outs)):
            table[i] = (s.meshlets.data_ptr(), s.bits.data_ptr(), s.reuse.data_ptr(), o.data_ptr(),
                        s.meshlet_count, 0, s.bits.numel(), s.reuse.numel(), s.strip_triangles)
        self.table = torch.from_numpy(table.view(np.uint8).reshape(-1)).to(device)
        if host_meshlets is None:
            host_meshlets = [s.meshlets.cpu().numpy().view(MESHLET_DTYPE) for s in self.streams]
        items = plan_batch(host_meshlets, target_tris)
        self.work_items = int(items.shape[0])
        self.work = torch.from_numpy(items.view(np.uint8).reshape(-1).copy()).to(device)
        self.mesh_count = n
        self.workspace = torch.zeros(BATCHED_WORKSPACE_BYTES, dtype=torch.uint8, device=device)
        self._graphs = []

    def launch(self, stream=None, cfg=None):
        L = lib()
        _check(L.decode_meshlets_batched(self.table.data_ptr(), self.mesh_count, self.work.data_ptr(),
                                         self.work_items, self.workspace.data_ptr(), self.workspace.numel(),
                                         _cfg(cfg), _stream_handle(stream)))
        return self.outs

    def graph(self, cfg=None):
        """Capture the batched decode once; returns a callable launching it."""
        L = lib()
        h = C.c_void_p()
        _check(L.gtsr_batched_graph_create(self.table.data_ptr(), self.mesh_count, self.work.data_ptr(),
                                           self.work_items, self.workspace.data_ptr(), self.workspace.numel(),
                                           FORMAT_REUSE, _cfg(cfg), C.byref(h)))
        g = Graph(h, keep=(self.table, self.work, self.workspace))
        self._graphs.append(g)
        return g


class Graph:
    """A captured batched decode.  It holds the tensors whose addresses the
    graph baked in (mesh table, work list), so they outlive it; a ``Pool``
    closes its graphs when it is re-planned."""

    def __init__(self, handle, keep=()):
        self.handle = handle
        self._keep = keep

    def __call__(self, stream=None):
        if not self.handle:
            raise RuntimeError("this graph was closed (its pool was re-planned or closed): capture a new one")
        _check(lib().gtsr_graph_launch(self.handle, _stream_handle(stream)))

    def close(self):
        if self.handle:
            lib().gtsr_graph_destroy(self.handle)
            self.handle = None
        self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_calib(src, dst, stream=None, cfg=None) -> int:
    """One launch of the bandwidth calibration kernel (``gtsr_stream_calib``):
    reads 4 KiB of ``src`` and writes 13 KiB of ``dst`` (device uint8
    tensors) per step; returns the step count (17408 bytes moved per step)."""
    steps = C.c_uint64()
    _check(lib().gtsr_stream_calib(src.data_ptr(), src.numel(), dst.data_ptr(), dst.numel(), _cfg(cfg),
                                   C.byref(steps), _stream_handle(stream)))
    return int(steps.value)


def device_cu_count() -> int:
    return int(lib().gtsr_device_cu_count())


class Pool:
    """Many encoded meshes resident on the device in one allocation per array.

    Each mesh's descriptors, flag chunks and reuse bytes sit at 16-byte
    aligned offsets of three shared uint8 tensors; ``out`` holds every mesh's
    decoded triples back to back.  ``table`` is the device mesh table of the
    batched decoder, ``streams`` the per-mesh ``StreamDesc`` structs (device
    pointers) of the plain decoder."""

    def __init__(self, encs, device="cuda", out=True):
        torch = _torch()

        def pad16(n):
            return (n + 15) // 16 * 16

        n = len(encs)
        self.mesh_count = n
        formats = {e.format for e in encs}
        if len(formats) > 1:
            raise ValueError("a Pool holds streams of one format")
        self.format = formats.pop() if formats else FORMAT_REUSE
        self.meshlet_counts = np.array([e.meshlet_count for e in encs], np.uint32)
        self.strip_tris = np.array([e.strip_triangles for e in encs], np.uint64)
        self.input_tris = np.array([e.stats["input_triangles"] for e in encs], np.uint64)
        d_sz = np.array([e.meshlets.nbytes for e in encs], np.uint64)
        b_sz = np.array([e.bits.nbytes for e in encs], np.uint64)
        r_sz = np.array([e.reuse.nbytes for e in encs], np.uint64)
        d_off = np.concatenate([[0], np.cumsum([pad16(int(x)) for x in d_sz])]).astype(np.uint64)
        b_off = np.concatenate([[0], np.cumsum([pad16(int(x)) for x in b_sz])]).astype(np.uint64)
        r_off = np.concatenate([[0], np.cumsum([pad16(int(x)) for x in r_sz])]).astype(np.uint64)
        o_off = np.concatenate([[0], np.cumsum(3 * self.strip_tris)]).astype(np.uint64)
        hd = np.zeros(int(d_off[-1]) + 16, np.uint8)
        hb = np.zeros(int(b_off[-1]) + 16, np.uint8)
        hr = np.zeros(int(r_off[-1]) + 16, np.uint8)
        for i, e in enumerate(encs):
            hd[int(d_off[i]):int(d_off[i]) + int(d_sz[i])] = e.meshlets.view(np.uint8).reshape(-1)
            hb[int(b_off[i]):int(b_off[i]) + int(b_sz[i])] = e.bits
            hr[int(r_off[i]):int(r_off[i]) + int(r_sz[i])] = e.reuse
        self.host_meshlets = [e.meshlets for e in encs]
        self.d_meshlets = torch.from_numpy(hd).to(device)
        self.d_bits = torch.from_numpy(hb).to(device)
        self.d_reuse = torch.from_numpy(hr).to(device)
        self.out_offsets = o_off
        self.out = torch.empty(int(o_off[-1]) + 16, dtype=torch.uint8, device=device) if out else None
        self.stored_bytes = int(d_sz.sum() + b_sz.sum() + r_sz.sum())
        dm, db, dr = self.d_meshlets.data_ptr(), self.d_bits.data_ptr(), self.d_reuse.data_ptr()
        do = self.out.data_ptr() if out else 0
        table = np.zeros(n, MESH_ENTRY_DTYPE)
        table["meshlets"] = dm + d_off[:-1]
        table["bits"] = db + b_off[:-1]
        table["reuse"] = dr + r_off[:-1]
        table["out"] = do + o_off[:-1]
        table["meshlet_count"] = self.meshlet_counts
        table["bits_bytes"] = b_sz
        table["reuse_bytes"] = r_sz
        table["strip_triangles"] = self.strip_tris
        self.host_table = table
        self.table = torch.from_numpy(table.view(np.uint8).reshape(-1).copy()).to(device)
        self.streams = (StreamDesc * max(n, 1))()
        for i in range(n):
            self.streams[i] = StreamDesc(int(table["meshlets"][i]), int(table["bits"][i]),
                                         int(table["reuse"][i]), int(self.meshlet_counts[i]), 0,
                                         int(b_sz[i]), int(r_sz[i]), int(self.strip_tris[i]))
        self.out_ptrs = (C.c_void_p * max(n, 1))(*[int(x) for x in table["out"]])
        self.out_bytes = (C.c_uint64 * max(n, 1))(*[int(x) for x in 3 * self.strip_tris])
        self.work = None
        self.work_items = 0
        self.workspace = torch.zeros(BATCHED_WORKSPACE_BYTES, dtype=torch.uint8, device=device)
        self._graphs = []

    def output(self, i: int):
        """Decoded triples of mesh ``i`` (a view into ``out``)."""
        a, b = int(self.out_offsets[i]), int(self.out_offsets[i + 1])
        return self.out[a:b].view(-1, 3)

    def plan(self, target_tris: int = 768):
        torch = _torch()
        # graphs captured before hold the old work list's address and length
        for g in self._graphs:
            g.close()
        self._graphs = []
        items = plan_batch(self.host_meshlets, target_tris)
        self.work_items = int(items.shape[0])
        self.work = torch.from_numpy(items.view(np.uint8).reshape(-1).copy()).to(self.table.device) \
            if items.size else torch.zeros(16, dtype=torch.uint8, device=self.table.device)
        return self

    # candidate work-item sizes (strip triangles), in order of preference: the
    # tuner takes the first within 1% of the fastest, and with the XCD stripes
    # 1536 measured 0.6-1.3% faster than 768 on the mixed batched workload
    TUNE_TARGETS = (1536, 768, 3072, 384)

    def tune_key(self) -> str:
        """The autotune cache key of this pool: device (architecture, CU
        count), stream format, and the workload's size class (meshes,
        strip triangles, strip triangles per meshlet, each rounded to a
        power-of-two or 8-triangle bucket)."""
        torch = _torch()
        props = torch.cuda.get_device_properties(self.table.device)
        return tune_key(getattr(props, "gcnArchName", props.name), props.multi_processor_count, self.format,
                        self.mesh_count, int(self.strip_tris.sum()), int(self.meshlet_counts.sum()))

    def autotune(self, targets=None, cfgs=None, reps: int = 5, stream=None, mode=None, cache=None):
        """Measure the batched decoder over work-list targets x launch shapes
        (``gtsr_autotune_batched``) and keep the fastest: the pool's work list
        becomes the winning one (planned and uploaded before measuring, so no
        host work separates tuning from use).  Returns ``(best_cfg, best,
        points)``: ``best_cfg`` is a dict for ``decode_batched`` /
        ``batched_graph``; ``best`` and ``points`` are ``TunePoint.as_dict()``
        records whose ``target_tris`` is the target (not the list index).

        ``mode`` (default: the ``GTSR_AUTOTUNE`` environment variable, else
        "search"): "search" always measures and records the pick in the
        cache file, if one is named; "cache" takes the pick recorded for this
        pool's ``tune_key()`` without measuring (``points`` is then empty)
        and measures only when there is none; "off" measures nothing and
        plans the default work list with the default shape.  ``cache``: a
        JSON file (default: ``GTSR_AUTOTUNE_CACHE``)."""
        mode = mode or os.environ.get("GTSR_AUTOTUNE", "search")
        cache = cache or os.environ.get("GTSR_AUTOTUNE_CACHE")
        if mode not in ("search", "cache", "off"):
            raise ValueError(f"autotune mode must be search, cache or off, not {mode!r}")
        if mode == "off":
            self.plan()
            return {"waves_per_group": 0, "groups_per_cu": 0, "run_tris": 0, "items_per_claim": 0}, None, []
        key = self.tune_key() if cache else None
        if mode == "cache" and cache:
            hit = tune_cache_get(cache, key)
            if hit is not None:
                self.plan(hit["target_tris"])
                return dict(hit["cfg"]), dict(hit["best"]), []
        cfg, best, points = self._measure(targets, cfgs, reps, stream)
        if cache:
            tune_cache_put(cache, key, {"target_tris": best["target_tris"], "cfg": cfg, "best": best})
        return cfg, best, points

    def _measure(self, targets, cfgs, reps, stream):
        torch = _torch()
        L = lib()
        tg = [int(t) for t in (targets or self.TUNE_TARGETS)]
        lists = [plan_batch(self.host_meshlets, t) for t in tg]
        dev = [torch.from_numpy(x.view(np.uint8).reshape(-1).copy()).to(self.table.device) if x.size
               else torch.zeros(16, dtype=torch.uint8, device=self.table.device) for x in lists]
        ptrs = (C.c_void_p * len(tg))(*[d.data_ptr() for d in dev])
        counts = np.array([x.shape[0] for x in lists], np.uint32)
        cf = (LaunchCfg * max(len(cfgs or []), 1))()
        for i, c in enumerate(cfgs or []):
            cf[i] = LaunchCfg(int(c.get("waves_per_group", 0)), 0, int(c.get("groups_per_cu", 0)),
                              int(c.get("run_tris", 0)), int(c.get("items_per_claim", 0)))
        cap = len(tg) * max(1, len(cfgs or []) or 21)   # at most 21 built-in shapes
        pts = (TunePoint * cap)()
        cnt = C.c_uint32()
        best = TunePoint()
        _check(L.gtsr_autotune_batched(self.table.data_ptr(), self.mesh_count, self.format, ptrs,
                                       counts.ctypes.data, len(tg), self.workspace.data_ptr(), self.workspace.numel(),
                                       cf if cfgs else None, len(cfgs or []), reps, pts, cap, C.byref(cnt),
                                       C.byref(best), _stream_handle(stream)))
        k = int(best.target_tris)
        for g in self._graphs:
            g.close()
        self._graphs = []
        self.work, self.work_items = dev[k], int(counts[k])
        cfg = {"waves_per_group": int(best.cfg.waves_per_group), "groups_per_cu": int(best.cfg.groups_per_cu),
               "run_tris": int(best.cfg.run_tris), "items_per_claim": int(best.cfg.items_per_claim)}

        def rec(p):
            d = p.as_dict()
            d["target_tris"] = tg[int(p.target_tris)]
            return d
        return cfg, rec(best), [rec(pts[i]) for i in range(min(cnt.value, cap))]

    def decode_batched(self, stream=None, cfg=None):
        if self.work is None:
            self.plan()
        f = lib().gtsr_decode_gts_batched if self.format == FORMAT_GTS else lib().decode_meshlets_batched
        _check(f(self.table.data_ptr(), self.mesh_count, self.work.data_ptr(), self.work_items,
                 self.workspace.data_ptr(), self.workspace.numel(), _cfg(cfg), _stream_handle(stream)))

    def batched_graph(self, cfg=None):
        if self.work is None:
            self.plan()
        h = C.c_void_p()
        _check(lib().gtsr_batched_graph_create(self.table.data_ptr(), self.mesh_count, self.work.data_ptr(),
                                               self.work_items, self.workspace.data_ptr(), self.workspace.numel(),
                                               self.format, _cfg(cfg), C.byref(h)))
        g = Graph(h, keep=(self.table, self.work, self.workspace))
        self._graphs.append(g)
        return g

    def decode_per_mesh(self, stream=None, cfg=None):
        """One plain launch per mesh, back to back (enqueued from C)."""
        _check(lib().gtsr_decode_meshlets_many(self.streams, self.out_ptrs, self.out_bytes, self.mesh_count,
                                               _cfg(cfg), _stream_handle(stream)))


class Server:
    """Decode-request server over a ``Pool`` (``gtsr_server_*``): requests are
    admitted first-come first-served while their output fits the device arena
    of ``arena_bytes`` (the HBM budget for outputs in flight) and decoded in
    batches, up to ``max_inflight`` batches on the device at once."""

    def __init__(self, pool: "Pool", arena_bytes: int, max_inflight: int = 4, max_batch: int = 256,
                 target_tris: int = 768, max_items: int = 0, cfg=None):
        torch = _torch()
        self.pool = pool
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=pool.table.device)
        base = self.arena.data_ptr()
        self._arena_base = (base + 255) // 256 * 256
        c = LaunchCfg(0, 0, 0, 0, 0)
        if cfg:
            c = LaunchCfg(int(cfg.get("waves_per_group", 0)), 0, int(cfg.get("groups_per_cu", 0)),
                          int(cfg.get("run_tris", 0)))
        p = ServerParams(self._arena_base, int(arena_bytes), max_inflight, max_batch, target_tris, max_items,
                         c, 0, 0)
        n = pool.mesh_count
        self._arrs = [np.ascontiguousarray(a, MESHLET_DTYPE) for a in pool.host_meshlets]
        ptrs = (C.c_void_p * max(n, 1))(*[a.ctypes.data if a.size else None for a in self._arrs])
        table = np.ascontiguousarray(pool.host_table)
        h = C.c_void_p()
        _check(lib().gtsr_server_create(table.ctypes.data, ptrs, n, C.byref(p), C.byref(h)))
        self._h = h
        self._buf = np.zeros(1024, COMPLETION_DTYPE)

    def submit(self, mesh: int, tag: int):
        _check(lib().gtsr_server_submit(self._h, int(mesh), int(tag)))

    def poll(self, timeout_us: int = 0) -> np.ndarray:
        """Finished requests (``COMPLETION_DTYPE``), oldest first."""
        cnt = C.c_uint32()
        _check(lib().gtsr_server_poll(self._h, self._buf.ctypes.data, self._buf.size, C.byref(cnt),
                                      int(timeout_us)))
        return self._buf[:cnt.value].copy()

    def output(self, completion):
        """The decoded triples of a finished, unreleased request (a view into the arena)."""
        off = self._arena_base - self.arena.data_ptr() + int(completion["out_offset"])
        return self.arena[off:off + int(completion["out_bytes"])].view(-1, 3)

    def release(self, tag: int):
        _check(lib().gtsr_server_release(self._h, int(tag)))

    def cancel(self, tag: int) -> bool:
        """Withdraw a request not yet admitted (``gtsr_server_cancel``): True if
        it left the queue (poll reports it with status ``ECANCELED``), False if
        it was already admitted and completes normally."""
        rc = lib().gtsr_server_cancel(self._h, int(tag))
        if rc == EBUSY:
            return False
        _check(rc)
        return True

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().gtsr_server_get_stats(self._h, C.byref(st)))
        return {n: int(getattr(st, n)) for n, _ in ServerStats._fields_}

    def replay(self, arrival_ns: np.ndarray, meshes: np.ndarray, tag_base: int = 0):
        """Open-loop replay of an arrival trace (``gtsr_server_replay``); returns
        ``(completions, start_ns)``."""
        arr = np.ascontiguousarray(arrival_ns, np.uint64)
        ms = np.ascontiguousarray(meshes, np.uint32)
        out = np.zeros(arr.size, COMPLETION_DTYPE)
        start = C.c_uint64()
        _check(lib().gtsr_server_replay(self._h, arr.ctypes.data, ms.ctypes.data, arr.size, int(tag_base),
                                        out.ctypes.data, C.byref(start)))
        return out, int(start.value)

    def close(self):
        if self._h:
            lib().gtsr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- vertex attributes

@dataclass
class QuantizedAttrs:
    """Crack-free fixed-point attributes of one encoded mesh (host arrays)."""

    origin: np.ndarray    # float32[n]
    delta: np.ndarray     # float32[n]
    lowest: np.ndarray    # int32[M, n]
    offsets: np.ndarray   # uint16[sum V, n]
    vert_off: np.ndarray  # uint64[M + 1]


def quantize_attributes(attrs: np.ndarray, enc: Encoded, bits: int = 16) -> QuantizedAttrs:
    """``gtsr_quantize_attributes`` over the meshlets of ``enc``;
    ``attrs``: float32[vertex_count, channels]."""
    attrs = np.ascontiguousarray(attrs, np.float32)
    nv, n = attrs.shape
    M = enc.meshlet_count
    vert_off = np.ascontiguousarray(enc.vert_off, np.uint64)
    verts = np.ascontiguousarray(enc.verts, np.uint32)
    # the quantizer reads M + 1 offsets and vert_off[M] vertex ids
    if vert_off.size != M + 1 or verts.size != int(vert_off[-1]):
        raise ValueError("quantize_attributes: the encoding lacks its vertex lists (stream-only Encoded)")
    origin = np.zeros(n, np.float32)
    delta = np.zeros(n, np.float32)
    lowest = np.zeros((M, n), np.int32)
    offsets = np.zeros((int(vert_off[-1]) if M else 0, n), np.uint16)
    ptr = lambda a: a.ctypes.data if a.size else None
    _check(lib().gtsr_quantize_attributes(ptr(attrs), nv, n, ptr(verts), ptr(vert_off), M, bits, ptr(origin),
                                          ptr(delta), ptr(lowest), ptr(offsets)))
    return QuantizedAttrs(origin, delta, lowest, offsets, vert_off)


@dataclass
class DeviceAttrs:
    """``QuantizedAttrs`` resident on the device (torch tensors)."""

    lowest: object
    offsets: object
    vert_off: object
    origin: object
    delta: object
    meshlet_count: int
    channels: int
    offset_count: int

    def desc(self) -> AttrStream:
        return AttrStream(self.lowest.data_ptr(), self.offsets.data_ptr(), self.vert_off.data_ptr(),
                          self.origin.data_ptr(), self.delta.data_ptr(), self.meshlet_count, self.channels,
                          self.offset_count)

    @property
    def elements(self) -> int:
        return self.offset_count


def attrs_to_device(q: QuantizedAttrs, device="cuda") -> DeviceAttrs:
    up = lambda a: upload_padded(np.ascontiguousarray(a), device)
    return DeviceAttrs(up(q.lowest), up(q.offsets), up(q.vert_off), up(q.origin), up(q.delta),
                       int(q.lowest.shape[0]), int(q.origin.shape[0]), int(q.offsets.size))


def dequantize(da: DeviceAttrs, out=None, stream=None, cfg=None):
    """``gtsr_dequantize``: float32[sum V, channels] on the device."""
    torch = _torch()
    if out is None:
        out = torch.empty((da.elements // max(da.channels, 1), da.channels), dtype=torch.float32,
                          device=da.offsets.device)
    d = da.desc()
    _check(lib().gtsr_dequantize(C.byref(d), out.data_ptr(), out.numel(), _cfg(cfg), _stream_handle(stream)))
    return out
