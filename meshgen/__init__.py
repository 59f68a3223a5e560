"""Seeded synthetic triangle meshes for the meshlet-connectivity codec.

This module only produces input connectivity (``uint32[T, 3]`` CCW triangle
lists plus a vertex count).  It holds none of the codec's arithmetic: no
meshlet building, no strips, no bit packing, no decoding.  Both the oracle
side (tests) and the product side (bench) draw their inputs from here.

The paper evaluates on six scanned meshes that are not available here; these
generators stand in for them with the shapes of its workloads (regular grids,
subdivided spheres, irregular Delaunay patches), as listed per workload below.

Every generator takes a ``numpy.random.Generator``; ``rng_for(workload, i)``
builds the one used for mesh ``i`` of a workload, so each mesh is reproducible
on its own.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = (2404, 6359)

HERE = os.path.dirname(os.path.abspath(__file__))
# MESHGEN_LIBRARY names another build of meshgen.c (the sanitized one, see
# build_sanitized); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("MESHGEN_LIBRARY") or os.path.join(HERE, "libmeshgen.so")
SANITIZED_PATH = os.path.join(os.path.dirname(HERE), "_build", "sanitize", "libmeshgen.so")
_lib = None
_lib_lock = threading.Lock()


def build() -> str:
    """Compile ``meshgen.c`` (plain C, gcc) into ``libmeshgen.so``."""
    tmp = f"{LIB_PATH}.{os.getpid()}.tmp"   # private per process: test workers may build at once
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp,
                    os.path.join(HERE, "meshgen.c"), "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_sanitized() -> str:
    """``meshgen.c`` with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc), into ``_build/sanitize/libmeshgen.so``, for CPU test runs."""
    os.makedirs(os.path.dirname(SANITIZED_PATH), exist_ok=True)
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-shared", "-fPIC", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", f"{SANITIZED_PATH}.{os.getpid()}.tmp",
                    os.path.join(HERE, "meshgen.c"), "-lm"], check=True)
    os.replace(f"{SANITIZED_PATH}.{os.getpid()}.tmp", SANITIZED_PATH)
    return SANITIZED_PATH


def _clib():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            L = C.CDLL(LIB_PATH)
            vp = C.c_void_p
            L.mg_grid.argtypes = [C.c_uint32, C.c_uint32, vp, vp, vp]
            L.mg_grid.restype = None
            L.mg_icosphere.argtypes = [C.c_uint32, vp, vp]
            L.mg_icosphere.restype = C.c_int
            L.mg_sphere_patch.argtypes = [vp, C.c_uint64, vp, C.c_uint64, C.c_uint64, vp, vp,
                                          C.POINTER(C.c_uint32)]
            L.mg_sphere_patch.restype = C.c_int
            _lib = L
    return _lib


def rng_for(workload: int, i: int = 0) -> np.random.Generator:
    """Generator for mesh ``i`` of workload ``workload`` (1..5)."""
    return np.random.default_rng(np.random.SeedSequence([*SEED_ROOT, workload, i]))


@dataclass
class Mesh:
    """A triangle list: ``tri[t] = (a, b, c)`` counter-clockwise, ids < ``nverts``."""

    tri: np.ndarray  # uint32[T, 3], C-contiguous
    nverts: int
    kind: str = ""
    max_vertices: int = 64
    max_triangles: int = 126
    meta: dict = field(default_factory=dict)

    @property
    def ntri(self) -> int:
        return int(self.tri.shape[0])


def _finish(tri: np.ndarray, nverts: int, rng: np.random.Generator | None,
            permute: bool) -> np.ndarray:
    tri = np.asarray(tri, dtype=np.int64)
    if permute and nverts > 0:
        perm = rng.permutation(nverts).astype(np.int64)
        tri = perm[tri]
    return np.ascontiguousarray(tri, dtype=np.uint32)


# --------------------------------------------------------------------------
# Regular grid
# --------------------------------------------------------------------------

def grid(nx: int, ny: int, rng: np.random.Generator, permute: bool = True) -> Mesh:
    """``nx`` x ``ny`` quads on an ``(nx+1)`` x ``(ny+1)`` lattice.

    Each quad is split along a diagonal picked by ``rng.integers(2)``; vertex
    ids are shuffled by ``rng.permutation`` when ``permute`` is set.  Triangles
    keep generation order (quad by quad, row-major), two per quad.
    """
    if nx <= 0 or ny <= 0:
        return Mesh(np.zeros((0, 3), np.uint32), 0, "grid")
    diag = np.ascontiguousarray(rng.integers(0, 2, size=nx * ny).astype(np.uint8))
    nverts = (nx + 1) * (ny + 1)
    perm = np.ascontiguousarray(rng.permutation(nverts).astype(np.uint32)) if permute else None
    tri = np.empty((2 * nx * ny, 3), np.uint32)
    _clib().mg_grid(nx, ny, diag.ctypes.data, perm.ctypes.data if perm is not None else None,
                    tri.ctypes.data)
    return Mesh(tri, nverts, "grid")


# --------------------------------------------------------------------------
# Icosphere
# --------------------------------------------------------------------------

_ico_cache: dict = {}
_ico_lock = threading.Lock()


def icosphere(level: int):
    """Unit icosphere after ``level`` 1-to-4 subdivisions (outward CCW).

    Returns ``(positions float64[V,3], faces uint32[20*4**level, 3])`` with
    ``V = 10*4**level + 2``.  Cached per level; callers must not modify.
    """
    with _ico_lock:
        hit = _ico_cache.get(level)
        if hit is None:
            nv, nf = 10 * 4 ** level + 2, 20 * 4 ** level
            v = np.empty((nv, 3), np.float64)
            f = np.empty((nf, 3), np.uint32)
            if _clib().mg_icosphere(level, v.ctypes.data, f.ctypes.data) != 0:
                raise MemoryError("icosphere")
            v.setflags(write=False)
            f.setflags(write=False)
            hit = _ico_cache[level] = (v, f)
    return hit


def sphere(level: int, rng: np.random.Generator, permute: bool = True,
           jitter: float = 0.1) -> Mesh:
    """Whole icosphere, vertex ids shuffled.  Positions get per-coordinate
    Gaussian jitter of ``jitter`` x the mean edge length; connectivity does not
    depend on them and the codec never reads them."""
    v, f = icosphere(level)
    nverts = v.shape[0]
    edge = np.linalg.norm(v[f[:, 0]] - v[f[:, 1]], axis=1).mean()
    pos = v + rng.normal(0.0, jitter * edge, size=v.shape)
    tri = np.asarray(f)
    if permute:
        perm = rng.permutation(nverts).astype(np.uint32)
        tri = perm[tri]
        inv = np.empty_like(perm)
        inv[perm] = np.arange(nverts)
        pos = pos[inv]
    return Mesh(np.ascontiguousarray(tri, np.uint32), nverts, "sphere",
                meta={"positions": pos, "level": level})


def vertex_attributes(mesh: Mesh) -> np.ndarray:
    """Eight float32 channels per vertex (position xyz, unit normal xyz,
    texture uv) for meshes that carry positions: a sphere's jittered
    positions with radial normals and spherical uv, or a Delaunay mesh's
    points at z = 0 with normal +z and uv = xy."""
    if "positions" in mesh.meta:
        p = np.asarray(mesh.meta["positions"], np.float64)
        nrm = p / np.linalg.norm(p, axis=1, keepdims=True)
        uv = np.stack([np.arctan2(nrm[:, 1], nrm[:, 0]) / (2 * math.pi) + 0.5,
                       np.arccos(np.clip(nrm[:, 2], -1.0, 1.0)) / math.pi], 1)
    elif "points" in mesh.meta:
        xy = np.asarray(mesh.meta["points"], np.float64)
        p = np.concatenate([xy, np.zeros((xy.shape[0], 1))], 1)
        nrm = np.tile([0.0, 0.0, 1.0], (xy.shape[0], 1))
        uv = xy
    else:
        raise ValueError("mesh carries no positions")
    return np.ascontiguousarray(np.concatenate([p, nrm, uv], 1), np.float32)


def sphere_patch(n: int, rng: np.random.Generator, permute: bool = True) -> Mesh:
    """About ``n`` connected triangles cut from the smallest icosphere with at
    least ``n`` faces: the ``n`` faces whose centroids lie closest to a seeded
    direction (a spherical cap), vertex ids compacted then shuffled."""
    n = max(1, int(n))
    level = 0
    while 20 * 4 ** level < n:
        level += 1
    v, f = icosphere(level)
    d = rng.normal(size=3)
    d = np.ascontiguousarray(d / np.linalg.norm(d))
    tri = np.empty((n, 3), np.uint32)
    nv = C.c_uint32()
    rc = _clib().mg_sphere_patch(v.ctypes.data, v.shape[0], f.ctypes.data, f.shape[0], n,
                                 d.ctypes.data, tri.ctypes.data, C.byref(nv))
    if rc != 0:
        raise MemoryError("sphere_patch")
    nverts = int(nv.value)
    if permute:
        perm = rng.permutation(nverts).astype(np.uint32)
        tri = perm[tri]
    return Mesh(np.ascontiguousarray(tri, np.uint32), nverts, "patch", meta={"level": level})


# --------------------------------------------------------------------------
# Delaunay
# --------------------------------------------------------------------------

def delaunay(n: int, rng: np.random.Generator) -> Mesh:
    """Delaunay triangulation (Qhull via scipy) of about ``(n+2)/2`` uniform
    random points in the unit square, every triangle turned counter-clockwise.
    Yields roughly ``n`` irregular triangles; point order is already random."""
    from scipy.spatial import Delaunay

    p = max(3, (int(n) + 2) // 2 + int(2.0 * math.sqrt(max(n, 1))))
    pts = rng.random((p, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    a, b, c = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    neg = cross < 0
    tri[neg] = tri[neg][:, [0, 2, 1]]
    return Mesh(np.ascontiguousarray(tri, np.uint32), p, "delaunay", meta={"points": pts})


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

CAPS = ((32, 64), (64, 126), (128, 256))


def loguniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def grid_for(n: int, rng: np.random.Generator, permute: bool = True) -> Mesh:
    w = max(1, math.ceil(math.sqrt(n / 2)))
    h = max(1, math.ceil(n / (2 * w)))
    return grid(w, h, rng, permute=permute)


def workload1() -> Mesh:
    """Single 64x64 quad grid: 4225 vertices, 8192 triangles, caps 64v/126t."""
    m = grid(64, 64, rng_for(1, 0))
    m.max_vertices, m.max_triangles = 64, 126
    return m


def workload2(level: int = 9) -> Mesh:
    """Single icosphere at level 9: 5,242,880 triangles, 2,621,442 vertices,
    caps 64v/126t."""
    m = sphere(level, rng_for(2, 0))
    m.max_vertices, m.max_triangles = 64, 126
    return m


def workload3_spec(count: int = 2000, lo: float = 1e3, hi: float = 2e6):
    """Per-mesh recipe of the batched workload: ``(kind, n, caps)`` for each of
    ``count`` meshes, drawn from ``rng_for(3, i)`` (so any prefix is stable)."""
    out = []
    for i in range(count):
        r = rng_for(3, i)
        n = loguniform_int(r, lo, hi)
        kind = "grid" if r.integers(2) == 0 else "patch"
        caps = CAPS[int(r.integers(3))]
        out.append((kind, n, caps))
    return out


def workload3_mesh(i: int, lo: float = 1e3, hi: float = 2e6) -> Mesh:
    """Mesh ``i`` of the batched workload (jittered grid or sphere patch with
    triangle count log-uniform in [lo, hi], caps uniform over the three)."""
    r = rng_for(3, i)
    n = loguniform_int(r, lo, hi)
    kind = "grid" if r.integers(2) == 0 else "patch"
    caps = CAPS[int(r.integers(3))]
    m = grid_for(n, r) if kind == "grid" else sphere_patch(n, r)
    m.max_vertices, m.max_triangles = caps
    m.meta["target_n"] = n
    return m


def workload4_mesh(i: int, lo: float = 5e4, hi: float = 1e6) -> Mesh:
    """Mesh ``i`` of the stress workload: Delaunay of uniform random points with
    triangle count log-uniform in [lo, hi], caps 64v/126t."""
    r = rng_for(4, i)
    n = loguniform_int(r, lo, hi)
    m = delaunay(n, r)
    m.max_vertices, m.max_triangles = 64, 126
    m.meta["target_n"] = n
    return m


def workload4(count: int = 200, threads: int = 1) -> list:
    """The stress workload: meshes 0..count-1 of ``workload4_mesh``, generated
    on ``threads`` threads (Qhull runs outside the interpreter lock)."""
    if threads <= 1:
        return [workload4_mesh(i) for i in range(count)]
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(workload4_mesh, range(count)))


SERVE_LO, SERVE_HI, SERVE_LEVELS = 1e4, 2e7, 16


def workload5_prototype(kind: int, cap: int, level: int) -> Mesh:
    """Prototype of the serving pool: ``kind`` 0 = grid, 1 = sphere patch; caps
    ``CAPS[cap]``; triangle count at the centre of log-size level ``level`` of
    ``SERVE_LEVELS`` equal steps over [1e4, 2e7]."""
    r = rng_for(5, 100000 + (kind * 3 + cap) * SERVE_LEVELS + level)
    step = math.log(SERVE_HI / SERVE_LO) / SERVE_LEVELS
    n = int(round(SERVE_LO * math.exp((level + 0.5) * step)))
    m = grid_for(n, r) if kind == 0 else sphere_patch(n, r)
    m.max_vertices, m.max_triangles = CAPS[cap]
    m.meta["target_n"] = n
    return m


def workload5_entries(count: int = 5000) -> np.ndarray:
    """Pool entry i -> prototype index ``(kind * 3 + cap) * SERVE_LEVELS + level``:
    its triangle count is drawn log-uniform in [1e4, 2e7] and rounded to the
    nearest level, kind and caps uniform."""
    out = np.zeros(count, np.int64)
    step = math.log(SERVE_HI / SERVE_LO) / SERVE_LEVELS
    for i in range(count):
        r = rng_for(5, i)
        u = r.uniform(0.0, math.log(SERVE_HI / SERVE_LO))
        level = min(SERVE_LEVELS - 1, int(u / step))
        kind, cap = int(r.integers(2)), int(r.integers(3))
        out[i] = (kind * 3 + cap) * SERVE_LEVELS + level
    return out


def workload5_spec(count: int = 5000, lo: float = 1e4, hi: float = 2e7):
    """Per-mesh recipe of the serving pool of distinct meshes: ``(kind, n,
    caps)`` for mesh ``i`` of ``count``, the draws ``workload5_mesh(i)`` makes
    before it builds the mesh."""
    out = []
    for i in range(count):
        r = rng_for(5, i)
        n = loguniform_int(r, lo, hi)
        kind = "grid" if r.integers(2) == 0 else "patch"
        out.append((kind, n, CAPS[int(r.integers(3))]))
    return out


def workload5_mesh(i: int, lo: float = 1e4, hi: float = 2e7, permute: bool = True) -> Mesh:
    """Mesh ``i`` of the serving pool: like the batched workload, triangle
    count log-uniform in [lo, hi].  ``permute=False`` keeps the generator's
    vertex numbering instead of shuffling it (the shuffle is the last draw, so
    the triangles are otherwise the same; the encoded streams do not depend on
    global vertex ids, only the vertex lists do)."""
    r = rng_for(5, i)
    n = loguniform_int(r, lo, hi)
    kind = "grid" if r.integers(2) == 0 else "patch"
    caps = CAPS[int(r.integers(3))]
    m = grid_for(n, r, permute) if kind == "grid" else sphere_patch(n, r, permute)
    m.max_vertices, m.max_triangles = caps
    m.meta["target_n"] = n
    return m


# --------------------------------------------------------------------------
# Small shapes for tests
# --------------------------------------------------------------------------

def fan(k: int, rng: np.random.Generator | None = None) -> Mesh:
    """``k`` triangles around hub vertex 0 (an open fan), CCW."""
    tri = np.stack([np.zeros(k, np.int64), np.arange(1, k + 1), np.arange(2, k + 2)], 1)
    return Mesh(np.ascontiguousarray(tri, np.uint32), k + 2, "fan")


def disjoint(k: int) -> Mesh:
    """``k`` triangles that share no vertex."""
    tri = np.arange(3 * k, dtype=np.int64).reshape(k, 3)
    return Mesh(np.ascontiguousarray(tri, np.uint32), 3 * k, "disjoint")
