"""Build raw GTS-Reuse stream bytes from per-meshlet flag lists (test inputs).

The layout (little-endian): a 16-byte descriptor per meshlet
``{u32 chunk_off, u32 reuse_off, u32 out_off, u16 T_s, u16 V}``; per 64 strip
triangles one 16-byte chunk ``{u64 LR, u64 INC}`` (bit i = triangle 64c+i,
LR 1 = R, INC 1 = new vertex, triangle 0 has no INC bit); reuse bytes meshlet
by meshlet.  This only packs bits given to it; it decodes nothing.
"""
from __future__ import annotations

import itertools

import numpy as np

L, R = 0, 1


def pack(meshlets):
    """``meshlets``: iterable of ``(f, g, r)``; ``f`` and ``g`` have length
    T_s (``g[0]`` ignored, stored 0), ``r`` lists the reuse bytes.
    Returns ``(desc, bits, reuse, strip_triangles)`` as uint8 arrays + int."""
    desc, bits, reuse = bytearray(), bytearray(), bytearray()
    chunk = 0
    out = 0
    for f, g, r in meshlets:
        T = len(f)
        V = 3 + sum(g[1:])
        nch = (T + 63) // 64
        desc += (chunk.to_bytes(4, "little") + len(reuse).to_bytes(4, "little") +
                 out.to_bytes(4, "little") + T.to_bytes(2, "little") + V.to_bytes(2, "little"))
        for c in range(nch):
            lr = inc = 0
            for i in range(64):
                t = 64 * c + i
                if t >= T:
                    break
                lr |= (f[t] & 1) << i
                if t >= 1:
                    inc |= (g[t] & 1) << i
            bits += lr.to_bytes(8, "little") + inc.to_bytes(8, "little")
        reuse += bytes(r)
        chunk += nch
        out += T
    return (np.frombuffer(bytes(desc), np.uint8).copy(), np.frombuffer(bytes(bits), np.uint8).copy(),
            np.frombuffer(bytes(reuse), np.uint8).copy(), out)


def all_streams(T: int):
    """Every meshlet stream with T_s = T: all flag words, all increment words,
    and at each reuse slot every vertex already introduced (0..s_t)."""
    for f in itertools.product((L, R), repeat=T):
        for gt in itertools.product((0, 1), repeat=T - 1):
            g = (0,) + gt
            # reuse slots and their choice ranges
            ranges = []
            s = 2
            for t in range(1, T):
                if g[t]:
                    s += 1
                else:
                    ranges.append(range(0, s + 1))
            for r in itertools.product(*ranges):
                yield list(f), list(g), list(r)


def random_stream(rng: np.random.Generator, T: int, p_inc: float = 0.55, p_r: float = 0.5):
    """A random valid meshlet stream with T_s = T (V capped at 256)."""
    f = [int(x) for x in (rng.random(T) < p_r)]
    g = [0]
    s = 2
    r = []
    for t in range(1, T):
        inc = (rng.random() < p_inc) and s < 255
        g.append(int(inc))
        if inc:
            s += 1
        else:
            r.append(int(rng.integers(0, s + 1)))
    return f, g, r


def pack_gts(meshlets):
    """Plain GTS stream bytes. ``meshlets``: iterable of ``(f, idx)``; ``f`` has
    length T_s, ``idx`` the T_s - 1 index bytes of triangles 1..T_s-1.  Layout:
    16-byte descriptor ``{u32 word_off, u32 index_off, u32 out_off, u16 T_s,
    u16 V}`` (V = 1 + largest index, at least 3), one u64 L/R word per 64 strip
    triangles, index bytes meshlet by meshlet.  Returns ``(desc, words, index,
    strip_triangles)``."""
    desc, words, index = bytearray(), bytearray(), bytearray()
    word = out = 0
    for f, idx in meshlets:
        T = len(f)
        assert len(idx) == T - 1
        V = max([2] + list(idx)) + 1
        nw = (T + 63) // 64
        desc += (word.to_bytes(4, "little") + len(index).to_bytes(4, "little") + out.to_bytes(4, "little") +
                 T.to_bytes(2, "little") + V.to_bytes(2, "little"))
        for w in range(nw):
            lr = 0
            for i in range(64):
                t = 64 * w + i
                if t < T:
                    lr |= (f[t] & 1) << i
            words += lr.to_bytes(8, "little")
        index += bytes(idx)
        word += nw
        out += T
    return (np.frombuffer(bytes(desc), np.uint8).copy(), np.frombuffer(bytes(words), np.uint8).copy(),
            np.frombuffer(bytes(index), np.uint8).copy(), out)
