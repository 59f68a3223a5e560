"""Closed-form (data-parallel) GTS-Reuse decode, pure Python -- TEST INFRASTRUCTURE.

This is the per-triangle formulation of Sec. 4.2 / 4.3 of the paper, written
so that each triangle is computed on its own, without the result of the
triangle before it (the property the paper's data-parallel decoder needs):

* index stream (Sec. 4.3): ``I[0], I[1], I[2] = 0, 1, 2``; for ``t >= 1`` the
  inclusive prefix sum of the increment flags gives ``s_t = 2 + sum(g[1..t])``
  (the first triangle contributes the implicit 2); a set flag makes
  ``I[t+2] = s_t``, a clear flag reads the reuse array at ``t + 1 - s_t``;
* pivot (Sec. 4.2, the search for the last L/R flip): ``k_t`` is the last
  position before ``t`` whose flag differs from ``f[t]`` (``-1`` if none) and
  the pivot vertex is ``X_t = I[k_t + 1]``;
* orientation (Sec. 4.2): flag L gives ``(X_t, I[t+1], I[t+2])``, flag R gives
  ``(I[t+1], X_t, I[t+2])``.

It shares nothing with ``oracle.c``'s sequential walk; the tests check that the
two agree on every tiny stream.  Pure-Python loops: tiny inputs only.
"""
from __future__ import annotations

L, R = 0, 1


def decode_meshlet_closed_form(f, g, r):
    """Decode one meshlet.

    ``f``: list of L/R flags, length T_s.  ``g``: increment flags, length T_s
    (``g[0]`` ignored).  ``r``: reuse bytes.  Returns a list of T_s triples.
    """
    T = len(f)
    I = [0, 1, 2] + [None] * (T - 1)
    for t in range(1, T):
        s = 2 + sum(g[1:t + 1])
        I[t + 2] = s if g[t] else r[t + 1 - s]
    out = []
    for t in range(T):
        k = -1
        for q in range(t - 1, -1, -1):
            if f[q] != f[t]:
                k = q
                break
        X = I[k + 1]
        if f[t] == L:
            out.append((X, I[t + 1], I[t + 2]))
        else:
            out.append((I[t + 1], X, I[t + 2]))
    return out


def unpack_meshlet(desc16: bytes, bits: bytes, reuse: bytes):
    """Parse one meshlet's descriptor, flags and reuse bytes from raw bytes."""
    chunk_off = int.from_bytes(desc16[0:4], "little")
    reuse_off = int.from_bytes(desc16[4:8], "little")
    out_off = int.from_bytes(desc16[8:12], "little")
    T = int.from_bytes(desc16[12:14], "little")
    V = int.from_bytes(desc16[14:16], "little")
    f, g = [], []
    for t in range(T):
        c = chunk_off + t // 64
        lr = int.from_bytes(bits[16 * c:16 * c + 8], "little")
        inc = int.from_bytes(bits[16 * c + 8:16 * c + 16], "little")
        f.append((lr >> (t % 64)) & 1)
        g.append((inc >> (t % 64)) & 1)
    n_ru = T + 2 - V
    r = list(reuse[reuse_off:reuse_off + n_ru])
    return out_off, f, g, r


def decode_closed_form(desc: bytes, bits: bytes, reuse: bytes):
    """Decode a whole stream; returns a flat list of triples in output order."""
    desc, bits, reuse = bytes(desc), bytes(bits), bytes(reuse)
    out = []
    for m in range(len(desc) // 16):
        _, f, g, r = unpack_meshlet(desc[16 * m:16 * m + 16], bits, reuse)
        out.extend(decode_meshlet_closed_form(f, g, r))
    return out
