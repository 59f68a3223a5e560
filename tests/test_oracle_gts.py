"""CPU pins for the oracle's plain GTS decoder and degenerate compaction.

Plain GTS (Sec. 4.2, Fig. "Strip Encoding" (c)) keeps the L/R flags and stores
the local index every triangle after the first adds, one byte each; 0, 1, 2
are implicit.  Compaction drops the four degenerate triangles each restart
adds (Sec. 4.2).  Pins: textbook strips and fans written out by hand, the
GTS-Reuse closed form on every tiny stream, the payload arithmetic, round
trips to the input mesh and the disjoint-triangle restart closed form.
"""
import numpy as np
import pytest

import meshgen
import oracle as O
from oracle import defn
from streams import L, R, all_streams, pack, pack_gts, random_stream


def gts_walk(meshlets):
    desc, words, index, ts = pack_gts(meshlets)
    return O.decode_gts(O.GtsStream(desc, words, index, ts))


@pytest.mark.parametrize("T", [1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200, 254])
def test_gts_textbook_strip(T):
    """Alternating flags with indices 3, 4, 5, ...: triangle t is (t, t+1,
    t+2), winding flipped on odd t."""
    f = [L if t % 2 == 0 else R for t in range(T)]
    got = gts_walk([(f, [t + 3 for t in range(T - 1)])])
    expect = [(t, t + 1, t + 2) if t % 2 == 0 else (t + 1, t, t + 2) for t in range(T)]
    np.testing.assert_array_equal(got, np.array(expect, np.uint8))


@pytest.mark.parametrize("T", [2, 31, 32, 33, 63, 64, 65, 127, 128, 200, 253])
def test_gts_encoder_shaped_fan(T):
    """Flags L, R, L, L, ... (the hub becomes vertex 2): (0,1,2), (2,1,3),
    then (2, t+1, t+2); fans longer than the 32- and 64-bit words."""
    f = [L, R] + [L] * (T - 2)
    got = gts_walk([(f, [t + 3 for t in range(T - 1)])])
    expect = [(0, 1, 2), (2, 1, 3)] + [(2, t + 1, t + 2) for t in range(2, T)]
    np.testing.assert_array_equal(got, np.array(expect, np.uint8))


def test_gts_reused_index_is_taken_verbatim():
    """A byte naming an earlier vertex lands in the new slot as is: flags
    L,R,L,R with indices 3, 1, 0 give (0,1,2), (2,1,3), (2,3,1), (1,3,0)."""
    got = gts_walk([([L, R, L, R], [3, 1, 0])])
    np.testing.assert_array_equal(got, np.array([(0, 1, 2), (2, 1, 3), (2, 3, 1), (1, 3, 0)], np.uint8))


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5])
def test_gts_equals_reuse_closed_form_exhaustive(T):
    """Every GTS-Reuse stream with T_s <= 5, re-encoded as plain GTS, decodes to
    the closed form of the reuse stream; the index bytes are I[3..T_s+1]."""
    ms = list(all_streams(T))
    desc, bits, reuse, ts = pack(ms)
    g = O.gts_from_reuse(desc, bits, reuse, ts)
    got = O.decode_gts(g)
    expect = np.array([tri for m in ms for tri in defn.decode_meshlet_closed_form(*m)], np.uint8)
    np.testing.assert_array_equal(got, expect)
    # index bytes: the vertex each triangle adds = third vertex of its triple
    np.testing.assert_array_equal(g.index, expect.reshape(len(ms), T, 3)[:, 1:, 2].reshape(-1))


def test_gts_random_long_and_sizes():
    rng = np.random.default_rng(77)
    ms = [random_stream(rng, int(rng.integers(1, 257)), float(rng.uniform(0.1, 0.9))) for _ in range(400)]
    desc, bits, reuse, ts = pack(ms)
    g = O.gts_from_reuse(desc, bits, reuse, ts)
    np.testing.assert_array_equal(O.decode_gts(g), O.decode_arrays(desc, bits, reuse, ts))
    Ts = np.array([len(m[0]) for m in ms])
    # 8 bytes of L/R flags per 64 strip triangles, one index byte per triangle after the first
    assert g.words.size == 8 * int(((Ts + 63) // 64).sum())
    assert g.index.size == int((Ts - 1).sum())
    # payload bits: T_s flags + 8 (T_s - 1) index bits (Fig. "Strip Encoding" (c))
    assert 8 * g.index.size + int(Ts.sum()) == int((9 * Ts - 8).sum())


MESHES = {
    "grid": lambda: meshgen.workload1(),
    "sphere4": lambda: meshgen.sphere(4, meshgen.rng_for(2, 3)),
    "delaunay": lambda: meshgen.delaunay(6000, meshgen.rng_for(4, 3)),
    "patch": lambda: meshgen.sphere_patch(5000, meshgen.rng_for(3, 3)),
}


@pytest.mark.parametrize("caps", [(32, 64), (64, 126), (128, 256)])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_compaction_keeps_exactly_the_input_triangles(name, caps):
    """Compacted output: one triple per input triangle (T = T_s - 4 restarts),
    in strip order, and the round trip gives back the mesh with its winding."""
    m = MESHES[name]()
    s = O.encode(m.tri, m.nverts, *caps)
    full = O.decode(s)
    kept, offs = O.compact(full, s.desc)
    assert kept.shape[0] == m.ntri == s.strip_triangles - 4 * s.stats["restarts"]
    # the kept triples are the non-degenerate ones, in order
    nondeg = (full[:, 0] != full[:, 1]) & (full[:, 1] != full[:, 2]) & (full[:, 0] != full[:, 2])
    np.testing.assert_array_equal(kept, full[nondeg])
    # per-meshlet offsets: meshlet m's triangles are kept[offs[m]:offs[m+1]]
    _, _, out_off, T, _ = s.fields()
    tri_meshlet = np.repeat(np.arange(s.meshlets), (offs[1:] - offs[:-1]).astype(np.int64))
    base = s.vert_off[:-1].astype(np.int64)[tri_meshlet]
    g = s.verts.astype(np.int64)[base[:, None] + kept.astype(np.int64)]
    np.testing.assert_array_equal(O.canonical(g), O.canonical(m.tri))
    assert offs[-1] == kept.shape[0] and (np.diff(offs.astype(np.int64)) >= 1).all()


def test_compaction_disjoint_triangles_closed_form():
    """k disjoint triangles in one meshlet: the restarts leave exactly the k
    triangles (3i, 3i+1, 3i+2) after compaction."""
    for k in (1, 2, 5, 51):
        f, g, r = [L], [0], []
        for i in range(1, k):
            c_prev, d, e = 3 * i - 1, 3 * i, 3 * i + 1
            f += [L, R, L, R, L]
            g += [0, 1, 0, 1, 1]
            r += [c_prev, d]
            del e
        desc, bits, reuse, ts = pack([(f, g, r)])
        kept, offs = O.compact(O.decode_arrays(desc, bits, reuse, ts), desc)
        np.testing.assert_array_equal(kept, np.array([(3 * i, 3 * i + 1, 3 * i + 2) for i in range(k)], np.uint8))
        assert list(offs) == [0, k]
