"""Pins for the oracle (CPU only).

The oracle decoder is the sequential strip walk (``oracle.c``).  It is checked
here against things other than itself:

* the data-parallel closed form of Sec. 4.2 / 4.3 (``oracle/defn.py``: flip
  search for the pivot, prefix count of increments, reuse read at t+1-s),
  exhaustively on every stream with T_s <= 6 and on random long streams;
* triples worked out by hand from the definitions (``golden/handworked_streams.txt``);
* the textbook triangle strip and triangle fan (consecutive-index triangles,
  alternating winding; hub-vertex triangles), which are special cases of a
  generalized strip (Sec. 2);
* encode -> decode round trips that must reproduce every input triangle with
  its winding, on generated meshes and on every small connected subset of a
  grid patch;
* exact counting invariants (four degenerates per restart, Table 1; bits per
  triangle accounting, Table 2).
"""
import itertools
import os

import numpy as np
import pytest

import meshgen
import oracle as O
from oracle import defn
from streams import L, R, all_streams, pack, random_stream


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()
    O._lib = None
    O.lib()


def walk(meshlets):
    desc, bits, reuse, ts = pack(meshlets)
    return O.decode_arrays(desc, bits, reuse, ts)


def closed(meshlets):
    out = []
    for f, g, r in meshlets:
        out.extend(defn.decode_meshlet_closed_form(f, g, r))
    return np.array(out, np.uint8).reshape(-1, 3)


# ----------------------------------------------------------- closed form pins

@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6])
def test_walk_equals_closed_form_exhaustive(T):
    ms = list(all_streams(T))
    assert len(ms) > 0
    np.testing.assert_array_equal(walk(ms), closed(ms))


def test_walk_equals_closed_form_random_long():
    rng = np.random.default_rng(7)
    ms = []
    for T in list(range(6, 70)) + [127, 128, 129, 191, 192, 193, 255, 256] * 4:
        for p in (0.1, 0.5, 0.9):
            ms.append(random_stream(rng, T, p_inc=0.55, p_r=p))
    np.testing.assert_array_equal(walk(ms), closed(ms))


def test_stream_count_exhaustive_small():
    # T_s = 1: two flag values, no increments, no reuse.
    assert len(list(all_streams(1))) == 2
    # T_s = 2: 4 flag words x (inc: 1 stream, reuse: 3 choices of 0..2) = 16.
    assert len(list(all_streams(2))) == 16


def _read_handworked(golden_dir):
    cases = []
    with open(os.path.join(golden_dir, "handworked_streams.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, flags, incs, reuse, tris = [x.strip() for x in line.split("|")]
            f = [R if c == "R" else L for c in flags]
            g = [0] + ([int(c) for c in incs] if incs != "-" else [])
            r = [int(x) for x in reuse.split()] if reuse != "-" else []
            t = [tuple(int(x) for x in tri.split()) for tri in tris.split(",")]
            cases.append((name, (f, g, r), t))
    return cases


def test_handworked_fixtures(golden_dir):
    cases = _read_handworked(golden_dir)
    assert len(cases) >= 8
    for name, m, expect in cases:
        got = [tuple(int(v) for v in row) for row in walk([m])]
        assert got == expect, name
        assert defn.decode_meshlet_closed_form(*m) == expect, name


@pytest.mark.parametrize("T", [1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200, 254])
def test_textbook_strip(T):
    """Alternating flags L,R,L,R,... with only new vertices: triangle t is made
    of the three consecutive indices t, t+1, t+2, with the winding flipped on
    every odd triangle (the classic triangle strip, Sec. 2)."""
    f = [L if t % 2 == 0 else R for t in range(T)]
    g = [0] + [1] * (T - 1)
    got = walk([(f, g, [])])
    expect = [(t, t + 1, t + 2) if t % 2 == 0 else (t + 1, t, t + 2) for t in range(T)]
    np.testing.assert_array_equal(got, np.array(expect, np.uint8))


@pytest.mark.parametrize("T", [1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200, 254])
def test_textbook_fan(T):
    """Constant L flags: every triangle shares hub vertex 0, (0, t+1, t+2);
    constant R: the mirrored fan (t+1, 0, t+2); R then L...: hub vertex 1."""
    g = [0] + [1] * (T - 1)
    np.testing.assert_array_equal(walk([([L] * T, g, [])]),
                                  np.array([(0, t + 1, t + 2) for t in range(T)], np.uint8))
    np.testing.assert_array_equal(walk([([R] * T, g, [])]),
                                  np.array([(t + 1, 0, t + 2) for t in range(T)], np.uint8))
    got = walk([([R] + [L] * (T - 1), g, [])])
    expect = [(1, 0, 2)] + [(1, t + 1, t + 2) for t in range(1, T)]
    np.testing.assert_array_equal(got, np.array(expect, np.uint8))


def test_restart_pattern_disjoint_triangles():
    """k disjoint triangles in one meshlet: after each, four degenerates
    (slots c, d, d, e with flags L,R,L,R, then f with L) start the next one
    (Sec. 4.2).  Expect T_s = 5k-4, V = 3k, 2(k-1) reuse bytes, and after
    dropping degenerates exactly the k triangles (3i, 3i+1, 3i+2)."""
    for k in (1, 2, 3, 17, 51):
        f, g, r = [L], [0], []
        for i in range(1, k):
            c_prev, d, e = 3 * i - 1, 3 * i, 3 * i + 1
            f += [L, R, L, R, L]
            g += [0, 1, 0, 1, 1]
            r += [c_prev, d]
        assert len(f) == 5 * k - 4 and 3 + sum(g[1:]) == 3 * k and len(r) == 2 * (k - 1)
        out = walk([(f, g, r)])
        keep = [tuple(int(x) for x in t) for t in out if len(set(t.tolist())) == 3]
        assert keep == [(3 * i, 3 * i + 1, 3 * i + 2) for i in range(k)]
        assert len(out) - len(keep) == 4 * (k - 1)


# --------------------------------------------- the pins catch planted mistakes

def _mutant(kind):
    def dec(f, g, r):
        T = len(f)
        I = [0, 1, 2] + [None] * (T - 1)
        for t in range(1, T):
            s = 2 + sum(g[1:t + 1])
            if kind == "scan_offset":
                s = 1 + sum(g[1:t + 1])
            if g[t]:
                I[t + 2] = s
            else:
                idx = t - s if kind == "reuse_index" else t + 1 - s
                I[t + 2] = r[idx] if 0 <= idx < len(r) else 0
        out = []
        for t in range(T):
            k = -1
            for q in range(t - 1, -1, -1):
                if (f[q] == f[t]) if kind == "flip_sign" else (f[q] != f[t]):
                    k = q
                    break
            X = I[k] if kind == "pivot_index" and k >= 0 else I[k + 1]
            if (f[t] == L) != (kind == "orientation"):
                out.append((X, I[t + 1], I[t + 2]))
            else:
                out.append((I[t + 1], X, I[t + 2]))
        return out
    return dec


@pytest.mark.parametrize("kind", ["scan_offset", "reuse_index", "flip_sign", "pivot_index",
                                  "orientation"])
def test_planted_mistakes_are_caught(kind):
    """A closed form with one plausible mistake must disagree with the walk on
    the exhaustive T_s <= 4 set (so the comparison above has teeth)."""
    ms = [m for T in (1, 2, 3, 4) for m in all_streams(T)]
    ref = walk(ms)
    dec = _mutant(kind)
    got = np.array([x for m in ms for x in dec(*m)], np.uint8).reshape(-1, 3)
    assert not np.array_equal(got, ref)


# ------------------------------------------------------------------- encoder

def _roundtrip(mesh, maxv, maxt):
    s = O.encode(mesh.tri, mesh.nverts, maxv, maxt)
    d = O.decode(s)
    np.testing.assert_array_equal(O.round_trip_triangles(s, d), O.canonical(mesh.tri))
    return s, d


def _invariants(s, d, maxv, maxt):
    M = s.meshlets
    chunk_off, reuse_off, out_off, T, V = s.fields()
    assert O.check_stream(s.desc, s.bits, s.reuse, s.strip_triangles) == 0
    assert np.all(T <= maxt) and np.all(V <= maxv) and np.all(V >= 3)
    # every meshlet opens with the implicit (0,1,2) (Sec. 4.3)
    np.testing.assert_array_equal(d[out_off], np.tile([0, 1, 2], (M, 1)))
    # degenerate triples are exactly four per restart (Sec. 4.2, Table 1)
    degen = ((d[:, 0] == d[:, 1]) | (d[:, 1] == d[:, 2]) | (d[:, 0] == d[:, 2])).sum()
    assert degen == 4 * s.stats["restarts"]
    assert s.strip_triangles == s.stats["input_triangles"] + 4 * s.stats["restarts"]
    # increments introduce every vertex once, in order: the largest local id
    # in each meshlet is V-1 and V = 3 + (number of increment bits)
    bits = s.bits.reshape(-1, 16)
    inc_pop = np.array([bin(int.from_bytes(b[8:].tobytes(), "little")).count("1") for b in bits])
    pop_per_meshlet = np.add.reduceat(inc_pop, chunk_off) if M else np.zeros(0)
    np.testing.assert_array_equal(pop_per_meshlet, V - 3)
    mx = np.maximum.reduceat(d.max(axis=1), out_off) if M else np.zeros(0)
    np.testing.assert_array_equal(mx, V - 1)
    # bits per triangle: counted from the arrays, from the formula, from stats
    n_ru = T - V + 2
    assert n_ru.sum() == s.reuse.size == s.stats["reuse_count"]
    payload = int((T + (T - 1) + 8 * n_ru).sum())
    assert payload == int((10 * T - 8 * V + 15).sum()) == s.stats["payload_bits"]
    assert s.stats["stored_bytes"] == int((16 + 16 * ((T + 63) // 64) + n_ru).sum())
    assert s.bits.size == 16 * int(((T + 63) // 64).sum())


def _reuse_address_pin(s):
    """Sec. 4.3: at a reuse slot t the reuse array is read at t + 1 - s_t with
    s_t the inclusive increment scan plus 2; it must equal the number of reuse
    slots before t, i.e. reuse bytes are consumed in order."""
    chunk_off, reuse_off, out_off, T, V = s.fields()
    for m in range(min(s.meshlets, 300)):
        lr = [int.from_bytes(s.bits[16 * c: 16 * c + 8].tobytes(), "little")
              for c in range(chunk_off[m], chunk_off[m] + (T[m] + 63) // 64)]
        inc = [int.from_bytes(s.bits[16 * c + 8: 16 * c + 16].tobytes(), "little")
               for c in range(chunk_off[m], chunk_off[m] + (T[m] + 63) // 64)]
        del lr
        s_t, n_prev = 2, 0
        for t in range(1, T[m]):
            g = (inc[t // 64] >> (t % 64)) & 1
            s_t += g
            if not g:
                assert t + 1 - s_t == n_prev
                n_prev += 1
        assert n_prev == T[m] - V[m] + 2


MESHES = {
    "grid64": lambda: meshgen.workload1(),
    "sphere4": lambda: meshgen.sphere(4, meshgen.rng_for(2, 99)),
    "patch": lambda: meshgen.sphere_patch(5000, meshgen.rng_for(3, 5)),
    "delaunay": lambda: meshgen.delaunay(6000, meshgen.rng_for(4, 3)),
    "fan300": lambda: meshgen.fan(300),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("caps", [(32, 64), (64, 126), (128, 256), (256, 256), (3, 1), (8, 7)])
def test_encode_roundtrip_and_invariants(name, caps):
    mesh = MESHES[name]()
    s, d = _roundtrip(mesh, *caps)
    _invariants(s, d, *caps)
    _reuse_address_pin(s)
    # the closed form agrees with the walk on real encoder output too
    if s.strip_triangles <= 20000:
        cf = defn.decode_closed_form(s.desc.tobytes(), s.bits.tobytes(), s.reuse.tobytes())
        np.testing.assert_array_equal(np.array(cf, np.uint8).reshape(-1, 3), d)


@pytest.mark.parametrize("k", [31, 32, 33, 63, 64, 65, 127, 128, 200, 254])
def test_encoder_fan_crosses_words(k):
    """A fan of k triangles becomes one strip with no restart; every decoded
    triangle holds the hub; lengths straddle 32- and 64-bit flag words
    (Sec. 4.2 notes fans longer than one flag word)."""
    mesh = meshgen.fan(k)
    s, d = _roundtrip(mesh, 256, 256)
    assert s.meshlets == 1 and s.stats["restarts"] == 0 and s.strip_triangles == k
    hub_local = int(np.where(s.verts == 0)[0][0])
    assert np.all((d == hub_local).any(axis=1))


def test_single_triangle_payload():
    """One triangle: T_s = 1, V = 3, no reuse, payload 1 bit (its L/R flag):
    10*1 - 8*3 + 15 = 1."""
    s = O.encode(np.array([[4, 9, 2]], np.uint32), 10, 64, 126)
    assert s.meshlets == 1 and s.strip_triangles == 1 and s.reuse.size == 0
    assert s.stats["payload_bits"] == 1
    np.testing.assert_array_equal(O.decode(s), [[0, 1, 2]])
    np.testing.assert_array_equal(s.verts, [4, 9, 2])


def test_empty_mesh():
    s = O.encode(np.zeros((0, 3), np.uint32), 0, 64, 126)
    assert s.meshlets == 0 and s.strip_triangles == 0


def _connected_subsets(adj, max_size):
    n = len(adj)
    seen = set()
    out = []

    def extend(cur, frontier):
        key = frozenset(cur)
        if key in seen:
            return
        seen.add(key)
        out.append(sorted(cur))
        if len(cur) == max_size:
            return
        for x in sorted(frontier):
            nf = (frontier | adj[x]) - cur - {x}
            extend(cur | {x}, nf)

    for s in range(n):
        extend({s}, set(adj[s]))
    return out


def test_brute_force_small_subsets():
    """Every connected subset of <= 6 triangles of a 3x3 quad patch, under a
    random vertex relabelling and several caps, round-trips."""
    base = meshgen.grid(3, 3, meshgen.rng_for(1, 123), permute=False)
    tri = base.tri.astype(np.int64)
    adj = [set() for _ in range(len(tri))]
    edges = {}
    for t, (a, b, c) in enumerate(tri):
        for u, v in ((a, b), (b, c), (c, a)):
            edges.setdefault((min(u, v), max(u, v)), []).append(t)
    for ts in edges.values():
        if len(ts) == 2:
            adj[ts[0]].add(ts[1])
            adj[ts[1]].add(ts[0])
    subsets = _connected_subsets(adj, 6)
    assert len(subsets) > 400   # 439 for this patch (every connected subset of its 18 triangles)
    rng = np.random.default_rng(11)
    for sub in subsets:
        t = tri[sub]
        perm = rng.permutation(base.nverts)
        t = perm[t]
        # triangle order and starting corner shuffled too
        t = t[rng.permutation(len(t))]
        rot = rng.integers(0, 3, len(t))
        t = np.array([np.roll(x, -k) for x, k in zip(t, rot)], np.uint32)
        mesh = meshgen.Mesh(t, base.nverts)
        for caps in ((256, 256), (4, 2), (6, 6)):
            _roundtrip(mesh, *caps)


def test_non_manifold_and_flipped_edges_roundtrip():
    """Edges used by three triangles or twice in the same direction are not
    crossed by strips or meshlet growth; the round trip still holds."""
    tri = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4],      # edge (0,1) used 3 times
                    [2, 1, 5], [1, 2, 6],                  # (1,2) used forward twice... and (2,1)
                    [5, 6, 7], [6, 5, 8]], np.uint32)
    _roundtrip(meshgen.Mesh(tri, 9), 64, 126)


def test_encode_errors():
    assert_code = lambda rc, *a: pytest.raises(O.OracleError, O.encode, *a)
    with pytest.raises(O.OracleError) as e:
        O.encode(np.array([[0, 1, 1]], np.uint32), 3, 64, 126)
    assert e.value.code == O.EDEGENERATE
    with pytest.raises(O.OracleError) as e:
        O.encode(np.array([[0, 1, 5]], np.uint32), 3, 64, 126)
    assert e.value.code == O.EINVAL
    for caps in ((2, 126), (257, 126), (64, 0), (64, 257)):
        with pytest.raises(O.OracleError) as e:
            O.encode(np.array([[0, 1, 2]], np.uint32), 3, *caps)
        assert e.value.code == O.ELIMIT
    del assert_code


def test_check_stream_rejects_corruption():
    mesh = meshgen.workload1()
    s = O.encode(mesh.tri, mesh.nverts, 64, 126)
    ok = (s.desc, s.bits, s.reuse, s.strip_triangles)
    assert O.check_stream(*ok) == 0

    def bad(desc=None, bits=None, reuse=None, ts=None):
        return O.check_stream(s.desc if desc is None else desc, s.bits if bits is None else bits,
                              s.reuse if reuse is None else reuse,
                              s.strip_triangles if ts is None else ts)

    d = s.desc.copy(); d[12:14] = [0, 0]                       # T_s = 0
    assert bad(desc=d) == O.ECORRUPT
    d = s.desc.copy(); d[16 + 8] ^= 1                           # out_off not contiguous
    assert bad(desc=d) == O.ECORRUPT
    d = s.desc.copy(); d[14] = 2; d[15] = 0                     # V = 2
    assert bad(desc=d) == O.ECORRUPT
    b = s.bits.copy(); b[8] |= 1                                # INC bit of triangle 0
    assert bad(bits=b) == O.ECORRUPT
    _, _, _, T, _ = s.fields()
    last_chunk = s.bits.size // 16 - 1
    t_last = int(T[-1]) % 64
    if t_last:
        b = s.bits.copy(); b[16 * last_chunk + 7] |= 0x80       # LR bit past T_s
        assert bad(bits=b) == O.ECORRUPT
    r = s.reuse.copy(); r[0] = 255                              # reuse of a vertex not yet introduced
    assert bad(reuse=r) == O.ECORRUPT
    assert bad(reuse=s.reuse[:-1]) == O.ECORRUPT                # truncated reuse
    assert bad(ts=s.strip_triangles + 1) == O.ECORRUPT
    b = s.bits.copy(); b[8] ^= 2                                # flip one increment bit
    assert bad(bits=b) == O.ECORRUPT


def test_check_stream_reuse_rule_exhaustive():
    """Every one-meshlet stream with T_s <= 4, every flag and increment word,
    reuse bytes 0..6: the checker accepts exactly the streams whose reuse
    bytes each name a vertex already introduced (Sec. 4.3: a clear increment
    flag takes the next reuse entry, an index of a vertex seen before), that
    is, a value below 3 plus the increments before its slot."""
    import itertools

    checked = accepted = 0
    for T in range(1, 5):
        for f in itertools.product((L, R), repeat=T):
            for gt in itertools.product((0, 1), repeat=T - 1):
                g = (0,) + gt
                seen, limits = 3, []
                for t in range(1, T):
                    if g[t]:
                        seen += 1
                    else:
                        limits.append(seen)
                for r in itertools.product(range(7), repeat=len(limits)):
                    valid = all(x < n for x, n in zip(r, limits))
                    desc, bits, reuse, ts = pack([(list(f), list(g), list(r))])
                    assert (O.check_stream(desc, bits, reuse, ts) == 0) == valid, (f, g, r)
                    checked += 1
                    accepted += valid
    assert checked == 8738 and 0 < accepted < checked


# ---------------------------------------------------------------- paper values

def _rows(path):
    out = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            out.append(line.split())
    return out


def test_table1_four_degenerates_per_restart(golden_dir):
    rows = _rows(os.path.join(golden_dir, "table1_restarts.txt"))
    assert len(rows) == 3
    for name, restarts, degen, meshlets, extra in rows:
        assert int(degen) == 4 * int(restarts), name
    # the same rule holds for the oracle encoder's output
    mesh = meshgen.sphere(5, meshgen.rng_for(2, 5))
    s, d = _roundtrip(mesh, 128, 256)
    degen = ((d[:, 0] == d[:, 1]) | (d[:, 1] == d[:, 2]) | (d[:, 0] == d[:, 2])).sum()
    assert degen == 4 * s.stats["restarts"] > 0


def test_table2_bits_per_triangle_denominator(golden_dir):
    """With T taken from the 96-bpt vertex-pipeline column, the basic column
    is 24 bpt and the GTS / GTS-Reuse columns reproduce their printed bpt to
    the printed precision: bpt is counted per input triangle."""
    rows = _rows(os.path.join(golden_dir, "table2_index_buffer.txt"))
    assert len(rows) == 6
    mib = 2 ** 20 * 8
    for name, vm, vb, bm, bb, gm, gb, rm, rb in rows:
        T = float(vm) * mib / 96.0
        assert abs(float(bm) * mib / T - 24.0) < 0.15, name
        assert abs(float(gm) * mib / T - float(gb)) < 0.06, name
        assert abs(float(rm) * mib / T - float(rb)) < 0.06, name
        # 4:1, ~10:1, ~16:1 compression versus the vertex pipeline
        assert abs(float(vm) / float(bm) - 4.0) < 0.05, name


def test_teaser_ladder(golden_dir):
    rows = {r[0]: r for r in _rows(os.path.join(golden_dir, "teaser_bpt.txt"))}
    assert float(rows["vertex"][1]) == int(rows["vertex"][2]) * int(rows["vertex"][3]) == 96
    assert float(rows["basic"][1]) == int(rows["basic"][2]) * int(rows["basic"][3]) == 24
    # the decode output is the basic layout: 3 bytes per strip triangle
    mesh = meshgen.workload1()
    s = O.encode(mesh.tri, mesh.nverts, 64, 126)
    assert O.decode(s).nbytes * 8 == 24 * s.strip_triangles
    # the payload stays well under the basic layout (compression happens)
    assert s.stats["payload_bits"] / mesh.ntri < 8.0
