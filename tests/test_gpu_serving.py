"""GPU: the decode-request server.  Each request's output is the same byte for
byte whether the mesh is decoded alone or among many concurrent requests
under a tight output budget, and equals the oracle's decode of its stream."""
import sys
import time

import numpy as np
import pytest

import meshgen
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2404_06359_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pool():
    meshes = []
    for i in range(10):
        r = meshgen.rng_for(5, 500 + i)
        n = meshgen.loguniform_int(r, 300, 80000)
        m = meshgen.grid_for(n, r) if i % 2 else meshgen.sphere_patch(n, r)
        meshes.append((m, meshgen.CAPS[i % 3]))
    meshes.append((meshgen.delaunay(30000, meshgen.rng_for(4, 77)), (64, 126)))
    meshes.append((meshgen.fan(1), (3, 1)))
    encs = [P.encode(m.tri, m.nverts, *caps) for m, caps in meshes]
    refs = [O.decode_arrays(e.desc_bytes, e.bits, e.reuse, e.strip_triangles) for e in encs]
    return P.Pool(encs, out=False), refs


def drain(srv, expect, keep=True, timeout_s=30.0):
    """Poll until `expect` requests finished; returns {tag: host output}."""
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < expect:
        assert time.time() < t_end, f"only {len(got)} of {expect} requests finished"
        for c in srv.poll(timeout_us=1000):
            assert c["status"] == 0, c
            assert c["t_submit_ns"] <= c["t_admit_ns"] <= c["t_done_ns"]
            got[int(c["tag"])] = srv.output(c).cpu().numpy().copy() if keep else None
            srv.release(int(c["tag"]))
    return got


def test_alone_equals_mix_equals_oracle(pool):
    pool_, refs = pool
    largest = max(r.nbytes for r in refs)
    # room for about two of the largest outputs: admission has to wait for releases
    srv = P.Server(pool_, arena_bytes=2 * largest + 4096, max_inflight=3, max_batch=4, target_tris=512)
    alone = {}
    for i in range(len(refs)):
        say(f"[gpu] serving alone: mesh {i}")
        srv.submit(i, 1000 + i)
        out = drain(srv, 1)
        alone[i] = out[1000 + i]
        np.testing.assert_array_equal(alone[i], refs[i])
    rng = np.random.default_rng(11)
    order = rng.permutation(np.repeat(np.arange(len(refs)), 5))
    say(f"[gpu] serving mix: {order.size} requests")
    got = {}
    pending = list(enumerate(order))
    # submit in bursts while earlier requests are still decoding
    while pending or len(got) < order.size:
        for _ in range(min(7, len(pending))):
            tag, mesh = pending.pop(0)
            srv.submit(int(mesh), tag)
        got.update(drain(srv, 1))
    for tag, mesh in enumerate(order):
        assert np.array_equal(got[tag], alone[int(mesh)]), f"request {tag} (mesh {mesh}) differs from alone"
    st = srv.stats()
    say(f"[gpu] serving stats {st}")
    assert st["completed"] == st["submitted"] == len(refs) + order.size
    assert st["max_batch_seen"] > 1
    assert st["max_arena_used"] <= 2 * largest + 4096
    assert st["arena_used"] == 0 and st["pending"] == 0
    srv.close()


def test_replay_poisson_trace(pool):
    pool_, refs = pool
    srv = P.Server(pool_, arena_bytes=64 << 20)
    rng = np.random.default_rng(5)
    n = 400
    arrivals = np.cumsum(rng.exponential(100e3, n)).astype(np.uint64)   # 10k requests/s
    meshes = rng.integers(0, len(refs), n).astype(np.uint32)
    say(f"[gpu] replay {n} requests")
    comp, start = srv.replay(arrivals, meshes)
    assert (comp["status"] == 0).all()
    assert np.array_equal(comp["tag"], np.arange(n))
    assert np.array_equal(comp["mesh"], meshes)
    assert (comp["t_submit_ns"] >= start + arrivals).all()
    lat = (comp["t_done_ns"] - comp["t_submit_ns"]) / 1e3
    say(f"[gpu] replay latency p50 {np.percentile(lat, 50):.1f} us, p99 {np.percentile(lat, 99):.1f} us")
    assert srv.stats()["arena_used"] == 0
    srv.close()


def test_server_errors(pool):
    pool_, refs = pool
    small = min(r.nbytes for r in refs if r.nbytes > 0)
    srv = P.Server(pool_, arena_bytes=small + 256, max_inflight=1)
    big = int(np.argmax([r.nbytes for r in refs]))
    with pytest.raises(P.GtsrError) as e:
        srv.submit(big, 1)
    assert e.value.code == P.ELIMIT
    with pytest.raises(P.GtsrError) as e:
        srv.submit(len(refs), 2)
    assert e.value.code == P.EINVAL
    with pytest.raises(P.GtsrError) as e:
        srv.release(12345)
    assert e.value.code == P.EINVAL
    i = int(np.argmin([r.nbytes if r.nbytes else 1 << 60 for r in refs]))
    srv.submit(i, 7)
    with pytest.raises(P.GtsrError) as e:
        srv.submit(i, 7)
    assert e.value.code == P.EINVAL
    out = drain(srv, 1)
    np.testing.assert_array_equal(out[7], refs[i])
    srv.close()


def test_server_arena_units(pool):
    """An output takes whole 256-byte units of the arena: a mesh whose output
    fits the arena only unrounded is refused at submit, not queued for ever
    (it would block every request behind it)."""
    pool_, refs = pool
    i = len(refs) - 1                    # the one-triangle fan: 3 output bytes
    assert refs[i].nbytes == 3
    srv = P.Server(pool_, arena_bytes=255, max_inflight=1)
    with pytest.raises(P.GtsrError) as e:
        srv.submit(i, 1)
    assert e.value.code == P.ELIMIT
    srv.close()
    srv = P.Server(pool_, arena_bytes=256, max_inflight=1)
    srv.submit(i, 1)
    out = drain(srv, 1)
    np.testing.assert_array_equal(out[1], refs[i])
    srv.close()


def test_cancel_unblocks_the_queue(pool):
    """A request that does not fit blocks the ones behind it until it is
    withdrawn: cancelling it lets the next request through, reports it with
    ECANCELED, and a request already admitted cannot be withdrawn."""
    pool_, refs = pool
    big = int(np.argmax([r.nbytes for r in refs]))
    small = int(np.argmin([r.nbytes if r.nbytes else 1 << 60 for r in refs]))
    span = lambda n: max(256, (n + 255) // 256 * 256)
    srv = P.Server(pool_, arena_bytes=span(refs[big].nbytes) + span(refs[small].nbytes), max_inflight=2)
    srv.submit(big, 1)
    first = []
    t_end = time.time() + 30
    while not first:
        assert time.time() < t_end
        first = list(srv.poll(timeout_us=1000))
    assert int(first[0]["tag"]) == 1 and first[0]["status"] == 0
    np.testing.assert_array_equal(srv.output(first[0]).cpu().numpy(), refs[big])
    srv.submit(big, 2)      # cannot fit while request 1 holds its range
    srv.submit(small, 3)    # would fit, but waits behind request 2
    assert len(srv.poll(timeout_us=20000)) == 0
    assert srv.stats()["pending"] == 2
    assert srv.cancel(1) is False           # admitted (finished, unreleased)
    assert srv.cancel(2) is True
    with pytest.raises(P.GtsrError) as e:
        srv.cancel(2)
    assert e.value.code == P.EINVAL
    got = {}
    t_end = time.time() + 30
    while len(got) < 2:
        assert time.time() < t_end
        for c in srv.poll(timeout_us=1000):
            got[int(c["tag"])] = c
            if c["status"] == 0:
                np.testing.assert_array_equal(srv.output(c).cpu().numpy(), refs[small])
    assert got[2]["status"] == P.ECANCELED and got[2]["out_bytes"] == 0
    assert got[3]["status"] == 0
    for t in (1, 3):
        srv.release(t)
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 2 and st["failed"] == 0 and st["arena_used"] == 0
    srv.close()
