"""GPU parity at the benchmark's full sizes.

* The batched workload (2000 meshes, 526M input triangles, mixed caps):
  decoded by one graph launch in the shape the benchmark times (autotuned),
  by the untuned default launch, by a persistent claiming launch and by one
  plain launch per mesh; every
  output byte equals the oracle's decode of the same stream.
* The same meshes as plain GTS streams, tuned and replayed from a graph.
* The serving pool (5000 meshes, 12.8G triangles, 13.8 GB of streams) under
  the 64 GB budget with the benchmark's server settings: a burst of requests
  decoded together equals the oracle, and a sample of them equals its own
  decode as a lone request.
"""
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import meshgen
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import bench  # noqa: E402
import paper_2404_06359_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_decodes(encs, threads):
    """The oracle's decode of each stream (the C decoder runs outside the GIL)."""
    refs = [None] * len(encs)

    def one(i):
        e = encs[i]
        refs[i] = O.decode_arrays(e.desc_bytes, e.bits, e.reuse, e.strip_triangles)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(len(encs))))
    return refs


@pytest.fixture(scope="module")
def batched():
    threads = bench.host_threads()
    say(f"[gpu] full size: encoding the 2000-mesh batched workload on {threads} threads")
    encs = bench.build_batched(2000, threads)
    refs = oracle_decodes(encs, threads)
    say(f"[gpu] full size: {sum(e.stats['input_triangles'] for e in encs)} input triangles, "
        f"{sum(e.strip_triangles for e in encs)} strip triangles, oracle decoded")
    return encs, refs


def assert_pool_output(pool, refs, what):
    torch.cuda.synchronize()
    got = pool.out.cpu().numpy()
    for i, ref in enumerate(refs):
        a, b = int(pool.out_offsets[i]), int(pool.out_offsets[i + 1])
        mine = got[a:b].reshape(-1, 3)
        if not np.array_equal(mine, ref):
            bad = np.nonzero((mine != ref).any(axis=1))[0] if mine.shape == ref.shape else np.arange(1)
            pytest.fail(f"{what}: mesh {i}: {bad.size} triangles differ, first {bad[:5]}")


@pytest.mark.timeout(900)
def test_batched_workload_full_size(batched):
    encs, refs = batched
    pool = P.Pool(encs)
    pool.plan(768)
    cfg, best, points = pool.autotune()
    say(f"[gpu] full size: autotuned over {len(points)} shapes: {best}")
    g = pool.batched_graph(cfg)
    for fill in (0xAA, 0x55):           # two replays, the output cleared between them
        pool.out.fill_(fill)
        g()
        assert_pool_output(pool, refs, f"graph replay (fill {fill:#x})")
    g.close()
    say("[gpu] full size: untuned default launch")
    pool.plan(768)
    pool.out.fill_(0xAA)
    pool.decode_batched()
    assert_pool_output(pool, refs, "default batched launch")
    say("[gpu] full size: persistent grid claiming 4 items at a time")
    pool.out.fill_(0x55)
    pool.decode_batched(cfg={"waves_per_group": 1, "groups_per_cu": 32, "items_per_claim": 4})
    assert_pool_output(pool, refs, "claiming launch")
    say("[gpu] full size: one plain launch per mesh")
    pool.out.fill_(0x55)
    pool.decode_per_mesh()
    assert_pool_output(pool, refs, "per-mesh launches")


@pytest.mark.timeout(900)
def test_plain_gts_batched_full_size(batched):
    """The same 2000 meshes as plain GTS streams (library conversion), tuned
    and replayed from a captured graph: every triple equals the oracle's
    decode of the original GTS-Reuse stream (same strips, same flags)."""
    encs, refs = batched
    say("[gpu] full size: plain GTS conversion of the batched workload")
    gts = [P.gts_from_reuse(e) for e in encs]
    pool = P.Pool(gts)
    assert pool.format == P.FORMAT_GTS
    cfg, best, points = pool.autotune(mode="search", cache=None)
    say(f"[gpu] full size: plain GTS autotuned over {len(points)} shapes: {best}")
    g = pool.batched_graph(cfg)
    for fill in (0xAA, 0x55):
        pool.out.fill_(fill)
        g()
        assert_pool_output(pool, refs, f"plain GTS graph replay (fill {fill:#x})")
    g.close()


@pytest.mark.timeout(900)
def test_serving_full_pool():
    threads = bench.host_threads()
    say(f"[gpu] serving pool: encoding 96 prototypes on {threads} threads")
    protos = bench.build_serve_prototypes(threads)
    entries = meshgen.workload5_entries(5000)
    pool = P.Pool([protos[int(k)] for k in entries], out=False)
    pool_bytes = int(pool.d_meshlets.numel() + pool.d_bits.numel() + pool.d_reuse.numel())
    say(f"[gpu] serving pool: {pool_bytes / 1e9:.2f} GB of streams on the device")
    assert 10e9 < pool_bytes < 20e9
    srv = P.Server(pool, arena_bytes=int(64e9) - pool_bytes, max_inflight=4, max_batch=256, target_tris=768)
    rng = meshgen.rng_for(6, 4242)
    burst = rng.integers(0, len(entries), 300)
    sample = set(int(t) for t in rng.choice(len(burst), 20, replace=False))
    keys = sorted(set(int(entries[m]) for m in burst))
    refs = dict(zip(keys, oracle_decodes([protos[k] for k in keys], threads)))

    def drain(expect, keep):
        got, done = {}, 0
        t_end = time.time() + 120.0
        while done < expect:
            assert time.time() < t_end, f"only {done} of {expect} requests finished"
            for c in srv.poll(timeout_us=100000):
                assert c["status"] == 0, c
                tag = int(c["tag"])
                out = srv.output(c).cpu().numpy()
                np.testing.assert_array_equal(out, refs[int(entries[burst[tag]])], err_msg=f"request {tag}")
                if tag in keep:
                    got[tag] = out.copy()
                srv.release(tag)
                done += 1
        return got

    say(f"[gpu] serving pool: burst of {burst.size} requests")
    for tag, m in enumerate(burst):
        srv.submit(int(m), tag)
    mixed = drain(burst.size, sample)
    st = srv.stats()
    say(f"[gpu] serving pool: {st}")
    assert st["completed"] == burst.size and st["max_batch_seen"] > 1
    say(f"[gpu] serving pool: {len(sample)} sampled requests alone")
    for tag in sorted(sample):
        srv.submit(int(burst[tag]), tag)
        alone = drain(1, {tag})
        np.testing.assert_array_equal(alone[tag], mixed[tag], err_msg=f"request {tag} alone vs mixed")
    srv.close()
