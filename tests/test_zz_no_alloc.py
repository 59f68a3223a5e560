"""GPU: gtsr_decode_batched_noalloc, the batched decode whose claim counters
live in the library's static device array, equals decode_meshlets_batched
(caller workspace) byte for byte, on two calls in a row, the second with a
smaller input (the array keeps the first call's counts; the call must clear
them)."""
import ctypes as C
import sys

import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2404_06359_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pool(count, seed, fmt):
    encs = []
    for i in range(count):
        r = meshgen.rng_for(7, seed + i)
        n = meshgen.loguniform_int(r, 300, 40000)
        m = meshgen.grid_for(n, r) if i % 2 else meshgen.sphere_patch(n, r)
        e = P.encode(m.tri, m.nverts, *meshgen.CAPS[i % 3])
        encs.append(P.gts_from_reuse(e) if fmt == P.FORMAT_GTS else e)
    return P.Pool(encs)


def _noalloc(pool, cfg):
    P._check(P.lib().gtsr_decode_batched_noalloc(pool.table.data_ptr(), pool.mesh_count, pool.work.data_ptr(),
                                                 pool.work_items, pool.format, P._cfg(cfg), P._stream_handle(None)))


@pytest.mark.parametrize("fmt", [P.FORMAT_REUSE, P.FORMAT_GTS])
def test_noalloc_equals_workspace_entry_point_twice(fmt):
    big, small = _pool(16, 100, fmt), _pool(5, 300, fmt)
    for pool, label in ((big, "first, larger"), (small, "second, smaller")):
        for cfg in (None, {"items_per_claim": 1, "groups_per_cu": 8}, {"items_per_claim": 4, "waves_per_group": 2}):
            pool.plan(300)
            n_out = int(pool.out_offsets[-1])
            say(f"[gpu] noalloc {label} format={fmt} cfg={cfg} items={pool.work_items}")
            pool.out.fill_(0xAA)
            ws_cfg = dict(cfg or {})
            ws_cfg.setdefault("items_per_claim", 2)
            pool.decode_batched(cfg=ws_cfg)
            torch.cuda.synchronize()
            ref = pool.out[:n_out].clone()
            pool.out.fill_(0x55)
            _noalloc(pool, cfg)
            torch.cuda.synchronize()
            assert torch.equal(pool.out[:n_out], ref)
            # and the workspace entry point's claiming output equals its static split
            pool.out.fill_(0x55)
            pool.decode_batched()
            torch.cuda.synchronize()
            assert torch.equal(pool.out[:n_out], ref)
