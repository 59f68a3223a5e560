"""Encoded meshes saved to a ``.gtsr`` file and loaded back decode on the GPU
to the oracle's bytes for the original streams, in both formats, through the
batched launch and a captured graph (the path a pool encoded once and
reloaded takes)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import meshgen  # noqa: E402
import oracle as O  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2404_06359_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)


def _meshes():
    return [(meshgen.workload1(), (64, 126)), (meshgen.fan(300), (64, 126)),
            (meshgen.delaunay(6000, meshgen.rng_for(4, 17)), (128, 256)),
            (meshgen.sphere_patch(20000, meshgen.rng_for(3, 17)), (32, 64)), (meshgen.disjoint(50), (32, 64))]


@pytest.mark.parametrize("fmt", ["reuse", "gts"])
def test_saved_pool_decodes_to_the_oracle(tmp_path, fmt):
    encs = [P.encode(m.tri, m.nverts, *caps) for m, caps in _meshes()]
    if fmt == "gts":
        encs = [P.gts_from_reuse(e) for e in encs]
        refs = [O.decode_gts(O.GtsStream(e.desc_bytes, e.bits, e.reuse, e.strip_triangles)) for e in encs]
    else:
        refs = [O.decode_arrays(e.desc_bytes, e.bits, e.reuse, e.strip_triangles) for e in encs]
    path = str(tmp_path / f"pool_{fmt}.gtsr")
    P.save(path, encs)
    back = P.load(path)
    assert [e.format for e in back] == [e.format for e in encs]
    pool = P.Pool(back)
    for rep, fill in enumerate((0xAA, 0x55)):
        say(f"[gpu] .gtsr {fmt} pool, batched launch, fill {fill:#x}")
        pool.out.fill_(fill)
        pool.decode_batched()
        torch.cuda.synchronize()
        for i, ref in enumerate(refs):
            np.testing.assert_array_equal(pool.output(i).cpu().numpy(), ref)
    g = pool.batched_graph()
    for rep in range(3):
        say(f"[gpu] .gtsr {fmt} pool, graph replay {rep}")
        pool.out.fill_(0x55 if rep % 2 else 0xAA)
        torch.cuda.synchronize()
        g()
        torch.cuda.synchronize()
        for i, ref in enumerate(refs):
            np.testing.assert_array_equal(pool.output(i).cpu().numpy(), ref)
