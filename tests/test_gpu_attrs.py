"""GPU: dequantization of crack-free fixed-point attributes, bit for bit
against the oracle's float64 fused multiply-add, and no cracks."""
import sys

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


def check(m, caps, bits, cfgs=(None,)):
    A = meshgen.vertex_attributes(m)
    enc = P.encode(m.tri, m.nverts, *caps)
    q = P.quantize_attributes(A, enc, bits)
    ref = O.dequantize(O.Quantized(q.origin, q.delta, q.lowest, q.offsets), q.vert_off)
    da = P.attrs_to_device(q)
    for cfg in cfgs:
        say(f"[gpu] dequantize {m.kind} caps={caps} bits={bits} cfg={cfg} elements={ref.size}")
        out = torch.full(ref.shape, float("nan"), dtype=torch.float32, device="cuda")
        P.dequantize(da, out=out, cfg=cfg)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    # every copy of a vertex has the same bits
    order = np.argsort(enc.verts, kind="stable")
    sv = enc.verts[order]
    first = np.r_[True, sv[1:] != sv[:-1]]
    rep = np.maximum.accumulate(np.where(first, np.arange(sv.size), 0))
    bitsv = got.view(np.uint32)[order]
    np.testing.assert_array_equal(bitsv, bitsv[rep])
    return enc, q, ref


@pytest.mark.parametrize("bits", [16, 9])
@pytest.mark.parametrize("caps", [(32, 64), (64, 126), (128, 256)])
@pytest.mark.parametrize("kind", ["sphere", "delaunay"])
def test_dequantize_parity(kind, caps, bits):
    m = meshgen.sphere(5, meshgen.rng_for(2, 11)) if kind == "sphere" else \
        meshgen.delaunay(30000, meshgen.rng_for(4, 11))
    check(m, caps, bits, cfgs=(None, {"waves_per_group": 1, "meshlets_per_wave": 1},
                               {"waves_per_group": 4, "meshlets_per_wave": 64}))


def test_dequantize_short_output_skips_tail():
    m = meshgen.sphere(4, meshgen.rng_for(2, 12))
    A = meshgen.vertex_attributes(m)
    enc = P.encode(m.tri, m.nverts, 64, 126)
    q = P.quantize_attributes(A, enc, 16)
    ref = O.dequantize(O.Quantized(q.origin, q.delta, q.lowest, q.offsets), q.vert_off)
    half = int(q.vert_off[len(q.vert_off) // 2])
    out = torch.full((half + 3, 8), -1.0, dtype=torch.float32, device="cuda")
    P.dequantize(P.attrs_to_device(q), out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[:half], ref[:half])
    assert (got[half:] == -1.0).all()


def test_dequantize_full_size_sphere():
    """The 5.2M-triangle icosphere's eight channels (about 25M elements)."""
    m = meshgen.workload2()
    say(f"[gpu] dequantize full-size sphere: {m.nverts} vertices")
    enc, q, ref = check(m, (64, 126), 16)
    assert ref.shape[0] == int(enc.vert_off[-1])


def test_dequantize_offset_count_bounds_meshlets():
    """Meshlets whose vertex range passes the offsets array's stated length
    are skipped even when the output is large enough (the stated length
    here is shorter than the real array, so every read stays in bounds)."""
    m = meshgen.sphere(4, meshgen.rng_for(2, 13))
    A = meshgen.vertex_attributes(m)
    enc = P.encode(m.tri, m.nverts, 64, 126)
    q = P.quantize_attributes(A, enc, 16)
    ref = O.dequantize(O.Quantized(q.origin, q.delta, q.lowest, q.offsets), q.vert_off)
    da = P.attrs_to_device(q)
    half = int(q.vert_off[len(q.vert_off) // 2])
    da.offset_count = half * 8 + 5            # not a whole vertex past the half: the next meshlet fails too
    out = torch.full((int(q.vert_off[-1]), 8), -1.0, dtype=torch.float32, device="cuda")
    say(f"[gpu] dequantize with offset_count {da.offset_count} of {q.offsets.size}")
    P.dequantize(da, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[:half], ref[:half])
    assert (got[half:] == -1.0).all()
