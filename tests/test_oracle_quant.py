"""CPU pins for the oracle's crack-free fixed-point attribute quantization
(Sec. 4.4): a hand-worked two-meshlet example, the b-bit offset bound, the
error bound of the global grid, identical bits for every copy of a vertex
(no cracks), and the information-content relation of the section."""
import math

import numpy as np
import pytest

import meshgen
import oracle as O


def test_handworked_two_meshlets():
    """One channel; meshlet 0 spans 0..65535, meshlet 1 spans 65535..100000:
    w = 65535, so the spacing is exactly 1, the grid is the values
    themselves, L = (0, 65535) and the offsets are the values minus L."""
    attrs = np.array([[0.0], [65535.0], [100000.0], [1234.0]], np.float32)
    verts = np.array([0, 3, 1, 1, 2], np.uint32)
    vert_off = np.array([0, 3, 5], np.uint64)
    qz = O.quantize(attrs, verts, vert_off, 16)
    assert qz.delta[0] == 1.0 and qz.origin[0] == 0.0
    np.testing.assert_array_equal(qz.L[:, 0], [0, 65535])
    np.testing.assert_array_equal(qz.q[:, 0], [0, 1234, 65535, 0, 34465])
    np.testing.assert_array_equal(O.dequantize(qz, vert_off)[:, 0], attrs[verts, 0])


def test_flat_channel():
    attrs = np.full((5, 2), 3.5, np.float32)
    attrs[:, 1] = [0, 1, 2, 3, 4]
    verts = np.arange(5, dtype=np.uint32)
    qz = O.quantize(attrs, verts, np.array([0, 2, 5], np.uint64), 16)
    assert qz.delta[0] == 1.0 and (qz.q[:, 0] == 0).all()
    np.testing.assert_array_equal(O.dequantize(qz, np.array([0, 2, 5], np.uint64))[:, 0], 3.5)


MESHES = {
    "sphere5": lambda: meshgen.sphere(5, meshgen.rng_for(2, 5)),
    "delaunay": lambda: meshgen.delaunay(20000, meshgen.rng_for(4, 5)),
}


@pytest.mark.parametrize("b", [16, 12, 8])
@pytest.mark.parametrize("caps", [(32, 64), (128, 256)])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_quantization_bounds_and_no_cracks(name, caps, b):
    m = MESHES[name]()
    A = meshgen.vertex_attributes(m)
    s = O.encode(m.tri, m.nverts, *caps)
    qz = O.quantize(A, s.verts, s.vert_off, b)
    out = O.dequantize(qz, s.vert_off)
    truth = A[s.verts.astype(np.int64)]
    top = (1 << b) - 1
    assert int(qz.q.max()) <= top
    # no cracks: every copy of a vertex decodes to the same bits
    order = np.argsort(s.verts, kind="stable")
    sv = s.verts[order]
    first = np.r_[True, sv[1:] != sv[:-1]]
    rep = np.maximum.accumulate(np.where(first, np.arange(sv.size), 0))
    bits = out.view(np.uint32)[order]
    np.testing.assert_array_equal(bits, bits[rep])
    M = s.meshlets
    for i in range(A.shape[1]):
        ext = [float(np.ptp(truth[int(s.vert_off[k]):int(s.vert_off[k + 1]), i].astype(np.float64))) for k in range(M)]
        w = max(ext)
        if w == 0:
            assert qz.delta[i] == 1.0
            continue
        d = float(qz.delta[i])
        # spacing: w / (2^b - 1), rounded up to float32 (widened only by rounding)
        assert w / top <= d <= w / top * (1 + 1e-5)
        # the widest meshlet uses (almost) the whole b-bit range
        assert int(qz.q[:, i].max()) >= top - 1
        # floor onto the global grid: 0 <= truth - decoded < spacing (+ float32 rounding)
        err = truth[:, i].astype(np.float64) - out[:, i].astype(np.float64)
        tol = np.spacing(np.abs(truth[:, i]).max()).astype(np.float64) * 2
        assert err.min() >= -tol and err.max() < d + tol
        # information content log2(W / delta) = log2(W / w) + log2(2^b - 1): at
        # least log2(2^b - 1) (the section's ">= b" up to that -1), more when
        # the mesh is wider than its widest meshlet
        W = float(A[:, i].max() - A[:, i].min())
        info = math.log2(W / d)
        assert abs(info - (math.log2(W / w) + math.log2(top))) < 1e-4
        assert info >= math.log2(top) - 1e-4


def test_local_grids_would_crack():
    """Planted mistake: quantizing each meshlet on its own grid (spacing from
    its own extent) gives different bits for shared vertices -- the crack the
    global grid prevents."""
    m = MESHES["sphere5"]()
    A = meshgen.vertex_attributes(m)
    s = O.encode(m.tri, m.nverts, 64, 126)
    qz = O.quantize(A, s.verts, s.vert_off, 16)
    out = O.dequantize(qz, s.vert_off)
    local = np.empty_like(out)
    for k in range(s.meshlets):
        a, z = int(s.vert_off[k]), int(s.vert_off[k + 1])
        v = A[s.verts[a:z].astype(np.int64), 0].astype(np.float64)
        lo, d = v.min(), max(np.ptp(v), 1e-30) / 65535
        local[a:z, 0] = (np.floor((v - lo) / d) * d + lo).astype(np.float32)
    order = np.argsort(s.verts, kind="stable")
    sv = s.verts[order]
    first = np.r_[True, sv[1:] != sv[:-1]]
    rep = np.maximum.accumulate(np.where(first, np.arange(sv.size), 0))
    assert (local[order, 0] != local[order, 0][rep]).any()
    assert (out[order, 0] == out[order, 0][rep]).all()
