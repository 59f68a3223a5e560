"""CPU pins for the oracle's meshlet normal cones and culling decision
(Sec. 3: cone culling in the amplification shader): a flat patch has a
zero-angle cone, every triangle normal lies inside its meshlet's cone, a
culled meshlet has only triangles facing away (checked triangle by triangle),
on a sphere fewer than half of the meshlets face away from any direction, and
a hand-worked two-triangle meshlet fixes the axis as the sum of unit (not
area-weighted) normals."""
import numpy as np
import pytest

import meshgen
import oracle as O


def stream_and_decode(m, caps=(64, 126)):
    s = O.encode(m.tri, m.nverts, *caps)
    return s, O.decode(s)


def tri_normals(m, s, dec, mi):
    """Unit normals of meshlet mi's non-degenerate triangles (float64)."""
    _, _, out_off, T, _ = s.fields()
    tris = dec[out_off[mi]:out_off[mi] + T[mi]]
    keep = (tris[:, 0] != tris[:, 1]) & (tris[:, 1] != tris[:, 2]) & (tris[:, 0] != tris[:, 2])
    g = s.verts[int(s.vert_off[mi]) + tris[keep].astype(np.int64)]
    p = meshgen.vertex_attributes(m)[:, :3].astype(np.float64)[g]
    n = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def test_flat_patch_cone():
    m = meshgen.delaunay(3000, meshgen.rng_for(4, 21))
    s, dec = stream_and_decode(m)
    c = O.cones(s, dec, meshgen.vertex_attributes(m)[:, :3])
    np.testing.assert_array_equal(c[:, :3], np.tile([0, 0, 1], (s.meshlets, 1)).astype(np.float32))
    assert np.allclose(c[:, 3], 1e-5, atol=1e-7)
    assert O.cull(c, (0, 0, 1)).all()
    assert not O.cull(c, (0, 0, -1)).any()
    assert not O.cull(c, (1, 0, 0)).any()


@pytest.mark.parametrize("caps", [(32, 64), (128, 256)])
def test_cones_contain_normals_and_culling_is_conservative(caps):
    m = meshgen.sphere(4, meshgen.rng_for(2, 21))
    s, dec = stream_and_decode(m, caps)
    c = O.cones(s, dec, meshgen.vertex_attributes(m)[:, :3])
    rng = np.random.default_rng(21)
    views = rng.normal(size=(12, 3))
    views /= np.linalg.norm(views, axis=1, keepdims=True)
    for mi in range(s.meshlets):
        n = tri_normals(m, s, dec, mi)
        if c[mi, 3] >= 2:
            continue
        half = np.arcsin(min(1.0, float(c[mi, 3]) - 1e-5))
        ang = np.arccos(np.clip(n @ c[mi, :3].astype(np.float64), -1, 1))
        assert ang.max() <= half + 1e-5
    fr = []
    for v in views:
        culled = O.cull(c, v.astype(np.float32))
        fr.append(culled.mean())
        for mi in np.nonzero(culled)[0]:
            assert (tri_normals(m, s, dec, mi) @ v > 0).all()
    # jittered positions widen the cones; still a share of the meshlets faces away, never half
    assert 0.05 < np.mean(fr) < 0.5


def test_two_triangle_roof_axis_bisects_unit_normals():
    """Hand-worked: triangle (A, B, C) in the plane z = 0, normal +z, area 8,
    and triangle (B, A, D) across edge AB tilted by 60 degrees, normal
    (0, sin 60, cos 60), area 2.  The sum of the unit normals bisects them:
    axis (0, sin 30, cos 30), both normals 30 degrees off it, cutoff
    sin 30 + 1e-5.  An area-weighted sum would lean toward +z (about 11
    degrees) and fail; so would a dropped or doubled triangle."""
    t = np.radians(60.0)
    pos = np.array([[0, 0, 0], [4, 0, 0], [0, 4, 0], [2, -np.cos(t), np.sin(t)]], np.float32)
    tri = np.array([[0, 1, 2], [1, 0, 3]], np.uint32)
    s = O.encode(tri, 4, 64, 126)
    assert s.meshlets == 1
    c = O.cones(s, O.decode(s), pos)
    np.testing.assert_allclose(c[0, :3], [0.0, 0.5, np.sqrt(3) / 2], atol=2e-6)
    np.testing.assert_allclose(c[0, 3], 0.5 + 1e-5, atol=2e-6)
    # culled when the view direction lies within 60 degrees of the axis (every
    # normal then within 90 degrees of it: both triangles face away)
    for v in ([0.0, 0.5, np.sqrt(3) / 2], [0.0, 0.0, 1.0]):
        assert O.cull(c, np.array(v, np.float32))[0], v
    # not culled when a triangle faces the viewer: (0, 1, -0.2) sees the flat one
    for v in ([0.0, -1.0, 0.0], [0.0, 1.0 / np.hypot(1, 0.2), -0.2 / np.hypot(1, 0.2)]):
        assert not O.cull(c, np.array(v, np.float32))[0], v
