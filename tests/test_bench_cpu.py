"""The benchmark's host-side pieces, on the CPU: its algorithmic byte count
against the per-meshlet figure of the method (flag chunks, reuse bytes,
descriptors read once; three output bytes per strip triangle written once),
the rule that reads committed traffic counters only for the kernel source
they were taken on, the serving pool of distinct meshes, and its one-GPU
contract."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import meshgen  # noqa: E402
import paper_2404_06359_amd as P  # noqa: E402


def test_algorithmic_bytes_follow_the_per_meshlet_figure():
    """Per meshlet the method reads its 16-byte descriptor, 16 bytes per 64
    strip triangles of flags and T_s - V + 2 reuse bytes (every strip slot
    after the first three that is not a first use), and writes 3 T_s bytes;
    the streams hold nothing else."""
    meshes = [(meshgen.workload1(), (64, 126)), (meshgen.fan(200), (64, 126)), (meshgen.disjoint(40), (32, 64)),
              (meshgen.delaunay(3000, meshgen.rng_for(4, 5)), (128, 256))]
    encs = []
    want = 0
    for m, caps in meshes:
        e = P.encode(m.tri, m.nverts, *caps)
        encs.append(e)
        d = e.meshlets
        T = d["tri_count"].astype(np.int64)
        V = d["vert_count"].astype(np.int64)
        want += int((16 + 16 * ((T + 63) // 64) + (T - V + 2) + 3 * T).sum())
    assert bench.algorithmic_bytes(encs) == want


def test_traffic_is_read_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "paper_2404_06359_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "decode.hip").write_text("// a comment\nint x;\n\nint y;  // trailing\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_source_hash()
    (prof / "traffic_k_w.txt").write_text(f"# header: ignored\nkernel_source_sha256_16: {h}\n"
                                          "hbm_bytes_per_launch: 1234\n")
    assert bench.read_traffic("k", "w") == 1234.0
    assert bench.read_traffic("k", "other") is None            # no file for this workload
    # comments and blank lines do not change the hash; code does
    (src / "decode.hip").write_text("int x;\n// another comment\nint y;\n")
    assert bench.read_traffic("k", "w") == 1234.0
    (src / "decode.hip").write_text("int x;\nint z;\n")
    assert bench.read_traffic("k", "w") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""



def test_distinct_serving_pool_follows_its_recipe(monkeypatch):
    """workload5_spec gives the (kind, size, caps) that workload5_mesh builds;
    the distinct pool holds each mesh's own streams and counts -- the bytes a
    plain encode of the shuffled mesh gives, though the pool encodes the
    unshuffled one -- but not its vertex lists or triangle ids."""
    spec = meshgen.workload5_spec(60)
    small = [i for i, (_, n, _) in enumerate(spec) if n < 60000][:5]
    assert len(small) >= 3 and {spec[i][0] for i in small} == {"grid", "patch"}
    build = meshgen.workload5_mesh
    meshes = [build(i) for i in small]
    for i, m in zip(small, meshes):
        kind, n, caps = spec[i]
        assert (m.kind, m.meta["target_n"], (m.max_vertices, m.max_triangles)) == (kind, n, caps)
        plain = build(i, permute=False)
        assert plain.ntri == m.ntri and not np.array_equal(plain.tri, m.tri)
    # a pool of just those meshes: mesh j of the patched recipe is mesh small[j]
    monkeypatch.setattr(meshgen, "workload5_spec", lambda count: [spec[i] for i in small][:count])
    monkeypatch.setattr(meshgen, "workload5_mesh", lambda j, permute=True: build(small[j], permute=permute))
    encs = bench.build_serve_distinct(len(small), 2)
    for e, m in zip(encs, meshes):
        full = P.encode(m.tri, m.nverts, m.max_vertices, m.max_triangles)
        np.testing.assert_array_equal(e.meshlets, full.meshlets)
        np.testing.assert_array_equal(e.bits, full.bits)
        np.testing.assert_array_equal(e.reuse, full.reuse)
        assert e.stats["input_triangles"] == full.stats["input_triangles"] == m.ntri
        assert e.strip_triangles == full.strip_triangles
        assert e.verts.size == 0 and e.kept_off is None and e.tri_ids is None
