"""Binary STL writer: the file against a numpy serialisation of the same
device mesh (vertices bit for bit, normals to the rounding their
conditioning allows), chunking (many chunks with a ragged tail give the same
bytes as one), the empty mesh and a bad index."""

import numpy as np
import pytest

import latgen

pytestmark = pytest.mark.gpu

REC = np.dtype([("n", "<f4", (3,)), ("v", "<f4", (3, 3)), ("attr", "<u2")])


def _line(msg):
    print(msg, flush=True)


def _read(path):
    data = open(path, "rb").read()
    assert len(data) >= 84
    assert not data[:5].lower().startswith(b"solid")
    count = int(np.frombuffer(data[80:84], "<u4")[0])
    assert len(data) == 84 + 50 * count
    assert REC.itemsize == 50
    return count, np.frombuffer(data[84:], REC)


def _check_against_mesh(recs, xyz, tri):
    v = xyz[tri]  # [T, 3, 3] float32
    assert np.array_equal(recs["v"].view(np.uint32), v.view(np.uint32))
    assert (recs["attr"] == 0).all()
    v64 = v.astype(np.float64)
    e1 = v64[:, 1] - v64[:, 0]
    e2 = v64[:, 2] - v64[:, 0]
    c = np.cross(e1, e2)
    cl = np.linalg.norm(c, axis=1)
    ok = cl > 0
    ref = np.zeros_like(c)
    ref[ok] = c[ok] / cl[ok, None]
    # FP32 cross product: relative error of the normal ~ eps32 |e1||e2| / |e1 x e2|
    cond = np.linalg.norm(e1, axis=1) * np.linalg.norm(e2, axis=1) / np.maximum(cl, 1e-300)
    err = np.linalg.norm(recs["n"].astype(np.float64) - ref, axis=1)
    tol = 1e-6 + 1e-6 * cond
    assert (err[ok] <= tol[ok]).all(), float(np.max(err[ok] / tol[ok]))


def test_stl_file_matches_mesh(tmp_path):
    import torch

    from paper_2405_15197_amd import Mesher

    lat = latgen.config(2, scale=3, seed=5)
    M = Mesher(lat)
    try:
        r = M.run(8)
        t = r.totals
        _line(f"stl: {t['n_triangles']} triangles, {t['n_mesh_vertices']} mesh vertices")
        one = tmp_path / "one.stl"
        many = tmp_path / "many.stl"
        s1 = M.write_stl(r, str(one))
        # the smallest chunk: 256 triangles, so the last chunk is ragged
        s2 = M.write_stl(r, str(many), chunk_bytes=256 * 50)
        s3 = M.write_stl(r, None, chunk_bytes=256 * 50)
        torch.cuda.synchronize()
        xyz = r.mesh_xyz.cpu().numpy()
        tri = r.tri.cpu().numpy()
    finally:
        M.close()
    T = tri.shape[0]
    assert T % 256 != 0
    assert s1["n_chunks"] == 1 and s2["n_chunks"] == (T + 255) // 256 == s3["n_chunks"]
    assert s1["n_bytes"] == s2["n_bytes"] == 84 + 50 * T
    assert one.read_bytes() == many.read_bytes()
    count, recs = _read(one)
    assert count == T
    _check_against_mesh(recs, xyz, tri)


def test_stl_empty_and_bad_index(tmp_path):
    import torch

    from paper_2405_15197_amd.latmesh import LM_ERR_INVALID_ARG, LatmeshError, write_stl

    xyz = torch.rand((10, 3), device="cuda")
    empty = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    p = tmp_path / "empty.stl"
    st = write_stl(xyz, empty, str(p))
    assert st["n_bytes"] == 84 and st["n_chunks"] == 0
    count, recs = _read(p)
    assert count == 0 and len(recs) == 0
    # a small mesh written in full, then one index out of range
    tri = torch.tensor([[0, 1, 2], [3, 4, 5], [7, 8, 9]], dtype=torch.int32, device="cuda")
    p2 = tmp_path / "small.stl"
    write_stl(xyz, tri, str(p2))
    count, recs = _read(p2)
    _check_against_mesh(recs, xyz.cpu().numpy(), tri.cpu().numpy())
    bad = torch.tensor([[0, 1, 2], [3, 4, 10]], dtype=torch.int32, device="cuda")
    with pytest.raises(LatmeshError) as e:
        write_stl(xyz, bad, str(tmp_path / "bad.stl"))
    assert e.value.code == LM_ERR_INVALID_ARG
