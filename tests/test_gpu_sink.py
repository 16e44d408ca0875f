"""Sink mode (chunked meshing reduced to per-chunk counts and hashes)
against the oracle and against the stored mode.

Exact: triangles, the triangle-key sum, mesh vertices and bad nodes per
chunk (where the GPU's triangulation equals the oracle's), and the vertex-key
sum against the same hash over the stored mode's FP32 mesh.  The fixed-point
coordinate sums differ from the oracle's FP64 ones by rounding only: at most
one unit of 2^-20 per vertex plus the vertex position tolerance.
"""

import types

import numpy as np
import pytest

import latgen
import oracle

pytestmark = pytest.mark.gpu


def _vert_hash_stored(mesh_xyz, node_off_mesh):
    """The sink's vertex-key sum per node over the stored mode's mesh."""
    xyz = np.ascontiguousarray(mesh_xyz, np.float32)
    n = len(node_off_mesh) - 1
    node_of = np.repeat(np.arange(n), np.diff(node_off_mesh))
    local = np.arange(len(node_of)) - node_off_mesh[node_of]
    vid = (node_of.astype(np.uint64) << np.uint64(21)) | local.astype(np.uint64)
    b = xyz.view(np.uint32).astype(np.uint64)
    with np.errstate(over="ignore"):
        k = oracle._mix(oracle._mix(oracle._mix(vid) ^ (b[:, 0] | (b[:, 1] << np.uint64(32)))) ^ b[:, 2])
    return node_of, k


CASES = [
    ("bcc4", lambda: latgen.config(2, scale=4, seed=7), 16),
    ("octet3", lambda: latgen.config(4, scale=3, seed=7), 12),
]


@pytest.mark.parametrize("name,make,k", CASES, ids=[c[0] for c in CASES])
def test_sink_matches_oracle_and_stored(name, make, k):
    import torch

    from paper_2405_15197_amd import Mesher

    lat = make()
    R = oracle.run(lat, k)
    M = Mesher(lat)
    try:
        r = M.run(k, meta=False)
        torch.cuda.synchronize()
        moff = r.node_off[3].cpu().numpy()
        tri = r.tri.cpu().numpy().astype(np.int64)
        node = np.searchsorted(moff, tri, side="right") - 1
        same = np.array_equal(np.stack([node, tri - moff[node]], -1),
                              np.stack([np.searchsorted(R.mesh_off, R.tris, side="right") - 1,
                                        R.tris - R.mesh_off[np.searchsorted(R.mesh_off, R.tris, side="right") - 1]],
                                       -1))
        assert same, "GPU and oracle triangulations differ on this lattice"
        node_of, vk = _vert_hash_stored(r.mesh_xyz.cpu().numpy(), moff)
        totals = None
        for chunk in (lat.n_nodes, 97, 31):
            got = M.sink(k, chunk)
            exp = oracle.sink_words(R, chunk, lat.strut_a, lat.strut_b)
            assert got.shape == exp.shape
            for f in (0, 1, 2, 7):
                assert np.array_equal(got[:, f], exp[:, f]), (name, chunk, f, got[:, f], exp[:, f])
            # vertex keys: the stored mode's FP32 mesh, hashed the same way
            ch = node_of // chunk
            for c in range(got.shape[0]):
                with np.errstate(over="ignore"):
                    assert got[c, 3] == np.sum(vk[ch == c], dtype=np.uint64)
            d = (got[:, 4:7].view(np.int64) - exp[:, 4:7].view(np.int64)).astype(np.float64)
            lim = exp[:, 2].astype(np.float64)[:, None] * (1.0 + 1e-5 * 0.12 * 1048576.0)
            assert (np.abs(d) <= lim).all(), (d, lim)
            with np.errstate(over="ignore"):
                tot = got.sum(axis=0, dtype=np.uint64)
            if totals is None:
                totals = tot
            assert np.array_equal(tot, totals), "sink totals depend on the chunking"
    finally:
        M.close()


def test_sink_billion_family_device_generated():
    """The billion-strut family (BCC, radii 0.08 (1 +- 0.1), no jitter, nodes
    numbered layer by layer) at 24^3 cells, generated on the device: every
    node is meshed (the oracle meshes all of them), the totals do not depend
    on the chunking (slabs of layers, and chunks that cut layers), and the
    stored mesh of the same lattice is closed and outward oriented with
    chi = 2N - 2S, its triangle and vertex counts equal to the sink's."""
    import latgen.device
    from paper_2405_15197_amd import Mesher
    from parity import check_closed, result_np

    lat = latgen.device.config(3, scale=24)
    M = Mesher(lat)
    try:
        tots = []
        for chunk in (lat.n_nodes, 4099, 2 * (25 * 25 + 24 * 24)):
            w = M.sink(12, chunk)
            assert int(w[:, 7].sum()) == 0, "nodes without a mesh"
            with np.errstate(over="ignore"):
                tots.append(w.sum(axis=0, dtype=np.uint64))
        assert np.array_equal(tots[0], tots[1]) and np.array_equal(tots[0], tots[2])
        G = result_np(M.run(12, meta=False), meta=False)
    finally:
        M.close()
    assert int(tots[0][0]) == G["totals"]["n_triangles"] and int(tots[0][2]) == G["totals"]["n_mesh_vertices"]
    host = types.SimpleNamespace(n_nodes=lat.n_nodes, n_struts=lat.n_struts)
    chi, vol = check_closed(G, host)
    print(f"billion family 24^3: closed, chi {chi}, volume {vol:.4g}", flush=True)
