"""Adjoint (fixed-topology gradient of a mesh loss) on the GPU against the
FP64 oracle's gradient (central differences with frozen topology).

Tolerance, from the arithmetic: the GPU works in FP32 (relative rounding
about 1e-7 per operation, amplified by the conditioning of the tie solves
and of the hole-centre normalisation), the oracle's gradient is accurate to
about 1e-9.  A parameter passes when |g_gpu - g_oracle| <= 1e-3 |g_oracle|
+ 1e-4 max|g_oracle|.
"""

import numpy as np
import pytest

import latgen
import oracle

pytestmark = pytest.mark.gpu

W3 = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
CASES = [
    ("octet2", lambda: latgen.config(4, scale=2, seed=6), 12),
    ("bcc3", lambda: latgen.config(2, scale=3, seed=3), 16),
]


def _gpu_grad(lat, k, weights):
    import torch

    from paper_2405_15197_amd import Mesher

    M = Mesher(lat)
    try:
        r = M.run(k, meta=False)
        terms, dl = M.loss(r, weights)
        gx, gr = M.backward(dl)
        torch.cuda.synchronize()
        tri = r.tri.cpu().numpy().astype(np.int64)
        moff = r.node_off[3].cpu().numpy()
        return (terms.cpu().numpy(), gx.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64),
                (tri, moff))
    finally:
        M.close()


def _as_local(tri, moff):
    node = np.searchsorted(moff, tri, side="right") - 1
    return np.stack([node, tri - moff[node]], -1)


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, make, k = request.param
    lat = make()
    R = oracle.run(lat, k)
    assert (R.status == 0).all()
    params = [(n, c) for n in range(lat.n_nodes) for c in range(4)]
    G, ok = oracle.fd_gradient(lat, k, params, weights=W3)
    return lat, k, R, params, G, ok


@pytest.mark.parametrize("wi", [0, 1, 2], ids=["area", "volume", "sq_norm"])
def test_gradient_matches_oracle(case, wi):
    lat, k, R, params, G, ok = case
    terms, gx, gr, (tri, moff) = _gpu_grad(lat, k, W3[wi])
    # the same triangulation as the oracle's, so the same loss function
    assert np.array_equal(_as_local(tri, moff), _as_local(R.tris, R.mesh_off))
    # loss terms against the oracle's mesh
    area = oracle.mesh_area(R.mesh, R.tris)
    v = R.mesh[R.tris]
    vol = float(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0)
    sq = oracle.mesh_sq(R.mesh)
    np.testing.assert_allclose(terms, [area, vol, sq], rtol=2e-5)
    g_gpu = np.array([gx[n, c] if c < 3 else gr[n] for n, c in params])
    g_orc = G[:, wi]
    sel = ok
    assert sel.mean() > 0.95
    tol = 1e-3 * np.abs(g_orc[sel]) + 1e-4 * np.abs(g_orc[sel]).max()
    err = np.abs(g_gpu[sel] - g_orc[sel])
    worst = int(np.argmax(err / tol))
    assert (err <= tol).all(), (
        f"{int((err > tol).sum())} of {sel.sum()} parameters off; worst {np.array(params)[sel][worst]} "
        f"gpu {g_gpu[sel][worst]:.6g} oracle {g_orc[sel][worst]:.6g}")


@pytest.mark.parametrize("wi,degree", [(0, 2), (1, 3), (2, 2)], ids=["area", "volume", "sq_norm"])
def test_gradient_euler_identity(case, wi, degree):
    """sum_j theta_j dL/dtheta_j = degree * L for the GPU's own gradient."""
    lat, k, R, params, G, ok = case
    terms, gx, gr, _ = _gpu_grad(lat, k, W3[wi])
    theta = np.stack([lat.x, lat.y, lat.z], 1).astype(np.float64)
    lhs = float((theta * gx).sum() + (lat.radius.astype(np.float64) * gr).sum())
    L = float(terms[wi])
    assert abs(lhs - degree * L) <= 1e-4 * abs(degree * L) + 1e-5, (lhs, degree * L)


def test_autograd_function_matches_loss_path():
    import torch

    from paper_2405_15197_amd import Mesher
    from paper_2405_15197_amd.latmesh import mesh_function

    lat = latgen.config(4, scale=2, seed=2)
    k = 12
    M = Mesher(lat)
    try:
        r = M.alloc(M.count(k), meta=False)
        xyz = torch.tensor(np.stack([lat.x, lat.y, lat.z], 1), device="cuda", requires_grad=True)
        rad = torch.tensor(lat.radius, device="cuda", requires_grad=True)
        verts = mesh_function().apply(xyz, rad, M, k, r)
        tri = r.tri[: M.totals["n_triangles"]].long()
        v = verts[: M.totals["n_mesh_vertices"]]
        a, b, c = v[tri[:, 0]], v[tri[:, 1]], v[tri[:, 2]]
        area = 0.5 * torch.linalg.cross(b - a, c - a).norm(dim=1).sum()
        area.backward()
        terms, dl = M.loss(r, (1.0, 0.0, 0.0))
        gx, gr = M.backward(dl)
        torch.cuda.synchronize()
        assert abs(area.item() - terms[0].item()) <= 1e-5 * terms[0].item()
        np.testing.assert_allclose(xyz.grad.cpu().numpy(), gx.cpu().numpy(), rtol=1e-3, atol=1e-4)
        np.testing.assert_allclose(rad.grad.cpu().numpy(), gr.cpu().numpy(), rtol=1e-3, atol=1e-4)
    finally:
        M.close()


def test_adjoint_is_bit_reproducible():
    """The node and half-edge partials are summed per node in adjacency order
    (no atomics between nodes), and the loss terms per node in a fixed order:
    repeated runs give identical bits."""
    import torch

    from paper_2405_15197_amd import Mesher

    lat = latgen.config(4, scale=6, seed=9)
    M = Mesher(lat)
    try:
        r = M.run(16, meta=False)
        outs = []
        for _ in range(3):
            terms, dl = M.loss(r, (1.0, 0.3, 0.1))
            gx, gr = M.backward(dl)
            torch.cuda.synchronize()
            outs.append((terms.cpu().numpy().copy(), dl.cpu().numpy().copy(), gx.cpu().numpy().copy(),
                         gr.cpu().numpy().copy()))
        for o in outs[1:]:
            for a, b in zip(outs[0], o):
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    finally:
        M.close()


def test_gradient_config_size_octet32():
    """The differentiation workload at its size: octet 32^3 (137,313 nodes,
    798,720 struts, radii U[0.04, 0.10], jitter 0.03), k = 16; 64 seeded
    random parameters (node coordinate or radius) against the oracle's FP64
    central differences (h = 1e-6), which re-mesh only the stars around each
    parameter's node.  Tolerance as for the small lattices above."""
    import torch

    from paper_2405_15197_amd import Mesher

    lat = latgen.config(4)
    k = 16
    rng = np.random.default_rng(64)
    nodes = rng.choice(lat.n_nodes, size=64, replace=False)
    comps = rng.integers(0, 4, size=64)
    params = [(int(n), int(c)) for n, c in zip(nodes, comps)]
    print(f"octet32: {lat.n_nodes} nodes, {lat.n_struts} struts; oracle FD on 64 parameters", flush=True)
    G, ok = oracle.fd_gradient(lat, k, params, weights=W3)
    M = Mesher(lat)
    try:
        r = M.run(k, meta=False)
        assert r.totals["n_bad_nodes"] == 0
        for wi in range(3):
            terms, dl = M.loss(r, W3[wi])
            gx, gr = M.backward(dl)
            torch.cuda.synchronize()
            gx, gr = gx.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
            g_gpu = np.array([gx[n, c] if c < 3 else gr[n] for n, c in params])
            g_orc = G[:, wi]
            sel = ok
            assert sel.mean() > 0.9
            tol = 1e-3 * np.abs(g_orc[sel]) + 1e-4 * np.abs(g_orc[sel]).max()
            err = np.abs(g_gpu[sel] - g_orc[sel])
            assert (err <= tol).all(), (wi, int((err > tol).sum()), float((err / tol).max()))
    finally:
        M.close()
