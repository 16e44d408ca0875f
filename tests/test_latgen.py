"""The seeded lattice generator (CPU): the two BCC node orders describe the
same lattice, and in layer order a range of whole layers has only the next
corner layer as higher-id neighbours outside it (the sink-mode halo)."""

import numpy as np

import latgen


def _geometry(lat):
    pts = np.stack([lat.x, lat.y, lat.z], 1).astype(np.float64)
    key = lambda p: tuple(np.round(p, 6))  # noqa: E731
    nodes = {key(p) for p in pts}
    edges = {tuple(sorted((key(pts[a]), key(pts[b])))) for a, b in zip(lat.strut_a, lat.strut_b)}
    return nodes, edges


def test_bcc_orders_same_lattice():
    g = latgen.bcc(4, order="grid")
    layer = latgen.bcc(4, order="layer")
    assert g.n_nodes == layer.n_nodes == 5**3 + 4**3 and g.n_struts == layer.n_struts == 8 * 4**3
    assert _geometry(g) == _geometry(layer)


def test_bcc_layer_halo_is_one_corner_layer():
    n = 5
    lat = latgen.bcc(n, order="layer")
    B = (n + 1) ** 2 + n**2  # ids per layer below the top one
    for l0, l1 in ((0, 2), (1, 3), (2, 5)):
        n0, n1 = l0 * B, min(l1 * B, lat.n_nodes)
        a, b = lat.strut_a.astype(np.int64), lat.strut_b.astype(np.int64)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        halo = np.unique(hi[(lo >= n0) & (lo < n1) & (hi >= n1)])
        # exactly the corners of layer l1 (when it exists)
        if l1 <= n:
            assert np.array_equal(halo, np.arange(l1 * B, l1 * B + (n + 1) ** 2))
            assert np.allclose(lat.z[halo], l1)


def test_billion_config_uses_layer_order():
    lat = latgen.config(3, scale=3)
    ref = latgen.bcc(3, radius=("rel", 0.08, 0.1), jitter=0.0, seed=1, order="layer")
    for f in ("x", "y", "z", "radius", "strut_a", "strut_b"):
        assert np.array_equal(getattr(lat, f), getattr(ref, f)), f
