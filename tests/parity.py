"""Element-by-element comparison of the GPU path with the FP64 oracle.

Combinatorial output (per-node counts, vertex names, arc labels and end
vertices, band and fan triangles as (node, local vertex) triples) must be
identical on every node whose oracle margins are above the comparison
thresholds (and every strut whose two end nodes and zipper margin are).
Positions must agree to 1e-5 of the node radius in node-local coordinates;
absolute mesh positions additionally carry the FP32 rounding of c + w (one
ulp of |x|).

Thresholds, per margin kind (oracle.c MK_*), from the FP32 path's measured
errors (vertex positions within 1e-6 rho, arc parameters within 1e-6 rad,
the tests' own statistics) with a factor of about ten:
  conic extremum |F| / rho 1e-5, runner-up gap at a vertex 1e-5, tie-root
  separation 1e-5, phi step along a loop 1e-5 rad: errors of about 1e-6;
  Eq. 11 floor, distance of k dt / 2 pi to an integer: 1.5e-6 k (the error
  of dt times k / 2 pi);
  ellipse (|e . n| - |sigma|), hole barycentre and strut-frame near ties:
  1e-4 (rare; not measured below that);
  zipper phi gaps between the two loops of a strut: 1e-5 rad.
Exact ties that both sides decide by the same rule (equal |e_j| in the strut
frame, whole tangency circles sampled at the same parameters) carry no
margin in the oracle.
"""

from __future__ import annotations

import numpy as np

import oracle

TAU = 1e-4  # a single threshold for every margin kind (when given)
STRUT_TAU = 1e-5
GEOM_TOL = 1e-5  # relative to the node radius

# margin kinds of oracle.c, column kind - 1 of OracleResult.kmargin
MK_ELLIPSE, MK_CONIC, MK_FRAME, MK_ROOTS, MK_GAP, MK_FLOOR, MK_HOLE, MK_STEP = range(1, 9)


def node_tau(k):
    """Comparison threshold of each margin kind at resolution k."""
    t = np.full(8, 1e-4)
    for kind in (MK_CONIC, MK_ROOTS, MK_GAP, MK_STEP):
        t[kind - 1] = 1e-5
    t[MK_FLOOR - 1] = 1.5e-6 * k
    return t


def above_margin(R, k, tau=None):
    """Nodes whose margins are all above the thresholds (tau: one value for
    every kind instead of the per-kind ones)."""
    if tau is not None:
        return R.margin >= tau
    return (R.kmargin >= node_tau(k)[None, :]).all(axis=1)


def gpu_result(lat, k, meta=True, kappa_max=None):
    import torch

    from paper_2405_15197_amd import Mesher

    M = Mesher(lat, kappa_max=kappa_max)
    try:
        out = result_np(M.run(k, meta=meta), meta)
    finally:
        M.close()
    return out


def result_np(r, meta=True):
    """Host copies of a trimmed MeshResult."""
    import torch

    torch.cuda.synchronize()
    out = {
        "totals": r.totals,
        "mesh": r.mesh_xyz.cpu().numpy().astype(np.float64),
        "tri": r.tri.cpu().numpy().astype(np.int64),
        "node_off": r.node_off.cpu().numpy(),
        "status": r.node_status.cpu().numpy().astype(np.int64),
        "strut_off": r.strut_off.cpu().numpy(),
    }
    if meta:
        out["vert_name"] = r.vert_name.cpu().numpy().view(np.uint32)
        out["vert_xyz"] = r.vert_xyz.cpu().numpy().T.astype(np.float64)
        out["arc_f32"] = r.arc_f32.cpu().numpy().T.astype(np.float64)
        out["arc_u32"] = r.arc_u32.cpu().numpy().view(np.uint32).T.copy()
    return out


def _sel(counts, mask):
    return np.repeat(mask, counts)


def _node_local(ids, moff):
    node = np.searchsorted(moff, ids, side="right") - 1
    return node, ids - moff[node]


def compare(lat, k, R=None, G=None, tau=None, strut_tau=None, check_all_status=True, geom_tol=GEOM_TOL,
            kappa_max=None):
    """Assert parity; returns a dict of statistics.  Nodes are compared when
    their margins are above the per-kind thresholds (or all at least ``tau``
    when given), struts when their zipper margin is at least ``strut_tau``
    (default STRUT_TAU, or ``tau`` when given)."""
    if strut_tau is None:
        strut_tau = STRUT_TAU if tau is None else tau
    R = R if R is not None else oracle.run(lat, k)
    G = G if G is not None else gpu_result(lat, k, kappa_max=kappa_max)
    N, S = lat.n_nodes, lat.n_struts
    rho = lat.radius.astype(np.float64)
    xyz = lat.xyz64()
    off = G["node_off"]
    gnv, gne, gnc, gnm, gnf = (np.diff(off[c]) for c in range(5))
    gst = G["status"]
    above = above_margin(R, k, tau)
    stable = (R.status == 0) & above
    stats = {"nodes": N, "stable": int(stable.sum()), "oracle_bad": int((R.status != 0).sum()),
             "fp64_nodes": int(G["totals"]["n_fp64_nodes"])}
    # status
    assert (gst[stable] == 0).all(), f"GPU flags stable nodes: {np.nonzero(gst[stable])[0][:10]}"
    if check_all_status:
        conf = (R.status != 0) & above
        assert (gst[conf] != 0).all(), "GPU misses an oracle flag"
    # counts
    for name, g, o in (("nv", gnv, R.nv), ("ne", gne, R.ne), ("nc", gnc, R.nc), ("nmesh", gnm, R.nmesh),
                       ("nfan", gnf, R.nfan)):
        bad = np.nonzero(stable & (g != o))[0]
        assert len(bad) == 0, f"count {name} differs at nodes {bad[:10]}: gpu {g[bad[:10]]} oracle {o[bad[:10]]}"
    # meta-mesh vertices
    if "vert_name" in G:
        gm = _sel(gnv, stable)
        om = _sel(R.nv, stable)
        assert np.array_equal(G["vert_name"][gm], R.vert_name[om]), "vertex names differ"
        rv = np.repeat(rho, R.nv)[om]
        err = np.abs(G["vert_xyz"][gm] - R.vert_w[om]).max(axis=1) / rv
        stats["vert_err"] = float(err.max()) if len(err) else 0.0
        assert stats["vert_err"] <= geom_tol, f"vertex position error {stats['vert_err']:.3g} rho"
        # arcs
        gm = _sel(gne, stable)
        om = _sel(R.ne, stable)
        gu = G["arc_u32"][gm]
        oi = R.arc_int[om]
        assert np.array_equal(gu[:, 0] & 0xFF, oi[:, 0]) and np.array_equal((gu[:, 0] >> 8) & 0xFF, oi[:, 1])
        assert np.array_equal((gu[:, 0] >> 16) & 1, oi[:, 6]), "whole-conic flags differ"
        assert np.array_equal(gu[:, 1] & 0xFFFF, oi[:, 2]) and np.array_equal(gu[:, 1] >> 16, oi[:, 3])
        ra = np.repeat(rho, R.ne)[om]
        gf = G["arc_f32"][gm]
        od = R.arc_dbl[om]
        # centre and semi-axis lengths are always well defined; the axis
        # directions and t-range only for circles (strut frame) and for
        # ellipses that are not nearly circular
        la, lb = np.linalg.norm(od[:, 3:6], axis=1), np.linalg.norm(od[:, 6:9], axis=1)
        gla, glb = np.linalg.norm(gf[:, 3:6], axis=1), np.linalg.norm(gf[:, 6:9], axis=1)
        # the conic's fields are FP32 numbers of their own size (a long thin
        # seam ellipse has |o| and |a| far above rho): their error is
        # measured against rho plus 2^-20 of that size
        size = np.maximum(np.linalg.norm(od[:, 0:3], axis=1), la) / ra
        scale = 1.0 + (2.0 ** -20 / geom_tol) * size if len(gf) else np.zeros(0)
        e_o = np.abs(gf[:, 0:3] - od[:, 0:3]).max(axis=1) / ra / scale if len(gf) else np.zeros(0)
        e_l = np.maximum(np.abs(gla - la), np.abs(glb - lb)) / ra / scale if len(gf) else np.zeros(0)
        axes = (oi[:, 0] == 0) | ((la - lb) / ra > 1e-3)
        e_v = np.abs(gf[:, 3:9] - od[:, 3:9]).max(axis=1) / ra / scale if len(gf) else np.zeros(0)
        stats["arc_err"] = float(max(e_o.max(initial=0), e_l.max(initial=0), e_v[axes].max(initial=0)))
        stats["arc_size_max"] = float(size.max(initial=0))
        assert stats["arc_err"] <= geom_tol, f"arc geometry error {stats['arc_err']:.3g} rho (size-scaled)"
        dt = np.abs((gf[axes, 9:11] - od[axes, 9:11] + np.pi) % (2 * np.pi) - np.pi)
        stats["arc_t_err"] = float(dt.max(initial=0))
        assert stats["arc_t_err"] <= 5e-5, f"arc parameter error {stats['arc_t_err']:.3g}"
    # mesh vertices (absolute)
    gm = _sel(gnm, stable)
    om = _sel(R.nmesh, stable)
    gx = G["mesh"][gm]
    ox = R.mesh[om]
    rv = np.repeat(rho, R.nmesh)[om]
    ulp = np.spacing(np.abs(ox).max(axis=1).astype(np.float32)).astype(np.float64)
    err = np.abs(gx - ox).max(axis=1)
    rel = np.maximum(err - ulp, 0) / rv
    stats["mesh_err_rho"] = float(rel.max()) if len(err) else 0.0
    if stats["mesh_err_rho"] > geom_tol:
        i = int(np.argmax(rel))
        node = np.repeat(np.arange(N), R.nmesh)[om][i]
        loc = i - int(np.searchsorted(np.repeat(np.arange(N), R.nmesh)[om], node))
        kind = "vertex" if loc < R.nv[node] else ("hole centre" if loc >= R.nmesh[node] - R.nc[node] else "interior")
        raise AssertionError(f"mesh vertex error {stats['mesh_err_rho']:.3g} rho beyond 1 ulp at node {node} local "
                             f"{loc} ({kind}; nv {R.nv[node]} nc {R.nc[node]} valence {R.valence[node]} "
                             f"margin {R.margin[node]:.3g}) gpu {gx[i]} oracle {ox[i]}")
    # band triangles per strut, as (node, local) triples
    gso = G["strut_off"]
    sa, sb = lat.strut_a.astype(np.int64), lat.strut_b.astype(np.int64)
    sst = stable[sa] & stable[sb] & (R.strut_margin >= strut_tau) & (R.strut_status == 0)
    gbc, obc = np.diff(gso), np.diff(R.band_off)
    bad = np.nonzero(sst & (gbc != obc))[0]
    assert len(bad) == 0, f"band triangle counts differ at struts {bad[:10]}"
    gt = G["tri"][: gso[-1]][_sel(gbc, sst)]
    ot = R.tris[: R.n_band][_sel(obc, sst)]
    gnode, gloc = _node_local(gt, off[3])
    onode, oloc = _node_local(ot, R.mesh_off)
    assert np.array_equal(gnode, onode) and np.array_equal(gloc, oloc), "band triangles differ"
    # struts between two compared nodes whose loops tie in phi (exactly, for
    # loop vertices of both ends on one generator, or within the threshold):
    # the apex choices may differ, the band's size and vertex set may not
    tie = stable[sa] & stable[sb] & (R.strut_status == 0) & ~sst
    bad = np.nonzero(tie & (gbc != obc))[0]
    assert len(bad) == 0, f"band triangle counts differ at tied struts {bad[:10]}"
    for s_ in np.nonzero(tie)[0][:2000]:
        gt_ = G["tri"][gso[s_]:gso[s_ + 1]].ravel()
        ot_ = R.tris[R.band_off[s_]:R.band_off[s_ + 1]].ravel()
        gn_, gl_ = _node_local(gt_, off[3])
        on_, ol_ = _node_local(ot_, R.mesh_off)
        assert np.array_equal(np.unique(gn_ * (1 << 24) + gl_), np.unique(on_ * (1 << 24) + ol_)), \
            f"band vertices differ at tied strut {s_}"
    stats["struts"] = S
    stats["stable_struts"] = int(sst.sum())
    stats["tied_struts"] = int(tie.sum())
    # fans per node
    gf_ = G["tri"][gso[-1]:][_sel(gnf, stable)]
    of_ = R.tris[R.n_band:][_sel(R.nfan, stable)]
    gnode, gloc = _node_local(gf_, off[3])
    onode, oloc = _node_local(of_, R.mesh_off)
    assert np.array_equal(gnode, onode) and np.array_equal(gloc, oloc), "fan triangles differ"
    return stats


def check_closed(G, lat):
    """The GPU mesh of a lattice whose nodes are all meshed is a closed,
    consistently oriented surface: every directed edge is used once and has
    its opposite twin (watertight, oriented, manifold along edges), every
    mesh vertex is used, the Euler characteristic is 2N - 2S (each node a
    sphere, each strut a handle), and the enclosed volume is positive
    (normals outward).  Returns (chi, volume)."""
    tri = G["tri"].astype(np.int64)
    M = int(G["totals"]["n_mesh_vertices"])
    assert G["totals"]["n_bad_nodes"] == 0 and G["totals"]["n_skipped_struts"] == 0
    e0 = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    e1 = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    key = np.sort(e0 * M + e1)
    assert (key[1:] != key[:-1]).all(), "a directed edge is used twice"
    rkey = e1 * M + e0
    pos = np.searchsorted(key, rkey).clip(max=len(key) - 1)
    assert (key[pos] == rkey).all(), "an edge has no opposite twin"
    assert len(np.unique(tri)) == M, "unused mesh vertices"
    chi = M - len(key) // 2 + len(tri)
    assert chi == 2 * lat.n_nodes - 2 * lat.n_struts, (chi, 2 * lat.n_nodes - 2 * lat.n_struts)
    v = G["mesh"][tri] - G["mesh"].mean(axis=0)
    vol = float(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0)
    assert vol > 0, "mesh oriented inward"
    return chi, vol


def sub_lattice(lat, centre_nodes):
    """The stars of ``centre_nodes``: those nodes, their neighbours and every
    strut incident to a centre node, with node and strut order preserved (so
    labels, strut frames and loop starts are unchanged for the centres).
    Returns (sub lattice, node map old->new (-1 if absent), strut ids kept)."""
    import latgen

    sa, sb = lat.strut_a.astype(np.int64), lat.strut_b.astype(np.int64)
    cen = np.zeros(lat.n_nodes, bool)
    cen[centre_nodes] = True
    keep_s = np.nonzero(cen[sa] | cen[sb])[0]
    nodes = np.unique(np.concatenate([sa[keep_s], sb[keep_s], np.asarray(centre_nodes)]))
    nmap = np.full(lat.n_nodes, -1, np.int64)
    nmap[nodes] = np.arange(len(nodes))
    sub = latgen.lattice_from_arrays(
        np.stack([lat.x[nodes], lat.y[nodes], lat.z[nodes]], 1).astype(np.float64),
        lat.radius[nodes].astype(np.float64),
        np.stack([nmap[sa[keep_s]], nmap[sb[keep_s]]], 1),
    )
    # keep the exact FP32 inputs
    sub.x, sub.y, sub.z, sub.radius = lat.x[nodes], lat.y[nodes], lat.z[nodes], lat.radius[nodes]
    return sub, nmap, keep_s
