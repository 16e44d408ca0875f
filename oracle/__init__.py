"""FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``oracle.c`` (plain C, double precision), which
shares no code with the GPU library.  See the header of ``oracle.c`` for the
method and the paper passages each step follows.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_INVALID_STRUT = 1
ST_NON_ELLIPTIC = 2
ST_LOOP = 4
ST_TOPOLOGY = 8
ST_ISOLATED = 16
ST_VALENCE = 32
ST_DUPLICATE = 64

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.orc_run.restype = P
    lib.orc_run.argtypes = [ctypes.c_int64, ctypes.c_int64] + [P] * 6 + [ctypes.c_int, ctypes.c_int]
    lib.orc_run_f64.restype = P
    lib.orc_run_f64.argtypes = [ctypes.c_int64, ctypes.c_int64] + [P] * 6 + [ctypes.c_int, ctypes.c_int]
    lib.orc_free.argtypes = [P]
    lib.orc_sizes.argtypes = [P, P]
    lib.orc_nodes.argtypes = [P, P, P]
    lib.orc_node_margins.argtypes = [P, P]
    lib.orc_vertices.argtypes = [P, P, P, P]
    lib.orc_arcs.argtypes = [P, P, P]
    lib.orc_loops.argtypes = [P, P, P, P]
    lib.orc_adjacency.argtypes = [P, P, P]
    lib.orc_mesh.argtypes = [P] * 8
    lib.orc_ellipse.restype = ctypes.c_int
    lib.orc_ellipse.argtypes = [P, ctypes.c_double, P, ctypes.c_double, P, ctypes.c_double, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class OracleResult:
    k: int
    n_nodes: int
    n_struts: int
    # per node
    status: np.ndarray  # int32 [N]
    valence: np.ndarray
    nv: np.ndarray
    ne: np.ndarray
    nc: np.ndarray
    nmesh: np.ndarray
    nfan: np.ndarray
    margin: np.ndarray  # float64 [N]
    margin_kind: np.ndarray  # int32 [N] (MK_* codes of oracle.c)
    kmargin: np.ndarray  # float64 [N, 8]: smallest margin of each kind MK_* = 1..8 (column kind - 1)
    # meta-mesh (node order; per-node offsets from nv / ne)
    vert_off: np.ndarray
    vert_name: np.ndarray  # uint32 [V]
    vert_w: np.ndarray  # float64 [V,3] local to the node
    vert_cond: np.ndarray  # float64 [V,2] root separation, runner-up gap (rho units)
    arc_off: np.ndarray
    arc_int: np.ndarray  # int32 [E,7]: p q vs ve nseg contour full
    arc_dbl: np.ndarray  # float64 [E,11]: o a b t1 t2 (local)
    loop_off: np.ndarray  # int64 [2S+1]
    loop_arc: np.ndarray
    loop_dir: np.ndarray
    adj_off: np.ndarray
    adj: np.ndarray
    # mesh
    mesh: np.ndarray  # float64 [M,3]
    tris: np.ndarray  # int64 [T,3]; bands (strut order) then fans (node order)
    mesh_off: np.ndarray  # int64 [N+1]
    band_off: np.ndarray  # int64 [S+1]
    fan_off: np.ndarray  # int64 [N+1] (relative to the first fan triangle)
    strut_margin: np.ndarray
    strut_status: np.ndarray

    @property
    def n_band(self) -> int:
        return int(self.band_off[-1])

    @property
    def ok(self) -> np.ndarray:
        return self.status == 0


def run(lat, k: int, threads: int | None = None) -> OracleResult:
    """Meta-mesh and triangulate ``lat`` (a latgen.Lattice) at k segments per turn."""
    lib = _load()
    if threads is None:
        threads = os.cpu_count() or 1
    # FP32 lattices are promoted; FP64 arrays (finite differences) are used as given
    f64 = np.asarray(lat.x).dtype == np.float64
    dt = np.float64 if f64 else np.float32
    x = np.ascontiguousarray(lat.x, dtype=dt)
    y = np.ascontiguousarray(lat.y, dtype=dt)
    z = np.ascontiguousarray(lat.z, dtype=dt)
    r = np.ascontiguousarray(lat.radius, dtype=dt)
    sa = np.ascontiguousarray(lat.strut_a, dtype=np.int32)
    sb = np.ascontiguousarray(lat.strut_b, dtype=np.int32)
    N, S = x.shape[0], sa.shape[0]
    entry = lib.orc_run_f64 if f64 else lib.orc_run
    h = entry(N, S, _p(x), _p(y), _p(z), _p(r), _p(sa), _p(sb), int(k), int(threads))
    if not h:
        raise ValueError("oracle rejected the lattice (strut index out of range or k < 1)")
    try:
        sz = np.zeros(7, np.int64)
        lib.orc_sizes(h, _p(sz))
        nV, nE, nC, nM, nB, nF, nL = (int(v) for v in sz)
        cnt = np.zeros((N, 8), np.int32)
        mg = np.zeros(N, np.float64)
        lib.orc_nodes(h, _p(cnt), _p(mg))
        kmg = np.zeros((N, 8), np.float64)
        lib.orc_node_margins(h, _p(kmg))
        vn = np.zeros(nV, np.uint32)
        vw = np.zeros((nV, 3), np.float64)
        vc = np.zeros((nV, 2), np.float64)
        lib.orc_vertices(h, _p(vn), _p(vw), _p(vc))
        ai = np.zeros((nE, 7), np.int32)
        ad = np.zeros((nE, 11), np.float64)
        lib.orc_arcs(h, _p(ai), _p(ad))
        lo = np.zeros(2 * S + 1, np.int64)
        la = np.zeros(max(nL, 1), np.int32)
        ld = np.zeros(max(nL, 1), np.int32)
        lib.orc_loops(h, _p(lo), _p(la), _p(ld))
        aoff = np.zeros(N + 1, np.int64)
        adj = np.zeros(max(int(2 * S), 1), np.int32)
        lib.orc_adjacency(h, _p(aoff), _p(adj))
        mesh = np.zeros((nM, 3), np.float64)
        tris = np.zeros((nB + nF, 3), np.int64)
        moff = np.zeros(N + 1, np.int64)
        boff = np.zeros(S + 1, np.int64)
        foff = np.zeros(N + 1, np.int64)
        smg = np.zeros(S, np.float64)
        sst = np.zeros(S, np.int32)
        lib.orc_mesh(h, _p(mesh), _p(tris), _p(moff), _p(boff), _p(foff), _p(smg), _p(sst))
    finally:
        lib.orc_free(h)
    off = lambda c: np.concatenate([[0], np.cumsum(c.astype(np.int64))])  # noqa: E731
    return OracleResult(
        k=int(k), n_nodes=N, n_struts=S,
        status=cnt[:, 0].copy(), valence=cnt[:, 1].copy(), nv=cnt[:, 2].copy(), ne=cnt[:, 3].copy(),
        nc=cnt[:, 4].copy(), nmesh=cnt[:, 5].copy(), nfan=cnt[:, 6].copy(), margin=mg,
        margin_kind=cnt[:, 7].copy(), kmargin=kmg,
        vert_off=off(cnt[:, 2]), vert_name=vn, vert_w=vw, vert_cond=vc,
        arc_off=off(cnt[:, 3]), arc_int=ai, arc_dbl=ad,
        loop_off=lo, loop_arc=la[:nL], loop_dir=ld[:nL], adj_off=aoff, adj=adj[: 2 * S],
        mesh=mesh, tris=tris, mesh_off=moff, band_off=boff, fan_off=foff,
        strut_margin=smg, strut_status=sst,
    )


def ellipse(c, r0, cp, rp, cq, rq):
    """Eq. 7 ellipse of strut (c -> cp) cut by its auxiliary plane with strut
    (c -> cq).  Returns (o, a, b) local to c, or None if not an ellipse."""
    lib = _load()
    c = np.ascontiguousarray(c, np.float64)
    cp = np.ascontiguousarray(cp, np.float64)
    cq = np.ascontiguousarray(cq, np.float64)
    out = np.zeros(9, np.float64)
    rc = lib.orc_ellipse(_p(c), float(r0), _p(cp), float(rp), _p(cq), float(rq), _p(out))
    if rc < 0:
        return None
    return out[0:3], out[3:6], out[6:9]


# ---------------------------------------------------------------------------
# mesh-level quantities (plain numpy on the oracle's output)


def mesh_area(verts: np.ndarray, tris: np.ndarray) -> float:
    v = verts[tris]
    return float(0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1).sum())


def mesh_volume(verts: np.ndarray, tris: np.ndarray) -> float:
    ref = verts.mean(axis=0) if len(verts) else np.zeros(3)
    v = verts[tris] - ref
    return float(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0)


def mesh_sq(verts: np.ndarray) -> float:
    """Sum of squared norms of the mesh vertices (each stored once)."""
    return float((verts * verts).sum())


# ---------------------------------------------------------------------------
# gradients at fixed topology (the adjoint's reference)
#
# The loss is L = w_area * Area + w_vol * Vol + w_sq * sum |v|^2 over the
# triangle mesh, Vol taken about a fixed point p0.  Its derivative with
# respect to a node coordinate or radius is the limit of difference
# quotients with the mesh topology (labels, arcs, segment counts, triangles)
# held fixed; here it is evaluated by central differences in FP64 with one
# Richardson step, on the stars around the perturbed node, and only where
# the perturbed meshes keep the topology.


def _star_lattice(lat64, centre):
    """Stars of the nodes in ``centre`` with node and strut order kept."""
    import latgen

    sa, sb = lat64.strut_a.astype(np.int64), lat64.strut_b.astype(np.int64)
    cen = np.zeros(lat64.n_nodes, bool)
    cen[centre] = True
    keep = np.nonzero(cen[sa] | cen[sb])[0]
    nodes = np.unique(np.concatenate([sa[keep], sb[keep], np.asarray(centre, np.int64)]))
    nmap = np.full(lat64.n_nodes, -1, np.int64)
    nmap[nodes] = np.arange(len(nodes))
    sub = latgen.Lattice(
        x=lat64.x[nodes].copy(), y=lat64.y[nodes].copy(), z=lat64.z[nodes].copy(),
        radius=lat64.radius[nodes].copy(),
        strut_a=nmap[sa[keep]].astype(np.int32), strut_b=nmap[sb[keep]].astype(np.int32),
    )
    return sub, nodes, nmap


def _local_loss(R, owner_mask_local, weights, p0):
    """Loss terms over the triangles that touch a vertex of an owner node,
    and the squared norms of the owner nodes' vertices (one value per row
    of ``weights``)."""
    node_of = np.repeat(np.arange(R.n_nodes), np.diff(R.mesh_off))
    own_v = owner_mask_local[node_of]
    t = R.tris
    sel = own_v[t].any(axis=1)
    v = R.mesh[t[sel]] - p0
    cr = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0
    sq = (R.mesh[own_v] ** 2).sum()
    return weights @ np.array([area, vol, sq])


def _topology(R, owner_mask_local):
    node_of = np.repeat(np.arange(R.n_nodes), np.diff(R.mesh_off))
    sel = owner_mask_local[node_of][R.tris].any(axis=1)
    t = R.tris[sel]
    return np.stack([node_of[t], t - R.mesh_off[node_of[t]]], -1), R.status[owner_mask_local]


def fd_gradient(lat, k, params, weights=(1.0, 0.0, 0.0), h=1e-6, p0=None):
    """Derivative of the loss with respect to each (node, component)
    in ``params`` (component 0..2: x, y, z; 3: radius) at fixed topology.
    ``weights`` is one (w_area, w_vol, w_sq) or a list of them.  Returns
    (values [len(params)] or [len(params), len(weights)], ok) where ok is
    False where a perturbation changed the topology (or left a node
    unmeshed)."""
    import latgen

    lat64 = latgen.Lattice(
        x=np.asarray(lat.x, np.float64), y=np.asarray(lat.y, np.float64), z=np.asarray(lat.z, np.float64),
        radius=np.asarray(lat.radius, np.float64), strut_a=lat.strut_a, strut_b=lat.strut_b,
    )
    if p0 is None:
        p0 = np.zeros(3)
    sa, sb = lat64.strut_a.astype(np.int64), lat64.strut_b.astype(np.int64)
    nbr = [[] for _ in range(lat64.n_nodes)]
    for a_, b_ in zip(sa, sb):
        nbr[a_].append(b_)
        nbr[b_].append(a_)
    weights = np.asarray(weights, np.float64)
    single = weights.ndim == 1
    weights = np.atleast_2d(weights)
    out = np.zeros((len(params), len(weights)))
    ok = np.ones(len(params), bool)
    for i, (node, comp) in enumerate(params):
        owners = np.unique(np.array([node] + nbr[node], np.int64))
        ring = np.unique(np.concatenate([owners] + [np.array(nbr[o], np.int64) for o in owners]))
        sub, nodes, nmap = _star_lattice(lat64, ring)
        own_local = np.zeros(len(nodes), bool)
        own_local[nmap[owners]] = True
        j = nmap[node]
        field = (sub.x, sub.y, sub.z, sub.radius)[comp]
        base = field[j]
        R0 = run(sub, k, threads=1)
        topo0, st0 = _topology(R0, own_local)
        vals = {}
        for step in (h, -h, 2 * h, -2 * h):
            field[j] = base + step
            Rs = run(sub, k, threads=1)
            field[j] = base
            topo, st = _topology(Rs, own_local)
            if topo.shape != topo0.shape or not np.array_equal(topo, topo0) or (st != 0).any() or (st0 != 0).any():
                ok[i] = False
                break
            vals[step] = _local_loss(Rs, own_local, weights, p0)
        if not ok[i]:
            continue
        d1 = (vals[h] - vals[-h]) / (2 * h)
        d2 = (vals[2 * h] - vals[-2 * h]) / (4 * h)
        out[i] = (4 * d1 - d2) / 3  # Richardson: O(h^4)
    return (out[:, 0] if single else out), ok


# ---------------------------------------------------------------------------
# per-chunk counts and order-independent hashes (the sink mode's reference)

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_G = np.uint64(0x9E3779B97F4A7C15)


def _mix(z):
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def tri_keys(v):
    """Keys of triangles given as uint64 vertex ids [T, 3] (orientation kept,
    smallest id rotated first)."""
    r = np.argmin(v, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    w = np.take_along_axis(v, idx, axis=1)
    with np.errstate(over="ignore"):
        return _mix(_mix(_mix(w[:, 0] + _G) ^ w[:, 1]) ^ w[:, 2])


def sink_words(R, chunk_nodes, strut_a, strut_b):
    """Per chunk of node ids: [triangles, sum of triangle keys, mesh vertices,
    0 (vertex keys need the GPU's FP32 positions), sums of round(2^20 x),
    round(2^20 y), round(2^20 z), nodes without a mesh] as uint64 [C, 8]."""
    N = R.n_nodes
    nch = max((N + chunk_nodes - 1) // chunk_nodes, 1)
    out = np.zeros((nch, 8), np.uint64)
    node_of = np.repeat(np.arange(N), np.diff(R.mesh_off))
    local = np.arange(len(node_of)) - R.mesh_off[node_of]
    vid = (node_of.astype(np.uint64) << np.uint64(21)) | local.astype(np.uint64)
    keys = tri_keys(vid[R.tris]) if len(R.tris) else np.zeros(0, np.uint64)
    # owner node of each triangle: bands by the strut's lower node, fans by node
    sa, sb = np.asarray(strut_a, np.int64), np.asarray(strut_b, np.int64)
    lo = np.minimum(sa, sb)
    band_owner = np.repeat(lo, np.diff(R.band_off))
    fan_owner = np.repeat(np.arange(N), np.diff(R.fan_off))
    owner = np.concatenate([band_owner, fan_owner])
    ch = owner // chunk_nodes
    out[:, 0] = np.bincount(ch, minlength=nch).astype(np.uint64)
    for c in range(nch):
        with np.errstate(over="ignore"):
            out[c, 1] = np.sum(keys[ch == c], dtype=np.uint64)
    vch = node_of // chunk_nodes
    out[:, 2] = np.bincount(vch, minlength=nch).astype(np.uint64)
    fix = np.rint(R.mesh * 1048576.0).astype(np.int64)
    for d in range(3):
        for c in range(nch):
            with np.errstate(over="ignore"):
                out[c, 4 + d] = np.sum(fix[vch == c, d].view(np.uint64), dtype=np.uint64)
    bad = np.nonzero(R.status != 0)[0]
    out[:, 7] = np.bincount(bad // chunk_nodes, minlength=nch).astype(np.uint64)
    return out
