"""Seeded synthetic strut lattices.

This module only builds inputs: node positions, nodal-sphere radii and strut
endpoint pairs.  It contains none of the meta-meshing arithmetic, so both the
FP64 oracle (``oracle/``) and the GPU path draw identical inputs from it.

Random numbers are counter based: a value is SplitMix64 applied to a key made
from (seed, entity id, field), uniform = (z >> 11) * 2**-53.  Every quantity is
generated in FP64 and rounded once to FP32; the FP32 arrays are the lattice.

Lattice families stand in for the paper's tetgen-built test lattices (Sec. 6),
which are not available: simple cubic, body-centred cubic (corner + body-centre
nodes joined by the 8 half body diagonals of each cell) and octet truss (FCC
sites joined to their 12 nearest neighbours).  Struts are round cones tangent to
the two nodal spheres (Sec. 4.1), so one radius per node defines every strut.
"""

from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Lattice",
    "uniform",
    "cubic",
    "bcc",
    "octet",
    "lattice_from_arrays",
    "two_strut",
    "star",
    "knn",
    "union",
    "config",
    "parts",
]

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)

FIELD_JX, FIELD_JY, FIELD_JZ, FIELD_R = 0, 1, 2, 3


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, ids: np.ndarray, field: int) -> np.ndarray:
    """U[0,1) in FP64 for each entity id, keyed by (seed, id, field)."""
    ids = np.asarray(ids, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = _splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(field))
        z = _splitmix64(ids ^ k)
        z = _splitmix64(z + np.uint64(field + 1))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclasses.dataclass
class Lattice:
    x: np.ndarray  # float32 [N]
    y: np.ndarray  # float32 [N]
    z: np.ndarray  # float32 [N]
    radius: np.ndarray  # float32 [N]   nodal-sphere radius per node
    strut_a: np.ndarray  # int32 [S]
    strut_b: np.ndarray  # int32 [S]
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_struts(self) -> int:
        return int(self.strut_a.shape[0])

    def xyz64(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1).astype(np.float64)


def lattice_from_arrays(xyz, radius, struts, name="") -> Lattice:
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3).astype(np.float32)
    radius = np.broadcast_to(np.asarray(radius, dtype=np.float64), (xyz.shape[0],))
    struts = np.asarray(struts, dtype=np.int64).reshape(-1, 2)
    return Lattice(
        x=np.ascontiguousarray(xyz[:, 0]),
        y=np.ascontiguousarray(xyz[:, 1]),
        z=np.ascontiguousarray(xyz[:, 2]),
        radius=np.ascontiguousarray(radius.astype(np.float32)),
        strut_a=np.ascontiguousarray(struts[:, 0].astype(np.int32)),
        strut_b=np.ascontiguousarray(struts[:, 1].astype(np.int32)),
        name=name,
    )


def _radii(seed, n, spec, cell):
    ids = np.arange(n, dtype=np.uint64)
    if np.isscalar(spec):
        return np.full(n, float(spec) * cell)
    kind = spec[0]
    if kind == "uniform":  # ("uniform", lo, hi): U[lo, hi] * cell
        u = uniform(seed, ids, FIELD_R)
        return (spec[1] + (spec[2] - spec[1]) * u) * cell
    if kind == "rel":  # ("rel", base, frac): base * (1 + U[-frac, frac]) * cell
        u = uniform(seed, ids, FIELD_R)
        return spec[1] * (1.0 + spec[2] * (2.0 * u - 1.0)) * cell
    raise ValueError(f"unknown radius spec {spec!r}")


def _jitter(seed, n, jitter, cell):
    if jitter == 0:
        return np.zeros((n, 3))
    ids = np.arange(n, dtype=np.uint64)
    out = np.empty((n, 3))
    for c, f in enumerate((FIELD_JX, FIELD_JY, FIELD_JZ)):
        out[:, c] = (2.0 * uniform(seed, ids, f) - 1.0) * jitter * cell
    return out


def _finish(pos, seed, radius, jitter, cell, struts, name):
    n = pos.shape[0]
    pos = pos * cell + _jitter(seed, n, jitter, cell)
    rad = _radii(seed, n, radius, cell)
    return lattice_from_arrays(pos, rad, struts, name=name)


def cubic(n, radius=0.1, jitter=0.0, seed=1, cell=1.0) -> Lattice:
    """Simple cubic lattice of n^3 cells: (n+1)^3 nodes, 3 n (n+1)^2 struts."""
    m = n + 1
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    pos = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    nid = lambda a, b, c: a + m * (b + m * c)  # noqa: E731
    st = []
    ii, jj, kk = i.ravel(), j.ravel(), k.ravel()
    for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        ok = (ii + di < m) & (jj + dj < m) & (kk + dk < m)
        st.append(np.stack([nid(ii[ok], jj[ok], kk[ok]), nid(ii[ok] + di, jj[ok] + dj, kk[ok] + dk)], 1))
    return _finish(pos, seed, radius, jitter, cell, np.concatenate(st), f"cubic{n}")


def bcc(n, radius=0.1, jitter=0.0, seed=1, cell=1.0, order="grid") -> Lattice:
    """Body-centred cubic lattice of n^3 cells.

    Nodes: (n+1)^3 cell corners and n^3 body centres.  Struts: the 8 half
    body diagonals of every cell (corner -> centre), 8 n^3 in total, cell by
    cell.  ``order`` numbers the nodes: "grid" lists all corners (x fastest),
    then all centres; "layer" lists layer z = 0, 1, ..., n, each as its corners
    followed by the centres just above it, so that a range of consecutive node
    ids is a slab whose only higher-id neighbours outside it are the next
    corner layer.  Random draws are keyed by the node id in either order.
    """
    m = n + 1
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    corners = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = i.ravel(), j.ravel(), k.ravel()
    centres = np.stack([ci, cj, ck], axis=1).astype(np.float64) + 0.5
    if order == "grid":
        corner_id = lambda a, b, c: a + m * (b + m * c)  # noqa: E731
        cid = m**3 + ci + n * (cj + n * ck)
        pos = np.concatenate([corners, centres])
    elif order == "layer":
        B = m * m + n * n  # ids per layer below the top one
        corner_id = lambda a, b, c: c * B + a + m * b  # noqa: E731
        cid = ck * B + m * m + ci + n * cj
        pos = np.empty((m**3 + n**3, 3))
        pos[corner_id(corners[:, 0].astype(np.int64), corners[:, 1].astype(np.int64),
                      corners[:, 2].astype(np.int64))] = corners
        pos[cid] = centres
    else:
        raise ValueError(f"unknown node order {order!r}")
    st = np.empty((n**3, 8, 2), dtype=np.int64)
    for c in range(8):
        di, dj, dk = c & 1, (c >> 1) & 1, (c >> 2) & 1
        st[:, c, 0] = corner_id(ci + di, cj + dj, ck + dk)
        st[:, c, 1] = cid
    return _finish(pos, seed, radius, jitter, cell, st.reshape(-1, 2), f"bcc{n}" + ("" if order == "grid" else "L"))


def octet(n, radius=0.1, jitter=0.0, seed=1, cell=1.0) -> Lattice:
    """Octet-truss lattice of n^3 cells: FCC sites joined to nearest neighbours.

    Sites are the points of the doubled grid [0, 2n]^3 with even coordinate sum
    (cell corners and face centres); struts join sites at distance sqrt(2)/2.
    """
    g = 2 * n + 1
    Z, Y, X = np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    keep = (X + Y + Z) % 2 == 0
    lin = np.full(g**3, -1, dtype=np.int64)
    lin[keep] = np.arange(int(keep.sum()))
    X, Y, Z = X[keep], Y[keep], Z[keep]
    pos = np.stack([X, Y, Z], axis=1).astype(np.float64) * 0.5
    offs = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]
    st = []
    for dx, dy, dz in offs:
        X2, Y2, Z2 = X + dx, Y + dy, Z + dz
        ok = (X2 >= 0) & (X2 < g) & (Y2 >= 0) & (Y2 < g) & (Z2 >= 0) & (Z2 < g)
        a = lin[X[ok] + g * (Y[ok] + g * Z[ok])]
        b = lin[X2[ok] + g * (Y2[ok] + g * Z2[ok])]
        st.append(np.stack([np.minimum(a, b), np.maximum(a, b)], 1))
    return _finish(pos, seed, radius, jitter, cell, np.concatenate(st), f"octet{n}")


def knn(n, kn, radius=0.1, seed=1, cell=1.0) -> Lattice:
    """Random lattice: n^3 points uniform in an n^3-cell box (density one per
    cell, a binomial stand-in for a Poisson process), each joined to its kn
    nearest neighbours, symmetrised (an edge if either end chose it)."""
    from scipy.spatial import cKDTree

    N = n**3
    ids = np.arange(N, dtype=np.uint64)
    pos = np.stack([uniform(seed, ids, f) for f in (FIELD_JX, FIELD_JY, FIELD_JZ)], axis=1) * n
    kk = min(kn, N - 1)
    if kk < 1:
        return _finish(pos, seed, radius, 0.0, cell, np.zeros((0, 2), np.int64), f"knn{n}_{kn}")
    _, nb = cKDTree(pos).query(pos, k=kk + 1)
    a = np.repeat(np.arange(N), kk)
    b = nb[:, 1:].ravel()
    e = np.unique(np.stack([np.minimum(a, b), np.maximum(a, b)], 1), axis=0)
    return _finish(pos, seed, radius, 0.0, cell, e, f"knn{n}_{kn}")


FIELD_PART = 16  # fields of the per-part draws


def _part_specs(n_parts, seed, n_max, n_min):
    """(kind, cells, resolution, k-NN degree, seed) of every part."""
    pid = np.arange(n_parts, dtype=np.uint64)
    u = [uniform(seed, pid, FIELD_PART + f) for f in range(4)]
    out = []
    for p in range(n_parts):
        kind = min(int(u[0][p] * 4), 3)
        n = n_min + min(int(u[1][p] * (n_max - n_min + 1)), n_max - n_min)
        res = (8, 16, 32)[min(int(u[2][p] * 3), 2)]
        kn = 3 + min(int(u[3][p] * 18), 17)
        out.append((kind, n, res, kn, seed * 1000003 + p))
    return out


def _make_part(spec):
    kind, n, res, kn, s = spec
    rad = ("uniform", 0.04, 0.12)
    if kind == 0:
        lat = cubic(n, radius=rad, jitter=0.0, seed=s)
    elif kind == 1:
        lat = bcc(n, radius=rad, jitter=0.0, seed=s)
    elif kind == 2:
        lat = octet(n, radius=rad, jitter=0.0, seed=s)
    else:
        lat = knn(n, kn, radius=rad, seed=s)
    return lat, res


def parts(n_parts=512, seed=1, n_max=64, n_min=4, workers=1, start="fork"):
    """The batched workload: ``n_parts`` lattice parts, each a cubic, BCC,
    octet or random k-NN lattice (uniform choice) with cells per side drawn
    from {n_min..n_max}, k-NN degree from {3..20}, node radii U[0.04, 0.12],
    and a resolution from {8, 16, 32}.  Returns a list of (Lattice, k).
    ``workers`` > 1 builds the parts in that many processes (same result),
    started by ``start`` ("spawn" from a process that has used the GPU)."""
    specs = _part_specs(n_parts, seed, n_max, n_min)
    if workers <= 1 or n_parts < 2:
        return [_make_part(s) for s in specs]
    import multiprocessing as mp

    # largest parts first, so the pool's tail is short
    order = sorted(range(n_parts), key=lambda i: -specs[i][1])
    with mp.get_context(start).Pool(workers) as pool:
        made = pool.map(_make_part, [specs[i] for i in order], chunksize=1)
    out = [None] * n_parts
    for i, r in zip(order, made):
        out[i] = r
    return out


def union(lattices):
    """Disjoint union of lattices (node ids offset part by part); returns the
    union and the node offsets of the parts [n_parts + 1]."""
    off = np.zeros(len(lattices) + 1, np.int64)
    soff = np.zeros(len(lattices) + 1, np.int64)
    for i, lat in enumerate(lattices):
        off[i + 1] = off[i] + lat.n_nodes
        soff[i + 1] = soff[i] + lat.n_struts
    if off[-1] >= 2**31:
        raise ValueError("union has 2^31 nodes or more")
    cat = lambda f: np.concatenate([getattr(l, f) for l in lattices])  # noqa: E731
    sa = np.empty(soff[-1], np.int32)
    sb = np.empty(soff[-1], np.int32)
    for i, l in enumerate(lattices):
        np.add(l.strut_a, np.int32(off[i]), out=sa[soff[i]:soff[i + 1]], dtype=np.int32)
        np.add(l.strut_b, np.int32(off[i]), out=sb[soff[i]:soff[i + 1]], dtype=np.int32)
    return Lattice(x=cat("x"), y=cat("y"), z=cat("z"), radius=cat("radius"), strut_a=sa, strut_b=sb,
                   name=f"union{len(lattices)}"), off


def two_strut(angle_deg=90.0, length=1.0, radius=0.1, radii=None) -> Lattice:
    """Three nodes: a centre node at the origin joined to two free ends.

    The first strut runs along +x; the second lies in the xy plane at
    ``angle_deg`` from the first.  ``radii`` overrides (centre, end1, end2).
    """
    a = np.deg2rad(angle_deg)
    xyz = [(0.0, 0.0, 0.0), (length, 0.0, 0.0), (length * np.cos(a), length * np.sin(a), 0.0)]
    r = radii if radii is not None else (radius, radius, radius)
    return lattice_from_arrays(xyz, r, [(0, 1), (0, 2)], name=f"two_strut{angle_deg}")


def star(directions, length=1.0, radius=0.1, radii=None) -> Lattice:
    """A centre node (id 0) joined to one free end per direction vector."""
    d = np.asarray(directions, dtype=np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    xyz = np.concatenate([np.zeros((1, 3)), d * length])
    r = radii if radii is not None else radius
    st = [(0, i + 1) for i in range(d.shape[0])]
    return lattice_from_arrays(xyz, r, st, name=f"star{d.shape[0]}")


def config(i: int, seed: int = 1, scale: int | None = None) -> Lattice:
    """The synthetic workloads, by number.

    1: simple cubic 6^3, radius 0.1, jitter 0.02 (resolution k = 8).
    2: BCC 64^3, node radii U[0.05, 0.12], jitter 0.05 (k = 16).
    3: BCC 512^3, node radii 0.08 (1 + U[-0.1, 0.1]), no jitter (k = 12), nodes
       numbered layer by layer (sink-mode chunks are slabs).
    4: octet 32^3, node radii U[0.04, 0.10], jitter 0.03 (k = 16).
    ``scale`` replaces the cell count n (same family and distributions).
    """
    if i == 1:
        return cubic(scale or 6, radius=0.1, jitter=0.02, seed=seed)
    if i == 2:
        return bcc(scale or 64, radius=("uniform", 0.05, 0.12), jitter=0.05, seed=seed)
    if i == 3:
        return bcc(scale or 512, radius=("rel", 0.08, 0.1), jitter=0.0, seed=seed, order="layer")
    if i == 4:
        return octet(scale or 32, radius=("uniform", 0.04, 0.10), jitter=0.03, seed=seed)
    raise ValueError(f"no config {i}")


CONFIG_K = {1: 8, 2: 16, 3: 12, 4: 16}
