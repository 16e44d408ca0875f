"""Pins of the FP64 oracle against facts fixed by geometry, not by the oracle.

* hand-derived worked cases (tests/golden/worked_cases.json): L-joint and
  orthogonal corner: vertex names and positions, arc spans, semi-axes;
* closed-form limits: band (strut) area of the L-joint, corner and conical
  capsule, capsule fan area and enclosed volume, approached at O(k^-2);
* Eq. 7 against an independent test: every point of the ellipse lies on both
  round cones, measured by distance to the strut axis;
* brute-force classification: points of kept arcs lie on the boundary of the
  union of round cones (the solid itself, evaluated as a union of linearly
  interpolated spheres), points of trimmed parts of each conic do not;
* invariants on whole lattices: per-node Euler relation, watertight and
  consistently oriented output, Euler characteristic 2N - 2S, positive
  volume, triangle count 2 * sum of segment counts;
* inside/outside of the mesh (generalised winding number) against the exact
  solid away from the surface.
"""

import json
import math
import os

import numpy as np
import pytest

import latgen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "worked_cases.json")))


def _name(p, q, r, root):
    return (p << 24) | (q << 16) | (r << 8) | root


# ---------------------------------------------------------------------------
# independent geometry: the solid as a union of round cones


def cone_distance(x, c0, r0, c1, r1, n=64):
    """min over t in [0,1] of |x - c(t)| - r(t) for linearly interpolated
    spheres; negative inside the round cone (convex hull of the two balls).
    The function of t is convex: golden-section search, vectorised over x."""
    x = np.atleast_2d(x)
    lo = np.zeros(len(x))
    hi = np.ones(len(x))
    f = lambda t: np.linalg.norm(x - (c0 + t[:, None] * (c1 - c0)), axis=1) - (r0 + t * (r1 - r0))  # noqa
    gr = (math.sqrt(5) - 1) / 2
    for _ in range(n):
        a = hi - gr * (hi - lo)
        b = lo + gr * (hi - lo)
        fa, fb = f(a), f(b)
        left = fa < fb
        hi = np.where(left, b, hi)
        lo = np.where(left, lo, a)
    t = 0.5 * (lo + hi)
    return np.minimum(np.minimum(f(t), f(np.zeros(len(x)))), f(np.ones(len(x))))


def solid_distance(lat, x):
    """Signed distance-like function of the whole lattice solid (< 0 inside)."""
    xyz = lat.xyz64()
    r = lat.radius.astype(np.float64)
    d = np.full(len(np.atleast_2d(x)), np.inf)
    for a, b in zip(lat.strut_a, lat.strut_b):
        d = np.minimum(d, cone_distance(x, xyz[a], r[a], xyz[b], r[b]))
    return d


def winding_number(verts, tris, pts):
    """Generalised winding number of a closed triangle mesh (solid angle sum)."""
    out = np.zeros(len(pts))
    for i in range(0, len(pts), 256):
        p = pts[i : i + 256][:, None, :]
        a = verts[tris[:, 0]][None] - p
        b = verts[tris[:, 1]][None] - p
        c = verts[tris[:, 2]][None] - p
        la, lb, lc = (np.linalg.norm(v, axis=2) for v in (a, b, c))
        num = np.einsum("ijk,ijk->ij", a, np.cross(b, c))
        den = la * lb * lc + np.einsum("ijk,ijk->ij", a, b) * lc + np.einsum("ijk,ijk->ij", b, c) * la
        den += np.einsum("ijk,ijk->ij", c, a) * lb
        out[i : i + 256] = (2 * np.arctan2(num, den)).sum(axis=1) / (4 * math.pi)
    return out


def mesh_checks(R, lat):
    """Watertight + consistently oriented, Euler characteristic, volume > 0."""
    t = R.tris
    nm = len(R.mesh)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = e[:, 0] * nm + e[:, 1]
    rkey = e[:, 1] * nm + e[:, 0]
    assert len(np.unique(key)) == len(key), "a directed edge is used twice"
    assert np.isin(rkey, key).all(), "an edge has no oppositely oriented twin"
    und = np.unique(np.sort(e, axis=1)[:, 0] * nm + np.sort(e, axis=1)[:, 1])
    used = len(np.unique(t))
    assert used == nm, "unreferenced mesh vertex"
    chi = nm - len(und) + len(t)
    assert chi == 2 * lat.n_nodes - 2 * lat.n_struts
    import oracle

    assert oracle.mesh_volume(R.mesh, R.tris) > 0


# ---------------------------------------------------------------------------
# worked cases


@pytest.mark.parametrize("case", ["ljoint", "corner"])
def test_worked_case_structure(orc, case):
    g = GOLD[case]
    lat = latgen.star(g["directions"], length=g["length"], radius=g["rho"])
    R = orc.run(lat, 9)
    assert (R.status == 0).all()
    sc = float(np.float32(g["rho"])) / g["rho"]  # inputs are rounded to FP32
    c = g["centre"]
    assert (R.nv[0], R.ne[0], R.nc[0]) == (c["nv"], c["ne"], c["nc"])
    names = R.vert_name[: R.nv[0]]
    w = R.vert_w[: R.nv[0]]
    for (p, q, r, root), pos in g["vertices"]:
        i = np.nonzero(names == _name(p, q, r, root))[0]
        assert len(i) == 1, f"vertex {(p, q, r, root)} missing"
        np.testing.assert_allclose(w[i[0]], np.array(pos) * sc, atol=1e-15)
    ai = R.arc_int[: R.ne[0]]
    ad = R.arc_dbl[: R.ne[0]]
    for want in g["arcs"]:
        j = np.nonzero((ai[:, 0] == want["p"]) & (ai[:, 1] == want["q"]))[0]
        assert len(j) == 1
        span = ad[j[0], 10] - ad[j[0], 9]
        assert abs(span - want["span"]) < 1e-12
        if "semi_major" in want:
            a, b = ad[j[0], 3:6], ad[j[0], 6:9]
            assert abs(np.linalg.norm(a) - want["semi_major"] * sc) < 1e-15
            assert abs(np.linalg.norm(b) - want["semi_minor"] * sc) < 1e-15
            assert abs(a @ b) < 1e-14
    for pq, n in g["nseg_k9"].items():
        if pq.startswith("_"):
            continue
        p, q = (int(x) for x in pq.split("-"))
        j = np.nonzero((ai[:, 0] == p) & (ai[:, 1] == q))[0]
        assert ai[j[0], 4] == n


def test_hole_centre_closed_form(orc):
    """Eq. 13 on an asymmetric lune (two cones): the contour is two circular
    arcs of different radii; the sum of N+1 equally spaced points on an arc
    has the closed form (Dirichlet kernel) sin((N+1) d/2) / sin(d/2) times
    the unit vector at the mid angle, so the projected barycentre follows
    without summing points."""
    import oracle

    ang = np.deg2rad(100.0)
    e1 = np.array([1.0, 0, 0])
    e2 = np.array([np.cos(ang), np.sin(ang), 0.0])
    lat = latgen.lattice_from_arrays([(0, 0, 0), tuple(e1), tuple(e2 * 0.9)], [0.1, 0.06, 0.15], [(0, 1), (0, 2)])
    k = 11
    R = orc.run(lat, k)
    assert R.status[0] == 0 and R.nc[0] == 1
    xyz = lat.xyz64()
    rad = lat.radius.astype(np.float64)
    rho = rad[0]
    struts = [(xyz[0], rad[0], xyz[i], rad[i]) for i in (1, 2)]
    # the two vertices: on the sphere and on both tangency planes e.w = rho s
    es, ss = [], []
    for i in (1, 2):
        L = np.linalg.norm(xyz[i])
        es.append(xyz[i] / L)
        ss.append((rho - rad[i]) / L)
    n = np.cross(es[0], es[1])
    A = np.stack([es[0], es[1]])
    w0 = np.linalg.lstsq(A, rho * np.array(ss), rcond=None)[0]
    lam = np.sqrt((rho * rho - w0 @ w0) / (n @ n))
    verts = [w0 - lam * n, w0 + lam * n]
    total = np.zeros(3)
    count = 0
    for i in range(2):
        e, s = es[i], ss[i]
        ctr = rho * s * e
        Rc = rho * np.sqrt(1 - s * s)
        u = verts[0] - ctr
        u /= np.linalg.norm(u)
        v = np.cross(e, u)
        phib = np.arctan2((verts[1] - ctr) @ v, (verts[1] - ctr) @ u) % (2 * np.pi)
        # the kept arc is the one outside the other strut
        mid = ctr + Rc * (np.cos(phib / 2) * u + np.sin(phib / 2) * v)
        other = struts[1 - i]
        if cone_distance(mid + xyz[0], *other)[0] < 0:
            lo, span = phib, 2 * np.pi - phib
        else:
            lo, span = 0.0, phib
        N = int(np.floor(k * span / (2 * np.pi))) + 1
        d = span / N
        kern = np.sin((N + 1) * d / 2) / np.sin(d / 2)
        pm = lo + span / 2
        total += (N + 1) * ctr + Rc * kern * (np.cos(pm) * u + np.sin(pm) * v)
        count += N + 1
    total -= verts[0] + verts[1]  # the two vertices were counted twice
    count -= 2
    b = total / count
    apex = rho * b / np.linalg.norm(b)
    got = R.mesh[R.mesh_off[1] - 1] - xyz[0]
    np.testing.assert_allclose(got, apex, atol=1e-14)


@pytest.mark.parametrize("case", ["ljoint", "corner"])
def test_band_area_converges_to_closed_form(orc, case):
    g = GOLD[case]
    lat = latgen.star(g["directions"], length=g["length"], radius=g["rho"])
    rho32 = float(np.float32(g["rho"]))
    # the closed form at the FP32-rounded radius the oracle actually sees
    exact = g["band_area_limit"]["value"] + (rho32 - g["rho"]) * (
        len(g["directions"]) * 2 * math.pi * g["length"])
    exact -= (rho32**2 - g["rho"] ** 2) * (4.0 if case == "ljoint" else 3 * (2 + math.sqrt(2)))
    errs = []
    import oracle

    for k in (17, 33, 65, 129):
        R = orc.run(lat, k)
        errs.append(exact - oracle.mesh_area(R.mesh, R.tris[: R.n_band]))
    errs = np.array(errs)
    assert (errs > 0).all()  # inscribed polygons lose area
    ratios = errs[:-1] / errs[1:]
    assert np.all((ratios > 3.0) & (ratios < 5.0)), ratios  # O(k^-2)
    assert errs[-1] / exact < 1e-3


def test_capsule_cone_closed_forms(orc):
    """Round cone between two free ends: band = frustum lateral area, fans =
    cones from the poles over the tangency circles, volume = frustum + cones."""
    import oracle

    d = np.array([1.0, 0.3, 0.2])
    d /= np.linalg.norm(d)
    lat = latgen.lattice_from_arrays([(0, 0, 0), tuple(d)], [0.1, 0.06], [(0, 1)])
    ra, rb = (float(v) for v in lat.radius)  # FP32-rounded inputs
    L = float(np.linalg.norm(lat.xyz64()[1]))
    s = (ra - rb) / L
    kap = math.sqrt(1 - s * s)
    band = math.pi * kap * (ra + rb) * math.sqrt(L * L - (ra - rb) ** 2)
    fan_a = math.pi * ra * kap * ra * math.sqrt(2 + 2 * s)
    fan_b = math.pi * rb * kap * rb * math.sqrt(2 - 2 * s)
    hf = L * kap * kap
    r1, r2 = ra * kap, rb * kap
    vol = math.pi * hf * (r1 * r1 + r1 * r2 + r2 * r2) / 3
    vol += math.pi * r1 * r1 * ra * (1 + s) / 3 + math.pi * r2 * r2 * rb * (1 - s) / 3
    prev = None
    for k in (16, 32, 64, 128):
        R = orc.run(lat, k)
        assert (R.status == 0).all()
        # full tangency circles get k segments (Eq. 11 capped at one turn):
        # per node one vertex, k - 1 interior points, one hole centre
        assert len(R.mesh) == 2 * (k + 1) and len(R.tris) == 4 * k
        nb = R.n_band
        eb = band - oracle.mesh_area(R.mesh, R.tris[:nb])
        ef = (fan_a + fan_b) - oracle.mesh_area(R.mesh, R.tris[nb:])
        ev = vol - oracle.mesh_volume(R.mesh, R.tris)
        for e in (eb, ef, ev):
            assert e > 0
        if prev is not None:
            for e, ep in zip((eb, ef, ev), prev):
                assert 3.5 < ep / e < 4.5
        prev = (eb, ef, ev)
    assert eb / band < 1e-3 and ev / vol < 1e-3


def test_free_end_fan_apex_on_hole(orc):
    """Eq. 13 reading: when the node sphere is the larger one the contour
    barycentre lies on the strut side; the apex must still land on the hole."""
    lat = latgen.lattice_from_arrays([(0, 0, 0), (1, 0, 0)], [0.12, 0.05], [(0, 1)])
    R = orc.run(lat, 16)
    apex0 = R.mesh[R.mesh_off[1] - 1]  # hole centre is the last local vertex
    r = lat.radius.astype(np.float64)
    np.testing.assert_allclose(apex0, [-r[0], 0, 0], atol=1e-15)
    apex1 = R.mesh[R.mesh_off[2] - 1]
    np.testing.assert_allclose(apex1, [1 + r[1], 0, 0], atol=1e-15)


# ---------------------------------------------------------------------------
# Eq. 7 against the round cones themselves


def _axis_dist_minus_radius(x, c0, r0, c1, r1):
    """Distance of x from the cone surface along the radial direction, using
    only the axis line and the linear radius profile of the tangent cone."""
    L = np.linalg.norm(c1 - c0)
    e = (c1 - c0) / L
    s = (r0 - r1) / L
    kap = math.sqrt(1 - s * s)
    z = (x - c0) @ e
    rad = np.linalg.norm((x - c0) - np.outer(z, e), axis=1)
    rz = r0 * kap - (s / kap) * (z - r0 * s)
    return rad - rz


def test_eq7_ellipse_lies_on_both_cones(orc):
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(300):
        c = rng.normal(size=3)
        r0 = rng.uniform(0.05, 0.15)
        dp, dq = rng.normal(size=3), rng.normal(size=3)
        dp /= np.linalg.norm(dp)
        dq /= np.linalg.norm(dq)
        if dp @ dq > 0.8:
            continue
        cp = c + dp * rng.uniform(0.6, 1.5)
        cq = c + dq * rng.uniform(0.6, 1.5)
        rp, rq = rng.uniform(0.05, 0.15), rng.uniform(0.05, 0.15)
        res = orc.ellipse(c, r0, cp, rp, cq, rq)
        if res is None:
            continue
        o, a, b = res
        t = np.linspace(0, 2 * np.pi, 37)
        x = c + o + np.outer(np.sin(t), a) + np.outer(np.cos(t), b)
        assert np.abs(_axis_dist_minus_radius(x, c, r0, cp, rp)).max() < 1e-12
        assert np.abs(_axis_dist_minus_radius(x, c, r0, cq, rq)).max() < 1e-12
        assert abs(a @ b) < 1e-12 * max(1, a @ a)  # principal axes
        assert np.linalg.norm(a) >= np.linalg.norm(b) - 1e-14
        nrm = np.cross(a, b)
        assert np.abs((x - c - o) @ nrm).max() < 1e-13  # planar
        checked += 1
    assert checked > 150


def test_eq7_matches_quadric_section_eigensystem(orc):
    """The plane section of a cone, written as a quadratic form in plane
    coordinates, has principal axes along its eigenvectors; compare."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        c = np.zeros(3)
        r0 = 0.1
        dp = np.array([1.0, 0, 0])
        dq = rng.normal(size=3)
        dq /= np.linalg.norm(dq)
        if dp @ dq > 0.5:
            continue
        rp, rq = rng.uniform(0.06, 0.14, size=2)
        cp, cq = dp * 1.0, dq * 0.9
        res = orc.ellipse(c, r0, cp, rp, cq, rq)
        if res is None:
            continue
        o, a, b = res
        n = np.cross(a, b)
        n /= np.linalg.norm(n)
        # plane basis and points of the cone p in the plane: solve on rays
        u1 = np.cross(n, [0.3, 0.5, 0.7])
        u1 /= np.linalg.norm(u1)
        u2 = np.cross(n, u1)
        # quadric of cone p: |w|^2 - r0^2 - P^2 with P from the tangent cone
        Lp = np.linalg.norm(cp)
        e = cp / Lp
        s = (r0 - rp) / Lp
        kap = math.sqrt(1 - s * s)
        g, h = e / kap, r0 * s / kap
        # restrict w = o + x u1 + y u2 : Q(x,y) = [x y 1] M [x y 1]^T
        B = np.stack([u1, u2, o], axis=1)  # 3x3 (columns)
        M = B.T @ B - np.outer(B.T @ g, B.T @ g)
        M[2, 2] -= r0 * r0
        pv = B.T @ g
        M[2, :] += h * pv
        M[:, 2] += h * pv
        M[2, 2] -= h * h
        # centre of the conic is where the gradient vanishes (o itself -> 0)
        ctr = np.linalg.solve(M[:2, :2], -M[:2, 2])
        assert np.linalg.norm(ctr) < 1e-10
        evals, evecs = np.linalg.eigh(M[:2, :2])
        k0 = -M[2, 2] + M[:2, 2] @ ctr
        semi = np.sqrt(k0 / evals)  # along the eigenvectors
        ax = sorted(semi)[::-1]
        assert abs(ax[0] - np.linalg.norm(a)) < 1e-10
        assert abs(ax[1] - np.linalg.norm(b)) < 1e-10
        major = evecs[:, np.argmin(evals)]
        dirm = major[0] * u1 + major[1] * u2
        assert abs(abs(dirm @ a) / np.linalg.norm(a) - 1) < 1e-9


# ---------------------------------------------------------------------------
# brute-force classification against the solid


def _random_star(rng, v):
    while True:
        d = rng.normal(size=(v, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        cosm = d @ d.T - 2 * np.eye(v)
        if cosm.max() < 0.7:
            break
    r = rng.uniform(0.08, 0.16, size=v + 1)
    L = rng.uniform(0.8, 1.2, size=v)
    xyz = np.concatenate([np.zeros((1, 3)), d * L[:, None]])
    return latgen.lattice_from_arrays(xyz, r, [(0, i + 1) for i in range(v)])


@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_kept_arcs_are_on_the_solid_boundary(orc, v):
    rng = np.random.default_rng(100 + v)
    done = 0
    for trial in range(12):
        lat = _random_star(rng, v)
        R = orc.run(lat, 8)
        if R.status[0] != 0 or R.margin[0] < 1e-6:
            continue
        xyz = lat.xyz64()
        rad = lat.radius.astype(np.float64)
        c = xyz[0]
        ai = R.arc_int[: R.ne[0]]
        ad = R.arc_dbl[: R.ne[0]]
        struts = [(xyz[0], rad[0], xyz[i + 1], rad[i + 1]) for i in range(v)]
        for (p, q, *_), dv in zip(ai, ad):
            o, a, b, t1, t2 = dv[0:3], dv[3:6], dv[6:9], dv[9], dv[10]
            # kept part: inner samples on the boundary of both faces
            t = t1 + (t2 - t1) * np.linspace(0.02, 0.98, 25)
            x = c + o + np.outer(np.sin(t), a) + np.outer(np.cos(t), b)
            ds = np.stack([cone_distance(x, *s) for s in struts], axis=1)
            dsph = np.linalg.norm(x - c, axis=1) - rad[0]
            for lab in (p, q):
                on = dsph if lab == 0 else ds[:, lab - 1]
                assert np.abs(on).max() < 1e-9
            others = [j for j in range(v) if j + 1 not in (p, q)]
            if others:
                assert ds[:, others].min() > -1e-9
        # every conic's trimmed remainder lies inside another strut or off
        # the faces: sample whole conics and compare with the kept set
        for (p, q, *_), dv in zip(ai, ad):
            o, a, b = dv[0:3], dv[3:6], dv[6:9]
            t = np.linspace(0, 2 * np.pi, 400, endpoint=False)
            x = c + o + np.outer(np.sin(t), a) + np.outer(np.cos(t), b)
            ds = np.stack([cone_distance(x, *s) for s in struts], axis=1)
            dsph = np.linalg.norm(x - c, axis=1) - rad[0]
            allds = np.concatenate([dsph[:, None], ds], axis=1)
            on_boundary = (np.abs(allds[:, p]) < 1e-9) & (np.abs(allds[:, q]) < 1e-9)
            others = [j for j in range(v + 1) if j not in (p, q)]
            on_boundary &= allds[:, others].min(axis=1) > 1e-9
            sel = (ai[:, 0] == p) & (ai[:, 1] == q)
            kept = np.zeros(len(t), bool)
            for dd in ad[sel]:
                tt = (t - dd[9]) % (2 * np.pi)
                kept |= tt < (dd[10] - dd[9])
            assert not (on_boundary & ~kept).any(), "boundary point missed by the arcs"
        done += 1
    assert done >= 4


# ---------------------------------------------------------------------------
# lattice invariants


LATTICES = {
    "cubic_cfg1": lambda: latgen.config(1),
    "bcc3": lambda: latgen.config(2, scale=3),
    "octet2": lambda: latgen.config(4, scale=2),
    "cubic_cones": lambda: latgen.cubic(3, radius=("uniform", 0.05, 0.15), jitter=0.04, seed=5),
    "bcc_cyl": lambda: latgen.bcc(2, radius=0.1, jitter=0.05, seed=9),
}


@pytest.mark.parametrize("name", sorted(LATTICES))
@pytest.mark.parametrize("k", [5, 8, 16])
def test_lattice_invariants(orc, name, k):
    lat = LATTICES[name]()
    R = orc.run(lat, k)
    assert (R.status == 0).all()
    assert np.array_equal(R.nv - R.ne + R.nc, 2 - R.valence)  # per-node Euler
    # T = 2 * sum of segment counts (each arc borders two loops or a loop and
    # a hole)
    assert len(R.tris) == 2 * int(R.arc_int[:, 4].sum())
    mesh_checks(R, lat)


def test_inside_outside_matches_solid(orc):
    lat = latgen.bcc(1, radius=("uniform", 0.12, 0.2), jitter=0.05, seed=4)
    k = 24
    R = orc.run(lat, k)
    assert (R.status == 0).all()
    rng = np.random.default_rng(11)
    lo, hi = lat.xyz64().min(0) - 0.3, lat.xyz64().max(0) + 0.3
    pts = rng.uniform(lo, hi, size=(3000, 3))
    d = solid_distance(lat, pts)
    rmax = float(lat.radius.max())
    # mesh deviates from the solid by the chord sagitta on struts and by the
    # flat fans on holes (up to (1 - 1/sqrt 2) rho for a hemispherical cap)
    delta = 0.3 * rmax + rmax * (1 - math.cos(math.pi / k))
    far = np.abs(d) > delta
    wn = winding_number(R.mesh, R.tris, pts[far])
    inside = wn > 0.5
    assert np.array_equal(inside, d[far] < 0)
    assert np.abs(wn - np.round(wn)).max() < 1e-6
    assert far.sum() > 1500 and inside.sum() > 50
