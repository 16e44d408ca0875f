"""FP64 reference of the lossy 128-bit arc codec (test infrastructure).

Only the tests may import this module.  It follows the compressive arc
representation of Sec. 4.2.1: an arc x(t) = c + a sin t + b cos t,
t in [t1, t2], keeps

* the semi-major axis a as spherical coordinates: radial distance r in
  [R_min, 4 R_max] on n = 12 bits, polar angle theta in [0, pi] on m = 15
  bits, azimuth phi in [0, 2 pi) on m + 1 = 16 bits;
* of the semi-minor axis b only its length, in [0.1 R_min, R_max] on 12
  bits: its direction is perpendicular to a and to a reference direction d
  known from the lattice, b = |b| (a / |a|) x d / |(a / |a|) x d|;
* the centre c as spherical coordinates, r in [0, R_max] on 12 bits, theta
  and phi as for a;
* t1 on 15 bits over [0, 2 pi) and the span t2 - t1 on 15 bits over
  [0, 2 pi]

= 128 bits.  An arc outside these ranges is kept uncompressed (fallback).
Quantisation is the fixed-point one the paper cites: a value in [lo, hi] on
k bits is the nearest of 2^k evenly spaced levels with both ends included
(round half to even); a periodic angle is the nearest of 2^k levels with
step 2 pi / 2^k.  The error bound is Eq. 5.

Readings (the paper is silent on them):

* d, the reference direction: for the tangency circle of strut q (p = 0) the
  strut's own direction (from the lower to the higher node id); for the seam
  ellipse of struts p < q the normal of its plane, (g_p - g_q) / |g_p - g_q|
  with g = e / kappa (the plane P_p = P_q of the local model).  The sign of b
  follows from the order (a, d) of the cross product.
* t1 is periodic, the span is not (a whole circle has span 2 pi).
"""

from __future__ import annotations

import math

import numpy as np

N_R = 12   # bits of a radial distance
M_TH = 15  # bits of a polar angle
M_PH = 16  # bits of an azimuth
N_T = 15   # bits of t1 and of the span
FIELDS = (("ra", N_R), ("tha", M_TH), ("pha", M_PH), ("rb", N_R), ("rc", N_R), ("thc", M_TH), ("phc", M_PH),
          ("t1", N_T), ("span", N_T))
assert sum(b for _, b in FIELDS) == 128


def eq5_bound(n: int = N_R, m: int = M_TH) -> float:
    """Eq. 5: the largest distance between a point of the arc and the point
    of the decoded arc at the same t, in units of R_max."""
    s1 = math.sqrt(17.0 / 2 ** (2 * n + 2) + 32.0 * math.pi ** 2 / 2 ** (2 * m + 2))
    s2 = math.sqrt(1.0 / 2 ** (2 * n + 2) + 32.0 * math.pi ** 2 / 2 ** (2 * m + 2))
    return s1 + s2


def _qlin(v, lo, hi, bits):
    levels = (1 << bits) - 1
    s = (v - lo) / (hi - lo) * levels
    return np.rint(np.clip(s, 0.0, levels)).astype(np.int64)


def _dlin(q, lo, hi, bits):
    return lo + q.astype(np.float64) * (hi - lo) / ((1 << bits) - 1)


def _qper(ang, bits):
    n = 1 << bits
    return np.rint(ang / (2.0 * math.pi) * n).astype(np.int64) % n


def _dper(q, bits):
    return q.astype(np.float64) * (2.0 * math.pi) / (1 << bits)


def _sph(v):
    r = np.linalg.norm(v, axis=1)
    z = np.where(r > 0, v[:, 2] / np.where(r > 0, r, 1.0), 1.0)
    th = np.arccos(np.clip(z, -1.0, 1.0))
    ph = np.arctan2(v[:, 1], v[:, 0])
    ph = np.where(ph < 0, ph + 2.0 * math.pi, ph)
    return r, th, ph


def _cart(r, th, ph):
    return r[:, None] * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def _unit_cross(a, d):
    x = np.cross(a, d)
    n = np.linalg.norm(x, axis=1)
    return x / np.where(n > 0, n, 1.0)[:, None], n


def encode(arcs, d, r_min, r_max):
    """arcs [E, 11] (c.xyz, a.xyz, b.xyz, t1, t2), d [E, 3] unit reference
    directions.  Returns (fields dict of int64 arrays, fallback bool [E],
    the pre-rounding values of every field for tie checks)."""
    arcs = np.asarray(arcs, np.float64)
    c, a, b = arcs[:, 0:3], arcs[:, 3:6], arcs[:, 6:9]
    t1, t2 = arcs[:, 9], arcs[:, 10]
    ra, tha, pha = _sph(a)
    rb = np.linalg.norm(b, axis=1)
    rc, thc, phc = _sph(c)
    span = t2 - t1
    bh, crossn = _unit_cross(a / np.where(ra > 0, ra, 1.0)[:, None], d)
    bdir = b / np.where(rb > 0, rb, 1.0)[:, None]
    fb = ~((ra >= r_min) & (ra <= 4.0 * r_max) & (rb >= 0.1 * r_min) & (rb <= r_max) & (rc <= r_max)
           & (t1 >= 0.0) & (t1 < 2.0 * math.pi) & (span >= 0.0) & (span <= 2.0 * math.pi)
           & (crossn > 1e-6) & (np.linalg.norm(bh - bdir, axis=1) <= 1e-3))
    raw = {
        "ra": (ra - r_min) / (4.0 * r_max - r_min) * ((1 << N_R) - 1),
        "tha": tha / math.pi * ((1 << M_TH) - 1),
        "pha": pha / (2.0 * math.pi) * (1 << M_PH),
        "rb": (rb - 0.1 * r_min) / (r_max - 0.1 * r_min) * ((1 << N_R) - 1),
        "rc": rc / r_max * ((1 << N_R) - 1),
        "thc": thc / math.pi * ((1 << M_TH) - 1),
        "phc": phc / (2.0 * math.pi) * (1 << M_PH),
        "t1": t1 / (2.0 * math.pi) * (1 << N_T),
        "span": span / (2.0 * math.pi) * ((1 << N_T) - 1),
    }
    q = {
        "ra": _qlin(ra, r_min, 4.0 * r_max, N_R),
        "tha": _qlin(tha, 0.0, math.pi, M_TH),
        "pha": _qper(pha, M_PH),
        "rb": _qlin(rb, 0.1 * r_min, r_max, N_R),
        "rc": _qlin(rc, 0.0, r_max, N_R),
        "thc": _qlin(thc, 0.0, math.pi, M_TH),
        "phc": _qper(phc, M_PH),
        "t1": _qper(t1, N_T),
        "span": _qlin(span, 0.0, 2.0 * math.pi, N_T),
    }
    return q, fb, raw


def pack(q) -> np.ndarray:
    """Fields into 4 little-endian 32-bit words per arc, least significant
    bit first in the order of FIELDS."""
    E = len(next(iter(q.values())))
    lo = np.zeros(E, np.uint64)
    hi = np.zeros(E, np.uint64)
    pos = 0
    for name, bits in FIELDS:
        v = q[name].astype(np.uint64)
        for b in range(bits):  # bit by bit: obviously correct, small inputs only
            bit = (v >> np.uint64(b)) & np.uint64(1)
            p = pos + b
            if p < 64:
                lo |= bit << np.uint64(p)
            else:
                hi |= bit << np.uint64(p - 64)
        pos += bits
    w = np.zeros((E, 4), np.uint32)
    w[:, 0] = (lo & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    w[:, 1] = (lo >> np.uint64(32)).astype(np.uint32)
    w[:, 2] = (hi & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    w[:, 3] = (hi >> np.uint64(32)).astype(np.uint32)
    return w


def unpack(w) -> dict:
    w = np.asarray(w, np.uint32).astype(np.uint64)
    lo = w[:, 0] | (w[:, 1] << np.uint64(32))
    hi = w[:, 2] | (w[:, 3] << np.uint64(32))
    q = {}
    pos = 0
    for name, bits in FIELDS:
        v = np.zeros(len(w), np.uint64)
        for b in range(bits):
            p = pos + b
            bit = ((lo >> np.uint64(p)) if p < 64 else (hi >> np.uint64(p - 64))) & np.uint64(1)
            v |= bit << np.uint64(b)
        q[name] = v.astype(np.int64)
        pos += bits
    return q


def decode(q, d, r_min, r_max) -> np.ndarray:
    """Fields (dict) and reference directions [E, 3] -> arcs [E, 11]."""
    a = _cart(_dlin(q["ra"], r_min, 4.0 * r_max, N_R), _dlin(q["tha"], 0.0, math.pi, M_TH), _dper(q["pha"], M_PH))
    c = _cart(_dlin(q["rc"], 0.0, r_max, N_R), _dlin(q["thc"], 0.0, math.pi, M_TH), _dper(q["phc"], M_PH))
    ah = a / np.maximum(np.linalg.norm(a, axis=1), 1e-300)[:, None]
    bh, _ = _unit_cross(ah, d)
    b = _dlin(q["rb"], 0.1 * r_min, r_max, N_R)[:, None] * bh
    t1 = _dper(q["t1"], N_T)
    t2 = t1 + _dlin(q["span"], 0.0, 2.0 * math.pi, N_T)
    return np.concatenate([c, a, b, t1[:, None], t2[:, None]], axis=1)


def arc_error(arcs, dec, samples: int = 17) -> np.ndarray:
    """Largest distance between the arc and the decoded arc at equal t over
    samples evenly spaced t in [t1, t2] (the E of the error analysis)."""
    arcs = np.asarray(arcs, np.float64)
    dec = np.asarray(dec, np.float64)
    s = np.linspace(0.0, 1.0, samples)
    t = arcs[:, 9:10] + (arcs[:, 10:11] - arcs[:, 9:10]) * s[None, :]
    st, ct = np.sin(t)[:, :, None], np.cos(t)[:, :, None]
    p = arcs[:, None, 0:3] + arcs[:, None, 3:6] * st + arcs[:, None, 6:9] * ct
    pd = dec[:, None, 0:3] + dec[:, None, 3:6] * st + dec[:, None, 6:9] * ct
    return np.linalg.norm(p - pd, axis=2).max(axis=1)


def reference_dirs(lat, node, p, q):
    """d for arcs of node `node` with strut labels p (0: tangency circle) and
    q: labels count a node's incident struts in increasing strut id."""
    x = np.stack([lat.x, lat.y, lat.z], 1).astype(np.float64)
    rad = np.asarray(lat.radius, np.float64)
    sa = np.asarray(lat.strut_a, np.int64)
    sb = np.asarray(lat.strut_b, np.int64)
    S = len(sa)
    ends = np.concatenate([sa, sb])
    far = np.concatenate([sb, sa])
    sid = np.concatenate([np.arange(S), np.arange(S)])
    order = np.lexsort((sid, ends))
    ends, far, sid = ends[order], far[order], sid[order]
    start = np.searchsorted(ends, np.arange(len(rad)))

    def entry(n, lab):
        h = start[n] + lab - 1
        f = far[h]
        dv = x[f] - x[n]
        L = np.linalg.norm(dv, axis=1)
        e = dv / L[:, None]
        sig = (rad[n] - rad[f]) / L
        kap = np.sqrt((1 - sig) * (1 + sig))
        g = e / kap[:, None]
        lo = np.where(f > n, n, f)
        hi = np.where(f > n, f, n)
        es = x[hi] - x[lo]
        es = es / np.linalg.norm(es, axis=1)[:, None]
        return g, es

    node = np.asarray(node, np.int64)
    p = np.asarray(p, np.int64)
    q = np.asarray(q, np.int64)
    gq, esq = entry(node, q)
    d = esq.copy()
    ell = p > 0
    if ell.any():
        gp, _ = entry(node[ell], p[ell])
        nv = gp - gq[ell]
        d[ell] = nv / np.linalg.norm(nv, axis=1)[:, None]
    return d
