"""Pins of the FP64 arc-codec reference against the paper's error analysis
(Sec. 4.2.1, Eq. 5) and plain facts of the format."""

import math

import numpy as np

import latgen
import oracle
from oracle import codec


def test_eq5_bound_gives_the_papers_bit_choice():
    # 12 bits for r and 15 / 16 for the angles give a bound under 0.001 R_max
    # (8.69e-4), and one bit fewer in either misses it: the paper's choice
    b = codec.eq5_bound(12, 15)
    assert abs(b - 8.69e-4) < 5e-7
    assert b < 1e-3
    assert codec.eq5_bound(11, 15) > 1e-3
    assert codec.eq5_bound(12, 14) > 1e-3


def test_pack_layout_and_roundtrip():
    rng = np.random.default_rng(1)
    E = 200
    q = {name: rng.integers(0, 1 << bits, E) for name, bits in codec.FIELDS}
    w = codec.pack(q)
    back = codec.unpack(w)
    for name, _ in codec.FIELDS:
        assert np.array_equal(back[name], q[name])
    # one field all ones: the bits land where the field order puts them
    z = {name: np.zeros(1, np.int64) for name, _ in codec.FIELDS}
    z["ra"][0] = (1 << 12) - 1
    assert list(codec.pack(z)[0]) == [0xFFF, 0, 0, 0]
    z["ra"][0] = 0
    z["span"][0] = (1 << 15) - 1  # the last 15 bits of the 128
    assert list(codec.pack(z)[0]) == [0, 0, 0, 0xFFFE0000]


def _random_arcs(rng, E, r_min, r_max):
    def unit(n):
        v = rng.normal(size=(n, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]

    d = unit(E)
    ah = unit(E)
    ah = ah - d * np.sum(ah * d, axis=1)[:, None]  # a perpendicular to d, as for the seams
    ah /= np.linalg.norm(ah, axis=1)[:, None]
    ra = rng.uniform(r_min, 4 * r_max, E)
    rb = rng.uniform(0.1 * r_min, r_max, E)
    bh = np.cross(ah, d)
    c = unit(E) * rng.uniform(0, r_max, E)[:, None]
    t1 = rng.uniform(0, 2 * math.pi, E)
    t2 = t1 + rng.uniform(0, 2 * math.pi, E)
    arcs = np.concatenate([c, ah * ra[:, None], bh * rb[:, None], t1[:, None], t2[:, None]], axis=1)
    return arcs, d


def test_roundtrip_error_within_eq5():
    rng = np.random.default_rng(7)
    r_min, r_max = 0.05, 0.12
    arcs, d = _random_arcs(rng, 20000, r_min, r_max)
    q, fb, _ = codec.encode(arcs, d, r_min, r_max)
    assert not fb.any()
    dec = codec.decode(codec.unpack(codec.pack(q)), d, r_min, r_max)
    err = codec.arc_error(arcs, dec)
    assert err.max() <= codec.eq5_bound() * r_max
    # the end parameters move by at most half a step
    assert np.abs(dec[:, 9] - arcs[:, 9]).max() <= math.pi / 2 ** 15 + 1e-12
    assert np.abs((dec[:, 10] - dec[:, 9]) - (arcs[:, 10] - arcs[:, 9])).max() <= math.pi / (2 ** 15 - 1) + 1e-12


def test_grid_values_decode_exactly():
    r_min, r_max = 0.05, 0.12
    lv = 1000
    ra = r_min + lv * (4 * r_max - r_min) / 4095
    # a along +z (theta 0), b along z x y = -x, d = +y, centre at the origin
    arcs = np.array([[0, 0, 0, 0, 0, ra, -r_max, 0, 0, 0.0, 2 * math.pi]])
    d = np.array([[0.0, 1.0, 0.0]])
    q, fb, _ = codec.encode(arcs, d, r_min, r_max)
    assert not fb.any()
    assert q["ra"][0] == lv and q["tha"][0] == 0 and q["rb"][0] == 4095 and q["rc"][0] == 0
    assert q["t1"][0] == 0 and q["span"][0] == 2 ** 15 - 1
    dec = codec.decode(q, d, r_min, r_max)
    np.testing.assert_allclose(dec, arcs, rtol=0, atol=1e-15)


def test_fallback_cases():
    r_min, r_max = 0.05, 0.12
    rng = np.random.default_rng(3)
    arcs, d = _random_arcs(rng, 4, r_min, r_max)
    arcs[0, 3:6] *= 5 * r_max / np.linalg.norm(arcs[0, 3:6])  # semi-major beyond 4 R_max
    arcs[1, 6:9] = -arcs[1, 6:9]  # b against the orientation the format implies
    arcs[2, 0:3] *= 2 * r_max / np.linalg.norm(arcs[2, 0:3])  # centre beyond R_max
    _, fb, _ = codec.encode(arcs, d, r_min, r_max)
    assert list(fb) == [True, True, True, False]


def test_oracle_arcs_and_reference_directions():
    """The meta-mesh the oracle computes fits the format: b lies where the
    reference direction puts it, and the decoded arcs stay within Eq. 5."""
    lat = latgen.config(2, scale=4, seed=3)
    R = oracle.run(lat, 8)
    node = np.repeat(np.arange(lat.n_nodes), R.ne)
    p, q = R.arc_int[:, 0], R.arc_int[:, 1]
    d = codec.reference_dirs(lat, node, p, q)
    r_min, r_max = float(np.min(lat.radius)), float(np.max(lat.radius))
    qq, fb, _ = codec.encode(R.arc_dbl, d, r_min, r_max)
    # orientation is never the reason to fall back on this lattice
    arcs = R.arc_dbl
    ah = arcs[:, 3:6] / np.linalg.norm(arcs[:, 3:6], axis=1)[:, None]
    bh = arcs[:, 6:9] / np.linalg.norm(arcs[:, 6:9], axis=1)[:, None]
    x = np.cross(ah, d)
    assert np.abs(x / np.linalg.norm(x, axis=1)[:, None] - bh).max() < 1e-9
    assert fb.mean() < 0.05
    dec = codec.decode(qq, d, r_min, r_max)
    err = codec.arc_error(arcs[~fb], dec[~fb])
    assert err.max() <= codec.eq5_bound() * r_max
