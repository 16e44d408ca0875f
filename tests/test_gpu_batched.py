"""Batched parts (one plan, per-part resolutions, all parts in one node pass
from a global work queue) against the FP64 oracle: every part's sink words
equal oracle.sink_words of that part alone (counts and triangle-key sums
exactly, fixed-point coordinate sums to the position tolerance), for several
wave mappings; and against each part meshed alone by lm_forward_sink.

The mix has cubic, BCC, octet and k-NN parts, the k-NN ones with k up to 20
(nodes of up to about 40 struts, in the multi-wave class)."""

import numpy as np
import pytest

import latgen
import oracle
from parity import STRUT_TAU, above_margin

pytestmark = pytest.mark.gpu

RAD = ("uniform", 0.04, 0.12)


def _parts():
    """12 parts of the batched workload's four families at small sizes; the
    regular ones jittered (seeded), so that nearly every node is above the
    comparison margin and the words can be compared exactly."""
    return [
        (latgen.cubic(3, radius=RAD, jitter=0.03, seed=40), 8),
        (latgen.bcc(3, radius=RAD, jitter=0.04, seed=32), 16),
        (latgen.octet(2, radius=RAD, jitter=0.03, seed=40), 32),
        (latgen.knn(4, 20, radius=RAD, seed=4020), 16),
        (latgen.bcc(2, radius=RAD, jitter=0.05, seed=34), 8),
        (latgen.knn(5, 17, radius=RAD, seed=48), 8),
        (latgen.cubic(4, radius=RAD, jitter=0.04, seed=41), 16),
        (latgen.knn(3, 9, radius=RAD, seed=3009), 32),
        (latgen.octet(3, radius=RAD, jitter=0.02, seed=43), 12),
        (latgen.knn(5, 19, radius=RAD, seed=5019), 12),
        (latgen.knn(4, 6, radius=RAD, seed=4006), 16),
        (latgen.bcc(4, radius=RAD, jitter=0.05, seed=37), 12),
    ]


def _stable(R):
    """(nodes, struts): every node (meshed or flagged) above the comparison
    thresholds; every strut between two meshed nodes above the zipper
    threshold as well.  The triangle count, mesh-vertex count, unmeshed-node
    count and coordinate sums depend on the nodes only; the triangle-key sum
    also on the zipper's apex choices, which exact phi ties between the two
    loops of a strut leave open (three mutually adjacent nodes put loop
    vertices of both ends on one generator)."""
    ok_struts = R.strut_status == 0
    nodes = bool(above_margin(R, R.k).all())
    return nodes, nodes and bool((R.strut_margin[ok_struts] >= STRUT_TAU).all())


def _check_part(got, R, lat, name):
    exp = oracle.sink_words(R, max(lat.n_nodes, 1), lat.strut_a, lat.strut_b)[0]
    nodes, struts = _stable(R)
    if nodes:
        for f in (0, 2, 7):
            assert got[f] == exp[f], (name, f, got[f], exp[f])
        d = (got[4:7].view(np.int64) - exp[4:7].view(np.int64)).astype(np.float64)
        lim = float(exp[2]) * (1.0 + 1e-5 * 0.12 * 1048576.0)
        assert (np.abs(d) <= lim).all(), (name, d, lim)
    else:
        assert abs(int(got[2]) - int(exp[2])) <= 0.02 * int(exp[2]) + 8, (name, got[2], exp[2])
    if struts:
        assert got[1] == exp[1], (name, "triangle keys", got[1], exp[1])
    return nodes, struts


def test_batched_matches_oracle_and_per_part():
    from paper_2405_15197_amd import Mesher
    from paper_2405_15197_amd.latmesh import lm_tuning

    parts = _parts()
    lat, off = latgen.union([p[0] for p in parts])
    ks = np.array([p[1] for p in parts], np.int32)
    Rs = [oracle.run(pl, int(k)) for pl, k in parts]
    ref = []
    for pl, k in parts:
        M = Mesher(pl)
        try:
            ref.append(M.sink(int(k), max(pl.n_nodes, 1))[0])
        finally:
            M.close()
    ref = np.stack(ref)
    n_nodes = n_keys = 0
    for i, ((pl, k), R) in enumerate(zip(parts, Rs)):
        a, b = _check_part(ref[i], R, pl, f"part {i} alone")
        n_nodes += a
        n_keys += b
    print(f"parts compared: counts and sums {n_nodes} of {len(parts)}, triangle keys {n_keys}", flush=True)
    assert n_nodes == len(parts) and n_keys >= 6
    M = Mesher(lat)
    try:
        for tune in (None, lm_tuning(0, 8, 0), lm_tuning(4, 4, 300), lm_tuning(0, 0, 1)):
            got = M.batched(off, ks, tune)
            assert got.shape == ref.shape
            for i, ((pl, k), R) in enumerate(zip(parts, Rs)):
                _check_part(got[i], R, pl, f"part {i} batched")
            bad = np.nonzero((got != ref).any(axis=1))[0]
            assert len(bad) == 0, (tune and (tune.v_four_per_wave, tune.v_two_per_wave, tune.group_nodes), bad,
                                   got[bad[:2]], ref[bad[:2]])
    finally:
        M.close()


def test_autotune_picks_a_candidate():
    from paper_2405_15197_amd.autotune import tune

    parts = latgen.parts(8, seed=4, n_max=4, n_min=2)
    best, times = tune(parts, latgen.union, sample=8, repeats=1, groups=(64, 1 << 21))
    assert (best.v_four_per_wave, best.v_two_per_wave, best.group_nodes) in times
    assert all(t > 0 for t in times.values())


def test_batched_512_parts_unmeshed_nodes_equal_oracle():
    """The full 512-part workload in one batched pass: the nodes each part
    leaves without a mesh (word 7) equal the oracle's count for that part,
    stored in tests/golden/batched512_oracle_flags.json by
    tests/golden/make_batched_flags.py from the oracle alone (k-NN nodes of
    up to 52 struts included)."""
    import json
    import os

    from paper_2405_15197_amd import Mesher

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batched512_oracle_flags.json")))
    parts = latgen.parts(512, seed=1, workers=16, start="spawn")
    assert [[p[0].n_nodes, int(p[1])] for p in parts] == [g[1:] for g in gold["per_part"]]
    lat, off = latgen.union([p[0] for p in parts])
    ks = np.array([p[1] for p in parts], np.int32)
    del parts
    M = Mesher(lat)
    try:
        got = M.batched(off, ks)
    finally:
        M.close()
    want = [g[0] for g in gold["per_part"]]
    assert [int(x) for x in got[:, 7]] == want, sum(int(x) for x in got[:, 7])
    print(f"512 parts: {sum(want)} nodes without a mesh, as the oracle", flush=True)
