"""Batched parts (one plan, per-part resolutions, node passes shared by the
parts of a group) against each part meshed on its own in sink mode: every
word of every part identical, for several wave mappings and group sizes."""

import numpy as np
import pytest

import latgen

pytestmark = pytest.mark.gpu


def test_batched_matches_per_part():
    from paper_2405_15197_amd import Mesher
    from paper_2405_15197_amd.latmesh import lm_tuning

    parts = latgen.parts(12, seed=3, n_max=5, n_min=2)
    lat, off = latgen.union([p[0] for p in parts])
    ks = np.array([p[1] for p in parts], np.int32)
    ref = []
    for pl, k in parts:
        M = Mesher(pl)
        try:
            ref.append(M.sink(int(k), max(pl.n_nodes, 1))[0])
        finally:
            M.close()
    ref = np.stack(ref)
    M = Mesher(lat)
    try:
        for tune in (None, lm_tuning(0, 8, 0), lm_tuning(4, 4, 300), lm_tuning(0, 0, 1)):
            got = M.batched(off, ks, tune)
            assert got.shape == ref.shape
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
