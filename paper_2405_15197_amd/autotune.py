"""Autotuner of the batched entry point: picks the wave-to-node mapping (the
valence limits of the four- and two-nodes-per-wave classes) and the group
size (nodes per node pass) by timing lm_batched on samples of the parts.

Successive halving: every candidate is timed on a small sample of the parts;
the faster half is kept and timed again on a sample twice as large, until
one candidate is left or the sample holds every part allowed.  Timings of
every round are returned."""

from __future__ import annotations

import itertools
import time

import numpy as np

from .latmesh import Mesher, lm_tuning

# (v_four_per_wave, v_two_per_wave): 0 sends no node to the four-per-wave
# class, 8 is the two-per-wave class's capacity
MAPPINGS = ((4, 8), (3, 8), (2, 8), (0, 8), (4, 6), (0, 6), (4, 4), (0, 0))
GROUPS = (0, 1 << 21, 1 << 23)  # 0: all parts in one node pass when they fit


def _time(M, off, ks, cand, repeats):
    import torch

    tn = lm_tuning(*cand)
    M.batched(off, ks, tn)  # warm-up
    best = float("inf")
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.batched(off, ks, tn)
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def tune(parts, union_fn, sample: int = 32, seed: int = 0, repeats: int = 2, mappings=MAPPINGS, groups=GROUPS,
         first_sample: int | None = None):
    """``parts``: list of (lattice, k).  ``union_fn``: lattices -> (union,
    part_off).  Successive halving over every (mapping, group) candidate,
    from ``first_sample`` parts (default sample / 4, at least 1) up to
    ``sample`` parts, drawn evenly from the list.  Returns (best lm_tuning,
    {(t4, t8, group): ms} of the largest sample each candidate reached)."""
    cands = list(itertools.product(mappings, groups))
    cands = [(t4, t8, g) for (t4, t8), g in cands]
    n = max(1, min(first_sample or max(1, sample // 4), len(parts)))
    times = {}
    while True:
        idx = np.linspace(0, len(parts) - 1, min(n, len(parts))).round().astype(int)
        sub = [parts[i] for i in idx]
        lat, off = union_fn([p[0] for p in sub])
        ks = np.array([p[1] for p in sub], np.int32)
        M = Mesher(lat)
        try:
            for c in cands:
                times[c] = _time(M, off, ks, c, repeats)
        finally:
            M.close()
        cands.sort(key=lambda c: times[c])
        if len(cands) == 1 or n >= min(sample, len(parts)):
            break
        cands = cands[: max(1, (len(cands) + 1) // 2)]
        n = min(2 * n, sample, len(parts))
    t4, t8, g = cands[0]
    return lm_tuning(t4, t8, g), times
