"""Autotuner of the batched entry point: picks the wave-to-node mapping (the
valence limits of the four- and two-nodes-per-wave classes) and the group
size (nodes per node pass) by timing lm_batched on a sample of the parts."""

from __future__ import annotations

import itertools
import time

import numpy as np

from .latmesh import Mesher, lm_tuning

MAPPINGS = ((4, 8), (0, 8), (4, 4), (0, 0))  # (v_four_per_wave, v_two_per_wave)
GROUPS = (1 << 21, 1 << 22, 1 << 23)


def tune(parts, union_fn, sample: int = 32, seed: int = 0, repeats: int = 2, mappings=MAPPINGS, groups=GROUPS):
    """``parts``: list of (lattice, k).  ``union_fn``: lattices -> (union,
    part_off).  Times every (mapping, group) on ``sample`` parts drawn
    evenly from the list; returns (best lm_tuning, {(t4, t8, group): ms})."""
    import torch

    idx = np.linspace(0, len(parts) - 1, min(sample, len(parts))).round().astype(int)
    sub = [parts[i] for i in idx]
    lat, off = union_fn([p[0] for p in sub])
    ks = np.array([p[1] for p in sub], np.int32)
    M = Mesher(lat)
    times = {}
    try:
        for (t4, t8), g in itertools.product(mappings, groups):
            tn = lm_tuning(t4, t8, g)
            M.batched(off, ks, tn)  # warm-up
            best = float("inf")
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                M.batched(off, ks, tn)
                best = min(best, time.perf_counter() - t0)
            times[(t4, t8, g)] = best * 1e3
    finally:
        M.close()
    t4, t8, g = min(times, key=times.get)
    return lm_tuning(t4, t8, g), times
