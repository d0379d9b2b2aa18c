"""The projection range operator of the parallel PCC algorithm (Sec. III).

P_i(C) is the set of coordinates that cluster C occupies along axis i, kept
as a sorted list of disjoint closed integer intervals.  When two clusters
merge, their ranges are united; a cluster percolates along axis i (extension
rule, periodic boundaries) when its range is the whole of [0, L-1].

This is a second, independent formulation of the oracle's percolation test:
``sw_oracle.c`` tests the full coordinate set of each cluster directly; the
tests check that both agree and that this one reproduces the worked example
of Sec. III (Fig. 5).  Test infrastructure only.
"""
from __future__ import annotations

from typing import Iterable, List, Tuple

Interval = Tuple[int, int]


def normalise(intervals: Iterable[Interval]) -> List[Interval]:
    """Sort and merge overlapping or touching closed integer intervals."""
    out: List[Interval] = []
    for lo, hi in sorted((int(a), int(b)) for a, b in intervals):
        if lo > hi:
            raise ValueError("empty interval")
        if out and lo <= out[-1][1] + 1:
            out[-1] = (out[-1][0], max(out[-1][1], hi))
        else:
            out.append((lo, hi))
    return out


def merge(a: Iterable[Interval], b: Iterable[Interval]) -> List[Interval]:
    """Range of the union of two clusters."""
    return normalise(list(a) + list(b))


def covers(rng: Iterable[Interval], L: int) -> bool:
    """True when the range is exactly [0, L-1]."""
    return normalise(rng) == [(0, L - 1)]


def cluster_ranges(labels, coords, L: int) -> dict:
    """Build every cluster's range along one axis by merging one site at a time.

    labels[i] is the cluster of site i and coords[i] its coordinate along the
    axis; sites are merged into their cluster's range in index order, as the
    incremental bookkeeping of Sec. III does when clusters are joined.
    """
    ranges: dict = {}
    for lab, c in zip(labels, coords):
        ranges[int(lab)] = merge(ranges.get(int(lab), []), [(int(c), int(c))])
    return ranges


def percolates(labels, dim: int, L: int) -> bool:
    """Extension rule with periodic boundaries over all axes, via ranges."""
    import numpy as np

    labels = np.asarray(labels).reshape(-1)
    idx = np.arange(labels.size)
    stride = 1
    for _ in range(dim):
        coords = (idx // stride) % L
        for rng in cluster_ranges(labels, coords, L).values():
            if covers(rng, L):
                return True
        stride *= L
    return False
