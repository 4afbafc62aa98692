"""Exact one-step transition probabilities of the paper-literal zone model on
one small rail (test infrastructure only).

For a state X (strictly increasing 1-based columns of the ions of one rail)
every ion draws two independent trials (SI S2.1, "Random Sampling and
Exclusion Rules"): a right move with probability P_right(z) when the column to
its right is free and inside the rail, and a left move with probability
P_left(z) under the same condition on its left.  Its move is M_right - M_left;
all ions move at once, and two ions that would land on the same column (gap
2, the left one moving right and the right one moving left) both stay.  Here
every combination of the 4^N trial outcomes is enumerated with its
probability instead of sampled, which gives the exact distribution of the next
state.  The per-zone probabilities come from the oracle's table (pinned on its
own); this module pins the sampling, the exclusion and the update.
"""
from __future__ import annotations

import itertools
from typing import Dict, Tuple

import numpy as np

from . import ZoneParams, zone_index, zone_table


def step_distribution(p: ZoneParams, X: Tuple[int, ...], V: float) -> Dict[Tuple[int, ...], float]:
    """{next state: probability} of one step of a single rail from X."""
    L, Z = p.sites, p.zones
    counts = np.zeros(Z, dtype=np.int64)
    for x in X:
        counts[zone_index(x, L, Z) - 1] += 1
    pl, pr, _ = zone_table(p, V, counts)
    n = len(X)
    per_ion = []
    for j, x in enumerate(X):
        z = zone_index(x, L, Z) - 1
        right_free = (X[j + 1] if j + 1 < n else L + 1) - x > 1
        left_free = x - (X[j - 1] if j > 0 else 0) > 1
        a = pr[z] if right_free else 0.0
        b = pl[z] if left_free else 0.0
        per_ion.append([((1, 0), a * (1 - b)), ((0, 1), (1 - a) * b), ((1, 1), a * b), ((0, 0), (1 - a) * (1 - b))])
    out: Dict[Tuple[int, ...], float] = {}
    for combo in itertools.product(*per_ion):
        prob = 1.0
        move = []
        for (mr, ml), q in combo:
            prob *= q
            move.append(mr - ml)
        if prob == 0.0:
            continue
        for j in range(n - 1):
            if move[j] == 1 and move[j + 1] == -1 and X[j + 1] - X[j] == 2:
                move[j] = move[j + 1] = 0
        nxt = tuple(x + m for x, m in zip(X, move))
        out[nxt] = out.get(nxt, 0.0) + prob
    return out
