"""Minimal-recomputation counts for reversing a time-stepping loop with a
fixed number of stored states (test infrastructure only).

The paper offers "optimal checkpointing" (§2.1, forward-wavefield management;
refs. Symes 2007, Griewank & Walther 2000) to save selected time steps and
recompute the rest.  Two independent statements of the optimum are given
here so that a schedule produced elsewhere can be checked:

* the closed form of Griewank & Walther: with s snapshots (the initial state
  held in one of them) and l steps to reverse, let t be the smallest integer
  with beta(s, t) >= l, beta(s, t) = C(s + t, s); the least number of forward
  steps is  t * l - beta(s + 1, t - 1);
* a dynamic programme over the first split: cost(l, c) is the least number of
  forward steps to reverse l steps from a stored start state with c further
  free slots; cost(1, c) = 0, cost(l, 0) = l (l - 1) / 2 and
  cost(l, c) = min_j [ j + cost(l - j, c - 1) + cost(j, c) ].
The two agree with cost(l, s - 1) = closed form(l, s).
"""
from __future__ import annotations

from math import comb

import numpy as np


def binomial(s: int, t: int) -> int:
    """beta(s, t) = C(s + t, s)."""
    if s < 0 or t < 0:
        return 0
    return comb(s + t, s)


def forward_steps_closed_form(l: int, s: int) -> int:
    """Least forward steps to reverse l steps with s snapshots (s >= 1)."""
    if l <= 1:
        return 0
    if s < 1:
        raise ValueError("need at least one snapshot")
    t = 0
    while binomial(s, t) < l:
        t += 1
    return t * l - binomial(s + 1, t - 1)


def optimal_cost_table(lmax: int, cmax: int) -> np.ndarray:
    """cost[l, c] by the dynamic programme above (small sizes only)."""
    INF = np.iinfo(np.int64).max // 4
    cost = np.full((lmax + 1, cmax + 1), INF, dtype=np.int64)
    for c in range(cmax + 1):
        cost[0, c] = 0
        cost[1, c] = 0
    for l in range(2, lmax + 1):
        cost[l, 0] = l * (l - 1) // 2
        for c in range(1, cmax + 1):
            best = INF
            for j in range(1, l):
                v = j + cost[l - j, c - 1] + cost[j, c]
                if v < best:
                    best = v
            cost[l, c] = best
    return cost
