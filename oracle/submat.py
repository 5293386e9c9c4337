"""Redundancy references (App. A) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module; the product path never does.  Plain Python loops,
written from the appendix's description, for small arrays.

Definitions (App. A; readings where the text leaves a choice):

* baselines are the pairs (i, j), i <= j, in lexicographic order (the sets
  hold no reverse pairs; autocorrelations included, N (N + 1) / 2 pairs);
* two baselines are redundant when both antennas carry the same beams
  (beam(i) = beam(k), beam(j) = beam(l)) and their vectors agree,
  b_ij = x_i - x_j = b_kl, here to within tol metres in every component
  (reading: positions are measured, so exact equality is relaxed to a
  tolerance).  Groups are built in pair order: a pair joins the earliest
  group whose representative it matches, otherwise it founds a new group and
  is its representative -- so the representative is the group's first pair
  in lexicographic order, as the appendix suggests;
* the sub-matrix heuristic (steps 1-5 of App. A) sorts the first antennas alpha
  of the unique pairs by multiplicity, descending (reading: ties by antenna
  index, ascending), and places N_sub - 1 cuts: for each cut, n_x grows from 1
  while the density D_x = |U within V_x| / |V_x| stays at or above tau (reading:
  the cut is placed after the last n with D_x >= tau, at least one antenna per
  sub-matrix and one left for every later one); the rest forms the last
  sub-matrix; if its density does not exceed tau, tau is lowered (reading:
  tau_k = 1 - k * tau_step, tau_step = 0.01) and the cuts are placed again.
  beta_x is sorted by antenna index (reading).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def pair_list(n_ant: int) -> List[Tuple[int, int]]:
    """All baselines (i, j), i <= j, in lexicographic order."""
    return [(i, j) for i in range(n_ant) for j in range(i, n_ant)]


def redundant_groups(antpos, beam_idx, tol: float):
    """(group id of every pair in pair_list order, representative pairs)."""
    x = np.asarray(antpos, dtype=np.float64)
    n = x.shape[0]
    bi = np.zeros(n, dtype=np.int64) if beam_idx is None else np.asarray(beam_idx, dtype=np.int64)
    reps: List[Tuple[int, int]] = []
    group = []
    for (i, j) in pair_list(n):
        b = x[i] - x[j]
        found = -1
        for g, (k, l) in enumerate(reps):
            if bi[i] != bi[k] or bi[j] != bi[l]:
                continue
            d = b - (x[k] - x[l])
            if abs(d[0]) <= tol and abs(d[1]) <= tol and abs(d[2]) <= tol:
                found = g
                break
        if found < 0:
            found = len(reps)
            reps.append((i, j))
        group.append(found)
    return np.array(group, dtype=np.int32), reps


def _density(count: int, n_rows: int, n_cols: int) -> float:
    return count / float(n_rows * n_cols)


def submatrix_plan(pairs: Sequence[Tuple[int, int]], n_sub: int, tau_step: float = 0.01):
    """App. A heuristic.  Returns (alpha', sizes n_x, [(A_x, B_x, D_x)])."""
    mult = {}
    for a, _ in pairs:
        mult[a] = mult.get(a, 0) + 1
    alpha = sorted(mult, key=lambda a: (-mult[a], a))
    seconds = {}
    for a, b in pairs:
        seconds.setdefault(a, set()).add(b)
    n_sub = max(1, min(n_sub, len(alpha)))

    def stats(lo, hi):
        cnt = sum(mult[a] for a in alpha[lo:hi])
        beta = set()
        for a in alpha[lo:hi]:
            beta |= seconds[a]
        return cnt, beta

    k = 0
    while True:
        tau = 1.0 - k * tau_step
        sizes = []
        start = 0
        for x in range(n_sub - 1):
            max_n = len(alpha) - start - (n_sub - 1 - x)
            best = 1
            for n in range(1, max_n + 1):
                cnt, beta = stats(start, start + n)
                if _density(cnt, n, len(beta)) >= tau:
                    best = n
                else:
                    break
            sizes.append(best)
            start += best
        sizes.append(len(alpha) - start)
        cnt, beta = stats(start, len(alpha))
        d_last = _density(cnt, sizes[-1], len(beta))
        if d_last > tau or tau <= 0.0:
            break
        k += 1
    subs = []
    start = 0
    for n in sizes:
        cnt, beta = stats(start, start + n)
        A = alpha[start:start + n]
        B = sorted(beta)
        subs.append((A, B, _density(cnt, n, len(B))))
        start += n
    return alpha, sizes, subs
