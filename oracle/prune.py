"""Decision rule of one pruning round, FP64.  Test infrastructure only.

The paper's iterative pruning (Alg. 2, Sec. 5.2) removes processors whose
bypass leaves the matching loss within a tolerance of the best loss so far.
This build evaluates a round's trials as one batch, read as follows (the
paper tests candidates one after another with an accumulating mask; the
reading keeps its guarantee that everything removed in a round is jointly
within tolerance):

  1. candidates: the first ``max_candidates`` remaining processors ordered by
     (effective dry/wet weight ascending, processor index) - low w first, as
     the paper's dry/wet sampler prefers;
  2. each candidate j alone: L_j = L_a with j bypassed; keep those with
     L_j - L_min < tau * L_min, ordered by (L_j - L_min, index);
  3. prefixes of that order bypassed together: accept the longest prefix k
     whose loss L_k < L_min (1 + tau); L_min <- min(L_min, L_k).

The loss of a mask is supplied by the caller (``loss_of``), so the rule can
be pinned on synthetic loss tables as well as on the console.
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple


def candidates(w: Sequence[float], alive: Sequence[bool], max_candidates: int) -> List[int]:
    idx = [p for p in range(len(w)) if alive[p]]
    idx.sort(key=lambda p: (float(w[p]), p))
    return idx[:max_candidates]


def order_within_tolerance(cand: Sequence[int], L_cand: Sequence[float], L_min: float, tau: float) -> List[int]:
    ok = [(float(L) - L_min, j) for j, L in zip(cand, L_cand) if float(L) - L_min < tau * L_min]
    ok.sort()
    return [j for _, j in ok]


def accept_prefix(L_prefix: Sequence[float], L_min: float, tau: float) -> int:
    k = 0
    for i, L in enumerate(L_prefix):
        if float(L) < L_min * (1.0 + tau):
            k = i + 1
    return k


def prune_round(loss_of: Callable[[Sequence[bool]], float], alive: Sequence[bool], w: Sequence[float],
                L_min: float, tau: float = 1e-3, max_candidates: int = 64) -> Tuple[List[bool], float, dict]:
    """One round.  loss_of(alive_mask) returns L_a with every processor whose
    entry is False bypassed.  Returns (new alive mask, new L_min, details)."""
    alive = [bool(a) for a in alive]
    cand = candidates(w, alive, max_candidates)
    L_cand = []
    for j in cand:
        m = list(alive)
        m[j] = False
        L_cand.append(float(loss_of(m)))
    order = order_within_tolerance(cand, L_cand, L_min, tau)
    L_prefix = []
    for k in range(1, len(order) + 1):
        m = list(alive)
        for j in order[:k]:
            m[j] = False
        L_prefix.append(float(loss_of(m)))
    k = accept_prefix(L_prefix, L_min, tau)
    new = list(alive)
    for j in order[:k]:
        new[j] = False
    L_new = min(L_min, L_prefix[k - 1]) if k else L_min
    return new, L_new, {"candidates": cand, "L_cand": L_cand, "order": order, "L_prefix": L_prefix, "k": k}
