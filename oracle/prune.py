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

The tolerance test takes tau relative to L_min (L < L_min (1 + tau), the
benchmark configuration's 1e-3) or absolute (L < L_min + tau, the paper's
0.001 / 0.01 / 0.1; Sec. 6.1 tolerance study).

The dry/wet sampler (Alg. 3, Sec. 6.2 "Candidate Sampling") and the hybrid
schedule (the batched brute-force round every 4th round, the dry/wet sampler
otherwise) follow ``drywet_round`` and ``hybrid_method``.
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence, Tuple


def candidates(w: Sequence[float], alive: Sequence[bool], max_candidates: int) -> List[int]:
    idx = [p for p in range(len(w)) if alive[p]]
    idx.sort(key=lambda p: (float(w[p]), p))
    return idx[:max_candidates]


def _tol(L_min: float, tau: float, relative: bool) -> float:
    return tau * L_min if relative else tau


def order_within_tolerance(cand: Sequence[int], L_cand: Sequence[float], L_min: float, tau: float,
                           relative: bool = True) -> List[int]:
    ok = [(float(L) - L_min, j) for j, L in zip(cand, L_cand) if float(L) - L_min < _tol(L_min, tau, relative)]
    ok.sort()
    return [j for _, j in ok]


def within(L: float, L_min: float, tau: float, relative: bool = True) -> bool:
    """The acceptance test of a trial: L < L_min (1 + tau), or L < L_min + tau."""
    return float(L) < (L_min * (1.0 + tau) if relative else L_min + tau)


def accept_prefix(L_prefix: Sequence[float], L_min: float, tau: float, relative: bool = True) -> int:
    k = 0
    for i, L in enumerate(L_prefix):
        if within(L, L_min, tau, relative):
            k = i + 1
    return k


def prune_round(loss_of: Callable[[Sequence[bool]], float], alive: Sequence[bool], w: Sequence[float],
                L_min: float, tau: float = 1e-3, max_candidates: int = 64,
                relative: bool = True) -> Tuple[List[bool], float, dict]:
    """One round.  loss_of(alive_mask) returns L_a with every processor whose
    entry is False bypassed.  Returns (new alive mask, new L_min, details)."""
    alive = [bool(a) for a in alive]
    cand = candidates(w, alive, max_candidates)
    L_cand = []
    for j in cand:
        m = list(alive)
        m[j] = False
        L_cand.append(float(loss_of(m)))
    order = order_within_tolerance(cand, L_cand, L_min, tau, relative)
    L_prefix = []
    for k in range(1, len(order) + 1):
        m = list(alive)
        for j in order[:k]:
            m[j] = False
        L_prefix.append(float(loss_of(m)))
    k = accept_prefix(L_prefix, L_min, tau, relative)
    new = list(alive)
    for j in order[:k]:
        new[j] = False
    L_new = min(L_min, L_prefix[k - 1]) if k else L_min
    return new, L_new, {"candidates": cand, "L_cand": L_cand, "order": order, "L_prefix": L_prefix, "k": k}


# ---------------------------------------------------------------------------
# Alg. 3: the dry/wet method
# ---------------------------------------------------------------------------
def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


def drywet_round(loss_of: Callable[[Sequence[bool]], float], alive: Sequence[bool], w: Sequence[float],
                 types: Sequence[str], L_min: float, tau: float, uniforms: Sequence[float],
                 relative: bool = False, r0: float = 0.1) -> Tuple[List[bool], float, dict]:
    """One pruning iteration of the dry/wet method (Alg. 3).

    Per processor type t present among the alive processors: V_t its alive
    processors, N_t = |V_t| at the start, r_t = r0.  While some type is left,
    a type is drawn uniformly from those left (the i-th draw uses
    uniforms[i] in [0, 1): the (floor(u |T|))-th remaining type in the order
    e c n x s g d r); its floor(N_t r_t + 1/2) processors of least weight
    (ties by index; at least one, at most |V_t|) are bypassed together with
    everything bypassed so far.  If the loss passes the tolerance test, they
    are pruned (removed from V_t) and L_min <- min(L_min, L); the type leaves
    the set once V_t is empty.  Otherwise r_t is halved while floor(N_t r_t +
    1/2) > 1, and the type leaves the set when it is not.

    Readings: the count is at least one (a count of zero tests nothing and
    never ends), the type leaves once all its processors are pruned, and w
    (the weights after training, fixed within the iteration) orders the
    candidates.  Returns (new alive mask, new L_min, details)."""
    alive = [bool(a) for a in alive]
    order = [t for t in "ecnxsgdr" if any(alive[p] and types[p] == t for p in range(len(alive)))]
    V = {t: [p for p in range(len(alive)) if alive[p] and types[p] == t] for t in order}
    N = {t: len(V[t]) for t in order}
    r = {t: r0 for t in order}
    m = list(alive)
    trials = []
    i = 0
    while order:
        if i >= len(uniforms):
            raise ValueError("ran out of uniform draws")
        t = order[int(math.floor(float(uniforms[i]) * len(order)))]
        i += 1
        k_raw = _round_half_up(N[t] * r[t])
        k = min(max(1, k_raw), len(V[t]))
        cand = sorted(V[t], key=lambda p: (float(w[p]), p))[:k]
        trial = list(m)
        for p in cand:
            trial[p] = False
        L = float(loss_of(trial))
        ok = within(L, L_min, tau, relative)
        trials.append({"type": t, "candidates": cand, "L": L, "accepted": ok})
        if ok:
            L_min = min(L_min, L)
            m = trial
            V[t] = [p for p in V[t] if p not in cand]
            if not V[t]:
                order.remove(t)
        elif k_raw > 1:
            r[t] /= 2.0
        else:
            order.remove(t)
    return m, L_min, {"trials": trials, "draws": i}


def hybrid_method(round_index: int) -> str:
    """The paper's default sampler (Sec. 6.2): the brute-force method on every
    4th pruning iteration (1-based), the dry/wet method on the others."""
    return "brute" if round_index % 4 == 0 else "drywet"
