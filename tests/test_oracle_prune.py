"""Pins of the oracle's pruning-round rule (oracle/prune.py): a hand-worked
additive example, tie-breaking, limiting tolerances, and brute force over
every mask of a small console evaluated by the oracle itself."""
import itertools

import numpy as np
import pytest
import torch

import synth
from oracle import console as OC
from oracle import loss as LS
from oracle import prune as PR
from oracle import train as TR


def additive(L0, c):
    """L(mask) = L0 + sum of c_j over bypassed j."""
    return lambda alive: L0 + sum(cj for cj, a in zip(c, alive) if not a)


def test_hand_worked_round():
    # w orders the candidates p1 (0.1), p5 (0.2), p3 (0.3), p2 (0.5); p2 costs
    # more than tau * L0 = 1e-3 alone; the others in Delta order p3, p5, p1
    # give prefix losses 1.0002, 1.0006, 1.0011, so the first two go.
    w = [0.9, 0.1, 0.5, 0.3, 0.7, 0.2]
    c = [0.0, 0.0005, 0.002, 0.0002, 0.0, 0.0004]
    alive, L_new, info = PR.prune_round(additive(1.0, c), [True] * 6, w, 1.0, tau=1e-3, max_candidates=4)
    assert info["candidates"] == [1, 5, 3, 2]
    assert info["order"] == [3, 5, 1]
    assert np.allclose(info["L_prefix"], [1.0002, 1.0006, 1.0011])
    assert info["k"] == 2
    assert alive == [True, True, True, False, True, False]
    assert L_new == 1.0


def test_improving_bypass_lowers_the_best_loss():
    alive, L_new, info = PR.prune_round(additive(2.0, [-0.5, 0.0001]), [True, True], [0.2, 0.1], 2.0, tau=1e-3)
    assert info["order"] == [0, 1]           # Delta -0.5 first, then 1e-4
    assert alive == [False, False]
    assert L_new == pytest.approx(1.5001)


def test_ties_break_by_index():
    w = [0.5, 0.5, 0.5]
    c = [1e-5, 1e-5, 1e-5]
    _, _, info = PR.prune_round(additive(1.0, c), [True] * 3, w, 1.0, tau=1e-3, max_candidates=2)
    assert info["candidates"] == [0, 1]
    assert info["order"] == [0, 1]


def test_dead_processors_are_not_candidates():
    _, _, info = PR.prune_round(additive(1.0, [0, 0, 0]), [True, False, True], [0.1, 0.0, 0.2], 1.0)
    assert info["candidates"] == [0, 2]


def test_limits_of_the_tolerance():
    c = [0.01, 0.02, 0.03]
    alive, _, _ = PR.prune_round(additive(1.0, c), [True] * 3, [0.1, 0.2, 0.3], 1.0, tau=1e9)
    assert alive == [False, False, False]
    alive, _, info = PR.prune_round(additive(1.0, c), [True] * 3, [0.1, 0.2, 0.3], 1.0, tau=0.0)
    assert alive == [True, True, True] and info["order"] == []


def _small_console():
    cfg = synth.small_config(seconds=0.3, fs=8000, n_tracks=2, n_subgroups=1, chain="eg", stereo_tracks=False,
                             eq_taps=63, loss_ffts=(256, 512))
    g, dry, noise = synth.song(11, cfg)
    return cfg, g, dry, noise


def test_brute_force_over_every_mask_of_a_small_console():
    """Every mask of a 6-processor console evaluated by the oracle; the round's
    result must be jointly within tolerance, maximal along its order, and made
    of processors that were each within tolerance alone."""
    cfg, g, dry, noise = _small_console()
    procs = g.processors()
    P = len(procs)
    assert P <= 8
    gt, gw = synth.ground_truth_params(111, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw)
    th, we = synth.random_params(11, g, cfg, std=0.3)
    table = {}
    for bits in itertools.product([True, False], repeat=P):
        mask = {v: (1.0 if b else 0.0) for v, b in zip(procs, bits)}
        table[bits] = TR.losses(g, cfg, dry, noise, target, th, we, mask)["La"]
    L_min = table[(True,) * P]
    w = [1.0 / (1.0 + np.exp(-we[v])) for v in procs]
    # a tolerance that lets some, not all, processors go
    deltas = sorted(table[tuple(i != j for i in range(P))] - L_min for j in range(P))
    tau = float(np.median(deltas) / L_min)
    if tau <= 0:
        tau = 1e-3
    alive, L_new, info = PR.prune_round(lambda a: table[tuple(bool(x) for x in a)], [True] * P, w, L_min, tau=tau)
    k = info["k"]
    if k:
        assert table[tuple(alive)] < L_min * (1 + tau)
        assert L_new == min(L_min, table[tuple(alive)])
    for kk in range(k + 1, len(info["order"]) + 1):
        m = [True] * P
        for j in info["order"][:kk]:
            m[j] = False
        assert table[tuple(m)] >= L_min * (1 + tau)
    for j in info["order"]:
        single = tuple(i != j for i in range(P))
        assert table[single] - L_min < tau * L_min
    dropped = [j for j in range(P) if not alive[j]]
    assert dropped == sorted(info["order"][:k])


def test_bypass_mask_equals_the_pruned_graph():
    """Sec. 1.2: bypassing a processor (w = 0) and deleting it with its edges
    rerouted give the same mix."""
    cfg, g, dry, noise = _small_console()
    th, we = synth.random_params(12, g, cfg, std=0.3)
    drop = g.processors()[1]
    mix_masked = TR.render(g, cfg, dry, noise, th, we, {drop: 0.0})
    keep = [v for v in range(g.n_nodes) if v != drop]
    new_id = {v: i for i, v in enumerate(keep)}
    edges = []
    for s, d in g.edges:
        if d == drop:
            continue
        if s == drop:
            for s2, d2 in g.edges:
                if d2 == drop:
                    edges.append((new_id[s2], new_id[d]))
        else:
            edges.append((new_id[s], new_id[d]))
    g2 = synth.Graph([g.types[v] for v in keep], edges, {new_id[v]: t for v, t in g.track_of_input.items()})
    th2 = {new_id[v]: p for v, p in th.items() if v != drop}
    we2 = {new_id[v]: x for v, x in we.items() if v != drop}
    mix_pruned = TR.render(g2, cfg, dry, noise, th2, we2)
    assert np.array_equal(mix_masked, mix_pruned)


# ---------------------------------------------------------------------------
# Alg. 3, the dry/wet method
# ---------------------------------------------------------------------------
def test_drywet_hand_worked_binary_search():
    """One type, 40 processors, weights increasing with the index; the 10
    lowest-weight ones are free to prune, every other costs 1 (absolute tau
    0.01).  r = 0.1 gives 4 per trial: 4 and 8 pruned, the third trial (2 free
    + 2 costly) fails; r halves to 0.05 (count 2): 10 pruned; the next pair
    fails, r = 0.025 (count 1) fails and the type leaves.  Six trials, exactly
    the 10 free processors pruned."""
    P = 40
    c = [0.0] * 10 + [1.0] * 30
    w = [0.01 * (i + 1) for i in range(P)]
    alive, L_new, info = PR.drywet_round(additive(0.5, c), [True] * P, w, ["e"] * P, 0.5, 0.01,
                                         uniforms=[0.3] * 10, relative=False)
    assert [len(t["candidates"]) for t in info["trials"]] == [4, 4, 4, 2, 2, 1]
    assert [t["accepted"] for t in info["trials"]] == [True, True, False, True, False, False]
    assert alive == [False] * 10 + [True] * 30
    assert L_new == 0.5
    assert info["draws"] == 6


def test_drywet_type_leaves_once_pruned_out_and_counts_at_least_one():
    """Three free processors of type g (count floor(3 * 0.1 + 1/2) = 0, read as
    1): pruned one per trial, and the type leaves when none is left; type e
    (2 processors, both costly) fails once with a count of 1 and leaves."""
    types = ["g", "e", "g", "e", "g"]
    c = [0.0, 5.0, 0.0, 5.0, 0.0]
    w = [0.3, 0.1, 0.2, 0.4, 0.1]
    # draws: first e (index 0 of [e, g]), then g thrice (index 0 of [g])
    alive, _, info = PR.drywet_round(additive(1.0, c), [True] * 5, w, types, 1.0, 0.01,
                                     uniforms=[0.2, 0.9, 0.0, 0.0], relative=False)
    assert [(t["type"], t["candidates"], t["accepted"]) for t in info["trials"]] == [
        ("e", [1], False), ("g", [4], True), ("g", [2], True), ("g", [0], True)]
    assert alive == [False, True, False, True, False]


def test_drywet_relative_and_absolute_tolerance():
    c = [0.004]
    # absolute tau 0.01 accepts +0.004, relative 1e-3 of L_min = 1 does not
    a_abs, _, _ = PR.drywet_round(additive(1.0, c), [True], [0.5], ["r"], 1.0, 0.01, [0.0], relative=False)
    a_rel, _, _ = PR.drywet_round(additive(1.0, c), [True], [0.5], ["r"], 1.0, 1e-3, [0.0], relative=True)
    assert a_abs == [False] and a_rel == [True]


@pytest.mark.parametrize("seed", range(6))
def test_drywet_invariants_on_random_tables(seed):
    """On random loss tables (interacting terms included): the pruned set of
    every type is a least-weight prefix of that type, the final mask's loss
    is the last accepted trial's and passes the test against the initial
    L_min, and L_min only falls."""
    rng = np.random.default_rng(seed)
    P = 12
    types = [str(t) for t in rng.choice(list("ecsgdr"), size=P)]
    w = rng.random(P).tolist()
    base = rng.normal(scale=0.01, size=P)
    pair = rng.normal(scale=0.01, size=(P, P))

    def loss(alive):
        off = [i for i in range(P) if not alive[i]]
        return 1.0 + sum(base[i] for i in off) + sum(pair[i, j] for i in off for j in off if i < j)

    u = rng.random(200).tolist()
    alive0 = [True] * P
    new, L_new, info = PR.drywet_round(loss, alive0, w, types, 1.0, 0.01, u, relative=False)
    for t in set(types):
        idx = sorted([p for p in range(P) if types[p] == t], key=lambda p: (w[p], p))
        pruned = [p for p in idx if not new[p]]
        assert pruned == idx[:len(pruned)]
    acc = [tr for tr in info["trials"] if tr["accepted"]]
    if acc:
        assert loss(new) == pytest.approx(acc[-1]["L"], abs=1e-15)
        assert loss(new) < 1.0 + 0.01
        assert L_new == min([1.0] + [tr["L"] for tr in acc])
    else:
        assert new == alive0


def test_drywet_brute_force_over_every_draw_sequence():
    """A 6-processor console of two types: enumerate every sequence of type
    draws (the draws decide only which remaining type goes next) and check
    each run against a direct simulation of Alg. 3 written as an explicit
    state walk over (V_t, r_t, T)."""
    types = ["e", "g", "e", "g", "e", "g"]
    w = [0.1, 0.6, 0.3, 0.2, 0.5, 0.4]
    c = [0.001, 0.0, 0.02, 0.003, 0.0, 0.05]
    L0, tau = 1.0, 0.01
    loss = additive(L0, c)

    def walk(choices):
        # state: remaining processors of each type (least weight first), r, the set of types
        V = {t: sorted([p for p in range(6) if types[p] == t], key=lambda p: w[p]) for t in "eg"}
        N = {t: len(V[t]) for t in "eg"}
        r = {"e": 0.1, "g": 0.1}
        T = ["e", "g"]
        off, Lmin, trace = set(), L0, []
        for ch in choices:
            if not T:
                break
            t = T[ch % len(T)]
            kr = int(N[t] * r[t] + 0.5)
            k = min(max(kr, 1), len(V[t]))
            cand = V[t][:k]
            L = loss([p not in off | set(cand) for p in range(6)])
            trace.append((t, tuple(cand), L < Lmin + tau))
            if L < Lmin + tau:
                Lmin, off = min(Lmin, L), off | set(cand)
                V[t] = V[t][k:]
                if not V[t]:
                    T.remove(t)
            elif kr > 1:
                r[t] /= 2
            else:
                T.remove(t)
        return off, trace

    n = 0
    for choices in itertools.product([0, 1], repeat=8):
        u = [(ch + 0.5) / 2.0 for ch in choices]   # u in the ch-th half of [0, 1)
        # with one type left, floor(u * 1) = 0 picks it whatever u is
        alive, _, info = PR.drywet_round(loss, [True] * 6, w, types, L0, tau, u + [0.0] * 8, relative=False)
        off, trace = walk(list(choices) + [0] * 8)
        assert {p for p in range(6) if not alive[p]} == off
        assert [(t["type"], tuple(t["candidates"]), t["accepted"]) for t in info["trials"]] == trace
        n += 1
    assert n == 256


def test_hybrid_runs_brute_force_every_fourth_round():
    assert [PR.hybrid_method(i) for i in range(1, 13)] == ["drywet"] * 3 + ["brute"] + ["drywet"] * 3 + \
        ["brute"] + ["drywet"] * 3 + ["brute"]
